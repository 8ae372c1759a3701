"""Host: the library's FP64 ln u and sin/cos 2 pi u at the Box-Muller uniforms u = (b + 1/2) 2^-21
(lb_rng.h: u21_ln, u21_sincos_turn), built for the host from the same header and evaluated at
every 21-bit b.  Both use only correctly rounded operations (products, sums, fma, one division,
bit manipulation), so the host build gives the device's bits.  Against references reduced
exactly in long double: within 5e-16 relative (measured 2.2e-16 for ln, 2.6e-16 for sin and cos);
against the double libm calls of the oracle: sin and cos within 2e-15 absolute (the oracle
rounds 2 pi u first)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_u21_transcendentals_over_every_argument(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "u21_check")
    subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17",
                    "-I", os.path.join(ROOT, "paper_1009_0254_amd", "csrc"),
                    os.path.join(ROOT, "tests", "u21_math_check.cpp"), "-o", exe],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([exe, "5e-16"], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
