"""Checks of the library's gfx950 device code as the compiler emits it (host only: hipcc
cross-compiles to assembly, no GPU is touched).

* No packed FP32 instructions anywhere (the build disables the feature; the checks would
  catch a build line that loses the flag).
* The step kernels address their population loads with scalar offsets: a value the compiler
  takes for divergent in a scalar operand becomes a waterfall loop (read the first lane's value,
  compare, mask, issue, repeat) around every such load, which cost the two-step kernel 5% of
  its throughput while its idle-wave test was not known to be wave-uniform.
* The step kernels and the sampler's kernels keep everything in registers and LDS (no
  private-segment scratch: a spill would put per-lane memory traffic into the hot loops).
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_1009_0254_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1009_0254_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

pytestmark = pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="hipcc not installed")

HOT = ["lb_step2.hip", "lb_kernels.hip", "lb_sk.hip", "lb_fft.hip"]


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    d = tmp_path_factory.mktemp("asm")
    flags = [f for f in B.FLAGS if f not in ("-shared", "-fPIC")]
    out = {}
    for src in HOT:
        s = str(d / (src + ".s"))
        subprocess.run([HIPCC, *flags, "--cuda-device-only", "-S", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                        os.path.join(CSRC, src), "-o", s], check=True, capture_output=True, text=True)
        out[src] = open(s).read()
    return out


def kernels(text):
    """(mangled name, body) of every kernel in an assembly listing."""
    return re.findall(r"^(_Z\S+):\s*;\s*@\S+\n(.*?)^\.Lfunc_end", text, flags=re.S | re.M)


def kernel_meta(text, name, key):
    m = re.search(r"\.amdhsa_kernel " + re.escape(name) + r"\n(.*?)\.end_amdhsa_kernel", text, flags=re.S)
    assert m, name
    v = re.search(r"\." + key + r"\s+(\d+)", m.group(1))
    assert v, (name, key)
    return int(v.group(1))


def waterfall_loops(body):
    """Loops of the form readfirstlane -> compare with the lane's own value -> and_saveexec."""
    lines = [ln.strip() for ln in body.split("\n") if ln.strip() and not ln.strip().startswith(";")]
    n = 0
    for i, ln in enumerate(lines):
        if ln.startswith("v_readfirstlane_b32"):
            win = lines[i + 1:i + 5]
            if any(w.startswith("v_cmp_eq_u32") for w in win) and any(w.startswith("s_and_saveexec") for w in win):
                n += 1
    return n


def test_every_hot_file_has_kernels(asm):
    for src, text in asm.items():
        assert kernels(text), src


def test_no_packed_fp32(asm):
    for src, text in asm.items():
        found = sorted(set(re.findall(r"\bv_pk_(?:add|mul|fma)_f32\b", text)))
        assert not found, (src, found)


@pytest.mark.parametrize("src,prefix", [("lb_step2.hip", "_ZN3lbf7k_step2"), ("lb_kernels.hip", "_ZN3lbf6k_step")])
def test_step_kernels_have_no_waterfall_loops(asm, src, prefix):
    ks = [(n, b) for n, b in kernels(asm[src]) if n.startswith(prefix)]
    assert ks, prefix
    for name, body in ks:
        assert waterfall_loops(body) == 0, name


@pytest.mark.parametrize("src,prefix", [("lb_step2.hip", "_ZN3lbf7k_step2"), ("lb_kernels.hip", "_ZN3lbf6k_step"),
                                        ("lb_sk.hip", "_ZN3lbf12_GLOBAL__N_19k_sk_"),
                                        ("lb_fft.hip", "_ZN3lbf8k_cn_")])
def test_hot_kernels_do_not_spill(asm, src, prefix):
    ks = [n for n, _ in kernels(asm[src]) if n.startswith(prefix)]
    assert ks, prefix
    for name in ks:
        assert kernel_meta(asm[src], name, "amdhsa_private_segment_fixed_size") == 0, name


def test_waterfall_detector_finds_one():
    body = """
    v_readfirstlane_b32 s6, v14
    s_nop 1
    v_cmp_eq_u32_e32 vcc, s6, v14
    s_and_saveexec_b64 vcc, vcc
    buffer_load_dword v81, v8, s[12:15], s6 offen
    s_xor_b64 exec, exec, vcc
    s_cbranch_execnz .LBB5_71
    """
    assert waterfall_loops(body) == 1
    assert waterfall_loops(body.replace("v_cmp_eq_u32_e32", "v_add_u32_e32")) == 0
