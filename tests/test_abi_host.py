"""Host-side checks of the C ABI: the library loads, exports every declared entry point,
the Python struct matches the C layout, and parameter validation rejects what the
model forbids (tau <= 1/2 by the stability requirement of Sec. III.A; a noise matrix
Xi(0) that is not positive semi-definite, Sec. III.C).  No GPU is touched."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1009_0254_amd import lbfluct as L
from paper_1009_0254_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbfluct.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:lb_status|void|const char \*)\s*\**\s*(lb_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for want in ("lb_workspace_size", "lb_init", "lb_step", "lb_moments", "lb_structure_factor",
                 "lb_status_flags", "lb_free", "lb_strerror"):
        assert want in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(lb_\w+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_param_struct_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "lbfluct.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(lb_params), offsetof(lb_params, rho0), offsetof(lb_params, kT),
         offsetof(lb_params, seed), offsetof(lb_params, init_kind), offsetof(lb_params, init_arg));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    P = L.LbParams
    assert got == [ctypes.sizeof(P), P.rho0.offset, P.kT.offset, P.seed.offset, P.init_kind.offset,
                   P.init_arg.offset]


def test_header_is_strict_c99_and_cxx(tmp_path):
    """The header compiles alone as pedantic C99 and as C++11, with every warning an error."""
    src = tmp_path / "h.c"
    src.write_text('#include "lbfluct.h"\nint main(void) { lb_handle *h = 0; lb_free(h); return (int)sizeof(lb_params) == 0; }\n')
    inc = ["-I", os.path.join(ROOT, "include")]
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", *inc, "-c", str(src),
                    "-o", str(tmp_path / "h.o")], check=True)
    subprocess.run(["g++", "-std=c++11", "-x", "c++", "-Wall", "-Wextra", "-pedantic", "-Werror", *inc, "-c",
                    str(src), "-o", str(tmp_path / "hpp.o")], check=True)


def test_c_client_builds_against_the_header_and_library(tmp_path):
    """A C program that uses only the header, the library and the HIP runtime compiles and
    links; run without arguments it prints its usage (no device call)."""
    from conftest import build_c_client
    exe = build_c_client(tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 2 and "usage" in r.stderr


def test_strerror():
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert isinstance(L.lb_strerror(code), str) and L.lb_strerror(code)
    assert L.lb_strerror(-99) == "unknown status"


def test_workspace_size_counts_both_population_buffers():
    c = W.single_phase(64, 32)
    n = 64 * 32
    b64 = L.lb_workspace_size([c], L.LB_FP64)
    b32 = L.lb_workspace_size([c], L.LB_FP32_SHIFTED)
    assert b64 >= 2 * 9 * n * 8 and b32 >= 2 * 9 * n * 4 and b64 > b32
    bsk = L.lb_workspace_size([c], L.LB_FP32_SHIFTED, L.LB_FEATURE_STRUCTURE_FACTOR)
    # accumulators [9][33][32] plus the row spectra of all nine modes (FP32 complex for FP32
    # storage, FP64 complex for FP64 storage)
    assert bsk >= b32 + 9 * 32 * 33 * 8 + 9 * 32 * 33 * 8
    bsk64 = L.lb_workspace_size([c], L.LB_FP64, L.LB_FEATURE_STRUCTURE_FACTOR)
    assert bsk64 >= b64 + 9 * 32 * 33 * 8 + 9 * 32 * 33 * 16
    two = L.lb_workspace_size([c, W.single_phase(128, 128)], L.LB_FP32_SHIFTED)
    assert two >= b32 + 2 * 9 * 128 * 128 * 4


@pytest.mark.parametrize("over,code", [
    (dict(tau_shear=0.5), L.LB_EINVAL),
    (dict(tau_bulk=0.3), L.LB_EINVAL),
    (dict(tau_eps=float("nan")), L.LB_EINVAL),
    (dict(nx=2), L.LB_EINVAL),
    (dict(ny=0), L.LB_EINVAL),
    (dict(rho0=0.0), L.LB_EINVAL),
    (dict(kT=-1e-6), L.LB_EINVAL),
    (dict(A=0.5), L.LB_ENOTPSD),          # c_s^2 = 0.83 > 2/3 makes Xi_44 negative
    (dict(c0sq=1.0), L.LB_ENOTPSD),
    (dict(noise="correlated", nx=48), L.LB_EINVAL),        # correlated noise needs powers of two
    (dict(replica=0x80000000), L.LB_EINVAL),              # top bit names the correlated stream
    # Xi(k) not PSD at large k: kappa large enough that c_s^2(k) > 2/3 near the zone corner
    (dict(noise="correlated", kappa=0.1), L.LB_ENOTPSD),
])
def test_validation_rejects(over, code):
    c = W.single_phase(16, 16)
    c.update(over)
    with pytest.raises(L.LbError) as e:
        L.lb_workspace_size([c], L.LB_FP32_SHIFTED)
    assert e.value.status == code


def test_validation_rejects_bad_precision_and_count():
    arr = (L.LbParams * 1)()
    arr[0] = L.make_params(W.single_phase(16, 16))
    n = ctypes.c_size_t(0)
    assert L.lib().lb_workspace_size(arr, 1, 7, 0, ctypes.byref(n)) == L.LB_EINVAL
    assert L.lib().lb_workspace_size(arr, 0, 0, 0, ctypes.byref(n)) == L.LB_EINVAL
    h = ctypes.c_void_p()
    # a misaligned workspace pointer is rejected before any device call
    assert L.lib().lb_init(arr, 1, 0, 0, 8, 1 << 30, None, ctypes.byref(h)) == L.LB_EINVAL
    assert L.lib().lb_noise_normals(1, 0, 0, -1, 0, None, None) == L.LB_EINVAL
    assert L.lib().lb_philox(0, 0, 0, 0, 0, -5, None, None) == L.LB_EINVAL


def test_all_workloads_validate():
    for cfg in (W.single_phase_64(), W.slab_2048(), W.single_phase_8192(), W.quench_16384(), W.uncorrelated_sec5a(), W.correlated_sec5a()):
        assert L.lb_workspace_size([cfg], L.LB_FP32_SHIFTED) > 0
    reps = W.ensemble_336()
    assert len(reps) == 336
    assert sum(r["nx"] * r["ny"] for r in reps) == 12_582_912
    assert L.lb_workspace_size(reps, L.LB_FP32_SHIFTED) > 2 * 9 * 12_582_912 * 4


def test_structure_factor_feature_size_rules():
    F = L.LB_FEATURE_STRUCTURE_FACTOR
    for nx, ny in [(16384, 16), (16, 16384), (4, 4), (256, 128)]:
        assert L.lb_workspace_size([W.single_phase(nx, ny)], L.LB_FP32_SHIFTED, F) > 0
    for nx, ny in [(48, 32), (32768, 4), (2, 8), (64, 3)]:
        with pytest.raises(L.LbError) as e:
            L.lb_workspace_size([W.single_phase(nx, ny)], L.LB_FP32_SHIFTED, F)
        assert e.value.status == L.LB_EINVAL
    # unknown feature bits
    with pytest.raises(L.LbError) as e:
        L.lb_workspace_size([W.single_phase(16, 16)], L.LB_FP32_SHIFTED, 2)
    assert e.value.status == L.LB_EINVAL
    # the 16384^2 workspace: two FP32 population buffers, the FP64 initial density, the
    # accumulators and the FP32 complex row spectra of the nine modes
    n = 16384 * 16384
    want = 2 * 9 * n * 4 + n * 8 + 9 * 16384 * 8193 * 8 + 9 * 16384 * 8193 * 8
    b = L.lb_workspace_size([W.quench_16384()], L.LB_FP32_SHIFTED, F)
    assert want <= b < want + (64 << 20)


def test_diagonal_noise_needs_only_a_nonnegative_diagonal():
    """Near c_s^2 = 2/3 the 4-9 block of Xi(0) is not PSD (its determinant turns negative
    before Xi_44 does), so the Cholesky noise is rejected; the diagonal variant of Sec. IV is
    valid there.  Past c_s^2 = 2/3, Xi_44 < 0 and both are rejected."""
    near = W.single_phase(16, 16, c0sq=0.6, A=0.05)        # c_s^2 = 0.65
    with pytest.raises(L.LbError) as e:
        L.lb_workspace_size([near], L.LB_FP32_SHIFTED)
    assert e.value.status == L.LB_ENOTPSD
    assert L.lb_workspace_size([dict(near, noise="diagonal")], L.LB_FP32_SHIFTED) > 0
    past = W.single_phase(16, 16, c0sq=0.7, A=0.05)        # c_s^2 = 0.75
    with pytest.raises(L.LbError) as e:
        L.lb_workspace_size([dict(past, noise="diagonal")], L.LB_FP32_SHIFTED)
    assert e.value.status == L.LB_ENOTPSD


def test_correlated_noise_validation_follows_the_fig2_region():
    """lb_init's PSD check of Xi(k) over the lattice agrees with the closed-form boundary of
    Fig. 2 for tau = 1 (c_s^2 + 16/3 kappa <= 3/5; a 16 x 16 lattice contains the corner)."""
    for kappa in (0.0, 0.03, 0.06, 0.09):
        for cs in (0.1, 0.3, 0.5, 0.7, 0.75):
            margin = cs * cs + 16.0 / 3.0 * kappa - 0.6
            if abs(margin) < 5e-3:
                continue
            cfg = dict(W.single_phase(16, 16, c0sq=cs * cs, A=0.0, B=0.0, kappa=kappa, kT=1e-7),
                       tau_bulk=1.0, tau_shear=1.0, tau_q=1.0, tau_eps=1.0, noise="correlated")
            if margin < 0:
                assert L.lb_workspace_size([cfg], L.LB_FP32_SHIFTED) > 0
            else:
                with pytest.raises(L.LbError) as e:
                    L.lb_workspace_size([cfg], L.LB_FP32_SHIFTED)
                assert e.value.status == L.LB_ENOTPSD, (kappa, cs)


def test_bench_traffic_is_tied_to_the_profiled_kernel_workload_and_tile(tmp_path, monkeypatch):
    """bench.py reports counter-measured HBM bytes only for the kernel source, workload and
    launch configuration (width, rows, steps per launch) the committed counters were taken
    with; anything else gives null."""
    import json
    import sys
    sys.path.insert(0, ROOT)
    import bench
    sha = bench.kernel_sha()
    c = {"kernel_src_sha": sha, "workload_key": "single_phase_8192", "hbm_bytes_per_launch": 1.0,
         "per_tile": {"512,8,1": {"hbm_bytes_per_launch": 5.0}, "256,16,2": {"hbm_bytes_per_launch": 4.0}}}
    f = tmp_path / "c.json"
    f.write_text(json.dumps(c))
    monkeypatch.setattr(bench, "COUNTERS", str(f))
    assert bench.traffic_from_counters("single_phase_8192", (512, 8, 1)) == 5.0
    assert bench.traffic_from_counters("single_phase_8192", (256, 16, 2)) == 4.0
    assert bench.traffic_from_counters("single_phase_8192", (256, 16, 1)) is None
    assert bench.traffic_from_counters("single_phase_8192", (128, 8, 1)) is None
    assert bench.traffic_from_counters("ensemble_336", (512, 8, 1)) is None
    c["kernel_src_sha"] = "0" * 16
    f.write_text(json.dumps(c))
    assert bench.traffic_from_counters("single_phase_8192", (512, 8, 1)) is None
    assert len(sha) == 16


def test_committed_counters_name_their_workload_and_tiles():
    import json
    c = json.load(open(os.path.join(ROOT, "profiles", "k_step2_fp32s_8192_counters.json")))
    assert c["workload_key"] == "single_phase_8192" and c["tile"] in c["per_tile"]
    for t, v in c["per_tile"].items():
        w, r, k = (int(s) for s in t.split(","))
        # a launch moves at least one read and one write of every population (two steps per
        # launch move the same bytes as one)
        assert w % 64 == 0 and r >= 4 and k in (1, 2) and v["hbm_bytes_per_launch"] > 72 * 8192 * 8192 * 0.9
