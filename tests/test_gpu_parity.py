"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same
seeded inputs, element by element.

Tolerances, derived from the arithmetic of each side:

* FP64 storage: absolute |m_a^gpu - m_a^oracle| <= 2e-12 max(1, max|m_a|).  The oracle
  keeps absolute populations f_i ~ w_i, so its own rounding grows like eps sqrt(t): an
  80-bit build of the same oracle differs from the FP64 oracle by 1.2e-13 after 400 steps
  of a 1e-4 wave.  The GPU works on deviations f_i - w_i rho0 and is the more precise of
  the two (it agrees with the 80-bit build to that level).
* FP32-shifted storage (deviations from the rest state fbar_i = T^-1 m^eq(rho0, u = 0)),
  noise-free runs: the required 1e-5, relative to the fluctuation,
  err_a = max_r |m_a^gpu - m_a^oracle| / max_r |m_a^oracle - mean(m_a^oracle)|, for rho, j_x,
  j_y: single-phase waves, the two-phase slab's density and the spinodal quench (measured
  3e-7 to 1.4e-6).  One derived floor remains: a 0.02 uniform flow carries populations
  ~0.02 w_i away from rest, whose FP32 rounding (~1e-9) is ~1e-4 of the 1e-4 wave riding on
  j_x (measured 2.0e-4; gate 6e-4).
* Noisy runs in FP32: the single-precision Box-Muller (hardware log2/sin/cos) differs from
  the FP64 normals by <= 3e-6 per draw, which the trajectories integrate; every case is
  deterministic (same seeds, same bits run after run), so each gate is about 3x the error
  measured for its case (single phase 1.8e-7 to 2.5e-7; the two-phase slab, whose bulk phases
  hold O(0.5) deviations from rest, 8.9e-6).
* Integer work (Philox) is compared bit for bit.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from oracle import theory as th  # noqa: E402
from paper_1009_0254_amd import workloads as W  # noqa: E402


def _L():
    from paper_1009_0254_amd import lbfluct as L
    return L


def say(*a):
    print("[gpu-parity]", *a, file=sys.stderr, flush=True)


def rel_err(mg, mo):
    out = []
    for a in range(9):
        rng = np.abs(mo[a] - mo[a].mean()).max()
        out.append(np.abs(mg[a] - mo[a]).max() / max(rng, 1e-300))
    return np.array(out)


def abs_ok(mg, mo, tol=2e-12):
    scale = np.maximum(1.0, np.abs(mo).reshape(9, -1).max(axis=1))
    err = np.abs(mg - mo).reshape(9, -1).max(axis=1) / scale
    return err.max() <= tol, err


def run_pair(cfg, precision, steps, chunks=1):
    L = _L()
    say("case", cfg.get("nx"), cfg.get("ny"), cfg.get("init"), "kT", cfg["kT"], precision, "steps", steps)
    lat = L.Lattice(cfg, precision=precision)
    ora = O.Oracle(cfg)
    per = steps // chunks
    for _ in range(chunks):
        lat.step(per)
        ora.step(per)
    mg = lat.moments()
    mo = ora.moments()
    lat.close()
    return mg, mo


# ------------------------------------------------------------------ RNG


def test_philox_bitwise():
    L = _L()
    n = 4096
    out = torch.zeros(4 * n, dtype=torch.int32, device="cuda")
    L.lb_philox(7, 123456789, 0xFFFFFFFF, 0xDEADBEEF, 0x01234567, n, out)
    got = out.cpu().numpy().view(np.uint32).reshape(n, 4)
    for k in list(range(0, n, 97)) + [n - 1]:
        assert list(got[k]) == O.philox4x32_10([k, 7, 123456789, 0xFFFFFFFF], [0xDEADBEEF, 0x01234567])
    # published known answers through the GPU path
    for ln in open(os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")):
        if ln.startswith("#") or not ln.strip():
            continue
        v = [int(s, 16) for s in ln.split()]
        if v[0] != 0:
            continue
        L.lb_philox(v[1], v[2], v[3], v[4], v[5], 1, out)
        assert list(out[:4].cpu().numpy().view(np.uint32)) == v[6:10]


@pytest.mark.parametrize("precision,tol", [(0, 1e-14), (1, 3e-6)])
def test_normals_match_oracle(precision, tol):
    L = _L()
    n = 20000
    out = torch.zeros(6 * n, dtype=torch.float64, device="cuda")
    seed, rep, t = 0x1234_5678_9ABC, 5, 3_000_000_123
    L.lb_noise_normals(seed, rep, t, n, precision, out)
    got = out.cpu().numpy().reshape(n, 6)
    want = O.normals_batch(seed, rep, t, n)
    err = np.abs(got - want) / np.maximum(1.0, np.abs(want))
    say("normals precision", precision, "max err", err.max())
    assert err.max() < tol


# ------------------------------------------------------------------ initial state


@pytest.mark.parametrize("precision", [0, 2, 1])
@pytest.mark.parametrize("cfgf", [
    lambda: W.wave(W.single_phase(64, 40, kT=0), 2, 1, 1e-3, 2e-3, -1e-3, U=0.01),
    lambda: W.slab(48, 64, kT=0),
    lambda: W.spinodal(70, 33, kT=0, seed=4),
])
def test_initial_moments(cfgf, precision):
    cfg = cfgf()
    mg, mo = run_pair(cfg, precision, 0)
    if precision == 0:
        ok, err = abs_ok(mg, mo, 1e-14)
        say("init", cfg["init"], "fp64 abs err", err.max())
        assert ok
    else:
        e = rel_err(mg, mo)
        say("init", cfg["init"], precision, e[:3])
        # one FP32 rounding of each stored value: |d rho| <= 9 max|s_i| 2^-24, s_i the
        # deviation from the rest state (FP32-shifted; measured <= 3.4e-7 of the range) or the
        # population itself (plain FP32)
        assert e[:3].max() < {2: 1e-6, 1: 1e-4}[precision]


# ------------------------------------------------------------------ deterministic dynamics


DET = [
    # label, config, steps, FP32-shifted gate on (rho, jx, jy)
    ("wave64", lambda: W.wave(W.single_phase(64, 64, kT=0), 1, 0, 1e-4, 0, 1e-4), 400, 1e-5),
    ("wave_ragged", lambda: W.wave(W.single_phase(100, 37, kT=0, tau_bulk=0.7, tau_q=0.9), 3, 2, 1e-4, 1e-4, 0),
     100, 1e-5),
    ("tiny", lambda: W.wave(W.single_phase(3, 5, kT=0), 1, 1, 1e-4, 1e-4, 0), 4, 1e-5),
    # the 3x5 lattice's slowest wave (k = 2 pi/5 along y) over 40 steps, in which it decays by
    # ~5e-3; compared about each side's mean (see MEAN_REMOVED)
    ("tiny_40", lambda: W.wave(W.single_phase(3, 5, kT=0), 0, 1, 1e-3, 1e-3, 0), 40, 1e-5),
    ("flow", lambda: W.wave(W.single_phase(96, 64, kT=0), 2, 1, 1e-4, 0, 1e-4, U=0.02), 300, 6e-4),
    ("slab", lambda: W.slab(64, 128, kT=0), 500, 1e-5),
    ("spinodal", lambda: W.spinodal(128, 96, kT=0, amp=0.01, seed=2), 300, 1e-5),
]


# Cases compared as fluctuations about each side's own lattice mean.  The means of rho, j_x and
# j_y are conserved totals, so in FP32-shifted storage they keep the one rounding of the stored
# initial state (~1e-11 per node at amplitude 1e-3) while the decaying wave's range shrinks below
# it; the totals have their own conservation tests.
MEAN_REMOVED = {"tiny_40"}


@pytest.mark.parametrize("label,cfgf,steps,tol32", DET, ids=[d[0] for d in DET])
@pytest.mark.parametrize("precision", [0, 2])
def test_deterministic_parity(label, cfgf, steps, tol32, precision):
    cfg = cfgf()
    mg, mo = run_pair(cfg, precision, steps, chunks=2)
    if label in MEAN_REMOVED:
        mg = mg - mg.mean(axis=(1, 2), keepdims=True)
        mo = mo - mo.mean(axis=(1, 2), keepdims=True)
    e = rel_err(mg, mo)
    if precision == 0:
        ok, err = abs_ok(mg, mo)
        say(label, "fp64 abs err per mode", err, "normalised rho,jx,jy", e[:3])
        assert ok
    else:
        say(label, "fp32s err rho,jx,jy", e[:3])
        # slab j_x is identically zero on both sides; its range is zero
        e3 = np.where(np.isfinite(e[:3]), e[:3], 0.0)
        if label == "slab":
            e3[2] = 0.0      # j_y across a static interface is rounding-level on both sides
        assert e3.max() < tol32


def test_fp32_plain_is_reported():
    cfg = W.wave(W.single_phase(64, 64, kT=0), 1, 0, 1e-4, 0, 1e-4)
    mg, mo = run_pair(cfg, 1, 400)
    e = rel_err(mg, mo)
    say("fp32 plain err rho,jx,jy", e[:3])
    assert np.isfinite(e).all() and e[:3].max() < 1e-2


# ------------------------------------------------------------------ noisy dynamics


NOISY = [
    # label, config, steps, FP32-shifted gate (all nine modes; ~3x the measured error)
    ("single_phase_64", lambda: W.single_phase_64(), 2000, 6e-7),
    ("ragged", lambda: W.single_phase(72, 50, kT=1e-5, seed=17, replica=3), 500, 6e-7),
    ("tiny", lambda: W.single_phase(3, 5, kT=1e-5, seed=2), 300, 8e-7),
    ("slab", lambda: W.slab(64, 128, kT=1e-6, seed=5), 500, 3e-5),
    ("uncorrelated_sec5a", lambda: W.uncorrelated_sec5a(64, 64, kT=1e-7), 500, 8e-7),
    ("diagonal", lambda: W.single_phase(64, 48, kT=1e-5, seed=9, c0sq=0.0, A=0.05, noise="diagonal"), 400, 7e-7),
]


@pytest.mark.parametrize("label,cfgf,steps,tol32", NOISY, ids=[d[0] for d in NOISY])
@pytest.mark.parametrize("precision", [0, 2])
def test_noisy_parity(label, cfgf, steps, tol32, precision):
    cfg = cfgf()
    mg, mo = run_pair(cfg, precision, steps, chunks=2)
    e = rel_err(mg, mo)
    if precision == 0:
        ok, err = abs_ok(mg, mo)
        say(label, "fp64 abs err per mode", err, "normalised all", e)
        assert ok
    else:
        say(label, "fp32s err all modes", e)
        assert e.max() < tol32


# ------------------------------------------------------------------ ensembles, graphs, determinism


def test_ensemble_of_uneven_replicas():
    L = _L()
    cfgs = [W.single_phase(64, 64, kT=3e-5, seed=11, replica=0),
            W.single_phase(128, 96, kT=1e-6, seed=12, replica=1),
            W.slab(64, 128, kT=1e-6, seed=13, replica=2),
            W.wave(W.single_phase(40, 24, kT=0), 1, 1, 1e-4, 0, 1e-4)]
    lat = L.Lattice(cfgs, precision=0)
    lat.step(150)
    for r, c in enumerate(cfgs):
        o = O.Oracle(c)
        o.step(150)
        ok, err = abs_ok(lat.moments(r), o.moments())
        say("ensemble replica", r, err.max())
        assert ok
    lat.close()


@pytest.mark.parametrize("precision", [0, 2])
def test_plain_c_client_matches_binding_and_oracle(tmp_path, precision):
    """The library driven from a C program alone (tests/c_client.c: its own hipMalloc'd
    workspace and stream, no torch, the state advanced in two lb_step calls) returns the
    same bits as the Python binding and agrees with the oracle to the gates above; the
    error returns it checks along the way are those the header documents."""
    import subprocess
    from conftest import build_c_client
    L = _L()
    cfgs = [W.single_phase(72, 50, kT=1e-5, seed=17, replica=3),
            W.wave(W.single_phase(40, 24, kT=0), 1, 1, 1e-4, 0, 1e-4)]
    steps = 121
    exe = build_c_client(tmp_path)
    pf, out = tmp_path / "params.bin", tmp_path / "out.bin"
    pf.write_bytes(b"".join(bytes(L.make_params(c)) for c in cfgs))
    say("c client precision", precision, "steps", steps)
    r = subprocess.run([exe, str(pf), str(precision), str(steps), str(out)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    raw = out.read_bytes()
    lat = L.Lattice(cfgs, precision=precision)
    lat.step(steps)
    off = 0
    for rep, c in enumerate(cfgs):
        n9 = 9 * c["nx"] * c["ny"]
        mc = np.frombuffer(raw, np.float64, n9, off).reshape(9, c["ny"], c["nx"])
        tc = np.frombuffer(raw, np.float64, 6, off + 8 * n9)
        off += 8 * (n9 + 6)
        assert np.array_equal(mc, lat.moments(rep)) and np.array_equal(tc, lat.totals(rep))
        o = O.Oracle(c)
        o.step(steps)
        mo = o.moments()
        e = rel_err(mc, mo)
        if precision == 0:
            ok, err = abs_ok(mc, mo)
            say("c client replica", rep, "fp64 abs err", err.max())
            assert ok
        else:
            say("c client replica", rep, "fp32s err", e)
            assert (e.max() if c["kT"] > 0 else e[:3].max()) < (6e-7 if c["kT"] > 0 else 1e-5)
    flags = int(np.frombuffer(raw, np.uint32, 1, off)[0])
    step = int(np.frombuffer(raw, np.int64, 1, off + 4)[0])
    assert off + 12 == len(raw)
    assert (flags, step) == tuple(lat.lb_status_flags()) and step == steps
    lat.close()


def test_graph_replay_matches_single_steps_bitwise():
    L = _L()
    cfg = W.single_phase(96, 80, kT=1e-5, seed=3)
    a = L.Lattice(cfg, precision=2)
    a.step(70)                     # two graph replays + 6 single steps
    b = L.Lattice(cfg, precision=2)
    for _ in range(70):
        b.step(1)
    ma, mb = a.moments(), b.moments()
    assert np.array_equal(ma, mb)
    assert a.lb_status_flags()[1] == 70 and b.lb_status_flags()[1] == 70
    a.close()
    b.close()


def test_tile_shape_does_not_change_bits(monkeypatch):
    L = _L()
    cfg = W.single_phase(300, 130, kT=1e-5, seed=8)
    res = []
    for tile in ("64,8", "256,32", "128,16", "512,64", "256,8", "512,4", "64,4"):
        monkeypatch.setenv("LBF_TILE", tile)
        lat = L.Lattice(cfg, precision=2)
        lat.step(40)
        res.append(lat.moments())
        lat.close()
    for m in res[1:]:
        assert np.array_equal(m, res[0])


TWO_STEP_CASES = [
    ("strips", [W.single_phase(1100, 70, kT=1e-5, seed=8)]),
    ("mixed", [W.single_phase(128, 40, kT=1e-5, seed=21, replica=0),
               W.single_phase(64, 24, kT=2e-5, seed=22, replica=1),
               W.single_phase(100, 36, kT=1e-5, seed=23, replica=2),
               W.single_phase(600, 18, kT=1e-5, seed=24, replica=3),
               W.wave(W.single_phase(3, 9, kT=0), 1, 1, 1e-4, 0, 1e-4),
               W.slab(40, 64, kT=1e-6, seed=25, replica=5)]),
    ("tiny", [W.single_phase(3, 5, kT=1e-5, seed=2)]),
    ("correlated", [dict(W.correlated_sec5a(64, 32, kT=1e-6, seed=31), replica=0),
                    W.single_phase(100, 36, kT=1e-5, seed=32, replica=1),
                    dict(W.correlated_sec5a(512, 16, kT=1e-6, seed=33), replica=2)]),
]


@pytest.mark.parametrize("label,cfgs", TWO_STEP_CASES, ids=[c[0] for c in TWO_STEP_CASES])
@pytest.mark.parametrize("precision", [2, 0, 1])
def test_two_steps_per_launch_bitwise(monkeypatch, label, cfgs, precision):
    """The two-steps-per-launch kernel gives the bits of the one-step kernel, for every
    workgroup width and tile height: overlapping strips (a ragged last strip, tile heights
    that do not divide ny), whole rows packed 2 to 8 per workgroup with empty groups, a
    3 x 5 lattice whose tile wraps its rows twice, replicas with the exact Xi(k) noise (both
    steps' fields made before the launch) beside a k = 0 one, all three storages; odd step
    counts end with a one-step launch, 64 steps replay the captured graph.  Flags and time
    agree too."""
    L = _L()
    def run(env):
        for k in ("LBF_TILE", "LBF_TILE2", "LBF_STEPS_PER_LAUNCH"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        lat = L.Lattice(cfgs, precision=precision)
        tune = lat.lb_tuning()
        out = []
        for n in (37, 64):
            lat.step(n)
            out.append(([lat.moments(r) for r in range(len(cfgs))], lat.lb_status_flags()))
        lat.close()
        return tune, out
    t1, ref = run({"LBF_TILE": "256,16", "LBF_STEPS_PER_LAUNCH": "1"})
    assert t1[3] == 1
    for tile in ("512,32", "256,16", "128,8", "384,64", "448,24", "320,13"):
        say("two-step", label, "precision", precision, "tile", tile)
        t2, got = run({"LBF_TILE": "256,16", "LBF_TILE2": tile, "LBF_STEPS_PER_LAUNCH": "2"})
        assert t2[3] == 2 and t2[0] == int(tile.split(",")[0])
        for (mg, fg), (mr, fr) in zip(got, ref):
            assert fg == fr
            for r in range(len(cfgs)):
                assert np.array_equal(mg[r], mr[r]), (tile, r)
    if precision == 0:
        o = O.Oracle(cfgs[0])
        o.step(101)
        assert abs_ok(ref[1][0][0], o.moments())[0]


@pytest.mark.parametrize("precision", [2, 0])
def test_ensemble_tile_shapes_do_not_change_bits(monkeypatch, precision):
    """Replicas narrower than the strip (whole-row strips, idle waves past the row) and wider
    ones (halo columns) in one launch: every shape gives the same bits."""
    L = _L()
    cfgs = [W.single_phase(128, 40, kT=1e-5, seed=21, replica=0),
            W.single_phase(64, 24, kT=2e-5, seed=22, replica=1),
            W.single_phase(100, 36, kT=1e-5, seed=23, replica=2),
            W.single_phase(300, 20, kT=1e-5, seed=24, replica=3),
            W.wave(W.single_phase(3, 9, kT=0), 1, 1, 1e-4, 0, 1e-4)]
    res = []
    for tile in ("64,8", "128,4", "256,8", "512,16", "256,4"):
        monkeypatch.setenv("LBF_TILE", tile)
        lat = L.Lattice(cfgs, precision=precision)
        lat.step(37)
        res.append([lat.moments(r) for r in range(len(cfgs))])
        lat.close()
    for other in res[1:]:
        for r in range(len(cfgs)):
            assert np.array_equal(other[r], res[0][r]), r
    o = O.Oracle(cfgs[2])
    o.step(37)
    if precision == 0:
        assert abs_ok(res[0][2], o.moments())[0]


def test_conservation_fp64_and_fp32s():
    L = _L()
    # FP64: drift at rounding level; FP32-shifted: each node's populations are rounded to
    # FP32 every step, so sum j random-walks by ~1e-11 per node per sqrt(step)
    for prec, tol, jtol in ((0, 1e-13, 1e-11), (2, 1e-9, 1e-5)):
        cfg = W.single_phase(256, 256, kT=1e-5, seed=99)
        lat = L.Lattice(cfg, precision=prec)
        lat.step(3)
        t0 = lat.totals()
        lat.step(1)
        t1 = lat.totals()
        lat.step(200)
        t2 = lat.totals()
        say("totals", prec, t0, t1, t2)
        assert abs(t2[0] - t0[0]) / t0[0] < tol
        assert abs(t2[1] - t0[1]) < jtol and abs(t2[2] - t0[2]) < jtol
        # streaming flips the staggered momentum sums exactly in exact arithmetic
        assert abs(t1[4] + t0[4]) < jtol and abs(t1[5] + t0[5]) < jtol
        lat.close()


def test_status_flags_clean_and_clamp():
    L = _L()
    lat = L.Lattice(W.single_phase_64(), precision=2)
    lat.step(100)
    f, t = lat.lb_status_flags()
    assert f == 0 and t == 100
    lat.close()
    # a density field whose local c_s^2 exceeds 2/3 somewhere makes Xi_44 negative there:
    # the pivot is clamped (flag), never NaN
    cfg = W.spinodal(64, 64, kT=1e-6, seed=3, amp=0.05)
    cfg.update(c0sq=1.0 / 3.0, A=0.05, B=20.0)
    lat = L.Lattice(cfg, precision=0)
    lat.step(2)
    f, _ = lat.lb_status_flags()
    assert f & L.LB_FLAG_CLAMPED_PIVOT
    assert not (f & L.LB_FLAG_NAN)
    o = O.Oracle(cfg)
    o.step(2)
    assert o.flags[0] > 0
    ok, err = abs_ok(lat.moments(), o.moments())
    say("clamp case fp64 abs err", err.max())
    assert ok
    lat.close()


# ------------------------------------------------------------------ structure factor


def fp64_spectrum_tol(n, smax):
    """FP64 FFT rounding: the k = 0 coefficient (sum of a moment, ~ n) spreads errors of
    ~ eps log2(n) n over every output; relative to sqrt(n S_max) that bounds the error of
    S(k) / S_max, with a factor 8 of margin."""
    eps = 2.2e-16
    return 1e-10 + 8 * 2 * eps * np.log2(n) * n / np.sqrt(n * smax)


SK_SHAPES = [(64, 32), (16384, 16), (16, 16384), (16, 8192), (8, 4096), (2048, 8), (4096, 64), (8192, 16), (4, 4)]


@pytest.mark.parametrize("shape", SK_SHAPES, ids=[f"{a}x{b}" for a, b in SK_SHAPES])
@pytest.mark.parametrize("precision", [0, 2])
def test_structure_factor_matches_oracle_fft(precision, shape):
    """All nine |m_a(k)|^2 against numpy's FFT of the oracle's moments: rows of length 16384
    (real-to-complex split), columns of 4096, 8192 and 16384 (the last with one
    decimation-in-frequency stage; 4096 and 8192 on the compile-time-length transforms),
    all nine modes per pass (up to 2048 wide), rows of 4096 and 8192 whose FP32 moments stay
    in registers across mode groups (8 + 1 and 4 + 4 + 1), and the smallest lattice."""
    L = _L()
    nx, ny = shape
    cfg = W.single_phase(nx, ny, kT=1e-5, seed=31)
    lat = L.Lattice(cfg, precision=precision, structure_factor=True)
    ora = O.Oracle(cfg)
    acc = np.zeros((9, ny, nx // 2 + 1))
    for _ in range(5):
        lat.step(7)
        ora.step(7)
        lat.lb_structure_factor(L.LB_SK_SAMPLE, 0)
        acc += O.power_spectrum(ora.moments())
    S, ns = lat.lb_structure_factor(L.LB_SK_READ, 0)
    S = S.cpu().numpy()
    want = acc / 5
    assert ns == 5
    mask = np.ones_like(want, dtype=bool)
    mask[:, 0, 0] = False                     # k = 0 carries the conserved totals
    err = np.abs(S - want)[mask].max() / want[mask].max()
    tol = fp64_spectrum_tol(nx * ny, want[mask].max()) if precision == 0 else 1e-4
    say("S(k)", shape, "precision", precision, "err", err, "tol", tol)
    assert err < tol
    lat.lb_structure_factor(L.LB_SK_RESET, -1)
    S2, ns2 = lat.lb_structure_factor(L.LB_SK_READ, 0)
    assert ns2 == 0 and float(S2.abs().max()) == 0.0
    lat.close()


def test_ensemble_sample_is_batched_and_bitwise_per_replica():
    """One batched sample of replicas of different sizes equals sampling each alone, bit
    for bit, and the oracle's spectrum."""
    L = _L()
    cfgs = [W.single_phase(64, 32, kT=1e-5, seed=1), W.single_phase(128, 128, kT=2e-5, seed=2),
            dict(W.single_phase(16, 64, kT=1e-5, seed=3), replica=5), W.single_phase(256, 8, kT=1e-5, seed=4)]
    a = L.Lattice(cfgs, precision=2, structure_factor=True)
    b = L.Lattice(cfgs, precision=2, structure_factor=True)
    for _ in range(3):
        a.step(5)
        b.step(5)
        a.lb_structure_factor(L.LB_SK_SAMPLE, -1)
        for r in range(len(cfgs)):
            b.lb_structure_factor(L.LB_SK_SAMPLE, r)
    for r, c in enumerate(cfgs):
        Sa, na = a.lb_structure_factor(L.LB_SK_READ, r)
        Sb, nb = b.lb_structure_factor(L.LB_SK_READ, r)
        assert na == nb == 3
        assert torch.equal(Sa, Sb), r
    o = O.Oracle(cfgs[1])
    acc = np.zeros((9, 128, 65))
    for _ in range(3):
        o.step(5)
        acc += O.power_spectrum(o.moments())
    S1 = a.lb_structure_factor(L.LB_SK_READ, 1)[0].cpu().numpy()
    mask = np.ones_like(acc, dtype=bool)
    mask[:, 0, 0] = False
    err = np.abs(S1 - acc / 3)[mask].max() / (acc / 3)[mask].max()
    say("batched S(k) err", err)
    assert err < 1e-4
    a.close()
    b.close()


@pytest.mark.parametrize("every,first,steps", [(7, 5, 60), (300, 0, 700), (32, 64, 200)])
def test_sampling_inside_lb_step_equals_manual_sampling(every, first, steps):
    """lb_set_sampling: graphs of `every` steps plus a sample (every <= 256) and the eager
    path (every > 256) both equal stepping and sampling by hand, bit for bit."""
    L = _L()
    cfgs = [W.single_phase(64, 32, kT=1e-5, seed=8), W.single_phase(32, 32, kT=1e-5, seed=9)]
    a = L.Lattice(cfgs, precision=2, structure_factor=True)
    b = L.Lattice(cfgs, precision=2, structure_factor=True)
    a.lb_set_sampling(every, first)
    a.step(steps // 3)
    a.step(steps - steps // 3)
    t = 0
    times = [ts for ts in range(first, steps + 1, every) if ts > 0]
    for ts in times:
        b.step(ts - t)
        b.lb_structure_factor(L.LB_SK_SAMPLE, -1)
        t = ts
    b.step(steps - t)
    for r in range(2):
        Sa, na = a.lb_structure_factor(L.LB_SK_READ, r)
        Sb, nb = b.lb_structure_factor(L.LB_SK_READ, r)
        say("in-step sampling", every, first, steps, "samples", na, nb)
        assert na == nb == len(times)
        assert torch.equal(Sa, Sb)
        assert np.array_equal(a.moments(r), b.moments(r))
    a.lb_set_sampling(0)
    a.step(every + 1)
    assert a.lb_structure_factor(L.LB_SK_READ, 0)[1] == len(times)
    a.close()
    b.close()


SNAP_SHAPES = [(64, 64), (128, 32), (16384, 16), (16, 16384)]


@pytest.mark.parametrize("shape", SNAP_SHAPES, ids=[f"{a}x{b}" for a, b in SNAP_SHAPES])
@pytest.mark.parametrize("precision", [0, 2])
def test_radial_density_snapshot_matches_oracle(precision, shape):
    L = _L()
    nx, ny = shape
    cfg = W.spinodal(nx, ny, kT=1e-6, amp=1e-3, seed=21)
    lat = L.Lattice(cfg, precision=precision, structure_factor=True)
    ora = O.Oracle(cfg)
    lat.step(12)
    ora.step(12)
    out = lat.lb_structure_factor(L.LB_SK_SNAPSHOT, 0).cpu().numpy()
    mean, counts = O.radial_spectrum(ora.moments()[0])
    assert out.shape == (2, len(mean))
    assert np.array_equal(out[1], counts.astype(np.float64))
    err = np.abs(out[0] - mean).max() / mean.max()
    tol = fp64_spectrum_tol(nx * ny, mean.max()) if precision == 0 else 1e-4
    say("snapshot", shape, precision, "err", err, "tol", tol)
    assert err < tol
    lat.close()


def test_radial_snapshot_16384_plane_wave_closed_form():
    """The 16384^2 quench lattice in FP32-shifted storage: a density wave at (kx, ky) =
    (3, 4) puts |rho(+-k)|^2 = a^2 n / 4 into shell 5 and nothing elsewhere.

    Floor: the stored deviations from the rest state are of the wave's size, so their FP32
    rounding is ~1e-7 of the wave's power, and the FP32 transforms add ~2 x 3e-7 of it
    (measured 4.5e-8); gate 1e-6."""
    L = _L()
    nx = ny = 16384
    a = 0.02
    cfg = W.wave(W.quench_16384(), 3, 4, a)
    say("snapshot 16384^2 wave")
    lat = L.Lattice(cfg, precision=2, structure_factor=True)
    out = lat.lb_structure_factor(L.LB_SK_SNAPSHOT, 0).cpu().numpy()
    lat.close()
    nb = out.shape[1]
    assert nb == int(O.radial_shell(nx // 2, ny // 2, nx, ny)) + 1
    assert out[1].sum() == nx * ny - 1
    # the inner shells, counted by the oracle's shell function on a window around k = 0
    kk = np.arange(-12, 13)
    KX, KY = np.meshgrid(kk, kk)
    b = O.radial_shell(KX, KY, nx, ny)
    inner = np.bincount(b[(KX != 0) | (KY != 0)], minlength=12)[:11]
    assert np.array_equal(out[1][:11], inner.astype(np.float64))
    want = 2 * a * a * nx * ny / 4 / out[1][5]
    say("shell 5", out[0][5], "want", want, "others max", np.delete(out[0], 5).max())
    assert abs(out[0][5] / want - 1) < 1e-6
    assert np.delete(out[0], 5).max() < 1e-12 * want


# ------------------------------------------------------------------ full size, sampled


@pytest.mark.parametrize("precision", [2, 0])
def test_full_size_8192_sampled_parity(precision):
    """The bench workload (8192^2 single phase, autotuned tiles) in FP32-shifted storage and in
    the FP64 storage bench times beside it: one and two steps against the oracle on the full
    lattice, compared at sampled nodes (FP64: the absolute gate of the small FP64 cases)."""
    L = _L()
    cfg = W.single_phase_8192()
    lat = L.Lattice(cfg, precision=precision)
    ora = O.Oracle(cfg)
    rng = np.random.default_rng(0)
    idx = rng.integers(0, 8192 * 8192, size=200_000)
    for s in (1, 1):
        lat.step(s)
        ora.step(s)
        mg, _ = lat.lb_moments(0, True)
        mg = mg.reshape(9, -1)[:, torch.from_numpy(idx).to(mg.device)].cpu().numpy()
        mo = ora.moments().reshape(9, -1)[:, idx]
        if precision == 0:
            ok, err = abs_ok(mg, mo)
            say("8192^2 fp64 t=", ora.t, "abs err", err)
            assert ok
            continue
        scale = np.abs(mo - mo.mean(axis=1, keepdims=True)).max(axis=1)
        e = np.abs(mg - mo).max(axis=1) / scale
        say("8192^2 t=", ora.t, "err", e)
        assert e.max() < 1e-5
    t = lat.totals()
    assert abs(t[0] - 8192.0 * 8192.0) / (8192.0 * 8192.0) < 1e-9
    lat.close()


@pytest.mark.parametrize("shape,tile", [((1 << 24, 3), None), ((3, 1 << 24), "64,64")], ids=["widest", "tallest"])
def test_extreme_lattice_shapes_sampled(monkeypatch, shape, tile):
    """The widest lattice the ABI admits (nx = 2^24: a row of 9 nx FP64 values is the largest
    range a buffer descriptor addresses here) and a three-column lattice 2^24 rows tall, 50 M
    nodes each, noisy: two steps in FP32-shifted and FP64 storage against the oracle at
    sampled nodes, and exact mass conservation."""
    L = _L()
    if tile:
        monkeypatch.setenv("LBF_TILE", tile)
    nx, ny = shape
    cfg = W.wave(W.single_phase(nx, ny, kT=1e-5, seed=5), 3, 1, 1e-4, 1e-4, 0)
    ora = O.Oracle(cfg)
    ora.step(2)
    mo_all = ora.moments().reshape(9, -1)
    del ora
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.integers(0, nx * ny, size=200_000), [0, nx - 1, nx * ny - 1, nx * (ny - 1)]])
    mo = mo_all[:, idx]
    scale = np.abs(mo - mo.mean(axis=1, keepdims=True)).max(axis=1)
    for precision in (2, 0):
        say("extreme shape", nx, ny, "precision", precision)
        lat = L.Lattice(cfg, precision=precision)
        lat.step(1)
        lat.step(1)
        mg, _ = lat.lb_moments(0, True)
        mg = mg.reshape(9, -1)[:, torch.from_numpy(idx).to(mg.device)].cpu().numpy()
        t = lat.totals()
        assert lat.lb_status_flags() == (0, 2)
        lat.close()
        if precision == 0:
            err = np.abs(mg - mo).max(axis=1) / np.maximum(1.0, np.abs(mo).max(axis=1))
            say("  fp64 abs err", err.max())
            assert err.max() <= 2e-12
            assert abs(t[0] - nx * ny) / (nx * ny) < 1e-13
        else:
            e = np.abs(mg - mo).max(axis=1) / scale
            say("  fp32s err", e)
            assert e.max() < 5e-7
            assert abs(t[0] - nx * ny) / (nx * ny) < 1e-9


@pytest.mark.parametrize("precision", [2, 0])
def test_full_size_8192_structure_factor_sampled(precision):
    """One S(k) sample of the bench workload (8192^2 single phase, FP32-shifted storage, the
    batched launch bench.py times) after two steps against the oracle's |m_a(k)|^2 / n of its
    own moments at 36 k per mode: k = 0 (restored in FP64 by the column pass), kx = 1, the
    Nyquist column and row, and random k.  Gates: off k = 0, 1.5e-5 of the mode's variance (the
    mean of S_a over k != 0; the FP32 transforms' rounding, measured <= 4.5e-6).  At k = 0, relative to max(S_a(0), variance): 1e-5 for the
    conserved rho, jx, jy (their totals are exact on both sides; the FP32 transform rounds X(0)
    by ~ eps32 sqrt(log2 n) |m'|_2, ~6e-7 of the variance in S_a(0)); 1e-3 for the other modes,
    whose X(0) = sum_r m_a(r) adds the FP32 trajectory's per-node differences (1.6e-7 of the
    range after two steps) coherently, up to ~ sqrt(n) 1.6e-7 ~ 1e-2 in the worst case.
    FP64 storage (FP64 transforms): the trajectory agrees with the oracle to ~1e-15 per node, so
    off k = 0 S_a differs by ~ 2 sqrt(var) 1e-15 (~1e-12 of the variance) and at k = 0 by at most
    ~ 2 |X(0)| n 1e-15 / n; gates 1e-9 of the variance off k = 0 and 1e-7 at k = 0."""
    L = _L()
    cfg = W.single_phase_8192()
    nx, ny = cfg["nx"], cfg["ny"]
    lat = L.Lattice(cfg, precision=precision, structure_factor=True)
    ora = O.Oracle(cfg)
    lat.step(2)
    ora.step(2)
    lat.lb_structure_factor(L.LB_SK_SAMPLE, -1)
    S, ns = lat.lb_structure_factor(L.LB_SK_READ, 0)
    assert ns == 1
    rng = np.random.default_rng(11)
    kxs = [0, 1, nx // 2] + [int(v) for v in rng.integers(2, nx // 2, size=3)]
    kys = [0, 1, ny // 2] + [int(v) for v in rng.integers(2, ny, size=3)]
    px = [a for a in kxs for b in kys]
    py = [b for a in kxs for b in kys]
    got = S[:, torch.tensor(py, device=S.device), torch.tensor(px, device=S.device)].cpu().numpy()
    del S
    lat.close()
    mo = ora.moments()
    del ora
    e0, err = np.zeros(9), np.zeros(9)
    for a in range(9):
        # off k = 0 from the centred field (the same |m_a(k)|^2 in exact arithmetic): the DFT of
        # the raw rho ~ 1 + drho carries ~ n eps of the constant's zero transform into X(k)
        want = np.concatenate([O.power_at(mo[a], px[:1], py[:1]),
                               O.power_at(mo[a] - mo[a].mean(), px[1:], py[1:])])
        var = mo[a].var()
        e0[a] = abs(got[a, 0] - want[0]) / max(want[0], var)
        err[a] = np.abs(got[a, 1:] - want[1:]).max() / var
        worst = np.argsort(-np.abs(got[a] - want))[:3]
        say("8192^2 S(k) precision", precision, "mode", a, "k=0 rel err", e0[a], "err / var", err[a],
            "worst (kx, ky, got, want):", [(px[i], py[i], float(got[a, i]), float(want[i])) for i in worst])
    if precision == 0:
        assert e0.max() < 1e-7 and err.max() < 1e-9
        return
    assert e0[:3].max() < 1e-5 and e0[3:].max() < 1e-3
    assert err.max() < 1.5e-5


def test_full_size_8192_equipartition_transient():
    """The fluctuation spectrum of the bench workload at full size (8192^2, FP32-shifted, the
    launch bench.py times): one S(k) sample 200 steps after its quiescent start against the
    exact linear-theory covariance of that moment, sum_{s<200} M^s Q M^{H s} with the k = 0
    noise (the stationary one is still far away for the slow modes), at 60,000 random k of the
    half plane: per mode the k-summed ratio within 2% (standard error ~0.5%)."""
    L = _L()
    cfg = W.single_phase_8192()
    nx, ny, t = cfg["nx"], cfg["ny"], 200
    lat = L.Lattice(cfg, precision=2, structure_factor=True)
    lat.step(t)
    lat.lb_structure_factor(L.LB_SK_SAMPLE, -1)
    S, ns = lat.lb_structure_factor(L.LB_SK_READ, 0)
    assert ns == 1
    rng = np.random.default_rng(21)
    nh = nx // 2 + 1
    flat = rng.choice(ny * nh, size=60_000, replace=False)
    iy, ix = flat // nh, flat % nh
    keep = ((ix != 0) | (iy != 0)) & ~((ix == nx // 2) & (iy == 0)) & ~((ix == 0) & (iy == ny // 2))
    iy, ix = iy[keep], ix[keep]
    got = S[:, torch.from_numpy(iy).to(S.device), torch.from_numpy(ix).to(S.device)].cpu().numpy()
    del S
    lat.close()
    lam = th.relaxation_rates(cfg["tau_bulk"], cfg["tau_shear"], cfg["tau_q"], cfg["tau_eps"])
    cs2 = th.sound_speed2(cfg["rho0"], cfg["c0sq"], cfg["A"], cfg["B"], cfg["rhoc"])
    G = th.transient_covariance_batch(2 * np.pi * ix / nx, 2 * np.pi * iy / ny, lam, cs2, cfg["rho0"],
                                      cfg["kappa"], cfg["kT"], t)
    Gd = np.real(np.diagonal(G, axis1=1, axis2=2))
    r = got.sum(axis=1) / Gd.sum(axis=0)
    say("8192^2 t=200 S/G(t) per mode", np.round(r, 4))
    assert np.abs(r - 1).max() < 0.02


def test_full_size_8192_structure_factor_over_20k_steps():
    """The 8192^2 single-phase workload as stated (FP32-shifted, the bench's launch): 20,000
    steps with S(k) of all nine modes sampled inside lb_step every 20 steps from step 2000
    (901 samples, FP64 accumulators), against the linear model's covariance averaged over the
    same sampling times (eq. lb-lang-ft from rest with the k = 0 noise; the slow hydrodynamic
    modes at small k are still equilibrating and are included exactly), at 60,000 random k of
    the half plane.  Per mode the k-summed ratio within 1%; per |k| shell of width 0.25 with at
    least 200 points within 2.5% (the slowest shell holds ~300 points whose samples decorrelate
    over ~300 steps: ~0.8% one sigma)."""
    L = _L()
    cfg = W.single_phase_8192()
    nx, ny = cfg["nx"], cfg["ny"]
    say("8192^2, 20k steps, S(k) every 20 from 2000")
    lat = L.Lattice(cfg, precision=2, structure_factor=True)
    lat.lb_set_sampling(20, 2000)
    lat.step(20000)
    S, ns = lat.lb_structure_factor(L.LB_SK_READ, 0)
    f, t = lat.lb_status_flags()
    assert ns == 901 and t == 20000 and f == 0
    rng = np.random.default_rng(23)
    nh = nx // 2 + 1
    flat = rng.choice(ny * nh, size=60_000, replace=False)
    iy, ix = flat // nh, flat % nh
    keep = ((ix != 0) | (iy != 0)) & ~((ix == nx // 2) & (iy == 0)) & ~((ix == 0) & (iy == ny // 2))
    iy, ix = iy[keep], ix[keep]
    got = S[:, torch.from_numpy(iy).to(S.device), torch.from_numpy(ix).to(S.device)].cpu().numpy()
    del S
    lat.close()
    lam = th.relaxation_rates(cfg["tau_bulk"], cfg["tau_shear"], cfg["tau_q"], cfg["tau_eps"])
    cs2 = th.sound_speed2(cfg["rho0"], cfg["c0sq"], cfg["A"], cfg["B"], cfg["rhoc"])
    kx, ky = 2 * np.pi * ix / nx, 2 * np.pi * np.where(iy > ny // 2, iy - ny, iy) / ny
    G = th.sampled_mean_covariance_batch(kx, ky, lam, cs2, cfg["rho0"], cfg["kappa"], cfg["kT"], 2000, 20, ns)
    Gd = np.real(np.diagonal(G, axis1=1, axis2=2)).T
    r = got.sum(axis=1) / Gd.sum(axis=1)
    say("8192^2 20k steps k-summed S / G per mode", np.round(r, 5))
    assert np.abs(r - 1).max() < 0.01
    kmag = np.sqrt(kx ** 2 + ky ** 2)
    worst = 0.0
    for lo in np.arange(0.0, 4.5, 0.25):
        sel = (kmag >= lo) & (kmag < lo + 0.25)
        if sel.sum() < 200:
            continue
        rs = got[:, sel].sum(axis=1) / Gd[:, sel].sum(axis=1)
        worst = max(worst, np.abs(rs - 1).max())
        assert np.abs(rs - 1).max() < 0.025, (lo, sel.sum(), rs)
    say("worst |k| shell deviation", worst)


def test_full_size_16384_quench_growth_follows_linear_theory():
    """The 16384^2 quench (the bench's quench_16384 workload at full size, FP32-shifted) after 50 steps,
    radially binned: in shells across the unstable band and beyond it, S(t) = S(0)
    <|[M(k)^t v(k)]_rho|^2> + <G_rho,rho(k, t)> over the shell's k, with v(k) the linearised
    Table II of a pure density perturbation (the initial state) and G the noise's transient
    covariance (eq. lb-lang-ft).  Gate 3%: the noise part's sampling error is ~0.7% of the
    total and the nonlinear corrections at this amplitude (delta rho ~ 0.02) ~0.7%.  The shell
    counts equal the exact integer enumeration."""
    L = _L()
    cfg = W.quench_16384()
    nx, ny, t = cfg["nx"], cfg["ny"], 50
    lat = L.Lattice(cfg, precision=2, structure_factor=True)
    s0 = lat.lb_structure_factor(L.LB_SK_SNAPSHOT, 0).cpu().numpy()
    lat.step(t)
    s1 = lat.lb_structure_factor(L.LB_SK_SNAPSHOT, 0).cpu().numpy()
    lat.close()
    lam = th.relaxation_rates(cfg["tau_bulk"], cfg["tau_shear"], cfg["tau_q"], cfg["tau_eps"])
    cs2 = th.sound_speed2(cfg["rho0"], cfg["c0sq"], cfg["A"], cfg["B"], cfg["rhoc"])
    assert cs2 < 0
    shells = [200, 500, 900, 1300, 1700, 2400]
    B = max(shells) + 2
    kk = np.arange(-B, B + 1)
    KX, KY = np.meshgrid(kk, kk)
    b = O.radial_shell(KX, KY, nx, ny)
    for sh in shells:
        sel = b == sh
        assert sel.sum() == s1[1][sh] == s0[1][sh]
        kx, ky = KX[sel], KY[sel]
        half = (ky > 0) | ((ky == 0) & (kx > 0))      # |g|^2 and G are even in k
        qx, qy = 2 * np.pi * kx[half] / nx, 2 * np.pi * ky[half] / ny
        G, P = th.transient_covariance_batch(qx, qy, lam, cs2, cfg["rho0"], cfg["kappa"], cfg["kT"], t, power=True)
        v = np.stack([th.equilibrium_jacobian(a, c, cs2, cfg["rho0"], cfg["kappa"])[:, 0] for a, c in zip(qx, qy)])
        g2 = np.abs(np.einsum("kij,kj->ki", P, v)[:, 0]) ** 2
        want = s0[0][sh] * g2.mean() + G[:, 0, 0].real.mean()
        say("quench shell", sh, "|k| =", round(2 * np.pi * sh / nx, 3), "growth", round(g2.mean(), 3),
            "S(t) / want", s1[0][sh] / want)
        assert abs(s1[0][sh] / want - 1) < 0.03


def test_quench_16384_snapshots_fp32s_against_fp64_over_5000_steps():
    """The 16384^2 quench at the workload's snapshot cadence (the radially binned density
    spectrum every 1000 steps) for its first 5000 steps, FP32-shifted against FP64 storage on
    the GPU (FP64 being pinned to the oracle at 2e-12): at every snapshot, in the shells that
    hold 99% of the power, the relative difference of the shell means within 6e-5, ~3x the
    measured (1.4e-6 after 1000 steps, growing to 2.0e-5 after 5000 as the domains coarsen and
    the spectral peak moves from shell 480 to 112), and the same integer shell counts."""
    L = _L()
    cfg = W.quench_16384()
    snaps = {}
    for precision in (2, 0):
        lat = L.Lattice(cfg, precision=precision, structure_factor=True)
        out = []
        for _ in range(5):
            lat.step(1000)
            out.append(lat.lb_structure_factor(L.LB_SK_SNAPSHOT, 0).cpu().numpy())
        f, t = lat.lb_status_flags()
        lat.close()
        assert f == 0 and t == 5000
        snaps[precision] = out
    for i, (a, b) in enumerate(zip(snaps[2], snaps[0])):
        assert np.array_equal(a[1], b[1])
        order = np.argsort(-b[0])
        cum = np.cumsum(b[0][order] * b[1][order]) / np.sum(b[0] * b[1])
        top = order[: int(np.searchsorted(cum, 0.99)) + 1]
        rel = np.abs(a[0][top] / b[0][top] - 1)
        say("quench step", 1000 * (i + 1), "shells", len(top), "peak shell", int(order[0]),
            "max rel diff FP32s vs FP64", rel.max())
        assert rel.max() < 6e-5


FULL_GATES = {"slab_2048": 2e-5, "quench_16384": 8e-7}   # ~3x the measured FP32-shifted errors


@pytest.mark.parametrize("precision", [2, 0])
@pytest.mark.parametrize("name", ["slab_2048", "quench_16384"])
def test_full_size_two_phase_workloads_sampled(name, precision):
    """The 2048^2 slab and the 16384^2 spinodal quench at full size, in the launch configuration
    bench.py times (FP32-shifted, autotuned tiles): two steps against the oracle at 200,000
    sampled nodes, whose moments the oracle forms there from its pre-collision populations.
    Gates ~3x the measured errors (slab 7.3e-6: its bulk phases hold O(0.5) deviations from
    the rest state; quench 2.7e-7); FP64 storage (autotuned FP64 tiles) at the absolute gate of
    the small FP64 cases."""
    L = _L()
    cfg = getattr(W, name)()
    nx, ny = cfg["nx"], cfg["ny"]
    rng = np.random.default_rng(3)
    idx = rng.integers(0, nx * ny, size=200_000)
    lat = L.Lattice(cfg, precision=precision)
    lat.step(2)
    mg, _ = lat.lb_moments(0, True)
    mg = mg.reshape(9, -1)[:, torch.from_numpy(idx).to(mg.device)].cpu().numpy()
    lat.close()
    ora = O.Oracle(cfg)
    ora.step(2)
    T = O.tables()[0]
    mo = T @ ora.f.reshape(9, -1)[:, idx]
    del ora
    if precision == 0:
        ok, err = abs_ok(mg, mo)
        say(name, "full size fp64, 2 steps, abs err", err)
        assert ok
        return
    scale = np.abs(mo - mo.mean(axis=1, keepdims=True)).max(axis=1)
    e = np.abs(mg - mo).max(axis=1) / scale
    say(name, "full size, 2 steps, err", e)
    assert e.max() < FULL_GATES[name]


def test_slab_2048_at_its_length_fp32s_against_fp64():
    """The two-phase slab workload as stated (2048^2, kT = 1e-6, 10,000 steps) in FP32-shifted,
    plain FP32 and FP64 storage on the GPU (FP64 being pinned to the oracle at 2e-12): the
    FP32-shifted moments against FP64 after the full run within 1.2e-4 of each moment's range
    (measured 4.0e-5 for the density, 8e-6 for j_x and j_y; plain FP32 the same, 4.0e-5: after
    10k noisy steps the FP32 normals, not the storage, set the error), and the physics of
    Sec. II.A on the FP64 run: bulk densities 1 +- sqrt(-A/B) = 1.5 / 0.5 within 2e-3, the
    x-averaged lower wall a tanh of half-width sqrt(-2 kappa / A) = 2 (eq. interf-width) within
    5%."""
    from scipy.optimize import curve_fit
    L = _L()
    cfg = W.slab_2048()
    res = {}
    for prec in ("fp64", "fp32s", "fp32"):
        say("slab_2048 10k steps", prec)
        lat = L.Lattice(cfg, precision=prec)
        lat.step(10000)
        m, _ = lat.lb_moments(0, True)
        assert lat.lb_status_flags() == (0, 10000)
        lat.close()
        res[prec] = m[:3].cpu().numpy()
        del m
    ref = res["fp64"]
    rng_ = [np.abs(ref[a] - ref[a].mean()).max() for a in range(3)]
    e32s = [np.abs(res["fp32s"][a] - ref[a]).max() / rng_[a] for a in range(3)]
    e32 = [np.abs(res["fp32"][a] - ref[a]).max() / rng_[a] for a in range(3)]
    say("slab_2048 10k steps: fp32s err / range", e32s, "plain fp32", e32)
    assert max(e32s) < 1.2e-4 and max(e32) < 1e-3
    rho = ref[0].mean(axis=1)
    ny = rho.size
    liquid, vapour = rho[ny // 2 - 50: ny // 2 + 50].mean(), np.r_[rho[:50], rho[-50:]].mean()
    y = np.arange(ny)
    y1 = ny / 4 - 0.5
    sel = np.abs(y - y1) < 20
    p, _ = curve_fit(lambda yy, a, b, c, w: a + b * np.tanh((yy - c) / w), y[sel], rho[sel], p0=[1.0, 0.5, y1, 2.0])
    say("slab_2048 bulk", liquid, vapour, "tanh fit (mean, half-contrast, centre, half-width)", p)
    assert abs(liquid - 1.5) < 2e-3 and abs(vapour - 0.5) < 2e-3
    assert abs(p[3] / 2.0 - 1) < 0.05


@pytest.mark.parametrize("precision", [2, 0])
def test_full_size_ensemble_sampled_replicas(precision):
    """The bench's 336-replica ensemble (256 x 128^2, 64 x 256^2, 16 x 512^2, kT over two
    decades) in one launch, FP32-shifted and FP64: two steps against the oracle for the first
    and last replica of each size class."""
    L = _L()
    cfgs = W.ensemble_336()
    lat = L.Lattice(cfgs, precision=precision)
    lat.step(2)
    worst = 0.0
    for r in (0, 255, 256, 319, 320, 335):
        o = O.Oracle(cfgs[r])
        o.step(2)
        if precision == 0:
            ok, err = abs_ok(lat.moments(r), o.moments())
            say("ensemble fp64 replica", r, cfgs[r]["nx"], "kT", cfgs[r]["kT"], "abs err", err.max())
            assert ok
            continue
        e = rel_err(lat.moments(r), o.moments())
        say("ensemble replica", r, cfgs[r]["nx"], "kT", cfgs[r]["kT"], "err", e.max())
        worst = max(worst, e.max())
    lat.close()
    assert worst < 1e-5


# ------------------------------------------------------------------ equipartition on the GPU


def _unc_targets(cfg, kxv, kyv, mask, diagonal=False):
    lam = th.relaxation_rates(cfg["tau_bulk"], cfg["tau_shear"], cfg["tau_q"], cfg["tau_eps"])
    cs2 = th.sound_speed2(cfg["rho0"], cfg["c0sq"], cfg["A"], cfg["B"], cfg["rhoc"])
    Gu = np.full((9, len(kyv), len(kxv)), np.nan)
    Gp = np.full_like(Gu, np.nan)
    for iy, ky in enumerate(kyv):
        for ix, kx in enumerate(kxv):
            if not mask[iy, ix]:
                continue
            Gu[:, iy, ix] = np.diag(th.stationary_covariance_uncorrelated(
                kx, ky, lam, cs2, cfg["rho0"], cfg["kappa"], cfg["kT"], diagonal)).real
            Gp[:, iy, ix] = np.diag(th.equilibrium_correlations(kx, ky, cs2, cfg["rho0"], cfg["kappa"], cfg["kT"])).real
    return Gu, Gp


@pytest.mark.parametrize("noise", ["k0", "diagonal"])
@pytest.mark.parametrize("precision", [2, 0])
def test_equipartition_all_modes_within_one_percent(precision, noise):
    """S_a(k) of all nine modes from the GPU's FP64 S(k) accumulators equals the stationary
    covariance of the linear model driven by the noise the path uses (Xi(0), or its diagonal
    for the "ideal-gas-like" variant of Sec. IV at c_s^2 = 0.05, where Xi_49 is large) within 1%
    on average over k, and within sampling error per |k| shell; the paper's G(k)
    (eq. g-mat-yeo) is matched at small k."""
    L = _L()
    nx = ny = 64
    if noise == "k0":
        cfg = W.single_phase(nx, ny, kT=1e-5, seed=101 + precision)
    else:
        cfg = W.single_phase(nx, ny, kT=1e-5, seed=201 + precision, c0sq=0.0, A=0.05, noise="diagonal")
    lat = L.Lattice(cfg, precision=precision, structure_factor=True)
    lat.step(3000)
    lat.lb_structure_factor(L.LB_SK_RESET, 0)
    nsamp = 4000
    for _ in range(nsamp):
        lat.step(10)
        lat.lb_structure_factor(L.LB_SK_SAMPLE, 0)
    S, ns = lat.lb_structure_factor(L.LB_SK_READ, 0)
    S = S.cpu().numpy()
    f, _ = lat.lb_status_flags()
    lat.close()
    assert ns == nsamp and f == 0
    kyv = 2 * np.pi * np.fft.fftfreq(ny)
    kxv = 2 * np.pi * np.fft.rfftfreq(nx)
    KX, KY = np.meshgrid(kxv, kyv)
    mask = np.ones_like(KX, dtype=bool)
    mask[0, 0] = False
    undamped = ((np.abs(KX) == np.pi) & (KY == 0)) | ((KX == 0) & (np.abs(KY) == np.pi))
    mask &= ~undamped
    Gu, Gp = _unc_targets(cfg, kxv, kyv, mask, noise == "diagonal")
    ratio = S / Gu
    kmag = np.sqrt(KX ** 2 + KY ** 2)
    means = []
    for a in range(9):
        r = ratio[a][mask]
        means.append(r.mean())
        assert abs(r.mean() - 1) < 0.01, (a, r.mean())
        # shells of width 0.25: sampling error of a shell mean, with the 10-step sampling
        # interval well below the slowest correlation time only at small k
        for lo in np.arange(0.0, 4.5, 0.25):
            sel = mask & (kmag >= lo) & (kmag < lo + 0.25)
            if sel.sum() < 20:
                continue
            assert abs(ratio[a][sel].mean() - 1) < 0.05, (a, lo, ratio[a][sel].mean())
    small = mask & (kmag < 0.35)
    pg = [(S[a][small] / Gp[a][small]).mean() for a in range(9)]
    say("equipartition", noise, "precision", precision, "mean S/G_unc", np.round(means, 4), "S/G (|k|<0.35)", np.round(pg, 3))
    # the paper's G(k) at small k: the exact target meets it within 1% (deterministic) ...
    for a in range(3):
        assert np.abs(Gu[a][small] / Gp[a][small] - 1).max() < 0.01
    # ... and so does the data, within sampling error: ~18 independent k with |k| < 0.35
    # whose transverse momentum decorrelates over 250-1000 steps give ~2.5% (one sigma)
    for a in range(3):
        assert abs(pg[a] - 1) < 0.08


def _shell_means(R, kmag, mask, width=0.25):
    out = []
    for lo in np.arange(0.0, 4.5, width):
        sel = mask & (kmag >= lo) & (kmag < lo + width)
        if sel.sum():
            out.append((lo, R[:, sel].mean(axis=1)))
    return out


@pytest.mark.parametrize("precision", [2, 0])
def test_uncorrelated_noise_run_of_sec_VA_at_128(precision):
    """The uncorrelated-noise equilibration run of Sec. V.A (128^2, kappa = 0.03, c_s = 0.156,
    tau = 1, T = 1e-7, S(k) sampled inside lb_step).  S_a(k) follows the exact linear target
    G_unc (the stationary covariance driven by Xi(0)) within 1% per mode.  Against the paper's
    G(k): negligible errors for |k| < 0.8 (as the text says), momentum within its 10% at every
    |k|; the density error, however, grows to ~18% near |k| = 3 and ~28% at the zone corner,
    as G_unc / G predicts, where the text reports < 10%."""
    L = _L()
    nx = ny = 128
    cfg = W.uncorrelated_sec5a(nx, ny, kT=1e-7, seed=61 + precision)
    lat = L.Lattice(cfg, precision=precision, structure_factor=True)
    lat.lb_set_sampling(10, 15000)
    lat.step(15000 + 30000)
    S, ns = lat.lb_structure_factor(L.LB_SK_READ, 0)
    S = S.cpu().numpy()
    lat.close()
    assert ns == 3001
    kyv = 2 * np.pi * np.fft.fftfreq(ny)
    kxv = 2 * np.pi * np.fft.rfftfreq(nx)
    KX, KY = np.meshgrid(kxv, kyv)
    mask = np.ones_like(KX, dtype=bool)
    mask[0, 0] = False
    mask &= ~(((np.abs(KX) == np.pi) & (KY == 0)) | ((KX == 0) & (np.abs(KY) == np.pi)))
    Gu, Gp = _unc_targets(cfg, kxv, kyv, mask)
    kmag = np.sqrt(KX ** 2 + KY ** 2)
    for a in range(9):
        r = (S[a] / Gu[a])[mask]
        assert abs(r.mean() - 1) < 0.01, (a, r.mean())
    shells = _shell_means(S / Gp, kmag, mask)
    for lo, m in shells:
        say("E4 |k| >= %.2f S/G" % lo, np.round(m, 3))
    hydro = mask & (kmag < 0.8)
    assert np.abs(Gu[:, hydro] / Gp[:, hydro] - 1).max() < 0.025
    assert np.abs((S / Gp)[:, hydro].mean(axis=1) - 1).max() < 0.04
    for lo, m in shells:
        assert m[1] < 1.10 and m[2] < 1.10, (lo, m[1], m[2])
    dens = {round(lo, 2): m[0] for lo, m in shells}
    assert dens[3.0] > 1.12 and dens[4.25] > 1.2


# ------------------------------------------------------------------ spatially correlated noise


@pytest.mark.parametrize("precision", [0, 2])
def test_correlated_noise_parity(precision):
    """Exact Xi(k) noise: the GPU's FFT-filtered fields and step against the oracle's numpy-FFT
    fields and FP64 step, same Philox streams."""
    cfg = W.correlated_sec5a(32, 16, kT=1e-6, seed=12)
    cfg["replica"] = 3
    mg, mo = run_pair(cfg, precision, 120, chunks=2)
    e = rel_err(mg, mo)
    if precision == 0:
        ok, err = abs_ok(mg, mo)
        say("correlated fp64 abs err", err, "normalised", e)
        assert ok
    else:
        say("correlated fp32s err", e)
        assert e.max() < 7e-7


CN_SHAPES = [(8192, 16, 4), (16, 8192, 4), (2048, 2048, 2)]


@pytest.mark.parametrize("shape", CN_SHAPES, ids=[f"{a}x{b}" for a, b, _ in CN_SHAPES])
@pytest.mark.parametrize("precision", [2, 0])
def test_correlated_noise_parity_long_lines(precision, shape):
    """The correlated-noise filter at the bench's line lengths: 8192-point rows (one block per
    row) and columns (several adjacent columns per block for the 16 narrow ones), and a 2048^2
    lattice, on the bench's single-phase parameters with the exact Xi(k) noise, against the
    oracle's numpy-FFT fields and FP64 step.  FP32-shifted gate 9e-7 of the fluctuation range
    (measured 2.3e-7 to 3.0e-7): the fields go through FP32 transforms (rounding ~3e-7 of
    their scale) on top of FP32 normals (3e-6 per draw)."""
    nx, ny, steps = shape
    cfg = dict(W.single_phase_8192(), nx=nx, ny=ny, noise="correlated", seed=17)
    mg, mo = run_pair(cfg, precision, steps, chunks=2)
    e = rel_err(mg, mo)
    if precision == 0:
        ok, err = abs_ok(mg, mo)
        say("correlated", nx, ny, "fp64 abs err", err.max(), "normalised", e.max())
        assert ok
    else:
        say("correlated", nx, ny, "fp32s err", e)
        assert e.max() < 9e-7


def test_full_size_8192_correlated_noise_sampled():
    """The bench's correlated-noise leg at full size: the 8192^2 single-phase lattice with the
    exact Xi(k) noise, in FP32-shifted and FP64 storage and their autotuned launches, two steps
    against the oracle (numpy-FFT fields, FP64 step) at 200,000 sampled nodes.  Gates as for the
    long lines: 9e-7 of the fluctuation range (FP32-shifted), 2e-12 absolute (FP64)."""
    L = _L()
    cfg = dict(W.single_phase_8192(), noise="correlated", seed=17)
    rng = np.random.default_rng(5)
    idx = rng.integers(0, cfg["nx"] * cfg["ny"], size=200_000)
    ora = O.Oracle(cfg)
    ora.step(2)
    mo = O.tables()[0] @ ora.f.reshape(9, -1)[:, idx]
    del ora
    for precision in (2, 0):
        lat = L.Lattice(cfg, precision=precision)
        lat.step(2)
        mg, _ = lat.lb_moments(0, True)
        mg = mg.reshape(9, -1)[:, torch.from_numpy(idx).to(mg.device)].cpu().numpy()
        flags, t = lat.lb_status_flags()
        lat.close()
        assert flags == 0 and t == 2
        if precision == 0:
            ok, err = abs_ok(mg, mo)
            say("correlated 8192^2 fp64 abs err", err)
            assert ok
        else:
            scale = np.abs(mo - mo.mean(axis=1, keepdims=True)).max(axis=1)
            e = np.abs(mg - mo).max(axis=1) / scale
            say("correlated 8192^2 fp32s err", e)
            assert e.max() < 9e-7


CN_SMALL = [(4, 64, 6), (64, 4, 6), (4, 4, 8), (8, 2048, 3), (8, 4096, 3), (4096, 8, 3)]


@pytest.mark.parametrize("shape", CN_SMALL, ids=[f"{a}x{b}" for a, b, _ in CN_SMALL])
@pytest.mark.parametrize("precision", [2, 0])
def test_correlated_noise_parity_narrow_sides(precision, shape):
    """The filter's edge shapes: the smallest sides (4), a lattice whose mirror-pair columns
    all fit one drawing block (4 x 64), rows of a 4-row chunk (64 x 4), 2048-point columns
    of a narrow lattice, and 4096-point columns and rows (the compile-time-length
    transforms), against the oracle as above (same gates)."""
    nx, ny, steps = shape
    cfg = dict(W.single_phase_8192(), nx=nx, ny=ny, noise="correlated", seed=23)
    mg, mo = run_pair(cfg, precision, steps, chunks=1)
    e = rel_err(mg, mo)
    if precision == 0:
        ok, err = abs_ok(mg, mo)
        say("correlated", nx, ny, "fp64 abs err", err.max(), "normalised", e.max())
        assert ok
    else:
        say("correlated", nx, ny, "fp32s err", e)
        assert e.max() < 9e-7


def test_correlated_and_uncorrelated_replicas_in_one_handle():
    L = _L()
    cfgs = [W.correlated_sec5a(32, 32, kT=1e-6, seed=1), W.uncorrelated_sec5a(48, 40, kT=1e-7, seed=2),
            dict(W.correlated_sec5a(16, 64, kT=1e-6, seed=3), replica=2)]
    lat = L.Lattice(cfgs, precision=0)
    lat.step(70)
    for r, c in enumerate(cfgs):
        o = O.Oracle(c)
        o.step(70)
        ok, err = abs_ok(lat.moments(r), o.moments())
        say("mixed noise replica", r, err.max())
        assert ok
    lat.close()


@pytest.mark.parametrize("nx", [64, 128])
@pytest.mark.parametrize("precision", [2, 0])
def test_correlated_noise_equilibrates_to_paper_G_at_all_k(precision, nx):
    """The paper's headline (Sec. V.A, Fig. 3 parameters): with the exact Xi(k) all nine modes
    reach G(k) of eq. (g-mat-yeo) at every k -- here within 1% on average and 5% per shell."""
    L = _L()
    ny = nx
    cfg = W.correlated_sec5a(nx, ny, kT=1e-6, seed=77 + precision + nx)
    lat = L.Lattice(cfg, precision=precision, structure_factor=True)
    # burn-in and sampling interval grow with the slowest relaxation time, ~ (nx / 2 pi)^2 / nu
    burn, every, nsamp = (2000, 8, 3000) if nx == 64 else (8000, 20, 3000)
    lat.step(burn)
    lat.lb_structure_factor(L.LB_SK_RESET, 0)
    for _ in range(nsamp):
        lat.step(every)
        lat.lb_structure_factor(L.LB_SK_SAMPLE, 0)
    S, ns = lat.lb_structure_factor(L.LB_SK_READ, 0)
    S = S.cpu().numpy()
    lat.close()
    kyv = 2 * np.pi * np.fft.fftfreq(ny)
    kxv = 2 * np.pi * np.fft.rfftfreq(nx)
    KX, KY = np.meshgrid(kxv, kyv)
    cs2 = th.sound_speed2(cfg["rho0"], cfg["c0sq"], cfg["A"], cfg["B"], cfg["rhoc"])
    G = np.full_like(S, np.nan)
    for iy, ky in enumerate(kyv):
        for ix, kx in enumerate(kxv):
            if ix or iy:
                G[:, iy, ix] = np.diag(th.equilibrium_correlations(kx, ky, cs2, 1.0, cfg["kappa"], cfg["kT"])).real
    mask = np.ones_like(KX, dtype=bool)
    mask[0, 0] = False
    undamped = ((np.abs(KX) == np.pi) & (KY == 0)) | ((KX == 0) & (np.abs(KY) == np.pi))
    kmag = np.sqrt(KX ** 2 + KY ** 2)
    means = []
    for a in range(9):
        m = mask & ~undamped if a in (1, 2) else mask
        r = (S[a] / G[a])[m]
        means.append(r.mean())
        assert abs(r.mean() - 1) < 0.01, (a, r.mean())
        for lo in np.arange(0.0, 4.5, 0.25):
            sel = m & (kmag >= lo) & (kmag < lo + 0.25)
            if sel.sum() < 20:
                continue
            assert abs((S[a] / G[a])[sel].mean() - 1) < 0.05, (a, lo)
    say("correlated equipartition precision", precision, "mean S/G", np.round(means, 4))


# ------------------------------------------------------------------ capillary waves (Sec. V.B)


def _interface_heights(rho, half, windows):
    """h(x): where rho crosses `half` in each column, by linear interpolation between the two
    bracketing nodes, for a rising (lower wall) and a falling (upper wall) crossing."""
    out = []
    for lo, hi, rising in windows:
        r = rho[lo:hi]
        a, b = r[:-1], r[1:]
        cross = ((a - half) * (b - half) <= 0) & ((b > a) if rising else (b < a))
        assert bool(cross.any(dim=0).all())
        idx = torch.argmax(cross.to(torch.int32), dim=0)
        ra = a.gather(0, idx[None])[0]
        rb = b.gather(0, idx[None])[0]
        out.append(lo + idx.to(torch.float64) + (half - ra) / (rb - ra))
    return out


def test_capillary_full_size_and_cropped_parity():
    """The capillary run of Sec. V.B against the oracle: at full size (2048 x 400, every node)
    two steps, and a cropped copy (256 x 120, a 50-wide stripe) for 400 steps, in FP64 and
    FP32-shifted storage.  Gates: FP64 the absolute gate of the parity tests; FP32-shifted
    relative to the fluctuation range, ~3x the measured error (the vapour holds deviations of
    0.5 from the rest state rho0 = 1, as in the slab)."""
    for cfg, steps, tol32 in ((W.capillary(), 2, 6e-5), (W.capillary(256, 120, width=50, seed=9), 400, 9e-5)):
        for precision in (0, 2):
            mg, mo = run_pair(cfg, precision, steps)
            if precision == 0:
                ok, err = abs_ok(mg, mo)
                say("capillary", cfg["nx"], cfg["ny"], steps, "fp64 abs err", err.max())
                assert ok
            else:
                e = rel_err(mg, mo)
                say("capillary", cfg["nx"], cfg["ny"], steps, "fp32s err", e)
                assert e.max() < tol32


def test_capillary_height_spectrum_matches_oracle():
    """The height spectrum of Sec. V.B (eq. capill-static) computed by the oracle's definition
    (oracle.interface_heights: the rho = (rho_L + rho_V)/2 passage of each column, linearly
    interpolated; oracle.height_spectrum) from the GPU state and from the oracle's own state of
    the same cropped capillary run (256 x 120, 600 steps): equal to 1e-9 of the largest |h(k)|^2
    in FP64 storage (measured 5e-12) and to 2.5e-4 of it in FP32-shifted storage (measured
    7.9e-5); and the torch extraction that the
    long capillary run uses gives the oracle's h(x) on the GPU state to 1e-12."""
    L = _L()
    cfg = W.capillary(256, 120, width=50, seed=4)
    ora = O.Oracle(cfg)
    ora.step(600)
    mo = ora.moments()
    walls = (((15, 60), True), ((60, 105), False))
    ho = [O.interface_heights(mo[0], 0.75, r, up) for r, up in walls]
    So = [O.height_spectrum(h) for h in ho]
    for precision, tol in ((0, 1e-9), (2, 2.5e-4)):
        lat = L.Lattice(cfg, precision=precision)
        lat.step(600)
        m, _ = lat.lb_moments(0, True)
        lat.close()
        rho = m[0].cpu().numpy()
        hg = [O.interface_heights(rho, 0.75, r, up) for r, up in walls]
        Sg = [O.height_spectrum(h) for h in hg]
        for a, b in zip(Sg, So):
            err = np.abs(a - b).max() / b.max()
            say("capillary spectrum precision", precision, "err / max", err)
            assert err < tol
        ht = _interface_heights(m[0], 0.75, ((15, 60, True), (60, 105, False)))
        for a, b in zip(ht, hg):
            assert np.abs(a.cpu().numpy() - b).max() < 1e-12


def test_capillary_spectrum_sec_VB():
    """The capillary run of Sec. V.B (2048 x 400, a 180-wide liquid stripe, rho_L = 1,
    rho_V = 0.5, beta = 0.04, kappa = 0.03, T = 1e-7, uncorrelated noise at the local density):
    the height h(x) of the rho = (rho_L + rho_V)/2 contour of both walls has <|h(k)|^2> =
    kT / (sigma k^2) (eq. capill-static, sigma of eq. surf-tension) within 15% for
    0.025 <= k < 0.39 (the text: well described for k <~ 0.2), here without the Galilean
    corrections the paper adds (reading R4); larger k deviate upwards, the longest waves
    (compressible stripe, slow relaxation) stay below."""
    import math
    L = _L()
    cfg = W.capillary()
    nx, ny = cfg["nx"], cfg["ny"]
    sigma = th.surface_tension(0.03, 0.04, 1.0, 0.5)
    lat = L.Lattice(cfg, precision="fp32s")
    m = torch.empty((9, ny, nx), dtype=torch.float64, device="cuda")
    lat.step(50000)
    acc = torch.zeros(nx // 2 + 1, dtype=torch.float64, device="cuda")
    ns = 0
    for _ in range(7000):
        lat.step(50)
        L._check("lb_moments", L.lib().lb_moments(lat._h, 0, m.data_ptr(), None))
        for h in _interface_heights(m[0], 0.75, ((40, 200, True), (200, 360, False))):
            hk = torch.fft.rfft(h - h.mean()) / math.sqrt(nx)
            acc += hk.real ** 2 + hk.imag ** 2
            ns += 1
    flags, _ = lat.lb_status_flags()
    lat.close()
    assert flags == 0
    S = (acc / ns).cpu().numpy()
    k = 2 * np.pi * np.arange(nx // 2 + 1) / nx
    ratio = S[1:] * sigma * k[1:] ** 2 / cfg["kT"]
    bands = {}
    for lo, hi in [(1, 8), (8, 16), (16, 32), (32, 64), (64, 128), (128, 256), (256, 512), (512, 1025)]:
        bands[lo] = ratio[lo - 1:hi - 1].mean()
        say("capillary m in [%d, %d), k in [%.3f, %.3f): <|h|^2> sigma k^2 / kT = %.3f"
            % (lo, hi, k[lo], k[min(hi, nx // 2)], bands[lo]))
    for lo in (8, 16, 32, 64):
        assert abs(bands[lo] - 1) < 0.15, (lo, bands[lo])
    assert bands[512] > 1.3 and bands[1] < 0.85


# ------------------------------------------------------------------ ensemble equipartition


def test_ensemble_workload_averaged_structure_factor_over_20k_steps():
    """The 336-replica ensemble workload as stated (256 x 128^2, 64 x 256^2, 16 x 512^2, kT
    log-uniform in [1e-6, 1e-4], FP32-shifted, one handle): 20,000 steps with S(k) of every
    replica sampled inside lb_step every 20 steps from step 5000 (751 samples).  Per size class
    the ensemble average of S_a(k) / kT_r against the linear model's covariance at unit kT,
    averaged over the same sampling times from rest (eq. lb-lang-ft with the k = 0 noise; the
    target is linear in kT, and the slow modes of the 512^2 replicas are still equilibrating and
    are included exactly): per mode the k-summed ratio within 1%; per |k| shell of width 0.25
    holding at least 200 points within 2.5% (the 512^2 class's lowest shells: ~480 effective
    samples per k over 16 replicas, ~0.3% one sigma).  All k of the 128^2 and 256^2 half
    planes, 30,000 random k of the 512^2 one."""
    L = _L()
    cfgs = W.ensemble_336()
    lat = L.Lattice(cfgs, precision="fp32s", structure_factor=True)
    lat.lb_set_sampling(20, 5000)
    lat.step(20000)
    f, t = lat.lb_status_flags()
    assert f == 0 and t == 20000
    c0 = cfgs[0]
    lam = th.relaxation_rates(c0["tau_bulk"], c0["tau_shear"], c0["tau_q"], c0["tau_eps"])
    cs2 = th.sound_speed2(c0["rho0"], c0["c0sq"], c0["A"], c0["B"], c0["rhoc"])
    rng = np.random.default_rng(29)
    for side in (128, 256, 512):
        members = [r for r, c in enumerate(cfgs) if c["nx"] == side]
        acc = None
        for r in members:
            S, ns = lat.lb_structure_factor(L.LB_SK_READ, r)
            assert ns == 751
            v = S / cfgs[r]["kT"]
            acc = v if acc is None else acc + v
        Sm = (acc / len(members)).cpu().numpy()
        nh = side // 2 + 1
        flat = np.arange(side * nh) if side < 512 else rng.choice(side * nh, size=30_000, replace=False)
        iy, ix = flat // nh, flat % nh
        keep = ((ix != 0) | (iy != 0)) & ~((ix == side // 2) & (iy == 0)) & ~((ix == 0) & (iy == side // 2))
        iy, ix = iy[keep], ix[keep]
        got = Sm[:, iy, ix]
        kx = 2 * np.pi * ix / side
        ky = 2 * np.pi * np.where(iy > side // 2, iy - side, iy) / side
        G = th.sampled_mean_covariance_batch(kx, ky, lam, cs2, c0["rho0"], c0["kappa"], 1.0, 5000, 20, 751)
        Gd = np.real(np.diagonal(G, axis1=1, axis2=2)).T
        ratio = got.sum(axis=1) / Gd.sum(axis=1)
        say("ensemble", len(members), "x", side, "^2: k-summed S / (kT G) per mode", np.round(ratio, 5))
        assert np.abs(ratio - 1).max() < 0.01
        kmag = np.sqrt(kx ** 2 + ky ** 2)
        worst = 0.0
        for lo in np.arange(0.0, 4.5, 0.25):
            sel = (kmag >= lo) & (kmag < lo + 0.25)
            if sel.sum() < 200:
                continue
            rs = got[:, sel].sum(axis=1) / Gd[:, sel].sum(axis=1)
            worst = max(worst, np.abs(rs - 1).max())
            assert np.abs(rs - 1).max() < 0.025, (side, lo, sel.sum(), rs)
        say("ensemble", side, "^2 worst |k| shell deviation", worst)
    lat.close()


def test_ensemble_size_class_equipartition():
    """The ensemble workload's 128^2 size class (256 replicas, kT log-uniform in [1e-6, 1e-4],
    each with its own Philox stream): S(k) of all replicas sampled together inside lb_step;
    the per-class mean of S_a(k) / G_unc,aa(k; kT_r) (the exact target scales with kT in the
    linear model) is 1 within 0.5% for every mode, and the replicas agree with each other
    (the spread of the per-replica means is the sampling error's, not a kT trend)."""
    L = _L()
    reps = [r for r in W.ensemble_336() if r["nx"] == 128]
    assert len(reps) == 256
    lat = L.Lattice(reps, precision="fp32s", structure_factor=True)
    burn, every, nsamp = 16000, 20, 500
    lat.lb_set_sampling(every, burn)
    lat.step(burn + every * (nsamp - 1))
    nx = ny = 128
    kyv = 2 * np.pi * np.fft.fftfreq(ny)
    kxv = 2 * np.pi * np.fft.rfftfreq(nx)
    KX, KY = np.meshgrid(kxv, kyv)
    mask = np.ones_like(KX, dtype=bool)
    mask[0, 0] = False
    mask &= ~(((np.abs(KX) == np.pi) & (KY == 0)) | ((KX == 0) & (np.abs(KY) == np.pi)))
    unit = dict(reps[0], kT=1.0)
    Gu, _ = _unc_targets(unit, kxv, kyv, mask)
    per = np.zeros((len(reps), 9))
    for r, c in enumerate(reps):
        S, ns = lat.lb_structure_factor(L.LB_SK_READ, r)
        assert ns == nsamp
        ratio = S.cpu().numpy() / (Gu * c["kT"])
        per[r] = [ratio[a][mask].mean() for a in range(9)]
    f, _ = lat.lb_status_flags()
    lat.close()
    assert f == 0
    mean = per.mean(axis=0)
    say("ensemble 128^2 class: mean S/G_unc", np.round(mean, 4), "replica spread", np.round(per.std(axis=0), 4))
    assert np.abs(mean - 1).max() < 0.005
    # no dependence on kT across two decades: compare the low- and high-kT halves
    order = np.argsort([c["kT"] for c in reps])
    lo, hi = per[order[:128]].mean(axis=0), per[order[128:]].mean(axis=0)
    assert np.abs(lo - hi).max() < 0.01
