"""Python access to the FP64 CPU oracle (oracle/lbo.c) and its S(k) measurement.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg.  The product library never loads it.

The oracle state is the pre-collision population array f[9][ny][nx] (FP64), i.e. the
delta-m(t) of eq. (lb-lang-ft) of arXiv:1009.0254 after a moment transform.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbo.c")
LIB = os.path.join(HERE, "liblbo.so")

INIT_KINDS = {"uniform": 0, "slab": 1, "random": 2, "wave": 3}


class LboParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("rho0", ctypes.c_double), ("rhoc", ctypes.c_double),
        ("A", ctypes.c_double), ("B", ctypes.c_double),
        ("kappa", ctypes.c_double), ("c0sq", ctypes.c_double),
        ("tau_bulk", ctypes.c_double), ("tau_shear", ctypes.c_double),
        ("tau_q", ctypes.c_double), ("tau_eps", ctypes.c_double),
        ("kT", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("replica", ctypes.c_uint32),
        ("init_kind", ctypes.c_int32),
        ("noise_kind", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("init_arg", ctypes.c_double * 6),
    ]


NOISE_KINDS = {"k0": 0, "correlated": 1, "diagonal": 2}
# counter word 1 of the white fields behind the correlated noise: replica | 2^31
CORRELATED_STREAM = 0x80000000


def build(force: bool = False) -> str:
    """Compile oracle/lbo.c into oracle/liblbo.so with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER(LboParams)
        dp = ctypes.POINTER(ctypes.c_double)
        L.lbo_init.argtypes = [P, dp]
        L.lbo_step.argtypes = [P, dp, ctypes.c_int64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int64)]
        L.lbo_moments.argtypes = [P, dp, dp]
        L.lbo_stencils.argtypes = [P, dp, dp, dp, dp]
        L.lbo_equilibrium.argtypes = [P] + [ctypes.c_double] * 6 + [dp]
        L.lbo_pressure.argtypes = [P, ctypes.c_double]
        L.lbo_pressure.restype = ctypes.c_double
        L.lbo_sound_speed_sq.argtypes = [P, ctypes.c_double]
        L.lbo_sound_speed_sq.restype = ctypes.c_double
        L.lbo_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.lbo_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, dp]
        L.lbo_normals_batch.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, dp]
        L.lbo_noise_samples.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                        ctypes.c_int64, dp]
        L.lbo_tables.argtypes = [dp, dp, dp, dp]
        L.lbo_step_fields.argtypes = [P, dp, ctypes.c_uint64, dp, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(cfg: dict) -> LboParams:
    """Oracle parameter struct from a workload dict (see paper_1009_0254_amd.workloads)."""
    p = LboParams()
    p.nx, p.ny = int(cfg["nx"]), int(cfg["ny"])
    p.rho0 = cfg.get("rho0", 1.0)
    p.rhoc = cfg.get("rhoc", 1.0)
    p.A, p.B, p.kappa = cfg["A"], cfg["B"], cfg["kappa"]
    p.c0sq = cfg.get("c0sq", 1.0 / 3.0)
    p.tau_bulk, p.tau_shear = cfg["tau_bulk"], cfg["tau_shear"]
    p.tau_q, p.tau_eps = cfg.get("tau_q", 1.0), cfg.get("tau_eps", 1.0)
    p.kT = cfg["kT"]
    p.seed = int(cfg.get("seed", 1))
    p.replica = int(cfg.get("replica", 0))
    p.init_kind = INIT_KINDS[cfg.get("init", "uniform")]
    p.noise_kind = NOISE_KINDS[cfg.get("noise", "k0")]
    args = list(cfg.get("init_arg", [])) + [0.0] * 6
    for k in range(6):
        p.init_arg[k] = float(args[k])
    return p


def correlated_noise_fields(cfg: dict, t: int):
    """xi_4(r), xi_9(r) with <xi_a(k) xi_b(-k)> = Xi_ab(k) of eq. (noise-yeo) for a, b in {4, 9},
    built in Fourier space as Sec. IV (last paragraph) describes.

    At every lattice k: xi(k) = L(k) nu(k), with L(k) the lower Cholesky factor of the (4,9)
    block of Xi(k) at the homogeneous state (rho0, c_s^2(rho0)), c_s^2(k) = c_s^2 + rho0 kappa k^2
    and k^2 minus the App. B Laplacian symbol (eq. sound-speed-k), and nu(k) unit Gaussians with
    nu(-k) = conj(nu(k)) so that the fields are real: complex (g0 + i g1) / sqrt(2) for nu_4 and
    (g2 + i g3) / sqrt(2) for nu_9 where k != -k, real g0 and g1 at the four points k = -k.
    The pair k, -k takes the g's of the Philox block of the one with the smaller index
    ky nx + kx (counter (that index, replica | 2^31, t)), the other member its conjugate.
    Then one transform back to real space: xi(r) = n^-1/2 sum_k exp(-i k.r) xi(k), done for
    both fields at once as xi_4 + i xi_9 = n^-1/2 FFT(xi_4(k) + i xi_9(k))."""
    nx, ny = int(cfg["nx"]), int(cfg["ny"])
    n = nx * ny
    rep = int(cfg.get("replica", 0)) | CORRELATED_STREAM
    z = normals_batch(int(cfg.get("seed", 1)), rep, t, n)
    ix = np.arange(nx)[None, :]
    iy = np.arange(ny)[:, None]
    idx = iy * nx + ix
    midx = ((ny - iy) % ny) * nx + (nx - ix) % nx
    canon = np.minimum(idx, midx)
    g = z[canon.reshape(-1)].reshape(ny, nx, 6)
    selfconj = idx == midx
    nu4 = np.where(selfconj, g[..., 0], (g[..., 0] + 1j * g[..., 1]) / np.sqrt(2.0))
    nu9 = np.where(selfconj, g[..., 1], (g[..., 2] + 1j * g[..., 3]) / np.sqrt(2.0))
    mirror = idx > midx
    nu4 = np.where(mirror, np.conj(nu4), nu4)
    nu9 = np.where(mirror, np.conj(nu9), nu9)
    kx = 2 * np.pi * ix / nx
    ky = 2 * np.pi * iy / ny
    lap = ((4.0 / 9.0) * (np.cos(kx) + np.cos(ky)) + (2.0 / 9.0) * np.cos(kx) * np.cos(ky) - 10.0 / 9.0) * 3.0
    rho0 = cfg.get("rho0", 1.0)
    x = rho0 - cfg.get("rhoc", 1.0)
    cs2 = cfg.get("c0sq", 1.0 / 3.0) + rho0 * (cfg["A"] + 3.0 * cfg["B"] * x * x)
    cs2k = cs2 - rho0 * cfg["kappa"] * lap
    le = -1.0 / cfg["tau_bulk"]
    leps = -1.0 / cfg.get("tau_eps", 1.0)
    pref = -rho0 * cfg["kT"] * 3.0
    x44 = pref * 4.0 * (2.0 - 3.0 * cs2k) * le * (2.0 + le)
    x49 = pref * 12.0 * (cs2k - 1.0 / 3.0) * (le + leps + le * leps)
    x99 = pref * 16.0 * (1.25 - 0.75 * cs2k) * leps * (2.0 + leps)
    l44 = np.sqrt(np.maximum(x44, 0.0))
    l94 = np.where(l44 > 0, x49 / np.where(l44 > 0, l44, 1.0), 0.0)
    l99 = np.sqrt(np.maximum(x99 - l94 * l94, 0.0))
    Z = l44 * nu4 + 1j * (l94 * nu4 + l99 * nu9)
    out = np.fft.fft2(Z) / np.sqrt(n)
    return np.ascontiguousarray(out.real), np.ascontiguousarray(out.imag)


class Oracle:
    """Plain FP64 stepper: state f[9][ny][nx] pre-collision, time t."""

    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self.p = make_params(cfg)
        self.nx, self.ny = self.p.nx, self.p.ny
        self.f = np.zeros((9, self.ny, self.nx))
        self.t = 0
        self.flags = (ctypes.c_int64 * 2)(0, 0)
        lib().lbo_init(ctypes.byref(self.p), _dp(self.f))

    def step(self, nsteps: int):
        if self.cfg.get("noise", "k0") == "correlated" and self.cfg["kT"] > 0:
            for _ in range(int(nsteps)):
                xi4, xi9 = correlated_noise_fields(self.cfg, self.t)
                lib().lbo_step_fields(ctypes.byref(self.p), _dp(self.f), int(self.t), _dp(xi4), _dp(xi9))
                self.t += 1
            return
        lib().lbo_step(ctypes.byref(self.p), _dp(self.f), int(nsteps), int(self.t), self.flags)
        self.t += int(nsteps)

    def moments(self) -> np.ndarray:
        m = np.zeros_like(self.f)
        lib().lbo_moments(ctypes.byref(self.p), _dp(self.f), _dp(m))
        return m

    def totals(self) -> np.ndarray:
        """sum rho, sum jx, sum jy, sum |j|^2, sum (-1)^x jx, sum (-1)^y jy."""
        m = self.moments()
        sx = (-1.0) ** np.arange(self.nx)[None, :]
        sy = (-1.0) ** np.arange(self.ny)[:, None]
        return np.array([m[0].sum(), m[1].sum(), m[2].sum(), (m[1] ** 2 + m[2] ** 2).sum(),
                         (sx * m[1]).sum(), (sy * m[2]).sum()])


def stencils(cfg: dict, rho: np.ndarray):
    p = make_params(cfg)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    lap, gx, gy = (np.zeros_like(rho) for _ in range(3))
    lib().lbo_stencils(ctypes.byref(p), _dp(rho), _dp(lap), _dp(gx), _dp(gy))
    return lap, gx, gy


def equilibrium(cfg: dict, rho, jx, jy, lap, gx, gy) -> np.ndarray:
    p = make_params(cfg)
    out = np.zeros(9)
    lib().lbo_equilibrium(ctypes.byref(p), rho, jx, jy, lap, gx, gy, _dp(out))
    return out


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().lbo_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def normals(seed: int, node: int, replica: int, t: int) -> np.ndarray:
    out = np.zeros(6)
    lib().lbo_normals(seed, node, replica, t, _dp(out))
    return out


def normals_batch(seed: int, replica: int, t: int, n: int) -> np.ndarray:
    out = np.zeros((n, 6))
    lib().lbo_normals_batch(seed, replica, t, n, _dp(out))
    return out


def noise_samples(cfg: dict, rho: float, cs2: float, t: int, n: int) -> np.ndarray:
    p = make_params(cfg)
    out = np.zeros((n, 9))
    lib().lbo_noise_samples(ctypes.byref(p), rho, cs2, t, n, _dp(out))
    return out


def tables():
    T = np.zeros((9, 9)); N = np.zeros(9); Ti = np.zeros((9, 9)); w = np.zeros(9)
    lib().lbo_tables(_dp(T), _dp(N), _dp(Ti), _dp(w))
    return T, N, Ti, w


def power_spectrum(m: np.ndarray) -> np.ndarray:
    """|m_a(k)|^2 with a(k) = n^-1/2 sum_r e^{ik.r} a(r) (Sec. III, notation).

    Returned on the half plane [9][ny][nx//2+1]; for a real field the power at k
    equals that at -k, so the sign of the exponent does not matter."""
    n = m.shape[-1] * m.shape[-2]
    F = np.fft.rfft2(m, axes=(-2, -1))
    return (F.real ** 2 + F.imag ** 2) / n


def power_at(a: np.ndarray, kx, ky) -> np.ndarray:
    """|a(k)|^2 with a(k) = n^-1/2 sum_r e^{ik.r} a(r) (Sec. III notation) of one real field
    a[ny][nx], at the lattice wave vectors k = (2 pi kx / nx, 2 pi ky / ny) listed in kx, ky:
    the double sum itself, taken over x for each listed kx (two real matrix-vector products)
    and then over y."""
    ny, nx = a.shape
    x, y = np.arange(nx), np.arange(ny)
    rows = {}
    out = np.empty(len(kx))
    for i, (p, q) in enumerate(zip(kx, ky)):
        if p not in rows:
            ph = 2 * np.pi * ((p * x) % nx) / nx
            rows[p] = a @ np.cos(ph) + 1j * (a @ np.sin(ph))   # sum_x a(x, y) e^{i kx x}
        ph = 2 * np.pi * ((q * y) % ny) / ny
        c = np.dot(np.cos(ph) + 1j * np.sin(ph), rows[p])
        out[i] = (c.real ** 2 + c.imag ** 2) / (nx * ny)
    return out


def radial_shell(kx, ky, nx: int, ny: int):
    """Shell index of the lattice wave vector k = (2 pi kx / nx, 2 pi ky / ny) (integer kx, ky,
    any sign): b = floor(|k| L / 2 pi + 1/2) with L = min(nx, ny), i.e. shells of width
    2 pi / L centred on multiples of it.

    Exact: with q = (|k| L / 2 pi)^2 = (kx L / nx)^2 + (ky L / ny)^2 (a rational number),
    b - 1/2 <= sqrt(q) is (2b - 1)^2 <= 4 q, so b = (isqrt(floor(4 q)) + 1) // 2."""
    L = min(nx, ny)
    px, py = nx // L, ny // L
    kx = np.asarray(kx, dtype=np.int64)
    ky = np.asarray(ky, dtype=np.int64)
    den = (px * py) ** 2
    f4q = (4 * (kx * kx * py * py + ky * ky * px * px)) // den
    s = np.floor(np.sqrt(f4q.astype(np.float64))).astype(np.int64)
    s = np.where(s * s > f4q, s - 1, s)
    s = np.where((s + 1) * (s + 1) <= f4q, s + 1, s)
    return (s + 1) // 2


def radial_spectrum(rho: np.ndarray):
    """Isotropic average of S_rho(k) = |rho(k)|^2 (rho(k) = n^-1/2 sum_r e^{ik.r} rho(r),
    Sec. III notation) over the shells of radial_shell, on the full k plane without k = 0.
    Returns (mean per shell, number of k points per shell); the corner (pi, pi) lies in the
    last shell."""
    ny, nx = rho.shape
    F = np.fft.fft2(rho)
    S = (F.real ** 2 + F.imag ** 2) / (nx * ny)
    kx = np.rint(np.fft.fftfreq(nx, 1.0 / nx)).astype(np.int64)
    ky = np.rint(np.fft.fftfreq(ny, 1.0 / ny)).astype(np.int64)
    KX, KY = np.meshgrid(kx, ky)
    b = radial_shell(KX, KY, nx, ny)
    keep = ~((KX == 0) & (KY == 0))
    nb = int(radial_shell(nx // 2, ny // 2, nx, ny)) + 1
    sums = np.bincount(b[keep], weights=S[keep], minlength=nb)
    counts = np.bincount(b[keep], minlength=nb)
    return np.where(counts > 0, sums / np.maximum(counts, 1), 0.0), counts


def interface_heights(rho: np.ndarray, level: float, rows: int, rising: bool) -> np.ndarray:
    """The height h(x) of an interface (Sec. V.B): in every column x, the position y at which
    the density rho[y][x] passes `level` (for the capillary run the midpoint (rho_L + rho_V)/2),
    searched in rows [rows[0], rows[1]), rising (vapour below, liquid above) or falling, as the
    first such passage between two neighbouring nodes, placed on the straight line through
    them.  Plain loops over the columns."""
    lo, hi = rows
    ny, nx = rho.shape
    h = np.empty(nx)
    for x in range(nx):
        col = rho[lo:hi, x]
        found = False
        for j in range(hi - lo - 1):
            a, b = col[j], col[j + 1]
            if (a - level) * (b - level) <= 0 and ((b > a) if rising else (b < a)):
                h[x] = lo + j + (level - a) / (b - a)
                found = True
                break
        if not found:
            raise ValueError(f"no {'rising' if rising else 'falling'} passage of {level} in column {x}")
    return h


def height_spectrum(h: np.ndarray) -> np.ndarray:
    """|h(k)|^2 with h(k) = Lx^-1/2 sum_x (h(x) - <h>) e^{ikx}, k = 2 pi m / Lx, m = 0 .. Lx/2
    (the spectrum whose mean Sec. V.B compares with kT / (sigma k^2), eq. capill-static);
    numpy's real FFT as the sum."""
    H = np.fft.rfft(h - h.mean())
    return (H.real ** 2 + H.imag ** 2) / h.size
