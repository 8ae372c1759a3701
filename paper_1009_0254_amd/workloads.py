"""Seeded synthetic workloads: parameter sets only (no arithmetic of the method).

Both the HIP library binding and the FP64 oracle read these dicts.  Keys:

  nx, ny            periodic lattice size
  rho0              reference density (linearisation point, storage shift)
  rhoc, A, B, c0sq  free energy psi = c0sq rho ln rho + A/2 (rho-rhoc)^2 + B/4 (rho-rhoc)^4
  kappa             square-gradient coefficient
  tau_bulk, tau_shear, tau_q, tau_eps   relaxation times (lambda_a = -1/tau_a)
  kT                temperature (0 = deterministic)
  seed              Philox key
  replica           replica index (part of the Philox counter)
  init, init_arg    initial density / velocity field:
      uniform  rho = rho0
      slab     rho(y) = out + (in-out)/2 [tanh((y-y1)/w) - tanh((y-y2)/w)], arg = (in, out, y1, y2, w)
      random   rho = rho0 + amp * N(0,1) per node (Philox, reserved counter), arg = (amp,)
      wave     rho = rho0 + a_rho cos(th), u = (U + a_ux cos(th), a_uy cos(th)),
               th = 2 pi (kx x / nx + ky y / ny), arg = (kx, ky, a_rho, a_ux, a_uy, U)
  noise             "k0" (default): Xi(0) at the local density, uncorrelated in space;
                    "correlated": the exact Xi(k) at rho0 (modes 4 and 9 correlated)

The model is the paper's modified-equilibrium D2Q9 model; the five lattice workloads
are the fixed benchmark set of this project (single-phase 64^2, two-phase 2048^2 slab,
single-phase 8192^2, an uneven ensemble and a 16384^2 spinodal quench).  Free-energy
readings: the 64^2, 8192^2 and ensemble runs take the ideal term literally
(c0sq = 1/3); the two-phase runs take c0sq = 0, the paper's pure double well with
beta = B/4, rho_{L,V} = 1 +- sqrt(-A/B).
"""
from __future__ import annotations

import math

_SINGLE = dict(rho0=1.0, rhoc=1.0, A=0.05, B=0.04, kappa=0.02, c0sq=1.0 / 3.0,
               tau_bulk=0.8, tau_shear=0.8, tau_q=1.0, tau_eps=1.0)
_TWO = dict(rho0=1.0, rhoc=1.0, A=-0.01, B=0.04, kappa=0.02, c0sq=0.0,
            tau_bulk=0.8, tau_shear=0.8, tau_q=1.0, tau_eps=1.0)


def single_phase(nx: int, ny: int, kT: float = 1e-5, seed: int = 1, **kw) -> dict:
    d = dict(_SINGLE, nx=nx, ny=ny, kT=kT, seed=seed, init="uniform")
    d.update(kw)
    return d


def slab(nx: int, ny: int, kT: float = 1e-6, seed: int = 1, **kw) -> dict:
    """Liquid slab y in [ny/4, 3ny/4) with tanh walls of half-width sqrt(-2 kappa / A)."""
    d = dict(_TWO, nx=nx, ny=ny, kT=kT, seed=seed)
    delta = math.sqrt(-d["A"] / d["B"])
    w = math.sqrt(-2.0 * d["kappa"] / d["A"])
    d["init"] = "slab"
    d["init_arg"] = [d["rhoc"] + delta, d["rhoc"] - delta, ny / 4 - 0.5, 3 * ny / 4 - 0.5, w]
    d.update(kw)
    return d


def capillary(nx: int = 2048, ny: int = 400, width: int = 180, kT: float = 1e-7, seed: int = 3, **kw) -> dict:
    """The capillary-wave run of Sec. V.B: a liquid stripe of the given width parallel to x in a
    periodic nx x ny box, rho_L = 1, rho_V = 0.5, beta = 0.04, kappa = 0.03, T = 1e-7; every
    relaxation time 1 (the printed tau = 0.1 violates tau > 1/2 and is read as 1.0).  The
    free energy is the paper's f0 (eq. f0-bulk): c0sq = 0, B = 4 beta, A = -beta (rho_L - rho_V)^2,
    rhoc = (rho_L + rho_V) / 2; the walls start as tanh profiles of half-width
    sqrt(2 kappa / beta) / (rho_L - rho_V)."""
    beta, rl, rv, kappa = 0.04, 1.0, 0.5, 0.03
    d = dict(rho0=1.0, rhoc=0.5 * (rl + rv), A=-beta * (rl - rv) ** 2, B=4.0 * beta, kappa=kappa, c0sq=0.0,
             tau_bulk=1.0, tau_shear=1.0, tau_q=1.0, tau_eps=1.0, nx=nx, ny=ny, kT=kT, seed=seed)
    w = math.sqrt(2.0 * kappa / beta) / (rl - rv)
    y1 = (ny - width) / 2 - 0.5
    d["init"] = "slab"
    d["init_arg"] = [rl, rv, y1, y1 + width, w]
    d.update(kw)
    return d


def spinodal(nx: int, ny: int, kT: float = 1e-6, seed: int = 1, amp: float = 0.01, **kw) -> dict:
    d = dict(_TWO, nx=nx, ny=ny, kT=kT, seed=seed, init="random", init_arg=[amp])
    d.update(kw)
    return d


def wave(base: dict, kx: int, ky: int, a_rho: float = 0.0, a_ux: float = 0.0, a_uy: float = 0.0,
         U: float = 0.0) -> dict:
    d = dict(base)
    d["init"] = "wave"
    d["init_arg"] = [kx, ky, a_rho, a_ux, a_uy, U]
    return d


# the five lattice workloads, in order
def single_phase_64() -> dict:
    """64x64 single phase, kT = 1e-5, seed 1, 2000 steps, FP64."""
    return dict(single_phase(64, 64, kT=1e-5, seed=1), steps=2000, precision="fp64")


def slab_2048() -> dict:
    """2048x2048 two-phase slab, kT = 1e-6, 10k steps, FP64 vs FP32."""
    return dict(slab(2048, 2048, kT=1e-6, seed=1), steps=10000, precision="fp32s")


def single_phase_8192(seed: int = 7) -> dict:
    """8192x8192 single phase, kT = 1e-5, FP32-shifted vs FP64, S(k) over 20k steps."""
    return dict(single_phase(8192, 8192, kT=1e-5, seed=seed), steps=20000, precision="fp32s")


def ensemble_336(seed: int = 11) -> list:
    """Uneven ensemble: 256 x 128^2, 64 x 256^2, 16 x 512^2; kT log-uniform in [1e-6, 1e-4].

    The per-replica kT is drawn here from Python's own seeded generator; it is an input
    of both the GPU run and the oracle, never drawn by either."""
    import random
    rng = random.Random(seed)
    reps = []
    r = 0
    for count, size in ((256, 128), (64, 256), (16, 512)):
        for _ in range(count):
            kT = 10.0 ** (-6.0 + 2.0 * rng.random())
            reps.append(single_phase(size, size, kT=kT, seed=seed * 1000003 + r, replica=r))
            r += 1
    return reps


def quench_16384(seed: int = 5) -> dict:
    """16384x16384 spinodal quench, rho = 1 + 0.01 N(0,1), kT = 1e-6, FP32-shifted."""
    return dict(spinodal(16384, 16384, kT=1e-6, seed=seed), steps=50000, precision="fp32s")


def correlated_sec5a(nx: int = 128, ny: int = 128, kT: float = 1e-7, seed: int = 4) -> dict:
    """Correlated-noise equilibration run of Sec. V.A (kappa = 0.08, c_s ~ 0.265, tau = 1).

    Double well with rho_V = 0.5, rho_L = 1, beta = 0.14, run in the liquid at rho0 = 1."""
    beta, rv, rl = 0.14, 0.5, 1.0
    return dict(nx=nx, ny=ny, rho0=1.0, rhoc=0.5 * (rl + rv), A=-beta * (rl - rv) ** 2, B=4 * beta,
                kappa=0.08, c0sq=0.0, tau_bulk=1.0, tau_shear=1.0, tau_q=1.0, tau_eps=1.0,
                kT=kT, seed=seed, init="uniform", noise="correlated")


def uncorrelated_sec5a(nx: int = 128, ny: int = 128, kT: float = 1e-7, seed: int = 3) -> dict:
    """Uncorrelated-noise equilibration run of Sec. V.A (kappa = 0.03, c_s ~ 0.15, tau = 1).

    Double well with rho_V = 0.1, rho_L = 1, beta = 0.015, run in the liquid at rho0 = 1."""
    beta, rv, rl = 0.015, 0.1, 1.0
    return dict(nx=nx, ny=ny, rho0=1.0, rhoc=0.5 * (rl + rv), A=-beta * (rl - rv) ** 2, B=4 * beta,
                kappa=0.03, c0sq=0.0, tau_bulk=1.0, tau_shear=1.0, tau_q=1.0, tau_eps=1.0,
                kT=kT, seed=seed, init="uniform")
