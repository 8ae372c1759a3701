"""Closed-form linear theory of the fluctuating modified-equilibrium (Swift) D2Q9 model.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module; it is
used by tests/, by the oracle's own pins and by bench.py's cpu_baseline leg.

Everything here is written from Gross, Adhikari, Cates & Varnik, "Thermal
fluctuations in the lattice Boltzmann method for non-ideal fluids"
(arXiv:1009.0254).  Citations name the section / equation / table:

* velocity set, weights, basis T and lengths N_a ......... Sec. III.A, Table I, eq. (Tmat), eq. (scalar-prod)
* lattice Laplacian symbol ............................... App. B
* generalised sound speed c_s^2(k), d(k) ................. eq. (sound-speed-k), eq. (eq-mom-yeo)
* structure factor S(k) .................................. eq. (struct-fact)
* advection operator A(k) ................................ eq. (lb-adv)
* linearised collision operator Omega(k) ................. eq. (coll-op-yeo)
* LB-Langevin map in Fourier space ....................... eq. (lb-lang-ft)
* FDT for the noise matrix ............................... eq. (noise-matrix), eq. (noise-matrix-k0)
* equal-time correlations G(k) ........................... eq. (g-mat-yeo)
* closed-form noise matrix Xi(k) ......................... eq. (noise-yeo)
* hydrodynamic-limit stress-noise variances .............. App. C, eq. (e-fluct)
* bulk viscosity zeta(k) ................................. eq. (bulkv-yeo)
* interface width and surface tension .................... eq. (interf-width), eq. (surf-tension)

The stationary covariance for spatially uncorrelated (k=0) noise,
G_unc = M G_unc M^H + A(-k) Xi(0) A(-k)^H with M = A(-k)(I + Omega(k)), follows
from eq. (lb-lang-ft) by the same stationarity argument that gives eq. (noise-matrix)
(Sec. III.B); it is the exact target for a simulation that uses Xi(0).
"""
from __future__ import annotations

import numpy as np

SIGMA_S2 = 1.0 / 3.0  # sigma_s^2, ideal LB sound speed squared (Sec. III, notation)

# D2Q9 velocities in the column order of eq. (Tmat): c_1 .. c_9.
C = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1],
              [1, 1], [-1, 1], [-1, -1], [1, -1]], dtype=np.int64)
# Weights (Sec. III.A): w_1 = 4/9, w_2..5 = 1/9, w_6..9 = 1/36.
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def basis_T() -> np.ndarray:
    """Rows of Table I evaluated on the velocity set: T[a, i] (a, i = 0..8)."""
    cx = C[:, 0].astype(float)
    cy = C[:, 1].astype(float)
    c2 = cx * cx + cy * cy
    rows = [
        np.ones(9),                # 1           rho
        cx,                        # c_x         j_x
        cy,                        # c_y         j_y
        3 * c2 - 2,                # 3c^2-2      e
        2 * cx * cx - c2,          # 2c_x^2-c^2  p_ww
        cx * cy,                   # c_x c_y     p_xy
        (3 * c2 - 4) * cx,         # q_x
        (3 * c2 - 4) * cy,         # q_y
        9 * c2 * c2 - 15 * c2 + 2, # epsilon
    ]
    return np.array(rows)


T = basis_T()
N = (T * T) @ W                         # N_a = sum_i w_i T_ai^2, eq. (scalar-prod)
TINV = (W[:, None] * T.T) / N[None, :]  # (T^-1)_{ia} = w_i T_ai / N_a (Sec. III.A)


def relaxation_rates(tau_bulk, tau_shear, tau_q, tau_eps) -> np.ndarray:
    """lambda_a = -1/tau_a, Table I; conserved modes have lambda = 0."""
    lb, ls, lq, le = (-1.0 / tau_bulk, -1.0 / tau_shear, -1.0 / tau_q, -1.0 / tau_eps)
    return np.array([0.0, 0.0, 0.0, lb, ls, ls, lq, lq, le])


# ----------------------------------------------------------------------------
# thermodynamics of psi(rho) = c0sq rho ln rho + A/2 (rho-rc)^2 + B/4 (rho-rc)^4
# (Sec. II.A: p0 = rho psi' - psi, c_s^2 = dp0/drho = rho psi'')
# ----------------------------------------------------------------------------

def pressure(rho, c0sq, A, B, rhoc=1.0):
    x = rho - rhoc
    psi = c0sq * rho * np.log(rho) + 0.5 * A * x**2 + 0.25 * B * x**4
    dpsi = c0sq * (np.log(rho) + 1.0) + A * x + B * x**3
    return rho * dpsi - psi


def sound_speed2(rho, c0sq, A, B, rhoc=1.0):
    x = rho - rhoc
    return c0sq + rho * (A + 3.0 * B * x * x)


def paper_free_energy_to_AB(beta, rho_v, rho_l):
    """Map f0 = beta (rho-rho_V)^2 (rho-rho_L)^2 (eq. f0-bulk) onto (A, B, rhoc) with c0sq = 0.

    The two functions differ by an additive constant only."""
    rhoc = 0.5 * (rho_l + rho_v)
    B = 4.0 * beta
    A = -beta * (rho_l - rho_v) ** 2
    return A, B, rhoc


def interface_width(kappa, beta, rho_l, rho_v):
    """xi = sqrt(8 kappa / beta) / (rho_L - rho_V), eq. (interf-width)."""
    return np.sqrt(8.0 * kappa / beta) / (rho_l - rho_v)


def surface_tension(kappa, beta, rho_l, rho_v):
    """sigma = (rho_L - rho_V)^3 sqrt(2 kappa beta) / 6, eq. (surf-tension)."""
    return (rho_l - rho_v) ** 3 * np.sqrt(2.0 * kappa * beta) / 6.0


# ----------------------------------------------------------------------------
# lattice Fourier symbols (App. B)
# ----------------------------------------------------------------------------

def laplacian_symbol(kx, ky):
    """Fourier symbol of the 9-point Laplacian of App. B (equals -k^2 on the lattice)."""
    return ((4.0 / 9.0) * (np.cos(kx) + np.cos(ky))
            + (2.0 / 9.0) * np.cos(kx) * np.cos(ky) - 10.0 / 9.0) / SIGMA_S2


def k2_lattice(kx, ky):
    return -laplacian_symbol(kx, ky)


def cs2_k(kx, ky, cs2, rho0, kappa):
    """c_s^2(k) = c_s^2 + rho0 kappa k^2, eq. (sound-speed-k), lattice k^2."""
    return cs2 + rho0 * kappa * k2_lattice(kx, ky)


def d_k(kx, ky, cs2, rho0, kappa):
    """d(k) = 6 [c_s^2(k) - sigma_s^2], eq. (eq-mom-yeo)."""
    return 6.0 * (cs2_k(kx, ky, cs2, rho0, kappa) - SIGMA_S2)


def structure_factor(kx, ky, cs2, rho0, kappa, kT):
    """S(k) = rho0 kT / c_s^2(k), eq. (struct-fact) with the lattice k^2 (App. B)."""
    return rho0 * kT / cs2_k(kx, ky, cs2, rho0, kappa)


def shear_viscosity(rho0, tau_shear):
    """eta = rho0 sigma_s^2 (tau_s - 1/2), Sec. III.C."""
    return rho0 * SIGMA_S2 * (tau_shear - 0.5)


# ----------------------------------------------------------------------------
# 9x9 matrices in moment space
# ----------------------------------------------------------------------------

def advection(kx, ky):
    """A(k) = T diag(exp(-i k.c_j)) T^-1, eq. (lb-adv)."""
    phase = np.exp(-1j * (C[:, 0] * kx + C[:, 1] * ky))
    return T @ np.diag(phase) @ TINV


def equilibrium_jacobian(kx, ky, cs2, rho0, kappa, U=(0.0, 0.0)):
    """E = d m^eq / d m at the uniform state (rho0, j = rho0 U), Fourier mode k.

    Hand derivative of Table II (C_n = 0): the square-gradient terms enter linearly only
    through -kappa rho lap(rho) (lap -> -k^2 of App. B); (grad rho)^2 terms are quadratic."""
    ux, uy = U
    rho = rho0
    jx, jy = rho * ux, rho * uy
    k2 = k2_lattice(kx, ky)
    piso = cs2 - SIGMA_S2 + kappa * rho0 * k2       # d/d rho of (p0 - rho sigma_s^2 - kappa rho lap rho)
    E = np.zeros((9, 9), dtype=complex)
    E[0, 0] = 1.0
    E[1, 1] = 1.0
    E[2, 2] = 1.0
    # m4 = 3 |j|^2 / rho + 6 (...)
    E[3, 0] = -3.0 * (jx * jx + jy * jy) / rho**2 + 6.0 * piso
    E[3, 1] = 6.0 * jx / rho
    E[3, 2] = 6.0 * jy / rho
    # m5 = (jx^2 - jy^2) / rho
    E[4, 0] = -(jx * jx - jy * jy) / rho**2
    E[4, 1] = 2.0 * jx / rho
    E[4, 2] = -2.0 * jy / rho
    # m6 = jx jy / rho
    E[5, 0] = -jx * jy / rho**2
    E[5, 1] = jy / rho
    E[5, 2] = jx / rho
    # m9 = -6 (...)
    E[8, 0] = -6.0 * piso
    return E


def collision_operator_flow(kx, ky, lam, cs2, rho0, kappa, U):
    """Omega(k) around a uniform flow: m* = m + Lambda (m - m^eq) gives Omega = Lambda (I - E).

    At U = 0 this equals eq. (coll-op-yeo)."""
    E = equilibrium_jacobian(kx, ky, cs2, rho0, kappa, U)
    return np.diag(np.asarray(lam, dtype=complex)) @ (np.eye(9) - E)


def step_matrix_flow(kx, ky, lam, cs2, rho0, kappa, U):
    return advection(-kx, -ky) @ (np.eye(9) + collision_operator_flow(kx, ky, lam, cs2, rho0, kappa, U))


def collision_operator(kx, ky, lam, cs2, rho0, kappa):
    """Omega(k) of eq. (coll-op-yeo): diag(lambda) plus the d(k) couplings of modes 4 and 9 to rho."""
    d = d_k(kx, ky, cs2, rho0, kappa)
    om = np.diag(np.asarray(lam, dtype=complex))
    om[3, 0] = -lam[3] * d
    om[8, 0] = lam[8] * d
    return om


def equilibrium_correlations(kx, ky, cs2, rho0, kappa, kT):
    """G(k) of eq. (g-mat-yeo)."""
    S = structure_factor(kx, ky, cs2, rho0, kappa, kT)
    d = d_k(kx, ky, cs2, rho0, kappa)
    Tt = rho0 * kT / SIGMA_S2
    G = np.zeros((9, 9), dtype=complex)
    G[0, 0] = S
    G[1, 1] = G[2, 2] = Tt * SIGMA_S2
    G[0, 3] = G[3, 0] = S * d
    G[0, 8] = G[8, 0] = -S * d
    G[3, 3] = N[3] * S
    G[3, 8] = G[8, 3] = 2.0 * S * d
    G[4, 4] = N[4] * Tt
    G[5, 5] = N[5] * Tt
    G[6, 6] = N[6] * Tt
    G[7, 7] = N[7] * Tt
    G[8, 8] = N[8] * (S + 3.0 * Tt) / 4.0
    return G


def noise_matrix_fdt(kx, ky, lam, cs2, rho0, kappa, kT):
    """Xi(k) = A(k) G A(-k)^T - [I+Omega(k)] G [I+Omega(-k)]^T, eq. (noise-matrix)."""
    G = equilibrium_correlations(kx, ky, cs2, rho0, kappa, kT)
    A = advection(kx, ky)
    Am = advection(-kx, -ky)
    Op = np.eye(9) + collision_operator(kx, ky, lam, cs2, rho0, kappa)
    Om = np.eye(9) + collision_operator(-kx, -ky, lam, cs2, rho0, kappa)
    return A @ G @ Am.T - Op @ G @ Om.T


def noise_matrix_k0_fdt(lam, cs2, rho0, kT):
    """Xi(0) = -G Omega^T - Omega G - Omega G Omega^T at k -> 0, eq. (noise-matrix-k0)."""
    G = equilibrium_correlations(0.0, 0.0, cs2, rho0, 0.0, kT)
    Om = collision_operator(0.0, 0.0, lam, cs2, rho0, 0.0)
    return (-G @ Om.T - Om @ G - Om @ G @ Om.T).real


def noise_matrix_closed(kx, ky, lam, cs2, rho0, kappa, kT):
    """Closed form of eq. (noise-yeo)."""
    c2k = cs2_k(kx, ky, cs2, rho0, kappa)
    lt = lam * (2.0 + lam)                      # tilde-lambda_a = lambda_a (2 + lambda_a)
    le, leps = lam[3], lam[8]
    lt_ee = le + leps + le * leps               # tilde-lambda_{e eps}
    pref = -rho0 * kT / SIGMA_S2
    X = np.zeros((9, 9))
    X[3, 3] = N[3] * (2.0 - 3.0 * c2k) * lt[3]
    X[3, 8] = X[8, 3] = 12.0 * (c2k - SIGMA_S2) * lt_ee
    X[4, 4] = N[4] * lt[4]
    X[5, 5] = N[5] * lt[5]
    X[6, 6] = N[6] * lt[6]
    X[7, 7] = N[7] * lt[7]
    X[8, 8] = N[8] * (1.25 - 0.75 * c2k) * lt[8]
    return pref * X


def stress_noise_variances_appC(lam, cs2, rho0, kT):
    """<xi_4^2>, <xi_5^2>, <xi_6^2> from the hydrodynamic limit, App. C (h = 2 - c_s^2/sigma_s^2)."""
    lb, ls = lam[3], lam[4]
    h = 2.0 - cs2 / SIGMA_S2
    v4 = -36.0 * kT * rho0 * SIGMA_S2 * (2 * lb + lb * lb) * h
    v5 = -4.0 * kT * rho0 * SIGMA_S2 * (2 * ls + ls * ls)
    v6 = -1.0 * kT * rho0 * SIGMA_S2 * (2 * ls + ls * ls)
    return v4, v5, v6


def step_matrix(kx, ky, lam, cs2, rho0, kappa):
    """M(k) = A(-k) [I + Omega(k)]: one deterministic step in Fourier space, eq. (lb-lang-ft)."""
    return advection(-kx, -ky) @ (np.eye(9) + collision_operator(kx, ky, lam, cs2, rho0, kappa))


def stationary_covariance_uncorrelated(kx, ky, lam, cs2, rho0, kappa, kT, diagonal=False):
    """Stationary <dm(k) dm(k)^H> when the noise has the k-independent covariance Xi(0)
    (diagonal=True: only its diagonal, the "ideal-gas-like" noise of Sec. IV).

    Solves G = M G M^H + Q with Q = A(-k) Xi(0) A(-k)^H by vectorisation.
    Singular (undamped) directions make the system ill-posed; callers exclude k = 0 and
    the staggered-momentum points (pi, 0) / (0, pi)."""
    M = step_matrix(kx, ky, lam, cs2, rho0, kappa)
    Am = advection(-kx, -ky)
    X = noise_matrix_closed(0.0, 0.0, lam, cs2, rho0, 0.0, kT)
    if diagonal:
        X = np.diag(np.diag(X))
    Q = Am @ X @ Am.conj().T
    n = 9
    # vec(M G M^H) = (conj(M) kron M) vec(G) with column-major vec
    K = np.eye(n * n) - np.kron(M.conj(), M)
    g = np.linalg.solve(K, Q.reshape(-1, order="F"))
    return g.reshape(n, n, order="F")


def transient_covariance(kx, ky, lam, cs2, rho0, kappa, kT, t, noise="k0"):
    """sum_{s<t} M^s Q M^{H s}: covariance after t noisy steps from a noise-free start, with
    Q = A(-k) Xi A(-k)^H (eq. lb-lang-ft, one step at a time)."""
    M = step_matrix(kx, ky, lam, cs2, rho0, kappa)
    Am = advection(-kx, -ky)
    if noise == "k0":
        X = noise_matrix_closed(0.0, 0.0, lam, cs2, rho0, 0.0, kT)
    elif noise == "diagonal":
        X = np.diag(np.diag(noise_matrix_closed(0.0, 0.0, lam, cs2, rho0, 0.0, kT)))
    else:
        X = noise_matrix_closed(kx, ky, lam, cs2, rho0, kappa, kT)
    Q = Am @ X @ Am.conj().T
    G = np.zeros((9, 9), dtype=complex)
    for _ in range(t):
        G = M @ G @ M.conj().T + Q
    return G


def transient_covariance_batch(kx, ky, lam, cs2, rho0, kappa, kT, t, power=False):
    """The same sum for the k = 0 noise at many k (arrays kx, ky) by doubling:
    with P_s = M^s and G_s the covariance after s steps, G_{s1+s2} = G_{s2} + P_{s2} G_{s1}
    P_{s2}^H and P_{s1+s2} = P_{s2} P_{s1}; t is built from its binary digits.
    Returns [K, 9, 9], and with power=True also M^t [K, 9, 9]."""
    kx = np.atleast_1d(np.asarray(kx, dtype=float))
    ky = np.atleast_1d(np.asarray(ky, dtype=float))
    X = noise_matrix_closed(0.0, 0.0, lam, cs2, rho0, 0.0, kT)
    M = np.stack([step_matrix(a, b, lam, cs2, rho0, kappa) for a, b in zip(kx, ky)])
    Am = np.stack([advection(-a, -b) for a, b in zip(kx, ky)])
    Q = Am @ X @ np.conj(np.swapaxes(Am, 1, 2))
    H = lambda A: np.conj(np.swapaxes(A, 1, 2))
    # (Pd, Gd): 2^j steps; (Pa, Ga): the steps taken so far
    Pd, Gd = M, Q
    Pa = np.broadcast_to(np.eye(9, dtype=complex), M.shape).copy()
    Ga = np.zeros_like(Q)
    while t > 0:
        if t & 1:
            Ga = Gd + Pd @ Ga @ H(Pd)
            Pa = Pd @ Pa
        t >>= 1
        if t:
            Gd = Gd + Pd @ Gd @ H(Pd)
            Pd = Pd @ Pd
    return (Ga, Pa) if power else Ga


def sampled_mean_covariance_batch(kx, ky, lam, cs2, rho0, kappa, kT, t0, every, nsamples):
    """Mean of the covariance G(t) over the sampling times t = t0 + every s, s = 0 .. N - 1,
    after a noise-free start (G(0) = 0), for the k = 0 noise at many k (arrays kx, ky):
    what an S(k) accumulated at those times averages to in the linear model.

    With P = M^every and G(t) = sum_{u<t} M^u Q M^{Hu} (eq. lb-lang-ft from rest),
    G(t0 + every s) = P^s G(t0) P^{Hs} + G(every s) and G(every s) = sum_{v<s} P^v G(every) P^{Hv},
    so  N * mean = D_N(G(t0)) + (N - 1) D_N(G(every)) - E_N(G(every))  with
    D_m(Y) = sum_{v<m} P^v Y P^{Hv} and E_m(Y) = sum_{v<m} v P^v Y P^{Hv}.  A block of a terms
    followed by one of b combines as D_{a+b} = D_a + P^a D_b P^{Ha},
    E_{a+b} = E_a + P^a (E_b + a D_b) P^{Ha}; N is built from its binary digits.
    Returns [K, 9, 9]."""
    H = lambda A: np.conj(np.swapaxes(A, 1, 2))
    G0, _ = transient_covariance_batch(kx, ky, lam, cs2, rho0, kappa, kT, t0, power=True)
    Ge, P = transient_covariance_batch(kx, ky, lam, cs2, rho0, kappa, kT, every, power=True)
    eye = np.broadcast_to(np.eye(9, dtype=complex), P.shape).copy()

    def block_sums(Y):
        # (count, P^count, D, E) of the doubling block and of the running total
        cd, Pd, Dd, Ed = 1, P, Y.copy(), np.zeros_like(Y)
        ca, Pa, Da, Ea = 0, eye, np.zeros_like(Y), np.zeros_like(Y)
        n = int(nsamples)
        while n > 0:
            if n & 1:
                # running block (a = ca terms) followed by the doubling block (b = cd terms)
                Da, Ea = Da + Pa @ Dd @ H(Pa), Ea + Pa @ (Ed + ca * Dd) @ H(Pa)
                Pa, ca = Pd @ Pa, ca + cd
            n >>= 1
            if n:
                Dd, Ed = Dd + Pd @ Dd @ H(Pd), Ed + Pd @ (Ed + cd * Dd) @ H(Pd)
                Pd, cd = Pd @ Pd, 2 * cd
        return Da, Ea

    D0, _ = block_sums(G0)
    De, Ee = block_sums(Ge)
    return (D0 + (nsamples - 1) * De - Ee) / nsamples


def psd_all_k(kappa, cs2, lam, rho0=1.0, nk=97, tol=1e-12):
    """True when Xi(k) of eq. (noise-yeo) is positive semi-definite at every k with k_x, k_y in
    [0, pi] (the white region of Fig. 2); checked on an nk x nk grid of k (which includes the
    corner (pi, pi) where minus the App. B Laplacian symbol is largest)."""
    for kx in np.linspace(0.0, np.pi, nk):
        for ky in np.linspace(0.0, np.pi, nk):
            X = noise_matrix_closed(kx, ky, lam, cs2, rho0, kappa, 1.0).real
            if np.linalg.eigvalsh(X).min() < -tol * np.abs(X).max():
                return False
    return True


def interface_width_paper(kappa, cs2, rho0=1.0):
    """xi = 4 sqrt(rho0 kappa) / c_s (eq. interf-width); xi = 4 is the dashed curve of Fig. 2."""
    return 4.0 * np.sqrt(rho0 * kappa / cs2)
