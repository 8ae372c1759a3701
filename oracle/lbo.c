/*
 * lbo.c -- plain FP64 CPU reference ("oracle") for the fluctuating
 * modified-equilibrium (Swift) D2Q9 lattice Boltzmann model of
 * Gross, Adhikari, Cates & Varnik, arXiv:1009.0254.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into oracle/liblbo.so and is
 * loaded by tests/, by __graft_entry__.smoke() and by bench.py's cpu_baseline leg.
 * It shares no code, header, table or constant with the HIP library; it is slow
 * and written for readability: whole-lattice passes, one after another, in the
 * order the paper states the algorithm.
 *
 * One time step, state = pre-collision populations f_i(r,t) on a periodic nx*ny
 * lattice (the delta-m(t) of eq. lb-lang-ft):
 *   1. density and momentum, rho = sum f_i, j = sum c_i f_i       (Sec. III.A)
 *   2. grad rho and lap rho on the whole rho field:
 *        Laplacian: the 9-point stencil of App. B;
 *        gradient:  the paper gives none; we use the isotropic
 *                   d_a rho = 3 sum_i w_i c_ia rho(r + c_i)        (reading R3)
 *   3. local thermodynamics of psi = c0sq rho ln rho + A/2 x^2 + B/4 x^4,
 *      x = rho - rhoc: p0 = rho psi' - psi, c_s^2 = rho psi''       (Sec. II.A)
 *   4. moments m = T f and equilibrium moments of Table II (C_n = 0)
 *   5. noise xi = L nu with L L^T = Xi(0) of eq. (noise-yeo) at k = 0, evaluated
 *      with the local rho and c_s^2 (Sec. IV and Sec. V.B); or, for the "ideal-gas-like"
 *      variant of Sec. IV, L = the square root of the diagonal of Xi(0)
 *   6. m*_a = m_a + lambda_a (m_a - m^eq_a) + xi_a                  (eq. gen-lbe-m, fluct-lin-lbe)
 *   7. f*_i = sum_a (T^-1)_ia m*_a, (T^-1)_ia = w_i T_ai / N_a
 *   8. streaming f_i(r + c_i, t+1) = f*_i(r, t), periodic           (eq. gen-lbe)
 *
 * Spatially correlated noise (Sec. IV, last paragraph; Fig. 3): modes 4 and 9 take fields
 * xi_4(r), xi_9(r) built outside this file (oracle.py: nu(k) drawn per k, L(k) of
 * eq. noise-yeo, one transform back); modes 5..8, whose entries of Xi(k) do not depend on k,
 * stay uncorrelated with the homogeneous rho0 (lbo_step_fields).
 *
 * Random numbers (the paper only asks for independent unit Gaussians, Sec. IV):
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key = seed, counter =
 * (node, replica, t_lo, t_hi); the 128 output bits give six 21-bit uniforms
 * u = (b + 1/2) 2^-21, paired by Box-Muller into nu_4 .. nu_9.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 9

typedef struct {
    int32_t nx, ny;
    double rho0, rhoc, A, B, kappa, c0sq;
    double tau_bulk, tau_shear, tau_q, tau_eps;
    double kT;
    uint64_t seed;
    uint32_t replica;
    int32_t init_kind;
    int32_t noise_kind;   /* 0: Xi(0) at the local rho (uncorrelated); 1: exact Xi(k) (correlated);
                             2: the diagonal of Xi(0) at the local rho ("ideal-gas-like") */
    int32_t pad_;
    double init_arg[6];
} lbo_params;

enum { LBO_INIT_UNIFORM = 0, LBO_INIT_SLAB = 1, LBO_INIT_RANDOM = 2, LBO_INIT_WAVE = 3 };

/* velocity set in the column order of eq. (Tmat) */
static const int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

static double Wt[Q];        /* weights w_i */
static double Tm[Q][Q];     /* T[a][i], Table I */
static double Nn[Q];        /* N_a */
static double Ti[Q][Q];     /* T^-1 [i][a] */
static int tables_ready = 0;

static void build_tables(void)
{
    if (tables_ready) return;
    for (int i = 0; i < Q; i++) {
        double cx = CX[i], cy = CY[i], c2 = cx * cx + cy * cy;
        Wt[i] = (i == 0) ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        Tm[0][i] = 1.0;
        Tm[1][i] = cx;
        Tm[2][i] = cy;
        Tm[3][i] = 3.0 * c2 - 2.0;
        Tm[4][i] = 2.0 * cx * cx - c2;
        Tm[5][i] = cx * cy;
        Tm[6][i] = (3.0 * c2 - 4.0) * cx;
        Tm[7][i] = (3.0 * c2 - 4.0) * cy;
        Tm[8][i] = 9.0 * c2 * c2 - 15.0 * c2 + 2.0;
    }
    for (int a = 0; a < Q; a++) {
        Nn[a] = 0.0;
        for (int i = 0; i < Q; i++) Nn[a] += Wt[i] * Tm[a][i] * Tm[a][i];
    }
    for (int i = 0; i < Q; i++)
        for (int a = 0; a < Q; a++) Ti[i][a] = Wt[i] * Tm[a][i] / Nn[a];
    tables_ready = 1;
}

void lbo_tables(double *T_out, double *N_out, double *Tinv_out, double *w_out)
{
    build_tables();
    for (int a = 0; a < Q; a++) {
        N_out[a] = Nn[a];
        for (int i = 0; i < Q; i++) {
            T_out[a * Q + i] = Tm[a][i];
            Tinv_out[i * Q + a] = Ti[i][a];
        }
    }
    for (int i = 0; i < Q; i++) w_out[i] = Wt[i];
}

/* ---------------------------------------------------------------- Philox4x32-10 */

void lbo_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {            /* Weyl key schedule between rounds */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* six unit normals nu_4..nu_9 for (seed, node, replica, t) */
void lbo_normals(uint64_t seed, uint32_t node, uint32_t replica, uint64_t t, double nu[6])
{
    const double PI = 3.14159265358979323846;
    uint32_t ctr[4] = {node, replica, (uint32_t)t, (uint32_t)(t >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    lbo_philox4x32_10(ctr, key, x);
    uint32_t b[6];
    b[0] = x[0] >> 11;
    b[1] = x[1] >> 11;
    b[2] = x[2] >> 11;
    b[3] = x[3] >> 11;
    b[4] = ((x[0] & 0x7FFu) << 10) | ((x[1] & 0x7FFu) >> 1);
    b[5] = ((x[2] & 0x7FFu) << 10) | ((x[3] & 0x7FFu) >> 1);
    double u[6];
    for (int k = 0; k < 6; k++) u[k] = ((double)b[k] + 0.5) / 2097152.0;   /* 2^21 */
    for (int p = 0; p < 3; p++) {
        double r = sqrt(-2.0 * log(u[2 * p]));
        double th = 2.0 * PI * u[2 * p + 1];
        nu[2 * p] = r * cos(th);
        nu[2 * p + 1] = r * sin(th);
    }
}

/* batch helper for statistical tests: normals for nodes [0, n) at (seed, replica, t) */
void lbo_normals_batch(uint64_t seed, uint32_t replica, uint64_t t, int64_t n, double *out)
{
    for (int64_t k = 0; k < n; k++) lbo_normals(seed, (uint32_t)k, replica, t, out + 6 * k);
}

/* ---------------------------------------------------------------- model pieces */

static double lam_of(const lbo_params *p, int a)
{
    switch (a) {
    case 3: return -1.0 / p->tau_bulk;
    case 4: case 5: return -1.0 / p->tau_shear;
    case 6: case 7: return -1.0 / p->tau_q;
    case 8: return -1.0 / p->tau_eps;
    default: return 0.0;
    }
}

static double bulk_pressure(const lbo_params *p, double rho)
{
    double x = rho - p->rhoc;
    /* p0 = rho psi' - psi with psi = c0sq rho ln rho + A/2 x^2 + B/4 x^4; with c0sq = 0 (the
       paper's double well, eq. f0-bulk) psi has no rho ln rho term at all, and log rho, which
       has no value for rho <= 0, is not evaluated */
    const double lr = p->c0sq != 0.0 ? log(rho) : 0.0;
    double psi = p->c0sq * rho * lr + 0.5 * p->A * x * x + 0.25 * p->B * x * x * x * x;
    double dpsi = p->c0sq * (lr + 1.0) + p->A * x + p->B * x * x * x;
    return rho * dpsi - psi;
}

static double sound_speed_sq(const lbo_params *p, double rho)
{
    double x = rho - p->rhoc;
    return p->c0sq + rho * (p->A + 3.0 * p->B * x * x);
}

static int64_t idx(const lbo_params *p, int x, int y)
{
    x = ((x % p->nx) + p->nx) % p->nx;
    y = ((y % p->ny) + p->ny) % p->ny;
    return (int64_t)y * p->nx + x;
}

/* lap rho (App. B) and the isotropic gradient on a periodic field */
void lbo_stencils(const lbo_params *p, const double *rho, double *lap, double *gx, double *gy)
{
    build_tables();
    const double s2 = 1.0 / 3.0;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; y++) {
        for (int x = 0; x < p->nx; x++) {
            int64_t n = idx(p, x, y);
            double sl = 0.0, sx = 0.0, sy = 0.0;
            for (int i = 1; i < Q; i++) {
                double fwd = rho[idx(p, x + CX[i], y + CY[i])];
                double bwd = rho[idx(p, x - CX[i], y - CY[i])];
                sl += Wt[i] * (fwd + bwd - 2.0 * rho[n]);
                sx += Wt[i] * CX[i] * fwd;
                sy += Wt[i] * CY[i] * fwd;
            }
            lap[n] = sl / s2;
            gx[n] = 3.0 * sx;
            gy[n] = 3.0 * sy;
        }
    }
}

/* Table II with C_n = 0 */
static void equilibrium(const lbo_params *p, double rho, double jx, double jy,
                        double lap, double gx, double gy, double meq[Q])
{
    const double s2 = 1.0 / 3.0;
    double p0 = bulk_pressure(p, rho);
    double ux = jx / rho, uy = jy / rho;
    double piso = p0 - rho * s2 - p->kappa * rho * lap;
    meq[0] = rho;
    meq[1] = rho * ux;
    meq[2] = rho * uy;
    meq[3] = 3.0 * rho * (ux * ux + uy * uy) + 6.0 * piso;
    meq[4] = rho * (ux * ux - uy * uy) + p->kappa * (gx * gx - gy * gy);
    meq[5] = rho * ux * uy + p->kappa * gx * gy;
    meq[6] = 0.0;
    meq[7] = 0.0;
    meq[8] = -6.0 * piso - 3.0 * p->kappa * (gx * gx + gy * gy);
}

/* Xi(0) of eq. (noise-yeo) at k = 0 with local rho and c_s^2: the nonzero block
   entries X44, X49, X99 and the diagonal X55..X88 (indices are 0-based modes).  The
   "ideal-gas-like" variant of Sec. IV (noise_kind 2) keeps only the diagonal. */
static void noise_covariance(const lbo_params *p, double rho, double cs2, double X[Q][Q])
{
    const double s2 = 1.0 / 3.0;
    double lam[Q];
    for (int a = 0; a < Q; a++) lam[a] = lam_of(p, a);
    double lt[Q];
    for (int a = 0; a < Q; a++) lt[a] = lam[a] * (2.0 + lam[a]);
    double lt_ee = lam[3] + lam[8] + lam[3] * lam[8];
    double pref = -rho * p->kT / s2;
    memset(X, 0, sizeof(double) * Q * Q);
    X[3][3] = pref * Nn[3] * (2.0 - 3.0 * cs2) * lt[3];
    if (p->noise_kind != 2) X[3][8] = X[8][3] = pref * 12.0 * (cs2 - s2) * lt_ee;
    X[4][4] = pref * Nn[4] * lt[4];
    X[5][5] = pref * Nn[5] * lt[5];
    X[6][6] = pref * Nn[6] * lt[6];
    X[7][7] = pref * Nn[7] * lt[7];
    X[8][8] = pref * Nn[8] * (1.25 - 0.75 * cs2) * lt[8];
}

/* Cholesky of the lower-right 6x6 block (modes 4..9); a negative pivot is clamped to
   zero and counted.  xi = L nu. */
static int noise_from_normals(const lbo_params *p, double rho, double cs2, const double nu[6],
                              double xi[Q])
{
    double X[Q][Q], L[6][6];
    int clamped = 0;
    noise_covariance(p, rho, cs2, X);
    memset(L, 0, sizeof(L));
    for (int r = 0; r < 6; r++) {
        for (int c = 0; c <= r; c++) {
            double s = X[3 + r][3 + c];
            for (int k = 0; k < c; k++) s -= L[r][k] * L[c][k];
            if (r == c) {
                if (s < 0.0) { s = 0.0; clamped = 1; }
                L[r][r] = sqrt(s);
            } else {
                L[r][c] = (L[c][c] > 0.0) ? s / L[c][c] : 0.0;
            }
        }
    }
    for (int a = 0; a < 3; a++) xi[a] = 0.0;
    for (int r = 0; r < 6; r++) {
        double s = 0.0;
        for (int c = 0; c <= r; c++) s += L[r][c] * nu[c];
        xi[3 + r] = s;
    }
    return clamped;
}

/* samples of xi for given (rho, c_s^2) over nodes [0, n): statistical pin of the noise */
void lbo_noise_samples(const lbo_params *p, double rho, double cs2, uint64_t t, int64_t n,
                       double *xi_out)
{
    build_tables();
    for (int64_t k = 0; k < n; k++) {
        double nu[6];
        lbo_normals(p->seed, (uint32_t)k, p->replica, t, nu);
        noise_from_normals(p, rho, cs2, nu, xi_out + Q * k);
    }
}

/* ---------------------------------------------------------------- initial state */

static double initial_density(const lbo_params *p, int x, int y)
{
    const double PI = 3.14159265358979323846;
    switch (p->init_kind) {
    case LBO_INIT_SLAB: {
        double rin = p->init_arg[0], rout = p->init_arg[1];
        double y1 = p->init_arg[2], y2 = p->init_arg[3], w = p->init_arg[4];
        return rout + 0.5 * (rin - rout) * (tanh((y - y1) / w) - tanh((y - y2) / w));
    }
    case LBO_INIT_RANDOM: {
        double nu[6];
        lbo_normals(p->seed, (uint32_t)idx(p, x, y), p->replica, UINT64_MAX, nu);
        return p->rho0 + p->init_arg[0] * nu[0];
    }
    case LBO_INIT_WAVE: {
        double th = 2.0 * PI * (p->init_arg[0] * x / p->nx + p->init_arg[1] * y / p->ny);
        return p->rho0 + p->init_arg[2] * cos(th);
    }
    default:
        return p->rho0;
    }
}

static void initial_velocity(const lbo_params *p, int x, int y, double *ux, double *uy)
{
    const double PI = 3.14159265358979323846;
    *ux = 0.0;
    *uy = 0.0;
    if (p->init_kind == LBO_INIT_WAVE) {
        double th = 2.0 * PI * (p->init_arg[0] * x / p->nx + p->init_arg[1] * y / p->ny);
        *ux = p->init_arg[5] + p->init_arg[3] * cos(th);   /* arg[5]: uniform base flow along x */
        *uy = p->init_arg[4] * cos(th);
    }
}

/* f(r, 0) = T^-1 m^eq(rho_init, u_init, grad rho_init, lap rho_init) */
void lbo_init(const lbo_params *p, double *f)
{
    build_tables();
    int64_t n = (int64_t)p->nx * p->ny;
    double *rho = malloc(sizeof(double) * n), *lap = malloc(sizeof(double) * n);
    double *gx = malloc(sizeof(double) * n), *gy = malloc(sizeof(double) * n);
    for (int y = 0; y < p->ny; y++)
        for (int x = 0; x < p->nx; x++) rho[idx(p, x, y)] = initial_density(p, x, y);
    lbo_stencils(p, rho, lap, gx, gy);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; y++) {
        for (int x = 0; x < p->nx; x++) {
            int64_t k = idx(p, x, y);
            double ux, uy, meq[Q];
            initial_velocity(p, x, y, &ux, &uy);
            equilibrium(p, rho[k], rho[k] * ux, rho[k] * uy, lap[k], gx[k], gy[k], meq);
            for (int i = 0; i < Q; i++) {
                double s = 0.0;
                for (int a = 0; a < Q; a++) s += Ti[i][a] * meq[a];
                f[(int64_t)i * n + k] = s;
            }
        }
    }
    free(rho); free(lap); free(gx); free(gy);
}

/* ---------------------------------------------------------------- time stepping */

/* Advance f (pre-collision, [9][ny][nx]) from time t0 by nsteps.
   flags[0] += nodes with a clamped noise pivot, flags[1] += nodes with rho <= 0. */
void lbo_step(const lbo_params *p, double *f, int64_t nsteps, uint64_t t0, int64_t flags[2])
{
    build_tables();
    int64_t n = (int64_t)p->nx * p->ny;
    double *fn = malloc(sizeof(double) * Q * n);
    double *rho = malloc(sizeof(double) * n), *lap = malloc(sizeof(double) * n);
    double *gx = malloc(sizeof(double) * n), *gy = malloc(sizeof(double) * n);
    double lam[Q];
    for (int a = 0; a < Q; a++) lam[a] = lam_of(p, a);
    int64_t nclamp = 0, nneg = 0;

    for (int64_t s = 0; s < nsteps; s++) {
        uint64_t t = t0 + (uint64_t)s;
        /* 1. density */
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < n; k++) {
            double r = 0.0;
            for (int i = 0; i < Q; i++) r += f[(int64_t)i * n + k];
            rho[k] = r;
        }
        /* 2. stencils */
        lbo_stencils(p, rho, lap, gx, gy);
        /* 3-8. collide and stream */
#pragma omp parallel for schedule(static) reduction(+ : nclamp, nneg)
        for (int y = 0; y < p->ny; y++) {
            for (int x = 0; x < p->nx; x++) {
                int64_t k = idx(p, x, y);
                double fl[Q], m[Q], meq[Q], xi[Q], ms[Q];
                for (int i = 0; i < Q; i++) fl[i] = f[(int64_t)i * n + k];
                for (int a = 0; a < Q; a++) {
                    double s2 = 0.0;
                    for (int i = 0; i < Q; i++) s2 += Tm[a][i] * fl[i];
                    m[a] = s2;
                }
                equilibrium(p, rho[k], m[1], m[2], lap[k], gx[k], gy[k], meq);
                for (int a = 0; a < Q; a++) xi[a] = 0.0;
                if (p->kT > 0.0) {
                    double nu[6];
                    double r = rho[k];
                    if (r <= 0.0) { nneg++; r = 0.0; }
                    lbo_normals(p->seed, (uint32_t)k, p->replica, t, nu);
                    nclamp += noise_from_normals(p, r, sound_speed_sq(p, r), nu, xi);
                }
                for (int a = 0; a < Q; a++) ms[a] = m[a] + lam[a] * (m[a] - meq[a]) + xi[a];
                for (int i = 0; i < Q; i++) {
                    double v = 0.0;
                    for (int a = 0; a < Q; a++) v += Ti[i][a] * ms[a];
                    fn[(int64_t)i * n + idx(p, x + CX[i], y + CY[i])] = v;
                }
            }
        }
        memcpy(f, fn, sizeof(double) * Q * n);
    }
    if (flags) { flags[0] += nclamp; flags[1] += nneg; }
    free(fn); free(rho); free(lap); free(gx); free(gy);
}

/* One step with externally supplied noise of modes 4 and 9 (correlated noise): xi4, xi9
   are [ny][nx] fields for time t; modes 5..8 use the k-independent diagonal of Xi at the
   homogeneous state (rho0, c_s^2(rho0)) with the normals nu_5..nu_8 of (seed, node,
   replica, t). */
void lbo_step_fields(const lbo_params *p, double *f, uint64_t t, const double *xi4, const double *xi9)
{
    build_tables();
    int64_t n = (int64_t)p->nx * p->ny;
    double *fn = malloc(sizeof(double) * Q * n);
    double *rho = malloc(sizeof(double) * n), *lap = malloc(sizeof(double) * n);
    double *gx = malloc(sizeof(double) * n), *gy = malloc(sizeof(double) * n);
    double lam[Q], X[Q][Q];
    for (int a = 0; a < Q; a++) lam[a] = lam_of(p, a);
    noise_covariance(p, p->rho0, sound_speed_sq(p, p->rho0), X);
    for (int64_t k = 0; k < n; k++) {
        double r = 0.0;
        for (int i = 0; i < Q; i++) r += f[(int64_t)i * n + k];
        rho[k] = r;
    }
    lbo_stencils(p, rho, lap, gx, gy);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; y++) {
        for (int x = 0; x < p->nx; x++) {
            int64_t k = idx(p, x, y);
            double fl[Q], m[Q], meq[Q], xi[Q], ms[Q], nu[6];
            for (int i = 0; i < Q; i++) fl[i] = f[(int64_t)i * n + k];
            for (int a = 0; a < Q; a++) {
                double s2 = 0.0;
                for (int i = 0; i < Q; i++) s2 += Tm[a][i] * fl[i];
                m[a] = s2;
            }
            equilibrium(p, rho[k], m[1], m[2], lap[k], gx[k], gy[k], meq);
            lbo_normals(p->seed, (uint32_t)k, p->replica, t, nu);
            for (int a = 0; a < Q; a++) xi[a] = 0.0;
            xi[3] = xi4[k];
            xi[8] = xi9[k];
            for (int a = 4; a < 8; a++) xi[a] = sqrt(X[a][a]) * nu[a - 3];
            for (int a = 0; a < Q; a++) ms[a] = m[a] + lam[a] * (m[a] - meq[a]) + xi[a];
            for (int i = 0; i < Q; i++) {
                double v = 0.0;
                for (int a = 0; a < Q; a++) v += Ti[i][a] * ms[a];
                fn[(int64_t)i * n + idx(p, x + CX[i], y + CY[i])] = v;
            }
        }
    }
    memcpy(f, fn, sizeof(double) * Q * n);
    free(fn); free(rho); free(lap); free(gx); free(gy);
}

/* moments m_a = sum_i T_ai f_i of the state, [9][ny][nx] */
void lbo_moments(const lbo_params *p, const double *f, double *m)
{
    build_tables();
    int64_t n = (int64_t)p->nx * p->ny;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; k++) {
        for (int a = 0; a < Q; a++) {
            double s = 0.0;
            for (int i = 0; i < Q; i++) s += Tm[a][i] * f[(int64_t)i * n + k];
            m[(int64_t)a * n + k] = s;
        }
    }
}

/* equilibrium moments for given local fields (lets tests linearise Table II) */
void lbo_equilibrium(const lbo_params *p, double rho, double jx, double jy, double lap,
                     double gx, double gy, double meq[Q])
{
    build_tables();
    equilibrium(p, rho, jx, jy, lap, gx, gy, meq);
}

double lbo_pressure(const lbo_params *p, double rho) { return bulk_pressure(p, rho); }
double lbo_sound_speed_sq(const lbo_params *p, double rho) { return sound_speed_sq(p, rho); }
