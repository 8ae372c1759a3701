/*
 * lbfluct.h -- C ABI of the MI355X (gfx950) fluctuating non-ideal-fluid lattice
 * Boltzmann library.
 *
 * Model: the modified-equilibrium (Swift) D2Q9 model with thermal noise of
 * Gross, Adhikari, Cates & Varnik, "Thermal fluctuations in the lattice Boltzmann
 * method for non-ideal fluids" (arXiv:1009.0254):
 *   - velocity set, weights, moment basis T and lengths N_a: Sec. III.A, Table I, eq. (Tmat);
 *   - MRT update f_i(r + c_i, t+1) = T^-1 [m + lambda (m - m^eq) + xi]: eq. (gen-lbe-m),
 *     eq. (fluct-lin-lbe), with lambda_a = -1/tau_a (Sec. III.A);
 *   - equilibrium moments: Table II with the Galilean terms C_n = 0;
 *   - square-gradient terms: Laplacian of App. B; the gradient (the paper gives none)
 *     is the isotropic d_a rho = 3 sum_i w_i c_ia rho(r + c_i);
 *   - noise: by default spatially uncorrelated, covariance Xi(0) of eq. (noise-yeo) at
 *     k = 0, evaluated with the local density and sound speed (Sec. IV, Sec. V.B),
 *     realised as xi = L nu with L the Cholesky factor of the modes-4..9 block (Sec. IV);
 *     optionally spatially correlated with the exact Xi(k) of the homogeneous state
 *     (Sec. IV, last paragraph): modes 4 and 9 from white fields filtered in Fourier space
 *     by the Cholesky factor of their 2x2 block of Xi(k), modes 5..8 white;
 *   - nu: unit normals from Philox4x32-10 (Salmon et al., SC'11) keyed by the seed, with
 *     counter (node = y*nx + x, replica, t_lo, t_hi); the 128 bits give six 21-bit
 *     uniforms u = (b + 1/2) 2^-21 paired by Box-Muller (nu_4, nu_5), (nu_6, nu_7), (nu_8, nu_9).
 *
 * Conventions
 *   - The state "at time t" is the pre-collision (post-streaming) population f(r, t),
 *     the delta-m(t) of eq. (lb-lang-ft).  lb_moments reports that state.
 *   - Lattices are periodic, node index y*nx + x.  In device memory the populations of a
 *     replica are row-interleaved, [ny][9][nx]; moment planes returned to callers are
 *     [9][ny][nx].
 *   - Every function returns an lb_status (0 = success, < 0 = error); nothing throws
 *     or aborts.  Errors leave the handle usable unless stated otherwise.
 *   - Device memory and the stream belong to the caller.  The library never calls
 *     hipMalloc: it carves the caller's workspace.  The workspace must outlive the handle.
 *   - Functions enqueue work on the stream given to lb_init and return without
 *     waiting, except where marked "synchronous".
 *   - A handle must not be used from two host threads at once.
 */
#ifndef LBFLUCT_H
#define LBFLUCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lb_status;
enum {
    LB_OK = 0,
    LB_EINVAL = -1,     /* bad argument, size or parameter (tau <= 1/2, nx < 3, ...) */
    LB_ENOTPSD = -2,    /* Xi(0) at (rho0, c_s^2(rho0)) is not positive semi-definite (Sec. III.C) */
    LB_EUNSTABLE = -3,  /* reserved: parameters outside the stable range */
    LB_ENOMEM = -4,     /* workspace smaller than lb_workspace_size reports */
    LB_EDEVICE = -5,    /* a HIP call failed (device fault, launch error) */
    LB_ESTATE = -6      /* call not valid in the handle's state (e.g. S(k) not enabled) */
};

/* storage precision of the populations.  The shifted storages hold deviations from the
   model's rest state fbar = T^-1 m^eq(rho0, u = 0) (Table II at rest: density rho0, moment 4
   at 6 (p0(rho0) - rho0/3), moment 9 at its negative, all others zero), which is w_i rho0
   when p0(rho0) = rho0/3; the collision works on those deviations throughout. */
enum {
    LB_FP64 = 0,          /* double storage of f_i - fbar_i, double arithmetic */
    LB_FP32 = 1,          /* float storage of f_i, float arithmetic */
    LB_FP32_SHIFTED = 2   /* float storage of f_i - fbar_i, float arithmetic */
};

/* initial condition: f(r, 0) = T^-1 m^eq(rho_init, u_init) with Table II's square-gradient
   terms evaluated on rho_init */
enum {
    LB_INIT_UNIFORM = 0,  /* rho = rho0, u = 0 */
    LB_INIT_SLAB = 1,     /* rho(y) = a1 + (a0 - a1)/2 [tanh((y - a2)/a4) - tanh((y - a3)/a4)], u = 0 */
    LB_INIT_RANDOM = 2,   /* rho = rho0 + a0 * nu_4 with nu from Philox at t = 2^64 - 1, u = 0 */
    LB_INIT_WAVE = 3      /* th = 2 pi (a0 x/nx + a1 y/ny): rho = rho0 + a2 cos th,
                             u = (a5 + a3 cos th, a4 cos th) */
};

/* noise model of a replica (lb_params.noise_kind) */
enum {
    LB_NOISE_K0 = 0,          /* Xi(0) at the local rho and c_s^2(rho), uncorrelated in space */
    LB_NOISE_CORRELATED = 1,  /* exact Xi(k) at (rho0, c_s^2(rho0)); needs nx, ny powers of two
                                 in [4, 8192] and Xi(k) positive semi-definite at every lattice k */
    LB_NOISE_DIAGONAL = 2     /* the "ideal-gas-like" noise of Sec. IV: the diagonal of Xi(0) at the
                                 local rho and c_s^2, no 4-9 cross-correlation; needs only that
                                 diagonal to be non-negative */
};

/* optional features (bit mask for lb_workspace_size / lb_init) */
enum {
    LB_FEATURE_STRUCTURE_FACTOR = 1   /* reserve FFT buffers and S(k) accumulators; every
                                         replica's nx and ny must be powers of two in [4, 16384] */
};

/* lb_structure_factor operations */
enum {
    LB_SK_RESET = 0,      /* zero the accumulators of replica rep (or all, rep = -1) */
    LB_SK_SAMPLE = 1,     /* add |m_a(k)|^2 of the current state of rep (or all, rep = -1) */
    LB_SK_READ = 2,       /* copy <|m_a(k)|^2> (accumulated sum / nsamples) of rep to out */
    LB_SK_SNAPSHOT = 3    /* radially binned |rho(k)|^2 of the current state of rep (no averaging) */
};

/* device-side status flags (lb_status_flags) */
enum {
    LB_FLAG_CLAMPED_PIVOT = 1u,  /* a local Cholesky pivot of Xi(0) was negative and clamped to 0 */
    LB_FLAG_NONPOSITIVE_RHO = 2u,/* a node had rho <= 0 (its noise was set to zero) */
    LB_FLAG_NAN = 4u,            /* a node had a non-finite density */
    LB_FLAG_LOW_MACH = 8u        /* set by lb_init: some replica has kT >= 0.01 rho0 / 3, outside the
                                    small-fluctuation bound kT << sigma_s^2 rho0 of eq. (low-mach) */
};

/* One replica: a periodic nx*ny lattice with its own parameters.  The free energy
 * density is psi(rho) = c0sq rho ln rho + A/2 (rho - rhoc)^2 + B/4 (rho - rhoc)^4, so
 * p0 = rho psi' - psi and c_s^2 = rho psi'' (Sec. II.A); the paper's double well
 * beta (rho - rho_V)^2 (rho - rho_L)^2 (eq. f0-bulk) is c0sq = 0, B = 4 beta,
 * A = -beta (rho_L - rho_V)^2, rhoc = (rho_L + rho_V)/2, up to a constant. */
typedef struct lb_params {
    int32_t nx, ny;            /* lattice size, each >= 3; nx <= 2^24; nx*ny < 2^32 */
    double rho0;               /* reference density (> 0): noise-free rest state and storage shift */
    double rhoc, A, B, kappa, c0sq;
    double tau_bulk, tau_shear, tau_q, tau_eps;  /* each > 1/2 */
    double kT;                 /* >= 0; 0 gives the deterministic model */
    uint64_t seed;             /* Philox key */
    uint32_t replica;          /* Philox counter word 1: independent streams per replica, < 2^31
                                  (the white fields of correlated noise use replica | 2^31) */
    int32_t init_kind;         /* LB_INIT_* */
    int32_t noise_kind;        /* LB_NOISE_* */
    int32_t reserved;          /* must be 0 */
    double init_arg[6];
} lb_params;

typedef struct lb_handle lb_handle;

/* Bytes of device workspace needed for n_rep replicas p[0..n_rep-1] at `precision`
 * with `features`.  Host-only; no device call. */
lb_status lb_workspace_size(const lb_params *p, int32_t n_rep, int32_t precision,
                            uint32_t features, size_t *bytes);

/* Validate parameters, carve the device workspace d_workspace (>= bytes from
 * lb_workspace_size, 256-byte aligned), upload per-replica constants and write the
 * initial state f(r, 0) of every replica.  `stream` is a hipStream_t (NULL = default
 * stream).  Rejects: n_rep < 1, nx or ny < 3, rho0 <= 0, any tau <= 1/2, kT < 0,
 * unknown precision, init or noise kind, replica >= 2^31, correlated noise on a lattice
 * whose sides are not powers of two in [4, 8192] (LB_EINVAL); Xi(0) at rho0 not PSD (for
 * LB_NOISE_DIAGONAL: a negative diagonal entry), or for correlated noise Xi(k) not PSD at
 * some lattice k (LB_ENOTPSD).  It also picks the step's launch shape (lb_tuning) and
 * captures the HIP graph that lb_step replays.
 * Synchronous.  On success *out owns host memory and HIP graphs; release them with lb_free. */
lb_status lb_init(const lb_params *p, int32_t n_rep, int32_t precision, uint32_t features,
                  void *d_workspace, size_t bytes, void *stream, lb_handle **out);

/* Advance every replica by nsteps >= 0 time steps (collision with noise, then
 * streaming: eq. gen-lbe-m / fluct-lin-lbe).  Enqueued on the stream; long runs replay
 * a captured HIP graph of the fused step kernel (preceded, for replicas with correlated
 * noise, by the kernels that build that step's noise fields). */
lb_status lb_step(lb_handle *h, int64_t nsteps);

/* Moments of the current state of replica rep: if d_m9 != NULL it receives the nine
 * FP64 planes m_a(r) = sum_i T_ai f_i(r, t) as [9][ny][nx] (device pointer, caller-owned,
 * 9*nx*ny doubles).  If h_totals != NULL it receives, in FP64 and a fixed summation
 * order, { sum rho, sum j_x, sum j_y, sum |j|^2, sum (-1)^x j_x, sum (-1)^y j_y }
 * (host pointer, 6 doubles).  Synchronous. */
lb_status lb_moments(lb_handle *h, int32_t rep, double *d_m9, double *h_totals);

/* lb_moments for callers that cannot allocate device memory or hand the library scratch
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same outputs, bitwise, but the reduction's scratch -- the partial sums of
 * at most 1024 workgroups and the six totals, 48.3 KB -- lives in a fixed device array of the
 * library (one per GPU, held until the process ends, its address resolved by lb_init) instead
 * of the handle's workspace.  Allocates nothing.  Every lattice the library accepts fits that
 * scratch (its workgroups stride over the nodes); rep outside [0, n_rep) gives LB_EINVAL.
 * Calls that overlap on one GPU (two host threads, or two streams) share the array and race;
 * successive calls need no clearing (each writes all it reads).  Synchronous. */
lb_status lb_moments_static(lb_handle *h, int32_t rep, double *d_m9, double *h_totals);

/* Static structure factor of all nine modes, the equilibration measurement of Sec. V.A:
 * op = LB_SK_SAMPLE adds |m_a(k)|^2, with a(k) = n^-1/2 sum_r exp(i k.r) a(r) (Sec. III
 * notation), for k on the half plane kx = 0..nx/2, ky = 0..ny-1, to FP64 accumulators;
 * LB_SK_READ copies the mean, [9][ny][nx/2+1] FP64, to the device pointer out and the
 * sample count to *nsamples (synchronous); LB_SK_RESET zeroes.  rep = -1 addresses every
 * replica for RESET and SAMPLE (one batched pass over all of them).  The transforms run
 * in the storage precision (FP32 for LB_FP32 and LB_FP32_SHIFTED) on the moments relative
 * to a reference state (the mean of the pulled populations of row 0), so that their
 * rounding is ~1e-7 of the spectrum's scale; k = 0 and the accumulation are FP64.
 * LB_SK_SNAPSHOT (rep >= 0; synchronous) bins |rho(k)|^2 of the current state radially (an
 * isotropic average of S_rho(k), e.g. to follow density modes growing after a quench to
 * c_s^2 < 0, where M(k) of eq. lb-lang-ft has eigenvalues above 1): with L = min(nx, ny) and the shell
 * spacing 2 pi / L, k = (2 pi kx / nx, 2 pi ky / ny) falls in shell b = floor(|k| L / 2 pi + 1/2)
 * (decided in exact integer arithmetic).  *nsamples receives the number of shells nb (the
 * corner (pi, pi) lies in the last); if out != NULL (device pointer, 2 nb doubles) it
 * receives the mean of |rho(k)|^2 over each shell of the full k plane without k = 0, then
 * the number of k points in each shell.  It uses the sampler's scratch only; accumulators
 * and sample counts are untouched.
 * Needs LB_FEATURE_STRUCTURE_FACTOR at lb_init (LB_ESTATE otherwise). */
lb_status lb_structure_factor(lb_handle *h, int32_t op, int32_t rep, double *out, int64_t *nsamples);

/* S(k) sampling inside lb_step: from now on, each time lb_step brings the state to a time
 * t >= first_step with (t - first_step) divisible by every, it adds a sample of every
 * replica (as LB_SK_SAMPLE with rep = -1).  Intervals up to 256 steps are replayed as one
 * captured graph of the steps and the sample.  every = 0 switches sampling off.  Needs
 * LB_FEATURE_STRUCTURE_FACTOR for every > 0 (LB_ESTATE); every, first_step >= 0. */
lb_status lb_set_sampling(lb_handle *h, int64_t every, int64_t first_step);

/* Accumulated LB_FLAG_* bits since lb_init and the current time step t.  Synchronous. */
lb_status lb_status_flags(lb_handle *h, uint32_t *flags, int64_t *step);

/* The fused step's launch configuration chosen by lb_init: steps per launch (1: one step per
 * launch; 2: two steps per launch, the post-collision rows of the first kept on chip for the
 * second, so that HBM holds only every other state), and that kernel's workgroup (strip)
 * width in lanes, rows per tile and number of workgroups.  An odd step count ends with one
 * single-step launch.  For lattices of 2^22 nodes or more the configuration is picked by
 * timing candidates on the caller's stream (smaller ones take two steps per launch); the
 * environment variables LBF_TILE="width,rows" (one step per launch) and
 * LBF_TILE2="width,rows" (two) pin a shape, LBF_STEPS_PER_LAUNCH=1 or 2 the kernel.
 * Handles with correlated noise take one step per launch.  The configuration changes the
 * schedule only: results are bitwise identical for every shape and either kernel.
 * Host-only; any output pointer may be NULL. */
lb_status lb_tuning(lb_handle *h, int32_t *strip_width, int32_t *rows_per_tile, int32_t *ntiles,
                    int32_t *steps_per_launch);

/* The six unit normals nu_4..nu_9 (as [n][6] doubles, device pointer) that the fused
 * step draws at nodes 0..n-1 of a replica with (seed, replica) at time t, computed in
 * the arithmetic of `precision` (LB_FP64: double; otherwise float).  Lets a caller
 * check the noise stream against an independent Philox implementation. */
lb_status lb_noise_normals(uint64_t seed, uint32_t replica, uint64_t t, int64_t n,
                           int32_t precision, double *d_out, void *stream);

/* Raw Philox4x32-10 blocks for counters (i, c1, c2, c3), i = 0..n-1, key (k0, k1):
 * d_out[4*i .. 4*i+3] (device pointer).  Integer work, bit-exact by definition. */
lb_status lb_philox(uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1, int64_t n,
                    uint32_t *d_out, void *stream);

/* Release the handle's host memory and HIP graphs.  Does not touch the workspace. */
void lb_free(lb_handle *h);

/* Static string for a status code. */
const char *lb_strerror(lb_status s);

#ifdef __cplusplus
}
#endif

#endif /* LBFLUCT_H */
