// Private declarations shared by the library's translation units (kernels + C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbf {

constexpr int Q = 9;

// Per-replica constants of the collision in the arithmetic type R of a kernel (float or
// double), so that kernels read them as scalars without conversions.
template <typename R> struct Consts {
    R rho0;
    R xr0;           // rho0 - rhoc
    R A, B;
    R c0m;           // c0sq - 1/3
    R kappa;
    R lam_b, lam_s, lam_q, lam_e;   // lambda_a = -1/tau_a
    R kT3;           // 3 kT = rho kT / sigma_s^2 per unit density
    R k44, k49, k99; // Xi(0)/(3 rho kT): (4,4) = k44 (2 - 3 c_s^2), (4,9) = k49 (c_s^2 - 1/3),
                     // (9,9) = k99 (5/4 - 3 c_s^2 / 4)
    R l55, l66, l77, l88;   // sqrt of Xi(0)_aa / (3 rho kT), a = 5..8
    R sub[9];        // df_i = s_i - sub_i (see RepDesc)
};

// Per-replica description, uploaded once by lb_init.  The populations of replica r live
// at element offset `off` of each population buffer as planes [9][ny][nx].
// Stored value s_i and population f_i are related by f_i = s_i + shift_i; kernels work
// on the deviation df_i = f_i - w_i rho0 = s_i - sub_i with sub_i = w_i rho0 - shift_i.
struct RepDesc {
    int32_t nx, ny;
    int64_t off;          // element offset of plane 0 in a population buffer
    int64_t node_off;     // node offset of this replica in replica-concatenated node arrays
    uint32_t seed_lo, seed_hi, rep_id, noise;
    Consts<double> cd;
    Consts<float> cf;
    double shift[Q];
    int32_t init_kind, pad_;
    double init_arg[6];
};

template <typename R> __host__ __device__ inline const Consts<R> &consts(const RepDesc &d);
template <> __host__ __device__ inline const Consts<double> &consts<double>(const RepDesc &d) { return d.cd; }
template <> __host__ __device__ inline const Consts<float> &consts<float>(const RepDesc &d) { return d.cf; }

// A unit of work of the fused step: replica `rep`, columns [x0, x0 + blockDim.x)
// (wrapped modulo nx, stored only where < nx), rows [y0, y1).
struct Tile {
    int32_t rep, x0, y0, y1;
};

struct StepLaunch {
    const void *fin;
    void *fout;
    const RepDesc *reps;
    const Tile *tiles;
    const unsigned long long *tdev;
    unsigned *flags;
    int32_t toff;
    int32_t ntiles;
    int32_t bx;
};

// launchers (lb_kernels.hip); all return hipSuccess or the launch error
hipError_t launch_step(int precision, const StepLaunch &a, hipStream_t s);
hipError_t launch_advance_time(unsigned long long *tdev, long long by, hipStream_t s);
hipError_t launch_init(int precision, void *f, double *rho_tmp, const RepDesc *d_reps,
                       const RepDesc &h_rep, int rep_index, hipStream_t s);
hipError_t launch_moments(int precision, const void *f, const RepDesc *d_reps, const RepDesc &h_rep,
                          int rep_index, double *d_m9, double *partials, int nblocks, double *d_tot,
                          hipStream_t s);
hipError_t launch_normals(uint64_t seed, uint32_t replica, uint64_t t, int64_t n, int precision,
                          double *d_out, hipStream_t s);
hipError_t launch_philox(uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1, int64_t n,
                         uint32_t *d_out, hipStream_t s);

// structure factor (lb_fft.hip)
struct SkPlan {
    int nx, ny;
    int lognx, logny;
    double *twx, *twy;      // twiddles exp(-2 pi i k / n), k < n/2, as (re, im) pairs
};
hipError_t launch_twiddles(double *tw, int n, hipStream_t s);
hipError_t launch_sk_sample(int precision, const void *f, const RepDesc *d_reps, const RepDesc &h_rep,
                            int rep_index, const SkPlan &plan, double *work_a, double *work_b,
                            double *acc, hipStream_t s);
hipError_t launch_sk_read(const double *acc, double *out, int nx, int ny, double inv_ns, hipStream_t s);
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s);

}  // namespace lbf
