// Private declarations shared by the library's translation units (kernels + C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

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
    R dp1, dp2, dp3, dp4;   // pex(rho0 + d) - pex(rho0) = d (dp1 + d (dp2 + d (dp3 + d dp4))), with
                            // pex = p0 - rho sigma_s^2 (Taylor coefficients at rho0; exact, pex is quartic)
    R lam_b, lam_s, lam_q, lam_e;   // lambda_a = -1/tau_a
    R kT3;           // 3 kT = rho kT / sigma_s^2 per unit density
    R k44, k49, k99; // Xi(0)/(3 rho kT): (4,4) = k44 (2 - 3 c_s^2), (4,9) = k49 (c_s^2 - 1/3),
                     // (9,9) = k99 (5/4 - 3 c_s^2 / 4)
    R k44x2, k44n3, k49m, k99x125, k99n075;   // 2 k44, -3 k44, -k49/3, 5/4 k99, -3/4 k99
    R c0sq, B3;      // c0sq, 3 B: c_s^2 = c0sq + rho (A + 3 B x^2)
    R l55, l66, l77, l88;   // sqrt of Xi(0)_aa / (3 rho kT), a = 5..8
    R sq0;           // sqrt(3 kT rho0): noise scale of the homogeneous state (correlated noise)
    R cs2_0;         // c_s^2(rho0)
    R sub[9];        // df_i = s_i - sub_i (see RepDesc)
};

// Per-replica description, uploaded once by lb_init.  The populations of replica r live
// at element offset `off` of each population buffer, row-interleaved: element (i, x, y)
// at ((y * 9) + i) * nx + x, so that the nine populations of a lattice row are one
// contiguous 9 nx block (pop_at).
// Stored value s_i and population f_i are related by f_i = s_i + shift_i; kernels work
// on the deviation df_i = f_i - fbar_i = s_i - sub_i with sub_i = fbar_i - shift_i, where
// fbar = T^-1 m^eq(rho0, u = 0) is the model's rest state (Table II at rest: w_i rho0 when
// p0(rho0) = rho0 sigma_s^2).  shift = fbar for the shifted storages, 0 for LB_FP32.
struct RepDesc {
    int32_t nx, ny;
    int64_t off;          // element offset of plane 0 in a population buffer
    int64_t node_off;     // node offset of this replica in replica-concatenated node arrays
    uint32_t seed_lo, seed_hi, rep_id;
    uint32_t noise;       // 0: none (kT = 0); 1: Xi(0) at the local state; 2: correlated Xi(k);
                          // 3: the diagonal of Xi(0) at the local state
    int32_t lognx, logny; // for correlated noise (powers of two)
    int64_t xi_off;       // correlated noise: offset (in pairs) of this replica's xi_4 + i xi_9 plane
    int64_t tw_off;       // correlated noise: offset (in double2) of its twiddles [nx/2 | ny/2]
    Consts<double> cd;
    Consts<float> cf;
    double shift[Q];
    int32_t init_kind, pad_;
    double init_arg[6];
};

// offset of population i of node (x, y) inside a replica's block
__host__ __device__ inline long long pop_at(int nx, int i, int x, int y)
{
    return ((long long)y * 9 + i) * nx + x;
}

// pre-collision populations f_i(x, y) = f*_i(x - c_i, y - c_iy) of node (x, y) in FP64,
// including the storage shift (generic kernels: init checks, moments, S(k) rows)
template <typename S>
__device__ inline void pull_node(const S *P, int nx, int ny, int x, int y, const double *shift, double g[9])
{
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    g[0] = (double)P[pop_at(nx, 0, x, y)] + shift[0];
    g[1] = (double)P[pop_at(nx, 1, xm, y)] + shift[1];
    g[2] = (double)P[pop_at(nx, 2, x, ym)] + shift[2];
    g[3] = (double)P[pop_at(nx, 3, xp, y)] + shift[3];
    g[4] = (double)P[pop_at(nx, 4, x, yp)] + shift[4];
    g[5] = (double)P[pop_at(nx, 5, xm, ym)] + shift[5];
    g[6] = (double)P[pop_at(nx, 6, xp, ym)] + shift[6];
    g[7] = (double)P[pop_at(nx, 7, xp, yp)] + shift[7];
    g[8] = (double)P[pop_at(nx, 8, xm, yp)] + shift[8];
}

template <typename R> __host__ __device__ inline const Consts<R> &consts(const RepDesc &d);
template <> __host__ __device__ inline const Consts<double> &consts<double>(const RepDesc &d) { return d.cd; }
template <> __host__ __device__ inline const Consts<float> &consts<float>(const RepDesc &d) { return d.cf; }

// A unit of work of the fused step: replica `rep`, columns [x0, x0 + blockDim.x)
// (wrapped modulo nx, stored only where < nx), rows [y0, y1).
struct Tile {
    int32_t rep, x0, y0, y1;
};

struct StepLaunch {
    const void *xi;     // correlated-noise planes (pairs of the storage type) or nullptr
    const void *fin;
    void *fout;
    const RepDesc *reps;
    const Tile *tiles;
    const unsigned long long *tdev;
    unsigned *flags;
    int32_t toff;
    int32_t ntiles;
    int32_t bx;
    int32_t plain;   // 1: stored values are f_i (sub_i = fbar_i); 0: stored f_i - fbar_i
    int32_t whole;   // 1: some replica fits one strip (nx <= bx): launch the whole-row variant
};

// the fused step's tiles for strips of bx lanes and tiles of about h rows (lb_tiles.hip)
std::vector<Tile> make_tiles(const std::vector<RepDesc> &reps, int bx, double h);

// Two steps per launch (lb_step2.hip).  A workgroup of bx lanes holds G lane groups of bx / G
// lanes, each running one tile: workgroup w runs tiles[wgs[w] .. wgs[w + 1]), G = their
// count.  A tile's x0 is its first output column (strips of bx / G - 6 output columns); a
// replica whose row fits a group (nx <= bx / G) has x0 = 0 and whole-row tiles; rep < 0
// marks an empty group.
struct Step2Launch {
    const void *xi;       // correlated noise of step t (plane 0) and t + 1 (at xi_plane), or null
    int64_t xi_plane;     // elements of the storage type between the two planes
    const void *fin;
    void *fout;
    const RepDesc *reps;
    const Tile *tiles;
    const int32_t *wgs;
    const unsigned long long *tdev;
    unsigned *flags;
    int32_t toff;
    int32_t nwg;
    int32_t bx;
    int32_t max_groups;   // largest G of the list (sizes the LDS)
    int32_t plain;
};
constexpr int STEP2_MIN_BX = 128, STEP2_MIN_H = 8;
// tiles and workgroup prefix of the two-step kernel for workgroups of bx lanes and tiles of
// about h rows; returns the largest group count
int make_tiles2(const std::vector<RepDesc> &reps, int bx, double h, std::vector<Tile> &tiles,
                std::vector<int32_t> &wgs);
// upper bound of the tile count of make_tiles2 for any bx >= STEP2_MIN_BX, h >= STEP2_MIN_H
long long max_tiles2(const std::vector<int> &nx, const std::vector<int> &ny);
hipError_t launch_step2(int precision, const Step2Launch &a, hipStream_t s);
size_t step2_lds_bytes(int precision, int bx, int max_groups);
// resident two-step workgroups of bx lanes (max_groups lane groups) per CU (0 if unknown)
int step2_blocks_per_cu(int precision, bool plain, bool cn, int bx, int max_groups);
// allow k_step2 the dynamic LDS of its largest configuration (512 lanes in 8 groups)
hipError_t set_step2_lds_limit();

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

// twiddles exp(-2 pi i j / n), j < n/2, as (re, im) pairs (lb_fft.hip)
hipError_t launch_twiddles(double *tw, int n, hipStream_t s);
// correlated noise of one replica for step time tdev[0] + toff: fills its xi plane, using
// `work` (nx ny complex doubles) as scratch
hipError_t launch_correlated_noise(int precision, const RepDesc *d_reps, const RepDesc &h_rep, int rep_index,
                                   double *work, const double *tw_base, void *xi_base,
                                   const unsigned long long *tdev, int toff, hipStream_t s);
// LDS limits of the correlated-noise kernels for replicas up to max_nx x max_ny
hipError_t set_fft_lds_limit(int max_nx, int max_ny);

// structure factor (lb_sk.hip).  Replicas are sampled together: every pass covers a range
// [r0, r1) of replicas with one launch per kernel, whatever their sizes.
constexpr int SK_MAX = 16384;       // largest side the sampler transforms

struct SkRep {
    int32_t nx, ny, lognx, logny;
    int32_t split;      // column blocks per kx: 1, or 2 (one per output parity) when a column does not fit
    int32_t cpb;        // adjacent kx columns per column block (1 when split)
    int32_t rpb;        // rows per row block (a power of two)
    int32_t logrpb;     // log2(rpb)
    int64_t row0;       // first row block of this replica (prefix of ceil(ny / rpb))
    int64_t col0;       // first column block (prefix of split * ceil(nh / cpb)), nh = nx/2 + 1
    int64_t soff;       // offset (complex elements) of its spectrum (sk_at layout) inside one mode slot
    int64_t acc_off;    // offset (double) of its [9][nh][ny] accumulators
};

struct SkLaunch {
    const void *f;            // current population buffer
    const RepDesc *reps;
    const SkRep *sk;          // device copy of the table
    int32_t r0, r1;           // replica range
    int64_t row_base, rows;   // row blocks of the range
    int64_t col_base, cols;
    int32_t lds_rows;         // most row points per block in the range (rpb * nx)
    int32_t lds_cols;         // most column points per block in the range (cpb * ny, or ny/2 if split)
    int32_t G;                // modes per transform group of the row kernel
    int64_t Ptot;             // complex elements per mode slot (sum of ny * sk_nh_padded(nx) over all replicas)
    void *spec;               // nine mode slots of row spectra (float2 for FP32 storage, else double2)
    double *acc;
    double *base;             // [replica][18]: reference moments (FP64) and populations of the last sample
    const double *tw;         // exp(-2 pi i j / nmax), j < nmax/2
    int32_t nmax;
};
// sampler layout policy: bytes per complex transform element (16 for FP64 storage, else 8),
// modes per row pass, column blocks per kx, adjacent kx per column block
int sk_elem(int precision);
int sk_modes_per_pass(int precision, int max_nx);
int sk_split(int precision, int ny);
int sk_cols_per_block(int precision, int nx, int ny);
hipError_t set_sk_lds_limits(int precision, int G, int max_row, int max_col);
// add |m_a(k)|^2 / n, a = 0..8, of every replica in the range to its accumulators
hipError_t launch_sk_sample(int precision, const SkLaunch &a, hipStream_t s);
// |rho(k)|^2 / n of replica a.r0 (a one-replica range), radially binned into out[0..nbins)
// (means) and out[nbins..2 nbins) (counts); P, xwide describe the bin metric
hipError_t launch_sk_snapshot(int precision, const SkLaunch &a, int nx, int ny, int nbins, int P, int xwide,
                              double *out, hipStream_t s);
hipError_t launch_sk_read(const double *acc, double *out, int nx, int ny, double inv_ns, hipStream_t s);
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s);

}  // namespace lbf
