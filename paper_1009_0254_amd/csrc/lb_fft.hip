// Fourier-space helpers: twiddle tables, a fill kernel, and the spatially correlated
// noise of arXiv:1009.0254, Sec. IV (last paragraph), built each step by filtering white
// fields with the Cholesky factor of Xi(k).

#include "lb_fftcore.h"
#include "lb_internal.h"
#include "lb_rng.h"

#include <math.h>

#include <type_traits>

namespace lbf {


__global__ void k_twiddles(double2 *tw, int n)
{
    const int half = n / 2;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < half; k += gridDim.x * blockDim.x) {
        double s, c;
        sincospi(-2.0 * (double)k / (double)n, &s, &c);
        tw[k] = make_double2(c, s);
    }
}

__global__ void k_fill(double *p, long long n, double v)
{
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
        p[k] = v;
}

// ------------------------------------------------------------------ correlated noise
// Sec. IV (last paragraph): the noise is built in Fourier space and transformed back once
// per step.  At every lattice k, xi(k) = L(k) nu(k) with L the lower Cholesky factor of the
// (4,9) block of Xi(k) (eq. noise-yeo at the homogeneous state; modes 5..8 do not depend on
// k and stay per node in the step kernel) and nu(k) unit Gaussians with nu(-k) = conj nu(k):
// complex (g0 + i g1)/sqrt2, (g2 + i g3)/sqrt2 where k != -k, real g0, g1 where k = -k.  The
// pair k, -k uses the Philox block of the member with the smaller index ky nx + kx (counter
// (index, replica | 2^31, t)); the other member takes the conjugate.  Both real fields go
// back in one complex transform: xi_4 + i xi_9 = n^-1/2 sum_k exp(-i k.r) (xi_4(k) + i xi_9(k)),
// taken along ky in the kernel that draws the noise and then along kx in the kernel that
// stores the fields.
//
// The intermediate plane between the two passes is stored in chunks of CH = min(4, ny) rows:
// element (kx, y) at ((y / CH) nx + kx) CH + y mod CH.  The drawing kernel writes each column as
// runs of CH contiguous elements; the storing kernel reads two rows across kx from one contiguous
// region of nx CH elements, one 16-byte piece per kx at a stride of CH elements, so that a wave's
// reads touch 16 cache lines.  (At 8192^2: 16-row chunks, whose rows all read different lines,
// made the storing kernel 0.52 ms; 4-row chunks 0.41 ms, for 0.01 ms more in the drawing kernel,
// whose writes become 32-byte pieces; 2-row chunks moved the cost there.)

constexpr int CN_THREADS = 1024;
constexpr int CN_COL_POINTS = 4096;   // points per drawing block when columns are short
constexpr int CN_LDS_POINT_BYTES = 131072;   // largest transform batch of one block, in bytes (before its 1/16 pad)

int cn_threads(int points) { return points >= 4096 ? 1024 : 256; }

// Work of one drawing block.  Conjugate partners k, -k share one set of normals, so a block
// holds whole mirror pairs of columns when two columns fit in its LDS: pair p (0 < p < nx/2)
// is columns p and nx - p, pair 0 the two self-conjugate columns 0 and nx/2.  Otherwise
// (FP64 columns of 8192 points) a block holds one column, and each conjugate pair's normals
// are drawn once by each of its two blocks.
// rows per storing block: two adjacent rows when they fit
int cn_out_rows(int nx, size_t elem) { return 2 * (size_t)nx * elem <= (size_t)CN_LDS_POINT_BYTES ? 2 : 1; }

struct CnGen {
    bool paired;
    int per_block;   // pairs (paired) or columns per block
    int blocks;
    int points;      // transform points held by a block
};
CnGen cn_gen_shape(int nx, int ny, size_t elem)
{
    CnGen g;
    g.paired = 2 * (size_t)ny * elem <= (size_t)CN_LDS_POINT_BYTES;
    if (g.paired) {
        const int want = ny >= CN_COL_POINTS / 2 ? 1 : CN_COL_POINTS / (2 * ny);
        g.per_block = want < nx / 2 ? want : nx / 2;
        g.blocks = (nx / 2) / g.per_block;
        g.points = 2 * g.per_block * ny;
    } else {
        g.per_block = 1;
        g.blocks = nx;
        g.points = ny;
    }
    return g;
}

// cos(2 pi j / n) for j < n: FP64 for FP64 storage; the hardware cosine (argument in
// revolutions) in FP32
template <typename R> __device__ __forceinline__ R cos_2pi(int j, int n);
template <> __device__ __forceinline__ double cos_2pi<double>(int j, int n) { return cospi(2.0 * j / n); }
template <> __device__ __forceinline__ float cos_2pi<float>(int j, int n)
{
    return __builtin_amdgcn_cosf((float)j / (float)n);
}
__device__ __forceinline__ double sqrt_r(double v) { return sqrt(v); }
__device__ __forceinline__ float sqrt_r(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ double div_r(double a, double b) { return a / b; }
__device__ __forceinline__ float div_r(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// the first four normals of Philox block (idx, rep, t): the Box-Muller pairs of the top 21
// bits of words (0, 1) and (2, 3), as drawn for the per-node noise
template <typename R>
__device__ __forceinline__ void normals4(uint32_t idx, uint32_t rep, unsigned long long t, uint32_t k0, uint32_t k1,
                                         R g[4])
{
    const uint4 x = philox10(make_uint4(idx, rep, (uint32_t)t, (uint32_t)(t >> 32)), k0, k1);
    Gauss<R>::pair(x.x >> 11, x.y >> 11, g[0], g[1]);
    Gauss<R>::pair(x.z >> 11, x.w >> 11, g[2], g[3]);
}
template <typename R>
__device__ __forceinline__ void normals2(uint32_t idx, uint32_t rep, unsigned long long t, uint32_t k0, uint32_t k1,
                                         R &g0, R &g1)
{
    const uint4 x = philox10(make_uint4(idx, rep, (uint32_t)t, (uint32_t)(t >> 32)), k0, k1);
    Gauss<R>::pair(x.x >> 11, x.y >> 11, g0, g1);
}

// Cholesky factor of the (4,9) block of Xi(k) at k = (2 pi kx / nx, 2 pi ky / ny), a function
// of |k|^2 through the App. B Laplacian symbol, so equal at k and -k.  In R: double for FP64
// storage (parity with FP64 references), float otherwise (the step consumes the fields in
// float; their rounding, ~1e-7 of the noise amplitude, is far below the FP32 normals' 3e-6).
template <typename R> struct Chol49 {
    R l44, l94, l99;
};
template <typename R>
__device__ __forceinline__ Chol49<R> cn_chol(const RepDesc &d, const Consts<R> &c, int kx, int ky)
{
    // minus the App. B Laplacian symbol, and c_s^2(k) = c_s^2 + rho0 kappa k^2
    const R cx = cos_2pi<R>(kx, d.nx), cy = cos_2pi<R>(ky, d.ny);
    const R k2 = (R)-3 * ((R)(4.0 / 9.0) * (cx + cy) + (R)(2.0 / 9.0) * cx * cy - (R)(10.0 / 9.0));
    const R cs2k = c.cs2_0 + c.rho0 * c.kappa * k2;
    const R pre = c.kT3 * c.rho0;
    const R x44 = pre * c.k44 * ((R)2 - (R)3 * cs2k);
    const R x49 = pre * c.k49 * (cs2k - (R)(1.0 / 3.0));
    const R x99 = pre * c.k99 * ((R)1.25 - (R)0.75 * cs2k);
    Chol49<R> L;
    L.l44 = sqrt_r(x44 > 0 ? x44 : (R)0);
    L.l94 = L.l44 > 0 ? div_r(x49, L.l44) : (R)0;
    const R r99 = x99 - L.l94 * L.l94;
    L.l99 = sqrt_r(r99 > 0 ? r99 : (R)0);
    return L;
}

// Z = xi_4 + i xi_9 at both members k, -k of a conjugate pair from the normals of the member
// with the smaller index `own`: sg = +1 when k is that member, -1 when -k is (xi(-k) =
// conj xi(k)).  xi_4 = l44 nu_4, xi_9 = l94 nu_4 + l99 nu_9.
template <typename R>
__device__ __forceinline__ void cn_pair(const RepDesc &d, const Chol49<R> &L, uint32_t own, R sg, unsigned long long t,
                                        typename V2<R>::type &zk, typename V2<R>::type &zmk)
{
    R g[4];
    normals4<R>(own, d.rep_id | 0x80000000u, t, d.seed_lo, d.seed_hi, g);
    const R rs = (R)0.70710678118654752440;   // 1/sqrt(2)
    const R n4r = rs * g[0], n4i = sg * (rs * g[1]), n9r = rs * g[2], n9i = sg * (rs * g[3]);
    const R x4r = L.l44 * n4r, x4i = L.l44 * n4i;
    const R x9r = L.l94 * n4r + L.l99 * n9r, x9i = L.l94 * n4i + L.l99 * n9i;
    zk = mk2(x4r - x9i, x4i + x9r);
    zmk = mk2(x4r + x9i, x9r - x4i);
}

// Z at a self-conjugate k (k = -k): real normals g0, g1
template <typename R>
__device__ __forceinline__ typename V2<R>::type cn_self(const RepDesc &d, const Chol49<R> &L, uint32_t idx,
                                                        unsigned long long t)
{
    R g0, g1;
    normals2<R>(idx, d.rep_id | 0x80000000u, t, d.seed_lo, d.seed_hi, g0, g1);
    return mk2(L.l44 * g0, L.l94 * g0 + L.l99 * g1);
}

// Z at any k, drawing the normals of its pair (the unpaired drawing blocks)
template <typename R>
__device__ __forceinline__ typename V2<R>::type cn_z(const RepDesc &d, const Consts<R> &c, int kx, int ky,
                                                     unsigned long long t)
{
    const int nx = d.nx, ny = d.ny;
    const int mx = (nx - kx) & (nx - 1), my = (ny - ky) & (ny - 1);
    const uint32_t idx = (uint32_t)ky * nx + kx, midx = (uint32_t)my * nx + mx;
    const Chol49<R> L = cn_chol<R>(d, c, kx, ky);
    if (idx == midx) return cn_self<R>(d, L, idx, t);
    typename V2<R>::type zk, zmk;
    cn_pair<R>(d, L, idx < midx ? idx : midx, idx < midx ? (R)1 : (R)-1, t, zk, zmk);
    return zk;
}

// `count` transforms of length n = 2^logn in the 1/16-pad layout: radix 16, remainder last; the
// lengths of the large lattices with compile-time strides
template <typename R>
__device__ __forceinline__ void cn_fft(typename V2<R>::type *X, int logn, int count, const TwCacheT<R> &T, int n)
{
    if (logn == 13)
        fft_lds_c<false, R, 4, true, 13, LDS_PAD16>(X, count, T, n);
    else if (logn == 12)
        fft_lds_c<false, R, 4, true, 12, LDS_PAD16>(X, count, T, n);
    else
        fft_lds<false, R, 4, true>(X, n, logn, count, T, n, LDS_PAD16);
}

// the intermediate plane's chunk length and element index
__device__ __forceinline__ int cn_chunk_log(int logny) { return logny < 2 ? logny : 2; }
__device__ __forceinline__ long long cn_a_at(int kx, int y, int nx, int lch)
{
    return ((((long long)(y >> lch) * nx) + kx) << lch) | (y & ((1 << lch) - 1));
}

// Columns first: Z(k) of the block's columns, transformed along ky in LDS (in the storage
// precision R), stored to the intermediate plane.  PAIRED: `per` mirror pairs of columns
// (slots 2i, 2i + 1 hold pair p0 + i), each pair's normals drawn once; else `per` adjacent
// columns.
template <typename R, bool PAIRED>
__global__ void __launch_bounds__(CN_THREADS) k_cn_gen(void *__restrict__ Av, const RepDesc *__restrict__ reps,
                                                       int rep_index, int per, int nblocks,
                                                       const double2 *__restrict__ twy,
                                                       const unsigned long long *__restrict__ tdev, int toff)
{
    typedef typename V2<R>::type C;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ TwCacheT<R> T;
    C *X = reinterpret_cast<C *>(smem_raw);
    const RepDesc &d = reps[rep_index];
    const Consts<R> &c = consts<R>(d);
    const int nx = d.nx, ny = d.ny, logny = d.logny, half = nx >> 1;
    const long long lb = xcd_logical(nblocks);
    if (lb < 0) return;
    const int first = (int)lb * per;
    const unsigned long long t = tdev[0] + (unsigned long long)toff;
    tw_cache_load(T, twy, ny);
    // 1/16-pad layout, filled in destination order: lane e writes slot e of the bit-reversed
    // column (its ky is bitrev(e)), radix-16 passes with the remainder last
    const int sh = LDS_PAD16;
    const int cols = PAIRED ? 2 * per : per;
    if (PAIRED) {
        const int hy = ny >> 1;
        for (int e = threadIdx.x; e < (per << logny); e += blockDim.x) {
            const int i = e >> logny, r = e & (ny - 1), p = first + i;
            const int s0 = (2 * i) << logny, s1 = (2 * i + 1) << logny;
            if (p > 0) {
                // k = (p, j) and -k = (nx - p, ny - j mod ny), j = bitrev(r)
                const int j = (int)bitrev((unsigned)r, logny), my = (ny - j) & (ny - 1);
                const uint32_t idx = (uint32_t)j * nx + p, midx = (uint32_t)my * nx + (nx - p);
                const Chol49<R> L = cn_chol<R>(d, c, p, j);
                C zk, zmk;
                cn_pair<R>(d, L, idx < midx ? idx : midx, idx < midx ? (R)1 : (R)-1, t, zk, zmk);
                X[lds_at(s0 + r, sh)] = zk;
                X[lds_at(s1 + bitrev((unsigned)my, logny), sh)] = zmk;
            } else {
                // columns 0 (slot 0, threads r < ny/2) and nx/2 (slot 1): each column is its own
                // mirror; thread q > 0 takes ky = q and ny - q, thread 0 the real ky = 0, ny/2
                const int kx = r < hy ? 0 : half, sb = r < hy ? s0 : s1, q = r & (hy - 1);
                if (q > 0) {
                    const Chol49<R> L = cn_chol<R>(d, c, kx, q);
                    C zk, zmk;
                    cn_pair<R>(d, L, (uint32_t)q * nx + kx, (R)1, t, zk, zmk);
                    X[lds_at(sb + bitrev((unsigned)q, logny), sh)] = zk;
                    X[lds_at(sb + bitrev((unsigned)(ny - q), logny), sh)] = zmk;
                } else {
                    X[lds_at(sb, sh)] = cn_self<R>(d, cn_chol<R>(d, c, kx, 0), (uint32_t)kx, t);
                    X[lds_at(sb + bitrev((unsigned)hy, logny), sh)] =
                        cn_self<R>(d, cn_chol<R>(d, c, kx, hy), (uint32_t)hy * nx + kx, t);
                }
            }
        }
    } else {
        for (int e = threadIdx.x; e < (cols << logny); e += blockDim.x) {
            const int cc = e >> logny, ky = (int)bitrev((unsigned)(e & (ny - 1)), logny);
            X[lds_at(e, sh)] = cn_z<R>(d, c, first + cc, ky, t);
        }
    }
    __syncthreads();
    cn_fft<R>(X, logny, cols, T, ny);
    C *A = reinterpret_cast<C *>(Av);
    const int lch = cn_chunk_log(logny);
    for (int e = threadIdx.x; e < (cols << logny); e += blockDim.x) {
        const int sl = e >> logny, y = e & (ny - 1);
        int kx = first + sl;
        if (PAIRED) {
            const int p = first + (sl >> 1);
            kx = (sl & 1) ? (p > 0 ? nx - p : half) : p;
        }
        A[cn_a_at(kx, y, nx, lch)] = X[lds_at(e, sh)];
    }
}

// Rows second: ROWS adjacent rows y0 = ROWS * block (in one chunk) of the intermediate plane,
// read across kx as one ROWS-element vector per kx from one contiguous region of nx CH
// elements, transformed along kx, scaled by n^-1/2 and stored as the xi_4, xi_9 pairs of the
// rows (contiguous).  Consecutive blocks, which read the same cache lines, run at the same
// time on one XCD.  Two rows per block when they fit: the gather is bound by the number of
// requests (one per lane and kx), which the second row halves.
template <typename S, int ROWS>
__global__ void __launch_bounds__(CN_THREADS) k_cn_out(const void *__restrict__ Av, S *__restrict__ xi,
                                                       const RepDesc *__restrict__ reps, int rep_index,
                                                       const double2 *__restrict__ twx)
{
    typedef typename V2<S>::type C;
    typedef typename std::conditional<sizeof(S) == 4, float4, double4>::type Q;
    constexpr int U = 8;   // loads in flight per lane
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ TwCacheT<S> T;
    C *X = reinterpret_cast<C *>(smem_raw);
    const C *A = reinterpret_cast<const C *>(Av);
    const RepDesc &d = reps[rep_index];
    const int nx = d.nx, ny = d.ny, lognx = d.lognx;
    const long long lr = xcd_logical(ny / ROWS);
    if (lr < 0) return;
    const int y0 = (int)lr * ROWS;
    tw_cache_load(T, twx, nx);
    const int sh = LDS_PAD16, lch = cn_chunk_log(d.logny);
    const C *src = A + cn_a_at(0, y0, nx, lch);   // element kx of row y0 + r at src[(kx << lch) + r]
    // destination order: lane e fills slot e of each row's bit-reversed transform from kx = bitrev(e)
    for (int k0 = threadIdx.x; k0 < nx; k0 += U * blockDim.x) {
        C v[U][ROWS];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long kx = bitrev((unsigned)min(k0 + u * (int)blockDim.x, nx - 1), lognx);
            if constexpr (ROWS == 2) {
                const Q q = *reinterpret_cast<const Q *>(src + (kx << lch));
                v[u][0] = mk2(q.x, q.y);
                v[u][ROWS - 1] = mk2(q.z, q.w);
            } else {
                v[u][0] = src[kx << lch];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = k0 + u * (int)blockDim.x;
            if (e < nx)
#pragma unroll
                for (int r = 0; r < ROWS; ++r) X[lds_at((r << lognx) + e, sh)] = v[u][r];
        }
    }
    __syncthreads();
    cn_fft<S>(X, lognx, ROWS, T, nx);
    const S s = (S)rsqrt((double)nx * (double)ny);
    C *out = reinterpret_cast<C *>(xi + 2 * d.xi_off) + (long long)y0 * nx;
    for (int e = threadIdx.x; e < ROWS * nx; e += blockDim.x) {
        const C v = X[lds_at(e, sh)];
        out[e] = mk2(v.x * s, v.y * s);
    }
}

template <typename R> static hipError_t set_cn_limits(int max_nx, int max_ny)
{
    typedef typename V2<R>::type C;
    const CnGen g = cn_gen_shape(max_nx, max_ny, sizeof(C));
    const int gb = (int)(sizeof(C) * lds_padded16(g.points));
    const int ob = (int)(sizeof(C) * lds_padded16((long long)cn_out_rows(max_nx, sizeof(C)) * max_nx));
    hipError_t e = hipFuncSetAttribute((const void *)k_cn_gen<R, true>, hipFuncAttributeMaxDynamicSharedMemorySize, gb);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_cn_gen<R, false>, hipFuncAttributeMaxDynamicSharedMemorySize, gb);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_cn_out<R, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, ob);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_cn_out<R, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, ob);
    return e;
}

// the dynamic LDS of a block grows with nx and ny, so the largest sides bound every replica's
hipError_t set_fft_lds_limit(int max_nx, int max_ny)
{
    hipError_t e = set_cn_limits<double>(max_nx, max_ny);
    return e == hipSuccess ? set_cn_limits<float>(max_nx, max_ny) : e;
}

template <typename R>
static void launch_cn_t(const RepDesc *d_reps, const RepDesc &h, int rep_index, double *work, const double2 *twx,
                        const double2 *twy, R *xi, const unsigned long long *tdev, int toff, hipStream_t s)
{
    typedef typename V2<R>::type C;
    const CnGen g = cn_gen_shape(h.nx, h.ny, sizeof(C));
    const size_t gb = sizeof(C) * lds_padded16(g.points);
    if (g.paired)
        hipLaunchKernelGGL((k_cn_gen<R, true>), dim3(xcd_grid(g.blocks)), dim3(cn_threads(g.points)), gb,
                           s, (void *)work, d_reps, rep_index, g.per_block, g.blocks, twy, tdev, toff);
    else
        hipLaunchKernelGGL((k_cn_gen<R, false>), dim3(xcd_grid(g.blocks)), dim3(cn_threads(g.points)),
                           gb, s, (void *)work, d_reps, rep_index, g.per_block, g.blocks, twy, tdev, toff);
    const int rows = cn_out_rows(h.nx, sizeof(C));
    const size_t ob = sizeof(C) * lds_padded16((long long)rows * h.nx);
    if (rows == 2)
        hipLaunchKernelGGL((k_cn_out<R, 2>), dim3(xcd_grid(h.ny / 2)), dim3(cn_threads(2 * h.nx)), ob, s,
                           (const void *)work, xi, d_reps, rep_index, twx);
    else
        hipLaunchKernelGGL((k_cn_out<R, 1>), dim3(xcd_grid(h.ny)), dim3(cn_threads(h.nx)), ob, s, (const void *)work, xi,
                           d_reps, rep_index, twx);
}

hipError_t launch_correlated_noise(int precision, const RepDesc *d_reps, const RepDesc &h_rep, int rep_index,
                                   double *work, const double *tw_base, void *xi_base,
                                   const unsigned long long *tdev, int toff, hipStream_t s)
{
    const double2 *twx = (const double2 *)tw_base + h_rep.tw_off;
    const double2 *twy = twx + h_rep.nx / 2;
    if (precision == 0)
        launch_cn_t<double>(d_reps, h_rep, rep_index, work, twx, twy, (double *)xi_base, tdev, toff, s);
    else
        launch_cn_t<float>(d_reps, h_rep, rep_index, work, twx, twy, (float *)xi_base, tdev, toff, s);
    return hipGetLastError();
}

hipError_t launch_twiddles(double *tw, int n, hipStream_t s)
{
    const int g = (n / 2 + 255) / 256;
    hipLaunchKernelGGL(k_twiddles, dim3(g > 0 ? g : 1), dim3(256), 0, s, (double2 *)tw, n);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s)
{
    long long g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)g), dim3(256), 0, s, p, (long long)n, v);
    return hipGetLastError();
}

}  // namespace lbf
