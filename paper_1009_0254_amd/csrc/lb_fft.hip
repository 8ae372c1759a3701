// Fourier-space helpers: twiddle tables, a fill kernel, and the spatially correlated
// noise of arXiv:1009.0254, Sec. IV (last paragraph), built each step by filtering white
// fields with the Cholesky factor of Xi(k).

#include "lb_fftcore.h"
#include "lb_internal.h"
#include "lb_rng.h"

#include <math.h>

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
// taken along ky in the kernel that draws the noise (its columns stored contiguously) and
// then along kx in the kernel that stores the fields (its rows stored contiguously).

constexpr int CN_THREADS = 1024;
constexpr int CN_COL_POINTS = 4096;   // points per column block when columns are short

int cn_threads(int points) { return points >= 4096 ? 1024 : 256; }

// columns per column block: adjacent x, up to CN_COL_POINTS points (one column if longer)
int cn_cols_per_block(int nx, int ny) { return ny >= CN_COL_POINTS ? 1 : (CN_COL_POINTS / ny < nx ? CN_COL_POINTS / ny : nx); }

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

// Z = xi_4(k) + i xi_9(k) at k = (2 pi kx / nx, 2 pi ky / ny), step t.  The per-k Cholesky
// factors run in R: double for FP64 storage (parity with FP64 references), float otherwise
// (the step consumes the fields in float; their rounding, ~1e-7 of the noise amplitude, is
// far below the FP32 normals' 3e-6).
template <typename R>
__device__ __forceinline__ typename V2<R>::type cn_z(const RepDesc &d, const Consts<R> &c, int kx, int ky,
                                                     unsigned long long t)
{
    const int nx = d.nx, ny = d.ny;
    const int mx = (nx - kx) & (nx - 1), my = (ny - ky) & (ny - 1);
    const unsigned idx = (unsigned)ky * nx + kx, midx = (unsigned)my * nx + mx;
    R g[6];
    normals6<R>(idx < midx ? idx : midx, d.rep_id | 0x80000000u, t, d.seed_lo, d.seed_hi, g);
    const R rs = (R)0.70710678118654752440;   // 1/sqrt(2)
    R n4r, n4i, n9r, n9i;
    if (idx == midx) {
        n4r = g[0];
        n9r = g[1];
        n4i = n9i = 0;
    } else {
        const R sg = idx < midx ? (R)1 : (R)-1;
        n4r = rs * g[0];
        n4i = sg * rs * g[1];
        n9r = rs * g[2];
        n9i = sg * rs * g[3];
    }
    // minus the App. B Laplacian symbol, and c_s^2(k) = c_s^2 + rho0 kappa k^2
    const R cx = cos_2pi<R>(kx, nx), cy = cos_2pi<R>(ky, ny);
    const R k2 = (R)-3 * ((R)(4.0 / 9.0) * (cx + cy) + (R)(2.0 / 9.0) * cx * cy - (R)(10.0 / 9.0));
    const R cs2k = c.cs2_0 + c.rho0 * c.kappa * k2;
    const R pre = c.kT3 * c.rho0;
    const R x44 = pre * c.k44 * ((R)2 - (R)3 * cs2k);
    const R x49 = pre * c.k49 * (cs2k - (R)(1.0 / 3.0));
    const R x99 = pre * c.k99 * ((R)1.25 - (R)0.75 * cs2k);
    const R l44 = sqrt_r(x44 > 0 ? x44 : (R)0);
    const R l94 = l44 > 0 ? div_r(x49, l44) : (R)0;
    const R r99 = x99 - l94 * l94;
    const R l99 = sqrt_r(r99 > 0 ? r99 : (R)0);
    // xi_4 = l44 nu_4, xi_9 = l94 nu_4 + l99 nu_9
    const R x4r = l44 * n4r, x4i = l44 * n4i;
    const R x9r = l94 * n4r + l99 * n9r, x9i = l94 * n4i + l99 * n9i;
    return mk2(x4r - x9i, x4i + x9r);
}

// columns first: Z(k) of C adjacent kx columns, transformed along ky in LDS, stored to A as
// [kx][y] (each block's columns are one contiguous run).  Transforms in the storage
// precision R.
template <typename R>
__global__ void __launch_bounds__(CN_THREADS) k_cn_gen(void *__restrict__ Av, const RepDesc *__restrict__ reps,
                                                       int rep_index, int cpb, const double2 *__restrict__ twy,
                                                       const unsigned long long *__restrict__ tdev, int toff)
{
    typedef typename V2<R>::type C;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ TwCacheT<R> T;
    C *X = reinterpret_cast<C *>(smem_raw);
    const RepDesc &d = reps[rep_index];
    const Consts<R> &c = consts<R>(d);
    const int nx = d.nx, ny = d.ny, logny = d.logny;
    const long long lb = xcd_logical((nx + cpb - 1) / cpb);
    if (lb < 0) return;
    const int x0 = (int)lb * cpb, Cn = min(cpb, nx - x0);
    const unsigned long long t = tdev[0] + (unsigned long long)toff;
    tw_cache_load(T, twy, ny);
    const int tot = Cn << logny, sh = lds_pad_shift(logny);
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
        const int cc = e >> logny, ky = e & (ny - 1);
        X[lds_at(cc * ny + bitrev((unsigned)ky, logny), sh)] = cn_z<R>(d, c, x0 + cc, ky, t);
    }
    __syncthreads();
    fft_lds<false, R>(X, ny, logny, Cn, T, ny);
    C *A = reinterpret_cast<C *>(Av) + (long long)x0 * ny;
    for (int e = threadIdx.x; e < tot; e += blockDim.x) A[e] = X[lds_at(e, sh)];
}

// rows second: row y of A gathered across kx (stride ny; consecutive rows, which share
// cache lines, are kept on one XCD), transformed along kx, scaled by n^-1/2 and stored as
// the xi_4, xi_9 pairs of the row (contiguous).
template <typename S>
__global__ void __launch_bounds__(CN_THREADS) k_cn_out(const void *__restrict__ Av, S *__restrict__ xi,
                                                       const RepDesc *__restrict__ reps, int rep_index,
                                                       const double2 *__restrict__ twx)
{
    typedef typename V2<S>::type C;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ TwCacheT<S> T;
    C *X = reinterpret_cast<C *>(smem_raw);
    const C *A = reinterpret_cast<const C *>(Av);
    const RepDesc &d = reps[rep_index];
    const int nx = d.nx, ny = d.ny, lognx = d.lognx;
    const long long ly = xcd_logical(ny);
    if (ly < 0) return;
    const int y = (int)ly;
    tw_cache_load(T, twx, nx);
    const int sh = lds_pad_shift(lognx);
    for (int k0 = threadIdx.x; k0 < nx; k0 += 4 * blockDim.x) {
        C v[4];
        for (int u = 0; u < 4; ++u) v[u] = A[(long long)min(k0 + u * (int)blockDim.x, nx - 1) * ny + y];
        for (int u = 0; u < 4; ++u) {
            const int kx = k0 + u * (int)blockDim.x;
            if (kx < nx) X[lds_at(bitrev((unsigned)kx, lognx), sh)] = v[u];
        }
    }
    __syncthreads();
    fft_lds<false, S>(X, nx, lognx, 1, T, nx);
    const S s = (S)rsqrt((double)nx * (double)ny);
    C *out = reinterpret_cast<C *>(xi + 2 * d.xi_off) + (long long)y * nx;
    for (int x = threadIdx.x; x < nx; x += blockDim.x) {
        const C v = X[lds_at(x, sh)];
        out[x] = mk2(v.x * s, v.y * s);
    }
}

hipError_t set_fft_lds_limit(int max_nx, int max_col_points)
{
    const int rows = (int)(sizeof(double2) * lds_padded(max_nx)), cols = (int)(sizeof(double2) * lds_padded(max_col_points));
    hipError_t e = hipFuncSetAttribute((const void *)k_cn_out<double>, hipFuncAttributeMaxDynamicSharedMemorySize, rows);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_cn_out<float>, hipFuncAttributeMaxDynamicSharedMemorySize, rows);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_cn_gen<double>, hipFuncAttributeMaxDynamicSharedMemorySize, cols);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_cn_gen<float>, hipFuncAttributeMaxDynamicSharedMemorySize, cols);
    return e;
}

int cn_col_points(int nx, int ny) { return cn_cols_per_block(nx, ny) * ny; }

hipError_t launch_correlated_noise(int precision, const RepDesc *d_reps, const RepDesc &h_rep, int rep_index,
                                   double *work, const double *tw_base, void *xi_base,
                                   const unsigned long long *tdev, int toff, hipStream_t s)
{
    const int nx = h_rep.nx, ny = h_rep.ny;
    const double2 *twx = (const double2 *)tw_base + h_rep.tw_off;
    const double2 *twy = twx + nx / 2;
    const int cpb = cn_cols_per_block(nx, ny);
    const unsigned ncb = xcd_grid((nx + cpb - 1) / cpb);
    if (precision == 0) {
        hipLaunchKernelGGL(k_cn_gen<double>, dim3(ncb), dim3(cn_threads(cpb * ny)), sizeof(double2) * lds_padded(cpb * ny),
                           s, (void *)work, d_reps, rep_index, cpb, twy, tdev, toff);
        hipLaunchKernelGGL(k_cn_out<double>, dim3(xcd_grid(ny)), dim3(cn_threads(nx)), sizeof(double2) * lds_padded(nx),
                           s, (const void *)work, (double *)xi_base, d_reps, rep_index, twx);
    } else {
        hipLaunchKernelGGL(k_cn_gen<float>, dim3(ncb), dim3(cn_threads(cpb * ny)), sizeof(float2) * lds_padded(cpb * ny),
                           s, (void *)work, d_reps, rep_index, cpb, twy, tdev, toff);
        hipLaunchKernelGGL(k_cn_out<float>, dim3(xcd_grid(ny)), dim3(cn_threads(nx)), sizeof(float2) * lds_padded(nx),
                           s, (const void *)work, (float *)xi_base, d_reps, rep_index, twx);
    }
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
