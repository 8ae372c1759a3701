// Fourier-space helpers: twiddle tables, a fill kernel, and the spatially correlated
// noise of arXiv:1009.0254, Sec. IV (last paragraph), built each step by filtering white
// fields with the Cholesky factor of Xi(k).

#include "lb_fftcore.h"
#include "lb_internal.h"
#include "lb_rng.h"

#include <math.h>

namespace lbf {

constexpr int FFT_THREADS = 256;

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

// [rows][cols] -> [cols][rows], 32x32 tiles through LDS
__global__ void __launch_bounds__(256) k_transpose(const double2 *__restrict__ in, double2 *__restrict__ out, int rows,
                                                   int cols)
{
    __shared__ double2 tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int j = ty; j < 32; j += 8) {
        const int r = by + j, c = bx + tx;
        if (r < rows && c < cols) tile[j][tx] = in[(long long)r * cols + c];
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int c = bx + j, r = by + tx;
        if (r < rows && c < cols) out[(long long)c * rows + r] = tile[tx][j];
    }
}

// ------------------------------------------------------------------ correlated noise
// Sec. IV (last paragraph): for each step, white fields w4, w9 -> z = w4 + i w9 ->
// Z = FFT(z) -> Y(k) = a(k) Z(k) + b(k) conj(Z(-k)) -> xi4 + i xi9 = IFFT(Y) / n, with
// a = (L44 + L99 + i L94)/2, b = (L44 - L99 + i L94)/2 and L the lower Cholesky factor of
// the (4,9) block of Xi(k) (eq. noise-yeo) at the homogeneous state.  Since
// Z + conj(Z(-k)) = 2 W4 and Z - conj(Z(-k)) = 2i W9, Y = L44 W4 + i (L94 W4 + L99 W9).

__global__ void k_cn_white(double2 *__restrict__ z, const RepDesc *__restrict__ reps, int rep_index,
                           const unsigned long long *__restrict__ tdev, int toff)
{
    const RepDesc &d = reps[rep_index];
    const long long n = (long long)d.nx * d.ny;
    const unsigned long long t = tdev[0] + (unsigned long long)toff;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
        double nu[6];
        normals6<double>((uint32_t)k, d.rep_id | 0x80000000u, t, d.seed_lo, d.seed_hi, nu);
        z[k] = make_double2(nu[0], nu[1]);
    }
}

// transform every line of length L (lines are contiguous) in place
template <bool INV>
__global__ void __launch_bounds__(FFT_THREADS) k_fft_lines(double2 *__restrict__ data, int L, int logL,
                                                           const double2 *__restrict__ tw)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ TwCache T;
    double2 *X = reinterpret_cast<double2 *>(smem_raw);
    double2 *line = data + (long long)blockIdx.x * L;
    tw_cache_load(T, tw, L);
    for (int i = threadIdx.x; i < L; i += blockDim.x) X[bitrev((unsigned)i, logL)] = line[i];
    __syncthreads();
    fft_lds<INV>(X, L, logL, 1, T, L);
    for (int i = threadIdx.x; i < L; i += blockDim.x) line[i] = X[i];
}

// A, B in the transposed layout [kx][ky]
__global__ void k_cn_combine(const double2 *__restrict__ A, double2 *__restrict__ B, const RepDesc *__restrict__ reps,
                             int rep_index)
{
    const RepDesc &d = reps[rep_index];
    const Consts<double> &c = d.cd;
    const int nx = d.nx, ny = d.ny;
    const long long n = (long long)nx * ny;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
        const int kx = (int)(k / ny), ky = (int)(k - (long long)kx * ny);
        const int mx = (nx - kx) & (nx - 1), my = (ny - ky) & (ny - 1);
        const double2 Z = A[k], Zm = A[(long long)mx * ny + my];
        // minus the App. B Laplacian symbol, and c_s^2(k) = c_s^2 + rho0 kappa k^2
        const double cx = cospi(2.0 * kx / nx), cy = cospi(2.0 * ky / ny);
        const double k2 = -3.0 * ((4.0 / 9.0) * (cx + cy) + (2.0 / 9.0) * cx * cy - 10.0 / 9.0);
        const double cs2k = c.cs2_0 + c.rho0 * c.kappa * k2;
        const double pre = c.kT3 * c.rho0;
        const double x44 = pre * c.k44 * (2.0 - 3.0 * cs2k);
        const double x49 = pre * c.k49 * (cs2k - 1.0 / 3.0);
        const double x99 = pre * c.k99 * (1.25 - 0.75 * cs2k);
        const double l44 = sqrt(fmax(x44, 0.0));
        const double l94 = l44 > 0 ? x49 / l44 : 0.0;
        const double l99 = sqrt(fmax(x99 - l94 * l94, 0.0));
        const double ar = 0.5 * (l44 + l99), br = 0.5 * (l44 - l99), ai = 0.5 * l94;
        // Y = (ar + i ai) Z + (br + i ai) conj(Zm)
        const double yr = ar * Z.x - ai * Z.y + br * Zm.x + ai * Zm.y;
        const double yi = ar * Z.y + ai * Z.x - br * Zm.y + ai * Zm.x;
        B[k] = make_double2(yr, yi);
    }
}

template <typename S>
__global__ void k_cn_store(const double2 *__restrict__ A, S *__restrict__ xi, long long n, double inv_n)
{
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
        const double2 v = A[k];
        xi[2 * k] = (S)(v.x * inv_n);
        xi[2 * k + 1] = (S)(v.y * inv_n);
    }
}

hipError_t set_fft_lds_limit(int max_line)
{
    const int bytes = (int)sizeof(double2) * max_line;
    hipError_t e = hipFuncSetAttribute((const void *)k_fft_lines<false>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_fft_lines<true>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return e;
}

hipError_t launch_correlated_noise(int precision, const RepDesc *d_reps, const RepDesc &h_rep, int rep_index,
                                   double *work_a, double *work_b, const double *tw_base, void *xi_base,
                                   const unsigned long long *tdev, int toff, hipStream_t s)
{
    const int nx = h_rep.nx, ny = h_rep.ny;
    const long long n = (long long)nx * ny;
    const double2 *twx = (const double2 *)tw_base + h_rep.tw_off;
    const double2 *twy = twx + nx / 2;
    double2 *A = (double2 *)work_a, *B = (double2 *)work_b;
    long long g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_cn_white, dim3((unsigned)g), dim3(256), 0, s, A, d_reps, rep_index, tdev, toff);
    // forward along x (rows of [ny][nx]), then along y in the transposed layout [nx][ny]
    hipLaunchKernelGGL(k_fft_lines<false>, dim3(ny), dim3(FFT_THREADS), sizeof(double2) * nx, s, A, nx, h_rep.lognx, twx);
    hipLaunchKernelGGL(k_transpose, dim3((nx + 31) / 32, (ny + 31) / 32), dim3(256), 0, s, (const double2 *)A, B, ny, nx);
    hipLaunchKernelGGL(k_fft_lines<false>, dim3(nx), dim3(FFT_THREADS), sizeof(double2) * ny, s, B, ny, h_rep.logny, twy);
    hipLaunchKernelGGL(k_cn_combine, dim3((unsigned)g), dim3(256), 0, s, (const double2 *)B, A, d_reps, rep_index);
    // inverse along y, back to [ny][nx], inverse along x
    hipLaunchKernelGGL(k_fft_lines<true>, dim3(nx), dim3(FFT_THREADS), sizeof(double2) * ny, s, A, ny, h_rep.logny, twy);
    hipLaunchKernelGGL(k_transpose, dim3((ny + 31) / 32, (nx + 31) / 32), dim3(256), 0, s, (const double2 *)A, B, nx, ny);
    hipLaunchKernelGGL(k_fft_lines<true>, dim3(ny), dim3(FFT_THREADS), sizeof(double2) * nx, s, B, nx, h_rep.lognx, twx);
    const double inv_n = 1.0 / (double)n;
    if (precision == 0)
        hipLaunchKernelGGL(k_cn_store<double>, dim3((unsigned)g), dim3(256), 0, s, (const double2 *)B,
                           (double *)xi_base + 2 * h_rep.xi_off, n, inv_n);
    else
        hipLaunchKernelGGL(k_cn_store<float>, dim3((unsigned)g), dim3(256), 0, s, (const double2 *)B,
                           (float *)xi_base + 2 * h_rep.xi_off, n, inv_n);
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
