// Private: the in-LDS FFT shared by the structure-factor sampler and the correlated-noise
// filter.  Twiddles w^t = exp(-2 pi i t / N), t < N/2, come from a table in global memory
// (tw[t]) through a 3 KiB two-level copy in LDS: w^t = hi[t / 64] lo[t % 64] with
// lo[l] = w^l and hi[h] = w^(64 h).  A transform of length n <= N uses every (N/n)-th.
#pragma once

#include <hip/hip_runtime.h>

namespace lbf {

__device__ __forceinline__ unsigned bitrev(unsigned v, int bits) { return bits > 0 ? __brev(v) >> (32 - bits) : 0u; }

// complex pairs of float or double
template <typename T> struct V2;
template <> struct V2<float> { typedef float2 type; };
template <> struct V2<double> { typedef double2 type; };

__device__ __forceinline__ double2 mk2(double x, double y) { return make_double2(x, y); }
__device__ __forceinline__ float2 mk2(float x, float y) { return make_float2(x, y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b)
{
    return mk2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return mk2(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return mk2(a.x - b.x, a.y - b.y); }

// Workgroups are dealt to the 8 XCDs round robin; give each XCD a contiguous range of
// logical indices so that neighbouring rows / columns share its L2.  Returns -1 for the
// padding workgroups of the last range (launch xcd_grid(total) workgroups).
__device__ __forceinline__ long long xcd_logical(long long total)
{
    const long long g = blockIdx.x, per = (total + 7) >> 3;
    const long long l = (g & 7) * per + (g >> 3);
    return l < total ? l : -1;
}
inline unsigned xcd_grid(long long total) { return (unsigned)(((total + 7) >> 3) << 3); }

constexpr int TW_LO = 64, TW_HI = 128;   // N <= 2 * 64 * 128 = 16384

// LDS layout of a batch of length-n transforms: element i sits at lds_at(i, sh) = i + (i >> sh)
// with sh = lds_pad_shift(log2 n), one pad slot after every 2^sh elements.  The bit-reversed
// fill sends the 64 lanes of a wave to elements n / 64 apart, which without the pad share one
// LDS bank; with it they fall into distinct banks.
__host__ __device__ constexpr int lds_pad_shift(int logn) { return logn - 6 > 5 ? logn - 6 : 5; }
__device__ __forceinline__ int lds_at(int i, int sh) { return i + (i >> sh); }
// LDS elements that hold `total` elements of transforms of any length (pad at most 1/32)
constexpr long long lds_padded(long long total) { return total + (total >> 5) + 1; }

template <typename T> struct TwCacheT {
    typedef typename V2<T>::type C;
    C lo[TW_LO];
    C hi[TW_HI];
};
typedef TwCacheT<double> TwCache;

// fill T from tw (N/2 FP64 entries, rounded to T's precision); the caller's next barrier
// publishes it
template <typename T>
__device__ __forceinline__ void tw_cache_load(TwCacheT<T> &Tc, const double2 *__restrict__ tw, int N)
{
    const int half = N >> 1, nhi = N >= 2 * TW_LO ? N / (2 * TW_LO) : 1;
    for (int i = threadIdx.x; i < TW_LO; i += blockDim.x) {
        const double2 w = i < half ? tw[i] : make_double2(1.0, 0.0);
        Tc.lo[i] = mk2((T)w.x, (T)w.y);
    }
    for (int h = threadIdx.x; h < nhi; h += blockDim.x) {
        const double2 w = tw[h * TW_LO];
        Tc.hi[h] = mk2((T)w.x, (T)w.y);
    }
}

template <typename T>
__device__ __forceinline__ typename V2<T>::type twiddle(const TwCacheT<T> &Tc, int t)
{
    return cmul(Tc.hi[t >> 6], Tc.lo[t & (TW_LO - 1)]);
}

// `count` independent in-place decimation-in-time transforms of length n = 2^logn (n >= 2)
// stored back to back in X (through lds_at), each already in bit-reversed order, with the
// twiddles of an N-point table in T.  Pairs of radix-2 stages are fused into radix-4 passes
// (the second stage's odd twiddle is the first's times w_4 = -i), with one radix-2 pass when
// logn is odd.  INV uses the conjugate twiddles exp(+2 pi i k / n) and does not scale.  Ends
// with a barrier.
template <bool INV, typename T>
__device__ void fft_lds(typename V2<T>::type *X, int n, int logn, int count, const TwCacheT<T> &Tc, int N)
{
    typedef typename V2<T>::type C;
    const int sh = lds_pad_shift(logn);
    int s = 1;
    for (; s + 1 <= logn; s += 2) {
        const int lq = s - 1, q = 1 << lq;
        const int st1 = N >> s, st2 = N >> (s + 1);   // N / 2q and N / 4q
        const int n4 = n >> 2, total = n4 * count;
        for (int b = threadIdx.x; b < total; b += blockDim.x) {
            const int g = b >> (logn - 2), bb = b & (n4 - 1);
            const int pos = bb & (q - 1);
            const int base = g * n + ((bb >> lq) << (lq + 2)) + pos;
            const int i0 = lds_at(base, sh), i1 = lds_at(base + q, sh), i2 = lds_at(base + 2 * q, sh),
                      i3 = lds_at(base + 3 * q, sh);
            C w1 = twiddle(Tc, pos * st1), w2 = twiddle(Tc, pos * st2);
            if (INV) {
                w1.y = -w1.y;
                w2.y = -w2.y;
            }
            const C a = X[i0], bv = X[i1], c = X[i2], d = X[i3];
            const C b1 = cmul(w1, bv), d1 = cmul(w1, d);
            const C a1 = cadd(a, b1), bq = csub(a, b1), c1 = cadd(c, d1), dq = csub(c, d1);
            const C c2 = cmul(w2, c1);
            C d2 = cmul(w2, dq);
            d2 = INV ? mk2(-d2.y, d2.x) : mk2(d2.y, -d2.x);   // times +i / -i
            X[i0] = cadd(a1, c2);
            X[i2] = csub(a1, c2);
            X[i1] = cadd(bq, d2);
            X[i3] = csub(bq, d2);
        }
        __syncthreads();
    }
    if (s == logn) {
        const int half = 1 << (s - 1), st = N >> s, nb = n >> 1, total = nb * count;
        for (int b = threadIdx.x; b < total; b += blockDim.x) {
            const int g = b >> (logn - 1), bb = b & (nb - 1);
            const int pos = bb & (half - 1);
            const int e0 = g * n + ((bb >> (s - 1)) << s) + pos;
            const int i0 = lds_at(e0, sh), i1 = lds_at(e0 + half, sh);
            C w = twiddle(Tc, pos * st);
            if (INV) w.y = -w.y;
            const C u = X[i0], t = cmul(X[i1], w);
            X[i0] = cadd(u, t);
            X[i1] = csub(u, t);
        }
        __syncthreads();
    }
}

}  // namespace lbf
