// Private: the in-LDS FFT shared by the structure-factor sampler and the correlated-noise
// filter.  Twiddles w^t = exp(-2 pi i t / N), t < N/2, come from a table in global memory
// (tw[t]) through a 3 KiB two-level copy in LDS: w^t = hi[t / 64] lo[t % 64] with
// lo[l] = w^l and hi[h] = w^(64 h).  A transform of length n <= N uses every (N/n)-th.
// Transforms are in place, decimation in time on bit-reversed input, in passes of up to
// four radix-2 stages held in a lane's registers (radix 4, 8 or 16).
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

// LDS layout of a batch of length-n transforms: element i sits at lds_at(i, sh) = i + (i >> sh),
// one pad slot after every 2^sh elements.  Two periods are used:
//   sh = lds_pad_shift(log2 n) = max(log2 n - 6, 5): the bit-reversed fill by consecutive source
//     index sends the lanes of a wave to elements n / 64 apart, which the pad spreads over the
//     banks (the register-fed fill of the structure factor's rows);
//   sh = LDS_PAD16 = 4: for radix-16 passes with the remainder pass last (fft_lds REM_LAST) a
//     lane's 16 elements, or 16 lanes' elements of one stride, fall in 16 distinct bank pairs
//     (8-byte elements) in every pass, provided the bit-reversed fill goes in destination order
//     (lane e writes slot e, reading its source at bitrev(e)).
__host__ __device__ constexpr int lds_pad_shift(int logn) { return logn - 6 > 5 ? logn - 6 : 5; }
constexpr int LDS_PAD16 = 4;
__device__ __forceinline__ int lds_at(int i, int sh) { return i + (i >> sh); }
// LDS elements that hold `total` elements of transforms of any length (pad at most 1/32)
constexpr long long lds_padded(long long total) { return total + (total >> 5) + 1; }
// the same for the 1/16 pad
constexpr long long lds_padded16(long long total) { return total + (total >> 4) + 1; }

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

// w exp(-+2 pi i k / 16) (forward: minus; INV: plus), k a compile-time constant < 8
template <bool INV, int K, typename C> __device__ __forceinline__ C rot16(C w)
{
    constexpr double c16[8] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                               0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613};
    constexpr double s16[8] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                               1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173};
    typedef decltype(w.x) T;
    if (K == 0) return w;
    if (K == 4) return INV ? mk2(-w.y, w.x) : mk2(w.y, -w.x);   // times +i / -i
    return cmul(w, mk2((T)c16[K], INV ? (T)s16[K] : (T)-s16[K]));
}

// butterflies of stage t of a radix-2^RL pass for the pairs (j, j + 2^t) with j mod 2^t = M,
// twiddle w W_{2^(t+1)}^M, then the next M.  UNIT: w = 1 exactly (the first pass), so only
// the constant roots are applied.
template <bool INV, int RL, int t, int M, bool UNIT, typename C> __device__ __forceinline__ void stage_pairs(C *x, C w)
{
    if constexpr (M < (1 << t)) {
        typedef decltype(w.x) T;
        const C tw = rot16<INV, (M << (3 - t))>(UNIT ? mk2((T)1, (T)0) : w);
#pragma unroll
        for (int j0 = M; j0 < (1 << RL); j0 += 2 << t) {
            const C u = x[j0];
            const C v = UNIT && M == 0 ? x[j0 + (1 << t)] : cmul(tw, x[j0 + (1 << t)]);
            x[j0] = cadd(u, v);
            x[j0 + (1 << t)] = csub(u, v);
        }
        stage_pairs<INV, RL, t, M + 1, UNIT>(x, w);
    }
}

// stages t .. RL-1 of a radix-2^RL pass on x[0 .. 2^RL), stage s + t of the transform
template <bool INV, int RL, int t, bool UNIT, typename T>
__device__ __forceinline__ void pass_stages(typename V2<T>::type *x, int pos, int s, const TwCacheT<T> &Tc, int N)
{
    if constexpr (t < RL) {
        typename V2<T>::type w = mk2((T)1, (T)0);
        if (!UNIT) {
            w = twiddle(Tc, pos * (N >> (s + t)));
            if (INV) w.y = -w.y;
        }
        stage_pairs<INV, RL, t, 0, UNIT>(x, w);
        pass_stages<INV, RL, t + 1, UNIT>(x, pos, s, Tc, N);
    }
}

// Stages s .. s + RL - 1 (a radix-2^RL pass) of `count` in-place decimation-in-time
// transforms of length 2^logn held back to back in X (through lds_at).  Stage s + t pairs
// elements i and i + 2^t q (q = 2^(s-1)) with twiddle W_{2^(s+t)}^(i mod 2^t q); a lane takes
// the 2^RL elements base + j q, j < 2^RL, whose twiddles at stage t are W_{2^(s+t)}^pos (one
// table lookup) times the constant W_{2^(t+1)}^(j mod 2^t).  FIRST: s = 1, where pos = 0 and
// every looked-up twiddle is 1.  When q is a multiple of the pad period the lane's elements
// sit a uniform stride apart.  Ends with a barrier.
// Lane order of a pass: lane b takes butterfly group perm(b), perm a rotation right by r of the
// bit field [lo, lo + w) of b (packed lo | w << 4 | r << 8; 0: identity).  It changes only
// which lane computes which group, so the results are the same; chosen so that 16 consecutive
// lanes touch 16 distinct bank pairs where the layout alone does not give that.
__device__ __forceinline__ int lane_perm(int b, unsigned perm)
{
    if (perm == 0) return b;
    const int lo = perm & 15, w = (perm >> 4) & 15, r = perm >> 8;
    const int mask = (1 << w) - 1, f = (b >> lo) & mask;
    return (b & ~(mask << lo)) | ((((f >> r) | (f << (w - r))) & mask) << lo);
}

template <bool INV, int RL, bool FIRST, typename T>
__device__ __forceinline__ void fft_pass(typename V2<T>::type *X, int logn, int count, int s, int sh,
                                         const TwCacheT<T> &Tc, int N, unsigned perm = 0)
{
    typedef typename V2<T>::type C;
    constexpr int R = 1 << RL;
    const int lq = s - 1, q = 1 << lq;
    const int groups = (count << logn) >> RL, gmask = (1 << (logn - RL)) - 1;
    // a lane's elements sit a uniform stride apart when q is a multiple of the pad period, or
    // when all R of them lie inside one aligned block of 2^(lq + RL) <= 2^sh elements
    const bool wide = lq >= sh, narrow = lq + RL <= sh;
    const int stride = wide ? q + (q >> sh) : q;
    // a permutation of the lanes needs whole blocks of 2^(lo + w) groups (uniform: scalar)
    perm = __builtin_amdgcn_readfirstlane(perm);
    if (perm && (groups & ((1 << ((perm & 15) + ((perm >> 4) & 15))) - 1))) perm = 0;
    for (int b0 = threadIdx.x; b0 < groups; b0 += blockDim.x) {
        const int b = lane_perm(b0, perm);
        const int g = b >> (logn - RL), bb = b & gmask;
        const int pos = bb & (q - 1);
        const int base = (g << logn) + ((bb >> lq) << (lq + RL)) + pos;
        C x[R];
        if (wide || narrow) {
            const int a0 = lds_at(base, sh);
#pragma unroll
            for (int j = 0; j < R; ++j) x[j] = X[a0 + j * stride];
            pass_stages<INV, RL, 0, FIRST, T>(x, pos, s, Tc, N);
#pragma unroll
            for (int j = 0; j < R; ++j) X[a0 + j * stride] = x[j];
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j) x[j] = X[lds_at(base + j * q, sh)];
            pass_stages<INV, RL, 0, FIRST, T>(x, pos, s, Tc, N);
#pragma unroll
            for (int j = 0; j < R; ++j) X[lds_at(base + j * q, sh)] = x[j];
        }
    }
    __syncthreads();
}

struct NoLanePerm {
    __device__ unsigned operator()(int, int, int) const { return 0; }
};

// `count` independent in-place decimation-in-time transforms of length n = 2^logn (n >= 2)
// stored back to back in X (through lds_at with period 2^sh; sh < 0: lds_pad_shift(logn)),
// each already in bit-reversed order, with the twiddles of an N-point table in T: radix-2^RMAX
// passes (each lane keeps 2^RMAX points in registers for RMAX stages) and one pass of radix
// 2^(logn mod RMAX), first or (REM_LAST) last.  perm_of(logn, s, RL) gives each pass's lane
// permutation (lane_perm).  INV uses the conjugate twiddles exp(+2 pi i k / n) and does not
// scale.  Ends with a barrier.
template <bool INV, typename T, int RMAX = 4, bool REM_LAST = false, typename P = NoLanePerm>
__device__ __forceinline__ void fft_lds(typename V2<T>::type *X, int n, int logn, int count, const TwCacheT<T> &Tc,
                                        int N, int sh = -1, P perm_of = P())
{
    static_assert(RMAX >= 2 && RMAX <= 4, "radix 4, 8 or 16");
    if (sh < 0) sh = lds_pad_shift(logn);
    const int rem = logn % RMAX;
    (void)n;
    auto rem_pass = [&](int s, bool first) {
        const unsigned pm = perm_of(logn, s, rem);
        if (rem == 1) {
            if (first) fft_pass<INV, 1, true, T>(X, logn, count, s, sh, Tc, N, pm);
            else fft_pass<INV, 1, false, T>(X, logn, count, s, sh, Tc, N, pm);
        }
        if (RMAX > 2 && rem == 2) {
            if (first) fft_pass<INV, 2, true, T>(X, logn, count, s, sh, Tc, N, pm);
            else fft_pass<INV, 2, false, T>(X, logn, count, s, sh, Tc, N, pm);
        }
        if (RMAX > 3 && rem == 3) {
            if (first) fft_pass<INV, 3, true, T>(X, logn, count, s, sh, Tc, N, pm);
            else fft_pass<INV, 3, false, T>(X, logn, count, s, sh, Tc, N, pm);
        }
    };
    int s = 1;
    if (!REM_LAST && rem) {
        rem_pass(1, true);
        s += rem;
    }
    if (s == 1 && logn >= RMAX) {
        fft_pass<INV, RMAX, true, T>(X, logn, count, 1, sh, Tc, N, perm_of(logn, 1, RMAX));
        s += RMAX;
    }
    for (; s + RMAX - 1 <= logn; s += RMAX)
        fft_pass<INV, RMAX, false, T>(X, logn, count, s, sh, Tc, N, perm_of(logn, s, RMAX));
    if (REM_LAST && rem) rem_pass(s, s == 1);
}

// The same passes with the transform length and the pad period fixed at compile time: every
// stride is a constant, so a lane's LDS accesses are one base address plus immediate offsets
// (the runtime version computes an address per element).  For the lengths the large lattices
// use; fft_lds covers the rest.
template <bool INV, int RL, bool FIRST, typename T, int LOGN, int S, int SH>
__device__ __forceinline__ void fft_pass_c(typename V2<T>::type *X, int count, const TwCacheT<T> &Tc, int N,
                                           unsigned perm)
{
    typedef typename V2<T>::type C;
    constexpr int R = 1 << RL, lq = S - 1, q = 1 << lq;
    constexpr bool wide = lq >= SH, narrow = lq + RL <= SH;
    constexpr int stride = wide ? q + (q >> SH) : q;
    const int groups = (count << LOGN) >> RL;
    if (perm && (groups & ((1 << ((perm & 15) + ((perm >> 4) & 15))) - 1))) perm = 0;
    for (int b0 = threadIdx.x; b0 < groups; b0 += blockDim.x) {
        const int b = lane_perm(b0, perm);
        const int g = b >> (LOGN - RL), bb = b & ((1 << (LOGN - RL)) - 1);
        const int pos = bb & (q - 1);
        const int base = (g << LOGN) + ((bb >> lq) << (lq + RL)) + pos;
        C x[R];
        if constexpr (wide || narrow) {
            C *Xa = X + lds_at(base, SH);
#pragma unroll
            for (int j = 0; j < R; ++j) x[j] = Xa[j * stride];
            pass_stages<INV, RL, 0, FIRST, T>(x, pos, S, Tc, N);
#pragma unroll
            for (int j = 0; j < R; ++j) Xa[j * stride] = x[j];
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j) x[j] = X[lds_at(base + j * q, SH)];
            pass_stages<INV, RL, 0, FIRST, T>(x, pos, S, Tc, N);
#pragma unroll
            for (int j = 0; j < R; ++j) X[lds_at(base + j * q, SH)] = x[j];
        }
    }
    __syncthreads();
}

// radix-2^RMAX passes from stage S on, then the remainder (REM_LAST) or nothing
template <bool INV, typename T, int RMAX, bool REM_LAST, int LOGN, int SH, int S, typename P>
__device__ __forceinline__ void fft_passes_c(typename V2<T>::type *X, int count, const TwCacheT<T> &Tc, int N,
                                             P perm_of)
{
    if constexpr (S + RMAX - 1 <= LOGN) {
        fft_pass_c<INV, RMAX, S == 1, T, LOGN, S, SH>(X, count, Tc, N, perm_of(LOGN, S, RMAX));
        fft_passes_c<INV, T, RMAX, REM_LAST, LOGN, SH, S + RMAX>(X, count, Tc, N, perm_of);
    } else if constexpr (REM_LAST && S <= LOGN) {
        fft_pass_c<INV, LOGN - S + 1, S == 1, T, LOGN, S, SH>(X, count, Tc, N, perm_of(LOGN, S, LOGN - S + 1));
    }
}

// fft_lds for n = 2^LOGN and pad period 2^SH known at compile time (same passes, same order)
template <bool INV, typename T, int RMAX, bool REM_LAST, int LOGN, int SH, typename P = NoLanePerm>
__device__ __forceinline__ void fft_lds_c(typename V2<T>::type *X, int count, const TwCacheT<T> &Tc, int N,
                                          P perm_of = P())
{
    constexpr int rem = LOGN % RMAX;
    if constexpr (!REM_LAST && rem != 0) {
        fft_pass_c<INV, rem, true, T, LOGN, 1, SH>(X, count, Tc, N, perm_of(LOGN, 1, rem));
        fft_passes_c<INV, T, RMAX, false, LOGN, SH, 1 + rem>(X, count, Tc, N, perm_of);
    } else {
        fft_passes_c<INV, T, RMAX, REM_LAST, LOGN, SH, 1>(X, count, Tc, N, perm_of);
    }
}

}  // namespace lbf
