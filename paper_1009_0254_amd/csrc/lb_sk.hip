// Static structure factor of the nine LB modes, the equilibration measurement of
// arXiv:1009.0254, Sec. V.A: <|m_a(k)|^2> with a(k) = n^-1/2 sum_r exp(i k.r) a(r)
// (Sec. III notation).  For a real field |a(k)|^2 = |a(-k)|^2, so the transforms below
// use exp(-2 pi i k x / n) and keep the half plane kx = 0..nx/2.
//
// A sample covers a range of replicas of any sizes with two launches, whatever their sizes:
//   1. rows: one workgroup per lattice row of any replica in the range.  It pulls the
//      pre-collision populations, forms the nine moments relative to those of a reference
//      (the mean pulled populations of row 0, from a one-block-per-replica pre-pass) in the
//      transform precision (FP32 for FP32 storage, FP64 for FP64 storage) and turns
//      each real row of length nx into its half spectrum with one complex transform of
//      length nx/2 (even samples as real part, odd as imaginary, then the standard split),
//      G modes at a time in LDS until all nine are done (for FP32 rows up to 8192 the
//      moments stay in registers between groups; otherwise each group pulls again and the
//      repeats hit the caches), writing mode a to slot a of the spectra, [ny][nx/2+1] each;
//   2. columns: one workgroup per kx and mode reads its column of the row spectra in place
//      (consecutive kx share cache lines and are kept on one XCD), transforms along y
//      (a column longer than 64 KiB of LDS is split by one decimation-in-frequency stage
//      into two half-length transforms, one per output parity, so that it fits), restores
//      the k = 0 coefficient in FP64 and adds |X|^2 / n to the FP64 accumulators
//      [9][nx/2+1][ny].
// Subtracting a constant per mode moves only k = 0; with the row-0 mean as that constant the
// transforms see fluctuation-sized values whatever the mean state, and so do the row sums
// (kx = 0) and totals, whose remaining offset is of the order of their own fluctuation: in
// FP32 the rounding is ~1e-7 of the spectrum's scale.
// The transforms are lb_fftcore.h's radix-8 passes (radix 4 for the FP64 columns).
// The radially binned density spectrum (the isotropic average of S_rho(k), used to follow
// density modes after a quench to c_s^2 < 0, where M(k) of eq. (lb-lang-ft) has growing
// eigenvalues) reuses 1-3 for mode 0 of one replica and bins |rho(k)|^2 / n with integer
// shell arithmetic.

#include <algorithm>
#include <type_traits>

#include "lb_fftcore.h"
#include "lb_internal.h"
#include "lb_sklayout.h"

namespace lbf {

namespace {

constexpr int SK_THREADS = 1024;   // upper bound; launches use fewer for short lines

// lines of 4096 points or more get 1024 lanes; shorter ones 256
int sk_threads(int line) { return line >= 4096 ? 1024 : 256; }

template <int F> __device__ __forceinline__ long long sk_key(const SkRep &q)
{
    return F == 0 ? q.row0 : q.col0;
}

// replica of global block g: the last r in [r0, r1) whose prefix is <= g
template <int F> __device__ __forceinline__ int sk_find(const SkRep *__restrict__ sk, int r0, int r1, long long g)
{
    int lo = r0, hi = r1 - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sk_key<F>(sk[mid]) <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// the nine stored values that the pull of node (x, y) reads (pull_node without the shift)
template <typename S>
__device__ __forceinline__ void load_pull(const S *__restrict__ P, int nx, int ny, int x, int y, S v[9])
{
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    v[0] = P[pop_at(nx, 0, x, y)];
    v[1] = P[pop_at(nx, 1, xm, y)];
    v[2] = P[pop_at(nx, 2, x, ym)];
    v[3] = P[pop_at(nx, 3, xp, y)];
    v[4] = P[pop_at(nx, 4, x, yp)];
    v[5] = P[pop_at(nx, 5, xm, ym)];
    v[6] = P[pop_at(nx, 6, xp, ym)];
    v[7] = P[pop_at(nx, 7, xp, yp)];
    v[8] = P[pop_at(nx, 8, xm, yp)];
}

// m = T f with the integer rows of the moment basis of Table I
template <typename U> __device__ __forceinline__ void moments9(const U g[9], U m[9])
{
    const double sa = (g[1] + g[2]) + (g[3] + g[4]);
    const double sd = (g[5] + g[6]) + (g[7] + g[8]);
    const double ax = g[1] - g[3], ay = g[2] - g[4], d68 = g[5] - g[7], d97 = g[8] - g[6];
    m[0] = g[0] + sa + sd;
    m[1] = ax + d68 + d97;
    m[2] = ay + d68 - d97;
    m[3] = -2 * g[0] + sa + 4 * sd;
    m[4] = (g[1] + g[3]) - (g[2] + g[4]);
    m[5] = (g[5] + g[7]) - (g[6] + g[8]);
    m[6] = -ax + 2 * (d68 + d97);
    m[7] = -ay + 2 * (d68 - d97);
    m[8] = 2 * g[0] - 4 * sa + 8 * sd;
}

constexpr int SK_CACHE_PAIRS = 4;   // node pairs per lane whose moments stay in registers

// The nine moments of nodes (x, y) and (x + 1, y) relative to those of the reference, in Tt,
// packed as (even, odd) complex pairs: the differences of the pulled values come first (for
// values of one population they are exact or rounded at the fluctuation's own scale), then
// the integer combinations of Table I.
template <typename S, typename Tt>
__device__ __forceinline__ void pair_moments(const S *__restrict__ P, int nx, int ny, int x, int y,
                                             const Tt *vref, typename V2<Tt>::type m[9])
{
    S v[2][9];
    load_pull(P, nx, ny, x, y, v[0]);
    load_pull(P, nx, ny, x + 1, y, v[1]);
    Tt de[9], dd[9], me[9], mo[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        de[i] = (Tt)v[0][i] - vref[i];
        dd[i] = (Tt)v[1][i] - vref[i];
    }
    moments9(de, me);
    moments9(dd, mo);
#pragma unroll
    for (int a = 0; a < 9; ++a) m[a] = mk2(me[a], mo[a]);
}

// `count` transforms of length n = 2^logn, pad period 2^sh (the 1/16 pad with the remainder pass
// last when P16, else the wide pad with the remainder first); the lengths of the large lattices
// with compile-time strides
template <typename Tt, int RMAX, bool P16, bool FIXED = true, typename P = NoLanePerm>
__device__ __forceinline__ void sk_fft(typename V2<Tt>::type *X, int n, int logn, int count, const TwCacheT<Tt> &T,
                                       int nmax, int sh)
{
    constexpr int SH12 = P16 ? LDS_PAD16 : lds_pad_shift(12), SH13 = P16 ? LDS_PAD16 : lds_pad_shift(13);
    if (FIXED && logn == 12 && sh == SH12)
        fft_lds_c<false, Tt, RMAX, P16, 12, SH12>(X, count, T, nmax, P());
    else if (FIXED && logn == 13 && sh == SH13)
        fft_lds_c<false, Tt, RMAX, P16, 13, SH13>(X, count, T, nmax, P());
    else
        fft_lds<false, Tt, RMAX, P16>(X, n, logn, count, T, nmax, sh, P());
}

// Lane orders of the row transforms' passes (radix 8, remainder first, the wide pad
// lds_pad_shift(logn)) whose 16 consecutive lanes would otherwise share LDS bank pairs (4- and
// 2-way at 4096 points, 8- and 2-way at 8192): lane_perm rotations found by enumerating the
// lanes' slots, packed lo | w << 4 | r << 8.
struct SkRowPerm {
    __device__ unsigned operator()(int logn, int s, int) const
    {
        if (logn == 12) return s == 1 ? (1u | 5u << 4 | 3u << 8) : s == 4 ? (3u | 4u << 4 | 1u << 8) : 0u;
        if (logn == 11) return s == 1 ? (2u | 3u << 4 | 2u << 8) : s == 3 ? (2u | 4u << 4 | 2u << 8) : 0u;
        if (logn == 13) return s == 1 ? (3u | 4u << 4 | 1u << 8) : s == 2 ? (1u | 7u << 4 | 3u << 8) : 0u;
        return 0u;
    }
};

// The FP32 columns (radix 8, remainder last, 1/16 pad): the stride-8 pass puts 16 consecutive
// lanes on 8 bank pairs; swapping bits 3 and 4 of the lane's group index spreads them.
struct SkColPerm {
    __device__ unsigned operator()(int, int s, int rl) const { return s == 4 && rl == 3 ? (3u | 2u << 4 | 1u << 8) : 0u; }
};

// The rows' register-fed bit-reversed fill: lane e of a wave writes slot bitrev(pair) + pad,
// which for consecutive pairs puts 16 lanes on 4 bank pairs; lanes of a 16-lane group take
// pairs 4 apart instead (the wave still covers 64 consecutive pairs, so its loads touch the same
// cache lines).  Needs whole blocks of 64 pairs.
__device__ __forceinline__ int sk_fill_pair(int e, bool whole64)
{
    return whole64 ? (e & ~63) | ((e & 15) << 2) | ((e >> 4) & 3) : e;
}

constexpr int SK_REF_THREADS = 256;

// The reference of replica r: the mean over row 0 of each pulled population, in FP64 with a
// fixed-order reduction, rounded to the transform type: vref_i = base[18 r + 9 + i].  Every
// node's moments are transformed relative to m(vref), whose distance from the replica's mean
// is ~ sigma / sqrt(nx), so that neither the row sums (kx = 0) nor the totals carry an offset
// that FP32 would have to resolve against the fluctuations.  base[18 r + a] = m_a(vref + shift)
// in FP64, the constant the column pass restores at k = 0.
template <typename S, typename Tt>
__global__ void __launch_bounds__(SK_REF_THREADS)
    k_sk_ref(const S *__restrict__ f, const RepDesc *__restrict__ reps, const SkRep *__restrict__ sk, int r0,
             double *__restrict__ base)
{
    __shared__ double part[SK_REF_THREADS / 64][9];
    const int r = r0 + (int)blockIdx.x;
    const SkRep &q = sk[r];
    const RepDesc &d = reps[r];
    const S *P = f + d.off;
    double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int x = threadIdx.x; x < q.nx; x += blockDim.x) {
        S v[9];
        load_pull(P, q.nx, q.ny, x, 0, v);
#pragma unroll
        for (int i = 0; i < 9; ++i) s[i] += (double)v[i];
    }
#pragma unroll
    for (int i = 0; i < 9; ++i)
        for (int o = 32; o > 0; o >>= 1) s[i] += __shfl_xor(s[i], o);
    if ((threadIdx.x & 63) == 0)
        for (int i = 0; i < 9; ++i) part[threadIdx.x >> 6][i] = s[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        double g[9], m[9];
        for (int i = 0; i < 9; ++i) {
            double t = 0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += part[w][i];
            const double vr = (double)(Tt)(t / q.nx);
            base[18 * r + 9 + i] = vr;
            g[i] = vr + d.shift[i];
        }
        moments9(g, m);
        for (int a = 0; a < 9; ++a) base[18 * r + a] = m[a];
    }
}

// Transforms run in Tt (float for FP32 storage, double for FP64) on m_a(r) - m_a(vref) (the
// reference of k_sk_ref); a constant only moves the k = 0 coefficient, which the column pass
// restores in FP64 as X(0) + n m_a(vref + shift).  CACHE: a lane's node pairs (at most
// SK_CACHE_PAIRS) are pulled once and their nine moments kept in registers for all mode
// groups, which are GC modes each and fixed at compile time (so that a placed group's
// registers are free for the transforms); otherwise each group of G modes pulls the row
// again (the repeats hit L2 or the MALL).
template <typename S, typename Tt, int RMAX, bool CACHE, int GC>
__global__ void __launch_bounds__(SK_THREADS)
    k_sk_rows(const S *__restrict__ f, const RepDesc *__restrict__ reps, const SkRep *__restrict__ sk, int r0, int r1,
              long long row_base, long long nrows, int a_first, int a_count, int G, long long Ptot,
              typename V2<Tt>::type *__restrict__ spec, const double *__restrict__ base,
              const double2 *__restrict__ tw, int nmax)
{
    typedef typename V2<Tt>::type C;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ TwCacheT<Tt> T;
    __shared__ Tt vref[9];
    C *X = reinterpret_cast<C *>(smem_raw);
    const long long lr = xcd_logical(nrows);
    if (lr < 0) return;
    tw_cache_load(T, tw, nmax);
    const long long gr = row_base + lr;
    const int r = sk_find<0>(sk, r0, r1, gr);
    const SkRep &q = sk[r];
    const RepDesc &d = reps[r];
    const int nx = q.nx, ny = q.ny, M = nx >> 1, logM = q.lognx - 1;
    const int y0 = (int)(gr - q.row0) * q.rpb;
    const int R = min(q.rpb, ny - y0);          // rows of this block
    const int Rp = q.rpb, lRp = q.logrpb;       // transform (c, rr) at X[(c Rp + rr) M]
    const int pairs = R * M;
    const S *P = f + d.off;
    const int wstride = nmax / nx, sh = lds_pad_shift(logM);
    if (threadIdx.x < 9) vref[threadIdx.x] = (Tt)base[18 * r + 9 + threadIdx.x];
    __syncthreads();   // vref (the reference)
    // (the cached variant pulls once; pulling in the permuted order every group costs more than
    // the fill's bank conflicts)
    const bool whole64 = CACHE && (pairs & 63) == 0;
    C cm[CACHE ? SK_CACHE_PAIRS : 1][9];
    if (CACHE) {
#pragma unroll
        for (int j = 0; j < SK_CACHE_PAIRS; ++j) {
            const int e = threadIdx.x + j * (int)blockDim.x;
            if (e < pairs) {
                const int ep = sk_fill_pair(e, whole64), rr = ep >> logM, n = ep & (M - 1);
                pair_moments(P, nx, ny, 2 * n, y0 + rr, vref, cm[j]);
            }
        }
    }
    // one group of modes [a0, a0 + gcount): place them (bit-reversed), transform, untangle into
    // the spectra.  A0, GN: compile-time a0 and gcount (the cached variant, whose moments of a
    // placed group are then dead), or -1 for the runtime a0_rt, gn_rt.
    auto run_group = [&](auto A0, auto GN, int a0_rt, int gn_rt) {
        constexpr int a0c = decltype(A0)::value, gnc = decltype(GN)::value;
        const int a0 = a0c >= 0 ? a0c : a0_rt, gcount = gnc >= 0 ? gnc : gn_rt;
        if constexpr (CACHE) {
#pragma unroll
            for (int j = 0; j < SK_CACHE_PAIRS; ++j) {
                const int e = threadIdx.x + j * (int)blockDim.x;
                if (e < pairs) {
                    const int ep = sk_fill_pair(e, whole64), rr = ep >> logM, n = ep & (M - 1);
                    const unsigned jb = bitrev((unsigned)n, logM);
#pragma unroll
                    for (int c = a0c; c < a0c + gnc; ++c) X[lds_at((((c - a0c) << lRp) + rr) * M + jb, sh)] = cm[j][c];
                }
            }
        } else {
            for (int e = threadIdx.x; e < pairs; e += blockDim.x) {
                const int ep = sk_fill_pair(e, whole64), rr = ep >> logM, n = ep & (M - 1);
                C m[9];
                pair_moments(P, nx, ny, 2 * n, y0 + rr, vref, m);
                const unsigned jb = bitrev((unsigned)n, logM);
#pragma unroll
                for (int c = 0; c < 9; ++c)
                    if (c >= a0 && c < a0 + gcount) X[lds_at((((c - a0) << lRp) + rr) * M + jb, sh)] = m[c];
            }
        }
        __syncthreads();
        // slots rr >= R (the last rows of a replica) hold no data; their results are dropped
        const int nt = gcount << lRp;
        sk_fft<Tt, RMAX, false, true, SkRowPerm>(X, M, logM, nt, T, nmax, lds_pad_shift(logM));
        // X_k = E_k + W^k O_k with E = (Z_k + conj Z_{M-k}) / 2, O = (Z_k - conj Z_{M-k}) / 2i,
        // W = exp(-2 pi i / nx), for k = 0..M (Z has period M).  The partner M - k reuses both
        // reads and the twiddle: E_{M-k} = conj E_k, O_{M-k} = conj O_k, W^{M-k} = -conj W^k,
        // so X_{M-k} = conj(E_k - W^k O_k).  A lane takes k < M/2 and its partner; k = M/2 in
        // the second loop.
        const Tt h = (Tt)0.5;
        auto untangle = [&](int t, int k) {
            const int c = t >> lRp, rr = t & (Rp - 1);
            if (rr >= R) return;
            const C Zk = X[lds_at(t * M + k, sh)];
            const C Zm = X[lds_at(t * M + ((M - k) & (M - 1)), sh)];
            const C E = mk2(h * (Zk.x + Zm.x), h * (Zk.y - Zm.y));
            const C O = mk2(h * (Zk.y + Zm.y), -h * (Zk.x - Zm.x));
            const C WO = cmul(twiddle(T, k * wstride), O);
            typename V2<Tt>::type *out = spec + (a0 + c) * Ptot + q.soff;
            out[sk_at(y0 + rr, k, ny)] = cadd(E, WO);
            if (2 * k != M) {
                const C D = csub(E, WO);
                out[sk_at(y0 + rr, M - k, ny)] = mk2(D.x, -D.y);
            }
        };
        const int lh = logM - 1;   // M/2 = 2^lh
        for (int idx = threadIdx.x; idx < nt << lh; idx += blockDim.x) untangle(idx >> lh, idx & ((1 << lh) - 1));
        for (int t = threadIdx.x; t < nt; t += blockDim.x) untangle(t, M >> 1);
        __syncthreads();   // X is reused by the next group
    };
    if constexpr (CACHE) {
        // the nine modes (a_first = 0, a_count = 9) in groups of GC
        static_assert(GC == 4 || GC == 8, "cached rows run 4 + 4 + 1 or 8 + 1 modes");
        (void)a_first;
        (void)a_count;
        (void)G;
        run_group(std::integral_constant<int, 0>{}, std::integral_constant<int, GC>{}, 0, 0);
        run_group(std::integral_constant<int, GC>{}, std::integral_constant<int, 9 - GC < GC ? 9 - GC : GC>{}, 0, 0);
        if constexpr (2 * GC < 9)
            run_group(std::integral_constant<int, 2 * GC>{}, std::integral_constant<int, 9 - 2 * GC>{}, 0, 0);
    } else {
        for (int a0 = a_first; a0 < a_first + a_count; a0 += G)
            run_group(std::integral_constant<int, -1>{}, std::integral_constant<int, -1>{}, a0,
                      min(G, a_first + a_count - a0));
    }
}

// column transforms of every replica in the range, reading the row spectra in place;
// mode a = a_first + blockIdx.y.  A block takes cpb adjacent kx (reads coalesced along kx)
// or, for split lines, one kx and one output parity.  |X|^2 is formed in FP64, with the
// k = 0 coefficient restored to X(0) + n m_a(vref + shift) (the row pass transformed moments
// relative to the reference of k_sk_ref).  SNAP writes |X|^2 / n to plane ([nh][ny], one replica),
// otherwise adds it to the accumulators.
template <typename Tt, bool SNAP, int RMAX>
__global__ void __launch_bounds__(SK_THREADS)
    k_sk_cols(const typename V2<Tt>::type *__restrict__ spec, const SkRep *__restrict__ sk, int r0, int r1,
              long long col_base, long long ncols, long long Ptot, int a_first, double *__restrict__ acc,
              double *__restrict__ plane, const double *__restrict__ base, const double2 *__restrict__ tw, int nmax)
{
    typedef typename V2<Tt>::type C;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ TwCacheT<Tt> T;
    C *X = reinterpret_cast<C *>(smem_raw);
    const long long lc = xcd_logical(ncols);
    if (lc < 0) return;
    tw_cache_load(T, tw, nmax);
    __syncthreads();
    const long long gc = col_base + lc;
    const int r = sk_find<2>(sk, r0, r1, gc);
    const SkRep &q = sk[r];
    const int ny = q.ny, nh = q.nx / 2 + 1, split = q.split;
    const int local = (int)(gc - q.col0);
    const int grp = local / split, par = local - grp * split;
    const int kx0 = grp * q.cpb;
    const int C_ = min(q.cpb, nh - kx0);         // columns of this block
    const int a = a_first + blockIdx.y;
    const C *S0 = spec + a * Ptot + q.soff;    // (y, kx) at S0[sk_at(y, kx, ny)]
    const double inv_n = 1.0 / ((double)q.nx * (double)ny);
    // added to the real part of output 0 of this block when that output is k = 0
    const double k0 = kx0 == 0 && par == 0 ? (double)q.nx * (double)ny * base[18 * r + a] : 0.0;
    const int L = ny / split, logL = q.logny - (split - 1);
    // P16 (FP32): the 1/16-pad layout, filled in destination order (lane e writes slot e of the
    // bit-reversed line and reads its source at bitrev(e)), the remainder pass last; FP64 keeps
    // the wide pad and a source-ordered fill
    constexpr bool P16 = sizeof(Tt) == 4;
    const int sh = P16 ? LDS_PAD16 : lds_pad_shift(logL);
    if (split == 1) {
        if (P16) {
            const int tot = C_ << logL;
            for (int e0 = threadIdx.x; e0 < tot; e0 += 4 * blockDim.x) {
                C v[4];
                for (int u = 0; u < 4; ++u) {
                    const int e = min(e0 + u * (int)blockDim.x, tot - 1);
                    const int y = (int)bitrev((unsigned)(e & (L - 1)), logL);
                    v[u] = S0[sk_at32(y, kx0 + (e >> logL), ny)];
                }
                for (int u = 0; u < 4; ++u) {
                    const int e = e0 + u * (int)blockDim.x;
                    if (e < tot) X[lds_at(e, sh)] = v[u];
                }
            }
        } else {
            // lanes over (y, c) with c < Cp = 2^ceil(log2 C_); c >= C_ idle
            const int lCp = C_ > 1 ? 32 - __clz(C_ - 1) : 0, tot = ny << lCp;
            for (int e0 = threadIdx.x; e0 < tot; e0 += 4 * blockDim.x) {
                C v[4];
                for (int u = 0; u < 4; ++u) {
                    const int e = min(e0 + u * (int)blockDim.x, tot - 1), y = e >> lCp;
                    const int c = min(e & ((1 << lCp) - 1), C_ - 1);
                    v[u] = S0[sk_at(y, kx0 + c, ny)];
                }
                for (int u = 0; u < 4; ++u) {
                    const int e = e0 + u * (int)blockDim.x, y = e >> lCp, c = e & ((1 << lCp) - 1);
                    if (e < tot && c < C_) X[lds_at(c * ny + bitrev((unsigned)y, logL), sh)] = v[u];
                }
            }
        }
    } else {
        // X_{2k+p} = sum_n [x_n + (-1)^p x_{n+L}] W^{pn} exp(-2 pi i n k / L), W = exp(-2 pi i / ny)
        const int wstride = nmax / ny;
        for (int r = threadIdx.x; r < L; r += blockDim.x) {
            const int n = P16 ? (int)bitrev((unsigned)r, logL) : r;
            const C u = S0[sk_at32(n, kx0, ny)], v = S0[sk_at32(n + L, kx0, ny)];
            X[lds_at(P16 ? r : (int)bitrev((unsigned)n, logL), sh)] =
                par == 0 ? cadd(u, v) : cmul(csub(u, v), twiddle(T, n * wstride));
        }
    }
    __syncthreads();
    sk_fft<Tt, RMAX, P16, true, typename std::conditional<P16, SkColPerm, NoLanePerm>::type>(X, L, logL, split == 1 ? C_ : 1, T,
                                                                                         nmax, sh);
    const int tot = (split == 1 ? C_ : 1) * L;
    auto power = [&](int e) {
        const C v = X[lds_at(e, sh)];
        const double re = (double)v.x + (e == 0 ? k0 : 0.0), im = (double)v.y;
        return (re * re + im * im) * inv_n;
    };
    // output e of this block is k = e mod L of column kx0 + e / L: index c ny + k split + par,
    // that is e (one column per output parity when split, else L = ny)
    if (SNAP) {
        double *D = plane + (long long)kx0 * ny;
        for (int e = threadIdx.x; e < tot; e += blockDim.x) D[split == 1 ? e : 2 * e + par] = power(e);
    } else {
        double *A = acc + q.acc_off + (long long)a * nh * ny + (long long)kx0 * ny;
        for (int e0 = threadIdx.x; e0 < tot; e0 += 4 * blockDim.x) {
            double old[4];
            for (int u = 0; u < 4; ++u) {
                const int e = min(e0 + u * (int)blockDim.x, tot - 1);
                old[u] = A[split == 1 ? e : 2 * e + par];
            }
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * (int)blockDim.x;
                if (e < tot) A[split == 1 ? e : 2 * e + par] = old[u] + power(e);
            }
        }
    }
}

// smallest t >= 0 with m t^2 >= v (m > 0)
__device__ __forceinline__ long long ceil_root(long long v, long long m)
{
    if (v <= 0) return 0;
    long long t = (long long)ceil(sqrt((double)v / (double)m));
    while (t > 0 && m * (t - 1) * (t - 1) >= v) --t;
    while (m * t * t < v) ++t;
    return t;
}

// Shell b of the radial spectrum: with L = min(nx, ny), P = max(nx, ny) / L and
// R2 = wx kx^2 + wy ky^2 ((wx, wy) = (1, P^2) if nx >= ny, else (P^2, 1)), |k| / (2 pi / L)
// = sqrt(R2) / P, and k lies in shell b = floor(sqrt(R2) / P + 1/2), i.e.
// ((2b - 1) P)^2 <= 4 R2 < ((2b + 1) P)^2.  Means over the full k plane without k = 0;
// the half plane stands for its mirror image with weight 2 except at kx = 0 and nx/2.
__global__ void __launch_bounds__(256) k_sk_bins(const double *__restrict__ plane, int nx, int ny, int P, int xwide,
                                                 int nbins, double *__restrict__ out)
{
    __shared__ double ss[256], sc[256];
    const int b = blockIdx.x;
    const long long wx = xwide ? 1 : (long long)P * P, wy = xwide ? (long long)P * P : 1;
    const long long lo = b > 0 ? (long long)(2 * b - 1) * P * (2 * b - 1) * P : 0;
    const long long hi = (long long)(2 * b + 1) * P * (2 * b + 1) * P;
    const int hx = nx / 2, hy = ny / 2;
    double s = 0, c = 0;
    for (int kx = threadIdx.x; kx <= hx; kx += blockDim.x) {
        const long long ax = 4 * wx * (long long)kx * kx;
        if (ax >= hi) break;
        const long long y0 = ceil_root(lo - ax, 4 * wy);
        const long long y1 = min(ceil_root(hi - ax, 4 * wy), (long long)hy + 1);
        const double w = (kx == 0 || kx == hx) ? 1.0 : 2.0;
        const double *D = plane + (long long)kx * ny;
        for (long long ky = y0; ky < y1; ++ky) {
            if (kx == 0 && ky == 0) continue;
            s += w * D[ky];
            c += w;
            if (ky >= 1 && ky < hy) {
                s += w * D[ny - ky];
                c += w;
            }
        }
    }
    ss[threadIdx.x] = s;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            ss[threadIdx.x] += ss[threadIdx.x + h];
            sc[threadIdx.x] += sc[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[b] = sc[0] > 0 ? ss[0] / sc[0] : 0.0;
        out[nbins + b] = sc[0];
    }
}

__global__ void k_sk_read(const double *__restrict__ acc, double *__restrict__ out, int nx, int ny, double inv_ns)
{
    const int nh = nx / 2 + 1;
    const long long per = (long long)nh * ny;
    const long long total = 9 * per;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < total; k += (long long)gridDim.x * blockDim.x) {
        const long long a = k / per, rem = k - a * per;
        const long long ky = rem / nh, kx = rem - ky * nh;
        out[k] = acc[a * per + kx * ny + ky] * inv_ns;
    }
}

// radix of the in-LDS passes: 8, except 4 for the FP64 column transforms (at 8 their
// registers allow only one 1024-lane workgroup per CU; so would 16 for the FP32 columns)
template <typename Tt> constexpr int SK_ROW_RADIX = 3;
template <typename Tt> constexpr int SK_COL_RADIX = sizeof(Tt) == 4 ? 3 : 2;

template <typename S, typename Tt, int RMAX, bool CACHE, int GC = 0>
void rows_kernel(const SkLaunch &a, int a_first, int a_count, int G, int threads, hipStream_t s)
{
    const size_t lds = (size_t)sk_elem(sizeof(Tt) == 8 ? 0 : 1) * lds_padded((long long)G * (a.lds_rows / 2));
    hipLaunchKernelGGL((k_sk_rows<S, Tt, RMAX, CACHE, GC>), dim3(xcd_grid(a.rows)), dim3(threads), lds, s, (const S *)a.f,
                       a.reps, a.sk, a.r0, a.r1, (long long)a.row_base, (long long)a.rows, a_first, a_count, G,
                       (long long)a.Ptot, (typename V2<Tt>::type *)a.spec, a.base, (const double2 *)a.tw, a.nmax);
}

hipError_t launch_rows(int precision, const SkLaunch &a, int a_first, int a_count, hipStream_t s)
{
    if (precision == 0)
        hipLaunchKernelGGL((k_sk_ref<double, double>), dim3((unsigned)(a.r1 - a.r0)), dim3(SK_REF_THREADS), 0, s,
                           (const double *)a.f, a.reps, a.sk, a.r0, a.base);
    else
        hipLaunchKernelGGL((k_sk_ref<float, float>), dim3((unsigned)(a.r1 - a.r0)), dim3(SK_REF_THREADS), 0, s,
                           (const float *)a.f, a.reps, a.sk, a.r0, a.base);
    const int G = a_count < a.G ? a_count : a.G;
    const int threads = sk_threads(a.lds_rows);
    // FP32: with at most SK_CACHE_PAIRS node pairs per lane the nine moments stay in
    // registers across the mode groups (FP64 would spill)
    const bool cache = precision != 0 && a_first == 0 && a_count == 9 && (G == 4 || G == 8) &&
                       a.lds_rows / 2 <= SK_CACHE_PAIRS * threads;
    if (precision == 0)
        rows_kernel<double, double, SK_ROW_RADIX<double>, false>(a, a_first, a_count, G, threads, s);
    else if (cache && G == 4)
        rows_kernel<float, float, SK_ROW_RADIX<float>, true, 4>(a, a_first, a_count, G, threads, s);
    else if (cache)
        rows_kernel<float, float, SK_ROW_RADIX<float>, true, 8>(a, a_first, a_count, G, threads, s);
    else
        rows_kernel<float, float, SK_ROW_RADIX<float>, false>(a, a_first, a_count, G, threads, s);
    return hipGetLastError();
}

// dynamic LDS of a column block of `points` transform points (FP32: 1/16 pad)
size_t sk_col_lds_bytes(int precision, long long points)
{
    return (size_t)sk_elem(precision) * (size_t)(precision == 0 ? lds_padded(points) : lds_padded16(points));
}

template <typename Tt, bool SNAP>
void cols_kernel(int precision, const SkLaunch &a, unsigned modes, double *plane, hipStream_t s)
{
    hipLaunchKernelGGL((k_sk_cols<Tt, SNAP, SK_COL_RADIX<Tt>>), dim3(xcd_grid(a.cols), modes),
                       dim3(sk_threads(a.lds_cols)), sk_col_lds_bytes(precision, a.lds_cols), s,
                       (const typename V2<Tt>::type *)a.spec, a.sk, a.r0, a.r1, (long long)a.col_base,
                       (long long)a.cols, (long long)a.Ptot, 0, SNAP ? nullptr : a.acc, plane, (const double *)a.base,
                       (const double2 *)a.tw, a.nmax);
}

template <typename K> hipError_t lds_limit(K kernel, size_t bytes)
{
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename S, typename Tt> hipError_t lds_limits_of(size_t rows, size_t cols)
{
    hipError_t e = lds_limit(k_sk_rows<S, Tt, SK_ROW_RADIX<Tt>, false, 0>, rows);
    if constexpr (sizeof(Tt) == 4) {   // the register-cached row variants exist for FP32 only
        if (e == hipSuccess) e = lds_limit(k_sk_rows<S, Tt, SK_ROW_RADIX<Tt>, true, 4>, rows);
        if (e == hipSuccess) e = lds_limit(k_sk_rows<S, Tt, SK_ROW_RADIX<Tt>, true, 8>, rows);
    }
    if (e == hipSuccess) e = lds_limit(k_sk_cols<Tt, false, SK_COL_RADIX<Tt>>, cols);
    if (e == hipSuccess) e = lds_limit(k_sk_cols<Tt, true, SK_COL_RADIX<Tt>>, cols);
    return e;
}

}  // namespace

int sk_elem(int precision) { return precision == 0 ? (int)sizeof(double2) : (int)sizeof(float2); }

// LDS budgets: the row kernel holds G half-length transforms of its widest rows in at most
// 128 KiB; a column block holds at most 64 KiB (two blocks per CU)
constexpr int ROW_BUDGET = 131072, COL_BUDGET = 65536;

int sk_modes_per_pass(int precision, int max_nx)
{
    const int per_mode = sk_elem(precision) * (std::max(max_nx, 1024) / 2);
    return std::max(1, std::min(9, ROW_BUDGET / per_mode));
}

int sk_split(int precision, int ny) { return (long long)ny * sk_elem(precision) > COL_BUDGET ? 2 : 1; }

int sk_cols_per_block(int precision, int nx, int ny)
{
    const int pts = COL_BUDGET / sk_elem(precision);
    return ny >= pts ? 1 : std::min(pts / ny, nx / 2 + 1);
}

hipError_t set_sk_lds_limits(int precision, int G, int max_row, int max_col)
{
    const size_t rows = (size_t)sk_elem(precision) * lds_padded((long long)G * (max_row / 2)),
                 cols = sk_col_lds_bytes(precision, max_col);
    return precision == 0 ? lds_limits_of<double, double>(rows, cols) : lds_limits_of<float, float>(rows, cols);
}

hipError_t launch_sk_sample(int precision, const SkLaunch &a, hipStream_t s)
{
    hipError_t e = launch_rows(precision, a, 0, 9, s);
    if (e != hipSuccess) return e;
    if (precision == 0)
        cols_kernel<double, false>(precision, a, 9, nullptr, s);
    else
        cols_kernel<float, false>(precision, a, 9, nullptr, s);
    return hipGetLastError();
}

hipError_t launch_sk_snapshot(int precision, const SkLaunch &a, int nx, int ny, int nbins, int P, int xwide,
                              double *out, hipStream_t s)
{
    hipError_t e = launch_rows(precision, a, 0, 1, s);
    if (e != hipSuccess) return e;
    // the density's |X|^2 / n goes to spectrum slot 1 (unused here) as [nh][ny] doubles
    double *plane = (double *)((char *)a.spec + (size_t)sk_elem(precision) * a.Ptot);
    if (precision == 0)
        cols_kernel<double, true>(precision, a, 1, plane, s);
    else
        cols_kernel<float, true>(precision, a, 1, plane, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sk_bins, dim3((unsigned)nbins), dim3(256), 0, s, (const double *)plane, nx, ny, P, xwide,
                       nbins, out);
    return hipGetLastError();
}

hipError_t launch_sk_read(const double *acc, double *out, int nx, int ny, double inv_ns, hipStream_t s)
{
    const long long total = 9ll * (nx / 2 + 1) * ny;
    long long g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_sk_read, dim3((unsigned)g), dim3(256), 0, s, acc, out, nx, ny, inv_ns);
    return hipGetLastError();
}

}  // namespace lbf
