// Two time steps of the fluctuating D2Q9 update per launch (temporal blocking).
//
// The update of one step (eq. gen-lbe-m with the noise of eq. noise-yeo at k = 0) is the one
// of k_step: pull f_i(r, t) = f*_i(r - c_i, t - 1), density, 9-point stencils (App. B
// Laplacian, isotropic gradient), collision (lb_collide.h).  k_step2 applies it twice, the
// second time to the post-collision rows of the first while they are still on chip, so that
// HBM sees one read of f*(t - 1) and one write of f*(t + 1) per two steps: half the traffic
// of two launches of k_step.  Every node of every step goes through the same arithmetic as in
// k_step (the same collision, density and stencil expressions, the rounding to the storage
// type between the steps included), so the results are bitwise those of two k_step launches.
//
// A workgroup holds G lane groups of BG = blockDim.x / G lanes (BG a multiple of 64, so a
// wave is in one group).  Each group runs one tile: rows [y0, y1) of a replica, and either
//   - the whole row (nx <= BG; lane l is column l, neighbours wrap inside the group), or
//   - a strip (nx > BG) whose lane l is column x0 - 3 + l.  Each step loses one column at
//     each end (a lane needs its neighbours' densities for the stencils, and the second step
//     pulls from the neighbouring columns of the first step's output): the first step is
//     valid at lanes 1 .. BG - 2, the second step's densities at 2 .. BG - 3 and its results
//     at 3 .. BG - 4.  So strips overlap by six columns and store columns [x0, x0 + BG - 6).
// The group marches down the rows.  Stage 1 (step t) collides row r; its output row goes to
// LDS (populations 1, 3, 5, 6, 7, 8, which the pull of step t + 1 takes from the next
// column) and registers (0, 2, 4, which stay in the column).  Stage 2 (step t + 1) pulls row
// r - 2 for its density (the pull of row y reads output rows y - 1, y, y + 1), and collides
// row r - 3 (whose stencil needs the density of row r - 2), pulling that row again from the
// same LDS rows and registers, so that no pulled row is held across a barrier.  A tile of
// output rows [y0, y1) runs stage 1 on rows [y0 - 2, y1 + 2) and reads rows [y0 - 4, y1 + 4)
// of f*(t - 1).  Two workgroup barriers per row: after the stage-1 and stage-2 densities of
// a row are in LDS (A), and after the stage-1 output row is (B).
//
// LDS per group, each array padded by one slot on both sides of the BG lanes (W = BG + 2):
//   ring1[3][W]    rho(t) - rho0 of three consecutive rows
//   ring2[3][W]    rho(t+1) - rho0
//   F13[4][2][W]   populations 1, 3 of the last four stage-1 rows (stored type S)
//   F56[5][2][W]   populations 5, 6 of the last five
//   F78[3][2][W]   populations 7, 8 of the last three
// (each kept as long as a density pull or a collision pull still reads it).
//
// BGC > 0: the launch holds one group of BGC lanes per workgroup (a single lattice's strips), so
// W is a compile-time constant; F13 and F56 then hold six rows and the row loop is unrolled six
// times, which makes every ring slot a compile-time offset (an LDS instruction's immediate)
// instead of an address computed per access.

#include "lb_collide.h"
#include "lb_internal.h"
#include "lb_rng.h"

#include <type_traits>

namespace lbf {

template <typename S, typename R, int BGC = 0> constexpr unsigned step2_group_bytes(unsigned W)
{
    return W * (6 * (unsigned)sizeof(R) + (BGC ? 30u : 24u) * (unsigned)sizeof(S));
}

// CN: the replica set has correlated noise; replicas with noise == 2 add the fields of step t
// (xi) and t + 1 (xi + xi_plane) to modes 4 and 9 (see k_step).
template <typename S, typename R, bool PLAIN, bool CN, int BGC = 0>
__global__ void __launch_bounds__(512) k_step2(const S *__restrict__ xi, long long xi_plane,
                                               const S *__restrict__ fin, S *__restrict__ fout,
                                               const RepDesc *__restrict__ reps, const Tile *__restrict__ tiles,
                                               const int32_t *__restrict__ wgs,
                                               const unsigned long long *__restrict__ tdev,
                                               unsigned *__restrict__ flags, int toff)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const unsigned BX = BGC ? (unsigned)BGC : blockDim.x;
    const int gbeg = wgs[blockIdx.x];
    const unsigned G = BGC ? 1u : (unsigned)(wgs[blockIdx.x + 1] - gbeg);
    const unsigned BG = BX / G;
    const unsigned tid = threadIdx.x;
    const unsigned grp = BGC ? 0u : __builtin_amdgcn_readfirstlane(tid / BG);   // uniform per wave
    const unsigned l = tid - grp * BG;
    const unsigned W = BG + 2;

    // rows the workgroup marches over: the tallest of its tiles (every group keeps the barriers)
    int hmax = 0;
    for (unsigned g = 0; g < G; ++g) {
        const Tile q = tiles[gbeg + g];
        if (q.rep >= 0) hmax = max(hmax, q.y1 - q.y0);
    }
    const Tile tl = tiles[gbeg + grp];
    const bool gidle = tl.rep < 0;
    const RepDesc &d = reps[gidle ? 0 : tl.rep];
    const Consts<R> &c = consts<R>(d);
    const VConsts<R> vk = vconsts<R>(c);
    const unsigned nx = (unsigned)d.nx, ny = (unsigned)d.ny;
    const unsigned long long pitch = 9ull * nx;
    constexpr unsigned ES = sizeof(S);
    const unsigned rowb = 9u * nx * ES, nxb = nx * ES;
    const unsigned long long t = tdev[0] + (unsigned long long)toff;
    const S *__restrict__ P = fin + d.off;
    S *__restrict__ Qo = fout + d.off;

    unsigned char *gb = smem_raw + grp * step2_group_bytes<S, R, BGC>(W);
    R *ring1 = reinterpret_cast<R *>(gb);
    R *ring2 = ring1 + 3 * W;
    constexpr unsigned N13 = BGC ? 6 : 4, N56 = BGC ? 6 : 5;
    S *F13 = reinterpret_cast<S *>(ring2 + 3 * W);
    S *F56 = F13 + 2 * N13 * W;
    S *F78 = F56 + 2 * N56 * W;

    // columns.  whole: lane l is column l (lanes past the row duplicate column l mod nx and
    // never store; whole waves past it only keep the barriers).  strip: lane l is column
    // x0 - 3 + l (mod nx).  The last strip of a row stores columns [x0, nx), which need lanes
    // l < nx - x0 + 6 (its results at lanes 3 .. nx - x0 + 2 depend on lanes 0 .. nx - x0 + 5);
    // whole waves past them only keep the barriers.  The first idle lane's LDS slots are never
    // written, as the slots beyond a strip's ends are not: only lanes whose results are not
    // needed read them.
    const bool whole = nx <= BG;
    const int wl0 = (int)((tid - grp * BG) / 64 * 64);   // first lane of this wave in its group
    // uniform per wave; readfirstlane says so to the compiler, which otherwise treats branches on
    // it as divergent and moves the pull offsets into vector registers (a waterfall loop per load)
    const bool idle = __builtin_amdgcn_readfirstlane(
        (int)(gidle || (whole ? wl0 >= (int)nx : wl0 >= (int)nx - tl.x0 + 6))) != 0;
    unsigned xw;
    if (whole) {
        xw = l < nx ? l : l % nx;
    } else {
        const int xs = tl.x0 - 3 + (int)l;
        xw = (unsigned)(xs < 0 ? xs + (int)nx : (xs >= (int)nx ? xs - (int)nx : xs));
    }
    const unsigned cm = (xw == 0 ? nx - 1 : xw - 1) * ES;
    const unsigned c0 = xw * ES;
    const unsigned cp = (xw == nx - 1 ? 0 : xw + 1) * ES;
    // LDS slots of the lane and of its two neighbours (row arrays of W slots, lane l at l + 1)
    const unsigned i0 = l + 1;
    const unsigned im = whole ? (xw == 0 ? nx - 1 : xw - 1) + 1 : l;
    const unsigned ip = whole ? (xw == nx - 1 ? 0 : xw + 1) + 1 : l + 2;
    // ring1 of whole rows: the lane of column nx - 1 also writes slot 0 and the lane of
    // column 0 slot nx + 1, the wrap-around neighbours of columns 0 and nx - 1
    const bool xtra = whole && (l == 0 || l == nx - 1);
    const unsigned xslot = l == 0 ? nx + 1 : 0;
    // stage 2 stores lanes whose column is one of the tile's output columns
    const bool store2 = whole ? l < nx : (l >= 3 && l < BG - 3 && (unsigned)(tl.x0 - 3 + (int)l) < nx);

    // periodic row index; v is at most a few rows outside [0, ny) (more than one period only
    // for lattices a few rows tall), so the wrap is a short uniform loop, not a division
    auto wrapy = [ny](int v) -> unsigned {
        while (v < 0) v += (int)ny;
        while (v >= (int)ny) v -= (int)ny;
        return (unsigned)v;
    };
    struct Rows {
        __amdgpu_buffer_rsrc_t m, z, p;
    };
    auto rows_of = [&](int yy) -> Rows {
        return Rows{row_rsrc(P + (unsigned long long)wrapy(yy - 1) * pitch, rowb),
                    row_rsrc(P + (unsigned long long)wrapy(yy) * pitch, rowb),
                    row_rsrc(P + (unsigned long long)wrapy(yy + 1) * pitch, rowb)};
    };
    auto pull = [&](const Rows &rr, R f[Q]) {
        f[0] = (R)bld<S>(rr.z, c0, 0);
        f[1] = (R)bld<S>(rr.z, cm, nxb);
        f[2] = (R)bld<S>(rr.m, c0, 2 * nxb);
        f[3] = (R)bld<S>(rr.z, cp, 3 * nxb);
        f[4] = (R)bld<S>(rr.p, c0, 4 * nxb);
        f[5] = (R)bld<S>(rr.m, cm, 5 * nxb);
        f[6] = (R)bld<S>(rr.m, cp, 6 * nxb);
        f[7] = (R)bld<S>(rr.p, cp, 7 * nxb);
        f[8] = (R)bld<S>(rr.p, cm, 8 * nxb);
    };
    auto dens = [&](const R f[Q]) { return dens9<R, PLAIN>(f, c); };
    auto put1 = [&](unsigned slot, R v) {
        ring1[slot * W + i0] = v;
        if (xtra) ring1[slot * W + xslot] = v;
    };

    const int y0 = tl.y0, y1 = tl.y1;
    const int ys0 = y0 - 2, ys1 = y1 + 2;   // stage-1 rows [ys0, ys1)
    const int nit = hmax + 5;               // iterations r = ys0 + k, k < nit (uniform)
    unsigned st = 0;

    // stage-1 registers: pulled rows r (cur), r + 1 (nxt), r + 2 (in flight)
    R fa[Q], fb[Q], fc[Q];
    // stage-1 output populations that stay in the column: rings of three rows (row rho at
    // slot (rho - ys0) mod 3) and the population 2 of the row before the ring (F2x)
    S F0r[3], F2r[3], F4r[3], F2x = (S)0;
#pragma unroll
    for (int i = 0; i < 3; ++i) F0r[i] = F2r[i] = F4r[i] = (S)0;

    // prologue: densities of rows ys0 - 1 and ys0, populations of row ys0, loads of row
    // ys0 + 1 in flight
    {
        const Rows ra = rows_of(ys0 - 1), rb = rows_of(ys0);
        if (!idle) {
            pull(ra, fb);
            put1(0, dens(fb));
            pull(rb, fa);
            put1(1, dens(fa));
        }
        const Rows rc = rows_of(ys0 + 1);
        if (!idle) pull(rc, fb);
    }

    // the nine populations of step t + 1 pulled at row y (stored values, as a load would give
    // them) from the stage-1 output: own column rows y (0), y - 1 (2), y + 1 (4), LDS rows
    // y (1, 3), y - 1 (5, 6), y + 1 (7, 8)
    auto pull2 = [&](S v0, S v2, S v4, const S *f13, const S *f56, const S *f78, R g[Q]) {
        g[0] = (R)v0;
        g[1] = (R)f13[im];
        g[2] = (R)v2;
        g[3] = (R)f13[W + ip];
        g[4] = (R)v4;
        g[5] = (R)f56[im];
        g[6] = (R)f56[W + ip];
        g[7] = (R)f78[ip];
        g[8] = (R)f78[W + im];
    };
    // LDS row slots of the stage-1 output row rho = ys0 + k + J, for the iteration k whose index
    // in the unrolled group is U (k = U mod the group's length)
    constexpr int UN = BGC ? 6 : 3;
    auto s13 = [&](auto Uc, auto Jc, int k) {
        constexpr int U = decltype(Uc)::value, J = decltype(Jc)::value;
        if constexpr (BGC) return F13 + (unsigned)((U + J + 6) % 6) * 2 * W;
        else return F13 + (unsigned)((k + J) & 3) * 2 * W;
    };
    auto s56 = [&](auto Uc, auto Jc, int k) {
        constexpr int U = decltype(Uc)::value, J = decltype(Jc)::value;
        if constexpr (BGC) return F56 + (unsigned)((U + J + 6) % 6) * 2 * W;
        else return F56 + (unsigned)((k + J) % 5) * 2 * W;
    };
    auto s78 = [&](auto Uc, auto Jc, int) {
        constexpr int U = decltype(Uc)::value, J = decltype(Jc)::value;
        return F78 + (unsigned)((U + J + 6) % 3) * 2 * W;
    };
    using Jm4 = std::integral_constant<int, -4>;
    using Jm3 = std::integral_constant<int, -3>;
    using Jm2 = std::integral_constant<int, -2>;
    using Jm1 = std::integral_constant<int, -1>;
    using J0 = std::integral_constant<int, 0>;

    // one iteration; K = k mod 3 fixes the slots of the three-row rings (all modulo 3):
    //   ring1 (rho(t)):    row rho at slot (rho - ys0 + 1), so row r + j at K + 1 + j
    //   ring2 (rho(t+1)):  row rho at slot (rho - ys0), so row r - 2 + j at K + 1 + j
    //   F0r, F2r, F4r:     row rho at slot (rho - ys0), row r at K
    auto iter = [&](auto Uc, int k, R cur[Q], R nxt[Q], R nn[Q]) {
        constexpr unsigned K = decltype(Uc)::value % 3;
        const int r = ys0 + k;
        const bool s1 = !idle && r < ys1;                    // stage 1 on row r
        const bool p2 = !idle && r >= ys0 + 3 && r <= ys1;   // stage-2 density of row r - 2
        const bool c2 = !idle && r >= ys0 + 5 && r <= ys1;   // stage-2 collision of row r - 3
        // ---- phase 1: density of row r + 1 into ring1, loads of row r + 2, stage-2 density
        if (s1) put1((K + 2) % 3, dens(nxt));
        if (k + 1 < nit && r + 2 <= ys1) {
            const Rows rn = rows_of(r + 2);
            if (s1) pull(rn, nn);
        }
        if (p2) {
            R g[Q];
            pull2(F0r[(K + 1) % 3], F2r[K], F4r[(K + 2) % 3], s13(Uc, Jm2{}, k), s56(Uc, Jm3{}, k), s78(Uc, Jm1{}, k), g);
            ring2[((K + 1) % 3) * W + i0] = dens(g);
        }
        __syncthreads();
        // ---- phase 2: stage-2 collision of row r - 3 (pulled again), stage-1 collision of
        // row r and its output
        if (c2) {
            R g[Q];
            pull2(F0r[K], F2x, F4r[(K + 1) % 3], s13(Uc, Jm3{}, k), s56(Uc, Jm4{}, k), s78(Uc, Jm2{}, k), g);
            // densities of rows r - 4, r - 3, r - 2 at ring2 slots K + 2, K, K + 1
            const unsigned s0 = K * W, sm = ((K + 2) % 3) * W, sp = ((K + 1) % 3) * W;
            R lap, gx, gy;
            stencil9<R>(ring2[s0 + i0], ring2[s0 + ip], ring2[s0 + im], ring2[sp + i0], ring2[sp + ip],
                        ring2[sp + im], ring2[sm + i0], ring2[sm + ip], ring2[sm + im], lap, gx, gy);
            if (PLAIN) {
#pragma unroll
                for (int i = 0; i < Q; ++i) g[i] -= c.sub[i];
            }
            const unsigned y = (unsigned)(r - 3);   // inside [y0, y1): no wrap
            R xi4 = 0, xi9 = 0;
            if (CN && d.noise == 2) {
                const S *__restrict__ xr = xi + xi_plane + 2 * (d.xi_off + (long long)y * nx + xw);
                xi4 = (R)xr[0];
                xi9 = (R)xr[1];
            }
            const unsigned s2 = collide<R, CN>(g, lap, gx, gy, c, vk, d.noise, y * nx + xw, d.rep_id, t + 1, d.seed_lo,
                                               d.seed_hi, xi4, xi9);
            const auto Wr = row_rsrc(Qo + (unsigned long long)y * pitch, rowb);
            if (store2) {
                st |= s2;
#pragma unroll
                for (int i = 0; i < Q; ++i) bst<S>(Wr, c0, i * nxb, (S)(PLAIN ? add_rn<R>(g[i], c.sub[i]) : g[i]));
            }
        }
        // keep the two collisions apart: interleaved, their temporaries would be live together
        __builtin_amdgcn_sched_barrier(0);
        if (s1) {
            const unsigned s0 = ((K + 1) % 3) * W, sm = (K % 3) * W, sp = ((K + 2) % 3) * W;
            R lap, gx, gy;
            stencil9<R>(ring1[s0 + i0], ring1[s0 + i0 + 1], ring1[s0 + i0 - 1], ring1[sp + i0], ring1[sp + i0 + 1],
                        ring1[sp + i0 - 1], ring1[sm + i0], ring1[sm + i0 + 1], ring1[sm + i0 - 1], lap, gx, gy);
            if (PLAIN) {
#pragma unroll
                for (int i = 0; i < Q; ++i) cur[i] -= c.sub[i];
            }
            const unsigned yr = wrapy(r);
            R xi4 = 0, xi9 = 0;
            if (CN && d.noise == 2) {
                const S *__restrict__ xr = xi + 2 * (d.xi_off + (long long)yr * nx + xw);
                xi4 = (R)xr[0];
                xi9 = (R)xr[1];
            }
            const unsigned s1f = collide<R, CN>(cur, lap, gx, gy, c, vk, d.noise, yr * nx + xw, d.rep_id, t, d.seed_lo,
                                                d.seed_hi, xi4, xi9);
            st |= s1f;
            S o[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) o[i] = (S)(PLAIN ? add_rn<R>(cur[i], c.sub[i]) : cur[i]);
            F0r[K] = o[0];
            F2x = F2r[K];
            F2r[K] = o[2];
            F4r[K] = o[4];
            S *f13 = s13(Uc, J0{}, k), *f56 = s56(Uc, J0{}, k), *f78 = s78(Uc, J0{}, k);
            f13[i0] = o[1];
            f13[W + i0] = o[3];
            f56[i0] = o[5];
            f56[W + i0] = o[6];
            f78[i0] = o[7];
            f78[W + i0] = o[8];
        }
        __syncthreads();
    };
    using U0 = std::integral_constant<int, 0>;
    using U1 = std::integral_constant<int, 1>;
    using U2 = std::integral_constant<int, 2>;
    using U3 = std::integral_constant<int, 3>;
    using U4 = std::integral_constant<int, 4>;
    using U5 = std::integral_constant<int, 5>;
    for (int k = 0; k < nit; k += UN) {
        iter(U0{}, k, fa, fb, fc);
        if (k + 1 < nit) iter(U1{}, k + 1, fb, fc, fa);
        if (k + 2 < nit) iter(U2{}, k + 2, fc, fa, fb);
        if constexpr (UN == 6) {
            if (k + 3 < nit) iter(U3{}, k + 3, fa, fb, fc);
            if (k + 4 < nit) iter(U4{}, k + 4, fb, fc, fa);
            if (k + 5 < nit) iter(U5{}, k + 5, fc, fa, fb);
        }
    }
    // the stage-1 results of a storing lane are those of nodes whose second step it stores (its
    // column; rows outside the tile are also other tiles' rows), so the flags of every node and
    // step reach the word through some storing lane
    if (st && store2) atomicOr(flags, st);
}

// the group-width specialisation a launch takes: BGC = bx for one group per workgroup of 256 or
// 512 lanes in FP32 storage (the FP64 loop unrolled six times would outgrow the instruction
// cache), else 0 (runtime group width)
static int step2_bgc(int precision, int bx, int max_groups)
{
    return precision != 0 && max_groups == 1 && (bx == 256 || bx == 512) ? bx : 0;
}

template <typename S, typename R, bool PLAIN, bool CN, int BGC> static void launch_step2_b(const Step2Launch &a, hipStream_t s)
{
    const size_t lds = (size_t)a.max_groups * step2_group_bytes<S, R, BGC>((unsigned)(a.bx / a.max_groups + 2));
    hipLaunchKernelGGL((k_step2<S, R, PLAIN, CN, BGC>), dim3(a.nwg), dim3(a.bx), lds, s, (const S *)a.xi,
                       (long long)a.xi_plane, (const S *)a.fin, (S *)a.fout, a.reps, a.tiles, a.wgs, a.tdev, a.flags,
                       a.toff);
}

template <typename S, typename R, bool PLAIN, bool CN> static void launch_step2_t(const Step2Launch &a, hipStream_t s)
{
    if constexpr (sizeof(S) == 4) {
        const int bgc = step2_bgc(1, a.bx, a.max_groups);
        if (bgc == 256) return launch_step2_b<S, R, PLAIN, CN, 256>(a, s);
        if (bgc == 512) return launch_step2_b<S, R, PLAIN, CN, 512>(a, s);
    }
    launch_step2_b<S, R, PLAIN, CN, 0>(a, s);
}

template <typename S, typename R, bool PLAIN, int BGC> static hipError_t set_step2_limit_b(int bytes)
{
    hipError_t e = hipFuncSetAttribute((const void *)k_step2<S, R, PLAIN, false, BGC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_step2<S, R, PLAIN, true, BGC>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return e;
}

template <typename S, typename R, bool PLAIN> static hipError_t set_step2_limit(int bytes)
{
    hipError_t e = set_step2_limit_b<S, R, PLAIN, 0>(bytes);
    if constexpr (sizeof(S) == 4) {
        if (e == hipSuccess) e = set_step2_limit_b<S, R, PLAIN, 256>((int)step2_group_bytes<S, R, 256>(258));
        if (e == hipSuccess) e = set_step2_limit_b<S, R, PLAIN, 512>((int)step2_group_bytes<S, R, 512>(514));
    }
    return e;
}

hipError_t set_step2_lds_limit()
{
    const int fp32 = (int)(8 * step2_group_bytes<float, float>(512 / 8 + 2));
    const int fp64 = (int)(8 * step2_group_bytes<double, double>(512 / 8 + 2));
    hipError_t e = set_step2_limit<double, double, false>(fp64);
    if (e == hipSuccess) e = set_step2_limit<float, float, false>(fp32);
    if (e == hipSuccess) e = set_step2_limit<float, float, true>(fp32);
    return e;
}

template <typename K> static int blocks_per_cu(K kernel, int bx, size_t lds)
{
    int nb = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)kernel, bx, lds) == hipSuccess ? nb : 0;
}

template <bool PLAIN, int BGC> static int blocks_per_cu_f(bool cn, int bx, size_t lds)
{
    return cn ? blocks_per_cu(k_step2<float, float, PLAIN, true, BGC>, bx, lds)
              : blocks_per_cu(k_step2<float, float, PLAIN, false, BGC>, bx, lds);
}

int step2_blocks_per_cu(int precision, bool plain, bool cn, int bx, int max_groups)
{
    const size_t lds = step2_lds_bytes(precision, bx, max_groups);
    if (precision == 0)
        return cn ? blocks_per_cu(k_step2<double, double, false, true>, bx, lds)
                  : blocks_per_cu(k_step2<double, double, false, false>, bx, lds);
    const int bgc = step2_bgc(precision, bx, max_groups);
    if (plain)
        return bgc == 256 ? blocks_per_cu_f<true, 256>(cn, bx, lds)
                          : bgc == 512 ? blocks_per_cu_f<true, 512>(cn, bx, lds) : blocks_per_cu_f<true, 0>(cn, bx, lds);
    return bgc == 256 ? blocks_per_cu_f<false, 256>(cn, bx, lds)
                      : bgc == 512 ? blocks_per_cu_f<false, 512>(cn, bx, lds) : blocks_per_cu_f<false, 0>(cn, bx, lds);
}

size_t step2_lds_bytes(int precision, int bx, int max_groups)
{
    const unsigned W = (unsigned)(bx / max_groups + 2);
    if (precision == 0) return (size_t)max_groups * step2_group_bytes<double, double>(W);
    return (size_t)max_groups * (step2_bgc(precision, bx, max_groups) ? step2_group_bytes<float, float, 1>(W)
                                                                     : step2_group_bytes<float, float>(W));
}

template <typename S, typename R, bool PLAIN> static void launch_step2_cn(const Step2Launch &a, hipStream_t s)
{
    if (a.xi)
        launch_step2_t<S, R, PLAIN, true>(a, s);
    else
        launch_step2_t<S, R, PLAIN, false>(a, s);
}

hipError_t launch_step2(int precision, const Step2Launch &a, hipStream_t s)
{
    if (precision == 0)
        launch_step2_cn<double, double, false>(a, s);
    else if (a.plain)
        launch_step2_cn<float, float, true>(a, s);
    else
        launch_step2_cn<float, float, false>(a, s);
    return hipGetLastError();
}

}  // namespace lbf

