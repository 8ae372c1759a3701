// Kernels of the fluctuating modified-equilibrium (Swift) D2Q9 lattice Boltzmann step,
// Gross, Adhikari, Cates & Varnik, arXiv:1009.0254, for gfx950.
//
// Memory holds the post-collision populations f*(r, t-1); the fused step pulls
// f_i(r, t) = f*_i(r - c_i, t-1) (streaming, eq. gen-lbe), collides and writes f*(r, t).
// Each workgroup owns a strip of blockDim.x columns and marches down rows y0..y1-1,
// keeping the density of rows y-1, y, y+1 in a 4-slot LDS ring so that the 9-point
// stencils (App. B Laplacian; isotropic gradient) never re-read populations from HBM.
// The two halo columns of the strip are pulled by lanes 0 and 1 of the first wave (a strip
// that spans its whole row reads them from its own columns instead).
// Loads run two rows ahead: while row y collides, the populations of row y+2 are in
// flight (on gfx950 a workgroup barrier only waits for LDS, not for global loads).
// Populations are row-interleaved ([y][i][x], see pop_at): a row of the lattice is one
// contiguous block.  The tile list (lb_tiles.hip) keeps neighbouring tiles on one XCD.
// Every access goes through a buffer descriptor of its row (no per-lane 64-bit address
// arithmetic); stores carry the nontemporal policy.

#include "lb_collide.h"
#include "lb_internal.h"
#include "lb_rng.h"

#include <math.h>

namespace lbf {

// ------------------------------------------------------------------ fused step kernel

template <typename S, typename R, bool PLAIN, bool CN, bool WHOLE>
__global__ void __launch_bounds__(512) k_step(const S *__restrict__ xi, const S *__restrict__ fin, S *__restrict__ fout,
                                              const RepDesc *__restrict__ reps, const Tile *__restrict__ tiles,
                                              const unsigned long long *__restrict__ tdev,
                                              unsigned *__restrict__ flags, int toff)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R *ring = reinterpret_cast<R *>(smem_raw);
    const unsigned BX = blockDim.x;
    const unsigned WL = BX + 2;
    const Tile tl = tiles[blockIdx.x];
    const RepDesc &d = reps[tl.rep];
    const Consts<R> &c = consts<R>(d);
    const VConsts<R> vk = vconsts<R>(c);
    const unsigned nx = (unsigned)d.nx, ny = (unsigned)d.ny;
    const unsigned long long pitch = 9ull * nx;   // elements per lattice row
    constexpr unsigned ESZ = sizeof(S);
    const unsigned rowb = 9u * nx * ESZ, nxb = nx * ESZ;   // bytes per row and per population plane
    const unsigned long long t = tdev[0] + (unsigned long long)toff;
    const S *__restrict__ P = fin + d.off;
    S *__restrict__ Qo = fout + d.off;
    const unsigned tid = threadIdx.x;

    // lane columns (loop invariant); x may exceed nx in a ragged or narrow strip: it wraps
    // and such lanes only supply densities.  Columns are kept as byte offsets.
    constexpr unsigned ES = sizeof(S);
    const unsigned xg = (unsigned)tl.x0 + tid;
    const unsigned xw = xg % nx;
    const unsigned cm = (xw == 0 ? nx - 1 : xw - 1) * ES;
    const unsigned c0 = xw * ES;
    const unsigned cp = (xw == nx - 1 ? 0 : xw + 1) * ES;
    const bool store = xg < nx;
    // A strip that spans its whole row (x0 = 0, nx <= BX; only in the WHOLE variant) has its
    // halo densities among its own columns: the lane of column nx - 1 also writes the west
    // halo slot 0 and the lane of column 0 the east halo slot nx + 1, the slot that lane
    // nx - 1 reads.  Such a strip pulls no halo columns, and its whole waves past the row
    // (x >= nx) only keep the barriers.  Other strips pull the two halo columns with lanes 0
    // (left) and 1 (right).
    const bool whole = WHOLE && tl.x0 == 0 && nx <= BX;
    const bool idle = WHOLE && __builtin_amdgcn_readfirstlane(whole && (tid & ~63u) >= nx);   // uniform per wave
    const bool xtra = whole && (tid == 0 || tid == nx - 1);
    const unsigned xslot = tid == 0 ? nx + 1 : 0;
    const bool halo = !whole && tid < 2;
    const unsigned hxw = tid == 0 ? ((unsigned)tl.x0 + nx - 1) % nx : ((unsigned)tl.x0 + BX) % nx;
    const unsigned hcm = (hxw == 0 ? nx - 1 : hxw - 1) * ES;
    const unsigned hc0 = hxw * ES;
    const unsigned hcp = (hxw == nx - 1 ? 0 : hxw + 1) * ES;
    const unsigned hslot = tid == 0 ? 0 : BX + 1;

    auto wrapy = [ny](int v) -> unsigned { return (unsigned)(v < 0 ? v + (int)ny : (v >= (int)ny ? v - (int)ny : v)); };

    // pulled populations f_i(x, yy) = f*_i(x - c_i, yy - c_iy): uniform row pointers, lane
    // byte offsets
    // the three stored rows that the pull of row yy reads (descriptors built outside any
    // divergent branch, so that they stay in scalar registers)
    struct Rows {
        __amdgpu_buffer_rsrc_t m, z, p;
    };
    auto rows_of = [&](int yy) -> Rows {
        return Rows{row_rsrc(P + (unsigned long long)wrapy(yy - 1) * pitch, rowb),
                    row_rsrc(P + (unsigned long long)wrapy(yy) * pitch, rowb),
                    row_rsrc(P + (unsigned long long)wrapy(yy + 1) * pitch, rowb)};
    };
    auto pull = [&](const Rows &rr, unsigned o0, unsigned ol, unsigned orr, R f[Q]) {
        const auto Rm = rr.m, R0 = rr.z, Rp = rr.p;
        f[0] = (R)bld<S>(R0, o0, 0);
        f[1] = (R)bld<S>(R0, ol, nxb);
        f[2] = (R)bld<S>(Rm, o0, 2 * nxb);
        f[3] = (R)bld<S>(R0, orr, 3 * nxb);
        f[4] = (R)bld<S>(Rp, o0, 4 * nxb);
        f[5] = (R)bld<S>(Rm, ol, 5 * nxb);
        f[6] = (R)bld<S>(Rm, orr, 6 * nxb);
        f[7] = (R)bld<S>(Rp, orr, 7 * nxb);
        f[8] = (R)bld<S>(Rp, ol, 8 * nxb);
    };
    // density deviation of pulled (stored) values
    auto dens = [&](const R f[Q]) { return dens9<R, PLAIN>(f, c); };

    const int y0 = tl.y0, y1 = tl.y1;
    unsigned st = 0;

    // stencils from the LDS ring and the collision of row y (populations cur, pulled)
    auto finish_row = [&](int y, R cur[Q], unsigned sp) {
        const unsigned s0 = ((unsigned)y & 3u) * WL, sm = ((unsigned)(y - 1) & 3u) * WL;
        const R C = ring[s0 + tid + 1], E = ring[s0 + tid + 2], Wv = ring[s0 + tid];
        const R N = ring[sp + tid + 1], NE = ring[sp + tid + 2], NW = ring[sp + tid];
        const R Sv = ring[sm + tid + 1], SE = ring[sm + tid + 2], SW = ring[sm + tid];
        R lap, gx, gy;
        stencil9<R>(C, E, Wv, N, NE, NW, Sv, SE, SW, lap, gx, gy);
        if (PLAIN) {
#pragma unroll
            for (int i = 0; i < Q; ++i) cur[i] -= c.sub[i];
        }
        R xi4 = 0, xi9 = 0;
        if (CN && d.noise == 2) {
            const S *__restrict__ xr = xi + 2 * (d.xi_off + (long long)y * nx + xw);
            xi4 = (R)xr[0];
            xi9 = (R)xr[1];
        }
        st |= collide<R, CN>(cur, lap, gx, gy, c, vk, d.noise, (unsigned)y * nx + xw, d.rep_id, t, d.seed_lo, d.seed_hi,
                         xi4, xi9);
        const auto W = row_rsrc(Qo + (unsigned long long)(unsigned)y * pitch, rowb);
        if (store) {
#pragma unroll
            for (int i = 0; i < Q; ++i) bst<S>(W, c0, i * nxb, (S)(PLAIN ? add_rn<R>(cur[i], c.sub[i]) : cur[i]));
        }
    };

    R fa[Q], fb[Q], hv[Q];
    // prologue: densities of rows y0-1 and y0 (own and halo columns), populations of row y0
    const Rows ra = rows_of(y0 - 1), rb = rows_of(y0);
    // the lane's density of row yy into the ring (and, in a whole-row strip, into a halo slot)
    auto put = [&](int yy, R v) {
        const unsigned sl = ((unsigned)yy & 3u) * WL;
        ring[sl + tid + 1] = v;
        if (xtra) ring[sl + xslot] = v;
    };
    if (!idle) {
        pull(ra, c0, cm, cp, fb);
        put(y0 - 1, dens(fb));
        if (halo) {
            pull(ra, hc0, hcm, hcp, hv);
            ring[((unsigned)(y0 - 1) & 3u) * WL + hslot] = dens(hv);
            pull(rb, hc0, hcm, hcp, hv);
            ring[((unsigned)y0 & 3u) * WL + hslot] = dens(hv);
        }
        pull(rb, c0, cm, cp, fa);
        put(y0, dens(fa));
    }

    // row y+1 is already in flight when row y starts; row y+2 is issued before the barrier
    // and lands while row y collides
    R fcq[Q];
    const Rows rc = rows_of(y0 + 1);
    if (!idle) {
        pull(rc, c0, cm, cp, fb);
        if (halo) pull(rc, hc0, hcm, hcp, hv);
    }
    auto row = [&](int y, R cur[Q], R nxt[Q], R nn[Q]) {
        const unsigned sp = ((unsigned)(y + 1) & 3u) * WL;
        if (!idle) {
            put(y + 1, dens(nxt));
            if (halo) ring[sp + hslot] = dens(hv);
        }
        if (y + 1 < y1) {
            const Rows rn = rows_of(y + 2);
            if (!idle) {
                pull(rn, c0, cm, cp, nn);
                if (halo) pull(rn, hc0, hcm, hcp, hv);
            }
        }
        __syncthreads();
        if (!idle) finish_row(y, cur, sp);
    };
    for (int y = y0; y < y1; y += 3) {
        row(y, fa, fb, fcq);
        if (y + 1 < y1) row(y + 1, fb, fcq, fa);
        if (y + 2 < y1) row(y + 2, fcq, fa, fb);
    }
    if (st && store) atomicOr(flags, st);
}

__global__ void k_advance_time(unsigned long long *tdev, long long by)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) tdev[0] += (unsigned long long)by;
}

// ------------------------------------------------------------------ initial state

__device__ double init_density(const RepDesc &d, int x, int y, uint32_t rep_index)
{
    const double *a = d.init_arg;
    switch (d.init_kind) {
    case 1:
        return a[1] + 0.5 * (a[0] - a[1]) * (tanh((y - a[2]) / a[4]) - tanh((y - a[3]) / a[4]));
    case 2: {
        double nu[6];
        normals6<double>((uint32_t)y * (uint32_t)d.nx + (uint32_t)x, d.rep_id, ~0ull, d.seed_lo, d.seed_hi, nu);
        return d.cd.rho0 + a[0] * nu[0];
    }
    case 3: {
        const double th = 2.0 * (a[0] * x / d.nx + a[1] * y / d.ny);   // in units of pi
        return d.cd.rho0 + a[2] * cospi(th);
    }
    default:
        return d.cd.rho0;
    }
}

__global__ void k_init_rho(double *rho, const RepDesc *__restrict__ reps, int rep_index)
{
    const RepDesc &d = reps[rep_index];
    const long long n = (long long)d.nx * d.ny;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k / d.nx), x = (int)(k - (long long)y * d.nx);
        rho[k] = init_density(d, x, y, rep_index);
    }
}

// f(r, 0) = T^-1 m^eq(rho, u, grad rho, lap rho), written where the pull of the first
// step finds it: slot r - c_i of plane i
template <typename S>
__global__ void k_init_f(S *__restrict__ f, const double *__restrict__ rho, const RepDesc *__restrict__ reps,
                         int rep_index)
{
    const RepDesc &d = reps[rep_index];
    const int nx = d.nx, ny = d.ny;
    const long long n = (long long)nx * ny;
    S *P = f + d.off;
    const int cx[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int cy[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k / nx), x = (int)(k - (long long)y * nx);
        auto at = [&](int dx, int dy) {
            int xx = x + dx, yy = y + dy;
            xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
            yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
            return rho[(long long)yy * nx + xx];
        };
        const double C = at(0, 0), E = at(1, 0), W = at(-1, 0), N = at(0, 1), Sd = at(0, -1);
        const double NE = at(1, 1), NW = at(-1, 1), SW = at(-1, -1), SE = at(1, -1);
        const double lap = (4 * ((E + W) + (N + Sd)) + ((NE + NW) + (SW + SE)) - 20 * C) / 6.0;
        const double gx = (4 * (E - W) + (NE - NW) + (SE - SW)) / 12.0;
        const double gy = (4 * (N - Sd) + (NE - SE) + (NW - SW)) / 12.0;
        double ux = 0, uy = 0;
        if (d.init_kind == 3) {
            const double th = 2.0 * (d.init_arg[0] * x / nx + d.init_arg[1] * y / ny);
            const double c = cospi(th);
            ux = d.init_arg[5] + d.init_arg[3] * c;
            uy = d.init_arg[4] * c;
        }
        const double r = C;
        const double jx = r * ux, jy = r * uy;
        // Table II at (rho, j) with the square-gradient terms
        const Consts<double> &c = d.cd;
        const double xx = r - (c.rho0 - c.xr0);
        const double x2 = xx * xx;
        const double pex = c.c0m * r + r * xx * (c.A + c.B * x2) - x2 * (0.5 * c.A + 0.25 * c.B * x2);
        const double piso = pex - c.kappa * r * lap;
        double m[Q];
        m[0] = r;
        m[1] = jx;
        m[2] = jy;
        m[3] = 3 * (jx * jx + jy * jy) / r + 6 * piso;
        m[4] = (jx * jx - jy * jy) / r + c.kappa * (gx * gx - gy * gy);
        m[5] = jx * jy / r + c.kappa * gx * gy;
        m[6] = 0;
        m[7] = 0;
        m[8] = -6 * piso - 3 * c.kappa * (gx * gx + gy * gy);
        const double M1 = m[0], M2 = 3 * m[1], M3 = 3 * m[2], M4 = 0.25 * m[3], M5 = 2.25 * m[4];
        const double M6 = 9 * m[5], M7 = 1.5 * m[6], M8 = 1.5 * m[7], M9 = 0.0625 * m[8];
        double fo[Q];
        fo[0] = (M1 - 2 * M4 + 2 * M9) * (4.0 / 9.0);
        fo[1] = (M1 + M2 + M4 + M5 - M7 - 4 * M9) / 9.0;
        fo[2] = (M1 + M3 + M4 - M5 - M8 - 4 * M9) / 9.0;
        fo[3] = (M1 - M2 + M4 + M5 + M7 - 4 * M9) / 9.0;
        fo[4] = (M1 - M3 + M4 - M5 + M8 - 4 * M9) / 9.0;
        fo[5] = (M1 + M2 + M3 + 4 * M4 + M6 + 2 * M7 + 2 * M8 + 8 * M9) / 36.0;
        fo[6] = (M1 - M2 + M3 + 4 * M4 - M6 - 2 * M7 + 2 * M8 + 8 * M9) / 36.0;
        fo[7] = (M1 - M2 - M3 + 4 * M4 + M6 - 2 * M7 - 2 * M8 + 8 * M9) / 36.0;
        fo[8] = (M1 + M2 - M3 + 4 * M4 - M6 + 2 * M7 - 2 * M8 + 8 * M9) / 36.0;
        for (int i = 0; i < Q; ++i) {
            int xs = x - cx[i], ys = y - cy[i];
            xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
            ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
            P[pop_at(nx, i, xs, ys)] = (S)(fo[i] - d.shift[i]);
        }
    }
}

// ------------------------------------------------------------------ moments and totals

constexpr int RED_THREADS = 256;

// Pre-collision moments (pull, then m = T f in FP64) of one replica; optional planes
// [9][ny][nx]; per-block partial sums of (rho, jx, jy, |j|^2, (-1)^x jx, (-1)^y jy).
template <typename S>
__global__ void __launch_bounds__(RED_THREADS) k_moments(const S *__restrict__ f, const RepDesc *__restrict__ reps,
                                                         int rep_index, double *__restrict__ m9,
                                                         double *__restrict__ partials)
{
    const RepDesc &d = reps[rep_index];
    const int nx = d.nx, ny = d.ny;
    const long long n = (long long)nx * ny;
    const S *P = f + d.off;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k / nx), x = (int)(k - (long long)y * nx);
        double g[Q];
        pull_node(P, nx, ny, x, y, d.shift, g);
        const double sa = (g[1] + g[2]) + (g[3] + g[4]);
        const double sd = (g[5] + g[6]) + (g[7] + g[8]);
        double m[Q];
        m[0] = g[0] + sa + sd;
        const double ax = g[1] - g[3], ay = g[2] - g[4], d68 = g[5] - g[7], d97 = g[8] - g[6];
        m[1] = ax + d68 + d97;
        m[2] = ay + d68 - d97;
        m[3] = -2 * g[0] + sa + 4 * sd;
        m[4] = (g[1] + g[3]) - (g[2] + g[4]);
        m[5] = (g[5] + g[7]) - (g[6] + g[8]);
        m[6] = -ax + 2 * (d68 + d97);
        m[7] = -ay + 2 * (d68 - d97);
        m[8] = 2 * g[0] - 4 * sa + 8 * sd;
        if (m9) {
#pragma unroll
            for (int a = 0; a < Q; ++a) m9[a * n + k] = m[a];
        }
        acc[0] += m[0];
        acc[1] += m[1];
        acc[2] += m[2];
        acc[3] += m[1] * m[1] + m[2] * m[2];
        acc[4] += (x & 1) ? -m[1] : m[1];
        acc[5] += (y & 1) ? -m[2] : m[2];
    }
    __shared__ double red[6][RED_THREADS];
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int c = 0; c < 6; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 6; ++c) partials[blockIdx.x * 6 + c] = red[c][0];
}

__global__ void __launch_bounds__(RED_THREADS) k_reduce_partials(const double *__restrict__ partials, int nblocks,
                                                                 double *__restrict__ tot)
{
    __shared__ double red[6][RED_THREADS];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int c = 0; c < 6; ++c) acc[c] += partials[b * 6 + c];
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int c = 0; c < 6; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 6; ++c) tot[c] = red[c][0];
}

// ------------------------------------------------------------------ RNG exposure

template <typename R>
__global__ void k_normals(uint64_t seed, uint32_t replica, unsigned long long t, long long n, double *out)
{
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
        R nu[6];
        normals6<R>((uint32_t)k, replica, t, (uint32_t)seed, (uint32_t)(seed >> 32), nu);
        for (int j = 0; j < 6; ++j) out[6 * k + j] = (double)nu[j];
    }
}

__global__ void k_philox(uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1, long long n, uint32_t *out)
{
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
        const uint4 x = philox10(make_uint4((uint32_t)k, c1, c2, c3), k0, k1);
        out[4 * k + 0] = x.x;
        out[4 * k + 1] = x.y;
        out[4 * k + 2] = x.z;
        out[4 * k + 3] = x.w;
    }
}

// ------------------------------------------------------------------ launchers

static int grid_for(long long n, int threads, int cap = 65536)
{
    long long g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

template <typename S, typename R, bool PLAIN, bool CN>
static void launch_step_t(const StepLaunch &a, hipStream_t s)
{
    const dim3 grid(a.ntiles), block(a.bx);
    const size_t lds = 4 * (a.bx + 2) * sizeof(R);
    if (a.whole)
        hipLaunchKernelGGL((k_step<S, R, PLAIN, CN, true>), grid, block, lds, s, (const S *)a.xi, (const S *)a.fin,
                           (S *)a.fout, a.reps, a.tiles, a.tdev, a.flags, a.toff);
    else
        hipLaunchKernelGGL((k_step<S, R, PLAIN, CN, false>), grid, block, lds, s, (const S *)a.xi, (const S *)a.fin,
                           (S *)a.fout, a.reps, a.tiles, a.tdev, a.flags, a.toff);
}

hipError_t launch_step(int precision, const StepLaunch &a, hipStream_t s)
{
    // the correlated-noise read is compiled only into the variant for handles that have it,
    // the whole-row strip handling only into the variant for tile lists that have such strips
    const bool cn = a.xi != nullptr;
    if (precision == 0)
        cn ? launch_step_t<double, double, false, true>(a, s) : launch_step_t<double, double, false, false>(a, s);
    else if (a.plain)
        cn ? launch_step_t<float, float, true, true>(a, s) : launch_step_t<float, float, true, false>(a, s);
    else
        cn ? launch_step_t<float, float, false, true>(a, s) : launch_step_t<float, float, false, false>(a, s);
    return hipGetLastError();
}

hipError_t launch_advance_time(unsigned long long *tdev, long long by, hipStream_t s)
{
    hipLaunchKernelGGL(k_advance_time, dim3(1), dim3(64), 0, s, tdev, by);
    return hipGetLastError();
}

hipError_t launch_init(int precision, void *f, double *rho_tmp, const RepDesc *d_reps, const RepDesc &h_rep,
                       int rep_index, hipStream_t s)
{
    const long long n = (long long)h_rep.nx * h_rep.ny;
    const int g = grid_for(n, 256);
    hipLaunchKernelGGL(k_init_rho, dim3(g), dim3(256), 0, s, rho_tmp, d_reps, rep_index);
    if (precision == 0)
        hipLaunchKernelGGL(k_init_f<double>, dim3(g), dim3(256), 0, s, (double *)f, rho_tmp, d_reps, rep_index);
    else
        hipLaunchKernelGGL(k_init_f<float>, dim3(g), dim3(256), 0, s, (float *)f, rho_tmp, d_reps, rep_index);
    return hipGetLastError();
}

hipError_t launch_moments(int precision, const void *f, const RepDesc *d_reps, const RepDesc &h_rep, int rep_index,
                          double *d_m9, double *partials, int nblocks, double *d_tot, hipStream_t s)
{
    if (precision == 0)
        hipLaunchKernelGGL(k_moments<double>, dim3(nblocks), dim3(RED_THREADS), 0, s, (const double *)f, d_reps,
                           rep_index, d_m9, partials);
    else
        hipLaunchKernelGGL(k_moments<float>, dim3(nblocks), dim3(RED_THREADS), 0, s, (const float *)f, d_reps,
                           rep_index, d_m9, partials);
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(RED_THREADS), 0, s, partials, nblocks, d_tot);
    return hipGetLastError();
}

hipError_t launch_normals(uint64_t seed, uint32_t replica, uint64_t t, int64_t n, int precision, double *d_out,
                          hipStream_t s)
{
    const int g = grid_for(n, 256);
    if (precision == 0)
        hipLaunchKernelGGL(k_normals<double>, dim3(g), dim3(256), 0, s, seed, replica, (unsigned long long)t,
                           (long long)n, d_out);
    else
        hipLaunchKernelGGL(k_normals<float>, dim3(g), dim3(256), 0, s, seed, replica, (unsigned long long)t,
                           (long long)n, d_out);
    return hipGetLastError();
}

hipError_t launch_philox(uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1, int64_t n, uint32_t *d_out,
                         hipStream_t s)
{
    const int g = grid_for(n, 256);
    hipLaunchKernelGGL(k_philox, dim3(g), dim3(256), 0, s, c1, c2, c3, k0, k1, (long long)n, d_out);
    return hipGetLastError();
}

}  // namespace lbf
