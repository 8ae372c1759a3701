// The fused step's work list: which tile (replica, strip, rows) each workgroup runs, and in
// what order.  Host code; the list is uploaded by lb_init and shared by every launch.

#include "lb_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

namespace lbf {

namespace {

// rows [y0, y1) of tile j when a strip of ny rows is cut into tiles of height about h:
// ceil(ny / h) tiles whose heights differ by at most one
struct Bands {
    int nt, ny;
    Bands(int ny_, double h) : nt(std::max(1, (int)ceil(ny_ / h - 1e-9))), ny(ny_) {}
    int y0(int j) const { return (int)((long long)j * ny / nt); }
    int y1(int j) const { return (int)((long long)(j + 1) * ny / nt); }
};

}  // namespace

// Tiles of every replica for strip width bx and about h rows per tile.  Workgroup i runs on
// XCD i mod 8, each XCD with its own L2.  Tiles that share data -- horizontal neighbours
// share the cache lines that straddle a strip boundary (pulls from x +- 1, halo columns),
// vertical neighbours share their boundary rows -- should run on the same XCD, while the
// workgroups in flight should cover whole lattice rows (HBM page locality).  So each
// replica's strips are split into 8 contiguous groups, one per XCD (replicas with fewer
// than 8 strips go whole to the least-loaded XCD), every XCD walks its tiles in bands
// (segment-major, then strip), and the eight per-XCD queues are interleaved so that list
// position j * 8 + k holds the j-th tile of XCD k.
// LBF_TILE_ORDER=rows (plain full-width bands) and =xcd (strip-major runs per XCD) select
// the alternatives.
std::vector<Tile> make_tiles(const std::vector<RepDesc> &reps, int bx, double h)
{
    constexpr int X = 8;
    const char *ord = getenv("LBF_TILE_ORDER");
    const bool rows_only = ord && strcmp(ord, "rows") == 0;
    const bool xcd_runs = ord && strcmp(ord, "xcd") == 0;
    std::vector<Tile> seq;
    if (rows_only || xcd_runs) {
        for (size_t r = 0; r < reps.size(); ++r) {
            const RepDesc &d = reps[r];
            const Bands B(d.ny, h);
            if (xcd_runs) {
                for (int x0 = 0; x0 < d.nx; x0 += bx)
                    for (int j = 0; j < B.nt; ++j) seq.push_back(Tile{(int32_t)r, x0, B.y0(j), B.y1(j)});
            } else {
                for (int j = 0; j < B.nt; ++j)
                    for (int x0 = 0; x0 < d.nx; x0 += bx) seq.push_back(Tile{(int32_t)r, x0, B.y0(j), B.y1(j)});
            }
        }
        if (rows_only) return seq;
        const int T = (int)seq.size();
        std::vector<Tile> out;
        out.reserve(T);
        const int base = T / X, extra = T % X;
        std::vector<int> start(X + 1, 0);
        for (int k = 0; k < X; ++k) start[k + 1] = start[k] + base + (k < extra ? 1 : 0);
        for (int j = 0; j <= base; ++j)
            for (int k = 0; k < X; ++k)
                if (start[k] + j < start[k + 1]) out.push_back(seq[start[k] + j]);
        return out;
    }
    std::vector<std::vector<Tile>> q(X);
    std::vector<long long> load(X, 0);
    // larger replicas first, so that whole small replicas fill in the balance
    std::vector<int> order(reps.size());
    for (size_t r = 0; r < reps.size(); ++r) order[r] = (int)r;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (long long)reps[a].nx * reps[a].ny > (long long)reps[b].nx * reps[b].ny;
    });
    for (int r : order) {
        const RepDesc &d = reps[r];
        const Bands B(d.ny, h);
        const int ns = (d.nx + bx - 1) / bx;
        if (ns >= X) {
            for (int k = 0; k < X; ++k) {
                const int s0 = k * ns / X, s1 = (k + 1) * ns / X;
                for (int j = 0; j < B.nt; ++j)
                    for (int sidx = s0; sidx < s1; ++sidx) {
                        q[k].push_back(Tile{(int32_t)r, sidx * bx, B.y0(j), B.y1(j)});
                        load[k] += (long long)bx * (B.y1(j) - B.y0(j));
                    }
            }
        } else {
            const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            for (int j = 0; j < B.nt; ++j)
                for (int sidx = 0; sidx < ns; ++sidx) {
                    q[k].push_back(Tile{(int32_t)r, sidx * bx, B.y0(j), B.y1(j)});
                    load[k] += (long long)bx * (B.y1(j) - B.y0(j));
                }
        }
    }
    size_t common = q[0].size();
    for (int k = 1; k < X; ++k) common = std::min(common, q[k].size());
    std::vector<Tile> out;
    for (size_t j = 0; j < common; ++j)
        for (int k = 0; k < X; ++k) out.push_back(q[k][j]);
    // the uneven remainder keeps its per-XCD order; its XCD placement is no longer exact
    for (int k = 0; k < X; ++k)
        for (size_t j = common; j < q[k].size(); ++j) out.push_back(q[k][j]);
    return out;
}

// Lane groups per workgroup for a replica of width nx in workgroups of bx lanes: the most
// groups (at most 8) of a width that is a multiple of 64 and holds the whole row; 1 (a strip)
// when the row is wider than bx.
static int groups_for(int nx, int bx)
{
    for (int G = 8; G > 1; --G)
        if (bx % (64 * G) == 0 && bx / G >= nx) return G;
    return 1;
}

// The two-step kernel's work list.  Strips of a replica wider than a workgroup overlap by six
// columns (each stores bx - 6); whole rows of narrower replicas are packed G to a workgroup,
// G vertically adjacent tiles of one replica (they share boundary rows), with empty groups
// (rep = -1) after the last tile of a replica.  XCD placement as in make_tiles: a replica
// with at least 8 strips is split into 8 contiguous strip groups, one per XCD queue; smaller
// ones go whole to the least-loaded queue; the queues are interleaved (workgroup i runs on
// XCD i mod 8).
int make_tiles2(const std::vector<RepDesc> &reps, int bx, double h, std::vector<Tile> &tiles,
                std::vector<int32_t> &wgs)
{
    constexpr int X = 8;
    typedef std::vector<Tile> WG;
    std::vector<std::vector<WG>> q(X);
    std::vector<long long> load(X, 0);
    std::vector<int> order(reps.size());
    for (size_t r = 0; r < reps.size(); ++r) order[r] = (int)r;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (long long)reps[a].nx * reps[a].ny > (long long)reps[b].nx * reps[b].ny;
    });
    int gmax = 1;
    for (int r : order) {
        const RepDesc &d = reps[r];
        const Bands B(d.ny, h);
        if (d.nx > bx) {
            const int w2 = bx - 6;
            const int ns = (d.nx + w2 - 1) / w2;
            const int parts = ns >= X ? X : 1;
            for (int k = 0; k < parts; ++k) {
                const int qk = parts == X ? k : (int)(std::min_element(load.begin(), load.end()) - load.begin());
                const int s0 = k * ns / parts, s1 = (k + 1) * ns / parts;
                for (int j = 0; j < B.nt; ++j)
                    for (int sidx = s0; sidx < s1; ++sidx) {
                        q[qk].push_back(WG{Tile{(int32_t)r, sidx * w2, B.y0(j), B.y1(j)}});
                        load[qk] += (long long)bx * (B.y1(j) - B.y0(j));
                    }
            }
        } else {
            const int G = groups_for(d.nx, bx);
            gmax = std::max(gmax, G);
            const int qk = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            for (int j0 = 0; j0 < B.nt; j0 += G) {
                WG w;
                for (int g = 0; g < G; ++g)
                    w.push_back(j0 + g < B.nt ? Tile{(int32_t)r, 0, B.y0(j0 + g), B.y1(j0 + g)} : Tile{-1, 0, 0, 0});
                q[qk].push_back(w);
                load[qk] += (long long)bx * (B.y1(j0) - B.y0(j0));
            }
        }
    }
    tiles.clear();
    wgs.clear();
    size_t common = q[0].size();
    for (int k = 1; k < X; ++k) common = std::min(common, q[k].size());
    auto emit = [&](const WG &w) {
        wgs.push_back((int32_t)tiles.size());
        tiles.insert(tiles.end(), w.begin(), w.end());
    };
    for (size_t j = 0; j < common; ++j)
        for (int k = 0; k < X; ++k) emit(q[k][j]);
    for (int k = 0; k < X; ++k)
        for (size_t j = common; j < q[k].size(); ++j) emit(q[k][j]);
    wgs.push_back((int32_t)tiles.size());
    return gmax;
}

long long max_tiles2(const std::vector<int> &nx, const std::vector<int> &ny)
{
    long long t = 0;
    for (size_t r = 0; r < nx.size(); ++r) {
        const long long strips = nx[r] > STEP2_MIN_BX ? (nx[r] + STEP2_MIN_BX - 7) / (STEP2_MIN_BX - 6) : 1;
        t += strips * ((ny[r] + STEP2_MIN_H - 1) / STEP2_MIN_H) + 8;
    }
    return t;
}

}  // namespace lbf
