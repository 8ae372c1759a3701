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

}  // namespace lbf
