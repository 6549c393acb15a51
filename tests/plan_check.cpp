// Host checks of the symbolic plan of a panel class (plan.cpp), built with
// g++ by tests/test_plan_host.py: no device is involved.
//
// For several lateral grids, panel depths and leaf sizes it builds the
// nested-dissection fronts and checks what the solves and the factorisation
// rely on (Sec. 2.1-2.2: fronts of pivots and update sets, the extend-add
// between a child's update set and its parent front):
//  * the elimination order is a permutation of the panel's nodes, each front's
//    pivots consecutive, plane-major over its cell rectangle (s = cells * nz);
//  * each child's update entry has a distinct position in its parent front
//    (push map), at the same elimination position, and the parent's pull map
//    points back at it;
//  * the first child's entries that land on a parent pivot carry that pivot's
//    elimination position (the forward pass adds them into the parent's
//    right-hand side there), all others -1, so every entry has one writer;
//  * the per-front storage regions tile their buffers without overlap.
// Prints one line per case and exits 1 at the first failed check.
#include <cstdio>
#include <vector>

#include "plan.hpp"

using namespace hsw;

#define CHECK(cond, ...)                          \
    do {                                          \
        if (!(cond)) {                            \
            std::printf("FAIL " __VA_ARGS__);     \
            std::printf("\n");                    \
            return 1;                             \
        }                                         \
    } while (0)

// [off[k], off[k] + len[k]) over all k must tile [0, total) exactly.
static bool tiles(const std::vector<long long>& off, const std::vector<long long>& len, long long total) {
    std::vector<char> used(total > 0 ? total : 1, 0);
    long long sum = 0;
    for (size_t k = 0; k < off.size(); ++k) {
        if (off[k] < 0 || off[k] + len[k] > total) return false;
        for (long long i = off[k]; i < off[k] + len[k]; ++i) {
            if (used[i]) return false;
            used[i] = 1;
        }
        sum += len[k];
    }
    return sum == total;
}

static int check(int Nx, int Ny, int nz, int leaf) {
    LatTree lt = build_lateral_tree(Nx, Ny, leaf);
    PanelClass pc;
    const std::string err = build_class(lt, nz, pc);
    CHECK(err.empty(), "build_class %dx%dx%d: %s", Nx, Ny, nz, err.c_str());
    const int nf = pc.nfront, naux = pc.naux;
    CHECK(naux == Nx * Ny * nz, "naux %d", naux);
    // the elimination order
    std::vector<int> seen(naux, 0);
    for (int e = 0; e < naux; ++e) {
        const int b = pc.perm[e];
        CHECK(b >= 0 && b < naux && !seen[b]++, "perm at %d", e);
        CHECK(pc.iperm[b] == e, "iperm at %d", b);
    }
    std::vector<long long> po(nf), pl(nf);
    for (int k = 0; k < nf; ++k) {
        po[k] = pc.start[k];
        pl[k] = pc.s[k];
        const int cells = pc.cellw[k] >> 16, cw = pc.cellw[k] & 0xffff;
        const int x0 = pc.cell0[k] & 0xffff, y0 = pc.cell0[k] >> 16;
        CHECK(cells * nz == pc.s[k], "front %d: %d cells x %d planes != %d pivots", k, cells, nz, pc.s[k]);
        for (int e = 0; e < pc.s[k]; ++e) {
            const int c = e % cells, q = e / cells;
            const int b = x0 + c % cw + (y0 + c / cw) * Nx + q * Nx * Ny;
            CHECK(pc.perm[pc.start[k] + e] == b, "front %d pivot %d", k, e);
        }
    }
    CHECK(tiles(po, pl, naux), "pivot ranges do not tile the panel");
    // push, pull and right-hand-side maps
    std::vector<int> writers(naux, 0);
    for (int k = 0; k < nf; ++k) {
        const int p = pc.parent[k];
        if (p < 0) {
            CHECK(pc.u[k] == 0, "root %d has %d update entries", k, pc.u[k]);
            continue;
        }
        CHECK(pc.depth[k] == pc.depth[p] + 1, "depth of %d", k);
        const int np = pc.s[p] + pc.u[p];
        const int ci = pc.child0[p] == k ? 0 : pc.child1[p] == k ? 1 : -1;
        CHECK(ci >= 0, "front %d is not a child of its parent %d", k, p);
        std::vector<char> taken(np, 0);
        for (int j = 0; j < pc.u[k]; ++j) {
            const int e = pc.ulist[pc.uoff[k] + j];
            const int local = pc.pmap[pc.pmoff[k] + j];
            CHECK(local >= 0 && local < np && !taken[local]++, "front %d entry %d: parent position %d", k, j,
                  local);
            const int ep = local < pc.s[p] ? pc.start[p] + local : pc.ulist[pc.uoff[p] + local - pc.s[p]];
            CHECK(ep == e, "front %d entry %d: position %d holds %d, not %d", k, j, local, ep, e);
            CHECK(pc.cmap[pc.moff[p] + ci * np + local] == j, "pull map of %d at %d", p, local);
            const int want = (ci == 0 && local < pc.s[p]) ? pc.start[p] + local : -1;
            CHECK(pc.hmap[pc.pmoff[k] + j] == want, "front %d entry %d: h-map %d, expected %d", k, j,
                  pc.hmap[pc.pmoff[k] + j], want);
            if (want >= 0) CHECK(writers[want]++ == 0, "pivot %d has two writers", want);
        }
    }
    // storage: the [x_S; -x_U] regions, the child-contribution slots and the factor blocks
    std::vector<long long> wo(nf), wl(nf), co(nf), cl(nf), lo(nf), ll(nf);
    for (int k = 0; k < nf; ++k) {
        const long long n = pc.s[k] + pc.u[k];
        wo[k] = pc.woff[k] - pc.s[k];
        wl[k] = n;
        co[k] = pc.c2off[k];
        cl[k] = 2 * n;
        lo[k] = pc.loff[k];
        ll[k] = n * pc.s[k];
    }
    CHECK(tiles(wo, wl, pc.wsize), "vector regions do not tile");
    CHECK(tiles(co, cl, pc.c2size), "child slots do not tile");
    CHECK(tiles(lo, ll, pc.lsize), "factor blocks do not tile");
    int listed = 0;
    for (const auto& d : pc.at_depth) listed += (int)d.size();
    CHECK(listed == nf, "depth lists hold %d of %d fronts", listed, nf);
    std::printf("ok %dx%dx%d leaf %d: %d fronts, depth %d\n", Nx, Ny, nz, leaf, nf, pc.maxdepth);
    return 0;
}

int main() {
    const int cases[][4] = {{1, 1, 3, 4}, {3, 2, 2, 1}, {9, 8, 3, 2}, {14, 12, 7, 4},
                            {17, 5, 4, 3}, {30, 30, 14, 4}, {60, 60, 9, 4}};
    for (const auto& c : cases)
        if (check(c[0], c[1], c[2], c[3])) return 1;
    return 0;
}
