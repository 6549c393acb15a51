// Symbolic plan: nested dissection of the quasi-2D panels, front structure,
// extend-add maps and the level schedules of the factorisation and solves.
//
// A panel's auxiliary box is Nx x Ny laterally and nz planes deep.  The
// lateral box is dissected recursively (Sec. 2.1, Fig. 2.1): a box whose two
// extents are both <= leaf is a leaf; otherwise the longer axis (the first
// one on ties) is cut at x0 + floor(w/2) by a one-node-wide strip.  Because
// the shallow x3 dimension is never split, every supernode is a lateral cell
// set times all nz planes.  Supernodes are numbered in postorder, lower
// coordinates first; inside a supernode the nodes are ordered with i1
// fastest, then i2, then the plane index.  The update set of a supernode is
// the set of nodes laterally adjacent to its subtree's box, over all planes,
// in elimination order.
#pragma once

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

namespace hsw {

constexpr int TILE = 64;        // square tile of the front kernels
// Nested-dissection leaf extent given to a problem that asks for 0: the
// fastest of the leaves 2..8 timed on the 50^3 and 100^3 workloads.
constexpr int DEFAULT_LEAF = 4;
constexpr int NB = 64;          // pivot block of the blocked partial LDL^T
// Block shapes of the solve passes: rows (forward) or columns (backward) per
// workgroup and threads per workgroup.  Each tree depth of each panel class
// uses one shape per pass, picked by timing (autotuning) or by the default
// rule: the first shape for depths whose largest front has fewer than
// SOLVE_SMALL_BLOCK_N rows, the second otherwise.
struct PassShape {
    int block, threads;
};
constexpr int N_FWD_SHAPES = 8, N_BWD_SHAPES = 9;
constexpr PassShape FWD_SHAPES[N_FWD_SHAPES] = {{64, 256}, {16, 256}, {64, 512}, {16, 512}, {32, 256},
                                                {8, 256},  {8, 512},  {32, 512}};
constexpr PassShape BWD_SHAPES[N_BWD_SHAPES] = {{32, 256}, {8, 256}, {32, 512}, {8, 512}, {16, 256}, {4, 256},
                                                {64, 256}, {2, 128}, {4, 128}};
// The matrix-core passes take the right-hand sides in groups of MM_MIN_RHS
// = 16 (the last group padded with zeros); a solve takes them from
// MM_DEFAULT_FROM right-hand sides on (option mm_min_rhs), below that the
// single-vector passes.  Without tuning, the forward pass takes
// items of 64 rows (shape 0) in complex64, or of 16 rows (shape 1) in
// complex128 and in complex64 launches that would have fewer than
// MM_NARROW_BELOW workgroups of 64 rows; the backward pass takes 64 columns
// (shape 6) in launches of at least MM_TILES4_FROM workgroups of 64 columns,
// else 16 columns (shape 4).  Launches of fewer than MM_WIDE_BELOW
// workgroups take more waves per workgroup.
constexpr int MM_MIN_RHS = 16, MM_DEFAULT_FROM = 4;
constexpr int MM_BWD_SHAPE = 4, MM_BWD_SHAPE64 = 6;
constexpr int MM_NARROW_BELOW = 256, MM_TILES4_FROM = 512, MM_WIDE_BELOW = 512;
// The split-contraction forms divide each item's contraction over
// mm_split(items, groups) workgroups: about MM_SPLIT_TARGET workgroups per
// launch, at most MM_SPLIT_MAX shares per item.
constexpr int MM_SPLIT_TARGET = 512, MM_SPLIT_MAX = 8;
inline int mm_split(int items, int groups) {
    const int64_t w = std::max<int64_t>(1, (int64_t)items * groups);
    return (int)std::min<int64_t>(MM_SPLIT_MAX, std::max<int64_t>(1, (MM_SPLIT_TARGET + w - 1) / w));
}
static_assert(FWD_SHAPES[0].block == 64 && FWD_SHAPES[1].block == 16 && BWD_SHAPES[MM_BWD_SHAPE].block == 16 &&
                  BWD_SHAPES[MM_BWD_SHAPE64].block == 64,
              "the matrix-core passes take items of 64 or 16 rows (forward) and 16 or 64 columns (backward)");
constexpr int SOLVE_SMALL_BLOCK_N = 512;
// Depths with at least this many fronts (over all panels and problems) apply
// the Schur updates left-looking: each block column once, before its pivots
// are factored, and F_BR once at the end -- every entry is read and written
// once instead of once per earlier pivot block.  Shallower depths, with few
// large fronts, keep the right-looking order, which has more tiles per launch.
constexpr int LEFT_LOOKING_MIN_FRONTS = 64;

struct LatNode {
    int x0 = 0, x1 = 0, y0 = 0, y1 = 0;
    std::vector<int> cells;  // lateral index a1 + a2 * Nx, a1 fastest
    // the cells form a rectangle: first cell (cx0, cy0), cw cells per row
    int cx0 = 0, cy0 = 0, cw = 0;
    int child[2] = {-1, -1};
    int parent = -1;
    int depth = 0;
};

struct LatTree {
    int Nx = 0, Ny = 0, leaf = 0;
    std::vector<LatNode> nodes;  // postorder
    std::vector<int> owner;      // lateral cell -> supernode
    std::vector<int> cellidx;    // lateral cell -> position in its supernode's cell list
    int maxdepth = 0;
};

LatTree build_lateral_tree(int Nx, int Ny, int leaf);

// Fronts of one panel class: a lateral tree extended over nz planes.
struct PanelClass {
    int Nx = 0, Ny = 0, nz = 0, leaf = 0;
    int naux = 0, nfront = 0, maxdepth = 0;
    std::vector<int> perm, iperm;  // elimination position <-> box index a1 + a2 Nx + q Nx Ny
    // per front, its cell rectangle packed in 16-bit halves: (x0 | y0 << 16)
    // and (cells per row | cells << 16); pivot e of the front is cell e mod
    // cells of that rectangle (row-major) on plane e / cells
    std::vector<int> cell0, cellw;
    std::vector<int> start, s, u, parent, child0, child1, depth;
    std::vector<int> uoff, ulist;  // update sets, concatenated (elimination positions)
    std::vector<int> moff, cmap;   // per front 2 (s+u) entries: position in child 0 / 1 update set or -1
    std::vector<int> pmoff, pmap;  // per front u entries: position of each update entry in the parent front
    // per front u entries, parallel to pmap: for the parent's first child, the
    // elimination position of the parent pivot an update entry adds into
    // (its contribution joins the parent's right-hand side there), else -1
    std::vector<int> hmap;
    std::vector<int> c2off;        // per front: offset of its 2 (s+u) child-contribution slots
    int64_t c2size = 0;            // sum 2 (s+u)
    std::vector<int64_t> loff;     // per front: offset of its (s+u) x s block, relative to the panel
    std::vector<int> woff;         // per front: offset of its update vector (u entries per rhs),
                                   // which follows s entries of the front's own
    int64_t lsize = 0;             // sum (s+u) s
    int64_t wsize = 0;             // sum of s + u
    std::vector<std::vector<int>> at_depth;
    double factor_cmac = 0;  // complex multiply-adds of the panel's partial factorisations
};

// Returns an empty string on success, else an error message.
std::string build_class(const LatTree& lt, int nz, PanelClass& pc);

// Decomposition of a lower-triangular tile index t into (ti, tj), ti >= tj.
inline void tri_decode(int t, int& ti, int& tj) {
    int i = 0;
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    ti = i;
    tj = t - i * (i + 1) / 2;
}

}  // namespace hsw
