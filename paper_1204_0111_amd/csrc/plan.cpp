// Symbolic plan: see plan.hpp.
#include "plan.hpp"

#include <algorithm>
#include <cstdio>
#include <functional>

namespace hsw {

LatTree build_lateral_tree(int Nx, int Ny, int leaf) {
    LatTree t;
    t.Nx = Nx;
    t.Ny = Ny;
    t.leaf = leaf;
    std::function<int(int, int, int, int)> rec = [&](int x0, int x1, int y0, int y1) -> int {
        int w = x1 - x0, h = y1 - y0;
        LatNode nd;
        nd.x0 = x0; nd.x1 = x1; nd.y0 = y0; nd.y1 = y1;
        if (w <= leaf && h <= leaf) {
            for (int a2 = y0; a2 < y1; ++a2)
                for (int a1 = x0; a1 < x1; ++a1) nd.cells.push_back(a1 + a2 * Nx);
            nd.cx0 = x0;
            nd.cy0 = y0;
            nd.cw = w;
            t.nodes.push_back(nd);
            return (int)t.nodes.size() - 1;
        }
        int l, r;
        if (w >= h) {
            int cut = x0 + w / 2;
            l = rec(x0, cut, y0, y1);
            r = rec(cut + 1, x1, y0, y1);
            for (int a2 = y0; a2 < y1; ++a2) nd.cells.push_back(cut + a2 * Nx);
            nd.cx0 = cut;
            nd.cy0 = y0;
            nd.cw = 1;
        } else {
            int cut = y0 + h / 2;
            l = rec(x0, x1, y0, cut);
            r = rec(x0, x1, cut + 1, y1);
            for (int a1 = x0; a1 < x1; ++a1) nd.cells.push_back(a1 + cut * Nx);
            nd.cx0 = x0;
            nd.cy0 = cut;
            nd.cw = w;
        }
        nd.child[0] = l;
        nd.child[1] = r;
        t.nodes.push_back(nd);
        return (int)t.nodes.size() - 1;
    };
    rec(0, Nx, 0, Ny);
    int nn = (int)t.nodes.size();
    for (int k = 0; k < nn; ++k)
        for (int c : t.nodes[k].child)
            if (c >= 0) t.nodes[c].parent = k;
    for (int k = nn - 1; k >= 0; --k) {
        int p = t.nodes[k].parent;
        t.nodes[k].depth = p < 0 ? 0 : t.nodes[p].depth + 1;
        t.maxdepth = std::max(t.maxdepth, t.nodes[k].depth);
    }
    t.owner.assign((size_t)Nx * Ny, -1);
    t.cellidx.assign((size_t)Nx * Ny, -1);
    for (int k = 0; k < nn; ++k)
        for (size_t i = 0; i < t.nodes[k].cells.size(); ++i) {
            t.owner[t.nodes[k].cells[i]] = k;
            t.cellidx[t.nodes[k].cells[i]] = (int)i;
        }
    return t;
}

std::string build_class(const LatTree& lt, int nz, PanelClass& pc) {
    const int Nx = lt.Nx, Ny = lt.Ny;
    const int nf = (int)lt.nodes.size();
    pc.Nx = Nx; pc.Ny = Ny; pc.nz = nz; pc.leaf = lt.leaf;
    pc.nfront = nf;
    pc.maxdepth = lt.maxdepth;
    pc.naux = Nx * Ny * nz;
    pc.start.resize(nf); pc.s.resize(nf); pc.u.resize(nf);
    pc.parent.resize(nf); pc.child0.resize(nf); pc.child1.resize(nf); pc.depth.resize(nf);
    pc.perm.resize(pc.naux);
    pc.iperm.resize(pc.naux);
    int pos = 0;
    for (int k = 0; k < nf; ++k) {
        const LatNode& nd = lt.nodes[k];
        pc.start[k] = pos;
        pc.s[k] = (int)nd.cells.size() * nz;
        pc.parent[k] = nd.parent;
        pc.child0[k] = nd.child[0];
        pc.child1[k] = nd.child[1];
        pc.depth[k] = nd.depth;
        for (int q = 0; q < nz; ++q)
            for (int cell : nd.cells) {
                int b = cell + q * Nx * Ny;
                pc.perm[pos] = b;
                pc.iperm[b] = pos;
                ++pos;
            }
    }
    if (pos != pc.naux) return "elimination order does not cover the panel";
    // the solves compute box indices from the cell rectangle: check that
    // closed form against the elimination order
    pc.cell0.resize(nf);
    pc.cellw.resize(nf);
    for (int k = 0; k < nf; ++k) {
        const LatNode& nd = lt.nodes[k];
        const int nc = (int)nd.cells.size();
        if (nd.cw < 1 || nc % nd.cw != 0 || nd.cx0 >= (1 << 16) || nd.cy0 >= (1 << 16) ||
            nd.cw >= (1 << 16) || nc >= (1 << 16))
            return "supernode cells do not form a rectangle";
        for (int e = 0; e < pc.s[k]; ++e) {
            const int cell = e % nc, q = e / nc;
            const int b = nd.cx0 + cell % nd.cw + (nd.cy0 + cell / nd.cw) * Nx + q * Nx * Ny;
            if (pc.perm[pc.start[k] + e] != b) return "supernode order is not the cell rectangle";
        }
        pc.cell0[k] = nd.cx0 | (nd.cy0 << 16);
        pc.cellw[k] = nd.cw | (nc << 16);
    }
    // update sets: lateral neighbours of the subtree box, every plane
    auto elim = [&](int cell, int q) {
        int k = lt.owner[cell];
        return pc.start[k] + q * (int)lt.nodes[k].cells.size() + lt.cellidx[cell];
    };
    pc.uoff.resize(nf);
    for (int k = 0; k < nf; ++k) {
        const LatNode& nd = lt.nodes[k];
        std::vector<int> cells;
        for (int a2 = nd.y0; a2 < nd.y1; ++a2) {
            if (nd.x0 - 1 >= 0) cells.push_back(nd.x0 - 1 + a2 * Nx);
            if (nd.x1 < Nx) cells.push_back(nd.x1 + a2 * Nx);
        }
        for (int a1 = nd.x0; a1 < nd.x1; ++a1) {
            if (nd.y0 - 1 >= 0) cells.push_back(a1 + (nd.y0 - 1) * Nx);
            if (nd.y1 < Ny) cells.push_back(a1 + nd.y1 * Nx);
        }
        std::vector<int> U;
        for (int cell : cells)
            for (int q = 0; q < nz; ++q) U.push_back(elim(cell, q));
        std::sort(U.begin(), U.end());
        for (int e : U)
            if (e < pc.start[k] + pc.s[k]) return "update set entry not in an ancestor";
        pc.uoff[k] = (int)pc.ulist.size();
        pc.u[k] = (int)U.size();
        pc.ulist.insert(pc.ulist.end(), U.begin(), U.end());
    }
    // extend-add maps (pull form): for each parent local index, the position
    // in each child's update set
    pc.moff.resize(nf);
    for (int k = 0; k < nf; ++k) {
        int n = pc.s[k] + pc.u[k];
        pc.moff[k] = (int)pc.cmap.size();
        pc.cmap.resize(pc.cmap.size() + 2 * (size_t)n, -1);
        int cs[2] = {pc.child0[k], pc.child1[k]};
        for (int ci = 0; ci < 2; ++ci) {
            int c = cs[ci];
            if (c < 0) continue;
            const int* Uc = pc.ulist.data() + pc.uoff[c];
            int uc = pc.u[c];
            int found = 0;
            for (int r = 0; r < n; ++r) {
                int e = r < pc.s[k] ? pc.start[k] + r : pc.ulist[pc.uoff[k] + r - pc.s[k]];
                const int* it = std::lower_bound(Uc, Uc + uc, e);
                if (it != Uc + uc && *it == e) {
                    pc.cmap[pc.moff[k] + ci * n + r] = (int)(it - Uc);
                    ++found;
                }
            }
            if (found != uc) return "child update set not contained in parent front";
        }
    }
    // push form of the maps: each update entry's position in the parent front,
    // and the slots a parent keeps for its two children's contributions
    pc.pmoff.resize(nf);
    pc.c2off.resize(nf);
    pc.c2size = 0;
    for (int k = 0; k < nf; ++k) {
        pc.c2off[k] = (int)pc.c2size;
        pc.c2size += 2 * (int64_t)(pc.s[k] + pc.u[k]);
        pc.pmoff[k] = (int)pc.pmap.size();
        const int p = pc.parent[k];
        if (p < 0) {
            if (pc.u[k] != 0) return "root front with a nonempty update set";
            continue;
        }
        const int* Up = pc.ulist.data() + pc.uoff[p];
        for (int j = 0; j < pc.u[k]; ++j) {
            const int e = pc.ulist[pc.uoff[k] + j];
            int local;
            if (e >= pc.start[p] && e < pc.start[p] + pc.s[p]) {
                local = e - pc.start[p];
            } else {
                const int* it = std::lower_bound(Up, Up + pc.u[p], e);
                if (it == Up + pc.u[p] || *it != e) return "update entry missing from the parent front";
                local = pc.s[p] + (int)(it - Up);
            }
            pc.pmap.push_back(local);
            pc.hmap.push_back(pc.child0[p] == k && local < pc.s[p] ? pc.start[p] + local : -1);
        }
    }
    // storage offsets and work counts
    pc.loff.resize(nf);
    pc.woff.resize(nf);
    pc.lsize = 0;
    pc.wsize = 0;
    pc.at_depth.assign(pc.maxdepth + 1, {});
    for (int k = 0; k < nf; ++k) {
        double s = pc.s[k], u = pc.u[k];
        pc.loff[k] = pc.lsize;
        pc.lsize += (int64_t)(pc.s[k] + pc.u[k]) * pc.s[k];
        // each front's vector region holds its s pivot entries, then its u
        // update-set entries (woff points at the latter)
        pc.woff[k] = (int)(pc.wsize + pc.s[k]);
        pc.wsize += pc.s[k] + pc.u[k];
        pc.at_depth[pc.depth[k]].push_back(k);
        pc.factor_cmac += s * s * s / 6 + s * s * u / 2 + s * u * u / 2;
    }
    return "";
}

}  // namespace hsw
