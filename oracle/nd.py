"""Nested dissection of a quasi-2D panel and its supernodal structure (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

What the paper fixes
--------------------
* The auxiliary problems are factored by a multifrontal method over a
  supernodal elimination tree defined by nested dissection; the shallow x3
  dimension of the quasi-2D domain is never split, so every separator is a
  full-depth strip, and the tree is numbered in postorder (Sec. 2.1,
  Fig. 2.1, and Sec. 2.3 on extending supernodal subvectors by zero in x3).

Readings
--------
* The lateral box [x0, x1) x [y0, y1) is a leaf once both extents are at
  most `leaf`; otherwise its longer axis (axis 1 on ties) is cut at index
  x0 + floor(w/2), the separator being that one-node-wide strip, and the
  lower-coordinate half is numbered first.  Fig. 2.1 (31 supernodes, 5
  levels, alternating cuts) is reproduced by this rule.
* Inside a supernode the nodes are ordered with i1 fastest, then i2, then
  the depth index.
* The update set of a supernode is obtained here by symbolic elimination of
  the permuted matrix (the structure of the supernode's columns of L below
  the supernode), not by a geometric formula.
"""

import numpy as np


class Supernode:
    __slots__ = ("box", "cells", "children", "parent", "depth", "start", "size")

    def __init__(self, box, cells, children):
        self.box = box
        self.cells = cells
        self.children = children
        self.parent = -1
        self.depth = 0
        self.start = 0
        self.size = 0


def nested_dissection(Nx, Ny, leaf):
    """Supernodes of the lateral Nx x Ny box, in postorder."""
    assert leaf >= 2
    nodes = []

    def rec(x0, x1, y0, y1):
        w, hgt = x1 - x0, y1 - y0
        if w <= leaf and hgt <= leaf:
            cells = [(a1, a2) for a2 in range(y0, y1) for a1 in range(x0, x1)]
            nodes.append(Supernode((x0, x1, y0, y1), cells, []))
            return len(nodes) - 1
        if w >= hgt:
            cut = x0 + w // 2
            left = rec(x0, cut, y0, y1)
            right = rec(cut + 1, x1, y0, y1)
            cells = [(cut, a2) for a2 in range(y0, y1)]
        else:
            cut = y0 + hgt // 2
            left = rec(x0, x1, y0, cut)
            right = rec(x0, x1, cut + 1, y1)
            cells = [(a1, cut) for a1 in range(x0, x1)]
        nodes.append(Supernode((x0, x1, y0, y1), cells, [left, right]))
        return len(nodes) - 1

    root = rec(0, Nx, 0, Ny)
    assert root == len(nodes) - 1
    for k, nd in enumerate(nodes):
        for ch in nd.children:
            nodes[ch].parent = k
    for k in range(len(nodes) - 1, -1, -1):
        p = nodes[k].parent
        nodes[k].depth = 0 if p < 0 else nodes[p].depth + 1
    return nodes


def elimination_order(nodes, Nx, Ny, nz):
    """Permutation perm[e] = box index (a1 + a2 Nx + q Nx Ny) of the e-th eliminated node.

    Also fills node.start / node.size (contiguous elimination ranges).
    """
    perm = []
    for nd in nodes:
        nd.start = len(perm)
        for q in range(nz):
            for (a1, a2) in nd.cells:
                perm.append(a1 + a2 * Nx + q * Nx * Ny)
        nd.size = len(perm) - nd.start
    perm = np.asarray(perm, dtype=np.int64)
    assert len(perm) == Nx * Ny * nz and len(np.unique(perm)) == len(perm)
    return perm


def symbolic_structure(Ap):
    """Row structure below the diagonal of each column of L for pattern Ap.

    Ap: sparse matrix (any format) in elimination order.  Liu's elimination-tree
    recurrence: struct(j) = {i > j : A_ij != 0} U (union of struct(c) over
    children c of j in the elimination tree) minus {j}; parent(j) = min struct(j).
    """
    A = Ap.tocsc()
    n = A.shape[0]
    children = [[] for _ in range(n)]
    struct = [None] * n
    for j in range(n):
        rows = A.indices[A.indptr[j]:A.indptr[j + 1]]
        s = set(int(r) for r in rows if r > j)
        for c in children[j]:
            s |= struct[c]
        s.discard(j)
        struct[j] = s
        if s:
            children[min(s)].append(j)
    return struct


def update_sets(nodes, struct):
    """Sorted update set (elimination positions) of every supernode."""
    out = []
    for nd in nodes:
        S = range(nd.start, nd.start + nd.size)
        u = set()
        for j in S:
            u |= struct[j]
        u -= set(S)
        out.append(np.array(sorted(u), dtype=np.int64))
    return out
