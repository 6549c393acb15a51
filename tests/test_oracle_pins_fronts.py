"""Pins of the oracle's front blocks, selective inverse and moving PML.

Each check ties an oracle function to something other than itself:
- the defining identities and a closed form of a triangular inverse;
- a supernodal substitution built from the blocks, against a sparse LU solve;
- the physical PML, itself pinned by the outgoing Green's function;
- the exact outgoing half-line Schur complement of a quasi-1D problem.

The mutation tests plant plausible mistakes in copies of the oracle's
arithmetic, on the CPU only, and check that the pins reject them.
"""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import helmholtz as hz
from oracle import ldlt as ld
from oracle import nd
from oracle import panels as pn
from paper_1204_0111_amd import workloads as wl
from tests._cases import zero_diagonal_problem


def _unit_lower(s, seed):
    rng = np.random.default_rng(seed)
    L = np.tril(rng.standard_normal((s, s)) + 1j * rng.standard_normal((s, s)), -1) * 0.4
    return L + np.eye(s)


# ------------------------------------------------- selective inverse (Sec. 2.2)
def test_selective_inverse_defining_identities():
    """G_TL L_F = L_F G_TL = I, G_BL L_F = F_BL, G_TL unit lower (Sec. 2.2)."""
    s, u = 9, 6
    L_F = _unit_lower(s, 1)
    rng = np.random.default_rng(2)
    F_BL = rng.standard_normal((u, s)) + 1j * rng.standard_normal((u, s))
    G_TL, G_BL = ld.selective_inverse(L_F, F_BL)
    eye = np.eye(s)
    assert np.abs(G_TL @ L_F - eye).max() < 1e-12
    assert np.abs(L_F @ G_TL - eye).max() < 1e-12
    assert np.abs(G_BL @ L_F - F_BL).max() < 1e-12
    assert np.abs(np.triu(G_TL, 1)).max() == 0.0
    assert np.abs(np.diag(G_TL) - 1.0).max() < 1e-15
    # a transposed inverse or the bottom block on the wrong side fails these
    assert np.abs(G_TL.T @ L_F - eye).max() > 1e-3
    assert np.abs(F_BL @ np.linalg.inv(L_F).T @ L_F - F_BL).max() > 1e-3


def test_selective_inverse_of_bidiagonal_closed_form():
    """L_F = I - a J (J the shift) has inverse entries a^(i-j) below the diagonal."""
    s, a = 8, 0.7 - 0.2j
    L_F = np.eye(s, dtype=np.complex128) - a * np.eye(s, k=-1)
    F_BL = np.zeros((1, s), dtype=np.complex128)
    F_BL[0, 0] = 1.0  # F_BL = e_0^T, so G_BL = e_0^T L_F^{-1} is row 0 of the inverse
    G_TL, G_BL = ld.selective_inverse(L_F, F_BL)
    for i in range(s):
        for j in range(s):
            want = a ** (i - j) if i >= j else 0.0
            assert abs(G_TL[i, j] - want) < 1e-14
    # e_0^T L_F^{-1} = e_0^T (only the diagonal entry of row 0)
    assert np.abs(G_BL - np.eye(1, s)).max() < 1e-14


def _panel_factor_case(n=(6, 5, 6), gamma=2, d=2, i=1, leaf=3):
    n, h = n, wl.grid_h(n)
    c = wl.velocity_grf(n, h, 5)
    om = wl.omega_for_ppw(c, h)
    H, lo, hi, ga = pn.aux_operator(c, h, om, wl.ALPHA_DEFAULT, gamma, 4.0, d, i)
    N = hz.padded_shape(n, gamma)
    nz = ga + hi - lo
    nodes = nd.nested_dissection(N[0], N[1], leaf)
    perm = nd.elimination_order(nodes, N[0], N[1], nz)
    Hp = H[perm][:, perm].tocsc()
    U = nd.update_sets(nodes, nd.symbolic_structure(Hp))
    L, dd = ld.ldlt_unpivoted(Hp.toarray())
    return Hp, nodes, U, ld.front_blocks(L, dd, nodes, U)


def _substitution_error(inverse=ld.selective_inverse):
    """Forward pass y = G v_S per front in postorder, D^{-1}, backward pass
    x_S = G^T [z_S; -x_U] in reverse postorder, with G = [L_F^{-1}; F_BL L_F^{-1}]
    (Sec. 2.2, multifrontal solve with selective inversion); relative error
    against the sparse LU solution of the permuted auxiliary problem."""
    Hp, nodes, U, blocks = _panel_factor_case()
    b = wl.random_complex((Hp.shape[0], 2), 13)
    w = b.copy()
    Gs = []
    for x, u, (dF, LF, FBL) in zip(nodes, U, blocks):
        S = slice(x.start, x.start + x.size)
        G_TL, G_BL = inverse(LF, FBL)
        Gs.append((G_TL, G_BL))
        vS = w[S].copy()
        w[S] = G_TL @ vS
        w[u] -= G_BL @ vS
    d_all = np.concatenate([dF for dF, _, _ in blocks])
    order = np.concatenate([np.arange(x.start, x.start + x.size) for x in nodes])
    dvec = np.empty(Hp.shape[0], dtype=np.complex128)
    dvec[order] = d_all
    z = w / dvec[:, None]
    xsol = z.copy()
    for k in range(len(nodes) - 1, -1, -1):
        x, u = nodes[k], U[k]
        S = slice(x.start, x.start + x.size)
        G_TL, G_BL = Gs[k]
        xsol[S] = G_TL.T @ z[S] - G_BL.T @ xsol[u]
    ref = spla.spsolve(Hp, b)
    return np.linalg.norm(xsol - ref) / np.linalg.norm(ref)


def test_supernodal_substitution_with_selective_inverse_solves_panel():
    assert _substitution_error() <= 1e-10


def _inv(L):
    return np.linalg.inv(L)


@pytest.mark.parametrize("mutant", [
    lambda L, F: (_inv(L).T, F @ _inv(L)),          # transposed inverse
    lambda L, F: (_inv(L), F @ _inv(L).T),          # wrong-side (transposed) bottom block
    lambda L, F: (_inv(L), F),                      # bottom block not multiplied
    lambda L, F: (_inv(L), -F @ _inv(L)),           # sign of the coupling
])
def test_substitution_pin_rejects_planted_inverse_mistakes(mutant):
    assert _substitution_error(mutant) > 1e-3


def test_front_blocks_of_a_hand_built_factorisation():
    """A = L0 D0 L0^T with two leaves {0,1}, {2,3} under the root {4}: the
    unpivoted LDL^T is unique, so the blocks are L0 and D0's sub-blocks."""
    L0 = np.eye(5, dtype=np.complex128)
    L0[1, 0] = 0.5 + 1j
    L0[3, 2] = -0.25
    L0[4, 0], L0[4, 1], L0[4, 2], L0[4, 3] = 2.0, 1j, -1.5, 0.75 - 0.5j
    D0 = np.array([2.0, -1 + 1j, 3j, 0.5, 4.0 - 2j])
    A = L0 @ np.diag(D0) @ L0.T

    class Node:
        def __init__(self, start, size):
            self.start, self.size = start, size

    nodes = [Node(0, 2), Node(2, 2), Node(4, 1)]
    usets = [[4], [4], []]
    L, d = ld.ldlt_unpivoted(A)
    blocks = ld.front_blocks(L, d, nodes, usets)
    assert np.allclose(blocks[0][0], D0[0:2], atol=1e-14)
    assert np.allclose(blocks[0][1], L0[0:2, 0:2], atol=1e-14)
    assert np.allclose(blocks[0][2], L0[[4], 0:2], atol=1e-14)
    assert np.allclose(blocks[1][1], [[1, 0], [-0.25, 1]], atol=1e-14)
    assert np.allclose(blocks[1][2], [[-1.5, 0.75 - 0.5j]], atol=1e-14)
    assert np.allclose(blocks[2][0], [4.0 - 2j], atol=1e-13)
    assert blocks[2][2].shape == (0, 1)


# ----------------------------------------------------- padding of the velocity
def test_pad_velocity_axis_order_with_unequal_widths():
    """Widths (g1, g2, g3) pad axes x1, x2, x3; numpy shape is (n3, n2, n1)."""
    n1, n2, n3 = 4, 3, 2
    c = np.arange(n1 * n2 * n3, dtype=np.float64).reshape(n3, n2, n1) + 1.0
    g = (1, 2, 3)
    cp = hz.pad_velocity(c, g)
    assert cp.shape == (n3 + 6, n2 + 4, n1 + 2)
    # interior copy sits at offsets (g3, g2, g1)
    assert np.array_equal(cp[3:3 + n3, 2:2 + n2, 1:1 + n1], c)
    # clamping: every padded node takes the nearest interior node's value
    for a3 in range(cp.shape[0]):
        for a2 in range(cp.shape[1]):
            for a1 in range(cp.shape[2]):
                i3 = min(max(a3 - 3, 0), n3 - 1)
                i2 = min(max(a2 - 2, 0), n2 - 1)
                i1 = min(max(a1 - 1, 0), n1 - 1)
                assert cp[a3, a2, a1] == c[i3, i2, i1]


# -------------------------------------------------- the moving PML (Sec. 1.1)
def _translation_gap(tables=None, gamma=3, d=2, i=2, C=25.0):
    """max |H_i - J[first planes]| for constant velocity.

    Fig. 1.2: the auxiliary problem of panel i puts the PML right below the
    panel and ignores the planes after it.  With a constant velocity that is
    exactly the physical problem's first ga + (hi - lo) planes (the bottom
    PML followed by interior planes), with Dirichlet on the cut above.
    `tables` replaces the oracle's aux_x3_tables (mutation tests).
    """
    n = (4, 3, 12)
    h = 1.0 / 13
    c = np.full((n[2], n[1], n[0]), 1.7)
    om = 2 * math.pi * 1.7 / (10 * h)
    saved = pn.aux_x3_tables
    if tables is not None:
        pn.aux_x3_tables = tables
    try:
        H, lo, hi, ga = pn.aux_operator(c, h, om, wl.ALPHA_DEFAULT, gamma, C, d, i)
    finally:
        pn.aux_x3_tables = saved
    g3 = hz.gamma3(gamma)[2]
    N3 = n[2] + 2 * g3
    assert ga == g3 and lo >= g3 + d and hi <= N3 - g3  # a middle panel
    J = hz.helmholtz_operator(c, h, om, gamma, C, wl.ALPHA_DEFAULT)
    N = hz.padded_shape(n, gamma)
    nb = (ga + hi - lo) * N[0] * N[1]
    return abs(H - J[:nb, :nb]).max() / abs(J[:nb, :nb]).max()


@pytest.mark.parametrize("gamma", [3, (2, 1, 4)])
def test_artificial_pml_is_the_physical_pml_moved_to_the_panel(gamma):
    # equal up to the rounding of the depth, (a - g + 1) h against (ga - q) h
    assert _translation_gap(gamma=gamma) < 1e-14


def _quasi_1d_T(g, C, n3=40, tables=None):
    """T_i of a middle panel of a 1 x 1 x n3 grid (PML only along x3, d = 1),
    and the exact outgoing half-line value.

    Eliminating the half-line below a node with the outgoing solution
    u_q = z^(p0 - q) u_p0, z = e^{i theta}, cos theta = 1 - keff^2 h^2 / 2,
    leaves the Schur complement (2 - z)/h^2 - keff^2 = 1/(z h^2), so the exact
    T is z h^2.  The artificial PML of H_i must approach it as gamma grows.
    """
    h = 1.0 / (n3 + 1)
    keff = 2 * math.pi / (10 * h)
    om = math.sqrt(4.0 / h ** 2 + keff ** 2)  # lateral Dirichlet adds 4/h^2
    c = np.ones((n3, 1, 1))
    gam = (0, 0, g)
    i = len(pn.panel_bounds(n3, gam, 1)) // 2
    saved = pn.aux_x3_tables
    if tables is not None:
        pn.aux_x3_tables = tables
    try:
        H = pn.aux_operator(c, h, om, 0.0, gam, C, 1, i)[0]
    finally:
        pn.aux_x3_tables = saved
    e = np.zeros(H.shape[0], dtype=np.complex128)
    e[-1] = 1.0
    T = spla.spsolve(H.tocsc(), e)[-1]
    z = np.exp(1j * math.acos(1 - keff ** 2 * h ** 2 / 2))
    return abs(T - z * h * h) / abs(z * h * h)


def test_artificial_pml_approaches_outgoing_half_line():
    errs = [_quasi_1d_T(g, 80.0) for g in (4, 8, 16, 32)]
    assert errs[-1] < 2e-5, errs
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    # the layer reversed (an amplifier) is far off at every width
    assert min(_quasi_1d_T(g, -80.0) for g in (4, 8, 16)) > 0.5


def _mutated_tables(node_shift=0.0, half_shift=0.0, sign=1.0):
    """A copy of the artificial-layer tables with a planted mistake."""
    def tables(n3, gamma, h, C, omega, lo, hi, ga):
        e_node, e_half = pn.__dict__["_orig_tables"](n3, gamma, h, C, omega, lo, hi, ga)
        g = hz.gamma3(gamma)[2]
        eta = (g + 1) * h
        e_node, e_half = e_node.copy(), e_half.copy()
        for q in range(ga):
            e_node[q] = hz.stretch((ga - q + node_shift) * h, sign * C, eta, omega)
        for a in range(ga + 1):
            e_half[a] = hz.stretch((ga - a + 0.5 + half_shift) * h, sign * C, eta, omega)
        return e_node, e_half
    return tables


@pytest.mark.parametrize("mut", [dict(node_shift=1.0), dict(node_shift=-1.0),
                                 dict(half_shift=1.0), dict(half_shift=-1.0), dict(sign=-1.0)])
def test_pins_reject_planted_artificial_pml_mistakes(mut):
    """Off-by-one depths (nodes or half-nodes) and a reversed stretch break the
    translation pin; the reversed stretch also fails the half-line pin."""
    pn._orig_tables = pn.aux_x3_tables
    try:
        # the unmutated copy reproduces the oracle exactly
        assert _translation_gap(tables=_mutated_tables()) < 1e-14
        assert _translation_gap(tables=_mutated_tables(**mut)) > 1e-3
        if mut.get("sign", 1.0) < 0:
            assert _quasi_1d_T(16, 80.0, tables=_mutated_tables(**mut)) > 0.5
    finally:
        del pn._orig_tables


# ------------------------------------------- breakdown without pivoting (Sec. 2.5)
def test_zero_diagonal_case_breaks_the_unpivoted_factorisation():
    """At omega^2 = 6 c^2 / h^2 without PML the operator's diagonal is zero;
    the unpivoted LDL^T of panel 0 breaks down at its first pivot.  The
    parameters make the entries exact zeros in floating point."""
    P = zero_diagonal_problem()
    assert 1.0 / (P["h"] * P["h"]) == 24.0
    H, lo, hi, ga = pn.aux_operator(P["c"], P["h"], P["omega"], P["alpha"], P["gamma"], P["C"],
                                    P["d"], 0)
    assert np.abs(H.diagonal()).max() == 0.0
    N = hz.padded_shape(P["n"], P["gamma"])
    nodes = nd.nested_dissection(N[0], N[1], P["leaf"])
    perm = nd.elimination_order(nodes, N[0], N[1], ga + hi - lo)
    with pytest.raises(ld.BreakdownError, match="pivot at 0"):
        ld.ldlt_unpivoted(H[perm][:, perm].toarray())
