"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (Fig. 2.1), closed forms (the sine-transform spectrum of the
stencil, the discrete outgoing Green's function), exact identities (block
LDL^T = exact solve, the Schur complement identity of Eqs. 1.3-1.4, the
uniqueness of the unpivoted LDL^T), library routines on special cases
(Cholesky, dense solves) and brute force on tiny inputs (the GMRES
minimal-residual property).
"""

import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import gmres as gm
from oracle import helmholtz as hz
from oracle import ldlt as ld
from oracle import nd
from oracle import panels as pn
from oracle import sweep as sw
from paper_1204_0111_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _small(n=(7, 6, 8), model="grf", seed=3):
    h = wl.grid_h(n)
    c = wl.velocity_grf(n, h, seed) if model == "grf" else wl.velocity_constant(n)
    return n, h, c, wl.omega_for_ppw(c, h)


# ---------------------------------------------------------------- P1 symmetry
@pytest.mark.parametrize("alpha", [0.0, wl.ALPHA_DEFAULT])
def test_operator_complex_symmetric_bitwise(alpha):
    """The system is complex symmetric, not Hermitian (Sec. 1.1)."""
    n, h, c, om = _small()
    A = hz.helmholtz_operator(c, h, om, 3, 4.0, alpha)
    D = (A - A.T).tocoo()
    assert D.nnz == 0 or np.max(np.abs(D.data)) == 0.0
    assert abs(A - A.conj().T).max() > 0  # not Hermitian: the PML is complex
    for i in range(len(pn.panel_bounds(n[2], 3, 2))):
        H = pn.aux_operator(c, h, om, alpha, 3, 4.0, 2, i)[0]
        Dh = (H - H.T).tocoo()
        assert Dh.nnz == 0 or np.max(np.abs(Dh.data)) == 0.0


def test_operator_has_seven_point_pattern():
    n, h, c, om = _small()
    A = hz.helmholtz_operator(c, h, om, 2, 4.0)
    N = hz.padded_shape(n, 2)
    counts = np.diff(A.indptr)
    assert counts.max() == 7 and counts.min() == 4  # corners of the padded box
    assert A.nnz == N[0] * N[1] * N[2] + 2 * sum(
        (N[j] - 1) * N[(j + 1) % 3] * N[(j + 2) % 3] for j in range(3))


# ------------------------------------------------------- P2 DST-I closed forms
def _dst_mode(N, k):
    a = np.arange(N)
    return np.sin(k * math.pi * (a + 1) / (N + 1))


def test_stencil_sine_spectrum_without_pml():
    """C = 0, constant c: A is diagonalised by the 3D sine transform."""
    n, h, c, om = _small(n=(5, 6, 4), model="const")
    g = 2
    A = hz.helmholtz_operator(c, h, om, g, 0.0)
    N = hz.padded_shape(n, g)
    for k in [(1, 1, 1), (2, 3, 1), (N[0], 1, N[2]), (4, 2, 3)]:
        m = np.einsum("k,j,i->kji", _dst_mode(N[2], k[2]), _dst_mode(N[1], k[1]),
                      _dst_mode(N[0], k[0])).ravel()
        lam = sum(4.0 / h ** 2 * math.sin(k[j] * math.pi / (2 * (N[j] + 1))) ** 2
                  for j in range(3)) - om ** 2
        r = A @ m - lam * m
        assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(lam * m) + 1e-9


def test_sine_transform_solver_matches_lu():
    """A fast DST-I solver (library FFT) agrees with the sparse LU solve."""
    from scipy.fft import dstn, idstn
    n, h, c, om = _small(n=(6, 5, 7), model="const")
    g = 1
    A = hz.helmholtz_operator(c, h, om * 0.9, g, 0.0)
    N = hz.padded_shape(n, g)
    b = wl.random_complex(A.shape[0], 5)
    lam = np.zeros((N[2], N[1], N[0]))
    for ax, Nj in ((2, N[0]), (1, N[1]), (0, N[2])):
        k = np.arange(1, Nj + 1)
        shp = [1, 1, 1]
        shp[ax] = Nj
        lam = lam + (4.0 / h ** 2 * np.sin(k * math.pi / (2 * (Nj + 1))) ** 2).reshape(shp)
    lam = lam - (om * 0.9) ** 2
    B = b.reshape(N[2], N[1], N[0])
    u_fft = idstn(dstn(B, type=1) / lam, type=1).ravel()
    u_lu = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(u_fft - u_lu) <= 1e-12 * np.linalg.norm(u_lu)


def test_constant_stretch_spectrum_places_factors_per_axis():
    """Constant complex stretches e_j: eigenvalue sum_j (e_k e_l / e_j) mu_j - kappa^2 E / c^2.

    A transposed axis, a missing factor or a stretch on the wrong side of the
    difference changes the eigenvalue.
    """
    N = (5, 4, 6)
    h = 0.1
    e = [1.0 + 0.3j, 0.8 - 0.5j, 1.2 + 0.1j]
    e_node = [np.full(N[j], e[j]) for j in range(3)]
    e_half = [np.full(N[j] + 1, e[j]) for j in range(3)]
    kappa2 = (3.0 + 0.7j) ** 2
    cbox = np.full((N[2], N[1], N[0]), 1.3)
    M = hz.stencil_operator(h, e_node, e_half, kappa2, cbox)
    E = e[0] * e[1] * e[2]
    for k in [(1, 1, 1), (2, 3, 4), (5, 1, 2)]:
        m = np.einsum("k,j,i->kji", _dst_mode(N[2], k[2]), _dst_mode(N[1], k[1]),
                      _dst_mode(N[0], k[0])).ravel()
        mu = [4.0 / h ** 2 * math.sin(k[j] * math.pi / (2 * (N[j] + 1))) ** 2 for j in range(3)]
        lam = sum(E / e[j] ** 2 * mu[j] for j in range(3)) - kappa2 * E / 1.3 ** 2
        assert np.linalg.norm(M @ m - lam * m) <= 1e-12 * abs(lam) * np.linalg.norm(m)


def _quasi_1d_greens(C, sign=1.0, gam=24, n3=61):
    """Centre-source response of a 1 x 1 x n3 grid with PML only in x3."""
    h = 1.0 / (n3 + 1)
    keff = 2 * math.pi / (10 * h)
    om = math.sqrt(4.0 / h ** 2 + keff ** 2)       # lateral Dirichlet adds 4/h^2
    c = np.ones((n3, 1, 1))
    A = hz.helmholtz_operator(c, h, om, (0, 0, gam), sign * C)
    N3 = n3 + 2 * gam
    src = gam + n3 // 2
    b = np.zeros(N3, dtype=np.complex128)
    b[src] = 1.0 / h
    u = spla.spsolve(A.tocsc(), b)
    # exact discrete outgoing Green's function of -(D+ D-) - keff^2 on Z:
    # u_p = h z^|p| / (1/z - z), z = e^{i theta}, cos theta = 1 - keff^2 h^2 / 2
    theta = math.acos(1 - keff ** 2 * h ** 2 / 2)
    z = np.exp(1j * theta)
    p = np.arange(N3) - src
    g = h * z ** np.abs(p) / (1 / z - z)
    inner = slice(gam, gam + n3)
    return np.linalg.norm(u[inner] - g[inner]) / np.linalg.norm(g[inner])


def test_pml_absorbs_outgoing_waves():
    """The PML lets the discrete outgoing wave leave with little reflection.

    With e^{-i omega t} the outgoing wave is e^{+ik|x|}; the stretch
    1 + i sigma/omega makes it decay in the layer.  The reversed sign turns
    the layer into an amplifier and the interior response is far off.
    """
    err = _quasi_1d_greens(40.0)
    assert err < 1e-3, err
    bad = _quasi_1d_greens(40.0, sign=-1.0)
    assert bad > 10 * err
    # no layer at all (Dirichlet walls only): standing waves, large error
    assert _quasi_1d_greens(0.0) > 0.2


# ------------------------------------------------------------- P3 exact solve
def test_manufactured_solution_recovered_by_lu():
    n, h, c, om = _small(n=(8, 8, 8))
    A = hz.helmholtz_operator(c, h, om, 3, 4.0)
    u = wl.random_complex(A.shape[0], 11)
    b = A @ u
    x = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x - u) <= 1e-10 * np.linalg.norm(u)


# -------------------------------------------------------------- P4 PML tables
def test_pml_table_matches_hand_values():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "pml_profile_values.txt"))
            if l.strip() and not l.startswith("#")]
    e_node, e_half = hz.axis_stretch(4, 3, 0.1, 4.0, 5.0)
    for where, a, t, re, im in rows:
        val = (e_node if where == "node" else e_half)[int(a)]
        assert abs(val - complex(float(re), float(im))) < 1e-13, (where, a)


# --------------------------------------------------------- P5 one-panel sweep
def test_single_panel_sweep_is_exact_inverse():
    n, h, c, om = _small(n=(6, 5, 6))
    S = sw.Sweep(c, h, om, wl.ALPHA_DEFAULT, 2, 4.0, d=n[2])
    assert S.m == 1
    v = wl.random_complex(S.N_pad, 2)
    ref = spla.spsolve(S.J.tocsc(), v)
    assert np.linalg.norm(S.apply(v) - ref) <= 1e-10 * np.linalg.norm(ref)


def test_single_panel_undamped_gmres_one_iteration():
    n, h, c, om = _small(n=(6, 5, 6))
    S = sw.Sweep(c, h, om, 0.0, 2, 4.0, d=n[2])
    A = hz.helmholtz_operator(c, h, om, 2, 4.0)
    b = wl.random_complex(S.N_pad, 4)
    x, it, rr, _ = gm.gmres(lambda v: A @ v, S.apply, b, k=20, tol=1e-5)
    assert it == 1 and rr < 1e-10


# ------------------------------------------------- P6 exact-auxiliary sweep
@pytest.mark.parametrize("d", [1, 2, 3])
def test_exact_auxiliary_sweep_equals_lu(d):
    """With exact auxiliary problems Alg. 1.5 is the block LDL^T solve (Algs. 1.1-1.2)."""
    n, h, c, om = _small(n=(5, 6, 7))
    S = sw.Sweep(c, h, om, wl.ALPHA_DEFAULT, 2, 4.0, d=d, exact=True)
    v = wl.random_complex((S.N_pad, 2), 8)
    ref = spla.spsolve(S.J.tocsc(), v)
    assert np.linalg.norm(S.apply(v) - ref) <= 1e-10 * np.linalg.norm(ref)


def test_block_ldlt_of_algorithms_1_1_and_1_2():
    """Algs. 1.1-1.2 on a plane-blocked J reproduce J^{-1} (dense, tiny grid)."""
    n, h, c, om = _small(n=(3, 3, 4))
    J = hz.helmholtz_operator(c, h, om, 1, 4.0, wl.ALPHA_DEFAULT).toarray()
    N = hz.padded_shape(n, 1)
    pl = N[0] * N[1]
    nb = N[2]
    blk = lambda i, j: J[i * pl:(i + 1) * pl, j * pl:(j + 1) * pl]
    S = [blk(0, 0)]
    for i in range(nb - 1):
        S.append(blk(i + 1, i + 1) - blk(i + 1, i) @ np.linalg.solve(S[i], blk(i + 1, i).T))
    f = wl.random_complex(J.shape[0], 9)
    u = [f[i * pl:(i + 1) * pl].copy() for i in range(nb)]
    for i in range(nb - 1):
        u[i + 1] = u[i + 1] - blk(i + 1, i) @ np.linalg.solve(S[i], u[i])
    for i in range(nb):
        u[i] = np.linalg.solve(S[i], u[i])
    for i in range(nb - 2, -1, -1):
        u[i] = u[i] - np.linalg.solve(S[i], blk(i + 1, i).T @ u[i + 1])
    ref = np.linalg.solve(J, f)
    assert np.linalg.norm(np.concatenate(u) - ref) <= 1e-10 * np.linalg.norm(ref)
    # and the exact-auxiliary oracle sweep with one plane per panel is the same solve
    Sx = sw.Sweep(c, h, om, wl.ALPHA_DEFAULT, 1, 4.0, d=1, exact=True)
    assert np.linalg.norm(Sx.apply(f) - ref) <= 1e-10 * np.linalg.norm(ref)


# ------------------------------------------------------ P7 Schur identity T_i
@pytest.mark.parametrize("i", [0, 1, 2])
def test_T_equals_inverse_schur_complement(i):
    """H_i^{-1} = [* *; * S~_i^{-1}] with the panel unknowns last (Eqs. 1.3-1.4)."""
    n, h, c, om = _small(n=(4, 5, 6))
    g, d = 2, 2
    S = sw.Sweep(c, h, om, wl.ALPHA_DEFAULT, g, 4.0, d=d)
    H, lo, hi, ga = pn.aux_operator(c, h, om, wl.ALPHA_DEFAULT, g, 4.0, d, i)
    H = H.toarray()
    na = ga * S.plane
    Hpp, Hpa, Haa, Hap = H[na:, na:], H[na:, :na], H[:na, :na], H[:na, na:]
    Sch = Hpp - (Hpa @ np.linalg.solve(Haa, Hap) if na else 0)
    v = wl.random_complex((H.shape[0] - na, 3), 21)
    ref = np.linalg.solve(Sch, v)
    assert np.linalg.norm(S.T(i, v) - ref) <= 1e-10 * np.linalg.norm(ref)


def test_artificial_layer_is_prefixed_and_panel_is_last():
    n, h, c, om = _small(n=(4, 4, 9))
    b = pn.panel_bounds(n[2], 3, 2)
    N3 = n[2] + 6
    assert b[0] == (0, 5) and b[-1][1] == N3 and len(b) == 5
    assert all(b[i][1] == b[i + 1][0] for i in range(len(b) - 1))
    H, lo, hi, ga = pn.aux_operator(c, h, om, 0.0, 3, 4.0, 2, 2)
    assert ga == 3 and H.shape[0] == 10 * 10 * (ga + hi - lo)
    # with C = 0 the artificial layer is plain J on the planes below the panel
    H0 = pn.aux_operator(c, h, om, 0.0, 3, 0.0, 2, 2)[0]
    J0 = hz.helmholtz_operator(c, h, om, 3, 0.0)
    pl = 100
    ref = J0[(lo - ga) * pl:hi * pl, (lo - ga) * pl:hi * pl]
    assert abs(H0 - ref).max() == 0.0


# ----------------------------------------------------------- Fig. 2.1 and ND
def test_nested_dissection_reproduces_fig_2_1():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "fig2_1_sep_tree.txt"))
            if l.strip() and not l.startswith("#")]
    Nx = Ny = 15
    nodes = nd.nested_dissection(Nx, Ny, 3)
    assert len(nodes) == 31
    assert max(x.depth for x in nodes) == 4
    owner = {}
    for k, x in enumerate(nodes):
        for cell in x.cells:
            owner[cell] = k
    for lab, fx, fy, par in rows:
        cell = (int(float(fx) * Nx), int(float(fy) * Ny))
        assert owner[cell] == int(lab), (lab, cell)
        assert nodes[int(lab)].parent == int(par)


def test_elimination_order_is_a_permutation_with_full_depth_supernodes():
    nodes = nd.nested_dissection(9, 7, 2)
    perm = nd.elimination_order(nodes, 9, 7, 3)
    assert sorted(perm) == list(range(9 * 7 * 3))
    for x in nodes:
        ids = perm[x.start:x.start + x.size]
        q = ids // (9 * 7)
        assert list(q) == sorted(q) and set(q) == {0, 1, 2}  # depth slowest, never split


# ------------------------------------------------ P8 factors and LDL^T pins
def test_ldlt_matches_cholesky_on_spd():
    rng = np.random.default_rng(0)
    B = rng.standard_normal((12, 12))
    A = B @ B.T + 12 * np.eye(12)
    L, d = ld.ldlt_unpivoted(A)
    Lc = sla.cholesky(A, lower=True)
    assert np.allclose(L * np.sqrt(d.real)[None, :], Lc, atol=1e-12, rtol=0)


def test_ldlt_uses_transpose_not_conjugate():
    rng = np.random.default_rng(1)
    B = rng.standard_normal((10, 10)) + 1j * rng.standard_normal((10, 10))
    A = B + B.T + 8 * np.eye(10)
    L, d = ld.ldlt_unpivoted(A)
    assert np.allclose(L @ np.diag(d) @ L.T, A, atol=1e-12, rtol=0)
    assert np.allclose(np.triu(L, 1), 0) and np.allclose(np.diag(L), 1)


def test_ldlt_breakdown_on_zero_pivot():
    with pytest.raises(ld.BreakdownError):
        ld.ldlt_unpivoted(np.array([[0.0, 1.0], [1.0, 2.0]]))


def test_front_structure_contains_the_factor():
    """The dense L is zero outside every front's rows S u U (symbolic update sets)."""
    n, h, c, om = _small(n=(6, 5, 6))
    H, lo, hi, ga = pn.aux_operator(c, h, om, wl.ALPHA_DEFAULT, 2, 4.0, 2, 1)
    N = hz.padded_shape(n, 2)
    nz = ga + hi - lo
    nodes = nd.nested_dissection(N[0], N[1], 3)
    perm = nd.elimination_order(nodes, N[0], N[1], nz)
    Hp = H[perm][:, perm]
    struct = nd.symbolic_structure(Hp)
    U = nd.update_sets(nodes, struct)
    L, d = ld.ldlt_unpivoted(Hp.toarray())
    assert np.allclose(L @ np.diag(d) @ L.T, Hp.toarray(), atol=1e-9 * abs(d).max(), rtol=0)
    scale = np.abs(L).max()
    for x, u in zip(nodes, U):
        S = np.arange(x.start, x.start + x.size)
        mask = np.ones(L.shape[0], bool)
        mask[S] = False
        mask[u] = False
        mask[:x.start] = False
        assert np.abs(L[mask][:, S]).max(initial=0.0) <= 1e-13 * scale
        # the update set lies in the ancestors and is geometric: the lateral
        # neighbours of the subtree box at every depth
        assert np.all(u >= x.start + x.size)
    blocks = ld.front_blocks(L, d, nodes, U)
    for (dF, LF, FBL), x, u in zip(blocks, nodes, U):
        assert dF.shape == (x.size,) and LF.shape == (x.size, x.size)
        assert FBL.shape == (len(u), x.size)


def test_update_set_is_lateral_perimeter_of_subtree_box():
    """Symbolic update sets equal the nodes adjacent to the subtree box, full depth."""
    Nx, Ny, nz = 11, 9, 2
    nodes = nd.nested_dissection(Nx, Ny, 2)
    perm = nd.elimination_order(nodes, Nx, Ny, nz)
    c = np.ones((nz, Ny, Nx))
    e = [np.ones(Nx), np.ones(Ny), np.ones(nz)]
    eh = [np.ones(Nx + 1), np.ones(Ny + 1), np.ones(nz + 1)]
    H = hz.stencil_operator(0.1, e, eh, 1.0, c)
    U = nd.update_sets(nodes, nd.symbolic_structure(H[perm][:, perm]))
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    for x, u in zip(nodes, U):
        x0, x1, y0, y1 = x.box
        cells = set()
        for a2 in range(y0, y1):
            for a1 in (x0 - 1, x1):
                if 0 <= a1 < Nx:
                    cells.add((a1, a2))
        for a1 in range(x0, x1):
            for a2 in (y0 - 1, y1):
                if 0 <= a2 < Ny:
                    cells.add((a1, a2))
        expect = sorted(inv[a1 + a2 * Nx + q * Nx * Ny] for (a1, a2) in cells for q in range(nz))
        assert list(u) == expect


# -------------------------------------------------------------- GMRES pins
def test_gmres_residual_is_minimal_over_krylov_space():
    """Each in-cycle estimate equals min ||b - A M^{-1} K_j y|| (brute force)."""
    rng = np.random.default_rng(4)
    n = 30
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Minv = np.diag(1.0 / np.diag(A))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it, rr, hist = gm.gmres(lambda v: A @ v, lambda v: Minv @ v, b, k=25, tol=1e-14,
                               maxit=10)
    AM = A @ Minv
    K = [b]
    for j in range(1, 11):
        Kj = np.column_stack(K)
        y = np.linalg.lstsq(AM @ Kj, b, rcond=None)[0]
        best = np.linalg.norm(b - AM @ Kj @ y) / np.linalg.norm(b)
        assert abs(hist[j - 1] - best) <= 1e-8 * max(best, 1e-12)
        K.append(AM @ K[-1])
    assert abs(rr - np.linalg.norm(b - A @ x) / np.linalg.norm(b)) < 1e-14


def test_gmres_restarted_converges_to_direct_solution():
    n, h, c, om = _small(n=(5, 5, 5))
    A = hz.helmholtz_operator(c, h, om, 2, 4.0)
    b = wl.random_complex(A.shape[0], 6)
    S = sw.Sweep(c, h, om, wl.ALPHA_DEFAULT, 2, 4.0, d=2)
    x, it, rr, _ = gm.gmres(lambda v: A @ v, S.apply, b, k=5, tol=1e-10, maxit=400)
    ref = spla.spsolve(A.tocsc(), b)
    assert rr < 1e-10
    assert np.linalg.norm(x - ref) <= 1e-7 * np.linalg.norm(ref)


def _dense_case(n, p, seed):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Minv = np.diag(1.0 / np.diag(A))
    B = rng.standard_normal((n, p)) + 1j * rng.standard_normal((n, p))
    return A, Minv, B


def test_block_gmres_with_one_column_is_gmres():
    A, Minv, B = _dense_case(40, 1, 7)
    x, it, rr, hist = gm.gmres(lambda v: A @ v, lambda v: Minv @ v, B[:, 0], k=5, tol=1e-9,
                               maxit=60)
    X, its, rel, bh = gm.block_gmres(lambda V: A @ V, lambda V: Minv @ V, B, k=5, tol=1e-9,
                                     maxit=60)
    assert its[0] == it and abs(rel[0] - rr) <= 1e-12
    assert np.allclose(hist, bh, rtol=1e-9, atol=0)
    assert np.linalg.norm(X[:, 0] - x) <= 1e-12 * np.linalg.norm(x)


def test_block_gmres_residual_is_minimal_over_block_krylov_space():
    """Each in-cycle estimate equals, for the worst column, min ||r0_c - A M^{-1} K_j y||
    over the block Krylov space K_j = [R0, (AM) R0, ..., (AM)^{j-1} R0] (brute force)."""
    A, Minv, B = _dense_case(36, 3, 8)
    X, its, rel, hist = gm.block_gmres(lambda V: A @ V, lambda V: Minv @ V, B, k=20,
                                       tol=1e-14, maxit=8)
    AM = A @ Minv
    bn = np.linalg.norm(B, axis=0)
    K = [B]
    for j in range(1, 9):
        Kj = np.column_stack(K)
        worst = 0.0
        for c in range(3):
            y = np.linalg.lstsq(AM @ Kj, B[:, c], rcond=None)[0]
            worst = max(worst, np.linalg.norm(B[:, c] - AM @ Kj @ y) / bn[c])
        assert abs(hist[j - 1] - worst) <= 1e-8 * max(worst, 1e-12), (j, hist[j - 1], worst)
        K.append(AM @ K[-1])
    for c in range(3):
        assert abs(rel[c] - np.linalg.norm(B[:, c] - A @ X[:, c]) / bn[c]) < 1e-14


def test_block_gmres_terminates_in_n_over_p_steps():
    """The block Krylov space of p columns reaches dimension n after n/p steps."""
    A, Minv, B = _dense_case(24, 4, 9)
    X, its, rel, _ = gm.block_gmres(lambda V: A @ V, lambda V: Minv @ V, B, k=10, tol=1e-10)
    assert max(its) <= 6 and max(rel) < 1e-10


def test_block_gmres_needs_no_more_iterations_than_gmres_per_column():
    """K_j(AM, r_c) lies in the block space, so without restarts the block
    method never needs more steps than any column's own GMRES; on the sweep
    preconditioned Helmholtz problem it converges to the direct solution."""
    n, h, c, om = _small(n=(6, 5, 5))
    A = hz.helmholtz_operator(c, h, om, 2, 4.0)
    S = sw.Sweep(c, h, om, wl.ALPHA_DEFAULT, 2, 4.0, d=2)
    B = wl.random_complex((A.shape[0], 3), 11)
    X, its, rel, _ = gm.block_gmres(lambda V: A @ V, S.apply, B, k=60, tol=1e-10, maxit=60)
    for col in range(3):
        _, it, _, _ = gm.gmres(lambda v: A @ v, S.apply, B[:, col], k=60, tol=1e-10, maxit=60)
        assert its[col] <= it
        ref = spla.spsolve(A.tocsc(), B[:, col])
        assert np.linalg.norm(X[:, col] - ref) <= 1e-7 * np.linalg.norm(ref)


def test_givens_zeroes_subdiagonal():
    for a, b in [(1 + 2j, 0.5), (0.0, 2.0), (3 - 1j, 0.0), (1e-3j, 7.0)]:
        c, s = gm.givens(a, b)
        assert abs(-np.conj(s) * a + c * b) < 1e-14 * (abs(a) + abs(b))
        assert abs(c * c + abs(s) ** 2 - 1) < 1e-14


# ------------------------------------------------------ P9/P11 soft checks
def test_front_work_grows_like_n_cubed_per_panel():
    """Per-panel dense front work is O(gamma^3 n^3) (Sec. 1.1): doubling n gives ~8x."""
    def work(Nx):
        nodes = nd.nested_dissection(Nx, Nx, 4)
        f = 0.0
        for x in nodes:
            x0, x1, y0, y1 = x.box
            s = len(x.cells)
            u = 0
            u += (y1 - y0) * ((x0 > 0) + (x1 < Nx))
            u += (x1 - x0) * ((y0 > 0) + (y1 < Nx))
            f += s ** 3 / 6 + s * s * u / 2 + s * u * u / 2
        return f
    r1 = work(64) / work(32)
    r2 = work(128) / work(64)
    assert 6.0 < r1 < 10.0 and 6.0 < r2 < 10.0


def test_sweep_preconditioner_reduces_iterations():
    """Sec. 1.1: the sweep gives few iterations where unpreconditioned GMRES stalls."""
    n, h, c, om = _small(n=(8, 8, 8))
    A = hz.helmholtz_operator(c, h, om, 3, 4.0)
    S = sw.Sweep(c, h, om, wl.ALPHA_DEFAULT, 3, 4.0, d=2)
    b = wl.gaussian_sources(n, 3, h, [[0.5, 0.5, 0.5]])[0].ravel()
    _, it_s, rr_s, _ = gm.gmres(lambda v: A @ v, S.apply, b, k=20, tol=1e-5)
    _, it_0, rr_0, _ = gm.gmres(lambda v: A @ v, lambda v: v, b, k=20, tol=1e-5, maxit=150)
    assert rr_s < 1e-5 and it_s < 30 and it_0 > 3 * it_s
