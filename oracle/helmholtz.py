"""Grid, complex-stretched PML and the 7-point Helmholtz operator (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

What the paper fixes
--------------------
* The operator is A = -Delta - omega^2/c(x)^2 with time dependence
  e^{-i omega t} (Sec. 1, Eq. 1.1), discretised by second-order finite
  differences on a grid ordered lexicographically with i1 fastest, which
  makes the system block tridiagonal by x3 planes and complex symmetric,
  not Hermitian, because of the PML (Sec. 1.1, the block tridiagonal system).
* The preconditioner is built from the artificially damped operator
  J = -Delta - (omega + i alpha)^2/c(x)^2 (Sec. 1.1, Eq. 1.5).

Readings (the paper is silent; each is listed in the design notes)
-------------------------------------------------------------------
* Grid: interior nodes at x_j = i_j h, i_j = 1..n_j; gamma PML nodes are
  added past every face, so padded node a_j = 0..n_j+2gamma_j-1 sits at
  x_j = (a_j - gamma_j + 1) h; homogeneous Dirichlet just outside the padding.
* PML profile: depth past the last interior node t = max(0, h - x, x - n h),
  eta = (gamma + 1) h (the Dirichlet wall), sigma(t) = (C/eta) (t/eta)^2 and
  stretch e(x) = 1 + i sigma(t)/omega.  The sign makes outgoing waves
  e^{+ikx} decay under e^{-i omega t}.  An axis with gamma = 0 is not stretched.
* Symmetric stretched stencil: with E = e1 e2 e3 at the node and
  w_j^{+-} = e_k(x_k) e_l(x_l) / e_j(x_j +- h/2),
      (H u)_p = h^-2 sum_j [(w_j^+ + w_j^-) u_p - w_j^+ u_{p+e_j}
                            - w_j^- u_{p-e_j}] - kappa^2 E(p) u_p / c(p)^2,
  kappa^2 = omega^2 for A and (omega + i alpha)^2 for J.  The stretching uses
  the real omega in both, so damping enters only the mass term and
  J_{i+1,i} = A_{i+1,i}.
* c in the padding is the interior value at the nearest interior node.
"""

import numpy as np
import scipy.sparse as sp


def gamma3(gamma):
    """PML width per axis as a 3-tuple (an int means the same on all axes)."""
    if np.isscalar(gamma):
        return (int(gamma),) * 3
    g = tuple(int(v) for v in gamma)
    assert len(g) == 3
    return g


def padded_shape(n, gamma):
    """(N1, N2, N3): interior nodes plus gamma PML nodes past each face."""
    g = gamma3(gamma)
    return tuple(int(n[j]) + 2 * g[j] for j in range(3))


def pml_sigma(t, C, eta):
    """Quadratic PML damping profile sigma(t) = (C/eta) (t/eta)^2."""
    t = np.asarray(t, dtype=np.float64)
    return (C / eta) * (t / eta) ** 2


def stretch(t, C, eta, omega):
    """Complex coordinate stretch e = 1 + i sigma(t)/omega."""
    return 1.0 + 1j * pml_sigma(t, C, eta) / omega


def physical_depth(x, nj, h):
    """Distance of position x past the interior [h, nj h] along one axis."""
    x = np.asarray(x, dtype=np.float64)
    return np.maximum(0.0, np.maximum(h - x, x - nj * h))


def axis_stretch(nj, gj, h, C, omega):
    """Stretch factors along one padded axis.

    Returns (e_node, e_half): e_node[a] at padded node a (length nj+2gj);
    e_half[a] at the half-node between nodes a-1 and a (length nj+2gj+1,
    e_half[0] lies between the Dirichlet wall and node 0).
    """
    Nj = nj + 2 * gj
    a = np.arange(Nj, dtype=np.float64)
    x = (a - gj + 1) * h
    xh = np.concatenate([x - 0.5 * h, [x[-1] + 0.5 * h]])
    if gj == 0 or C == 0.0:
        return np.ones(Nj, dtype=np.complex128), np.ones(Nj + 1, dtype=np.complex128)
    eta = (gj + 1) * h
    e_node = stretch(physical_depth(x, nj, h), C, eta, omega)
    e_half = stretch(physical_depth(xh, nj, h), C, eta, omega)
    return e_node.astype(np.complex128), e_half.astype(np.complex128)


def pad_velocity(c, gamma):
    """Extend interior c (shape (n3, n2, n1)) into the padding by clamping."""
    g = gamma3(gamma)
    return np.pad(np.asarray(c, dtype=np.float64),
                  ((g[2], g[2]), (g[1], g[1]), (g[0], g[0])), mode="edge")


def stencil_operator(h, e_node, e_half, kappa2, c_box):
    """Symmetric stretched 7-point operator on a box (Dirichlet outside).

    e_node[j], e_half[j]: stretch at nodes / half-nodes along axis j of the box
    (axis 0 = x1, the fastest index).  c_box: velocity, numpy shape
    (N3, N2, N1).  Returns a CSR matrix of order N1 N2 N3, lexicographic with
    x1 fastest.
    """
    N3, N2, N1 = c_box.shape
    assert len(e_node[0]) == N1 and len(e_node[1]) == N2 and len(e_node[2]) == N3
    e1 = e_node[0][None, None, :]
    e2 = e_node[1][None, :, None]
    e3 = e_node[2][:, None, None]
    idx = np.arange(N1 * N2 * N3).reshape(N3, N2, N1)
    # products of the two other axes' node stretches, per axis j
    others = [e2 * e3, e1 * e3, e1 * e2]
    E = e1 * e2 * e3
    diag = -kappa2 * E / c_box ** 2
    rows, cols, vals = [], [], []
    inv_h2 = 1.0 / (h * h)
    # numpy axis for grid axis j: x1 -> 2, x2 -> 1, x3 -> 0
    for j, ax in ((0, 2), (1, 1), (2, 0)):
        eh = e_half[j]
        shp = [1, 1, 1]
        shp[ax] = len(eh) - 1
        eh_plus = eh[1:].reshape(shp)
        eh_minus = eh[:-1].reshape(shp)
        P = np.broadcast_to(others[j], (N3, N2, N1))
        wp = P / eh_plus
        wm = P / eh_minus
        diag = diag + (wp + wm) * inv_h2
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        lo, hi = tuple(lo), tuple(hi)
        # coupling p -> p + e_j (row p) and p + e_j -> p (row p + e_j)
        rows.append(idx[lo].ravel()); cols.append(idx[hi].ravel())
        vals.append((-wp[lo] * inv_h2).ravel())
        rows.append(idx[hi].ravel()); cols.append(idx[lo].ravel())
        vals.append((-wm[hi] * inv_h2).ravel())
    rows.append(idx.ravel()); cols.append(idx.ravel())
    vals.append(np.broadcast_to(diag, (N3, N2, N1)).ravel())
    n = N1 * N2 * N3
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    M.sum_duplicates()
    return M


def axis_tables(n, gamma, h, C, omega):
    """Physical (e_node, e_half) per axis for the padded grid."""
    g = gamma3(gamma)
    tabs = [axis_stretch(int(n[j]), g[j], h, C, omega) for j in range(3)]
    return [t[0] for t in tabs], [t[1] for t in tabs]


def helmholtz_operator(c, h, omega, gamma, C, alpha=0.0):
    """A (alpha = 0) or J (alpha > 0) on the whole padded grid (CSR).

    c: interior velocity, numpy shape (n3, n2, n1), x1 fastest.
    """
    c = np.asarray(c, dtype=np.float64)
    n = (c.shape[2], c.shape[1], c.shape[0])
    e_node, e_half = axis_tables(n, gamma, h, C, omega)
    kappa2 = (omega + 1j * alpha) ** 2
    return stencil_operator(h, e_node, e_half, kappa2, pad_velocity(c, gamma))


def padded_positions(n, gamma, h):
    """Coordinates (x1, x2, x3) of every padded node, each of numpy shape (N3, N2, N1)."""
    g = gamma3(gamma)
    N = padded_shape(n, g)
    ax = [(np.arange(N[j]) - g[j] + 1) * h for j in range(3)]
    X3, X2, X1 = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X1, X2, X3
