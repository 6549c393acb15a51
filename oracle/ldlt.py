"""Unpivoted complex-symmetric LDL^T and the frontal blocks (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

What the paper fixes
--------------------
* The auxiliary problems are complex symmetric, factored as L D L^T with
  transposes (never conjugates) and without pivoting (Sec. 1.1, the block
  tridiagonal system; Sec. 2.2; Sec. 2.5 on the lack of pivoting).
* For a front F = [F_TL *; F_BL F_BR] the partial factorisation overwrites
  F_TL by L_F and D_F, then F_BL := F_BL L_F^{-T}, Z := F_BL,
  F_BL := F_BL D_F^{-1}, F_BR := F_BR - Z F_BL^T (Sec. 2.2).  The result is
  exactly the corresponding block of the full factorisation of the permuted
  matrix, so the per-front blocks here are taken from the dense factorisation:
  D_F = D[S], L_F = L[S, S] and the final coupling F_BL = L[U, S].
* Selective inversion replaces each triangular solve with L_F by a product
  with L_F^{-1} (Sec. 2.2).  The blocks G_TL = L_F^{-1} and
  G_BL = F_BL L_F^{-1} are formed here for comparison with the device's
  inverted fronts.
"""

import numpy as np
import scipy.linalg as sla


class BreakdownError(ArithmeticError):
    pass


def ldlt_unpivoted(A):
    """Textbook right-looking LDL^T without pivoting (transpose, not conjugate).

    Returns (L, d) with L unit lower triangular and A = L diag(d) L^T.
    """
    A = np.array(A, dtype=np.complex128, copy=True)
    n = A.shape[0]
    L = np.eye(n, dtype=np.complex128)
    d = np.empty(n, dtype=np.complex128)
    for k in range(n):
        d[k] = A[k, k]
        if d[k] == 0 or not np.isfinite(d[k]):
            raise BreakdownError("zero or non-finite pivot at %d" % k)
        col = A[k + 1:, k].copy()
        L[k + 1:, k] = col / d[k]
        A[k + 1:, k + 1:] -= np.outer(L[k + 1:, k], col)
    return L, d


def front_blocks(L, d, nodes, usets):
    """Per-supernode (D_F, L_F, F_BL) from a dense factorisation in elimination order."""
    out = []
    for nd, U in zip(nodes, usets):
        S = slice(nd.start, nd.start + nd.size)
        out.append((d[S].copy(), L[S, S].copy(), L[np.asarray(U, dtype=np.int64), S].copy()))
    return out


def selective_inverse(L_F, F_BL):
    """(G_TL, G_BL) = (L_F^{-1}, F_BL L_F^{-1})."""
    s = L_F.shape[0]
    G_TL = sla.solve_triangular(L_F, np.eye(s, dtype=np.complex128), lower=True,
                                unit_diagonal=True)
    return G_TL, F_BL @ G_TL
