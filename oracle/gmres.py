"""Right-preconditioned GMRES(k) in FP64 (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

What the paper fixes
--------------------
* The preconditioned system is solved with GMRES(k) (Sec. 2.4) from a zero
  initial guess (Sec. 3) until the relative residual falls below the target
  (Sec. 3, Tables 3.1-3.2).

Readings
--------
* Right preconditioning, so the residual that is minimised is the true
  residual b - A x of the undamped operator A; Arnoldi by modified
  Gram-Schmidt with the Hermitian inner product; complex Givens rotations on
  the Hessenberg matrix (Saad and Schultz's GMRES).
* Each right-hand side runs its own GMRES.  The in-cycle estimate triggers a
  check of the true relative residual ||b - A x|| / ||b||, which decides.
* An iteration is one preconditioner application inside an Arnoldi step.
"""

import numpy as np


def givens(a, b):
    """(c, s) with c real so that [[c, s], [-conj(s), c]] [a, b]^T = [r, 0]^T."""
    if b == 0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    r = np.hypot(abs(a), abs(b))
    c = abs(a) / r
    s = (a / abs(a)) * np.conj(b) / r
    return c, s


def gmres(matvec, precond, b, k=20, tol=1e-5, maxit=1000):
    """Solve A x = b with x = M^{-1} y, GMRES(k).  Returns (x, iters, relres, history).

    matvec(v) = A v; precond(v) = M^{-1} v; b is one complex vector.
    history holds the in-cycle residual estimates (relative) per iteration.
    """
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bnorm == 0:
        return x, 0, 0.0, []
    iters = 0
    history = []
    r = b - matvec(x)
    while True:
        beta = np.linalg.norm(r)
        if beta / bnorm < tol or iters >= maxit:
            break
        V = [r / beta]
        H = np.zeros((k + 1, k), dtype=np.complex128)
        cs = np.zeros(k)
        sn = np.zeros(k, dtype=np.complex128)
        g = np.zeros(k + 1, dtype=np.complex128)
        g[0] = beta
        jdone = 0
        for j in range(k):
            w = matvec(precond(V[j]))
            iters += 1
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            hnext = np.linalg.norm(w)
            H[j + 1, j] = hnext
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            jdone = j + 1
            est = abs(g[j + 1]) / bnorm
            history.append(est)
            if est < tol or iters >= maxit:
                break
            if hnext == 0:
                break
            V.append(w / hnext)
        y = np.zeros(jdone, dtype=np.complex128)
        for i in range(jdone - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:jdone] @ y[i + 1:]) / H[i, i]
        Vy = np.zeros_like(b)
        for i in range(jdone):
            Vy = Vy + y[i] * V[i]
        x = x + precond(Vy)
        r = b - matvec(x)
        if np.linalg.norm(r) / bnorm < tol or iters >= maxit:
            break
    return x, iters, np.linalg.norm(r) / bnorm, history
