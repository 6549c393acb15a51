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


def block_gmres(matvec, precond, B, k=20, tol=1e-5, maxit=1000):
    """Block GMRES(k): the columns of B share one block Krylov space (Sec. 2.4
    names block variants as a way to lower the iteration count).

    matvec and precond act on blocks (N x q arrays).  B is N x p.  Returns
    (X, iters per column, relres per column, history of the largest in-cycle
    estimate per iteration).

    Readings (the paper only names the method):
    * Right preconditioning and a zero initial guess, as for GMRES(k); one
      iteration is one application of M^{-1} to the block of still active
      columns, and a column's count is the number of iterations it took part in.
    * Each cycle starts from the true residual block of the columns whose true
      relative residual is still >= tol (converged columns leave the block at
      a restart).  The residual block is split as R0 = V_0 S by a reduced QR.
    * Arnoldi step j: W = A M^{-1} V_j; block modified Gram-Schmidt against
      V_0..V_j (H_ij = V_i^H W, W -= V_i H_ij); reduced QR W = V_{j+1} H_{j+1,j}.
    * The block least-squares problem min ||E_1 S - H_j Y|| (Frobenius norm,
      which decouples by column) is solved by a library least-squares routine
      after every step; column c's estimate is the norm of its residual
      column, relative to ||b_c||.  The cycle ends when every active estimate
      is below tol, after k steps, or when a diagonal entry of H_{j+1,j} falls
      below 1e-14 times the largest one seen (the block Krylov space has
      become invariant: rank breakdown).
    * X += M^{-1} [V_0 .. V_j] Y, then the true residual decides.
    """
    B = np.asarray(B, dtype=np.complex128)
    N, p = B.shape
    bn = np.linalg.norm(B, axis=0)
    X = np.zeros_like(B)
    its = np.zeros(p, dtype=int)
    rel = np.where(bn > 0, 1.0, 0.0)
    history = []
    total = 0
    while True:
        R = B - matvec(X)
        for c in range(p):
            if bn[c] > 0:
                rel[c] = np.linalg.norm(R[:, c]) / bn[c]
        act = [c for c in range(p) if bn[c] > 0 and rel[c] >= tol]
        if not act or total >= maxit:
            break
        q = len(act)
        V0, S = np.linalg.qr(R[:, act])
        V = [V0]
        Hcols = []  # block column j: ((j+2) q) x q
        scale = np.max(np.abs(np.diag(S)))
        jdone = 0
        Y = None
        for j in range(k):
            W = matvec(precond(V[j]))
            total += 1
            its[act] += 1
            col = np.zeros(((j + 2) * q, q), dtype=np.complex128)
            for i in range(j + 1):
                Hij = V[i].conj().T @ W
                W = W - V[i] @ Hij
                col[i * q:(i + 1) * q] = Hij
            Vn, Rn = np.linalg.qr(W)
            col[(j + 1) * q:] = Rn
            Hcols.append(col)
            jdone = j + 1
            Hbar = np.zeros(((j + 2) * q, (j + 1) * q), dtype=np.complex128)
            for jj, cj in enumerate(Hcols):
                Hbar[:cj.shape[0], jj * q:(jj + 1) * q] = cj
            E = np.zeros(((j + 2) * q, q), dtype=np.complex128)
            E[:q] = S
            Y = np.linalg.lstsq(Hbar, E, rcond=None)[0]
            res = np.linalg.norm(E - Hbar @ Y, axis=0) / bn[act]
            history.append(float(res.max()))
            d = np.abs(np.diag(Rn))
            scale = max(scale, float(d.max()))
            if res.max() < tol or total >= maxit or d.min() <= 1e-14 * scale:
                break
            V.append(Vn)
        VY = np.zeros((N, q), dtype=np.complex128)
        for i in range(jdone):
            VY = VY + V[i] @ Y[i * q:(i + 1) * q]
        X[:, act] = X[:, act] + precond(VY)
    return X, its, rel, history
