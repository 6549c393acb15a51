"""Approximate Schur-complement inverses T_i and the sweep M^{-1} (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

What the paper fixes
--------------------
* T_i applies the approximate inverse Schur complement of panel i: extend
  the panel vector by zero over the artificial PML, solve with H_i, and
  extract the panel's entries, which is valid because the panel's unknowns
  come last in H_i (Sec. 1.1, Eqs. 1.3-1.4 and Alg. 1.3).
* The sweep (Sec. 1.1, Alg. 1.5) is a block forward and backward
  substitution over the panels of the block LDL^T form of J, with each exact
  inverse Schur complement replaced by T_i.  Going up, every panel's block is
  multiplied by its T_i and its coupling to the panel above is subtracted
  from that panel's block.  Going down, every panel but the last subtracts
  T_i applied to the transposed coupling of the already final block above it.
  The coupling blocks J_{i+1,i} are those of the damped operator J.

The solves with H_i use SciPy's sparse LU (a library primitive); nothing is
blocked or reordered beyond the steps above.  `exact=True` replaces every H_i
by J restricted to all planes up to the end of panel i (no artificial PML):
then T_i is the exact inverse Schur complement and the sweep is the exact
block LDL^T solve of Algs. 1.1-1.2, i.e. J^{-1}.
"""

import numpy as np
import scipy.sparse.linalg as spla

from . import helmholtz as hz
from . import panels as pn


class Sweep:
    def __init__(self, c, h, omega, alpha, gamma, C, d, exact=False):
        c = np.asarray(c, dtype=np.float64)
        self.n = (c.shape[2], c.shape[1], c.shape[0])
        N = hz.padded_shape(self.n, gamma)
        self.plane = N[0] * N[1]
        self.N_pad = N[0] * N[1] * N[2]
        self.J = hz.helmholtz_operator(c, h, omega, gamma, C, alpha)
        self.bounds = pn.panel_bounds(self.n[2], gamma, d)
        self.m = len(self.bounds)
        self.lus, self.ga = [], []
        for i, (lo, hi) in enumerate(self.bounds):
            if exact:
                H = self.J[:hi * self.plane, :hi * self.plane]
                ga_planes = lo
            else:
                H, lo2, hi2, ga_planes = pn.aux_operator(c, h, omega, alpha, gamma, C, d, i)
                assert (lo2, hi2) == (lo, hi)
            self.lus.append(spla.splu(H.tocsc()))
            self.ga.append(ga_planes)

    def rows(self, i):
        lo, hi = self.bounds[i]
        return slice(lo * self.plane, hi * self.plane)

    def J_block(self, i, j):
        """J_{i,j}: rows of panel i, columns of panel j."""
        return self.J[self.rows(i), self.rows(j)]

    def T(self, i, v):
        """Alg. 1.3: zero-extend over the artificial planes, solve, extract."""
        pre = self.ga[i] * self.plane
        v = np.asarray(v)
        shape_rhs = v.shape[1:]
        ext = np.zeros((pre + v.shape[0],) + shape_rhs, dtype=np.complex128)
        ext[pre:] = v
        sol = self.lus[i].solve(ext)
        return sol[pre:]

    def apply(self, f):
        """Alg. 1.5: u = M^{-1} f on the padded grid (vector or N_pad x nrhs block)."""
        f = np.asarray(f, dtype=np.complex128)
        u = [f[self.rows(i)].copy() for i in range(self.m)]
        for i in range(self.m - 1):
            u[i] = self.T(i, u[i])
            u[i + 1] = u[i + 1] - self.J_block(i + 1, i) @ u[i]
        u[self.m - 1] = self.T(self.m - 1, u[self.m - 1])
        for i in range(self.m - 2, -1, -1):
            u[i] = u[i] - self.T(i, self.J_block(i + 1, i).T @ u[i + 1])
        return np.concatenate(u, axis=0)
