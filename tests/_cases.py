"""Seeded parity cases shared by the GPU tests (inputs only, no method arithmetic)."""

import numpy as np

from paper_1204_0111_amd import workloads as wl


def case(n=(14, 12, 13), gamma=3, d=3, leaf=4, model="grf", seed=5, C=4.0, alpha=None):
    n = tuple(int(v) for v in n)
    h = wl.grid_h(n)
    c = {"grf": lambda: wl.velocity_grf(n, h, seed),
         "layered": lambda: wl.velocity_layered(n, h, seed),
         "constant": lambda: wl.velocity_constant(n),
         "barrier": lambda: wl.velocity_barrier(n, h),
         "wedge_paper": lambda: wl.velocity_wedge_paper(n, h),
         "two_layer": lambda: wl.velocity_two_layer(n, h),
         "waveguide": lambda: wl.velocity_waveguide(n, h)}[model]()
    return dict(name=model, src="paper", n=n, h=h, c=c, omega=wl.omega_for_ppw(c, h),
                alpha=wl.ALPHA_DEFAULT if alpha is None else alpha, gamma=gamma, C=C, d=d,
                leaf=leaf)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


TOL = {"c128": 1e-12, "c64": 1e-4}


# Constant velocity, no PML, alpha = 0 and omega^2 = 6 c^2 / h^2: every
# diagonal entry 6/h^2 - omega^2/c^2 of the 7-point operator is zero.  With
# this h, 1/h^2 is exactly 24 in floating point and omega^2 = 144, so the
# entries are exact zeros.
H_ZERO_DIAG = 0.2041241452319315
OMEGA_ZERO_DIAG = 12.0


def zero_diagonal_problem():
    n = (8, 7, 6)
    return dict(name="constant", src="paper", n=n, h=H_ZERO_DIAG, c=np.ones((n[2], n[1], n[0])),
                omega=OMEGA_ZERO_DIAG, alpha=0.0, gamma=2, C=0.0, d=2, leaf=3)
