"""Panels and their PML-padded auxiliary problems H_i (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

What the paper fixes
--------------------
* The x3 planes are grouped into m panels of O(gamma) contiguous planes
  (Sec. 1.1, the paragraph before Alg. 1.4).
* Setup: S_0 := J_{0,0} is factored as is; every later panel's auxiliary
  problem H_i is formed by prefixing PML to J_{i,i} and factored
  (Sec. 1.1, Alg. 1.4).  The artificial radiation condition is moved next to
  the panel, and the planes after the panel are ignored, i.e. a homogeneous
  Dirichlet condition is put on the cut (Sec. 1.1, Fig. 1.2).

Readings
--------
* m = ceil(n3/d).  Panel i owns the interior planes i3 in
  [i d + 1, min((i+1) d, n3)]; panel 0 also owns the gamma bottom physical
  PML planes and panel m-1 the gamma top ones.
* For i >= 1, H_i is J on the gamma grid planes just below panel i followed by
  panel i's planes.  On those gamma planes, and on the half-planes up to the
  panel, the x3 stretch is the artificial profile with depth measured from
  the panel's first plane p0, t = (p0 - p3) h, eta = (gamma + 1) h; the
  velocity there is the true (clamped) velocity of those planes.  Dirichlet
  holds below the artificial layer and above the panel.
* The lateral (x1, x2) PML is the physical one on every plane.
"""

import math

import numpy as np

from . import helmholtz as hz


def panel_bounds(n3, gamma, d):
    """Global padded plane ranges [lo, hi) of the m panels."""
    g = hz.gamma3(gamma)[2]
    N3 = int(n3) + 2 * g
    m = int(math.ceil(n3 / d))
    out = []
    for i in range(m):
        lo = 0 if i == 0 else g + i * d
        hi = N3 if i == m - 1 else g + (i + 1) * d
        out.append((lo, hi))
    return out


def artificial_planes(i, gamma):
    """Number of artificial PML planes prefixed to panel i (0 for panel 0)."""
    return 0 if i == 0 else hz.gamma3(gamma)[2]


def aux_x3_tables(n3, gamma, h, C, omega, lo, hi, ga):
    """x3 stretch tables (node, half-node) of an auxiliary problem.

    The box has ga artificial planes then the panel planes [lo, hi).
    """
    g = hz.gamma3(gamma)[2]
    _, gl_half = hz.axis_stretch(int(n3), g, h, C, omega)
    gl_node, _ = hz.axis_stretch(int(n3), g, h, C, omega)
    nz = ga + (hi - lo)
    eta = (g + 1) * h
    e_node = np.empty(nz, dtype=np.complex128)
    e_half = np.empty(nz + 1, dtype=np.complex128)
    for q in range(nz):
        if q < ga:
            e_node[q] = hz.stretch((ga - q) * h, C, eta, omega) if C != 0.0 else 1.0
        else:
            e_node[q] = gl_node[lo - ga + q]
    for a in range(nz + 1):
        if ga > 0 and a <= ga:
            e_half[a] = hz.stretch((ga - a + 0.5) * h, C, eta, omega) if C != 0.0 else 1.0
        else:
            e_half[a] = gl_half[lo - ga + a]
    return e_node, e_half


def aux_operator(c, h, omega, alpha, gamma, C, d, i):
    """H_i as CSR over its box (lateral padded grid x aux planes), x1 fastest.

    Returns (H, lo, hi, ga): panel plane range and the number of artificial
    planes in front of it.
    """
    c = np.asarray(c, dtype=np.float64)
    n = (c.shape[2], c.shape[1], c.shape[0])
    bounds = panel_bounds(n[2], gamma, d)
    lo, hi = bounds[i]
    ga = artificial_planes(i, gamma)
    e_node, e_half = hz.axis_tables(n, gamma, h, C, omega)
    e3n, e3h = aux_x3_tables(n[2], gamma, h, C, omega, lo, hi, ga)
    cpad = hz.pad_velocity(c, gamma)[lo - ga:hi]
    kappa2 = (omega + 1j * alpha) ** 2
    H = hz.stencil_operator(h, [e_node[0], e_node[1], e3n], [e_half[0], e_half[1], e3h],
                            kappa2, cpad)
    return H, lo, hi, ga
