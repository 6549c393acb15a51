"""Seeded synthetic inputs: problem configurations, velocity models, sources.

This module only produces inputs (velocity arrays on the interior grid,
right-hand sides on the padded grid, random vectors and the parameters of
each workload).  It holds none of the method's arithmetic and is shared by
the tests, the benchmark and the smoke check.

Velocity arrays have numpy shape (n3, n2, n1) (x1 fastest), float64.
Right-hand sides have numpy shape (nrhs, N3, N2, N1) on the padded grid,
complex128.  The paper's models (Sec. 3) are reproduced where they are
analytic; the Overthrust model is not available, so layered and
wedge-plus-inclusion models with its structure stand in for it.
"""

import math

import numpy as np

ALPHA_DEFAULT = 2.25 * math.pi   # damping used for Table 3.2 (Sec. 3)
PML_AMP_DEFAULT = 4.0            # PML amplitude C, the value most used in Table 3.1
# The workloads, by name.  `seed` offsets the generator seed 12040111 (sub
# problems of a batch add 1000 each); C is the PML amplitude frozen from a
# modest search on the FP64 path (as Sec. 3 did per problem): the value with
# the fewest GMRES(20) iterations to 1e-5, ties to the smallest residual.
WORKLOADS = {
    # 20^3, constant velocity, one plane per panel
    "const20": dict(seed=1, n=(20, 20, 20), gamma=5, d=1, leaf=8, model="constant", nrhs=1,
                    src="centre", C=15.0),
    # 50^3 Gaussian random field in [1, 3]
    "grf50": dict(seed=2, n=(50, 50, 50), gamma=8, d=4, leaf=4, model="grf", nrhs=1,
                  src="centre", C=30.0),
    # 100^3 layered model, 16 surface shots
    "layered100": dict(seed=3, n=(100, 100, 100), gamma=10, d=4, leaf=4, model="layered",
                       nrhs=16, src="surface", C=30.0),
    # one of 48 problems with per-axis sizes drawn from 30..70, 4 shots each
    "batch48": dict(seed=4, n=None, gamma=8, d=4, leaf=4, model="grf", nrhs=4, src="surface",
                    C=30.0, nprob=48),
    # 250^3 wedge with a salt body, 32 surface shots
    "wedge250": dict(seed=5, n=(250, 250, 250), gamma=12, d=4, leaf=4, model="wedge_salt",
                     nrhs=32, src="surface", C=30.0),
    # one GPU's share of it: the same lateral shape, PML and panel depth over
    # 40 planes (10 of its 63 panels), the same 32 shots
    "wedge250slab": dict(seed=5, n=(250, 250, 40), gamma=12, d=4, leaf=4, model="wedge_salt",
                         nrhs=32, src="surface", C=30.0),
    # the analytic models of Sec. 3 at 50^3 (5 PML points, 4 planes per panel
    # as in Table 3.1), each with the four forcings f0..f3 as one block; C is
    # the amplitude the search over {2,3,4,7.5,10,15,20,30,45,60} picked
    "barrier50": dict(seed=6, n=(50, 50, 50), gamma=5, d=4, leaf=4, model="barrier", nrhs=4,
                      src="paper", C=15.0),
    "wedge50": dict(seed=7, n=(50, 50, 50), gamma=5, d=4, leaf=4, model="wedge_paper", nrhs=4,
                    src="paper", C=20.0),
    "twolayer50": dict(seed=8, n=(50, 50, 50), gamma=5, d=4, leaf=4, model="two_layer", nrhs=4,
                       src="paper", C=15.0),
    "waveguide50": dict(seed=9, n=(50, 50, 50), gamma=5, d=4, leaf=4, model="waveguide", nrhs=4,
                        src="paper", C=15.0),
}


def seed_for(offset, sub=0):
    return 12040111 + 1000 * sub + offset


def grid_h(n):
    """One spacing for all axes: the largest axis spans the unit interval."""
    return 1.0 / (max(int(v) for v in n) + 1)


def omega_for_ppw(c, h, ppw=10.0):
    """Angular frequency resolving the shortest wavelength with ppw points."""
    cmin = float(np.min(c))
    return 2.0 * math.pi * cmin / (ppw * h)


def _axes(n, h):
    # interior node coordinates x_j = i_j h, i_j = 1..n_j
    return [np.arange(1, int(n[j]) + 1) * h for j in range(3)]


def _mesh(n, h):
    a = _axes(n, h)
    X3, X2, X1 = np.meshgrid(a[2], a[1], a[0], indexing="ij")
    return X1, X2, X3


def velocity_constant(n, value=1.0):
    return np.full((int(n[2]), int(n[1]), int(n[0])), float(value))


def velocity_grf(n, h, seed, corr=0.1, lo=1.0, hi=3.0):
    """Smooth Gaussian random field mapped affinely onto [lo, hi]."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((int(n[2]), int(n[1]), int(n[0])))
    s = gaussian_filter(w, sigma=corr / h, mode="reflect")
    s = (s - s.min()) / max(s.max() - s.min(), 1e-300)
    return lo + (hi - lo) * s


def velocity_layered(n, h, seed, layers=8, vmin=1.5, vmax=6.0, noise=0.05):
    """Dipping planar layers, velocity increasing with depth x3, +/- noise."""
    rng = np.random.default_rng(seed)
    X1, X2, X3 = _mesh(n, h)
    L = [(int(n[j]) + 1) * h for j in range(3)]
    z = np.sort(rng.uniform(0.05, 0.95, layers - 1))
    a = rng.uniform(-0.1, 0.1, layers - 1)
    b = rng.uniform(-0.1, 0.1, layers - 1)
    u1, u2, u3 = X1 / L[0], X2 / L[1], X3 / L[2]
    k = np.zeros(X1.shape, dtype=np.int64)
    for i in range(layers - 1):
        k += (u3 > z[i] + a[i] * (u1 - 0.5) + b[i] * (u2 - 0.5)).astype(np.int64)
    v = vmin + (vmax - vmin) * k / (layers - 1)
    return v * (1.0 + rng.uniform(-noise, noise, v.shape))


def velocity_wedge_salt(n, h, seed, noise=0.03):
    """Three dipping layers 2.0/3.0/4.5 and an ellipsoidal c = 4.5 inclusion."""
    rng = np.random.default_rng(seed)
    X1, X2, X3 = _mesh(n, h)
    L = [(int(n[j]) + 1) * h for j in range(3)]
    u1, u2, u3 = X1 / L[0], X2 / L[1], X3 / L[2]
    v = np.where(u3 <= 0.4 + 0.1 * u2, 2.0, np.where(u3 <= 0.8 - 0.2 * u2, 3.0, 4.5))
    cen = rng.uniform(0.3, 0.7, 3)
    ax = rng.uniform(0.1, 0.2, 3)
    inside = ((u1 - cen[0]) / ax[0]) ** 2 + ((u2 - cen[1]) / ax[1]) ** 2 \
        + ((u3 - cen[2]) / ax[2]) ** 2 <= 1.0
    v = np.where(inside, 4.5, v)
    return v * (1.0 + rng.uniform(-noise, noise, v.shape))


def velocity_barrier(n, h):
    """Sec. 3 barrier model: c = 1 except 1e10 in [0,1] x [0.25,0.3] x [0,0.75]."""
    X1, X2, X3 = _mesh(n, h)
    inside = (X2 >= 0.25) & (X2 <= 0.3) & (X3 <= 0.75)
    return np.where(inside, 1e10, 1.0)


def velocity_waveguide(n, h):
    """Sec. 3 waveguide model c = 1.25 (1 - 0.4 exp(-32 (|x1-.5|^2 + |x2-.5|^2)))."""
    X1, X2, X3 = _mesh(n, h)
    return 1.25 * (1.0 - 0.4 * np.exp(-32.0 * ((X1 - 0.5) ** 2 + (X2 - 0.5) ** 2)))


def velocity_wedge_paper(n, h):
    """Sec. 3 wedge model over the unit cube: c = 2 where x3 <= 0.4 + 0.1 x2,
    else 1.5 where x3 <= 0.8 - 0.2 x2, else 3."""
    X1, X2, X3 = _mesh(n, h)
    return np.where(X3 <= 0.4 + 0.1 * X2, 2.0, np.where(X3 <= 0.8 - 0.2 * X2, 1.5, 3.0))


def velocity_two_layer(n, h):
    """Sec. 3 two-layer model: c = 4 where x2 < 0.5, else 1."""
    X1, X2, X3 = _mesh(n, h)
    return np.where(X2 < 0.5, 4.0, 1.0)


# Points and direction of the four forcings of Sec. 3.
FORCING_X0 = (0.5, 0.5, 0.1)
FORCING_X1 = (0.25, 0.25, 0.1)
FORCING_X2 = (0.75, 0.75, 0.5)
FORCING_D = tuple(np.array([1.0, 1.0, -1.0]) / np.sqrt(3.0))


def paper_forcings(n, gamma, h, omega):
    """The four right-hand sides of Sec. 3 on the padded grid, zero outside
    the interior (the PML padding carries no source):
      f0 = m exp(-10 m |x - x0|^2)                  a shot,
      f1 = sum over x0, x1, x2 of the same shot     three shots,
      f2 = exp(i w x.d) exp(-4 w |x - x2|^2)        a Gaussian beam,
      f3 = exp(i w x.d)                             a plane wave,
    with m the number of interior points per axis (the largest axis).
    Returns (4, N3, N2, N1) complex128."""
    X1, X2, X3 = padded_coords(n, gamma, h)
    g = int(gamma)
    inside = np.zeros(X1.shape, dtype=bool)
    inside[g:g + int(n[2]), g:g + int(n[1]), g:g + int(n[0])] = True
    m = float(max(int(v) for v in n))

    def r2(p):
        return (X1 - p[0]) ** 2 + (X2 - p[1]) ** 2 + (X3 - p[2]) ** 2

    def shot(p):
        return m * np.exp(-10.0 * m * r2(p))

    phase = np.exp(1j * omega * (X1 * FORCING_D[0] + X2 * FORCING_D[1] + X3 * FORCING_D[2]))
    f = [shot(FORCING_X0), shot(FORCING_X0) + shot(FORCING_X1) + shot(FORCING_X2),
         phase * np.exp(-4.0 * omega * r2(FORCING_X2)), phase]
    return np.stack([np.where(inside, v, 0.0).astype(np.complex128) for v in f])


def padded_coords(n, gamma, h):
    """Coordinates of the padded nodes (x_j = (a_j - gamma + 1) h), numpy shape (N3, N2, N1)."""
    g = int(gamma)
    a = [(np.arange(int(n[j]) + 2 * g) - g + 1) * h for j in range(3)]
    X3, X2, X1 = np.meshgrid(a[2], a[1], a[0], indexing="ij")
    return X1, X2, X3


def gaussian_sources(n, gamma, h, centers_frac, sigma_h=2.0):
    """Gaussian point sources exp(-|x - x_s|^2 / (2 sigma^2)), sigma = sigma_h h.

    centers_frac: (nrhs, 3) positions as fractions of each axis extent
    (n_j + 1) h.  Returns (nrhs, N3, N2, N1) complex128 on the padded grid.
    """
    X1, X2, X3 = padded_coords(n, gamma, h)
    L = [(int(n[j]) + 1) * h for j in range(3)]
    sig = sigma_h * h
    out = []
    for cf in np.atleast_2d(centers_frac):
        xs = [cf[j] * L[j] for j in range(3)]
        r2 = (X1 - xs[0]) ** 2 + (X2 - xs[1]) ** 2 + (X3 - xs[2]) ** 2
        out.append(np.exp(-r2 / (2.0 * sig * sig)).astype(np.complex128))
    return np.stack(out)


def surface_centers(nrhs, seed, depth=0.1):
    """Shot positions at depth x3 = 0.1 (Sec. 3), (x1, x2) ~ U[0.1, 0.9]^2."""
    rng = np.random.default_rng(seed)
    xy = rng.uniform(0.1, 0.9, (nrhs, 2))
    return np.column_stack([xy, np.full(nrhs, depth)])


def random_complex(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def make_problem(name, scale_n=None, sub=0):
    """Inputs of one workload (a key of WORKLOADS).  Returns a dict with the
    velocity and parameters.

    scale_n overrides the interior size (reduced variants for parity tests
    keep everything else); sub selects one problem of the batch workload.
    """
    spec = WORKLOADS[name]
    n = spec["n"]
    if n is None:
        rng = np.random.default_rng(seed_for(spec["seed"], sub))
        n = tuple(int(v) for v in rng.integers(30, 71, 3))
    if scale_n is not None:
        n = tuple(int(v) for v in scale_n)
    h = grid_h(n)
    seed = seed_for(spec["seed"], sub)
    c = {"constant": lambda: velocity_constant(n), "grf": lambda: velocity_grf(n, h, seed),
         "layered": lambda: velocity_layered(n, h, seed),
         "wedge_salt": lambda: velocity_wedge_salt(n, h, seed),
         "barrier": lambda: velocity_barrier(n, h), "wedge_paper": lambda: velocity_wedge_paper(n, h),
         "two_layer": lambda: velocity_two_layer(n, h),
         "waveguide": lambda: velocity_waveguide(n, h)}[spec["model"]]()
    if spec["src"] == "centre":
        centers = np.array([[0.5, 0.5, 0.5]])
    elif spec["src"] == "paper":
        centers = None  # the four forcings of Sec. 3 (sources())
    else:
        centers = surface_centers(spec["nrhs"], seed + 7)
    return dict(name=name, n=n, h=h, c=c, omega=omega_for_ppw(c, h), alpha=ALPHA_DEFAULT,
                gamma=spec["gamma"], C=spec["C"], d=spec["d"], leaf=spec["leaf"],
                centers=centers, src=spec["src"], nrhs=spec["nrhs"] if centers is None else len(centers))


def sources(P):
    """Right-hand sides of a workload made by make_problem: (nrhs, N_pad) complex128."""
    if P["src"] == "paper":
        f = paper_forcings(P["n"], P["gamma"], P["h"], P["omega"])
    else:
        f = gaussian_sources(P["n"], P["gamma"], P["h"], P["centers"])
    return f.reshape(f.shape[0], -1)
