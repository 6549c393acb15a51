"""Host checks of the seeded inputs of Sec. 3 and of the PML study's selection rule.

The analytic models and the four forcings are checked against their
definitions at hand-picked points (a wrong threshold, axis or sign moves one
of them), and the forcings against properties fixed by their formulas: the
shot's peak value and width, the plane wave's unit modulus and phase step,
the beam's centre, and zero values in the PML padding.
"""

import ast
import os

import numpy as np
import pytest

from paper_1204_0111_amd import studies
from paper_1204_0111_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _at(c, n, h, x):
    """Value of a (N3, N2, N1) interior array at the node nearest x."""
    i = [int(round(x[j] / h)) - 1 for j in range(3)]
    return c[i[2], i[1], i[0]]


def test_wedge_layers_at_sample_points():
    n = (39, 39, 39)
    h = wl.grid_h(n)
    c = wl.velocity_wedge_paper(n, h)
    assert _at(c, n, h, (0.5, 0.0 + h, 0.3)) == 2.0      # below 0.4 + 0.1 x2
    assert _at(c, n, h, (0.5, 0.9, 0.475)) == 2.0        # 0.4 + 0.09 = 0.49 > 0.475
    assert _at(c, n, h, (0.5, 0.9, 0.55)) == 1.5         # between the two planes
    assert _at(c, n, h, (0.5, 0.1, 0.775)) == 1.5        # 0.8 - 0.02 = 0.78 > 0.775
    assert _at(c, n, h, (0.5, 0.9, 0.65)) == 3.0         # 0.8 - 0.18 = 0.62 < 0.65
    assert _at(c, n, h, (0.1, 0.5, 0.95)) == 3.0
    assert set(np.unique(c)) == {1.5, 2.0, 3.0}
    # invariant along x1
    assert np.array_equal(c, np.broadcast_to(c[:, :, :1], c.shape))


def test_two_layer_and_barrier_and_waveguide():
    n = (19, 19, 19)
    h = wl.grid_h(n)
    c = wl.velocity_two_layer(n, h)
    assert _at(c, n, h, (0.5, 0.45, 0.5)) == 4.0 and _at(c, n, h, (0.5, 0.55, 0.5)) == 1.0
    b = wl.velocity_barrier(n, h)
    assert _at(b, n, h, (0.5, 0.25, 0.5)) == 1e10 and _at(b, n, h, (0.5, 0.2, 0.5)) == 1.0
    assert _at(b, n, h, (0.5, 0.25, 0.8)) == 1.0   # the slab ends at x3 = 0.75
    g = wl.velocity_waveguide(n, h)
    assert abs(_at(g, n, h, (0.5, 0.5, 0.1)) - 1.25 * 0.6) < 1e-12
    r2 = (0.1 - 0.5) ** 2 + (0.2 - 0.5) ** 2
    assert abs(_at(g, n, h, (0.1, 0.2, 0.9)) - 1.25 * (1 - 0.4 * np.exp(-32 * r2))) < 1e-12


def test_forcings_match_their_definitions():
    n, gamma = (39, 39, 39), 3
    h = wl.grid_h(n)
    omega = 7.0
    f = wl.paper_forcings(n, gamma, h, omega)
    N = [v + 2 * gamma for v in n]
    assert f.shape == (4, N[2], N[1], N[0])
    g = gamma
    inner = (slice(g, g + n[2]), slice(g, g + n[1]), slice(g, g + n[0]))
    pad = np.ones(f.shape[1:], dtype=bool)
    pad[inner] = False
    assert np.all(f[:, pad] == 0)
    X1, X2, X3 = wl.padded_coords(n, gamma, h)

    def idx(x):
        return (int(round(x[2] / h)) - 1 + g, int(round(x[1] / h)) - 1 + g,
                int(round(x[0] / h)) - 1 + g)

    # f0: height m at x0 (x0 = (0.5, 0.5, 0.1) is a node of the 39^3 grid with
    # h = 1/40), and m exp(-10 m r^2) one node away along x1
    m = 39.0
    i0 = idx((0.5, 0.5, 0.1))
    assert abs(X1[i0] - 0.5) < 1e-12 and abs(X3[i0] - 0.1) < 1e-12
    assert abs(f[0][i0] - m) < 1e-12
    i1 = (i0[0], i0[1], i0[2] + 1)
    assert abs(f[0][i1] - m * np.exp(-10 * m * h * h)) < 1e-12
    # f1 = three shots: at x1 = (0.25, 0.25, 0.1) the value is the shot's peak
    # plus the others' (negligible) tails
    assert abs(f[1][idx((0.25, 0.25, 0.1))] - m) < 1e-9
    assert abs(f[1][idx((0.75, 0.75, 0.5))] - m) < 1e-9
    # f3: unit modulus, phase step exp(i w h d1) along x1
    ins = f[3][inner]
    assert np.allclose(np.abs(ins), 1.0, atol=1e-14)
    d1 = 1 / np.sqrt(3.0)
    assert np.allclose(ins[:, :, 1:] / ins[:, :, :-1], np.exp(1j * omega * h * d1), atol=1e-12)
    assert np.allclose(ins[1:, :, :] / ins[:-1, :, :], np.exp(-1j * omega * h * d1), atol=1e-12)
    # f2: the plane wave times a Gaussian exp(-4 w r^2) about x2
    i2 = idx((0.75, 0.75, 0.5))
    assert abs(abs(f[2][i2]) - 1.0) < 1e-12
    assert abs(f[2][i2] - f[3][i2]) < 1e-12
    i3 = (i2[0] + 2, i2[1], i2[2])
    assert abs(abs(f[2][i3]) - np.exp(-4 * omega * (2 * h) ** 2)) < 1e-12


def test_paper_workloads_are_well_formed():
    for name, ppw_c in [("barrier50", 1.0), ("wedge50", 1.5), ("twolayer50", 1.0),
                        ("waveguide50", 1.25 * 0.6)]:
        P = wl.make_problem(name)
        assert P["gamma"] == 5 and P["d"] == 4 and P["nrhs"] == 4 and P["src"] == "paper"
        # ten points per wavelength of the slowest velocity
        assert abs(P["omega"] - 2 * np.pi * P["c"].min() / (10 * P["h"])) < 1e-9
        assert abs(P["c"].min() - ppw_c) < 1e-2  # the waveguide axis falls between nodes
        b = wl.sources(P)
        assert b.shape == (4, int(np.prod([v + 10 for v in P["n"]])))


def _cand(v, its, conv=True):
    return dict(value=v, iters=max(its), iters_per_rhs=its, converged=conv)


def test_study_choice_rule():
    assert studies.choose([_cand(2.0, [9, 8]), _cand(4.0, [7, 7]), _cand(8.0, [7, 9])]) == 4.0
    # equal maxima: the fewer total iterations wins, then the smaller value
    assert studies.choose([_cand(2.0, [7, 6]), _cand(4.0, [7, 5])]) == 4.0
    assert studies.choose([_cand(2.0, [7, 5]), _cand(4.0, [7, 5])]) == 2.0
    # a candidate that did not converge loses even with a smaller count
    assert studies.choose([_cand(2.0, [3, 3], conv=False), _cand(4.0, [30, 30])]) == 4.0


@pytest.mark.parametrize("mod", ["hsweep.py", "studies.py", "workloads.py", "build.py",
                                 "__init__.py"])
def test_product_modules_do_not_import_the_oracle(mod):
    tree = ast.parse(open(os.path.join(ROOT, "paper_1204_0111_amd", mod)).read())
    for node in ast.walk(tree):
        names = []
        if isinstance(node, ast.Import):
            names = [a.name for a in node.names]
        elif isinstance(node, ast.ImportFrom):
            names = [node.module or ""]
        for nm in names:
            assert not nm.split(".")[0] == "oracle", (mod, nm)
