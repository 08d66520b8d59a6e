"""Pins of the oracle's heterogeneous sea (Sec. III eq. 1, 2) and Choppy Wave
Model displacement.

The tiling is checked against what the paper states of it: each TL corner
carries exactly its own T2L field (unit weight there, zero elsewhere), the
squared weights of the four fields add to one at every point (energy kept),
so a uniform sea state keeps its height variance everywhere, including tile
centres; the generator is chunk invariant.  The CWM displacement against the
trochoid closed form of one component (Eulerian mean level -k A^2 / 2,
horizontal excursion A) and against the Lagrangian kinematics (displacement
rate = the orbital velocity the facets carry).
"""
import math
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
import oracle as O

KEYS = ("z", "vx", "vy", "vz")


def node_field(sea, q, cwm=None):
    """Mode-1 sea made of node q's own homogeneous field."""
    return replace(sea, mode=1, hs=float(sea.node_hs[q]), dirs=sea.node_dirs[q],
                   phases=sea.node_phases[q], cwm=sea.cwm if cwm is None else cwm)


def vec(f, i):
    return np.array([f[k][i] for k in KEYS])


def small_hetero(seed=3, cwm=True):
    # 121 x 121 points at 5 m, tiles of 150 m: nodes fall on grid points
    return W.hetero_sea(121, 121, 5.0, seed, 150.0, cwm=cwm)


def test_corner_nodes_carry_their_own_field():
    sea = small_hetero()
    f = O.generate_facets(sea, 3)
    n1 = sea.ntx + 1
    X = (np.arange(121) - 60) * 5.0
    for q in (0, 7, 12, 24):
        i, j = q % n1, q // n1
        ix = int(np.argmin(np.abs(X - (sea.tile_x0 + i * sea.tile_L))))
        iy = int(np.argmin(np.abs(X - (sea.tile_y0 + j * sea.tile_L))))
        assert abs(X[ix] - (sea.tile_x0 + i * sea.tile_L)) < 1e-9
        g = O.generate_facets(node_field(sea, q), 3)
        p = iy * 121 + ix
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            assert abs(f[k][p] - g[k][p]) < 1e-12, (q, k)


def test_squared_weights_sum_to_one():
    """With one node's height set and the others zero, the field at a point
    is W_q times that node's own field; the four W_q of a tile are >= 0 and
    their squares add to 1 (eq. 2's energy condition)."""
    sea = small_hetero(cwm=False)
    n1 = sea.ntx + 1
    # points inside tile (1, 2): all four of its corners contribute
    corners = [2 * n1 + 1, 2 * n1 + 2, 3 * n1 + 1, 3 * n1 + 2]
    pts = [iy * 121 + ix for ix, iy in ((32, 62), (35, 70), (40, 80), (47, 89), (33, 88))]
    W2 = np.zeros(len(pts))
    for q in corners:
        hs = np.zeros_like(sea.node_hs)
        hs[q] = sea.node_hs[q]
        only = replace(sea, node_hs=hs)
        f = O.generate_facets(only, 3)
        g = O.generate_facets(node_field(sea, q), 3)
        for n, p in enumerate(pts):
            a, b = vec(f, p), vec(g, p)
            Wq = float(a @ b / (b @ b))
            assert Wq >= -1e-12
            assert np.allclose(a, Wq * b, atol=1e-12 * max(1.0, np.abs(b).max()))
            W2[n] += Wq * Wq
    assert np.max(np.abs(W2 - 1.0)) < 1e-10, W2


def test_uniform_sea_state_keeps_height_variance():
    """Uniform Hs: the variance of the height at tile centres (four fields of
    weight 1/2) equals that at the nodes, (Hs/4)^2; weights that are not
    square-root (e.g. 1/4 each) would give a quarter of it there."""
    hs = 2.0
    zc, zn = [], []
    for seed in range(6):
        sea = W.hetero_sea(241, 241, 10.0, seed, 100.0, hs_range=(hs, hs), turn_deg=0.0,
                           cwm=False)
        f = O.generate_facets(sea, seed)
        X = (np.arange(241) - 120) * 10.0
        z = f["z"].reshape(241, 241)
        off = (X - sea.tile_x0) / sea.tile_L
        cen = np.nonzero(np.abs(off - np.floor(off) - 0.5) < 1e-9)[0]
        nod = np.nonzero(np.abs(off - np.round(off)) < 1e-9)[0]
        zc.append(z[np.ix_(cen, cen)].ravel())
        zn.append(z[np.ix_(nod, nod)].ravel())
    vc, vn = np.var(np.concatenate(zc)), np.var(np.concatenate(zn))
    want = (hs / 4.0) ** 2
    assert abs(vc / want - 1.0) < 0.15, (vc, want)
    assert abs(vn / want - 1.0) < 0.15, (vn, want)


def test_chunk_invariance():
    sea = small_hetero()
    full = O.generate_facets(sea, 9)
    part = O.generate_facets(sea, 9, 17, 30, 50, 40)
    X = full["x"].reshape(121, 121)
    for k in full:
        np.testing.assert_array_equal(part[k].reshape(40, 50),
                                      full[k].reshape(121, 121)[30:70, 17:67])
    assert X.shape == (121, 121)


def one_component(cwm=True, phase=0.3):
    lam = 50.0
    k = 2 * math.pi / lam
    return W.Sea(nx=1001, ny=1, dx=lam / 1000, dy=1.0, mode=1, n_comp=1, k_min=k, k_max=k,
                 hs=4.0, dirs=np.array([0.0]), phases=np.array([phase]), cwm=cwm), k


def test_cwm_trochoid_of_one_component():
    """One component: x = X - A sin(theta), z = A cos(theta) (a trochoid);
    its Eulerian mean level over a wavelength is -k A^2 / 2 and the largest
    horizontal excursion is A (A = Hs sqrt(2) / 4)."""
    sea, k = one_component()
    f = O.generate_facets(sea, 1)
    A = 4.0 * math.sqrt(2.0) / 4.0
    X = (np.arange(1001) - 500) * sea.dx
    assert abs(np.max(np.abs(f["x"] - X)) - A) < 1e-4
    x, z = f["x"], f["z"]
    mean = np.sum(0.5 * (z[1:] + z[:-1]) * np.diff(x)) / (x[-1] - x[0])
    assert abs(mean - (-k * A * A / 2)) < 1e-5 * A, (mean, -k * A * A / 2)
    # without the CWM the facets stay on the grid and the mean level is 0
    g = O.generate_facets(one_component(cwm=False)[0], 1)
    np.testing.assert_array_equal(g["x"], X)
    assert abs(np.sum(0.5 * (g["z"][1:] + g["z"][:-1]) * np.diff(g["x"])) / 50.0) < 1e-5


def test_cwm_displacement_rate_is_the_facet_velocity():
    """Advancing every component's phase by -omega dt moves each facet by
    V dt to first order (the facets follow the orbital motion they carry)."""
    sea = W.wave_sea(60, 60, 3.0, seed=4)
    sea = replace(sea, cwm=True)
    _, _, om = O.wave_table(sea)
    dt = 1e-4
    f0 = O.generate_facets(sea, 4)
    f1 = O.generate_facets(replace(sea, phases=sea.phases - om * dt), 4)
    for a, b in (("x", "vx"), ("y", "vy"), ("z", "vz")):
        rate = (f1[a] - f0[a]) / dt
        assert np.max(np.abs(rate - f0[b])) < 2e-3 * np.max(np.abs(f0[b])), a
