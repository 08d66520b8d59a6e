"""Pins of the oracle's u-v gridded antenna patterns (Sec. III.B: patterns are
converted into u-v grids held in GPU memory; reading: a real field gain over
the direction cosines on the antenna's azimuth and elevation axes,
interpolated bilinearly, zero outside the table's half-open cells).

The interpolation reproduces the table at its nodes, is exact on any
bilinear function, converges to a smooth pattern at second order in the cell
size (so a grid sampled from the analytic pattern gives the analytic sum in
the limit), is zero outside the grid and behind the antenna, and its adjoint
matches finite differences.
"""
from dataclasses import replace

import numpy as np

import workloads as W
import oracle as O


def with_pattern(g, pats):
    ants = tuple(replace(a, pattern=p) for a, p in zip(g.antennas, pats))
    return replace(g, antennas=ants + g.antennas[len(ants):])


def direction_point(pa, frame, u, v, r=8.5e5):
    """The point at range r from pa whose direction cosines on (az, el) are
    (u, v), in front of the antenna."""
    b, az, el = frame
    w = np.sqrt(1.0 - u * u - v * v)
    return pa + r * (u * az + v * el + w * b)


def tx_setup(g):
    _, ptx, _, _ = O.pulse_geometry(g, 0, 0)
    return ptx, O.antenna_frame(g, 0)


def test_node_values():
    g = W.harmony_geometry(8, 256)
    pat = W.synthetic_pattern(g.antennas[0].beta_az, g.antennas[0].beta_el, seed=3,
                              nu=33, nv=17)
    gg = with_pattern(g, (pat,))
    ptx, fr = tx_setup(g)
    vals = pat.values.astype(np.float64)
    for i, j in ((1, 1), (5, 12), (16, 8), (31, 3), (20, 15)):
        u, v = pat.u0 + i * pat.du, pat.v0 + j * pat.dv
        f = O.gain(gg, 0, ptx, direction_point(ptx, fr, u, v))
        assert abs(f - vals[j, i]) < 1e-9 * max(1.0, abs(vals[j, i])), (i, j, f, vals[j, i])
        # a transposed reading of the table would give vals[i, j] (asymmetric table)
        if i < vals.shape[0] and j < vals.shape[1]:
            assert abs(vals[j, i] - vals[i, j]) > 1e-6 or i == j


def test_exact_on_bilinear_functions():
    g = W.harmony_geometry(8, 256)
    nu, nv = 21, 11
    u0, du, v0, dv = -0.02, 0.002, -0.3, 0.06
    uu = u0 + du * np.arange(nu)
    vv = v0 + dv * np.arange(nv)
    a, b, c, d = 0.7, 31.0, -1.3, 85.0
    f = lambda u, v: a + b * u + c * v + d * u * v
    vals = f(uu[None, :], vv[:, None]).astype(np.float32)
    pat = W.Pattern(u0, du, v0, dv, vals)
    gg = with_pattern(g, (pat,))
    ptx, fr = tx_setup(g)
    rng = np.random.default_rng(5)
    vd = vals.astype(np.float64)
    for _ in range(20):
        u = rng.uniform(uu[0], uu[-1])
        v = rng.uniform(vv[0], vv[-1])
        x = (u - u0) / du
        y = (v - v0) / dv
        i, j = int(x), int(y)
        fx, fy = x - i, y - j
        # the float32 table is bilinear in the cell: its own corners define it
        want = ((1 - fx) * (1 - fy) * vd[j, i] + fx * (1 - fy) * vd[j, i + 1] +
                (1 - fx) * fy * vd[j + 1, i] + fx * fy * vd[j + 1, i + 1])
        got, grad = O.gain(gg, 0, ptx, direction_point(ptx, fr, u, v), with_grad=True)
        assert abs(got - want) < 1e-9, (got, want)
        assert abs(got - f(u, v)) < 1e-6 * (1 + abs(f(u, v)))      # float32 nodes
        # dF/dX against central differences of the gain (smooth inside a cell)
        X = direction_point(ptx, fr, u, v)
        h = 0.5
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            fd = (O.gain(gg, 0, ptx, X + e) - O.gain(gg, 0, ptx, X - e)) / (2 * h)
            assert abs(fd - grad[k]) < 1e-6 * np.abs(grad).max() + 1e-12, (k, fd, grad[k])


def test_zero_outside_and_behind():
    g = W.harmony_geometry(8, 256)
    vals = np.ones((5, 9), np.float32)
    pat = W.Pattern(-0.01, 0.0025, -0.2, 0.1, vals)
    gg = with_pattern(g, (pat,))
    ptx, fr = tx_setup(g)
    inside = O.gain(gg, 0, ptx, direction_point(ptx, fr, 0.0, 0.0))
    assert inside == 1.0
    for u, v in ((-0.0101, 0.0), (0.0101, 0.0), (0.0, -0.21), (0.0, 0.21)):
        assert O.gain(gg, 0, ptx, direction_point(ptx, fr, u, v)) == 0.0, (u, v)
    # the upper edges are outside (half-open cells), the lower ones inside
    assert O.gain(gg, 0, ptx, direction_point(ptx, fr, -0.01 + 1e-12, 0.0)) == 1.0
    assert O.gain(gg, 0, ptx, direction_point(ptx, fr, 0.01 + 1e-9, 0.0)) == 0.0
    # behind the antenna: zero even where the table covers the direction cosines
    b, az, el = fr
    X = ptx - 8.5e5 * b
    assert O.gain(gg, 0, ptx, X) == 0.0


def sampled_analytic(g, ant, pa, n_u, n_v, span_u, span_v):
    """The oracle's analytic field of antenna `ant` sampled at grid nodes."""
    fr = O.antenna_frame(g, ant)
    a = g.antennas[ant]
    uu = np.linspace(-span_u * a.beta_az, span_u * a.beta_az, n_u)
    vv = np.linspace(-span_v * a.beta_el, span_v * a.beta_el, n_v)
    vals = np.array([[O.gain(g, ant, pa, direction_point(pa, fr, u, v)) for u in uu]
                     for v in vv])
    return W.Pattern(float(uu[0]), float(uu[1] - uu[0]), float(vv[0]), float(vv[1] - vv[0]),
                     vals.astype(np.float32))


def test_converges_to_the_analytic_pattern():
    """Tx and Rx grids sampled from the analytic sinc patterns: the facet sum
    with them approaches the analytic sum at second order in the cell size."""
    g = W.harmony_geometry(48, 256)
    f = {k: v.astype(np.float64) for k, v in W.scattered_facets(40, 120.0, 8).items()}
    ref = O.forward(g, f)
    _, ptx, prx, _ = O.pulse_geometry(g, 0, 0)
    errs = []
    # u cells of beta_az / 16, / 32, / 64.  The scene spans ~1e-4 in v, a
    # sliver of one v cell, where the v error is first order in the cell
    # size; a fine v grid (cells of beta_el / 320) keeps it out of the way.
    for n in (129, 257, 513):
        pt = sampled_analytic(g, 0, ptx, n, 33, 4.0, 0.05)
        pr = sampled_analytic(g, 1, prx, n, 33, 4.0, 0.05)
        errs.append(O.rel_l2(O.forward(with_pattern(g, (pt, pr)), f), ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.6 and 3.5 < r2 < 4.6, errs
    assert errs[2] < 2e-4, errs


def test_grid_adjoint_vs_richardson_fd():
    g = W.gridded_geometry(W.harmony_geometry(16, 128, receivers="AB"), seed=4)
    f = {k: v.astype(np.float64) for k, v in W.scattered_facets(10, 40.0, 41).items()}
    target = O.forward(g, {k: v.astype(np.float64)
                           for k, v in W.scattered_facets(10, 40.0, 42).items()})
    resid = O.forward(g, f) - target
    gr = O.adjoint(g, f, 2.0 * resid)
    for key, h in (("z", 2e-4), ("vx", 0.2), ("a_re", 1e-3)):
        for i in (0, 5, 9):
            d1 = O.fd_gradient(g, f, target, i, key, h, resid=resid)
            d2 = O.fd_gradient(g, f, target, i, key, h / 2, resid=resid)
            rich = (4 * d2 - d1) / 3
            scale = max(abs(gr[key][i]), 1e-6 * np.abs(gr[key]).max())
            tol = 1e-4 if key.startswith("v") else 1e-5
            assert abs(rich - gr[key][i]) < tol * scale + 1e-9, (key, i, rich, gr[key][i])


def test_gridded_sum_differs_from_analytic():
    """The synthetic grids change the sum (the pattern path is really taken)."""
    g = W.harmony_geometry(32, 256)
    gg = W.gridded_geometry(g, seed=1)
    f = {k: v.astype(np.float64) for k, v in W.scattered_facets(30, 80.0, 2).items()}
    assert O.rel_l2(O.forward(gg, f), O.forward(g, f)) > 1e-2
