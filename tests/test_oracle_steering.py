"""Pins of the oracle's time-dependent antenna patterns (Sec. III.B: patterns
are time dependent in the TOPSAR modes; reading: each antenna's frame turns
about its elevation axis at a constant rate).

Rotating the antenna by phi must act on a facet's gain exactly as rotating
the facet by -phi about the antenna's elevation axis through its phase
centre (Rodrigues' formula, written here), so a lone facet's steered rows
equal its unsteered rows times a gain ratio taken from the static pattern;
a zero rate is the stripmap model; the adjoint matches finite differences.
"""
from dataclasses import replace

import numpy as np

import workloads as W
import oracle as O


def rodrigues(v, k, phi):
    k = np.asarray(k, np.float64) / np.linalg.norm(k)
    return (v * np.cos(phi) + np.cross(k, v) * np.sin(phi) +
            k * np.dot(k, v) * (1.0 - np.cos(phi)))


def test_zero_rate_is_stripmap():
    g = W.harmony_geometry(20, 256, receivers="AB", n_pc=3)
    f = {k: v.astype(np.float64) for k, v in W.scattered_facets(30, 80.0, 2).items()}
    g0 = W.tops_geometry(g, 0.0)
    assert O.rel_l2(O.forward(g0, f), O.forward(g, f)) == 0.0


def test_steered_gain_is_a_rotated_facet():
    g = W.harmony_geometry(40, 256)
    gs = W.tops_geometry(g, 3.0)
    rate = gs.antennas[0].steer_rate
    X = np.array([40.0, -130.0, 0.5])
    f = dict(x=X[:1].copy(), y=X[1:2].copy(), z=X[2:].copy(), vx=np.zeros(1),
             vy=np.zeros(1), vz=np.zeros(1), a_re=np.ones(1), a_im=np.zeros(1))
    plain = O.forward(g, f)[0]
    steered = O.forward(gs, f)[0]
    _, _, el = O.antenna_frame(g, 0)
    for p in (0, 13, 39):
        t, ptx, prx, tau = O.pulse_geometry(g, 0, p)
        phi = rate * t
        Xr = ptx + rodrigues(X - ptx, el, -phi)
        ratio_want = O.gain(g, 0, ptx, Xr) / O.gain(g, 0, ptx, X)
        n = int(np.abs(plain[p]).argmax())
        ratio = steered[p, n] / plain[p, n]
        assert abs(ratio - ratio_want) < 1e-12, (p, ratio, ratio_want)
        assert abs(ratio_want - 1.0) > 1e-4 or p == 20    # the steering matters


def test_steering_turns_the_beam_forward():
    """A positive rate turns the Tx boresight towards +az: late in the burst
    the facets ahead (along-track) gain and those behind lose."""
    g = W.tops_geometry(W.harmony_geometry(200, 256), 6.0)
    ahead = dict(x=np.array([150.0]), y=np.zeros(1), z=np.zeros(1), vx=np.zeros(1),
                 vy=np.zeros(1), vz=np.zeros(1), a_re=np.ones(1), a_im=np.zeros(1))
    behind = dict(ahead, x=np.array([-150.0]))
    pa = np.abs(O.forward(g, ahead)[0]).max(axis=1)
    pb = np.abs(O.forward(g, behind)[0]).max(axis=1)
    assert pa[-1] > pa[0] and pb[-1] < pb[0]


def test_steered_adjoint_vs_richardson_fd():
    g = W.tops_geometry(W.harmony_geometry(16, 128, receivers="AB"), 20.0)
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


def test_steered_back_plane():
    """The back plane turns with the antenna: a facet just in front of the
    unsteered Tx back plane, behind it along-track, drops out once the frame
    has turned far enough (airborne geometry, whose scene reaches the plane),
    exactly when its rotated position is behind the static antenna."""
    plats = (W.Platform((0.0, -15000.0, 12000.0), (60.0, 0.0, 0.0)),
             W.Platform((400.0, -15000.0, 12000.0), (60.0, 0.0, 0.0)))
    g = W.tops_geometry(replace(W.harmony_geometry(64, 4096), platforms=plats), 60.0)
    rate = g.antennas[0].steer_rate
    b, az, el = O.antenna_frame(g, 0)
    P0 = np.array(plats[0].p0)
    x = -300.0
    # ground point on the static back plane at this x, moved 2 m in front of it
    y = P0[1] - ((x - P0[0]) * b[0] - P0[2] * b[2]) / b[1]
    X = np.array([x, y, 0.0])
    X = X + 2.0 * b / np.linalg.norm(b[:2]) * np.sign(b[1]) * np.array([0, 1, 0])
    f = dict(x=X[:1].copy(), y=X[1:2].copy(), z=np.zeros(1), vx=np.zeros(1), vy=np.zeros(1),
             vz=np.zeros(1), a_re=np.ones(1), a_im=np.zeros(1))
    rows = O.forward(g, f)[0]
    front = []
    for p in range(64):
        t, ptx, prx, tau = O.pulse_geometry(g, 0, p)
        Xr = ptx + rodrigues(X - ptx, el, -rate * t)
        front.append(float(np.dot(Xr - ptx, b)) > 0.0)
        if not front[-1]:
            assert np.abs(rows[p]).max() == 0.0, p
        else:
            assert np.abs(rows[p]).max() > 0.0, p
    assert any(front) and not all(front)
