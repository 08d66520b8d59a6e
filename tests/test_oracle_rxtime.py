"""Pins of the oracle's per-facet reception time (eq. 3 evaluates r_r at the
facet's own reception time t_r; the default reading takes the receiver at
the scene origin's echo time of each pulse).

The echo delay is checked against a 50-digit mpmath root of its defining
equation, written here from the platform trajectories; the forward against
that delay (the phase and sample shift of a lone facet relative to the
per-pulse receiver model) and against the static-receiver special case; the
adjoint's implicit-function gradient against Richardson finite differences.
"""
from dataclasses import replace

import mpmath as mp
import numpy as np
import pytest

import workloads as W
import oracle as O

mp.mp.dps = 50


def exact(g):
    return replace(g, rx_exact=True)


def mp_echo(g, ch, p, X):
    """Root of c tau = |X - P_tx(t_p)| + |X - P_rx(t_p + tau)| in 50 digits."""
    t = (mp.mpf(p) - mp.mpf(g.n_pulses - 1) / 2) / mp.mpf(g.prf)
    chan = g.channels[ch]
    tx = g.platforms[g.antennas[chan.tx].platform]
    rx = g.platforms[g.antennas[chan.rx].platform]
    Xm = [mp.mpf(float(v)) for v in X]

    def pos(pl, tt, off=(0.0, 0.0, 0.0)):
        return [mp.mpf(pl.p0[k]) + mp.mpf(pl.v[k]) * tt + mp.mpf(off[k]) for k in range(3)]

    def dist(a, b):
        return mp.sqrt(sum((a[k] - b[k]) ** 2 for k in range(3)))

    pt = pos(tx, t)
    c = mp.mpf(g.c)
    f = lambda tau: c * tau - dist(Xm, pt) - dist(Xm, pos(rx, t + tau, chan.pc_offset))
    return mp.findroot(f, mp.mpf("0.0057"))


@pytest.mark.parametrize("X", [(0.0, 0.0, 0.0), (250.0, -310.0, 1.5), (-480.0, 520.0, -2.0)])
def test_echo_time_matches_mpmath_root(X):
    g = W.harmony_geometry(64, 128, receivers="AB", n_pc=3)
    for ch, p in ((0, 0), (3, 40), (5, 63)):
        tau = O.echo_time(g, ch, p, X)
        ref = mp_echo(g, ch, p, X)
        assert abs(tau - float(ref)) < 4e-18, (ch, p, tau, float(ref))


def test_static_receiver_is_the_per_pulse_model():
    g = W.harmony_geometry(12, 128)
    plats = tuple(replace(p, v=(0.0, 0.0, 0.0)) for p in g.platforms)
    g = replace(g, platforms=plats)
    f = {k: v.astype(np.float64) for k, v in W.scattered_facets(40, 200.0, 5).items()}
    a = O.forward(g, f)
    b = O.forward(exact(g), f)
    assert O.rel_l2(b, a) < 1e-15


def test_lone_facet_phase_and_delay_shift():
    """Rows of a lone static facet: with the exact reception time the peak
    sample carries the phase -2 pi f0 tau_e instead of -2 pi f0 tau_p (tau_p:
    receiver at the origin's echo time), the taps shifted by (tau_e - tau_p) fs."""
    g = W.harmony_geometry(8, 256)
    X = (180.0, -420.0, 0.7)
    f = dict(x=np.array([X[0]]), y=np.array([X[1]]), z=np.array([X[2]]),
             vx=np.zeros(1), vy=np.zeros(1), vz=np.zeros(1),
             a_re=np.ones(1), a_im=np.zeros(1))
    plain = O.forward(g, f)[0]
    ex = O.forward(exact(g), f)[0]
    for p in (0, 5):
        t, ptx, prx, tau_ref = O.pulse_geometry(g, 0, p)
        Xm = [mp.mpf(v) for v in X]
        tau_p = (mp.sqrt(sum((Xm[k] - mp.mpf(ptx[k])) ** 2 for k in range(3))) +
                 mp.sqrt(sum((Xm[k] - mp.mpf(prx[k])) ** 2 for k in range(3)))) / mp.mpf(g.c)
        tau_e = mp_echo(g, 0, p, X)
        dphi = float(-2 * mp.pi * mp.mpf(g.f0) * (tau_e - tau_p))
        assert abs(dphi) > 0.05            # the effect is far above the 1e-4 target
        n = int(np.abs(plain[p]).argmax())
        # the ratio of the two rows at the peak: phase from the delay change,
        # modulus from the tap shift and the receiver-gain change (~1e-8)
        u_p = g.ref_sample + float((tau_p - mp.mpf(tau_ref)) * mp.mpf(g.fs))
        u_e = g.ref_sample + float((tau_e - mp.mpf(tau_ref)) * mp.mpf(g.fs))
        ratio = ex[p, n] / plain[p, n]
        tap_ratio = O.tap(n - u_e, g.kaiser_beta) / O.tap(n - u_p, g.kaiser_beta)
        d = np.angle(ratio * np.exp(-1j * dphi))
        assert abs(d) < 2e-7, (p, d)
        assert abs(abs(ratio) / abs(tap_ratio) - 1.0) < 1e-6


def test_exact_time_adjoint_vs_richardson_fd():
    g = exact(W.harmony_geometry(16, 128, receivers="AB"))
    f = {k: v.astype(np.float64) for k, v in W.scattered_facets(10, 40.0, 33).items()}
    target = O.forward(g, {k: v.astype(np.float64)
                           for k, v in W.scattered_facets(10, 40.0, 34).items()})
    resid = O.forward(g, f) - target
    gr = O.adjoint(g, f, 2.0 * resid)
    # The implicit factor 1 / (1 + u_r.V_rx/c) moves grad R by ~1e-5; the
    # height derivative's finite differences agree to ~4e-7, so a 2e-6 bar
    # on it resolves that factor.
    for key, h in (("z", 2e-4), ("vx", 0.2), ("vy", 0.2), ("a_re", 1e-3)):
        for i in (0, 3, 6, 9):
            d1 = O.fd_gradient(g, f, target, i, key, h, resid=resid)
            d2 = O.fd_gradient(g, f, target, i, key, h / 2, resid=resid)
            rich = (4 * d2 - d1) / 3
            scale = max(abs(gr[key][i]), 1e-6 * np.abs(gr[key]).max())
            tol = {"z": 2e-6, "a_re": 1e-5}.get(key, 1e-4)
            assert abs(rich - gr[key][i]) < tol * scale + 1e-9, (key, i, rich, gr[key][i])
