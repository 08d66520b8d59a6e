"""Pins of the oracle's intra-facet speckle (Sec. III.A eq. 7, 9, 10).

The construction (anchors every 64 pulses, eq. 10 pulse by pulse inside a
group, conditioned on the next anchor) is checked against the law eq. 10
defines: being linear in its draws, its exact covariance is obtained by
feeding unit draws and must equal b^|p - q| (the stationary AR(1)
autocorrelation exp(-|t| / tau_s)) to rounding, whatever b.  The draws are
checked statistically (Philox2x32-10 bit patterns are parity unpinned: no
known-answer vectors are available offline), the Doppler factor of eq. 7
against a closed form on a lone facet, and the speckle-carrying forward and
adjoint by linearity, a dot-product test and finite differences.
"""
import math

import numpy as np
import pytest
from scipy import stats

import workloads as W
import oracle as O


def exact_covariance(a, n_groups):
    """Covariance E[x(p) conj x(q)] of the construction over 64 n_groups
    pulses, from its linear map applied to unit draws (real unit vectors:
    the map has real coefficients and the draws are CN(0, 1))."""
    G = n_groups
    cols = []
    # anchor draws eta_0 .. eta_G
    for j in range(G + 1):
        eta = np.zeros(G + 1, complex)
        eta[j] = 1.0
        y = O.speckle_anchors(a, eta)
        cols.append(O.speckle_groups(a, 0, G, y, np.zeros(64 * G, complex)).real)
    # innovations e_1 .. e_{64 G}
    y0 = O.speckle_anchors(a, np.zeros(G + 1, complex))
    for j in range(64 * G):
        e = np.zeros(64 * G, complex)
        e[j] = 1.0
        cols.append(O.speckle_groups(a, 0, G, y0, e).real)
    M = np.stack(cols, 1)
    return M @ M.T


@pytest.mark.parametrize("a", [1.0 / 34.0, 0.004, 0.3, 2.0])
def test_construction_has_the_ar1_law(a):
    cov = exact_covariance(a, 3)
    p = np.arange(cov.shape[0])
    want = np.exp(-a * np.abs(p[:, None] - p[None, :]))
    assert np.max(np.abs(cov - want)) < 1e-12


def test_frozen_and_white_limits():
    # tau_s -> inf: x is one constant draw for all pulses
    cov = exact_covariance(0.0, 2)
    assert np.max(np.abs(cov - 1.0)) < 1e-12
    x = O.speckle_series(3, 17, 0.0, 0, 200)
    assert np.max(np.abs(x - x[0])) < 1e-15
    assert x[0] == O.speckle_draw(3, 17, 2 ** 31)      # the anchor y_0 = eta_0
    # tau_s -> 0: every pulse is its own draw (anchor at group starts)
    x = O.speckle_series(3, 17, 800.0, 0, 130)
    assert x[0] == O.speckle_draw(3, 17, 2 ** 31)
    assert abs(x[64] - O.speckle_draw(3, 17, 2 ** 31 + 1)) < 1e-15
    for p in (1, 5, 63, 65, 129):
        assert abs(x[p] - O.speckle_draw(3, 17, p)) < 1e-15


def test_series_is_independent_of_the_requested_range():
    a = 1.0 / 34.0
    full = O.speckle_series(9, 123456, a, 0, 700)
    for pa, pb in ((0, 1), (63, 64), (64, 65), (100, 250), (127, 129), (640, 700)):
        np.testing.assert_array_equal(O.speckle_series(9, 123456, a, pa, pb), full[pa:pb])


def test_draw_statistics():
    e = np.array([O.speckle_draw(5, i, s) for i in range(400) for s in (1, 2, 77, 2 ** 31)])
    # |e|^2 = -ln u1 is Exp(1); the angle is uniform; real and imaginary
    # parts are N(0, 1/2) each and uncorrelated
    assert stats.kstest(np.abs(e) ** 2, "expon").pvalue > 1e-4
    assert stats.kstest((np.angle(e) / (2 * np.pi)) % 1.0, "uniform").pvalue > 1e-4
    assert stats.kstest(e.real * np.sqrt(2.0), "norm").pvalue > 1e-4
    assert stats.kstest(e.imag * np.sqrt(2.0), "norm").pvalue > 1e-4
    assert abs(np.mean(e.real * e.imag)) < 4 * 0.5 / np.sqrt(e.size)
    # different slots and ids are different draws
    assert O.speckle_draw(5, 1, 2) != O.speckle_draw(5, 1, 3)
    assert O.speckle_draw(5, 1, 2) != O.speckle_draw(5, 2, 2)
    assert O.speckle_draw(5, 1, 2) != O.speckle_draw(6, 1, 2)
    # avalanche of the two-word generator
    flips = []
    for b in range(32):
        a0 = O.philox2x32_10([12345, 678], 99)
        a1 = O.philox2x32_10([12345 ^ (1 << b), 678], 99)
        flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a0, a1)))
    assert 26 < np.mean(flips) < 38


def test_empirical_autocorrelation_eq9():
    """E[s(t0) conj s(t0 + k dt)] over many facets = b^|k| exp(-2 pi j f_s k dt)
    (eq. 9 with the exponential form of eq. 10), across a group boundary."""
    a = 1.0 / 34.0
    dt = 1.0 / W.PRF
    fs = 5.7
    xs = np.array([O.speckle_series(2, i, a, 40, 110) for i in range(3000)])
    t = (np.arange(40, 110) - 0.0) * dt
    s = xs * np.exp(2j * np.pi * fs * t)[None, :]
    for p, k in ((0, 0), (20, 5), (10, 30), (23, 1), (0, 60)):
        r = np.mean(s[:, p] * np.conj(s[:, p + k]))
        want = np.exp(-a * k) * np.exp(-2j * np.pi * fs * k * dt)
        assert abs(r - want) < 5.0 / np.sqrt(xs.shape[0]), (p, k, r, want)


def lone_facet():
    return dict(x=np.array([3.0]), y=np.array([-2.0]), z=np.array([0.4]),
                vx=np.array([0.3]), vy=np.array([-0.2]), vz=np.array([0.1]),
                a_re=np.array([0.8]), a_im=np.array([-0.6]))


def test_lone_facet_speckle_factor_closed_form():
    """Frozen speckle (tau_s = inf) and Doppler f_s: every row of a lone
    facet is its speckle-free row times x(0) exp(j 2 pi f_s t_p)."""
    g = W.harmony_geometry(40, 128)
    f = lone_facet()
    sp = W.Speckle(tau_s=math.inf, seed=4, first_index=1000)
    fs = np.array([3.25])
    base = O.forward(g, f, 3, 30)
    got = O.forward(g, f, 3, 30, speckle=sp, f_s=fs)
    x0 = O.speckle_draw(4, 1000, 2 ** 31)
    t = np.array([O.pulse_time(g, p) for p in range(3, 33)])
    want = base * (x0 * np.exp(2j * np.pi * fs[0] * t))[None, :, None]
    # the Doppler phase joins the ~1.9e8 rad carrier phase before its sine and
    # cosine are taken, so agreement is at that phase's FP64 rounding (~3e-8)
    assert O.rel_l2(got, want) < 1e-7
    # with a finite tau_s each row is scaled by that pulse's x(p)
    sp2 = W.Speckle(tau_s=0.01, seed=4, first_index=1000)
    got2 = O.forward(g, f, 3, 30, speckle=sp2)
    xp = O.speckle_series(4, 1000, 1.0 / (W.PRF * 0.01), 3, 33)
    assert O.rel_l2(got2, base * xp[None, :, None]) < 1e-13


def test_speckle_forward_linearity_and_ids():
    g = W.harmony_geometry(24, 128, receivers="AB")
    f = {k: v.astype(np.float64) for k, v in W.scattered_facets(30, 50.0, 6).items()}
    sp = W.Speckle(tau_s=0.02, seed=8, first_index=500)
    fs = W.speckle_doppler(30, 8).astype(np.float64)
    full = O.forward(g, f, 0, 24, speckle=sp, f_s=fs)
    # split into two sets that keep their ids (first_index of the second part)
    f1 = {k: v[:12] for k, v in f.items()}
    f2 = {k: v[12:] for k, v in f.items()}
    part = (O.forward(g, f1, 0, 24, speckle=sp, f_s=fs[:12]) +
            O.forward(g, f2, 0, 24, speckle=W.Speckle(0.02, 8, 512), f_s=fs[12:]))
    assert O.rel_l2(part, full) < 1e-13
    # a different seed changes the result, the plain forward differs
    other = O.forward(g, f, 0, 24, speckle=W.Speckle(0.02, 9, 500), f_s=fs)
    assert O.rel_l2(other, full) > 0.1
    assert O.rel_l2(O.forward(g, f, 0, 24), full) > 0.1
    # pulse sub-ranges are row slices (the speckle is drawn on absolute pulses)
    sub = O.forward(g, f, 5, 13, speckle=sp, f_s=fs)
    assert O.rel_l2(sub, full[:, 5:18]) < 1e-13


def _speckle_problem(seed=21, n=10):
    g = W.harmony_geometry(20, 128, receivers="AB")
    f = {k: v.astype(np.float64) for k, v in W.scattered_facets(n, 40.0, seed).items()}
    sp = W.Speckle(tau_s=0.015, seed=seed, first_index=77)
    fs = W.speckle_doppler(n, seed).astype(np.float64)
    ft = {k: v.astype(np.float64) for k, v in W.scattered_facets(n, 40.0, seed + 1).items()}
    target = O.forward(g, ft, speckle=sp, f_s=fs)
    return g, f, sp, fs, target


def test_speckle_adjoint_dot_product_amplitude():
    g, f, sp, fs, _ = _speckle_problem()
    rng = np.random.default_rng(3)
    gi = rng.standard_normal((g.n_channels, 20, 128)) + \
        1j * rng.standard_normal((g.n_channels, 20, 128))
    da = rng.standard_normal(10) + 1j * rng.standard_normal(10)
    f0 = dict(f)
    f0["a_re"], f0["a_im"] = da.real.copy(), da.imag.copy()
    Ada = O.forward(g, f0, speckle=sp, f_s=fs)
    lhs = np.sum(gi.real * Ada.real + gi.imag * Ada.imag)
    gr = O.adjoint(g, f, gi, speckle=sp, f_s=fs)
    rhs = np.sum(gr["a_re"] * da.real + gr["a_im"] * da.imag)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


@pytest.mark.parametrize("key", ["z", "vx", "vz", "a_im"])
def test_speckle_adjoint_vs_richardson_fd(key):
    g, f, sp, fs, target = _speckle_problem()
    resid = O.forward(g, f, speckle=sp, f_s=fs) - target
    gr = O.adjoint(g, f, 2.0 * resid, speckle=sp, f_s=fs)
    h = {"z": 2e-4, "vx": 0.2, "vz": 0.05, "a_im": 1e-3}[key]
    for i in (0, 4, 9):
        d1 = O.fd_gradient(g, f, target, i, key, h, resid=resid, speckle=sp, f_s=fs)
        d2 = O.fd_gradient(g, f, target, i, key, h / 2, resid=resid, speckle=sp, f_s=fs)
        rich = (4 * d2 - d1) / 3
        scale = max(abs(gr[key][i]), 1e-6 * np.abs(gr[key]).max())
        tol = 1e-4 if key.startswith("v") else 1e-5
        assert abs(rich - gr[key][i]) < tol * scale + 1e-9, (i, rich, gr[key][i])


def test_grid_index_ids_make_chunking_invisible():
    """A generated scene split into unequal chunks, each facet taking the id
    first_index + (grid index) and the Doppler at that index, gives the
    speckle sum of the whole scene (the streamed entry points' rule): ids
    that restarted per chunk would not."""
    g = W.harmony_geometry(96, 512)
    sea = W.wave_sea(40, 30, 1.0, seed=2)
    sp = W.Speckle(tau_s=0.02, seed=7, first_index=500)
    fs_grid = W.speckle_doppler(sea.nx * sea.ny, 7).astype(np.float64)
    whole = O.generate_facets(sea, 2)
    ref = O.forward(g, whole, 10, 70, speckle=sp, f_s=fs_grid)
    chunks = [(0, 0, 25, 12), (25, 0, 15, 12), (0, 12, 40, 18)]
    parts = [O.generate_facets(sea, 2, *c) for c in chunks]
    f = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    gi = np.concatenate([(c[1] + np.arange(c[2] * c[3]) // c[2]) * sea.nx + c[0] +
                         np.arange(c[2] * c[3]) % c[2] for c in chunks])
    got = O.forward(g, f, 10, 70, speckle=sp, f_s=fs_grid[gi],
                    ids=(sp.first_index + gi) & 0xFFFFFFFF)
    assert O.rel_l2(got, ref) < 1e-13
    # per-chunk ids (each chunk from first_index) change the speckle
    bad_ids = np.concatenate([sp.first_index + np.arange(c[2] * c[3]) for c in chunks])
    bad = O.forward(g, f, 10, 70, speckle=sp, f_s=fs_grid[gi], ids=bad_ids & 0xFFFFFFFF)
    assert O.rel_l2(bad, ref) > 0.1
