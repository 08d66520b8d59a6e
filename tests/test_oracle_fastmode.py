"""Pins of the fast-mode oracle (oracle/fastmode.py; Sec. IV.B, the
fast-mode paragraph): the layout and eq. 2's weights in one dimension,
window pulses equal to the full-rate sum (so n_fast equal to the window
length gives the full-rate sum), Parseval and spectral support for a pure
Doppler tone, the cross-channel phase kept bin by bin, power interpolated
linearly between nodes, and, on a scene whose Doppler spectrum varies
slowly, the gate-averaged Doppler power spectrum of the fast-mode lines
against the full-rate lines within a statistical bound (with a negative
control that the bound rejects)."""
import math

import numpy as np
import pytest

import workloads as W
import oracle as O
from oracle import fastmode as FM


def test_layout_and_weights():
    starts, nodes, L_s = FM.layout(1000, 200)
    assert list(starts) == [0, 200, 400, 600, 800]
    assert list(nodes) == [32, 232, 432, 632, 832]
    assert L_s == 512 and L_s >= 2 * 200 + 64
    starts, nodes, L_s = FM.layout(2048, 256)
    assert starts[-1] + 64 <= 2048 and starts[-1] + 256 + 64 > 2048
    assert L_s == 1024
    d = np.linspace(0.0, 1.0, 101)
    wa, wb = FM.weights(d)
    assert np.allclose(wa ** 2 + wb ** 2, 1.0, atol=1e-15)
    assert wa[0] == 1.0 and wb[0] == 0.0 and wa[-1] == 0.0 and wb[-1] == 1.0
    assert np.all(np.diff(wa) < 0) and np.all(np.diff(wb) > 0)
    # the taper's squares sum to the window length (power normalisation)
    assert abs(np.sum(FM.taper() ** 2) - 64.0) < 1e-12
    with pytest.raises(ValueError):
        FM.layout(1000, 32)


def test_window_pulses_are_the_full_rate_sum(oracle_lib):
    g = W.harmony_geometry(320, 128)
    f = W.scattered_facets(300, 60.0, seed=3)
    F = {k: v.astype(np.float64) for k, v in f.items()}
    full = O.forward(g, F)
    fast = FM.fast_forward(g, F, 128, seed=9)
    starts, _, _ = FM.layout(320, 128)
    for s in starts:
        assert np.array_equal(fast[:, s:s + 64], full[:, s:s + 64])
    # synthesized pulses differ from the sum (they are a new realisation)
    assert O.rel_l2(fast[:, 64:128], full[:, 64:128]) > 0.3
    # n_fast equal to the window length: every pulse is a window pulse
    fast64 = FM.fast_forward(g, F, 64, seed=9)
    assert np.array_equal(fast64, full)


def test_pure_tone_parseval_and_support(oracle_lib):
    """A window holding one Doppler tone (bin 10 of 64) at amplitude 3 on
    every gate: the synthesized node signal's mean power over its period is
    the tone's power (Parseval), and the missing pulses' power lies within
    two window bins of the tone."""
    C, K, Wn, N = 1, 3, 64, 16
    m = np.arange(Wn)
    tone = 3.0 * np.exp(2j * math.pi * 10 * m / Wn)
    win = np.broadcast_to(tone[None, None, :, None], (C, K, Wn, N)).copy()
    n_fast, n_p = 256, 576
    starts, nodes, L_s = FM.layout(n_p, n_fast)
    g0 = FM.node_signal(FM.window_spectra(win[:, 0]), FM.node_phases(4, 0, N, L_s), L_s)
    assert np.allclose(np.mean(np.abs(g0) ** 2, axis=1), 9.0, rtol=1e-12)
    out = FM.synthesize(win, n_p, n_fast, seed=4)
    seg = out[0, 64:256]                                   # missing pulses, [192, N]
    hann = np.sin(math.pi * (np.arange(192) + 0.5) / 192)[:, None] ** 2
    spec = np.abs(np.fft.fft(seg * hann, n=1920, axis=0)) ** 2   # fine Doppler grid
    fbin = np.arange(1920) * 64 / 1920                     # in window-bin units
    near = np.abs(((fbin - 10 + 32) % 64) - 32) <= 2.0
    frac = spec[near].sum() / spec.sum()
    assert frac > 0.99, frac


def test_cross_channel_phase_is_kept():
    """Channel 1 = channel 0 times exp(i 0.7) in every window: the missing
    pulses of channel 1 are those of channel 0 times exp(i 0.7) (the
    along-track interferometric phase survives the synthesis)."""
    rng = np.random.default_rng(1)
    K, Wn, N = 3, 64, 8
    w0 = rng.standard_normal((K, Wn, N)) + 1j * rng.standard_normal((K, Wn, N))
    win = np.stack([w0, w0 * np.exp(0.7j)])
    out = FM.synthesize(win, 600, 256, seed=2)
    assert np.allclose(out[1], out[0] * np.exp(0.7j), rtol=1e-12, atol=1e-12)


def test_power_interpolates_between_nodes():
    """Windows of power 1 (node 0) and 4 (node 1), white in Doppler: the
    gate-averaged power of the missing pulses follows (1 - d) 1 + d 4."""
    rng = np.random.default_rng(5)
    K, Wn, N = 2, 64, 4000
    amp = np.array([1.0, 2.0])[:, None, None]
    w = amp * (rng.standard_normal((K, Wn, N)) + 1j * rng.standard_normal((K, Wn, N))) / math.sqrt(2)
    n_fast = 256
    out = FM.synthesize(w[None], 64 + n_fast, n_fast, seed=3)
    starts, nodes, _ = FM.layout(64 + n_fast, n_fast)
    for p in (80, 150, 250):
        d = (p - nodes[0]) / n_fast
        want = (1 - d) * np.mean(np.abs(w[0]) ** 2 * FM.taper()[:, None] ** 2) + \
            d * np.mean(np.abs(w[1]) ** 2 * FM.taper()[:, None] ** 2)
        got = np.mean(np.abs(out[0, p]) ** 2)
        assert abs(got / want - 1.0) < 0.1, (p, got, want)


def _gate_spectrum(iq, n_gates, p_lo, p_hi):
    """Gate-averaged Doppler power spectrum: Hann-tapered 64-pulse
    periodograms over [p_lo, p_hi) in steps of 32, all gates."""
    h = FM.taper()[:, None]
    segs = [np.abs(np.fft.fft(iq[0, s:s + 64] * h, axis=0)) ** 2
            for s in range(p_lo, p_hi - 63, 32)]
    return np.mean(segs, axis=0).mean(axis=1)


def test_doppler_spectrum_of_a_slowly_varying_scene(oracle_lib):
    """A scene longer along track than the beam's footprint moves through
    the beam with a stationary Doppler spectrum (the beam's Doppler band).
    Gate-averaged over the missing pulses, the fast-mode spectrum matches the
    full-rate one in relative L1 within 0.15: with about 100 independent
    gates, three nodes and 21 half-overlapping segments, each Doppler bin of
    the two averaged spectra carries a relative sampling error of about
    0.075 (periodogram bins are exponentially distributed), so their L1
    distance is expected near 0.06.  A synthesis with the spectrum shifted by
    a quarter of the PRF exceeds the bound."""
    g = W.harmony_geometry(832, 160)
    rng = np.random.default_rng(12)
    n = 24000
    f = dict(x=rng.uniform(-2500, 2500, n), y=rng.uniform(-250, 250, n),
             z=0.3 * rng.standard_normal(n), vx=0.5 * rng.standard_normal(n),
             vy=0.5 * rng.standard_normal(n), vz=0.5 * rng.standard_normal(n),
             a_re=rng.standard_normal(n) / math.sqrt(2), a_im=rng.standard_normal(n) / math.sqrt(2))
    F = {k: np.asarray(v, np.float64) for k, v in f.items()}
    full = O.forward(g, F)
    n_fast = 256
    fast = FM.fast_forward(g, F, n_fast, seed=17)
    starts, _, _ = FM.layout(832, n_fast)
    S_full = _gate_spectrum(full, 160, 64, 768)
    S_fast = _gate_spectrum(fast, 160, 64, 768)
    err = np.abs(S_fast - S_full).sum() / S_full.sum()
    # negative control: the same synthesis with every window's Doppler
    # spectrum moved by a quarter of the PRF
    wins = np.stack([full[:, s:s + 64] for s in starts], axis=1)
    m = np.arange(64)[None, None, :, None]
    shifted = FM.synthesize(wins * np.exp(2j * math.pi * 16 * m / 64), 832, n_fast, seed=17)
    bad = np.abs(_gate_spectrum(shifted, 160, 64, 768) - S_full).sum() / S_full.sum()
    print(f"fast-mode spectrum rel L1 {err:.3f}; shifted control {bad:.3f}")
    assert err < 0.15
    assert bad > 0.5
