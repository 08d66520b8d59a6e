"""GPU parity of the fast mode (Sec. IV.B, fast-mode paragraph;
sim_forward_fast) against the FP64 oracle's fast mode (oracle/fastmode.py),
element by element under the same counter-based phases: a two-channel scene
(window rows and synthesized rows, the cross-channel phase), n_fast = 64
(every pulse in a window: the full-rate sum), a spacing that is not a power
of two, the widest spacing (a synthesis workgroup holding 145 KB of LDS),
and workload 2 at full size on sampled gates, the oracle synthesizing from
the GPU's own window rows."""
import sys

import numpy as np
import pytest

import workloads as W
import oracle as O
from oracle import fastmode as FM

pytestmark = pytest.mark.gpu

IQ_TOL = 1e-4
FKEYS = ("x", "y", "z", "vx", "vy", "vz", "a_re", "a_im")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_09938_amd as hs
    hs.load()
    return torch, hs


def dev(torch, f):
    return {k: torch.from_numpy(np.ascontiguousarray(f[k], np.float32)).cuda() for k in FKEYS}


def f64(f):
    return {k: np.asarray(f[k], np.float32).astype(np.float64) for k in FKEYS}


def window_rows(n_pulses, n_fast):
    starts, _, _ = FM.layout(n_pulses, n_fast)
    rows = np.zeros(n_pulses, bool)
    for s in starts:
        rows[s:s + 64] = True
    return rows


@pytest.mark.parametrize("n_fast,n_pulses,n_samples,n_pc", [(128, 700, 256, 2), (320, 1000, 128, 1),
                                                            (1024, 2200, 64, 1)])
def test_fast_mode_matches_oracle(env, n_fast, n_pulses, n_samples, n_pc):
    torch, hs = env
    say(f"case: fast mode n_fast {n_fast}, {n_pulses} pulses x {n_samples} samples x {n_pc} ch")
    g = W.harmony_geometry(n_pulses, n_samples, receivers="A", n_pc=n_pc)
    f = W.scattered_facets(2500, 150.0, seed=n_fast, sigma_v=0.5, sigma_z=0.4)
    sim = hs.Simulator(g)
    d = dev(torch, f)
    plan = sim.plan(d["x"], d["y"], 8.0)
    got = sim.forward_fast(plan, d, n_fast, seed=1234 + n_fast).cpu().numpy()
    ref = FM.fast_forward(g, f64(f), n_fast, seed=1234 + n_fast)
    rows = window_rows(n_pulses, n_fast)
    e_all = O.rel_l2(got, ref)
    e_win = O.rel_l2(got[:, rows], ref[:, rows])
    e_syn = O.rel_l2(got[:, ~rows], ref[:, ~rows])
    say(f"n_fast {n_fast}: rel-L2 all {e_all:.3e}, window rows {e_win:.3e}, "
        f"synthesized rows {e_syn:.3e}")
    assert e_all < IQ_TOL and e_win < IQ_TOL and e_syn < IQ_TOL
    if n_pc > 1:
        for c in range(n_pc):
            assert O.rel_l2(got[c][~rows], ref[c][~rows]) < IQ_TOL, c


def test_fast_mode_spacing_64_is_the_full_rate_sum(env):
    torch, hs = env
    say("case: fast mode n_fast 64 (every pulse in a window) vs sim_forward")
    g = W.harmony_geometry(256, 256)
    f = W.scattered_facets(2000, 120.0, seed=2)
    sim = hs.Simulator(g)
    d = dev(torch, f)
    plan = sim.plan(d["x"], d["y"], 8.0)
    a = sim.forward_fast(plan, d, 64, seed=5).cpu().numpy()
    b = sim.forward(plan, d).cpu().numpy()
    diff = np.abs(a - b).max() / np.abs(b).max()
    say(f"n_fast 64 vs the full-rate sum: max rel diff {diff:.3e}")
    assert diff < 1e-5


def test_fast_mode_workload2_sampled_gates(env):
    """Workload 2 at full size with n_fast = 256: window rows against the
    full-rate sum of the same plan, and the synthesized rows of 12 sampled
    gates against the oracle's synthesis from those window rows."""
    torch, hs = env
    say("case: fast mode on workload 2 (1e6 facets, 2048 pulses), n_fast 256")
    wl = W.workload(2)
    sim = hs.Simulator(wl.geometry)
    f = sim.generate(wl.sea, wl.seed)
    plan = sim.plan(f["x"], f["y"], wl.block_edge)
    fast = sim.forward_fast(plan, f, 256, seed=99)
    full = sim.forward(plan, f)
    rows = window_rows(2048, 256)
    a, b = fast.cpu().numpy(), full.cpu().numpy()
    e_win = O.rel_l2(a[:, rows], b[:, rows])
    assert e_win < 1e-5, e_win
    # 12 gates drawn among those the scene reaches (most of the 4096 are empty)
    power = np.mean(np.abs(b[0]) ** 2, axis=0)
    live = np.flatnonzero(power > 0.01 * power.max())
    assert live.size > 50
    rng = np.random.default_rng(3)
    gates = np.sort(rng.choice(live, 12, replace=False))
    starts, _, _ = FM.layout(2048, 256)
    # the oracle synthesizes from the GPU's window rows
    wins_fast = np.stack([a[:, s:s + 64][:, :, gates] for s in starts], axis=1).astype(np.complex128)
    ref = FM.synthesize(wins_fast, 2048, 256, seed=99, gates=gates)
    got_syn = a[:, ~rows][:, :, gates]
    assert np.abs(got_syn).max() > 0
    e_syn = O.rel_l2(got_syn, ref[:, ~rows])
    say(f"workload 2: window rows vs full-rate {e_win:.3e}; synthesized rows of 12 gates "
        f"vs the oracle's synthesis {e_syn:.3e}")
    assert e_syn < 1e-5


@pytest.mark.parametrize("option", ["steering", "patterns", "rx_exact"])
def test_fast_mode_with_handle_options(env, option):
    """The fast mode on handles with the forward's other options (the window
    sums take the same kernel variants as the full-rate sum): a Tx beam
    steered at 3 deg/s, u-v gridded patterns, the receiver at each facet's
    echo time; against the oracle's fast mode on the same geometry."""
    from dataclasses import replace
    torch, hs = env
    say(f"case: fast mode n_fast 256 with {option}")
    g = W.harmony_geometry(900, 128, receivers="A", n_pc=1)
    if option == "steering":
        g = W.tops_geometry(g, 3.0)
    elif option == "patterns":
        g = W.gridded_geometry(g, seed=4)
    else:
        g = replace(g, rx_exact=True)
    f = W.scattered_facets(2000, 150.0, seed=44, sigma_v=0.5, sigma_z=0.4)
    sim = hs.Simulator(g)
    d = dev(torch, f)
    plan = sim.plan(d["x"], d["y"], 8.0)
    got = sim.forward_fast(plan, d, 256, seed=77).cpu().numpy()
    ref = FM.fast_forward(g, f64(f), 256, seed=77)
    rows = window_rows(900, 256)
    e_win = O.rel_l2(got[:, rows], ref[:, rows])
    e_syn = O.rel_l2(got[:, ~rows], ref[:, ~rows])
    say(f"{option}: window rows {e_win:.3e}, synthesized rows {e_syn:.3e}")
    assert e_win < IQ_TOL and e_syn < IQ_TOL
