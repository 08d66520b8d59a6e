"""GPU parity of the per-facet reception time (sim_config.rx_exact: the
receiver at each facet's own echo time, eq. 3's r_r(t_r)) against the FP64
oracle, which solves the echo equation per facet and pulse.

Bars as for the plain sum: IQ rel-L2 <= 1e-4 (and the 5e-5 budget of the
block-reference scheme), gradients <= 1e-3.  Each case also checks that the
option changes the result by far more than the bar.
"""
import sys
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
import oracle as O

pytestmark = pytest.mark.gpu

FKEYS = ("x", "y", "z", "vx", "vy", "vz", "a_re", "a_im")
GKEYS = ("z", "vx", "vy", "vz", "a_re", "a_im")
IQ_TOL = 1e-4
IQ_BUDGET = 5e-5
GRAD_TOL = 1e-3


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


def exact(g):
    return replace(g, rx_exact=True)


def test_rx_exact_cfg1_forward(env):
    torch, hs = env
    say("case: receiver at each facet's echo time, config-1 scene")
    wl = W.workload(1)
    g = exact(wl.geometry)
    f = W.iid_facets(64, 64, 5.0, seed=wl.seed)
    sim = hs.Simulator(g)
    d = dev(torch, f)
    plan = sim.plan(d["x"], d["y"], wl.block_edge)
    got = sim.forward(plan, d).cpu().numpy()
    ref = O.forward(g, f64(f))
    e = O.rel_l2(got, ref)
    moved = O.rel_l2(O.forward(wl.geometry, f64(f)), ref)
    say(f"rx_exact config 1 rel-L2 {e:.3e} (the option moves the result by {moved:.2e})")
    assert e < IQ_TOL and e < IQ_BUDGET
    assert moved > 1e-2


def test_rx_exact_multichannel_forward_adjoint(env):
    """Two receivers x 3 phase centres, pulses [37, 137), scattered facets
    with heights; forward and adjoint."""
    torch, hs = env
    say("case: rx_exact, 2000 scattered facets, 6 channels, pulses [37, 137)")
    g = exact(W.harmony_geometry(200, 512, receivers="AB", n_pc=3))
    f = W.scattered_facets(2000, 150.0, seed=13, sigma_v=0.6, sigma_z=0.7)
    sim = hs.Simulator(g)
    d = dev(torch, f)
    plan = sim.plan(d["x"], d["y"], 8.0)
    got = sim.forward(plan, d, 37, 100).cpu().numpy()
    F = f64(f)
    ref = O.forward(g, F, 37, 100)
    e = O.rel_l2(got, ref)
    say(f"rx_exact 6-channel forward rel-L2 {e:.3e}")
    assert e < IQ_TOL and e < IQ_BUDGET
    for c in range(6):
        assert O.rel_l2(got[c], ref[c]) < IQ_TOL, c
    rng = np.random.default_rng(14)
    gi = (rng.standard_normal(got.shape) + 1j * rng.standard_normal(got.shape)).astype(np.complex64)
    gr = sim.backward(plan, d, torch.from_numpy(gi).cuda(), 37, 100)
    refg = O.adjoint(g, F, gi.astype(np.complex128), 37, 100)
    for k in GKEYS:
        ek = O.rel_l2(gr[k].cpu().numpy(), refg[k])
        say(f"rx_exact adjoint {k} rel-L2 {ek:.3e}")
        assert ek < GRAD_TOL, k


def test_rx_exact_with_speckle_exact_elevation_mode(env):
    """Airborne geometry (every pattern factor per facet) with the speckle,
    forward and adjoint."""
    torch, hs = env
    say("case: rx_exact + speckle, airborne geometry (exact elevation mode)")
    plats = (W.Platform((0.0, -15000.0, 12000.0), (60.0, 0.0, 0.0)),
             W.Platform((400.0, -15000.0, 12000.0), (60.0, 0.0, 0.0)))
    g = exact(replace(W.harmony_geometry(70, 4096), platforms=plats))
    rng = np.random.default_rng(51)
    n = 1500
    f = dict(x=rng.uniform(-200, 200, n), y=rng.uniform(-24900, -24300, n),
             z=rng.normal(0, 0.3, n), vx=rng.normal(0, 0.3, n), vy=rng.normal(0, 0.3, n),
             vz=rng.normal(0, 0.3, n), a_re=rng.normal(0, 0.7, n), a_im=rng.normal(0, 0.7, n))
    f = {k: v.astype(np.float32) for k, v in f.items()}
    sp = W.Speckle(tau_s=0.01, seed=5, first_index=0)
    fs = W.speckle_doppler(n, 5)
    fsd = torch.from_numpy(fs).cuda()
    sim = hs.Simulator(g)
    d = dev(torch, f)
    plan = sim.plan(d["x"], d["y"], 2.0, speckle=True)
    assert not plan.el_const
    got = sim.forward(plan, d, 3, 60, speckle=sp, f_s=fsd).cpu().numpy()
    F = f64(f)
    ref = O.forward(g, F, 3, 60, speckle=sp, f_s=fs.astype(np.float64))
    e = O.rel_l2(got, ref)
    say(f"rx_exact + speckle airborne forward rel-L2 {e:.3e}")
    assert e < IQ_TOL
    gi = (rng.standard_normal(got.shape) + 1j * rng.standard_normal(got.shape)).astype(np.complex64)
    gr = sim.backward(plan, d, torch.from_numpy(gi).cuda(), 3, 60, speckle=sp, f_s=fsd)
    refg = O.adjoint(g, F, gi.astype(np.complex128), 3, 60, speckle=sp, f_s=fs.astype(np.float64))
    for k in ("z", "vx", "a_re"):
        ek = O.rel_l2(gr[k].cpu().numpy(), refg[k])
        say(f"rx_exact + speckle airborne adjoint {k} rel-L2 {ek:.3e}")
        assert ek < GRAD_TOL, k


def test_rx_exact_workload2_full_rows(env):
    """Workload 2 at full size with the facets' own reception times, as the
    benchmark's --rx-exact mode launches it; three sampled pulses."""
    torch, hs = env
    say("case: rx_exact, workload 2 at full size, pulses 0, 700, 2047")
    wl = W.workload(2)
    g = exact(wl.geometry)
    sim = hs.Simulator(g)
    f = sim.generate(wl.sea, wl.seed)
    plan = sim.plan(f["x"], f["y"], wl.block_edge)
    rc = sim.forward(plan, f)
    torch.cuda.synchronize()
    fo = {k: v.astype(np.float32).astype(np.float64)
          for k, v in O.generate_facets(wl.sea, wl.seed).items()}
    for p in (0, 700, 2047):
        ref = O.forward(g, fo, p, 1)
        e = O.rel_l2(rc[:, p:p + 1].cpu().numpy(), ref)
        say(f"workload 2 rx_exact row {p}: rel-L2 {e:.3e}")
        assert e < IQ_TOL and e < IQ_BUDGET
