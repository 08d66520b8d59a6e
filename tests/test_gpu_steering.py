"""GPU parity of time-dependent antenna patterns (frames turning about their
elevation axes at constant rates, TOPS-like steering) against the FP64
oracle: forward and adjoint, with steered transmit and receive antennas, in
both elevation modes (the airborne case also turns the Tx back plane across
the scene), combined with the speckle and the per-facet reception time, and
workload 2 at full size on sampled rows."""
import math
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


def steer(g, rates_deg_s):
    ants = tuple(replace(a, steer_rate=math.radians(r)) for a, r in zip(g.antennas, rates_deg_s))
    return replace(g, antennas=ants + g.antennas[len(ants):])


def test_steering_cfg1_forward(env):
    torch, hs = env
    say("case: Tx steered at 3 deg/s, config-1 scene")
    wl = W.workload(1)
    g = W.tops_geometry(wl.geometry, 3.0)
    f = W.iid_facets(64, 64, 5.0, seed=wl.seed)
    sim = hs.Simulator(g)
    d = dev(torch, f)
    plan = sim.plan(d["x"], d["y"], wl.block_edge)
    got = sim.forward(plan, d).cpu().numpy()
    ref = O.forward(g, f64(f))
    e = O.rel_l2(got, ref)
    moved = O.rel_l2(O.forward(wl.geometry, f64(f)), ref)
    say(f"steered config 1 rel-L2 {e:.3e} (the steering moves the result by {moved:.2e})")
    assert e < IQ_TOL and e < IQ_BUDGET
    assert moved > 1e-3


def test_steering_multichannel_forward_adjoint(env):
    """Tx at +2 deg/s, receiver A at -1 deg/s; 6 channels, pulses [37, 137)."""
    torch, hs = env
    say("case: Tx and Rx A steered, 2000 facets, 6 channels, pulses [37, 137)")
    g = steer(W.harmony_geometry(200, 512, receivers="AB", n_pc=3), (2.0, -1.0))
    f = W.scattered_facets(2000, 150.0, seed=17, sigma_v=0.6, sigma_z=0.7)
    sim = hs.Simulator(g)
    d = dev(torch, f)
    plan = sim.plan(d["x"], d["y"], 8.0)
    got = sim.forward(plan, d, 37, 100).cpu().numpy()
    F = f64(f)
    ref = O.forward(g, F, 37, 100)
    e = O.rel_l2(got, ref)
    say(f"steered 6-channel forward rel-L2 {e:.3e}")
    assert e < IQ_TOL and e < IQ_BUDGET
    rng = np.random.default_rng(18)
    gi = (rng.standard_normal(got.shape) + 1j * rng.standard_normal(got.shape)).astype(np.complex64)
    gr = sim.backward(plan, d, torch.from_numpy(gi).cuda(), 37, 100)
    refg = O.adjoint(g, F, gi.astype(np.complex128), 37, 100)
    for k in GKEYS:
        ek = O.rel_l2(gr[k].cpu().numpy(), refg[k])
        say(f"steered adjoint {k} rel-L2 {ek:.3e}")
        assert ek < GRAD_TOL, k


def test_steering_airborne_back_plane(env):
    """Airborne geometry (exact elevation mode) whose Tx back plane crosses
    the scene and turns with the antenna; forward and adjoint."""
    torch, hs = env
    say("case: steered Tx back plane across an airborne scene, forward and adjoint")
    plats = (W.Platform((0.0, -15000.0, 12000.0), (60.0, 0.0, 0.0)),
             W.Platform((400.0, -15000.0, 12000.0), (60.0, 0.0, 0.0)))
    g = W.tops_geometry(replace(W.harmony_geometry(48, 4096), platforms=plats), 60.0)
    rng = np.random.default_rng(61)
    n = 3000
    f = dict(x=rng.uniform(-300, 300, n), y=rng.uniform(-25400, -23800, n),
             z=rng.normal(0, 0.3, n), vx=rng.normal(0, 0.3, n), vy=rng.normal(0, 0.3, n),
             vz=rng.normal(0, 0.3, n), a_re=rng.normal(0, 0.7, n), a_im=rng.normal(0, 0.7, n))
    f = {k: v.astype(np.float32) for k, v in f.items()}
    sim = hs.Simulator(g)
    d = dev(torch, f)
    plan = sim.plan(d["x"], d["y"], 2.0)
    assert not plan.el_const
    got = sim.forward(plan, d).cpu().numpy()
    F = f64(f)
    ref = O.forward(g, F)
    e = O.rel_l2(got, ref)
    say(f"steered airborne forward rel-L2 {e:.3e}")
    assert e < IQ_TOL
    gi = (rng.standard_normal(got.shape) + 1j * rng.standard_normal(got.shape)).astype(np.complex64)
    gr = sim.backward(plan, d, torch.from_numpy(gi).cuda())
    refg = O.adjoint(g, F, gi.astype(np.complex128))
    for k in ("z", "vx", "a_re"):
        ek = O.rel_l2(gr[k].cpu().numpy(), refg[k])
        say(f"steered airborne adjoint {k} rel-L2 {ek:.3e}")
        assert ek < GRAD_TOL, k


def test_steering_with_speckle_and_rx_exact(env):
    torch, hs = env
    say("case: steering + speckle + per-facet reception time, 6 channels, forward and adjoint")
    g = replace(steer(W.harmony_geometry(130, 256, receivers="AB", n_pc=3), (3.0, 0.0, -2.0)),
                rx_exact=True)
    f = W.scattered_facets(1500, 100.0, seed=23, sigma_v=0.5, sigma_z=0.5)
    sp = W.Speckle(tau_s=0.02, seed=23, first_index=11)
    fs = W.speckle_doppler(1500, 23)
    fsd = torch.from_numpy(fs).cuda()
    sim = hs.Simulator(g)
    d = dev(torch, f)
    plan = sim.plan(d["x"], d["y"], 8.0, speckle=True)
    got = sim.forward(plan, d, 20, 100, speckle=sp, f_s=fsd).cpu().numpy()
    F = f64(f)
    ref = O.forward(g, F, 20, 100, speckle=sp, f_s=fs.astype(np.float64))
    e = O.rel_l2(got, ref)
    say(f"steering + speckle + rx_exact forward rel-L2 {e:.3e}")
    assert e < IQ_TOL and e < IQ_BUDGET
    rng = np.random.default_rng(24)
    gi = (rng.standard_normal(got.shape) + 1j * rng.standard_normal(got.shape)).astype(np.complex64)
    gr = sim.backward(plan, d, torch.from_numpy(gi).cuda(), 20, 100, speckle=sp, f_s=fsd)
    refg = O.adjoint(g, F, gi.astype(np.complex128), 20, 100, speckle=sp,
                     f_s=fs.astype(np.float64))
    for k in GKEYS:
        ek = O.rel_l2(gr[k].cpu().numpy(), refg[k])
        say(f"steering + speckle + rx_exact adjoint {k} rel-L2 {ek:.3e}")
        assert ek < GRAD_TOL, k


def test_steering_workload2_full_rows(env):
    torch, hs = env
    say("case: steered Tx (1.5 deg/s), workload 2 at full size, pulses 0, 1024, 2047")
    wl = W.workload(2)
    g = W.tops_geometry(wl.geometry, 1.5)
    sim = hs.Simulator(g)
    f = sim.generate(wl.sea, wl.seed)
    plan = sim.plan(f["x"], f["y"], wl.block_edge)
    rc = sim.forward(plan, f)
    torch.cuda.synchronize()
    fo = {k: v.astype(np.float32).astype(np.float64)
          for k, v in O.generate_facets(wl.sea, wl.seed).items()}
    for p in (0, 1024, 2047):
        ref = O.forward(g, fo, p, 1)
        e = O.rel_l2(rc[:, p:p + 1].cpu().numpy(), ref)
        say(f"workload 2 steered row {p}: rel-L2 {e:.3e}")
        assert e < IQ_TOL and e < IQ_BUDGET
