"""GPU parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times (whole scene generated on the device, one
plan, the whole pulse range in one call), checked on sampled outputs the
oracle computes one by one: whole (channel, pulse) rows of IQ for the
forward, whole facets for the adjoint.  The oracle generates the same scene
from the same seed and sea draws with its own code."""
import sys

import numpy as np
import pytest

import workloads as W
import oracle as O

pytestmark = pytest.mark.gpu

IQ_TOL = 1e-4
IQ_BUDGET = 5e-5
GRAD_TOL = 1e-3
GKEYS = ("z", "vx", "vy", "vz", "a_re", "a_im")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hs():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_09938_amd as hs
    hs.load()
    return hs


def oracle_scene(wl):
    f = O.generate_facets(wl.sea, wl.seed)
    return {k: v.astype(np.float32).astype(np.float64) for k, v in f.items()}


def sampled_pulses(n_pulses, k, seed):
    rng = np.random.default_rng(seed)
    mid = rng.choice(np.arange(1, n_pulses - 1), size=k - 2, replace=False)
    return sorted({0, n_pulses - 1, *mid.tolist()})


def check_rows(hs, k, n_rows, expect_el_const):
    import torch
    wl = W.workload(k)
    g = wl.geometry
    sim = hs.Simulator(g)
    f = sim.generate(wl.sea, wl.seed)
    plan = sim.plan(f["x"], f["y"], wl.block_edge)
    say(f"elevation mode: const {plan.el_const}, bound {plan.el_bound:.2e}")
    assert plan.el_const == expect_el_const
    rc = sim.forward(plan, f)
    raw = sim.apply_waveform(rc) if g.chirp_T > 0 else None
    torch.cuda.synchronize()
    pulses = sampled_pulses(g.n_pulses, n_rows, 100 + k)
    say(f"sampled pulses {pulses} x {g.n_channels} channels")
    fo = oracle_scene(wl)
    got_rc = np.stack([rc[:, p].cpu().numpy() for p in pulses], 1)
    ref_rc = np.concatenate([O.forward(g, fo, p, 1) for p in pulses], 1)
    e = O.rel_l2(got_rc, ref_rc)
    say(f"workload {k} rc rows rel-L2 {e:.3e}")
    assert e < IQ_TOL and e < IQ_BUDGET
    for c in range(g.n_channels):
        ec = O.rel_l2(got_rc[c], ref_rc[c])
        say(f"  channel {c}: rel-L2 {ec:.3e}")
        assert ec < IQ_TOL
    if raw is not None:
        got_raw = np.stack([raw[:, p].cpu().numpy() for p in pulses], 1)
        er = O.rel_l2(got_raw, O.waveform_fft(g, ref_rc))
        say(f"workload {k} raw rows rel-L2 {er:.3e}")
        assert er < IQ_TOL


def test_workload2_full_rows(hs):
    say("case: workload 2 at full size (1e6 facets, 2048 pulses, 4096 samples), 5 rows")
    check_rows(hs, 2, 5, True)


def test_workload3_full_rows(hs):
    say("case: workload 3 at full size (1.6e7 facets, 4096 pulses, 8192 samples, "
        "6 channels), 2 pulses")
    check_rows(hs, 3, 2, True)


def test_workload4_full_adjoint_sampled_facets(hs):
    """Adjoint over all 1024 pulses of the 1e6-facet scene; gradients of 256
    seed-drawn facets against the oracle adjoint of those facets alone (each
    facet's gradient depends only on itself and g)."""
    import torch
    say("case: workload 4 adjoint at full size (1e6 facets, 1024 pulses), 256 facets")
    wl = W.workload(4)
    g = wl.geometry
    sim = hs.Simulator(g)
    f = sim.generate(wl.sea, wl.seed)
    plan = sim.plan(f["x"], f["y"], wl.block_edge)
    shape = (g.n_channels, g.n_pulses, g.n_samples)
    gen = torch.Generator(device="cuda").manual_seed(41)
    gi = torch.complex(torch.randn(shape, device="cuda", generator=gen),
                       torch.randn(shape, device="cuda", generator=gen))
    gr = sim.backward(plan, f, gi)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(42).choice(f["x"].numel(), 256, replace=False))
    fo = {k: v[idx] for k, v in oracle_scene(wl).items()}
    ref = O.adjoint(g, fo, gi.cpu().numpy().astype(np.complex128))
    for k in GKEYS:
        e = O.rel_l2(gr[k].cpu().numpy()[idx], ref[k])
        say(f"workload 4 adjoint {k}: rel-L2 {e:.3e}")
        assert e < GRAD_TOL, k


def test_workload4_autograd_vs_fd_on_64_facets(hs):
    """Workload 4's check at full facet count: loss ||IQ - T||^2 with T from the
    same facets moved by a 0.1 m/s current, GPU autograd against central
    finite differences of the FP64 oracle's loss with h = 1e-3 on 64
    seed-drawn facets (Richardson h, h/2 for height, whose FD truncation at
    h = 1e-3 alone is about 0.5 %).  Pulses 480 .. 543 of the 1024 keep the
    oracle's full-scene forward within seconds; the GPU runs the same pulse
    range through the same plan."""
    import torch
    say("case: workload 4, 1e6 facets, pulses 480..543, autograd vs oracle FD on 64 facets")
    wl = W.workload(4)
    g = wl.geometry
    p0, npl = 480, 64
    sim = hs.Simulator(g)
    f = sim.generate(wl.sea, wl.seed)
    plan = sim.plan(f["x"], f["y"], wl.block_edge)
    psi = W.sea_draws(wl.seed)["perturb_heading"]
    cx, cy = np.float32(0.1 * np.cos(psi)), np.float32(0.1 * np.sin(psi))
    ft = dict(f)
    ft["vx"] = f["vx"] + float(cx)
    ft["vy"] = f["vy"] + float(cy)
    with torch.no_grad():
        tgt = sim.forward(plan, ft, p0, npl)
    for k in GKEYS:
        f[k].requires_grad_(True)
    iq = hs.simulate(sim, plan, f, p0, npl)
    ((iq - tgt).abs() ** 2).sum().backward()
    idx = np.sort(np.random.default_rng(44).choice(f["x"].numel(), 64, replace=False))
    gpu = {k: f[k].grad.cpu().numpy()[idx] for k in GKEYS}
    fo32 = {k: v.astype(np.float32) for k, v in O.generate_facets(wl.sea, wl.seed).items()}
    fto = dict(fo32)
    fto["vx"] = (fo32["vx"] + cx).astype(np.float32)
    fto["vy"] = (fo32["vy"] + cy).astype(np.float32)
    F = {k: v.astype(np.float64) for k, v in fo32.items()}
    T = O.forward(g, {k: v.astype(np.float64) for k, v in fto.items()}, p0, npl)
    resid = O.forward(g, F, p0, npl) - T
    for k in GKEYS:
        h = 1e-3
        fd = []
        for i in idx:
            d1 = O.fd_gradient(g, F, T, int(i), k, h, p0, npl, resid=resid)
            if k == "z":
                d2 = O.fd_gradient(g, F, T, int(i), k, h / 2, p0, npl, resid=resid)
                d1 = (4.0 * d2 - d1) / 3.0
            fd.append(d1)
        e = O.rel_l2(gpu[k], np.array(fd))
        say(f"workload 4 autograd {k} vs FD (h=1e-3{', Richardson' if k == 'z' else ''}): rel-L2 {e:.3e}")
        assert e < GRAD_TOL, k
