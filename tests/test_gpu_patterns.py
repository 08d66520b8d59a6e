"""GPU parity of u-v gridded antenna patterns (Sec. III.B: patterns converted
into u-v grids in GPU memory) against the FP64 oracle, which interpolates the
same float32 tables: forward and adjoint, with a grid on every antenna or on
some, over six channels, combined with steering, speckle and the per-facet
reception time, with the beam sweeping off the table's edge, across an
antenna back plane, and workload 2 at full size on sampled rows."""
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


def check_adjoint(torch, sim, plan, d, F, g, got, p0, npl, seed, keys=GKEYS, label="", **kw):
    rng = np.random.default_rng(seed)
    gi = (rng.standard_normal(got.shape) + 1j * rng.standard_normal(got.shape)).astype(np.complex64)
    gr = sim.backward(plan, d, torch.from_numpy(gi).cuda(), p0, npl, **kw)
    okw = {k: (v.cpu().numpy().astype(np.float64) if hasattr(v, "cpu") else v)
           for k, v in kw.items()}
    refg = O.adjoint(g, F, gi.astype(np.complex128), p0, npl, **okw)
    for k in keys:
        ek = O.rel_l2(gr[k].cpu().numpy(), refg[k])
        say(f"{label} adjoint {k} rel-L2 {ek:.3e}")
        assert ek < GRAD_TOL, k


def test_patterns_cfg1_forward(env):
    torch, hs = env
    say("case: gridded Tx and Rx patterns (129x65 nodes), config-1 scene")
    wl = W.workload(1)
    g = W.gridded_geometry(wl.geometry, seed=11)
    f = W.iid_facets(64, 64, 5.0, seed=wl.seed)
    sim = hs.Simulator(g)
    d = dev(torch, f)
    plan = sim.plan(d["x"], d["y"], wl.block_edge)
    got = sim.forward(plan, d).cpu().numpy()
    F = f64(f)
    ref = O.forward(g, F)
    e = O.rel_l2(got, ref)
    moved = O.rel_l2(O.forward(wl.geometry, F), ref)
    say(f"gridded config 1 rel-L2 {e:.3e} (the grids move the result by {moved:.2e})")
    assert e < IQ_TOL and e < IQ_BUDGET
    assert moved > 1e-2


def test_patterns_multichannel_forward_adjoint(env):
    """Grids on the Tx and on receiver B only (receiver A analytic); 6
    channels, pulses [37, 137)."""
    torch, hs = env
    say("case: grids on Tx and Rx B, 2000 facets, 6 channels, pulses [37, 137)")
    g0 = W.harmony_geometry(200, 512, receivers="AB", n_pc=3)
    gg = W.gridded_geometry(g0, seed=3)
    g = replace(g0, antennas=(gg.antennas[0], g0.antennas[1], gg.antennas[2]))
    f = W.scattered_facets(2000, 150.0, seed=17, sigma_v=0.6, sigma_z=0.7)
    sim = hs.Simulator(g)
    d = dev(torch, f)
    plan = sim.plan(d["x"], d["y"], 8.0)
    got = sim.forward(plan, d, 37, 100).cpu().numpy()
    F = f64(f)
    ref = O.forward(g, F, 37, 100)
    e = O.rel_l2(got, ref)
    say(f"gridded 6-channel forward rel-L2 {e:.3e}")
    assert e < IQ_TOL and e < IQ_BUDGET
    check_adjoint(torch, sim, plan, d, F, g, got, 37, 100, 18, label="gridded 6-channel")


def test_patterns_beam_leaves_the_table(env):
    """A table spanning +-0.15 azimuth beam widths: early and late in the dwell
    the scene is off the table (field 0), in between it crosses the edge.  The
    border nodes are 0, so the field is continuous across the edge and a
    facet within rounding of it contributes next to nothing on either side."""
    torch, hs = env
    say("case: narrow tables (+-0.15 beam widths in u), the scene crossing their edges")
    g0 = W.gridded_geometry(W.harmony_geometry(400, 512), seed=5, nu=33, nv=17, span_az=0.15)
    ants = []
    for a in g0.antennas:
        v = a.pattern.values.copy()
        v[[0, -1], :] = 0.0
        v[:, [0, -1]] = 0.0
        ants.append(replace(a, pattern=replace(a.pattern, values=v)))
    g = replace(g0, antennas=tuple(ants))
    f = W.scattered_facets(1500, 120.0, seed=9, sigma_v=0.5, sigma_z=0.5)
    sim = hs.Simulator(g)
    d = dev(torch, f)
    plan = sim.plan(d["x"], d["y"], 8.0)
    got = sim.forward(plan, d).cpu().numpy()
    F = f64(f)
    ref = O.forward(g, F)
    rows = np.abs(ref).max(axis=(0, 2))
    e = O.rel_l2(got, ref)
    say(f"narrow-table forward rel-L2 {e:.3e}; zero rows {int(np.sum(rows == 0))} of {rows.size}")
    assert np.sum(rows == 0) > 20 and np.sum(rows > 0) > 20
    assert e < IQ_TOL and e < IQ_BUDGET
    assert np.abs(got[:, rows == 0]).max() < 1e-6 * np.abs(got).max()
    check_adjoint(torch, sim, plan, d, F, g, got, 0, 400, 6, label="narrow-table")


def test_patterns_with_steering_speckle_rx_exact(env):
    torch, hs = env
    say("case: grids + steering + speckle + per-facet reception time, 6 channels")
    g0 = W.gridded_geometry(W.harmony_geometry(130, 256, receivers="AB", n_pc=3), seed=8)
    ants = list(g0.antennas)
    ants[0] = replace(ants[0], steer_rate=np.radians(3.0))
    ants[2] = replace(ants[2], steer_rate=np.radians(-2.0))
    g = replace(g0, antennas=tuple(ants), rx_exact=True)
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
    say(f"grids + steering + speckle + rx_exact forward rel-L2 {e:.3e}")
    assert e < IQ_TOL and e < IQ_BUDGET
    check_adjoint(torch, sim, plan, d, F, g, got, 20, 100, 24,
                  label="grids + steering + speckle + rx_exact", speckle=sp, f_s=fsd)


def test_patterns_airborne_back_plane(env):
    """Airborne geometry whose Tx back plane crosses the scene, with gridded
    patterns wide enough to cover it (grazing blocks take the per-facet test)."""
    torch, hs = env
    say("case: gridded patterns, Tx back plane across an airborne scene")
    plats = (W.Platform((0.0, -15000.0, 12000.0), (60.0, 0.0, 0.0)),
             W.Platform((400.0, -15000.0, 12000.0), (60.0, 0.0, 0.0)))
    g0 = replace(W.harmony_geometry(48, 4096), platforms=plats)
    # the scene sits near v = 1 on the elevation axis: tables over [-1.02, 1.02]
    wide = tuple(replace(a, beta_az=0.5, beta_el=0.6) for a in g0.antennas)
    g = W.gridded_geometry(replace(g0, antennas=wide), seed=2, span_az=1.9, span_el=1.7)
    rng = np.random.default_rng(61)
    n = 3000
    f = dict(x=rng.uniform(-300, 300, n), y=rng.uniform(-25400, -23800, n),
             z=rng.normal(0, 0.3, n), vx=rng.normal(0, 0.3, n), vy=rng.normal(0, 0.3, n),
             vz=rng.normal(0, 0.3, n), a_re=rng.normal(0, 0.7, n), a_im=rng.normal(0, 0.7, n))
    f = {k: v.astype(np.float32) for k, v in f.items()}
    sim = hs.Simulator(g)
    d = dev(torch, f)
    plan = sim.plan(d["x"], d["y"], 2.0)
    got = sim.forward(plan, d).cpu().numpy()
    F = f64(f)
    ref = O.forward(g, F)
    e = O.rel_l2(got, ref)
    say(f"gridded airborne forward rel-L2 {e:.3e}")
    assert e < IQ_TOL
    check_adjoint(torch, sim, plan, d, F, g, got, 0, 48, 62, keys=("z", "vx", "a_re"),
                  label="gridded airborne")


def test_patterns_workload2_full_rows(env):
    torch, hs = env
    say("case: gridded patterns, workload 2 at full size, pulses 0, 1024, 2047")
    wl = W.workload(2)
    g = W.gridded_geometry(wl.geometry, seed=12)
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
        say(f"workload 2 gridded row {p}: rel-L2 {e:.3e}")
        assert e < IQ_TOL and e < IQ_BUDGET


def test_patterns_streamed_scene(env):
    """Gridded patterns through the streamed entry points (chunks generated,
    planned and summed in the library), forward and dL/dV."""
    torch, hs = env
    say("case: gridded patterns, streamed scene of 3 chunks, 3 channels, 64 pulses")
    g = W.gridded_geometry(W.harmony_geometry(64, 1024, receivers="A", n_pc=3), seed=21)
    sea = W.wave_sea(120, 80, 1.0, seed=5, current_speed=0.5)
    chunks = [(0, 0, 70, 40), (70, 0, 50, 40), (0, 40, 120, 40)]
    sim = hs.Simulator(g)
    rc = sim.stream_forward(sea, 5, chunks, 8.0)
    parts = [O.generate_facets(sea, 5, *c) for c in chunks]
    fo = {k: np.concatenate([p[k] for p in parts]).astype(np.float32).astype(np.float64)
          for k in parts[0]}
    ref = O.forward(g, fo)
    got = rc.cpu().numpy()
    e = O.rel_l2(got, ref)
    say(f"gridded streamed rel-L2 {e:.3e}")
    assert e < IQ_TOL and e < IQ_BUDGET
    rng = np.random.default_rng(22)
    gi = (rng.standard_normal(got.shape) + 1j * rng.standard_normal(got.shape)).astype(np.complex64)
    gr = sim.stream_backward(sea, 5, chunks, torch.from_numpy(gi).cuda(), 8.0)
    refg = O.adjoint(g, fo, gi.astype(np.complex128))
    for k in ("vx", "vy", "vz"):
        ek = O.rel_l2(gr[k].cpu().numpy(), refg[k])
        say(f"gridded streamed adjoint {k} rel-L2 {ek:.3e}")
        assert ek < GRAD_TOL, k


def test_patterns_edges(env):
    """Gridded patterns on the edge cases of the plain path: a lone facet and
    a ragged 63-facet set, accumulation onto an existing IQ, taps leaving a
    narrow range window, an empty pulse range, and the adjoint of a lone
    facet."""
    torch, hs = env
    say("case: gridded edges (1 and 63 facets, accumulate, narrow window, empty range)")
    g = W.gridded_geometry(W.harmony_geometry(64, 128), seed=31)
    sim = hs.Simulator(g)
    rng = np.random.default_rng(32)
    for n in (1, 63):
        f = dict(x=rng.uniform(-300, 300, n), y=rng.uniform(-700, 700, n),
                 z=rng.normal(0, 0.5, n), vx=rng.normal(0, 0.5, n), vy=rng.normal(0, 0.5, n),
                 vz=rng.normal(0, 0.5, n), a_re=rng.normal(0, 0.7, n),
                 a_im=rng.normal(0, 0.7, n))
        f = {k: v.astype(np.float32) for k, v in f.items()}
        d = dev(torch, f)
        plan = sim.plan(d["x"], d["y"], 8.0)
        base = torch.full((1, 64, 128), 0.5 - 0.25j, dtype=torch.complex64, device="cuda")
        sim.forward(plan, d, 0, 64, out=base, accumulate=True)
        torch.cuda.synchronize()
        got = base.cpu().numpy().astype(np.complex128) - (0.5 - 0.25j)
        F = f64(f)
        ref = O.forward(g, F)
        scale = np.abs(ref).max()
        err = O.rel_l2(got, ref) if scale > 0 else np.abs(got).max()
        say(f"{n} facet(s), accumulate, narrow window: rel-L2 {err:.3e}")
        assert err < IQ_TOL
        empty = sim.forward(plan, d, 10, 0)
        assert empty.numel() == 0
        if n == 1 and scale > 0:
            check_adjoint(torch, sim, plan, d, F, g, sim.forward(plan, d).cpu().numpy(), 0, 64,
                          33, label="gridded lone facet")
