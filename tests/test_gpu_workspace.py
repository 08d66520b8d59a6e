"""GPU checks of the caller-owned workspaces of the C ABI: a plan built in a
workspace the caller allocated (explicit scene rectangle, block count and
outside-facet count read back), facets outside the plan's rectangle (counted,
still summed to the oracle's tolerance), one workspace reused in stream order
by two plans and by the streamed forward and adjoint, and the facet
generator writing its sea table into a caller workspace."""
import ctypes
import math
import sys

import numpy as np
import pytest

import workloads as W
import oracle as O

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


def outside_count(f, box, edge):
    """Facets whose lattice cell (floor(x / edge)) lies beyond the cells of
    the rectangle's corners (the library's rule), counted on the host."""
    cx = np.floor(f["x"].astype(np.float64) / edge)
    cy = np.floor(f["y"].astype(np.float64) / edge)
    out = ((cx < math.floor(box[0] / edge)) | (cx > math.floor(box[1] / edge)) |
           (cy < math.floor(box[2] / edge)) | (cy > math.floor(box[3] / edge)))
    return int(out.sum())


def test_plan_in_caller_workspace(env):
    torch, hs = env
    say("case: plan in a caller workspace, 3000 scattered facets, 2 channels, 96 pulses")
    g = W.harmony_geometry(96, 512, receivers="A", n_pc=2)
    f = W.scattered_facets(3000, 120.0, seed=41, sigma_v=0.6, sigma_z=0.6)
    d = dev(torch, f)
    sim = hs.Simulator(g)
    sim.device_init()
    ref = O.forward(g, f64(f))
    box = (-121.0, 121.0, -121.0, 121.0)
    plan = sim.plan(d["x"], d["y"], 8.0, box=box)
    assert plan.n_outside == 0
    assert plan.n_blocks >= 3000 // 64
    got = sim.forward(plan, d).cpu().numpy()
    e = O.rel_l2(got, ref)
    say(f"caller workspace: rel-L2 {e:.3e}, blocks {plan.n_blocks}")
    assert e < IQ_TOL
    # a rectangle 10 m short on every side: the facets beyond it are counted
    # and summed through the edge blocks of the lattice
    small = (-110.0, 110.0, -110.0, 110.0)
    p2 = sim.plan(d["x"], d["y"], 8.0, box=small)
    n_out = outside_count(f, small, 8.0)
    assert n_out > 0
    assert p2.n_outside == n_out
    e2 = O.rel_l2(sim.forward(p2, d).cpu().numpy(), ref)
    say(f"{n_out} facets outside a short rectangle: rel-L2 {e2:.3e}")
    assert e2 < IQ_TOL


def test_workspace_reused_in_stream_order(env):
    """Two plans of different facet sets built one after the other in the same
    workspace (the second overwrites the first after its sum, in stream order)
    give each set's own sum."""
    torch, hs = env
    say("case: one workspace, two facet sets planned and summed in turn")
    from paper_2405_09938_amd import _native as N
    g = W.harmony_geometry(64, 512)
    fa = W.scattered_facets(2000, 100.0, seed=3)
    fb = W.scattered_facets(1500, 80.0, seed=4)
    sim = hs.Simulator(g)
    box = (-101.0, 101.0, -101.0, 101.0)
    need = sim.workspace_size(2000, box, 8.0)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    lib = N.load()
    outs = []
    for f in (fa, fb):
        d = dev(torch, f)
        n = f["x"].size
        bx = N.SimBox(*box)
        p = ctypes.c_void_p()
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        N.check(lib.sim_plan_create(sim.handle, ctypes.c_void_p(d["x"].data_ptr()),
                                    ctypes.c_void_p(d["y"].data_ptr()), n, ctypes.byref(bx), 8.0,
                                    0, ctypes.c_void_p(ws.data_ptr()), need, stream,
                                    ctypes.byref(p)), "sim_plan_create")
        iq = torch.empty((1, 64, 512), dtype=torch.complex64, device="cuda")
        fs = N.SimFacets(n, *[ctypes.cast(d[k].data_ptr(), ctypes.POINTER(ctypes.c_float))
                              for k in FKEYS])
        N.check(lib.sim_forward(sim.handle, p, ctypes.byref(fs), 0, 64,
                                ctypes.c_void_p(iq.data_ptr()), 0, stream), "sim_forward")
        lib.sim_plan_destroy(p)      # host descriptor only: the sum still runs
        outs.append((iq, f, d))
    torch.cuda.synchronize()
    for iq, f, _ in outs:
        e = O.rel_l2(iq.cpu().numpy(), O.forward(g, f64(f)))
        say(f"reused workspace: rel-L2 {e:.3e}")
        assert e < IQ_TOL


def test_streamed_calls_share_one_workspace(env):
    """The streamed forward and adjoint run in one caller workspace; results
    match those with workspaces of their own."""
    torch, hs = env
    say("case: streamed forward then adjoint through one workspace, 3 chunks")
    g = W.harmony_geometry(48, 512, receivers="A", n_pc=3)
    sea = W.wave_sea(90, 60, 1.0, seed=8, current_speed=0.5)
    chunks = [(0, 0, 90, 20), (0, 20, 90, 30), (0, 50, 90, 10)]
    sim = hs.Simulator(g)
    need = sim.stream_workspace_size(sea, chunks, 8.0)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    rc = sim.stream_forward(sea, 8, chunks, 8.0, workspace=ws)
    gr = sim.stream_backward(sea, 8, chunks, rc, 8.0, workspace=ws)
    rc2 = sim.stream_forward(sea, 8, chunks, 8.0)
    gr2 = sim.stream_backward(sea, 8, chunks, rc2, 8.0)
    a, b = rc.cpu().numpy(), rc2.cpu().numpy()
    assert np.abs(a - b).max() <= 1e-5 * np.abs(b).max()
    for k in ("vx", "vy", "vz"):
        x, y = gr[k].cpu().numpy(), gr2[k].cpu().numpy()
        assert np.abs(x - y).max() <= 1e-5 * np.abs(y).max(), k
    parts = [O.generate_facets(sea, 8, *c) for c in chunks]
    fo = {k: np.concatenate([p_[k] for p_ in parts]).astype(np.float32).astype(np.float64)
          for k in parts[0]}
    e = O.rel_l2(a, O.forward(g, fo))
    say(f"streamed through one workspace: rel-L2 {e:.3e}")
    assert e < IQ_TOL


def test_generate_into_caller_workspace(env):
    """The generator's wave table goes through the caller's workspace; the
    facets match the oracle's generator to a float32 ulp, and a flat sea needs
    no workspace."""
    torch, hs = env
    say("case: generator with a caller workspace (waves) and without (flat)")
    sea = W.wave_sea(64, 48, 1.0, seed=12, current_speed=0.3)
    sim = hs.Simulator(W.harmony_geometry(8, 256))
    got = sim.generate(sea, 12, 10, 5, 40, 30)
    ref = O.generate_facets(sea, 12, 10, 5, 40, 30)
    for k in FKEYS:
        a = np.ascontiguousarray(got[k].cpu().numpy(), np.float32)
        b = np.ascontiguousarray(ref[k], np.float64).astype(np.float32)
        ulps = np.abs(a.view(np.int32).astype(np.int64) - b.view(np.int32).astype(np.int64))
        assert int(np.count_nonzero(ulps > 1)) == 0, k
    flat = W.flat_sea(20, 10, 2.0, sigma_v=0.5)
    f0 = sim.generate(flat, 3)
    r0 = O.generate_facets(flat, 3)
    assert np.array_equal(f0["x"].cpu().numpy(), r0["x"].astype(np.float32))
