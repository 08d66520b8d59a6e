"""The forward sum is deterministic: every window of a strip segment goes to
its own scratch slot and the lines add the windows in segment order, and a
cell's facets are summed in ascending index, so two launches give the same
bits, whatever order the GPU runs the work in.  Checked on workload 2 at
full size, on a planned-again copy of the scene (the plan's atomically
counted sort must come out the same), and on streamed workload-5 rows."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


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


def test_forward_is_bitwise_repeatable(env):
    torch, hs = env
    say("case: workload 2 forward, twice on one plan, once on a second plan")
    wl = W.workload(2)
    sim = hs.Simulator(wl.geometry)
    f = sim.generate(wl.sea, wl.seed)
    plan = sim.plan(f["x"], f["y"], wl.block_edge, box=sim.chunk_box(wl.sea))
    a = sim.forward(plan, f).cpu().numpy()
    b = sim.forward(plan, f).cpu().numpy()
    plan2 = sim.plan(f["x"], f["y"], wl.block_edge, box=sim.chunk_box(wl.sea))
    c = sim.forward(plan2, f).cpu().numpy()
    say(f"max |a - b| {np.abs(a - b).max():.3e}, max |a - c| {np.abs(a - c).max():.3e}")
    assert np.array_equal(a, b)
    assert np.array_equal(a, c)
    # accumulate adds the same bits on top
    base = torch.from_numpy(a).cuda()
    sim.forward(plan, f, out=base, accumulate=True)
    assert np.array_equal(base.cpu().numpy(), (a + a))


def test_streamed_forward_is_bitwise_repeatable(env):
    torch, hs = env
    say("case: workload 5, first chunk, 192 pulses at the dwell's start, twice")
    wl = W.workload(5)
    sim = hs.Simulator(wl.geometry)
    a = sim.stream_forward(wl.sea, wl.seed, wl.chunks[:1], wl.block_edge, 0, 192).cpu().numpy()
    b = sim.stream_forward(wl.sea, wl.seed, wl.chunks[:1], wl.block_edge, 0, 192).cpu().numpy()
    say(f"max |a - b| {np.abs(a - b).max():.3e}")
    assert np.abs(a).max() > 0
    assert np.array_equal(a, b)


def _dense_scene():
    """A cluster of 6000 facets in a 24 m square (9 cells of 8 m, ~670
    facets each: the LDS sort) over 2000 spread in a 150 m square (cells of
    a few facets: the register sort)."""
    a = W.scattered_facets(6000, 12.0, seed=31, sigma_v=0.6, sigma_z=0.7)
    b = W.scattered_facets(2000, 75.0, seed=32, sigma_v=0.6, sigma_z=0.7)
    return {k: np.concatenate([a[k], b[k]]) for k in a}


def test_dense_cells_repeatable_and_match_oracle(env):
    torch, hs = env
    import oracle as O
    say("case: dense cells (65..1024 facets) and sparse cells, 128 pulses x 512 samples")
    g = W.harmony_geometry(128, 512)
    f = _dense_scene()
    sim = hs.Simulator(g)
    d = {k: torch.from_numpy(np.ascontiguousarray(f[k], np.float32)).cuda() for k in f}
    plan = sim.plan(d["x"], d["y"], 8.0)
    a = sim.forward(plan, d).cpu().numpy()
    b = sim.forward(plan, d).cpu().numpy()
    c = sim.forward(sim.plan(d["x"], d["y"], 8.0), d).cpu().numpy()
    say(f"max |a - b| {np.abs(a - b).max():.3e}, max |a - c| {np.abs(a - c).max():.3e}")
    assert np.array_equal(a, b)
    assert np.array_equal(a, c)
    ref = O.forward(g, {k: np.asarray(f[k], np.float32).astype(np.float64) for k in f})
    err = O.rel_l2(a.astype(np.complex128), ref)
    say(f"dense cells rel-L2 vs the oracle {err:.3e}")
    assert err < 1e-4
