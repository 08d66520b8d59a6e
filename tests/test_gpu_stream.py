"""GPU parity of the streamed scene path (chunks generated, planned and
summed inside the library) against the FP64 oracle, which generates the same
chunks from the same seed and sea draws with its own code."""
import sys

import numpy as np
import pytest

import workloads as W
import oracle as O

pytestmark = pytest.mark.gpu

IQ_TOL = 1e-4
GRAD_TOL = 1e-3


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


def oracle_chunk_facets(sea, seed, chunks):
    parts = [O.generate_facets(sea, seed, *c) for c in chunks]
    f = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    return {k: v.astype(np.float32).astype(np.float64) for k, v in f.items()}


def test_stream_forward_and_backward(hs):
    import torch
    say("case: streamed scene, 4 chunks of 60x40 @1 m, 3 channels, 64 pulses, chirp")
    g = W.harmony_geometry(64, 1024, receivers="A", n_pc=3, chirp=True)
    sea = W.wave_sea(120, 80, 1.0, seed=5, current_speed=0.5)
    chunks = [(0, 0, 60, 40), (60, 0, 60, 40), (0, 40, 60, 40), (60, 40, 60, 40)]
    sim = hs.Simulator(g)
    rc = sim.stream_forward(sea, 5, chunks, 8.0)
    raw = sim.apply_waveform(rc).cpu().numpy()
    fo = oracle_chunk_facets(sea, 5, chunks)
    ref_rc = O.forward(g, fo)
    ref_raw = O.waveform_fft(g, ref_rc)
    e1 = O.rel_l2(rc.cpu().numpy(), ref_rc)
    e2 = O.rel_l2(raw, ref_raw)
    say(f"streamed rc rel-L2 {e1:.3e}, raw rel-L2 {e2:.3e}")
    assert e1 < IQ_TOL and e2 < IQ_TOL
    # one plan over the whole scene gives the same lines
    whole = sim.generate(sea, 5)
    plan = sim.plan(whole["x"], whole["y"], 8.0)
    one = sim.forward(plan, whole).cpu().numpy()
    e3 = O.rel_l2(rc.cpu().numpy(), one)
    say(f"streamed vs single plan rel-L2 {e3:.3e}")
    assert e3 < 1e-5
    # adjoint w.r.t. velocities, chunk order
    rng = np.random.default_rng(7)
    gi = (rng.standard_normal(rc.shape) + 1j * rng.standard_normal(rc.shape)).astype(np.complex64)
    gr = sim.stream_backward(sea, 5, chunks, torch.from_numpy(gi).cuda(), 8.0)
    ref = O.adjoint(g, fo, gi.astype(np.complex128))
    for k in ("vx", "vy", "vz"):
        e = O.rel_l2(gr[k].cpu().numpy(), ref[k])
        say(f"streamed adjoint {k}: rel-L2 {e:.3e}")
        assert e < GRAD_TOL


def test_streamed_workload5_pulse_subset(hs):
    """Full-size geometry of the 1.28e8-facet streamed workload: its first
    8e6-facet chunk, all 3 channels, 2 pulses from the middle of the dwell,
    in the launch configuration of the full run."""
    say("case: workload 5, chunk 0 (4000x2000 facets), pulses 8191..8192, 3 channels")
    wl = W.workload(5)
    g = wl.geometry
    sim = hs.Simulator(g)
    chunks = [wl.chunks[0]]
    p0, npl = g.n_pulses // 2 - 1, 2
    rc = sim.stream_forward(wl.sea, wl.seed, chunks, wl.block_edge, p0, npl).cpu().numpy()
    fo = oracle_chunk_facets(wl.sea, wl.seed, chunks)
    ref = O.forward(g, fo, p0, npl)
    e = O.rel_l2(rc, ref)
    say(f"workload 5 chunk 0 rel-L2 {e:.3e}")
    assert e < IQ_TOL
