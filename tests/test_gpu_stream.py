"""GPU parity of the streamed scene path (chunks generated, planned and
summed inside the library) against the FP64 oracle, which generates the same
chunks from the same seed and sea draws with its own code; with the
intra-facet speckle, whose facet ids and Doppler follow the grid index."""
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


IQ_BUDGET = 5e-5


@pytest.mark.parametrize("chunk_idx", [0, 15])
def test_streamed_workload5_dwell_ends(hs, chunk_idx):
    """Workload 5 at its own geometry where its precision is tightest: the
    first and last pulses of the 9.6 s dwell (|t_p| = 4.82 s, so each facet
    has drifted by V t_p from its position at t = 0), all 3 channels, on the
    first chunk and on the far-corner chunk of the 16 km x 8 km scene."""
    wl = W.workload(5)
    g = wl.geometry
    c = wl.chunks[chunk_idx]
    sim = hs.Simulator(g)
    say(f"case: workload 5, chunk {chunk_idx} {c}, dwell-end pulses, 3 channels")
    fo = oracle_chunk_facets(wl.sea, wl.seed, [c])
    for p0 in (0, g.n_pulses - 2):
        rc = sim.stream_forward(wl.sea, wl.seed, [c], wl.block_edge, p0, 2).cpu().numpy()
        ref = O.forward(g, fo, p0, 2)
        e = O.rel_l2(rc, ref)
        say(f"chunk {chunk_idx}, pulses {p0}..{p0 + 1}: rel-L2 {e:.3e}")
        assert e < IQ_TOL and e < IQ_BUDGET
        for ch in range(g.n_channels):
            ec = O.rel_l2(rc[ch], ref[ch])
            say(f"  channel {ch}: rel-L2 {ec:.3e}")
            assert ec < IQ_TOL


def test_streamed_workload5_velocity_adjoint_dwell_ends(hs):
    """The streamed velocity adjoint of workload 5 at its own geometry:
    32 pulses at each end of the dwell, all 3 channels, on a whole 8e6-facet
    chunk; dL/dV of 256 seed-drawn facets of the chunk against the FP64
    oracle adjoint of those facets alone (a facet's gradient depends only on
    itself and g)."""
    import torch
    wl = W.workload(5)
    g = wl.geometry
    sim = hs.Simulator(g)
    rng = np.random.default_rng(55)
    npl = 32
    for chunk_idx, p0 in ((0, g.n_pulses - npl), (15, 0)):
        c = wl.chunks[chunk_idx]
        say(f"case: workload 5 adjoint, chunk {chunk_idx} {c}, pulses [{p0}, {p0 + npl})")
        gi = (rng.standard_normal((g.n_channels, npl, g.n_samples))
              + 1j * rng.standard_normal((g.n_channels, npl, g.n_samples))).astype(np.complex64)
        gr = sim.stream_backward(wl.sea, wl.seed, [c], torch.from_numpy(gi).cuda(),
                                 wl.block_edge, p0, npl)
        sel = np.sort(rng.choice(c[2] * c[3], 256, replace=False))
        parts = [O.generate_facets(wl.sea, wl.seed, c[0] + int(s) % c[2], c[1] + int(s) // c[2],
                                   1, 1) for s in sel]
        fo = {k: np.concatenate([q[k] for q in parts]).astype(np.float32).astype(np.float64)
              for k in parts[0]}
        ref = O.adjoint(g, fo, gi.astype(np.complex128), p0, npl)
        for k in ("vx", "vy", "vz"):
            e = O.rel_l2(gr[k].cpu().numpy()[sel], ref[k])
            say(f"  dL/d{k}: rel-L2 {e:.3e}")
            assert e < GRAD_TOL


def grid_index(sea, chunks):
    """Grid index (iy * nx + ix) of every facet, chunk after chunk, each chunk
    row-major in its sub-rectangle."""
    out = []
    for ix0, iy0, cnx, cny in chunks:
        iy, ix = np.divmod(np.arange(cnx * cny), cnx)
        out.append((iy0 + iy) * sea.nx + ix0 + ix)
    return np.concatenate(out)


def test_stream_speckle_matches_whole_scene(hs):
    """Streamed speckle: facet ids and Doppler follow the grid index, so
    unequal chunks give the oracle's speckle sum of the whole scene and the
    same lines as one chunk or one non-streamed plan; adjoint w.r.t. V."""
    import torch
    say("case: streamed speckle, 3 unequal chunks of a 90x70 @1 m scene, 3 channels, "
        "pulses [37, 137)")
    g = W.harmony_geometry(160, 512, receivers="A", n_pc=3)
    sea = W.wave_sea(90, 70, 1.0, seed=9, current_speed=0.3)
    chunks = [(0, 0, 50, 30), (50, 0, 40, 30), (0, 30, 90, 40)]
    sp = W.Speckle(tau_s=0.02, seed=5, first_index=1000)
    fs_grid = W.speckle_doppler(sea.nx * sea.ny, 9)
    fsd = torch.from_numpy(fs_grid).cuda()
    p0, npl = 37, 100
    sim = hs.Simulator(g)
    rc = sim.stream_forward(sea, 9, chunks, 8.0, p0, npl, speckle=sp, f_s=fsd)
    torch.cuda.synchronize()
    fo = oracle_chunk_facets(sea, 9, chunks)
    gi = grid_index(sea, chunks)
    ids = (sp.first_index + gi) & 0xFFFFFFFF
    fs = fs_grid[gi].astype(np.float64)
    ref = O.forward(g, fo, p0, npl, speckle=sp, f_s=fs, ids=ids)
    got = rc.cpu().numpy()
    e = O.rel_l2(got, ref)
    moved = O.rel_l2(O.forward(g, fo, p0, npl), ref)
    say(f"streamed speckle rel-L2 {e:.3e} (the speckle moves the result by {moved:.2f})")
    assert e < IQ_TOL and e < 5e-5
    assert moved > 0.5
    one = sim.stream_forward(sea, 9, [(0, 0, sea.nx, sea.ny)], 8.0, p0, npl, speckle=sp,
                             f_s=fsd).cpu().numpy()
    whole = sim.generate(sea, 9)
    plan = sim.plan(whole["x"], whole["y"], 8.0, speckle=True)
    flat = sim.forward(plan, whole, p0, npl, speckle=sp, f_s=fsd).cpu().numpy()
    e1, e2 = O.rel_l2(got, one), O.rel_l2(got, flat)
    say(f"chunked vs one chunk {e1:.2e}, vs one plan {e2:.2e}")
    assert e1 < 1e-5 and e2 < 1e-5
    rng = np.random.default_rng(10)
    gg = (rng.standard_normal(got.shape) + 1j * rng.standard_normal(got.shape)).astype(np.complex64)
    gr = sim.stream_backward(sea, 9, chunks, torch.from_numpy(gg).cuda(), 8.0, p0, npl,
                             speckle=sp, f_s=fsd)
    refg = O.adjoint(g, fo, gg.astype(np.complex128), p0, npl, speckle=sp, f_s=fs, ids=ids)
    for k in ("vx", "vy", "vz"):
        ek = O.rel_l2(gr[k].cpu().numpy(), refg[k])
        say(f"streamed speckle adjoint {k}: rel-L2 {ek:.3e}")
        assert ek < GRAD_TOL
