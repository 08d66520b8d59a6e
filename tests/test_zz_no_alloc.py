"""GPU check of sim_stream_forward_noalloc, the streamed forward that keeps
its facets and plans in the library's fixed device scratch instead of a
caller workspace: through the C ABI, two calls in a row (the second with a
smaller scene, so it runs over what the first left in the scratch) against
sim_stream_forward with a caller workspace, and against the FP64 oracle."""
import ctypes
import sys

import numpy as np
import pytest

import workloads as W
import oracle as O

pytestmark = pytest.mark.gpu

IQ_TOL = 1e-4


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


def test_noalloc_matches_workspace_entry_point(env):
    torch, hs = env
    from paper_2405_09938_amd import _native as N
    lib = N.load()
    g = W.harmony_geometry(96, 1024, receivers="A", n_pc=2, chirp=False)
    sim = hs.Simulator(g)
    sim.device_init()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    cases = (
        ("large", W.wave_sea(300, 200, 1.0, seed=21, current_speed=0.5),
         [(0, 0, 300, 120), (0, 120, 300, 80)], 0),
        ("small", W.wave_sea(100, 60, 1.0, seed=22), [(0, 0, 100, 60)], 10),
    )
    for name, sea, chunks, p0 in cases:
        np_ = 96 - p0
        say(f"case: no-alloc streamed forward, {name} scene {sea.nx}x{sea.ny}, "
            f"{len(chunks)} chunks, pulses [{p0}, 96)")
        need = sim.stream_workspace_size(sea, chunks, 8.0)
        assert need <= 96 * 2 ** 20
        s, keep = sim._sea_struct(sea)
        ca, nc = sim._chunk_array(chunks)
        out = torch.full((2, np_, 1024), complex(3.0, -1.0), dtype=torch.complex64, device="cuda")
        N.check(lib.sim_stream_forward_noalloc(sim.handle, ctypes.byref(s), 7, ca, nc, 8.0, p0,
                                               np_, ctypes.c_void_p(out.data_ptr()), 0, stream),
                "sim_stream_forward_noalloc")
        ref = sim.stream_forward(sea, 7, chunks, 8.0, p0, np_)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        e_ws = O.rel_l2(a, b)
        parts = [O.generate_facets(sea, 7, *c) for c in chunks]
        fo = {k: np.concatenate([q[k] for q in parts]).astype(np.float32).astype(np.float64)
              for k in parts[0]}
        e_or = O.rel_l2(a, O.forward(g, fo, p0, np_))
        say(f"{name}: vs sim_stream_forward rel-L2 {e_ws:.3e}, vs FP64 oracle {e_or:.3e}")
        assert e_ws < 1e-5
        assert e_or < IQ_TOL


def test_noalloc_in_passes(env):
    """A call whose workspace would exceed the fixed scratch (2048 pulses x 2
    channels over a 400 m x 400 m scene: 132 MiB) runs with window slots for
    fewer pulse groups, in passes: the same bits as sim_stream_forward with a
    caller workspace (one pass), and the oracle's sums on sampled rows."""
    torch, hs = env
    from paper_2405_09938_amd import _native as N
    lib = N.load()
    g = W.harmony_geometry(2048, 1024, receivers="A", n_pc=2, chirp=False)
    sim = hs.Simulator(g)
    sim.device_init()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    sea = W.wave_sea(400, 400, 1.0, seed=23, current_speed=0.3)
    chunks = [(0, 0, 400, 200), (0, 200, 400, 200)]
    need = sim.stream_workspace_size(sea, chunks, 8.0)
    say(f"case: no-alloc in passes, 400x400 m in 2 chunks, 2048 pulses x 2 ch "
        f"(workspace {need / 2 ** 20:.0f} MiB)")
    assert need > 96 * 2 ** 20
    s, keep = sim._sea_struct(sea)
    ca, nc = sim._chunk_array(chunks)
    out = torch.full((2, 2048, 1024), complex(3.0, -1.0), dtype=torch.complex64, device="cuda")
    N.check(lib.sim_stream_forward_noalloc(sim.handle, ctypes.byref(s), 9, ca, nc, 8.0, 0, 2048,
                                           ctypes.c_void_p(out.data_ptr()), 0, stream),
            "sim_stream_forward_noalloc")
    ref = sim.stream_forward(sea, 9, chunks, 8.0, 0, 2048)
    torch.cuda.synchronize()
    a, b = out.cpu().numpy(), ref.cpu().numpy()
    say(f"max |noalloc - workspace| {np.abs(a - b).max():.3e}")
    assert np.array_equal(a, b)
    parts = [O.generate_facets(sea, 9, *c) for c in chunks]
    fo = {k: np.concatenate([q[k] for q in parts]).astype(np.float32).astype(np.float64)
          for k in parts[0]}
    for p0 in (0, 1023, 2045):
        e = O.rel_l2(a[:, p0:p0 + 3], O.forward(g, fo, p0, 3))
        say(f"rows [{p0}, {p0 + 3}): rel-L2 vs FP64 oracle {e:.3e}")
        assert e < IQ_TOL
