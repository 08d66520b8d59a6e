"""GPU parity of the heterogeneous sea (Sec. III eq. 1, 2) and the Choppy
Wave Model displacement: the library's generator against the oracle's
(within one float32 ulp, as for the homogeneous seas), chunk by chunk, and
the whole path (generate, plan, sum, chirp) on such a scene against the
oracle's own generator and sum."""
import sys
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
import oracle as O

pytestmark = pytest.mark.gpu

FKEYS = ("x", "y", "z", "vx", "vy", "vz", "a_re", "a_im")
IQ_TOL = 1e-4
IQ_BUDGET = 5e-5


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


def ulp_check(got, ref, label):
    for k in FKEYS:
        a = got[k].cpu().numpy()
        b = ref[k].astype(np.float32)
        ulps = np.abs(a.view(np.int32).astype(np.int64) - b.view(np.int32).astype(np.int64))
        say(f"{label} {k}: max ulp diff {int(ulps.max())}, exact {np.mean(ulps == 0):.6f}")
        assert int(np.count_nonzero(ulps > 1)) == 0, k


def test_generator_tiles_and_cwm(env):
    torch, hs = env
    say("case: generator, heterogeneous sea (5x4 tiles of 80 m) with CWM, and mode 1 with CWM")
    sim = hs.Simulator(W.harmony_geometry(4, 64))
    het = W.hetero_sea(300, 200, 1.3, seed=6, tile_L=80.0, current_speed=0.4)
    for sea, seed, sub, label in ((het, 11, (0, 0, 300, 200), "tiles+cwm"),
                                  (het, 11, (37, 50, 120, 90), "tiles+cwm chunk"),
                                  (replace(het, cwm=False), 12, (0, 0, 300, 200), "tiles"),
                                  (replace(W.wave_sea(200, 150, 1.0, seed=3), cwm=True), 13,
                                   (0, 0, 200, 150), "mode 1+cwm")):
        got = sim.generate(sea, seed, *sub)
        ref = O.generate_facets(sea, seed, *sub)
        ulp_check(got, ref, label)


def test_tiles_invalid_lattice_rejected(env):
    torch, hs = env
    sim = hs.Simulator(W.harmony_geometry(4, 64))
    het = W.hetero_sea(100, 100, 1.0, seed=1, tile_L=40.0)
    bad = replace(het, tile_x0=het.tile_x0 + 30.0)      # no longer covers the grid
    with pytest.raises(Exception):
        sim.generate(bad, 1)


def test_tiles_cwm_scene_end_to_end(env):
    """Generate, plan, sum and convolve a heterogeneous CWM scene on both
    sides from the same seed and node draws."""
    torch, hs = env
    say("case: end to end, heterogeneous CWM sea 240x240 @1 m (tiles of 60 m), 128 pulses, chirp")
    g = W.harmony_geometry(128, 1024, chirp=True)
    sea = W.hetero_sea(240, 240, 1.0, seed=8, tile_L=60.0, current_speed=0.3)
    sim = hs.Simulator(g)
    d = sim.generate(sea, 8)
    plan = sim.plan(d["x"], d["y"], 8.0)
    rc = sim.forward(plan, d)
    raw = sim.apply_waveform(rc).cpu().numpy()
    rc = rc.cpu().numpy()
    fo = O.as_float32(O.generate_facets(sea, 8))
    fo = {k: v.astype(np.float64) for k, v in fo.items()}
    ref_rc = O.forward(g, fo)
    ref_raw = O.waveform_fft(g, ref_rc)
    e1, e2 = O.rel_l2(rc, ref_rc), O.rel_l2(raw, ref_raw)
    say(f"tiles+cwm end-to-end rc rel-L2 {e1:.3e}, raw rel-L2 {e2:.3e}")
    assert e1 < IQ_TOL and e2 < IQ_TOL and e1 < IQ_BUDGET
