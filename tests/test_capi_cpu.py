"""CPU-side checks of the C ABI: the library loads, exports every function the
header declares, validates its arguments before touching a device, and its
host-side FP64 geometry (pulse times, echo delays) and waveform sizing agree
with the oracle.  No kernel is launched here."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import workloads as W
import oracle as O

# A stand-in workspace (aligned address, ample size) for checks that fail
# before any device work; nothing is ever written through it here.
WS = ctypes.c_void_p(1 << 20)
WSN = 1 << 40

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "heeps_sim.h")
LIB = os.path.join(ROOT, "paper_2405_09938_amd", "libheeps_sim.so")


@pytest.fixture(scope="module")
def native():
    if not os.path.exists(LIB):
        from paper_2405_09938_amd.build import build
        build()
    from paper_2405_09938_amd import _native as N
    N.load()
    return N


def _config(N, geom):
    plats = (N.SimTraj * len(geom.platforms))()
    for i, p in enumerate(geom.platforms):
        plats[i].p0 = N._d3(*p.p0)
        plats[i].v = N._d3(*p.v)
    ants = (N.SimAntenna * len(geom.antennas))()
    for i, a in enumerate(geom.antennas):
        ants[i] = N.SimAntenna(a.platform, a.beta_az, a.beta_el, a.steer_rate)
    chans = (N.SimChannel * len(geom.channels))()
    for i, ch in enumerate(geom.channels):
        chans[i] = N.SimChannel(ch.tx, ch.rx, N._d3(*ch.pc_offset))
    cfg = N.SimConfig()
    cfg.c, cfg.f0, cfg.fs, cfg.prf = geom.c, geom.f0, geom.fs, geom.prf
    cfg.n_samples, cfg.n_pulses, cfg.n_ref = geom.n_samples, geom.n_pulses, geom.n_ref
    cfg.kaiser_beta, cfg.chirp_bw, cfg.chirp_T = geom.kaiser_beta, geom.chirp_bw, geom.chirp_T
    cfg.n_platforms, cfg.platforms = len(geom.platforms), plats
    cfg.n_antennas, cfg.antennas = len(geom.antennas), ants
    cfg.n_channels, cfg.channels = len(geom.channels), chans
    cfg.rx_exact = 1 if geom.rx_exact else 0
    return cfg, (plats, ants, chans)


def test_exports_match_header(native):
    text = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char \*)\s*(sim_\w+)\s*\(", text, re.M))
    assert declared == set(native.EXPORTS)
    lib = ctypes.CDLL(LIB)
    for name in declared:
        assert hasattr(lib, name), name


def test_create_validates_before_any_device_call(native):
    L = native.load()
    h = ctypes.c_void_p()
    assert L.sim_create(None, ctypes.byref(h)) == native.SIM_EINVAL
    assert b"NULL" in L.sim_last_error()
    g = W.harmony_geometry(8, 64)
    for field, bad in (("n_samples", 1), ("prf", -1.0), ("f0", float("nan")),
                       ("kaiser_beta", 50.0), ("n_ref", 64), ("n_pulses", 0)):
        cfg, keep = _config(native, g)
        setattr(cfg, field, bad)
        assert L.sim_create(ctypes.byref(cfg), ctypes.byref(h)) == native.SIM_EINVAL, field
        assert len(L.sim_last_error()) > 0
    cfg, keep = _config(native, g)
    keep[2][0].rx_antenna = 7
    assert L.sim_create(ctypes.byref(cfg), ctypes.byref(h)) == native.SIM_EINVAL
    # an antenna narrower than kappa/500 rad is refused
    cfg, keep = _config(native, g)
    keep[1][0].beta_az = 1e-4
    assert L.sim_create(ctypes.byref(cfg), ctypes.byref(h)) == native.SIM_EUNSUPPORTED
    # a steering rate must be finite
    cfg, keep = _config(native, g)
    keep[1][0].steer_rate = float("nan")
    assert L.sim_create(ctypes.byref(cfg), ctypes.byref(h)) == native.SIM_EINVAL


def test_create_validates_pattern_grids(native):
    """Gridded patterns: node counts, steps, origin and values are checked by
    sim_create (no device work), a good grid is accepted and copied, and a
    grid lifts the kappa/500 width limit of the analytic pattern."""
    L = native.load()
    g = W.harmony_geometry(8, 64)
    vals = np.ones((5, 7), np.float32)

    def with_grid(v, nu, nv, u0=-0.01, du=0.003, v0=-0.2, dv=0.1, beta_az=None):
        cfg, keep = _config(native, g)
        a = keep[1][0]
        if beta_az is not None:
            a.beta_az = beta_az
        a.pattern = v.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        a.pattern_nu, a.pattern_nv = nu, nv
        a.pattern_u0, a.pattern_du, a.pattern_v0, a.pattern_dv = u0, du, v0, dv
        return cfg, keep

    h = ctypes.c_void_p()
    bad_vals = vals.copy()
    bad_vals[2, 3] = np.nan
    for kw, msg in (({"nu": 1, "nv": 5}, "nodes"), ({"nu": 7, "nv": 1}, "nodes"),
                    ({"nu": 7, "nv": 5, "du": 0.0}, "steps"),
                    ({"nu": 7, "nv": 5, "dv": float("inf")}, "steps"),
                    ({"nu": 7, "nv": 5, "u0": float("nan")}, "origin")):
        cfg, keep = with_grid(vals, **kw)
        assert L.sim_create(ctypes.byref(cfg), ctypes.byref(h)) == native.SIM_EINVAL, kw
        assert msg in L.sim_last_error().decode(), (kw, L.sim_last_error())
    cfg, keep = with_grid(bad_vals, 7, 5)
    assert L.sim_create(ctypes.byref(cfg), ctypes.byref(h)) == native.SIM_EINVAL
    assert "finite" in L.sim_last_error().decode()
    # a table reaching 2^14 cells from u = 0 is refused (FP32 cell coordinates)
    cfg, keep = with_grid(vals, 7, 5, u0=0.5, du=1e-5)
    assert L.sim_create(ctypes.byref(cfg), ctypes.byref(h)) == native.SIM_EUNSUPPORTED
    assert "2^14" in L.sim_last_error().decode()
    # accepted, also for a beam narrower than kappa/500 rad (no sinc argument)
    cfg, keep = with_grid(vals, 7, 5, beta_az=1e-4)
    assert L.sim_create(ctypes.byref(cfg), ctypes.byref(h)) == native.SIM_OK
    L.sim_destroy(h)


def test_entry_points_reject_null(native):
    L = native.load()
    p = ctypes.c_void_p()
    assert L.sim_plan_create(None, None, None, 10, None, 8.0, 0, None, 0, None,
                             ctypes.byref(p)) == native.SIM_EINVAL
    assert L.sim_device_init(None) == native.SIM_EINVAL
    assert L.sim_plan_info(None, None, None, None, None) == native.SIM_EINVAL
    assert L.sim_forward(None, None, None, 0, 1, None, 0, None) == native.SIM_EINVAL
    assert L.sim_backward(None, None, None, 0, 1, None, None, 0, None) == native.SIM_EINVAL
    assert L.sim_apply_waveform(None, None, None, 1, None) == native.SIM_EINVAL
    assert L.sim_plan_mode(None, None, None) == native.SIM_EINVAL
    assert L.sim_forward_speckle(None, None, None, None, 0, 1, None, 0, None) == native.SIM_EINVAL
    assert "speckle is NULL" in L.sim_last_error().decode()
    assert L.sim_backward_speckle(None, None, None, None, 0, 1, None, None, 0,
                                  None) == native.SIM_EINVAL
    sp = native.SimSpeckle(0.02, 1, 0, None)
    assert L.sim_forward_speckle(None, None, None, ctypes.byref(sp), 0, 1, None, 0,
                                 None) == native.SIM_EINVAL
    L.sim_destroy(None)
    L.sim_plan_destroy(None)


def test_host_geometry_matches_oracle(native):
    """The library's FP64 per-pulse geometry (host side) against the oracle."""
    L = native.load()
    g = W.harmony_geometry(300, 256, receivers="AB", n_pc=3, chirp=True)
    cfg, keep = _config(native, g)
    h = ctypes.c_void_p()
    assert L.sim_create(ctypes.byref(cfg), ctypes.byref(h)) == native.SIM_OK
    try:
        dp = ctypes.POINTER(ctypes.c_double)
        for ch in range(g.n_channels):
            t = np.zeros(300)
            tau = np.zeros(300)
            assert L.sim_pulse_info(h, ch, 0, 300, t.ctypes.data_as(dp),
                                    tau.ctypes.data_as(dp)) == native.SIM_OK
            for p in (0, 1, 150, 299):
                to, _, _, tauo = O.pulse_geometry(g, ch, p)
                assert abs(t[p] - to) <= 1e-15 * max(1.0, abs(to))
                assert abs(tau[p] - tauo) <= 1e-15 * tauo
        # pulse range validation
        assert L.sim_pulse_info(h, 0, 250, 100, None, None) == native.SIM_EINVAL
        assert L.sim_pulse_info(h, 6, 0, 1, None, None) == native.SIM_EINVAL
        Lc, M = ctypes.c_int(), ctypes.c_int()
        assert L.sim_waveform_info(h, ctypes.byref(Lc), ctypes.byref(M)) == native.SIM_OK
        assert Lc.value == O.chirp(g).size
        assert M.value == 1 << int(math.ceil(math.log2(256 + Lc.value - 1)))
    finally:
        L.sim_destroy(h)


def test_waveform_sizes_for_workloads(native):
    L = native.load()
    for k, (Lexp, Mexp) in ((2, (2000, 8192)), (3, (2000, 16384))):
        g = W.with_pulses(W.workload(k).geometry, 4)
        cfg, keep = _config(native, g)
        h = ctypes.c_void_p()
        assert L.sim_create(ctypes.byref(cfg), ctypes.byref(h)) == native.SIM_OK
        Lc, M = ctypes.c_int(), ctypes.c_int()
        L.sim_waveform_info(h, ctypes.byref(Lc), ctypes.byref(M))
        assert (Lc.value, M.value) == (Lexp, Mexp)
        L.sim_destroy(h)


def test_stream_entry_points_validate(native):
    """Chunks outside the grid or empty, a NULL sea and a bad pulse range are
    refused before any device work."""
    L = native.load()
    g = W.harmony_geometry(8, 64)
    cfg, keep = _config(native, g)
    h = ctypes.c_void_p()
    assert L.sim_create(ctypes.byref(cfg), ctypes.byref(h)) == native.SIM_OK
    try:
        sea = native.SimSea()
        sea.nx, sea.ny, sea.dx, sea.dy, sea.mode = 100, 50, 1.0, 1.0, 0
        bad = [(90, 0, 20, 10), (0, 0, 0, 10), (-1, 0, 5, 5), (0, 45, 10, 10)]
        for c in bad:
            arr = (ctypes.c_int * 4)(*c)
            rc = L.sim_stream_forward(h, ctypes.byref(sea), 1, arr, 1, 8.0, 0, 8,
                                      ctypes.c_void_p(16), 0, WS, WSN, None)
            assert rc == native.SIM_EINVAL, c
        ok = (ctypes.c_int * 4)(0, 0, 10, 10)
        assert L.sim_stream_forward(h, None, 1, ok, 1, 8.0, 0, 8, ctypes.c_void_p(16), 0,
                                    WS, WSN, None) == native.SIM_EINVAL
        assert L.sim_stream_forward(h, ctypes.byref(sea), 1, ok, 1, 8.0, 4, 8,
                                    ctypes.c_void_p(16), 0, WS, WSN, None) == native.SIM_EINVAL
        assert L.sim_stream_backward(h, ctypes.byref(sea), 1, ok, 0, 8.0, 0, 8, None, None,
                                     None, None, WS, WSN, None) == native.SIM_EINVAL
        # a workspace that is missing, misaligned or too small
        need = ctypes.c_size_t()
        assert L.sim_stream_workspace_size(h, ctypes.byref(sea), ok, 1, 8.0, 0,
                                           ctypes.byref(need)) == native.SIM_OK
        for ws, wsn, msg in ((None, WSN, "NULL"), (ctypes.c_void_p(4096 + 16), WSN, "aligned"),
                             (WS, need.value - 1, "too small")):
            assert L.sim_stream_forward(h, ctypes.byref(sea), 1, ok, 1, 8.0, 0, 8,
                                        ctypes.c_void_p(16), 0, ws, wsn,
                                        None) == native.SIM_EINVAL
            assert msg in L.sim_last_error().decode(), msg
        # speckle variants: NULL speckle, bad tau_s or first_index, then the
        # stream checks as above
        assert L.sim_stream_forward_speckle(h, ctypes.byref(sea), 1, ok, 1, 8.0, None, 0, 8,
                                            ctypes.c_void_p(16), 0, WS, WSN,
                                            None) == native.SIM_EINVAL
        assert "speckle is NULL" in L.sim_last_error().decode()
        assert L.sim_stream_backward_speckle(h, ctypes.byref(sea), 1, ok, 1, 8.0, None, 0, 8,
                                             ctypes.c_void_p(16), None, None, None,
                                             WS, WSN, None) == native.SIM_EINVAL
        for sp, msg in ((native.SimSpeckle(0.0, 1, 0, None), "tau_s"),
                        (native.SimSpeckle(float("nan"), 1, 0, None), "tau_s"),
                        (native.SimSpeckle(0.02, 1, -1, None), "first_index")):
            assert L.sim_stream_forward_speckle(h, ctypes.byref(sea), 1, ok, 1, 8.0,
                                                ctypes.byref(sp), 0, 8, ctypes.c_void_p(16), 0,
                                                WS, WSN, None) == native.SIM_EINVAL
            assert msg in L.sim_last_error().decode()
            assert L.sim_stream_backward_speckle(h, ctypes.byref(sea), 1, ok, 1, 8.0,
                                                 ctypes.byref(sp), 0, 8, ctypes.c_void_p(16),
                                                 None, None, None, WS, WSN,
                                                 None) == native.SIM_EINVAL
        sp = native.SimSpeckle(0.02, 1, 0, None)
        arr = (ctypes.c_int * 4)(90, 0, 20, 10)
        assert L.sim_stream_forward_speckle(h, ctypes.byref(sea), 1, arr, 1, 8.0,
                                            ctypes.byref(sp), 0, 8, ctypes.c_void_p(16), 0,
                                            WS, WSN, None) == native.SIM_EINVAL
        assert "chunk" in L.sim_last_error().decode()
    finally:
        L.sim_destroy(h)


def test_generate_validates_sea_before_any_device_call(native):
    """Bad sea descriptions (unknown mode, missing arrays, a tile lattice not
    covering the grid, a negative node height) are refused with SIM_EINVAL
    before the device is touched (there is none here: a device call would
    answer SIM_EHIP)."""
    L = native.load()
    g = W.harmony_geometry(8, 64)
    cfg, keep = _config(native, g)
    h = ctypes.c_void_p()
    assert L.sim_create(ctypes.byref(cfg), ctypes.byref(h)) == native.SIM_OK
    try:
        n = 40 * 30
        bufs = [np.zeros(n, np.float32) for _ in range(8)]
        out = native.SimFacetsOut(n, *[b.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
                                       for b in bufs])
        dp = ctypes.POINTER(ctypes.c_double)
        het = W.hetero_sea(40, 30, 2.0, seed=1, tile_L=20.0)
        hs_ = np.ascontiguousarray(het.node_hs, np.float64)
        d = np.ascontiguousarray(het.node_dirs, np.float64).ravel()
        ph = np.ascontiguousarray(het.node_phases, np.float64).ravel()

        def sea2(**kw):
            s = native.SimSea()
            s.nx, s.ny, s.dx, s.dy, s.mode, s.n_comp = 40, 30, 2.0, 2.0, 2, het.n_comp
            s.k_min, s.k_max, s.slope, s.hs, s.g = het.k_min, het.k_max, het.slope, 2.0, 9.81
            s.ntx, s.nty, s.tile_L, s.tile_x0, s.tile_y0 = (het.ntx, het.nty, het.tile_L,
                                                            het.tile_x0, het.tile_y0)
            s.node_hs, s.node_dirs, s.node_phases = (hs_.ctypes.data_as(dp), d.ctypes.data_as(dp),
                                                     ph.ctypes.data_as(dp))
            for k, v in kw.items():
                setattr(s, k, v)
            return s

        def rc(s):
            return L.sim_generate_facets(h, ctypes.byref(s), 1, 0, 0, 40, 30, ctypes.byref(out),
                                         WS, WSN, None)

        assert rc(sea2(mode=3)) == native.SIM_EINVAL
        assert rc(sea2(tile_x0=het.tile_x0 + 5.0)) == native.SIM_EINVAL
        assert b"cover" in L.sim_last_error()
        assert rc(sea2(ntx=0)) == native.SIM_EINVAL
        assert rc(sea2(node_hs=None)) == native.SIM_EINVAL
        assert rc(sea2(n_comp=0)) == native.SIM_EINVAL
        assert rc(sea2(mode=1)) == native.SIM_EINVAL       # mode 1 without dirs, phases
        neg = hs_.copy()
        neg[3] = -1.0
        assert rc(sea2(node_hs=neg.ctypes.data_as(dp))) == native.SIM_EINVAL
        # a valid description passes validation and then needs a device
        assert rc(sea2()) != native.SIM_EINVAL
        # ... and a workspace for its wave table
        tb = ctypes.c_size_t()
        assert L.sim_sea_table_size(ctypes.byref(sea2()), ctypes.byref(tb)) == native.SIM_OK
        assert tb.value >= 8 * 6 * het.n_comp * (het.ntx + 1) * (het.nty + 1)
        assert L.sim_generate_facets(h, ctypes.byref(sea2()), 1, 0, 0, 40, 30, ctypes.byref(out),
                                     None, 0, None) == native.SIM_EINVAL
        assert b"workspace" in L.sim_last_error()
    finally:
        L.sim_destroy(h)


def test_workspace_sizes(native):
    """Workspace size queries (host only): the plan's bytes grow with the
    facet count and the scene rectangle, the speckle flag adds its records and
    anchors, a generated chunk's box holds its cell centres (widened by the
    CWM displacement), and plan creation refuses a missing, misaligned or
    short workspace before any device work."""
    L = native.load()
    g = W.harmony_geometry(256, 512)
    cfg, keep = _config(native, g)
    h = ctypes.c_void_p()
    assert L.sim_create(ctypes.byref(cfg), ctypes.byref(h)) == native.SIM_OK
    try:
        def size(n, box, edge=8.0, flags=0):
            b = ctypes.c_size_t()
            bx = native.SimBox(*box)
            rc = L.sim_workspace_size(h, n, ctypes.byref(bx), edge, flags, ctypes.byref(b))
            return rc, b.value
        rc, s0 = size(4096, (-160.0, 160.0, -160.0, 160.0))
        assert rc == native.SIM_OK
        # permutation + sorted records alone are 36 bytes per facet
        assert s0 >= 36 * 4096
        assert size(8192, (-160.0, 160.0, -160.0, 160.0))[1] > s0
        assert size(4096, (-640.0, 640.0, -640.0, 640.0))[1] > s0
        rc, s1 = size(4096, (-160.0, 160.0, -160.0, 160.0), flags=native.SIM_PLAN_SPECKLE)
        assert rc == native.SIM_OK
        groups = (256 + 63) // 64 + 1
        assert s1 - s0 >= 4097 * (8 + 16 * groups)
        for bad in ((0, (-1.0, 1.0, -1.0, 1.0)), (10, (1.0, -1.0, -1.0, 1.0)),
                    (10, (float("nan"), 1.0, -1.0, 1.0)), (10, (-1.0, float("inf"), -1.0, 1.0))):
            assert size(*bad)[0] == native.SIM_EINVAL, bad
        assert size(10, (-1.0, 1.0, -1.0, 1.0), edge=0.0)[0] == native.SIM_EINVAL
        assert size(10, (-1.0, 1.0, -1.0, 1.0), flags=2)[0] == native.SIM_EINVAL
        # a lattice of more than 2^28 cells
        assert size(10, (-1e6, 1e6, -1e6, 1e6), edge=1.0)[0] == native.SIM_EUNSUPPORTED
        # plan creation: workspace checks come before any device call
        bx = native.SimBox(-160.0, 160.0, -160.0, 160.0)
        p = ctypes.c_void_p()
        fake = ctypes.c_void_p(1 << 24)
        for ws, n_ws, msg in ((None, s0, "NULL"), (ctypes.c_void_p((1 << 24) + 64), s0, "aligned"),
                              (fake, s0 - 1, "too small")):
            assert L.sim_plan_create(h, fake, fake, 4096, ctypes.byref(bx), 8.0, 0, ws, n_ws,
                                     None, ctypes.byref(p)) == native.SIM_EINVAL
            assert msg in L.sim_last_error().decode(), msg
        # generated chunks: the box holds the chunk's cell centres
        sea = W.wave_sea(120, 80, 1.0, seed=5, current_speed=0.5)
        from paper_2405_09938_amd.sim import Simulator   # the binding's struct marshalling
        s, skeep = Simulator._sea_struct(sea)
        b = native.SimBox()
        assert L.sim_chunk_box(ctypes.byref(s), 60, 40, 60, 40, ctypes.byref(b)) == native.SIM_OK
        xs = (np.arange(60, 120) - 59.5) * 1.0
        ys = (np.arange(40, 80) - 39.5) * 1.0
        assert b.x_min <= xs.min() and b.x_max >= xs.max()
        assert b.y_min <= ys.min() and b.y_max >= ys.max()
        assert b.x_max - b.x_min < 59.0 + 0.01 and b.y_max - b.y_min < 39.0 + 0.01
        s.cwm = 1
        bc = native.SimBox()
        assert L.sim_chunk_box(ctypes.byref(s), 60, 40, 60, 40, ctypes.byref(bc)) == native.SIM_OK
        assert bc.x_min < b.x_min - 0.1 and bc.y_max > b.y_max + 0.1
        assert L.sim_chunk_box(ctypes.byref(s), 60, 40, 61, 40, ctypes.byref(bc)) == native.SIM_EINVAL
        # streamed workspace: table + 8 arrays of the largest chunk + its plan
        chunks = (ctypes.c_int * 8)(0, 0, 60, 40, 60, 40, 60, 40)
        ns = ctypes.c_size_t()
        assert L.sim_stream_workspace_size(h, ctypes.byref(s), chunks, 2, 8.0, 0,
                                           ctypes.byref(ns)) == native.SIM_OK
        assert ns.value >= 32 * 2400 + 36 * 2400
    finally:
        L.sim_destroy(h)


def test_noalloc_entry_point_refuses_before_device_work(native):
    """sim_stream_forward_noalloc: a call needing more than its fixed scratch
    even with window slots for one pulse group is refused with the limit in
    the message, and a handle never initialised on a device is refused too
    (its set-up would allocate); both before any device work.  A call that
    fits only with slots for fewer groups is taken."""
    L = native.load()
    g = W.harmony_geometry(8, 64)
    cfg, keep = _config(native, g)
    h = ctypes.c_void_p()
    assert L.sim_create(ctypes.byref(cfg), ctypes.byref(h)) == native.SIM_OK
    try:
        sea = native.SimSea()
        sea.nx, sea.ny, sea.dx, sea.dy, sea.mode, sea.sigma_v = 3000, 1000, 1.0, 1.0, 0, 0.5
        big = (ctypes.c_int * 4)(0, 0, 3000, 1000)        # 3e6 facets in one chunk
        need = ctypes.c_size_t()
        assert L.sim_stream_workspace_size(h, ctypes.byref(sea), big, 1, 8.0, 0,
                                           ctypes.byref(need)) == native.SIM_OK
        assert need.value > 96 * 2 ** 20
        assert L.sim_stream_forward_noalloc(h, ctypes.byref(sea), 1, big, 1, 8.0, 0, 8,
                                            ctypes.c_void_p(16), 0, None) == native.SIM_EINVAL
        msg = L.sim_last_error().decode()
        assert str(96 * 2 ** 20) in msg and "scratch" in msg, msg
        small = (ctypes.c_int * 8)(0, 0, 500, 400, 500, 0, 500, 400)
        assert L.sim_stream_forward_noalloc(h, ctypes.byref(sea), 1, small, 2, 8.0, 0, 8,
                                            ctypes.c_void_p(16), 0, None) == native.SIM_EINVAL
        assert "sim_device_init" in L.sim_last_error().decode()
        assert L.sim_stream_forward_noalloc(None, ctypes.byref(sea), 1, small, 2, 8.0, 0, 8,
                                            ctypes.c_void_p(16), 0, None) == native.SIM_EINVAL
    finally:
        L.sim_destroy(h)
    # a call whose one-pass workspace exceeds the scratch is taken (window
    # slots for fewer pulse groups, summed in passes): refused here only for
    # the missing device set-up
    g = W.harmony_geometry(2048, 1024, receivers="A", n_pc=2)
    cfg, keep = _config(native, g)
    h = ctypes.c_void_p()
    assert L.sim_create(ctypes.byref(cfg), ctypes.byref(h)) == native.SIM_OK
    try:
        from paper_2405_09938_amd.sim import Simulator
        s, skeep = Simulator._sea_struct(W.wave_sea(400, 400, 1.0, seed=23, current_speed=0.3))
        two = (ctypes.c_int * 8)(0, 0, 400, 200, 0, 200, 400, 200)
        need = ctypes.c_size_t()
        assert L.sim_stream_workspace_size(h, ctypes.byref(s), two, 2, 8.0, 0,
                                           ctypes.byref(need)) == native.SIM_OK
        assert need.value > 96 * 2 ** 20
        assert L.sim_stream_forward_noalloc(h, ctypes.byref(s), 1, two, 2, 8.0, 0, 2048,
                                            ctypes.c_void_p(16), 0, None) == native.SIM_EINVAL
        assert "sim_device_init" in L.sim_last_error().decode()
    finally:
        L.sim_destroy(h)


@pytest.mark.parametrize("k", [2, 5])
def test_strip_windows_hold_every_tap(native, k):
    """The plan's range strips (sim_plan_geometry) against the oracle's FP64
    geometry: facets anywhere in a block (random points of the scene, heights
    and speeds in any direction up to the bounds sim_chunk_box derives from
    the sea) at random pulses of random bands (and of the half groups either
    side of a band that a unit of the band can reach) put all 8 taps inside the
    window the forward sum gives their block's strip, so none takes the
    global path.  Workload 2 and a chunk of workload 5 (its 9.6 s dwell: the
    largest drift)."""
    L = native.load()
    wl = W.workload(k)
    g = wl.geometry
    cfg, keep = _config(native, g)
    h = ctypes.c_void_p()
    assert L.sim_create(ctypes.byref(cfg), ctypes.byref(h)) == native.SIM_OK
    try:
        from paper_2405_09938_amd.sim import Simulator
        s, skeep = Simulator._sea_struct(wl.sea)
        sub = wl.chunks[0] if wl.chunks else (0, 0, wl.sea.nx, wl.sea.ny)
        bx = native.SimBox()
        assert L.sim_chunk_box(ctypes.byref(s), *sub, ctypes.byref(bx)) == native.SIM_OK
        n = sub[2] * sub[3]
        v = [ctypes.c_int() for _ in range(6)]
        assert L.sim_plan_geometry(h, n, ctypes.byref(bx), wl.block_edge,
                                   *[ctypes.byref(x) for x in v], None, None) == native.SIM_OK
        win_max, nb, bg, ns, _, _ = [x.value for x in v]
        C = g.n_channels
        bands = np.zeros(nb * C * 3)
        bwin = np.zeros(nb * C, np.int32)
        assert L.sim_plan_geometry(h, n, ctypes.byref(bx), wl.block_edge, None, None, None, None,
                                   None, None,
                                   bands.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   bwin.ctypes.data_as(ctypes.POINTER(ctypes.c_int))) == 0
        bands = bands.reshape(nb, C, 3)
        bwin = bwin.reshape(nb, C)
        assert bwin.max() <= win_max and set(np.unique(bwin)) <= {24, 26, 32, 48, 64}
        if k == 5:   # the long dwell: 24-sample windows mid-dwell, wider at the ends
            assert set(np.unique(bwin)) == {24, 26}
            assert bwin[nb // 2].max() == 24 and bwin[0].min() == 26
        # narrower windows than the widest only for strips of at least 1 sample
        assert np.all(bands[..., 1][bwin < win_max] >= 1.0 - 1e-9)
        assert np.all(bands[..., 1] >= 1.0 - 1e-9)
        fs_c = g.fs / g.c
        n_ref = g.n_ref if g.n_ref >= 0 else g.n_samples // 2
        rng = np.random.default_rng(k)
        edge = wl.block_edge
        worst = -1e9
        for _ in range(400):
            b = int(rng.integers(nb))
            ch = int(rng.integers(C))
            # a unit takes the band of its group's centre pulse, so its
            # lanes reach 32 pulses before the band and 31 after it
            p = int(rng.integers(max(b * bg * 64 - 32, 0),
                                 min((b + 1) * bg * 64 + 32, g.n_pulses)))
            pref = min(b * bg * 64 + bg * 32, g.n_pulses - 1)
            x = rng.uniform(bx.x_min, bx.x_max)
            y = rng.uniform(bx.y_min, bx.y_max)
            xc = (math.floor(x / edge) + 0.5) * edge
            yc = (math.floor(y / edge) + 0.5) * edge
            z = rng.uniform(-bx.z_max, bx.z_max)
            vel = rng.standard_normal(3)
            vel *= rng.uniform(0.0, bx.v_max) / np.linalg.norm(vel)

            def u_at(pp, X):
                t, ptx, prx, tau = O.pulse_geometry(g, ch, pp)
                R = np.linalg.norm(X - ptx) + np.linalg.norm(X - prx)
                return n_ref + (R - g.c * tau) * fs_c, t

            uc, _ = u_at(pref, np.array([xc, yc, 0.0]))
            t_p = O.pulse_geometry(g, ch, p)[0]
            uf, _ = u_at(p, np.array([x, y, z]) + vel * t_p)
            umin, S, margin = bands[b, ch]
            win = int(bwin[b, ch])
            strip = min(max(int(math.floor((uc - umin) / S)), 0), ns - 1)
            lo = math.floor(umin + strip * S - margin) - 3
            first, last = math.floor(uf) - 3, math.floor(uf) + 4
            assert first >= lo and last <= lo + win - 1, (b, ch, p, first, last, lo, win)
            worst = max(worst, lo - first, last - (lo + win - 1))
        print(f"workload {k}: windows {sorted(set(bwin.ravel().tolist()))}, "
              f"tightest tap {-worst} samples inside")
    finally:
        L.sim_destroy(h)


def test_chunk_box_height_and_speed_bounds(native):
    """sim_chunk_box's bounds on |z| and |V| hold for every facet the oracle's
    generator makes (the generator the GPU's is checked against): a wave sea
    with a current, a tiled sea (mode 2) and a flat sea's Gaussian speeds
    (6 sigma_v).  A gross overestimate fails too: each bound within 4x of
    the sample's largest value (the triangle inequality over 64 components
    of random phase gives about 2-3x), 6x in mode 2 (whose four corner
    weights may add up to 2, and whose bound takes the roughest node).  Boxes with negative or non-finite
    bounds are refused, and tighter bounds give fewer, wider strips."""
    L = native.load()
    from paper_2405_09938_amd.sim import Simulator
    cases = [(W.wave_sea(200, 150, 1.0, seed=5, current_speed=0.5), (20, 10, 150, 120)),
             (W.hetero_sea(300, 200, 1.3, seed=6, tile_L=80.0, current_speed=0.4), (0, 0, 300, 200)),
             (W.flat_sea(300, 300, 1.0, sigma_v=0.5), (0, 0, 300, 300))]
    for sea, sub in cases:
        s, keep = Simulator._sea_struct(sea)
        b = native.SimBox()
        assert L.sim_chunk_box(ctypes.byref(s), *sub, ctypes.byref(b)) == native.SIM_OK
        f = O.generate_facets(sea, 3, *sub)
        zmax = float(np.abs(f["z"]).max())
        vmax = float(np.sqrt(f["vx"] ** 2 + f["vy"] ** 2 + f["vz"] ** 2).max())
        print(f"mode {sea.mode}: |z| <= {zmax:.3f} (bound {b.z_max:.3f}), "
              f"|V| <= {vmax:.3f} (bound {b.v_max:.3f})")
        assert zmax <= b.z_max and vmax <= b.v_max
        loose = 6.0 if sea.mode == 2 else 4.0
        assert b.v_max <= loose * vmax
        if sea.mode >= 1:
            assert b.z_max <= loose * zmax
        else:
            assert b.z_max <= 1e-3
    g = W.harmony_geometry(64, 256)
    cfg, keep = _config(native, g)
    h = ctypes.c_void_p()
    assert L.sim_create(ctypes.byref(cfg), ctypes.byref(h)) == native.SIM_OK
    try:
        n = ctypes.c_size_t()
        for zv in ((-1.0, 0.0), (0.0, -0.5), (float("nan"), 1.0), (1.0, float("inf"))):
            bx = native.SimBox(-100.0, 100.0, -100.0, 100.0, *zv)
            assert L.sim_workspace_size(h, 1000, ctypes.byref(bx), 8.0, 0,
                                        ctypes.byref(n)) == native.SIM_EINVAL
            assert "z_max" in L.sim_last_error().decode()
        # tighter bounds: narrower margins, so wider strips (fewer of them)
        def strips(zv):
            bx = native.SimBox(-500.0, 500.0, -500.0, 500.0, *zv)
            v = [ctypes.c_int() for _ in range(6)]
            assert L.sim_plan_geometry(h, 100000, ctypes.byref(bx), 8.0,
                                       *[ctypes.byref(x) for x in v], None,
                                       None) == native.SIM_OK
            return v[3].value
        assert strips((0.5, 0.2)) < strips((0.0, 0.0)) < strips((8.0, 6.0))
    finally:
        L.sim_destroy(h)
