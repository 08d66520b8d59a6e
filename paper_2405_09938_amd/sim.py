"""PyTorch-facing API over the C ABI (include/heeps_sim.h).

PyTorch supplies device memory and the current HIP stream; every step of the
facet sum, its adjoint, the waveform convolution and the facet generation
runs in the library's own gfx950 kernels.  Nothing here computes any part of
the method: functions only marshal arguments, allocate outputs and call the
library.  If the library cannot be loaded, an exception is raised.
"""
from __future__ import annotations

import ctypes
from typing import Dict, Iterable, Optional

import numpy as np
import torch

from . import _native as N

FACET_KEYS = ("x", "y", "z", "vx", "vy", "vz", "a_re", "a_im")
GRAD_KEYS = ("z", "vx", "vy", "vz", "a_re", "a_im")


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _fptr(t: Optional[torch.Tensor]):
    if t is None:
        return ctypes.cast(None, ctypes.POINTER(ctypes.c_float))
    return ctypes.cast(t.data_ptr(), ctypes.POINTER(ctypes.c_float))


def _workspace(nbytes: int, device) -> torch.Tensor:
    """Caller-owned device workspace (torch allocations are 512-byte aligned)."""
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _box(b) -> "N.SimBox":
    """(x_min, x_max, y_min, y_max[, z_max, v_max]); missing or zero bounds on
    |z| and |V| take the library's defaults."""
    zv = (float(b[4]), float(b[5])) if len(b) > 4 else (0.0, 0.0)
    return N.SimBox(float(b[0]), float(b[1]), float(b[2]), float(b[3]), *zv)


def _check_f32(t: torch.Tensor, n: int, name: str, device) -> torch.Tensor:
    if t.dtype != torch.float32 or t.device != device or t.numel() != n:
        raise ValueError(f"{name}: need a float32 tensor of {n} elements on {device}")
    return t.contiguous()


class Simulator:
    """One acquisition (geometry, antennas, channels, waveform) on one GPU.

    ``geometry`` is any object with the attributes f0, fs, prf, n_samples,
    n_pulses, n_ref, kaiser_beta, chirp_bw, chirp_T, c and the sequences
    platforms (p0, v), antennas (platform, beta_az, beta_el) and channels
    (tx, rx, pc_offset).
    """

    def __init__(self, geometry):
        self.lib = N.load()
        self.device = torch.device("cuda", torch.cuda.current_device())
        g = geometry
        self._plats = (N.SimTraj * len(g.platforms))()
        for i, p in enumerate(g.platforms):
            self._plats[i].p0 = N._d3(*p.p0)
            self._plats[i].v = N._d3(*p.v)
        self._ants = (N.SimAntenna * len(g.antennas))()
        pat_keep = []      # gridded patterns (sim_create copies them)
        self._pat_keep = pat_keep
        for i, a in enumerate(g.antennas):
            self._ants[i] = N.SimAntenna(a.platform, a.beta_az, a.beta_el,
                                         float(getattr(a, "steer_rate", 0.0)))
            pat = getattr(a, "pattern", None)
            if pat is not None:
                vals = np.ascontiguousarray(pat.values, dtype=np.float32)
                if vals.ndim != 2:
                    raise ValueError("pattern values must be a 2-D [nv, nu] array")
                pat_keep.append(vals)
                ant = self._ants[i]
                ant.pattern = vals.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
                ant.pattern_nv, ant.pattern_nu = vals.shape
                ant.pattern_u0, ant.pattern_du = float(pat.u0), float(pat.du)
                ant.pattern_v0, ant.pattern_dv = float(pat.v0), float(pat.dv)
        self._chans = (N.SimChannel * len(g.channels))()
        for i, ch in enumerate(g.channels):
            self._chans[i] = N.SimChannel(ch.tx, ch.rx, N._d3(*ch.pc_offset))
        cfg = N.SimConfig()
        cfg.c, cfg.f0, cfg.fs, cfg.prf = g.c, g.f0, g.fs, g.prf
        cfg.n_samples, cfg.n_pulses, cfg.n_ref = g.n_samples, g.n_pulses, g.n_ref
        cfg.kaiser_beta, cfg.chirp_bw, cfg.chirp_T = g.kaiser_beta, g.chirp_bw, g.chirp_T
        cfg.n_platforms, cfg.platforms = len(g.platforms), self._plats
        cfg.n_antennas, cfg.antennas = len(g.antennas), self._ants
        cfg.n_channels, cfg.channels = len(g.channels), self._chans
        cfg.rx_exact = 1 if getattr(g, "rx_exact", False) else 0
        h = ctypes.c_void_p()
        N.check(self.lib.sim_create(ctypes.byref(cfg), ctypes.byref(h)), "sim_create")
        self.handle = h
        self.n_channels = len(g.channels)
        self.n_samples = g.n_samples
        self.n_pulses = g.n_pulses
        L, M = ctypes.c_int(), ctypes.c_int()
        N.check(self.lib.sim_waveform_info(h, ctypes.byref(L), ctypes.byref(M)),
                "sim_waveform_info")
        self.chirp_len, self.fft_len = L.value, M.value

    def close(self):
        if getattr(self, "handle", None):
            self.lib.sim_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- metadata ----------------------------------------------------------
    def pulse_info(self, ch: int, p0: int = 0, np_: Optional[int] = None):
        np_ = self.n_pulses - p0 if np_ is None else np_
        t = np.zeros(np_)
        tau = np.zeros(np_)
        dp = ctypes.POINTER(ctypes.c_double)
        N.check(self.lib.sim_pulse_info(self.handle, ch, p0, np_, t.ctypes.data_as(dp),
                                        tau.ctypes.data_as(dp)), "sim_pulse_info")
        return t, tau

    # -- facets ------------------------------------------------------------
    def _facets_struct(self, facets: Dict[str, torch.Tensor], n: int):
        keep = [_check_f32(facets[k], n, k, self.device) for k in FACET_KEYS]
        s = N.SimFacets(n, *[_fptr(t) for t in keep])
        return s, keep

    def device_init(self):
        """Upload the handle's constant tables (the one synchronising set-up step)."""
        N.check(self.lib.sim_device_init(self.handle), "sim_device_init")

    def workspace_size(self, n: int, box, block_edge: float = 8.0, speckle: bool = False) -> int:
        b = ctypes.c_size_t()
        bx = _box(box)
        N.check(self.lib.sim_workspace_size(self.handle, int(n), ctypes.byref(bx),
                                            float(block_edge),
                                            N.SIM_PLAN_SPECKLE if speckle else 0,
                                            ctypes.byref(b)), "sim_workspace_size")
        return b.value

    def plan(self, x: torch.Tensor, y: torch.Tensor, block_edge: float = 8.0, box=None,
             speckle: bool = False) -> "Plan":
        """Plan of the facet set (x, y) in a workspace allocated here.  box =
        (x_min, x_max, y_min, y_max) of the positions (taken from x, y when
        None, which waits for the stream); speckle makes room for the
        intra-facet speckle."""
        n = x.numel()
        x = _check_f32(x, n, "x", self.device)
        y = _check_f32(y, n, "y", self.device)
        if box is None:
            xa, ya = torch.aminmax(x), torch.aminmax(y)
            box = (float(xa.min), float(xa.max), float(ya.min), float(ya.max))
        flags = N.SIM_PLAN_SPECKLE if speckle else 0
        ws = _workspace(self.workspace_size(n, box, block_edge, speckle), self.device)
        bx = _box(box)
        p = ctypes.c_void_p()
        N.check(self.lib.sim_plan_create(self.handle, ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(y.data_ptr()), n, ctypes.byref(bx),
                                         float(block_edge), flags,
                                         ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                         _stream(), ctypes.byref(p)), "sim_plan_create")
        return Plan(self, p, n, ws, tuple(box))

    def chunk_box(self, sea, ix0: int = 0, iy0: int = 0, cnx: Optional[int] = None,
                  cny: Optional[int] = None):
        """Rectangle holding every facet generated for a grid sub-rectangle,
        with bounds on their |z| and |V|: (x_min, x_max, y_min, y_max, z_max,
        v_max)."""
        cnx = sea.nx - ix0 if cnx is None else cnx
        cny = sea.ny - iy0 if cny is None else cny
        s, keep = self._sea_struct(sea)
        bx = N.SimBox()
        N.check(self.lib.sim_chunk_box(ctypes.byref(s), ix0, iy0, cnx, cny, ctypes.byref(bx)),
                "sim_chunk_box")
        return (bx.x_min, bx.x_max, bx.y_min, bx.y_max, bx.z_max, bx.v_max)

    @staticmethod
    def _sea_struct(sea):
        s = N.SimSea()
        s.nx, s.ny, s.dx, s.dy = sea.nx, sea.ny, sea.dx, sea.dy
        s.mode, s.sigma_v, s.n_comp = sea.mode, sea.sigma_v, sea.n_comp
        s.k_min, s.k_max, s.slope, s.hs, s.g = sea.k_min, sea.k_max, sea.slope, sea.hs, sea.g
        keep = []
        if sea.mode == 1:
            d = np.ascontiguousarray(sea.dirs, np.float64)
            ph = np.ascontiguousarray(sea.phases, np.float64)
            keep = [d, ph]
            dp = ctypes.POINTER(ctypes.c_double)
            s.dirs, s.phases = d.ctypes.data_as(dp), ph.ctypes.data_as(dp)
        if sea.mode == 2:
            dp = ctypes.POINTER(ctypes.c_double)
            hs_ = np.ascontiguousarray(sea.node_hs, np.float64).ravel()
            d = np.ascontiguousarray(sea.node_dirs, np.float64).ravel()
            ph = np.ascontiguousarray(sea.node_phases, np.float64).ravel()
            keep = [hs_, d, ph]
            s.ntx, s.nty = sea.ntx, sea.nty
            s.tile_L, s.tile_x0, s.tile_y0 = sea.tile_L, sea.tile_x0, sea.tile_y0
            s.node_hs, s.node_dirs, s.node_phases = (hs_.ctypes.data_as(dp), d.ctypes.data_as(dp),
                                                     ph.ctypes.data_as(dp))
        s.cwm = 1 if getattr(sea, "cwm", False) else 0
        s.current[0], s.current[1] = sea.current
        return s, keep

    def generate(self, sea, seed: int, ix0: int = 0, iy0: int = 0, cnx: Optional[int] = None,
                 cny: Optional[int] = None) -> Dict[str, torch.Tensor]:
        """Facets of the grid sub-rectangle [ix0, ix0+cnx) x [iy0, iy0+cny)."""
        cnx = sea.nx - ix0 if cnx is None else cnx
        cny = sea.ny - iy0 if cny is None else cny
        n = cnx * cny
        out = {k: torch.empty(n, dtype=torch.float32, device=self.device) for k in FACET_KEYS}
        s, keep = self._sea_struct(sea)
        b = ctypes.c_size_t()
        N.check(self.lib.sim_sea_table_size(ctypes.byref(s), ctypes.byref(b)), "sim_sea_table_size")
        ws = _workspace(b.value, self.device)
        fo = N.SimFacetsOut(n, *[_fptr(out[k]) for k in FACET_KEYS])
        N.check(self.lib.sim_generate_facets(self.handle, ctypes.byref(s), int(seed), ix0, iy0,
                                             cnx, cny, ctypes.byref(fo),
                                             ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                             _stream()),
                "sim_generate_facets")
        del keep
        return out

    # -- streamed scenes (chunks generated, planned and summed in the library)
    @staticmethod
    def _chunk_array(chunks):
        flat = [int(v) for c in chunks for v in c]
        return (ctypes.c_int * len(flat))(*flat), len(chunks)

    def stream_workspace_size(self, sea, chunks, block_edge: float = 8.0,
                              speckle: bool = False) -> int:
        s, keep = self._sea_struct(sea)
        ca, nc = self._chunk_array(chunks)
        b = ctypes.c_size_t()
        N.check(self.lib.sim_stream_workspace_size(self.handle, ctypes.byref(s), ca, nc,
                                                   float(block_edge),
                                                   N.SIM_PLAN_SPECKLE if speckle else 0,
                                                   ctypes.byref(b)),
                "sim_stream_workspace_size")
        return b.value

    def _stream_ws(self, sea, chunks, block_edge, speckle, workspace):
        need = self.stream_workspace_size(sea, chunks, block_edge, speckle)
        if workspace is None:
            workspace = _workspace(need, self.device)
        elif workspace.numel() < need or workspace.device != self.device:
            raise ValueError(f"workspace needs {need} bytes on {self.device}")
        return workspace

    def stream_forward(self, sea, seed: int, chunks, block_edge: float = 8.0, p0: int = 0,
                       np_: Optional[int] = None, out: Optional[torch.Tensor] = None,
                       accumulate: bool = False, speckle=None,
                       f_s: Optional[torch.Tensor] = None,
                       workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
        """IQ_rc of the scene made of `chunks` = [(ix0, iy0, cnx, cny), ...];
        with `speckle` the intra-facet speckle sum, facet ids and f_s (float32
        device [ny * nx] or None) taken by grid index.  workspace: uint8
        device tensor of at least stream_workspace_size bytes (allocated here
        when None)."""
        np_ = self.n_pulses - p0 if np_ is None else np_
        shape = (self.n_channels, np_, self.n_samples)
        if out is None:
            out = torch.empty(shape, dtype=torch.complex64, device=self.device)
            accumulate = False
        elif out.shape != shape or out.dtype != torch.complex64 or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous complex64 tensor of shape {shape}")
        ws = self._stream_ws(sea, chunks, block_edge, speckle is not None, workspace)
        wsp, wsn = ctypes.c_void_p(ws.data_ptr()), ws.numel()
        s, keep = self._sea_struct(sea)
        ca, nc = self._chunk_array(chunks)
        if speckle is None:
            N.check(self.lib.sim_stream_forward(self.handle, ctypes.byref(s), int(seed), ca, nc,
                                                float(block_edge), p0, np_,
                                                ctypes.c_void_p(out.data_ptr()),
                                                int(accumulate), wsp, wsn, _stream()),
                    "sim_stream_forward")
        else:
            sp, f_keep = self._speckle_struct(speckle, f_s, int(sea.nx) * int(sea.ny))
            N.check(self.lib.sim_stream_forward_speckle(
                self.handle, ctypes.byref(s), int(seed), ca, nc, float(block_edge),
                ctypes.byref(sp), p0, np_, ctypes.c_void_p(out.data_ptr()), int(accumulate),
                wsp, wsn, _stream()), "sim_stream_forward_speckle")
        return out

    def stream_backward(self, sea, seed: int, chunks, g_rc: torch.Tensor,
                        block_edge: float = 8.0, p0: int = 0,
                        np_: Optional[int] = None, speckle=None,
                        f_s: Optional[torch.Tensor] = None,
                        workspace: Optional[torch.Tensor] = None) -> Dict[str, torch.Tensor]:
        """dL/dV of every facet of the streamed scene, chunk after chunk
        (speckle, f_s and workspace as in stream_forward)."""
        np_ = self.n_pulses - p0 if np_ is None else np_
        shape = (self.n_channels, np_, self.n_samples)
        if g_rc.shape != shape or g_rc.dtype != torch.complex64:
            raise ValueError(f"g_rc must be complex64 of shape {shape}")
        g_rc = g_rc.contiguous()
        n = sum(int(c[2]) * int(c[3]) for c in chunks)
        out = {k: torch.empty(n, dtype=torch.float32, device=self.device)
               for k in ("vx", "vy", "vz")}
        ws = self._stream_ws(sea, chunks, block_edge, speckle is not None, workspace)
        wsp, wsn = ctypes.c_void_p(ws.data_ptr()), ws.numel()
        s, keep = self._sea_struct(sea)
        ca, nc = self._chunk_array(chunks)
        outs = [ctypes.c_void_p(out[k].data_ptr()) for k in ("vx", "vy", "vz")]
        if speckle is None:
            N.check(self.lib.sim_stream_backward(self.handle, ctypes.byref(s), int(seed), ca, nc,
                                                 float(block_edge), p0, np_,
                                                 ctypes.c_void_p(g_rc.data_ptr()), *outs,
                                                 wsp, wsn, _stream()), "sim_stream_backward")
        else:
            sp, f_keep = self._speckle_struct(speckle, f_s, int(sea.nx) * int(sea.ny))
            N.check(self.lib.sim_stream_backward_speckle(
                self.handle, ctypes.byref(s), int(seed), ca, nc, float(block_edge),
                ctypes.byref(sp), p0, np_, ctypes.c_void_p(g_rc.data_ptr()), *outs, wsp, wsn,
                _stream()), "sim_stream_backward_speckle")
        return out

    # -- the facet sum and its adjoint -----------------------------------------
    def _speckle_struct(self, speckle, f_s: Optional[torch.Tensor], n: int):
        """C description of the intra-facet speckle (speckle: an object with
        tau_s, seed and first_index, e.g. workloads.Speckle; f_s: float32
        device [n] Doppler in Hz, or None)."""
        if f_s is not None:
            f_s = _check_f32(f_s, n, "f_s", self.device)
        sp = N.SimSpeckle(float(speckle.tau_s), int(speckle.seed), int(speckle.first_index),
                          _fptr(f_s))
        return sp, f_s

    def forward(self, plan: "Plan", facets: Dict[str, torch.Tensor], p0: int = 0,
                np_: Optional[int] = None, out: Optional[torch.Tensor] = None,
                accumulate: bool = False, speckle=None,
                f_s: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Range-compressed IQ, complex64 [C, np, N]; with `speckle` (and the
        per-facet Doppler f_s) the intra-facet speckle sum."""
        np_ = self.n_pulses - p0 if np_ is None else np_
        fs, keep = self._facets_struct(facets, plan.n)
        shape = (self.n_channels, np_, self.n_samples)
        if out is None:
            out = torch.empty(shape, dtype=torch.complex64, device=self.device)
            accumulate = False
        elif out.shape != shape or out.dtype != torch.complex64 or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous complex64 tensor of shape {shape}")
        if speckle is None:
            N.check(self.lib.sim_forward(self.handle, plan.ptr, ctypes.byref(fs), p0, np_,
                                         ctypes.c_void_p(out.data_ptr()), int(accumulate),
                                         _stream()), "sim_forward")
        else:
            sp, f_keep = self._speckle_struct(speckle, f_s, plan.n)
            N.check(self.lib.sim_forward_speckle(self.handle, plan.ptr, ctypes.byref(fs),
                                                 ctypes.byref(sp), p0, np_,
                                                 ctypes.c_void_p(out.data_ptr()),
                                                 int(accumulate), _stream()),
                    "sim_forward_speckle")
        return out

    def forward_fast(self, plan: "Plan", facets: Dict[str, torch.Tensor], n_fast: int,
                     seed: int, out: Optional[torch.Tensor] = None,
                     workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Fast-mode IQ_rc [C, N_p, N] over the whole acquisition: windows of 64
        full-rate pulses every n_fast pulses, the pulses in between generated
        from the windows' Doppler spectra (sim_forward_fast)."""
        fs, keep = self._facets_struct(facets, plan.n)
        shape = (self.n_channels, self.n_pulses, self.n_samples)
        if out is None:
            out = torch.empty(shape, dtype=torch.complex64, device=self.device)
        elif out.shape != shape or out.dtype != torch.complex64 or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous complex64 tensor of shape {shape}")
        b = ctypes.c_size_t()
        N.check(self.lib.sim_fast_workspace_size(self.handle, int(n_fast), ctypes.byref(b)),
                "sim_fast_workspace_size")
        if workspace is None:
            workspace = _workspace(b.value, self.device)
        elif workspace.numel() < b.value:
            raise ValueError(f"workspace needs {b.value} bytes")
        N.check(self.lib.sim_forward_fast(self.handle, plan.ptr, ctypes.byref(fs), int(n_fast),
                                          int(seed), ctypes.c_void_p(out.data_ptr()),
                                          ctypes.c_void_p(workspace.data_ptr()),
                                          workspace.numel(), _stream()), "sim_forward_fast")
        return out

    def backward(self, plan: "Plan", facets: Dict[str, torch.Tensor], g_rc: torch.Tensor,
                 p0: int = 0, np_: Optional[int] = None,
                 need: Iterable[str] = GRAD_KEYS, speckle=None,
                 f_s: Optional[torch.Tensor] = None) -> Dict[str, torch.Tensor]:
        """Facet gradients from g = dL/dRe(IQ_rc) + j dL/dIm(IQ_rc)."""
        np_ = self.n_pulses - p0 if np_ is None else np_
        fs, keep = self._facets_struct(facets, plan.n)
        shape = (self.n_channels, np_, self.n_samples)
        if g_rc.shape != shape or g_rc.dtype != torch.complex64:
            raise ValueError(f"g_rc must be complex64 of shape {shape}")
        g_rc = g_rc.contiguous()
        need = set(need)
        out = {k: torch.empty(plan.n, dtype=torch.float32, device=self.device)
               for k in GRAD_KEYS if k in need}
        gs = N.SimFacetGrads(plan.n, *[_fptr(out.get(k)) for k in GRAD_KEYS])
        if speckle is None:
            N.check(self.lib.sim_backward(self.handle, plan.ptr, ctypes.byref(fs), p0, np_,
                                          ctypes.c_void_p(g_rc.data_ptr()), ctypes.byref(gs),
                                          0, _stream()), "sim_backward")
        else:
            sp, f_keep = self._speckle_struct(speckle, f_s, plan.n)
            N.check(self.lib.sim_backward_speckle(self.handle, plan.ptr, ctypes.byref(fs),
                                                  ctypes.byref(sp), p0, np_,
                                                  ctypes.c_void_p(g_rc.data_ptr()),
                                                  ctypes.byref(gs), 0, _stream()),
                    "sim_backward_speckle")
        return out

    def apply_waveform(self, iq: torch.Tensor, out: Optional[torch.Tensor] = None,
                       adjoint: bool = False) -> torch.Tensor:
        if iq.dtype != torch.complex64 or iq.shape[-1] != self.n_samples:
            raise ValueError("iq must be complex64 [..., N]")
        iq = iq.contiguous()
        out = torch.empty_like(iq) if out is None else out
        n_lines = iq.numel() // self.n_samples
        fn = self.lib.sim_apply_waveform_adjoint if adjoint else self.lib.sim_apply_waveform
        N.check(fn(self.handle, ctypes.c_void_p(iq.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                   n_lines, _stream()), "sim_apply_waveform")
        return out


class Plan:
    """Block decomposition of one facet set (depends on x, y only); its
    device buffers are the workspace tensor it holds."""

    def __init__(self, sim: Simulator, ptr: ctypes.c_void_p, n: int, workspace: torch.Tensor,
                 box):
        self.sim, self.ptr, self.n, self.workspace, self.box = sim, ptr, n, workspace, box
        c = ctypes.c_longlong()
        N.check(sim.lib.sim_plan_info(ptr, None, None, ctypes.byref(c), None), "sim_plan_info")
        self.n_strips = c.value          # range strips per band and channel (a bound)
        m, bound = ctypes.c_int(), ctypes.c_double()
        N.check(sim.lib.sim_plan_mode(ptr, ctypes.byref(m), ctypes.byref(bound)), "sim_plan_mode")
        # elevation factors taken at block centres (error bound el_bound)
        self.el_const, self.el_bound = bool(m.value), bound.value

    def _counts(self):
        b, o = ctypes.c_longlong(), ctypes.c_longlong()
        N.check(self.sim.lib.sim_plan_info(self.ptr, None, ctypes.byref(b), None,
                                           ctypes.byref(o)), "sim_plan_info")
        return b.value, o.value

    @property
    def n_blocks(self) -> int:
        """Number of blocks (read back from the device: waits for the plan's stream)."""
        return self._counts()[0]

    @property
    def n_outside(self) -> int:
        """Facets outside the plan's box (read back from the device)."""
        return self._counts()[1]

    def n_beyond(self, stream=None) -> int:
        """Facets of the last forward or backward call (made on `stream`, the
        current stream by default) beyond the plan's bounds on |z| and |V|
        (read back from the device: waits for that stream)."""
        st = torch.cuda.current_stream(self.sim.device) if stream is None else stream
        v = ctypes.c_longlong()
        N.check(self.sim.lib.sim_plan_beyond(self.ptr, ctypes.c_void_p(st.cuda_stream),
                                             ctypes.byref(v)), "sim_plan_beyond")
        return v.value

    def close(self):
        if getattr(self, "ptr", None):
            self.sim.lib.sim_plan_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SimForward(torch.autograd.Function):
    """IQ = sum over facets (optionally convolved with the chirp), with the
    hand-written adjoint as backward.  Differentiable inputs: z, vx, vy, vz,
    a_re, a_im (x, y fix the plan).  Geometry is recomputed in backward; only
    the input tensors are saved."""

    @staticmethod
    def forward(ctx, sim, plan, p0, np_, waveform, speckle, f_s, x, y, z, vx, vy, vz, a_re,
                a_im):
        facets = dict(zip(FACET_KEYS, (x, y, z, vx, vy, vz, a_re, a_im)))
        iq = sim.forward(plan, facets, p0, np_, speckle=speckle, f_s=f_s)
        if waveform:
            iq = sim.apply_waveform(iq, out=iq)
        ctx.sim, ctx.plan, ctx.p0, ctx.np_, ctx.waveform = sim, plan, p0, np_, waveform
        ctx.speckle, ctx.f_s = speckle, f_s
        ctx.save_for_backward(x, y, z, vx, vy, vz, a_re, a_im)
        return iq

    @staticmethod
    def backward(ctx, g):
        sim = ctx.sim
        facets = dict(zip(FACET_KEYS, ctx.saved_tensors))
        g = g.contiguous()
        if ctx.waveform:
            g = sim.apply_waveform(g, adjoint=True)
        need = [k for k, f in zip(GRAD_KEYS, ctx.needs_input_grad[9:]) if f]
        grads = sim.backward(ctx.plan, facets, g, ctx.p0, ctx.np_, need=need,
                             speckle=ctx.speckle, f_s=ctx.f_s) if need else {}
        return (None,) * 9 + tuple(grads.get(k) for k in GRAD_KEYS)


def simulate(sim: Simulator, plan: Plan, facets: Dict[str, torch.Tensor], p0: int = 0,
             np_: Optional[int] = None, waveform: bool = False, speckle=None,
             f_s: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Differentiable facet sum (optionally with the chirp and the intra-facet
    speckle; the speckle inputs are not differentiated)."""
    np_ = sim.n_pulses - p0 if np_ is None else np_
    return SimForward.apply(sim, plan, p0, np_, waveform, speckle, f_s,
                            *[facets[k] for k in FACET_KEYS])
