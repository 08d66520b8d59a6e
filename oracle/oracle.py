"""ctypes wrapper of the FP64 oracle (oracle.c) plus NumPy FFT helpers.

TEST INFRASTRUCTURE ONLY (tests/, smoke(), bench.py's cpu_baseline leg).

Inputs are the descriptions of ``workloads`` (geometry, sea, facets); every
quantity the method computes is computed in oracle.c in double precision, or
here with NumPy's FP64 FFT for the waveform convolution of large lines.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB overrides the library path (used to check that the pins fail on
# deliberately broken builds of oracle.c).
_LIB_PATH = os.environ.get("ORACLE_LIB", os.path.join(_HERE, "liboracle.so"))

MAXP, MAXA, MAXC = 8, 8, 16

_d3 = ctypes.c_double * 3


class OgConfig(ctypes.Structure):
    _fields_ = [
        ("c", ctypes.c_double), ("f0", ctypes.c_double), ("fs", ctypes.c_double),
        ("prf", ctypes.c_double),
        ("n_samples", ctypes.c_int), ("n_pulses", ctypes.c_int), ("n_ref", ctypes.c_int),
        ("kaiser_beta", ctypes.c_double), ("chirp_bw", ctypes.c_double),
        ("chirp_T", ctypes.c_double),
        ("n_plat", ctypes.c_int),
        ("plat_p0", _d3 * MAXP), ("plat_v", _d3 * MAXP),
        ("n_ant", ctypes.c_int),
        ("ant_plat", ctypes.c_int * MAXA),
        ("ant_beta_az", ctypes.c_double * MAXA), ("ant_beta_el", ctypes.c_double * MAXA),
        ("n_ch", ctypes.c_int),
        ("ch_tx", ctypes.c_int * MAXC), ("ch_rx", ctypes.c_int * MAXC),
        ("ch_off", _d3 * MAXC),
        ("rx_exact", ctypes.c_int),
        ("ant_steer", ctypes.c_double * MAXA),
        ("ant_grid", ctypes.POINTER(ctypes.c_double) * MAXA),
        ("ant_gnu", ctypes.c_int * MAXA), ("ant_gnv", ctypes.c_int * MAXA),
        ("ant_gu0", ctypes.c_double * MAXA), ("ant_gdu", ctypes.c_double * MAXA),
        ("ant_gv0", ctypes.c_double * MAXA), ("ant_gdv", ctypes.c_double * MAXA),
    ]


class OgSea(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("mode", ctypes.c_int), ("sigma_v", ctypes.c_double),
        ("n_comp", ctypes.c_int),
        ("k_min", ctypes.c_double), ("k_max", ctypes.c_double),
        ("slope", ctypes.c_double), ("hs", ctypes.c_double), ("g", ctypes.c_double),
        ("dirs", ctypes.POINTER(ctypes.c_double)),
        ("phases", ctypes.POINTER(ctypes.c_double)),
        ("cur", ctypes.c_double * 2),
        ("ntx", ctypes.c_int), ("nty", ctypes.c_int),
        ("tile_L", ctypes.c_double), ("tile_x0", ctypes.c_double), ("tile_y0", ctypes.c_double),
        ("node_hs", ctypes.POINTER(ctypes.c_double)),
        ("node_dirs", ctypes.POINTER(ctypes.c_double)),
        ("node_phases", ctypes.POINTER(ctypes.c_double)),
        ("cwm", ctypes.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from .build import build
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        cfgp = P(OgConfig)
        L.og_num_threads.argtypes = []
        L.og_num_threads.restype = ctypes.c_int
        L.og_pulse_time.argtypes = [cfgp, ctypes.c_int]
        L.og_pulse_time.restype = ctypes.c_double
        L.og_pulse_geometry.argtypes = [cfgp, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp]
        L.og_echo_time.argtypes = [cfgp, ctypes.c_int, ctypes.c_int, dp]
        L.og_echo_time.restype = ctypes.c_double
        L.og_kappa.argtypes = []
        L.og_kappa.restype = ctypes.c_double
        L.og_antenna_frame.argtypes = [cfgp, ctypes.c_int, dp, dp, dp]
        L.og_gain.argtypes = [cfgp, ctypes.c_int, dp, dp, dp]
        L.og_gain.restype = ctypes.c_double
        L.og_tap.argtypes = [ctypes.c_double, ctypes.c_double]
        L.og_tap.restype = ctypes.c_double
        L.og_dtap.argtypes = [ctypes.c_double, ctypes.c_double]
        L.og_dtap.restype = ctypes.c_double
        L.og_forward.argtypes = [cfgp, ctypes.c_longlong] + [dp] * 8 + \
            [ctypes.c_int, ctypes.c_int, dp]
        L.og_adjoint.argtypes = [cfgp, ctypes.c_longlong] + [dp] * 8 + \
            [ctypes.c_int, ctypes.c_int, dp] + [dp] * 6
        L.og_chirp_len.argtypes = [cfgp]
        L.og_chirp_len.restype = ctypes.c_int
        L.og_chirp.argtypes = [cfgp, dp]
        L.og_waveform.argtypes = [cfgp, ctypes.c_longlong, dp, dp]
        L.og_waveform_adjoint.argtypes = [cfgp, ctypes.c_longlong, dp, dp]
        u32p = P(ctypes.c_uint32)
        L.og_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.og_philox2x32_10.argtypes = [u32p, ctypes.c_uint32, u32p]
        L.og_speckle_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, dp]
        L.og_speckle_anchors.argtypes = [ctypes.c_double, ctypes.c_int, dp, dp]
        L.og_speckle_groups.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.og_speckle_series.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double,
                                        ctypes.c_int, ctypes.c_int, dp]
        spk_args = [u32p, dp, ctypes.c_double, ctypes.c_uint64]
        L.og_forward_speckle.argtypes = [cfgp, ctypes.c_longlong] + [dp] * 8 + spk_args + \
            [ctypes.c_int, ctypes.c_int, dp]
        L.og_adjoint_speckle.argtypes = [cfgp, ctypes.c_longlong] + [dp] * 8 + spk_args + \
            [ctypes.c_int, ctypes.c_int, dp] + [dp] * 6
        L.og_wave_table.argtypes = [P(OgSea), dp, dp, dp]
        L.og_generate_facets.argtypes = [P(OgSea), ctypes.c_uint64, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int] + [dp] * 8
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_config(geom) -> OgConfig:
    """Marshal a workloads.Geometry into the oracle's C struct."""
    c = OgConfig()
    keep = []
    c._keep = keep          # gridded pattern tables referenced by the struct
    c.c, c.f0, c.fs, c.prf = geom.c, geom.f0, geom.fs, geom.prf
    c.n_samples, c.n_pulses = geom.n_samples, geom.n_pulses
    c.n_ref = geom.ref_sample
    c.kaiser_beta, c.chirp_bw, c.chirp_T = geom.kaiser_beta, geom.chirp_bw, geom.chirp_T
    assert len(geom.platforms) <= MAXP and len(geom.antennas) <= MAXA
    assert len(geom.channels) <= MAXC
    c.n_plat = len(geom.platforms)
    for i, p in enumerate(geom.platforms):
        for k in range(3):
            c.plat_p0[i][k] = p.p0[k]
            c.plat_v[i][k] = p.v[k]
    c.n_ant = len(geom.antennas)
    for i, a in enumerate(geom.antennas):
        c.ant_plat[i] = a.platform
        c.ant_beta_az[i] = a.beta_az
        c.ant_beta_el[i] = a.beta_el
        c.ant_steer[i] = getattr(a, "steer_rate", 0.0)
        pat = getattr(a, "pattern", None)
        if pat is not None:
            vals = np.ascontiguousarray(np.asarray(pat.values).astype(np.float64))
            assert vals.ndim == 2 and vals.shape[0] >= 2 and vals.shape[1] >= 2
            keep.append(vals)
            c.ant_grid[i] = _dptr(vals)
            c.ant_gnv[i], c.ant_gnu[i] = vals.shape
            c.ant_gu0[i], c.ant_gdu[i] = pat.u0, pat.du
            c.ant_gv0[i], c.ant_gdv[i] = pat.v0, pat.dv
    c.n_ch = len(geom.channels)
    for i, ch in enumerate(geom.channels):
        c.ch_tx[i], c.ch_rx[i] = ch.tx, ch.rx
        for k in range(3):
            c.ch_off[i][k] = ch.pc_offset[k]
    c.rx_exact = 1 if getattr(geom, "rx_exact", False) else 0
    return c


_FACET_KEYS = ("x", "y", "z", "vx", "vy", "vz", "a_re", "a_im")


def _facet_arrays(facets: Dict[str, np.ndarray]):
    return [np.ascontiguousarray(facets[k], dtype=np.float64) for k in _FACET_KEYS]


def num_threads() -> int:
    return int(lib().og_num_threads())


def pulse_time(geom, p: int) -> float:
    cfg = make_config(geom)
    return lib().og_pulse_time(ctypes.byref(cfg), p)


def pulse_geometry(geom, ch: int, p: int):
    """(t_p, P_tx(t_p), P_rx(t_p + tau_ref), tau_ref)."""
    cfg = make_config(geom)
    t = np.zeros(1)
    ptx, prx, tau = np.zeros(3), np.zeros(3), np.zeros(1)
    lib().og_pulse_geometry(ctypes.byref(cfg), ch, p, _dptr(t), _dptr(ptx), _dptr(prx),
                            _dptr(tau))
    return float(t[0]), ptx, prx, float(tau[0])


def echo_time(geom, ch: int, p: int, X) -> float:
    """Echo delay of point X with the receiver at the echo's own reception
    time (the fixed point used when geom.rx_exact is set)."""
    cfg = make_config(geom)
    X = np.ascontiguousarray(X, np.float64)
    return lib().og_echo_time(ctypes.byref(cfg), ch, p, _dptr(X))


def kappa() -> float:
    return lib().og_kappa()


def antenna_frame(geom, ant: int):
    cfg = make_config(geom)
    b, az, el = np.zeros(3), np.zeros(3), np.zeros(3)
    lib().og_antenna_frame(ctypes.byref(cfg), ant, _dptr(b), _dptr(az), _dptr(el))
    return b, az, el


def gain(geom, ant: int, pa, x, with_grad: bool = False):
    cfg = make_config(geom)
    pa = np.ascontiguousarray(pa, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    gr = np.zeros(3)
    f = lib().og_gain(ctypes.byref(cfg), ant, _dptr(pa), _dptr(x),
                      _dptr(gr) if with_grad else None)
    return (f, gr) if with_grad else f


def tap(t: float, beta: float) -> float:
    return lib().og_tap(float(t), float(beta))


def dtap(t: float, beta: float) -> float:
    return lib().og_dtap(float(t), float(beta))


def _speckle_args(speckle, n: int, f_s, ids):
    """(ids uint32 [n], f_s float64 [n] or None) of a speckle description."""
    if ids is None:
        ids = (int(speckle.first_index) + np.arange(n, dtype=np.int64)) & 0xFFFFFFFF
    ids = np.ascontiguousarray(ids, np.uint32)
    assert ids.size == n
    fs = None if f_s is None else np.ascontiguousarray(f_s, np.float64)
    assert fs is None or fs.size == n
    return ids, fs


def forward(geom, facets: Dict[str, np.ndarray], p0: int = 0,
            np_: Optional[int] = None, speckle=None, f_s=None, ids=None) -> np.ndarray:
    """Range-compressed IQ, complex128 [C, np, N], pulses [p0, p0 + np).

    speckle (workloads.Speckle, optional): intra-facet speckle of eq. 7 with
    per-facet Doppler f_s (Hz, default 0); facet i draws with counter id
    ids[i] (default speckle.first_index + i)."""
    np_ = geom.n_pulses - p0 if np_ is None else np_
    cfg = make_config(geom)
    arrs = _facet_arrays(facets)
    n = arrs[0].size
    out = np.zeros((geom.n_channels, np_, geom.n_samples, 2), np.float64)
    if speckle is None:
        lib().og_forward(ctypes.byref(cfg), n, *[_dptr(a) for a in arrs], p0, np_,
                         _dptr(out))
    else:
        idv, fs = _speckle_args(speckle, n, f_s, ids)
        lib().og_forward_speckle(ctypes.byref(cfg), n, *[_dptr(a) for a in arrs],
                                 idv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                 None if fs is None else _dptr(fs), float(speckle.tau_s),
                                 int(speckle.seed), p0, np_, _dptr(out))
    return out[..., 0] + 1j * out[..., 1]


def adjoint(geom, facets: Dict[str, np.ndarray], g: np.ndarray, p0: int = 0,
            np_: Optional[int] = None, speckle=None, f_s=None,
            ids=None) -> Dict[str, np.ndarray]:
    """dL/d(z, vx, vy, vz, a_re, a_im) given g = dL/dRe(IQ) + j dL/dIm(IQ)
    (speckle arguments as in ``forward``)."""
    np_ = geom.n_pulses - p0 if np_ is None else np_
    cfg = make_config(geom)
    arrs = _facet_arrays(facets)
    n = arrs[0].size
    g = np.asarray(g, np.complex128)
    assert g.shape == (geom.n_channels, np_, geom.n_samples)
    gi = np.ascontiguousarray(np.stack([g.real, g.imag], -1))
    outs = [np.zeros(n) for _ in range(6)]
    if speckle is None:
        lib().og_adjoint(ctypes.byref(cfg), n, *[_dptr(a) for a in arrs], p0, np_,
                         _dptr(gi), *[_dptr(o) for o in outs])
    else:
        idv, fs = _speckle_args(speckle, n, f_s, ids)
        lib().og_adjoint_speckle(ctypes.byref(cfg), n, *[_dptr(a) for a in arrs],
                                 idv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                 None if fs is None else _dptr(fs), float(speckle.tau_s),
                                 int(speckle.seed), p0, np_, _dptr(gi),
                                 *[_dptr(o) for o in outs])
    return dict(zip(("z", "vx", "vy", "vz", "a_re", "a_im"), outs))


def chirp(geom) -> np.ndarray:
    cfg = make_config(geom)
    L = lib().og_chirp_len(ctypes.byref(cfg))
    out = np.zeros((L, 2))
    lib().og_chirp(ctypes.byref(cfg), _dptr(out))
    return out[:, 0] + 1j * out[:, 1]


def waveform(geom, rc: np.ndarray) -> np.ndarray:
    """Direct O(N L) 'same'-mode convolution of each line with the chirp."""
    cfg = make_config(geom)
    rc = np.asarray(rc, np.complex128)
    shp = rc.shape
    assert shp[-1] == geom.n_samples
    x = np.ascontiguousarray(np.stack([rc.real, rc.imag], -1)).reshape(-1, geom.n_samples, 2)
    y = np.zeros_like(x)
    lib().og_waveform(ctypes.byref(cfg), x.shape[0], _dptr(x), _dptr(y))
    return (y[..., 0] + 1j * y[..., 1]).reshape(shp)


def waveform_adjoint(geom, graw: np.ndarray) -> np.ndarray:
    cfg = make_config(geom)
    graw = np.asarray(graw, np.complex128)
    shp = graw.shape
    x = np.ascontiguousarray(np.stack([graw.real, graw.imag], -1)).reshape(-1, geom.n_samples, 2)
    y = np.zeros_like(x)
    lib().og_waveform_adjoint(ctypes.byref(cfg), x.shape[0], _dptr(x), _dptr(y))
    return (y[..., 0] + 1j * y[..., 1]).reshape(shp)


def waveform_fft(geom, rc: np.ndarray) -> np.ndarray:
    """Same convolution as ``waveform`` via NumPy's FP64 FFT (large lines):
    full linear convolution with the chirp, then samples [L/2, L/2 + N)."""
    ch = chirp(geom)
    L, N = ch.size, geom.n_samples
    M = 1 << int(np.ceil(np.log2(N + L - 1)))
    X = np.fft.fft(np.asarray(rc, np.complex128), M, axis=-1)
    Cf = np.fft.fft(ch, M)
    y = np.fft.ifft(X * Cf, axis=-1)
    return y[..., L // 2: L // 2 + N]


def waveform_adjoint_fft(geom, graw: np.ndarray) -> np.ndarray:
    """Adjoint of ``waveform_fft``: correlation with the chirp."""
    ch = chirp(geom)
    L, N = ch.size, geom.n_samples
    M = 1 << int(np.ceil(np.log2(N + L - 1)))
    pad = np.zeros(graw.shape[:-1] + (M,), np.complex128)
    pad[..., L // 2: L // 2 + N] = graw
    G = np.fft.fft(pad, axis=-1)
    Cf = np.fft.fft(ch, M)
    r = np.fft.ifft(G * np.conj(Cf), axis=-1)
    return r[..., :N]


def philox4x32_10(ctr, key) -> np.ndarray:
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().og_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def philox2x32_10(ctr, key) -> np.ndarray:
    c = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in ctr])
    o = (ctypes.c_uint32 * 2)()
    lib().og_philox2x32_10(c, int(key) & 0xFFFFFFFF, o)
    return np.array(list(o), dtype=np.uint32)


def speckle_draw(seed: int, fid: int, slot: int) -> complex:
    o = np.zeros(2)
    lib().og_speckle_draw(int(seed), int(fid) & 0xFFFFFFFF, int(slot) & 0xFFFFFFFF, _dptr(o))
    return complex(o[0], o[1])


def speckle_anchors(a: float, eta: np.ndarray) -> np.ndarray:
    """Anchors y_0.. from complex draws eta (a = dt / tau_s)."""
    e = np.ascontiguousarray(np.stack([np.real(eta), np.imag(eta)], -1), np.float64)
    y = np.zeros_like(e)
    lib().og_speckle_anchors(float(a), e.shape[0], _dptr(e), _dptr(y))
    return y[:, 0] + 1j * y[:, 1]


def speckle_groups(a: float, g0: int, g1: int, y: np.ndarray, e: np.ndarray) -> np.ndarray:
    """x at pulses 64 g0 .. 64 g1 - 1 from anchors y_{g0..g1} and innovations
    e[64 (g - g0) + k - 1] = e_{64 g + k} (complex arrays)."""
    yy = np.ascontiguousarray(np.stack([np.real(y), np.imag(y)], -1), np.float64)
    ee = np.ascontiguousarray(np.stack([np.real(e), np.imag(e)], -1), np.float64)
    assert yy.shape[0] == g1 - g0 + 1 and ee.shape[0] == 64 * (g1 - g0)
    x = np.zeros((64 * (g1 - g0), 2))
    lib().og_speckle_groups(float(a), g0, g1, _dptr(yy), _dptr(ee), _dptr(x))
    return x[:, 0] + 1j * x[:, 1]


def speckle_series(seed: int, fid: int, a: float, pa: int, pb: int) -> np.ndarray:
    """x(p) of facet id `fid` for absolute pulses [pa, pb)."""
    x = np.zeros((max(pb - pa, 0), 2))
    if pb > pa:
        lib().og_speckle_series(int(seed), int(fid) & 0xFFFFFFFF, float(a), pa, pb, _dptr(x))
    return x[:, 0] + 1j * x[:, 1]


def _make_sea(sea):
    s = OgSea()
    s.nx, s.ny, s.dx, s.dy = sea.nx, sea.ny, sea.dx, sea.dy
    s.mode, s.sigma_v, s.n_comp = sea.mode, sea.sigma_v, sea.n_comp
    s.k_min, s.k_max, s.slope, s.hs, s.g = sea.k_min, sea.k_max, sea.slope, sea.hs, sea.g
    keep = []
    if sea.mode == 1:
        d = np.ascontiguousarray(sea.dirs, np.float64)
        ph = np.ascontiguousarray(sea.phases, np.float64)
        keep = [d, ph]
        s.dirs, s.phases = _dptr(d), _dptr(ph)
    if sea.mode == 2:
        hs = np.ascontiguousarray(sea.node_hs, np.float64).ravel()
        d = np.ascontiguousarray(sea.node_dirs, np.float64).ravel()
        ph = np.ascontiguousarray(sea.node_phases, np.float64).ravel()
        keep = [hs, d, ph]
        s.ntx, s.nty = sea.ntx, sea.nty
        s.tile_L, s.tile_x0, s.tile_y0 = sea.tile_L, sea.tile_x0, sea.tile_y0
        s.node_hs, s.node_dirs, s.node_phases = _dptr(hs), _dptr(d), _dptr(ph)
    s.cwm = 1 if getattr(sea, "cwm", False) else 0
    s.cur[0], s.cur[1] = sea.current
    return s, keep


def wave_table(sea) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    s, keep = _make_sea(sea)
    k, a, w = np.zeros(sea.n_comp), np.zeros(sea.n_comp), np.zeros(sea.n_comp)
    lib().og_wave_table(ctypes.byref(s), _dptr(k), _dptr(a), _dptr(w))
    return k, a, w


def generate_facets(sea, seed: int, ix0: int = 0, iy0: int = 0,
                    cnx: Optional[int] = None, cny: Optional[int] = None
                    ) -> Dict[str, np.ndarray]:
    """FP64 facets of a grid sub-rectangle (see og_generate_facets)."""
    cnx = sea.nx - ix0 if cnx is None else cnx
    cny = sea.ny - iy0 if cny is None else cny
    s, keep = _make_sea(sea)
    n = cnx * cny
    outs = [np.zeros(n) for _ in range(8)]
    lib().og_generate_facets(ctypes.byref(s), seed, ix0, iy0, cnx, cny,
                             *[_dptr(o) for o in outs])
    return dict(zip(_FACET_KEYS, outs))


def as_float32(facets: Dict[str, np.ndarray]) -> Dict[str, np.ndarray]:
    return {k: np.asarray(v, np.float32) for k, v in facets.items()}


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """||a - b|| / ||b||."""
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) /
                 max(np.linalg.norm(np.asarray(b).ravel()), 1e-300))


def loss(iq: np.ndarray, target: np.ndarray) -> float:
    d = iq - target
    return float(np.sum(d.real ** 2 + d.imag ** 2))


def fd_gradient(geom, facets: Dict[str, np.ndarray], target: np.ndarray, idx: int,
                key: str, h: float, p0: int = 0, np_: Optional[int] = None,
                resid: Optional[np.ndarray] = None, speckle=None, f_s=None) -> float:
    """Central finite difference of L = ||IQ - target||^2 w.r.t. facets[key][idx].

    Uses linearity of the sum: with r = IQ - target for all facets, changing
    one facet only changes its own contribution c_i, so
    L(theta) = ||r - c_i(theta0) + c_i(theta)||^2 and each evaluation costs one
    facet's contributions.  With speckle the facet keeps its own counter id
    and Doppler.
    """
    if resid is None:
        resid = forward(geom, facets, p0, np_, speckle, f_s)
        resid = resid - target
    one = {k: np.array([np.float64(v[idx])]) for k, v in facets.items()}
    kw = {}
    if speckle is not None:
        n = next(iter(facets.values())).size
        ids, fs = _speckle_args(speckle, n, f_s, None)
        kw = dict(speckle=speckle, ids=ids[idx:idx + 1],
                  f_s=None if fs is None else fs[idx:idx + 1])
    c0 = forward(geom, one, p0, np_, **kw)
    base = resid - c0
    vals = []
    for s in (+1.0, -1.0):
        o = {k: v.copy() for k, v in one.items()}
        o[key][0] += s * h
        vals.append(loss(base + forward(geom, o, p0, np_, **kw), 0.0))
    return (vals[0] - vals[1]) / (2.0 * h)
