"""ctypes binding of include/heeps_sim.h (argument marshalling only).

Loads the in-tree libheeps_sim.so.  There is no fallback: if the library is
missing, loading raises, and every entry point runs on the GPU.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libheeps_sim.so")

SIM_OK = 0
SIM_EINVAL = -1
SIM_ENOMEM = -2
SIM_EHIP = -3
SIM_EUNSUPPORTED = -4
MAX_PLATFORMS, MAX_ANTENNAS, MAX_CHANNELS = 8, 8, 16

_d3 = ctypes.c_double * 3
_fp = ctypes.POINTER(ctypes.c_float)


class SimTraj(ctypes.Structure):
    _fields_ = [("p0", _d3), ("v", _d3)]


class SimAntenna(ctypes.Structure):
    _fields_ = [("platform", ctypes.c_int), ("beta_az", ctypes.c_double),
                ("beta_el", ctypes.c_double), ("steer_rate", ctypes.c_double),
                ("pattern", ctypes.POINTER(ctypes.c_float)),
                ("pattern_nu", ctypes.c_int), ("pattern_nv", ctypes.c_int),
                ("pattern_u0", ctypes.c_double), ("pattern_du", ctypes.c_double),
                ("pattern_v0", ctypes.c_double), ("pattern_dv", ctypes.c_double)]


class SimChannel(ctypes.Structure):
    _fields_ = [("tx_antenna", ctypes.c_int), ("rx_antenna", ctypes.c_int),
                ("pc_offset", _d3)]


class SimConfig(ctypes.Structure):
    _fields_ = [
        ("c", ctypes.c_double), ("f0", ctypes.c_double), ("fs", ctypes.c_double),
        ("prf", ctypes.c_double),
        ("n_samples", ctypes.c_int), ("n_pulses", ctypes.c_int), ("n_ref", ctypes.c_int),
        ("kaiser_beta", ctypes.c_double), ("chirp_bw", ctypes.c_double),
        ("chirp_T", ctypes.c_double),
        ("n_platforms", ctypes.c_int), ("platforms", ctypes.POINTER(SimTraj)),
        ("n_antennas", ctypes.c_int), ("antennas", ctypes.POINTER(SimAntenna)),
        ("n_channels", ctypes.c_int), ("channels", ctypes.POINTER(SimChannel)),
        ("rx_exact", ctypes.c_int),
    ]


class SimFacets(ctypes.Structure):
    _fields_ = [("n", ctypes.c_longlong)] + [(k, _fp) for k in
                                              ("x", "y", "z", "vx", "vy", "vz", "a_re", "a_im")]


SimFacetsOut = SimFacets


class SimFacetGrads(ctypes.Structure):
    _fields_ = [("n", ctypes.c_longlong)] + [(k, _fp) for k in
                                              ("dz", "dvx", "dvy", "dvz", "da_re", "da_im")]


class SimSea(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("mode", ctypes.c_int), ("sigma_v", ctypes.c_double),
        ("n_comp", ctypes.c_int),
        ("k_min", ctypes.c_double), ("k_max", ctypes.c_double), ("slope", ctypes.c_double),
        ("hs", ctypes.c_double), ("g", ctypes.c_double),
        ("dirs", ctypes.POINTER(ctypes.c_double)), ("phases", ctypes.POINTER(ctypes.c_double)),
        ("current", ctypes.c_double * 2),
        ("ntx", ctypes.c_int), ("nty", ctypes.c_int),
        ("tile_L", ctypes.c_double), ("tile_x0", ctypes.c_double), ("tile_y0", ctypes.c_double),
        ("node_hs", ctypes.POINTER(ctypes.c_double)),
        ("node_dirs", ctypes.POINTER(ctypes.c_double)),
        ("node_phases", ctypes.POINTER(ctypes.c_double)),
        ("cwm", ctypes.c_int),
    ]


class SimBox(ctypes.Structure):
    _fields_ = [("x_min", ctypes.c_double), ("x_max", ctypes.c_double),
                ("y_min", ctypes.c_double), ("y_max", ctypes.c_double),
                ("z_max", ctypes.c_double), ("v_max", ctypes.c_double)]


SIM_PLAN_SPECKLE = 1


class SimSpeckle(ctypes.Structure):
    _fields_ = [("tau_s", ctypes.c_double), ("seed", ctypes.c_ulonglong),
                ("first_index", ctypes.c_longlong), ("f_s", _fp)]


EXPORTS = ("sim_create", "sim_destroy", "sim_last_error", "sim_device_init", "sim_pulse_info",
           "sim_waveform_info", "sim_workspace_size", "sim_plan_create", "sim_plan_destroy",
           "sim_plan_info", "sim_plan_beyond", "sim_plan_mode", "sim_sea_table_size", "sim_chunk_box",
           "sim_stream_workspace_size",
           "sim_generate_facets", "sim_forward", "sim_apply_waveform",
           "sim_apply_waveform_adjoint", "sim_backward", "sim_stream_forward",
           "sim_stream_backward", "sim_forward_speckle", "sim_backward_speckle",
           "sim_stream_forward_speckle", "sim_stream_backward_speckle",
           "sim_stream_forward_noalloc", "sim_fast_workspace_size", "sim_forward_fast",
           "sim_plan_geometry")

_lib = None


class SimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def load(path: str = LIB_PATH):
    """Load the library (the HIP runtime it needs is the one torch loaded)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it with `python -m paper_2405_09938_amd.build`")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    i, ll = ctypes.c_int, ctypes.c_longlong
    L.sim_create.argtypes = [P(SimConfig), P(vp)]
    L.sim_destroy.argtypes = [vp]
    L.sim_destroy.restype = None
    L.sim_last_error.argtypes = []
    L.sim_last_error.restype = ctypes.c_char_p
    L.sim_pulse_info.argtypes = [vp, i, i, i, P(ctypes.c_double), P(ctypes.c_double)]
    L.sim_waveform_info.argtypes = [vp, P(i), P(i)]
    sz = ctypes.c_size_t
    L.sim_device_init.argtypes = [vp]
    L.sim_workspace_size.argtypes = [vp, ll, P(SimBox), ctypes.c_double, i, P(sz)]
    L.sim_plan_create.argtypes = [vp, vp, vp, ll, P(SimBox), ctypes.c_double, i, vp, sz, vp,
                                  P(vp)]
    L.sim_plan_destroy.argtypes = [vp]
    L.sim_plan_destroy.restype = None
    L.sim_plan_info.argtypes = [vp, P(ll), P(ll), P(ll), P(ll)]
    L.sim_plan_beyond.argtypes = [vp, vp, P(ll)]
    L.sim_plan_mode.argtypes = [vp, P(i), P(ctypes.c_double)]
    L.sim_sea_table_size.argtypes = [P(SimSea), P(sz)]
    L.sim_chunk_box.argtypes = [P(SimSea), i, i, i, i, P(SimBox)]
    L.sim_generate_facets.argtypes = [vp, P(SimSea), ctypes.c_ulonglong, i, i, i, i,
                                      P(SimFacetsOut), vp, sz, vp]
    L.sim_forward.argtypes = [vp, vp, P(SimFacets), i, i, vp, i, vp]
    L.sim_apply_waveform.argtypes = [vp, vp, vp, ll, vp]
    L.sim_apply_waveform_adjoint.argtypes = [vp, vp, vp, ll, vp]
    L.sim_backward.argtypes = [vp, vp, P(SimFacets), i, i, vp, P(SimFacetGrads), i, vp]
    L.sim_forward_speckle.argtypes = [vp, vp, P(SimFacets), P(SimSpeckle), i, i, vp, i, vp]
    L.sim_backward_speckle.argtypes = [vp, vp, P(SimFacets), P(SimSpeckle), i, i, vp,
                                       P(SimFacetGrads), i, vp]
    ip = P(ctypes.c_int)
    L.sim_stream_workspace_size.argtypes = [vp, P(SimSea), ip, i, ctypes.c_double, i, P(sz)]
    L.sim_stream_forward.argtypes = [vp, P(SimSea), ctypes.c_ulonglong, ip, i, ctypes.c_double,
                                     i, i, vp, i, vp, sz, vp]
    L.sim_stream_backward.argtypes = [vp, P(SimSea), ctypes.c_ulonglong, ip, i, ctypes.c_double,
                                      i, i, vp, vp, vp, vp, vp, sz, vp]
    L.sim_stream_forward_speckle.argtypes = [vp, P(SimSea), ctypes.c_ulonglong, ip, i,
                                             ctypes.c_double, P(SimSpeckle), i, i, vp, i, vp, sz,
                                             vp]
    L.sim_stream_backward_speckle.argtypes = [vp, P(SimSea), ctypes.c_ulonglong, ip, i,
                                              ctypes.c_double, P(SimSpeckle), i, i, vp, vp, vp,
                                              vp, vp, sz, vp]
    L.sim_stream_forward_noalloc.argtypes = [vp, P(SimSea), ctypes.c_ulonglong, ip, i,
                                             ctypes.c_double, i, i, vp, i, vp]
    L.sim_fast_workspace_size.argtypes = [vp, i, P(sz)]
    L.sim_plan_geometry.argtypes = [vp, ll, P(SimBox), ctypes.c_double, P(i), P(i), P(i), P(i),
                                    P(i), P(i), P(ctypes.c_double), P(i)]
    L.sim_forward_fast.argtypes = [vp, vp, P(SimFacets), i, ctypes.c_ulonglong, vp, vp, sz, vp]
    for name in EXPORTS:
        if name not in ("sim_destroy", "sim_last_error", "sim_plan_destroy"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(rc: int, what: str):
    if rc != SIM_OK:
        msg = load().sim_last_error().decode(errors="replace")
        raise SimError(rc, f"{what}: {msg}")
