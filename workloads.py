"""Seeded synthetic inputs for the HEEPS/MARE facet-sum path.

This module is shared by the test-side FP64 oracle and by the GPU library's
callers (tests, bench).  It holds *no* arithmetic of the method: only the
acquisition geometry (platform trajectories, antenna widths, channel layout),
grid layouts, sizes and random draws.  Everything the method computes from
these inputs (pulse times, echo delays, ranges, gains, phases, wave spectra,
taps, chirps) lives separately in ``oracle/`` and in the HIP library.

Geometry follows the Harmony ATI formation (Sec. I, Fig. 1): Sentinel-1
transmits from 693 km altitude, the Harmony receivers fly on the same orbit
250 km ahead (and, for the two-receiver case, 250 km behind), and every antenna
points at the same surface target, the scene origin O.  The frame is a flat
local ENU frame at O: x along-track, y ground range away from the Tx track,
z up.  Straight-line trajectories at 7500 m/s.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Dict, List, Optional, Tuple

import numpy as np

C_LIGHT = 299_792_458.0
F0 = 5.405e9            # C-band carrier (Hz)
FS = 50e6               # range sampling rate (Hz)
PRF = 1700.0            # pulse repetition frequency (Hz)
ALT = 693_000.0         # orbit altitude (m)
INCIDENCE_DEG = 35.0    # incidence at the scene origin
V_ORBIT = 7500.0        # platform speed (m/s)
RX_LEAD = 250_000.0     # along-track separation of the Harmony receivers (m)
PC_SPACING = 3.3        # along-track phase-centre spacing on one receiver (m)
BEAM_AZ_DEG = 0.23      # one-way 3-dB azimuth width of the sinc^2 pattern
BEAM_EL_DEG = 15.0      # one-way 3-dB elevation width
KAISER_BETA = 5.653     # 8-tap Kaiser-windowed sinc interpolator
CHIRP_BW = 40e6         # chirp bandwidth (Hz)
CHIRP_T = 40e-6         # chirp duration (s)

# Sea-state description used by the wave-driven configurations.
SEA_N_COMP = 64
SEA_K_MIN = 2 * math.pi / 250.0
SEA_K_MAX = 2 * math.pi / 5.0
SEA_SLOPE = -4.0
SEA_HS = 2.0
SEA_G = 9.81
SEA_DIR_SPREAD_DEG = 25.0

# Intra-facet speckle (Sec. III.A eq. 7, 10).  tau_s = 20 ms is a correlation
# time of the order of the facet Doppler widths of C-band sea echoes (a few
# Hz); the intra-facet Doppler is drawn around +-5.7 Hz, the frequency of the
# first-order Bragg waves at 35 deg incidence, for waves moving towards or
# away from the radar.
SPECKLE_TAU_S = 0.02
SPECKLE_FD_HZ = 5.7
SPECKLE_FD_SPREAD_HZ = 0.5


@dataclass(frozen=True)
class Platform:
    p0: Tuple[float, float, float]      # position at t = 0 (m)
    v: Tuple[float, float, float]       # constant velocity (m/s)


@dataclass(frozen=True)
class Pattern:
    """A field pattern tabulated on a u-v grid (direction cosines on the
    antenna's azimuth and elevation axes): values[j, i] at u = u0 + i du,
    v = v0 + j dv (float32)."""
    u0: float
    du: float
    v0: float
    dv: float
    values: np.ndarray                  # float32 [nv, nu]


@dataclass(frozen=True)
class Antenna:
    platform: int
    beta_az: float                      # one-way 3-dB width in azimuth (rad)
    beta_el: float                      # one-way 3-dB width in elevation (rad)
    steer_rate: float = 0.0             # azimuth steering rate about the el axis (rad/s)
    pattern: Optional[Pattern] = None   # gridded field pattern (None: analytic)


@dataclass(frozen=True)
class Channel:
    tx: int                             # transmitting antenna index
    rx: int                             # receiving antenna index
    pc_offset: Tuple[float, float, float] = (0.0, 0.0, 0.0)  # Rx phase-centre offset (m)


@dataclass(frozen=True)
class Geometry:
    n_pulses: int
    n_samples: int
    platforms: Tuple[Platform, ...]
    antennas: Tuple[Antenna, ...]
    channels: Tuple[Channel, ...]
    f0: float = F0
    fs: float = FS
    prf: float = PRF
    n_ref: int = -1                     # window reference sample; -1 means N/2
    kaiser_beta: float = KAISER_BETA
    chirp_bw: float = 0.0
    chirp_T: float = 0.0                # 0 means range-compressed output only
    c: float = C_LIGHT
    # receiver position: False = at the scene origin's echo time of each
    # pulse (one position per pulse); True = at each facet's own echo time
    rx_exact: bool = False

    @property
    def n_channels(self) -> int:
        return len(self.channels)

    @property
    def ref_sample(self) -> int:
        return self.n_samples // 2 if self.n_ref < 0 else self.n_ref


@dataclass(frozen=True)
class Sea:
    """Sea-surface description for on-device facet generation.

    ``mode`` 0: flat sea, z = 0, velocities N(0, sigma_v^2) per axis.
    ``mode`` 1: 64 linear wave components plus a uniform current.
    ``mode`` 2: heterogeneous sea: square tiles of side ``tile_L`` whose
    corner nodes (``ntx + 1`` x ``nty + 1``, from ``tile_x0, tile_y0``) each
    carry their own significant height, component directions and phases.
    ``cwm``: facets displaced horizontally (Choppy Wave Model).
    Random draws of the method (component directions and phases) are inputs.
    """
    nx: int
    ny: int
    dx: float
    dy: float
    mode: int = 0
    sigma_v: float = 0.5
    n_comp: int = SEA_N_COMP
    k_min: float = SEA_K_MIN
    k_max: float = SEA_K_MAX
    slope: float = SEA_SLOPE
    hs: float = SEA_HS
    g: float = SEA_G
    dirs: Optional[np.ndarray] = None   # [n_comp] propagation directions (rad)
    phases: Optional[np.ndarray] = None  # [n_comp] initial phases (rad)
    current: Tuple[float, float] = (0.0, 0.0)
    ntx: int = 0
    nty: int = 0
    tile_L: float = 0.0
    tile_x0: float = 0.0
    tile_y0: float = 0.0
    node_hs: Optional[np.ndarray] = None      # [(ntx+1)(nty+1)]
    node_dirs: Optional[np.ndarray] = None    # [(ntx+1)(nty+1), n_comp]
    node_phases: Optional[np.ndarray] = None  # [(ntx+1)(nty+1), n_comp]
    cwm: bool = False


def harmony_geometry(n_pulses: int, n_samples: int, receivers: str = "A",
                     n_pc: int = 1, chirp: bool = False) -> Geometry:
    """Tx (Sentinel-1) + receivers 'A' (250 km ahead) and/or 'B' (behind)."""
    yg = ALT * math.tan(math.radians(INCIDENCE_DEG))
    plats = [Platform((0.0, -yg, ALT), (V_ORBIT, 0.0, 0.0))]
    ants = [Antenna(0, math.radians(BEAM_AZ_DEG), math.radians(BEAM_EL_DEG))]
    chans: List[Channel] = []
    for r in receivers:
        lead = RX_LEAD if r == "A" else -RX_LEAD
        plats.append(Platform((lead, -yg, ALT), (V_ORBIT, 0.0, 0.0)))
        ants.append(Antenna(len(plats) - 1, math.radians(BEAM_AZ_DEG),
                            math.radians(BEAM_EL_DEG)))
        if n_pc == 1:
            offs = [0.0]
        else:
            offs = [PC_SPACING * (k - (n_pc - 1) / 2) for k in range(n_pc)]
        for o in offs:
            chans.append(Channel(0, len(ants) - 1, (o, 0.0, 0.0)))
    return Geometry(n_pulses=n_pulses, n_samples=n_samples,
                    platforms=tuple(plats), antennas=tuple(ants),
                    channels=tuple(chans),
                    chirp_bw=CHIRP_BW if chirp else 0.0,
                    chirp_T=CHIRP_T if chirp else 0.0)


def grid_xy(nx: int, ny: int, dx: float, dy: Optional[float] = None,
            ix0: int = 0, iy0: int = 0, gnx: Optional[int] = None,
            gny: Optional[int] = None, cnx: Optional[int] = None,
            cny: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Cell centres of a grid centred on O, row-major (index = iy*nx + ix).

    With (ix0, iy0, cnx, cny) a sub-rectangle of the (gnx, gny) grid is returned.
    """
    dy = dx if dy is None else dy
    gnx = nx if gnx is None else gnx
    gny = ny if gny is None else gny
    cnx = nx if cnx is None else cnx
    cny = ny if cny is None else cny
    ix = np.arange(ix0, ix0 + cnx, dtype=np.float64)
    iy = np.arange(iy0, iy0 + cny, dtype=np.float64)
    xs = (ix - (gnx - 1) / 2.0) * dx
    ys = (iy - (gny - 1) / 2.0) * dy
    X, Y = np.meshgrid(xs, ys)
    return X.ravel().astype(np.float32), Y.ravel().astype(np.float32)


def iid_facets(nx: int, ny: int, dx: float, seed: int, sigma_v: float = 0.5,
               sigma_z: float = 0.0) -> Dict[str, np.ndarray]:
    """Facets on a grid: z ~ N(0, sigma_z^2) (0 = flat sea), V ~ N(0, sigma_v^2)
    per axis, a ~ CN(0, 1) (each component variance 1/2).  float32 SoA."""
    rng = np.random.default_rng(seed)
    x, y = grid_xy(nx, ny, dx)
    n = x.size
    z = (sigma_z * rng.standard_normal(n)).astype(np.float32) if sigma_z > 0 \
        else np.zeros(n, np.float32)
    v = (sigma_v * rng.standard_normal((3, n))).astype(np.float32)
    a = (rng.standard_normal((2, n)) / math.sqrt(2.0)).astype(np.float32)
    return dict(x=x, y=y, z=z, vx=v[0], vy=v[1], vz=v[2], a_re=a[0], a_im=a[1])


def scattered_facets(n: int, half_extent: float, seed: int, sigma_v: float = 0.5,
                     sigma_z: float = 0.5) -> Dict[str, np.ndarray]:
    """Facets at uniformly random positions in a square (not on a grid)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-half_extent, half_extent, n).astype(np.float32)
    y = rng.uniform(-half_extent, half_extent, n).astype(np.float32)
    z = (sigma_z * rng.standard_normal(n)).astype(np.float32)
    v = (sigma_v * rng.standard_normal((3, n))).astype(np.float32)
    a = (rng.standard_normal((2, n)) / math.sqrt(2.0)).astype(np.float32)
    return dict(x=x, y=y, z=z, vx=v[0], vy=v[1], vz=v[2], a_re=a[0], a_im=a[1])


def sea_draws(seed: int, n_comp: int = SEA_N_COMP) -> Dict[str, np.ndarray]:
    """Random draws of the sea state: component directions and phases, and the
    current / perturbation headings."""
    rng = np.random.default_rng(10_000 + seed)
    psi0 = rng.uniform(0.0, 2 * math.pi)
    dirs = psi0 + np.radians(SEA_DIR_SPREAD_DEG) * rng.standard_normal(n_comp)
    phases = rng.uniform(0.0, 2 * math.pi, n_comp)
    current_heading = rng.uniform(0.0, 2 * math.pi)
    perturb_heading = rng.uniform(0.0, 2 * math.pi)
    return dict(dirs=dirs, phases=phases, current_heading=current_heading,
                perturb_heading=perturb_heading)


def wave_sea(nx: int, ny: int, dx: float, seed: int, current_speed: float = 0.0,
             n_comp: int = SEA_N_COMP) -> Sea:
    d = sea_draws(seed, n_comp)
    h = d["current_heading"]
    cur = (current_speed * math.cos(h), current_speed * math.sin(h))
    return Sea(nx=nx, ny=ny, dx=dx, dy=dx, mode=1, n_comp=n_comp,
               dirs=d["dirs"], phases=d["phases"], current=cur)


def hetero_sea(nx: int, ny: int, dx: float, seed: int, tile_L: float,
               hs_range: Tuple[float, float] = (1.0, 3.0), turn_deg: float = 90.0,
               current_speed: float = 0.0, cwm: bool = True,
               n_comp: int = SEA_N_COMP) -> Sea:
    """Heterogeneous sea over the grid: tiles of side tile_L covering it, the
    node significant height growing linearly in x over hs_range and the mean
    wave direction turning by turn_deg across the scene in y (the kind of
    sharply varying swell field the tiling is meant for); every node draws its
    own directions (mean + N(0, 25 deg)) and phases."""
    ntx = max(1, math.ceil((nx - 1) * dx / tile_L))
    nty = max(1, math.ceil((ny - 1) * dx / tile_L))
    x0 = -0.5 * ntx * tile_L
    y0 = -0.5 * nty * tile_L
    rng = np.random.default_rng(20_000 + seed)
    psi0 = rng.uniform(0.0, 2 * math.pi)
    nn = (ntx + 1) * (nty + 1)
    hs = np.empty(nn)
    dirs = np.empty((nn, n_comp))
    phases = np.empty((nn, n_comp))
    for j in range(nty + 1):
        for i in range(ntx + 1):
            q = j * (ntx + 1) + i
            hs[q] = hs_range[0] + (hs_range[1] - hs_range[0]) * i / ntx
            mean = psi0 + math.radians(turn_deg) * j / nty
            dirs[q] = mean + np.radians(SEA_DIR_SPREAD_DEG) * rng.standard_normal(n_comp)
            phases[q] = rng.uniform(0.0, 2 * math.pi, n_comp)
    h = rng.uniform(0.0, 2 * math.pi)
    cur = (current_speed * math.cos(h), current_speed * math.sin(h))
    return Sea(nx=nx, ny=ny, dx=dx, dy=dx, mode=2, n_comp=n_comp, current=cur,
               ntx=ntx, nty=nty, tile_L=tile_L, tile_x0=x0, tile_y0=y0,
               node_hs=hs, node_dirs=dirs, node_phases=phases, cwm=cwm)


def flat_sea(nx: int, ny: int, dx: float, sigma_v: float = 0.5) -> Sea:
    return Sea(nx=nx, ny=ny, dx=dx, dy=dx, mode=0, sigma_v=sigma_v)


# ---------------------------------------------------------------------------
# The five workloads (sizes and seeds).  Config 1 is the small parity case.
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    geometry: Geometry
    sea: Sea
    seed: int
    block_edge: float               # spatial block edge for FP64 references (m)
    chunks: Tuple[Tuple[int, int, int, int], ...] = ()  # (ix0, iy0, cnx, cny)
    target_dv: float = 0.0          # adjoint target: velocity perturbation (m/s)

    @property
    def n_facets(self) -> int:
        return self.sea.nx * self.sea.ny

    @property
    def contributions(self) -> int:
        g = self.geometry
        return self.n_facets * g.n_pulses * g.n_channels


def workload(k: int) -> Workload:
    if k == 1:
        g = harmony_geometry(256, 512)
        return Workload("cfg1_tiny_4096f_256p_512s_1ch", g, flat_sea(64, 64, 5.0),
                        seed=1, block_edge=10.0)
    if k == 2:
        g = harmony_geometry(2048, 4096, chirp=True)
        return Workload("cfg2_1e6f_2048p_4096s_1ch_chirp", g,
                        wave_sea(1000, 1000, 1.0, seed=2), seed=2, block_edge=8.0)
    if k == 3:
        g = harmony_geometry(4096, 8192, receivers="AB", n_pc=3, chirp=True)
        return Workload("cfg3_1.6e7f_4096p_8192s_6ch_chirp", g,
                        wave_sea(4000, 4000, 1.0, seed=3, current_speed=0.5),
                        seed=3, block_edge=8.0)
    if k == 4:
        g = harmony_geometry(1024, 4096)
        return Workload("cfg4_adjoint_1e6f_1024p_4096s_1ch", g,
                        flat_sea(1000, 1000, 1.0), seed=4, block_edge=8.0,
                        target_dv=0.1)
    if k == 5:
        g = harmony_geometry(16384, 8192, receivers="A", n_pc=3, chirp=True)
        sea = wave_sea(16000, 8000, 1.0, seed=5, current_speed=0.5)
        chunks = tuple((4000 * (c % 4), 2000 * (c // 4), 4000, 2000)
                       for c in range(16))
        return Workload("cfg5_streamed_1.28e8f_16384p_8192s_3ch_chirp", g, sea,
                        seed=5, block_edge=8.0, chunks=chunks)
    raise ValueError(f"no workload {k}")


@dataclass(frozen=True)
class Speckle:
    """Intra-facet speckle inputs: correlation time tau_s (s; math.inf
    freezes the process), the Philox seed, and the counter id of facet 0
    (facet i draws with id first_index + i)."""
    tau_s: float = SPECKLE_TAU_S
    seed: int = 0
    first_index: int = 0


def speckle_doppler(n: int, seed: int) -> np.ndarray:
    """Per-facet intra-facet Doppler f_s (Hz, float32 [n]): +-SPECKLE_FD_HZ
    with equal odds plus N(0, SPECKLE_FD_SPREAD_HZ^2)."""
    rng = np.random.default_rng(seed + 7919)
    sign = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    return (sign * SPECKLE_FD_HZ + rng.normal(0.0, SPECKLE_FD_SPREAD_HZ, n)).astype(np.float32)


def tops_geometry(g: Geometry, rate_deg_s: float = 1.5) -> Geometry:
    """The same acquisition with the transmit antenna steered in azimuth at a
    constant rate (TOPS-like burst sweep; Sentinel-1 IW sweeps its beam by
    about +-0.6 deg over a burst of under a second)."""
    ants = list(g.antennas)
    ants[0] = replace(ants[0], steer_rate=math.radians(rate_deg_s))
    return replace(g, antennas=tuple(ants))


def synthetic_pattern(beta_az: float, beta_el: float, seed: int, nu: int = 129,
                      nv: int = 65, span_az: float = 4.0, span_el: float = 2.0,
                      ripple: float = 0.03) -> Pattern:
    """Stand-in for an industrial antenna model (the paper's patterns come
    from phased-array models that are not available): a Gaussian main beam
    with the given one-way 3-dB widths (field exp(-2 ln2 (x^2 + y^2)),
    x = u / beta_az, y = v / beta_el), an az-el coupling term 0.15 x y, and
    seeded per-node ripple of relative size `ripple` (element errors), on a
    grid spanning +-span_az beam widths in u and +-span_el in v."""
    rng = np.random.default_rng(seed + 104729)
    u = np.linspace(-span_az * beta_az, span_az * beta_az, nu)
    v = np.linspace(-span_el * beta_el, span_el * beta_el, nv)
    x = u[None, :] / beta_az
    y = v[:, None] / beta_el
    f = np.exp(-2.0 * math.log(2.0) * (x * x + y * y) + 0.15 * x * y)
    f = f * (1.0 + ripple * rng.standard_normal((nv, nu)))
    return Pattern(float(u[0]), float(u[1] - u[0]), float(v[0]), float(v[1] - v[0]),
                   f.astype(np.float32))


def gridded_geometry(g: Geometry, seed: int = 0, **kw) -> Geometry:
    """The same acquisition with every antenna's pattern given as a u-v grid
    (synthetic_pattern of its beam widths)."""
    ants = tuple(replace(a, pattern=synthetic_pattern(a.beta_az, a.beta_el, seed + i, **kw))
                 for i, a in enumerate(g.antennas))
    return replace(g, antennas=ants)


def with_pulses(g: Geometry, n_pulses: int) -> Geometry:
    return replace(g, n_pulses=n_pulses)
