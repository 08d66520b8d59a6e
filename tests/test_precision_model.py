"""Precision model of the FP32 facet geometry (CPU, NumPy only).

The carrier phase of one contribution is 2 pi f0 R / c with R ~ 1.7e6 m, and
the relative L2 error of a speckle sum is about the rms phase error of its
contributions.  The HIP path removes the large part of R per (block, pulse)
in FP64 and forms only the offset

    R - R_b = e.g + (|e|^2 - (e.d_t)^2) / (2 R_t) + (|e|^2 - (e.d_r)^2) / (2 R_r)

in float32, with e = X0 - x_b + V t_p the facet's offset from its block
centre.  This test emulates that expression in float32 with NumPy, measures
its rms phase error against the FP64 ranges, and checks it against two
bounds: with 8 m blocks it is at the 1e-5 rad level, which is the floor the
GPU parity tests measure (about 2e-5 rel-L2); with a single reference point
for a 1 km scene (the negative control) it is above 5e-4 rad, far past the
1e-4 target.  No code of the library or of the oracle is used: positions,
pulse geometry and ranges are recomputed here from the configuration.
"""
import math

import numpy as np

import workloads as W

F32 = np.float32


def pulse_positions(g, p):
    """Tx at t_p and Rx at t_p + tau_ref (scene origin echo), FP64."""
    t = (p - (g.n_pulses - 1) / 2) / g.prf
    tx, rx = g.platforms[0], g.platforms[g.antennas[g.channels[0].rx].platform]
    ptx = np.array(tx.p0) + np.array(tx.v) * t
    tau = 0.0
    for _ in range(8):
        prx = np.array(rx.p0) + np.array(rx.v) * (t + tau) + np.array(g.channels[0].pc_offset)
        tau = (np.linalg.norm(ptx) + np.linalg.norm(prx)) / g.c
    return t, ptx, prx


def phase_error_rms(g, x0, v, centres, pulses):
    """rms of 2 pi f0/c (dR_fp32 - dR_fp64) over facets and pulses."""
    errs = []
    for p in pulses:
        t, ptx, prx = pulse_positions(g, p)
        X = x0 + v * t
        # FP64 truth relative to each facet's reference point
        rt_b = np.linalg.norm(centres - ptx, axis=1)
        rr_b = np.linalg.norm(centres - prx, axis=1)
        dR64 = (np.linalg.norm(X - ptx, axis=1) + np.linalg.norm(X - prx, axis=1)) - (rt_b + rr_b)
        # float32 offset expansion, references rounded once to float32
        dt = ((centres - ptx) / rt_b[:, None]).astype(F32)
        dr = ((centres - prx) / rr_b[:, None]).astype(F32)
        gv = (dt + dr).astype(F32)
        e = ((x0 - centres).astype(F32) + v.astype(F32) * F32(t)).astype(F32)
        ee = np.sum(e * e, axis=1, dtype=F32)
        L = np.sum(e * gv, axis=1, dtype=F32)
        at = np.sum(e * dt, axis=1, dtype=F32)
        ar = (L - at).astype(F32)
        i2rt = (0.5 / rt_b).astype(F32)
        i2rr = (0.5 / rr_b).astype(F32)
        dR32 = L + ((ee - at * at) * i2rt + (ee - ar * ar) * i2rr).astype(F32)
        errs.append(2 * math.pi * g.f0 / g.c * (dR32.astype(np.float64) - dR64))
    return float(np.sqrt(np.mean(np.concatenate(errs) ** 2)))


def scene(n_side, spacing, seed):
    rng = np.random.default_rng(seed)
    ix, iy = np.meshgrid(np.arange(n_side), np.arange(n_side))
    x = (ix.ravel() - (n_side - 1) / 2) * spacing
    y = (iy.ravel() - (n_side - 1) / 2) * spacing
    x0 = np.stack([x, y, rng.normal(0, 0.5, x.size)], 1)
    v = rng.normal(0, 0.5, (x.size, 3))
    return x0, v


def test_block_references_meet_the_phase_budget():
    g = W.harmony_geometry(2048, 4096)
    x0, v = scene(128, 1.0, 3)
    edge = 8.0
    centres = np.stack([(np.floor(x0[:, 0] / edge) + 0.5) * edge,
                        (np.floor(x0[:, 1] / edge) + 0.5) * edge, np.zeros(len(x0))], 1)
    e = phase_error_rms(g, x0, v, centres, (0, 1023, 2047))
    print(f"8 m blocks: rms phase error {e:.2e} rad")
    assert 1e-6 < e < 5e-5


def test_single_reference_negative_control():
    g = W.harmony_geometry(2048, 4096)
    x0, v = scene(128, 8.0, 4)          # 1 km x 1 km
    centres = np.zeros_like(x0)
    e = phase_error_rms(g, x0, v, centres, (0, 1023, 2047))
    print(f"one reference for a 1 km scene: rms phase error {e:.2e} rad")
    assert e > 5e-4


def test_block_references_at_the_streamed_dwell_ends():
    """The streamed 16384-pulse workload: a 9.6 s dwell (|t_p| up to 4.82 s)
    over a scene reaching 8 km along-track and 4 km across, facets moving
    with wave orbital velocities plus a 0.5 m/s current, so the drift V t_p
    stretches the offsets from the block centres to ~5-10 m at the dwell ends
    and their float32 rounding grows with them (about ulp(|e|) of path per
    component).  With the orbital velocity of the workload's sea (k^-4
    spectrum scaled to Hs = 2 m over wavelengths 5-250 m: ~0.21 m/s rms per
    horizontal axis) the model gives ~3.5e-5 rad at the dwell ends, in the
    far corners as at the centre (2.3e-5 mid-dwell), inside the 5e-5 budget
    guard; with twice that velocity it stays below the 1e-4 target."""
    g = W.harmony_geometry(16384, 8192, receivers="A", n_pc=3)
    rng = np.random.default_rng(5)
    edge = 8.0
    psi = 0.7
    # orbital velocity rms per axis of the workload's sea: sum A^2 omega^2 / 2
    # over its 64 components, a half on each horizontal axis
    k = np.exp(np.linspace(np.log(W.SEA_K_MIN), np.log(W.SEA_K_MAX), W.SEA_N_COMP))
    dl = math.log(W.SEA_K_MAX / W.SEA_K_MIN) / (W.SEA_N_COMP - 1)
    a2 = 2.0 * k ** W.SEA_SLOPE * k * dl
    a2 *= (W.SEA_HS / 4.0) ** 2 / np.sum(0.5 * a2)
    sv = math.sqrt(np.sum(0.5 * a2 * W.SEA_G * k) / 2.0)
    print(f"orbital velocity rms per horizontal axis {sv:.3f} m/s")
    assert 0.2 < sv < 0.5
    for scale, bound in ((1.0, 5e-5), (2.0, 1e-4)):
        for corner in ((0.0, 0.0), (7500.0, 3500.0), (-7500.0, -3500.0)):
            n = 128 * 128
            x = corner[0] + rng.uniform(-400, 400, n)
            y = corner[1] + rng.uniform(-400, 400, n)
            x0 = np.stack([x, y, rng.normal(0, 0.5, n)], 1)
            v = rng.normal(0, scale * sv, (n, 3))
            v[:, 0] += 0.5 * math.cos(psi)
            v[:, 1] += 0.5 * math.sin(psi)
            centres = np.stack([(np.floor(x / edge) + 0.5) * edge,
                                (np.floor(y / edge) + 0.5) * edge, np.zeros(n)], 1)
            e = phase_error_rms(g, x0, v, centres, (0, 16383))
            print(f"velocity x{scale}, scene at {corner}: dwell-end rms phase error {e:.2e} rad")
            assert 1e-6 < e < bound
