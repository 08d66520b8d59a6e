"""Benchmark of the facet-sum hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 5]

Workload 5 (the default) is the largest single-GPU configuration: a streamed
scene of 1.28e8 facets in 16 chunks of 8e6, 16384 pulses x 8192 samples x 3
channels, chirp.  One step is one chunk of it: facet generation on the
device (Philox + linear waves + current), the range-binned block sort
(plan), the fused forward sum of every pulse and channel accumulated into
the resident IQ (3 GiB), and the chirp convolution of a sixteenth of the
lines, i.e. one sixteenth of the whole scene's forward work.  Steps cycle
through the chunks.  Workloads 1-4 (``--workload k``) are single scenes:
one step is the whole scene (generation, plan, sum, chirp).

`value` is forward throughput in G facet-pulse-channel contributions per
second (contributions per step / step time), every input generated in HBM
inside the step.  Consecutive steps are pipelined: the generation and plan
of step i+1 run on a side stream (default priority) while step i's sum runs;
every step still does all of its work.  A second timed loop of
forward+adjoint steps gives `fwd_adj`: the forward step, the loss gradient
and chirp adjoint of the step's share of the lines, and the adjoint sum over
the step's facets (workload 5: dL/dV of the chunk, loss 1/2 ||raw||^2;
workloads 1-4: dL/d(z, V, a), loss ||raw - T||^2 against a target from a
perturbed current).

`roofline` reports the fused forward kernel against the FP32 vector ALU:
achieved = W_alg slots per contribution x contributions per launch / average
launch time (HIP events on the launch stream), where a slot is one FP32
lane-operation of the full-rate FMA pipe and a transcendental costs four;
peak = 256 CUs x 128 lanes x 2.4 GHz (the 157.3 TFLOP/s FP32 figure counted
in FMAs).  `roofline_adjoint` does the same for the adjoint kernel with its
own frozen listing.  `cpu_baseline` times the FP64 oracle on a bounded pulse
subset of the same scene (workload 5: its first chunk) on the host's cores,
and `rel_l2_vs_fp64` compares those oracle lines with the GPU's.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic ALU slots per contribution of the forward sum at one channel,
# frozen from the per-contribution operation listing of the reformulated
# arithmetic (offset expansion of the range, one reciprocal for the pattern
# factors, even/odd tap polynomials): 116 FP32 operations at one slot and 7
# transcendentals (sin, cos, rcp), which gfx950 issues at a quarter of the
# FP32 FMA rate, at four slots each.  Where the plan takes the elevation
# pattern factors at block centres, two direction cosines, their two sines
# and four products leave the listing: 104 FP32 operations, 5
# transcendentals.  Loop control, window tests and LDS addressing are
# overhead, not counted.
W_ALG_SLOTS = 116.0 + 7 * 4.0
W_ALG_SLOTS_EL_CONST = 104.0 + 5 * 4.0
# With u-v gridded patterns (--patterns) the four scaled direction cosines
# become four cell coordinates (16 operations, no sines) and the sinc product
# becomes two bilinear lookups of 17 operations each (2 floors, 2 fractions,
# 4 bounds tests, index, 64-bit address, 3 lerps, select; one 16-byte load)
# plus the field product, spreading and amplitude (4): 144 FP32 operations and
# 2 transcendentals (sin, cos of the phase).
W_ALG_SLOTS_GRID = 144.0 + 2 * 4.0
# With the intra-facet speckle of eq. 7 (--speckle), per contribution: one
# Philox2x32-10 evaluation (10 rounds of one 32 x 32 -> 64-bit product, which
# gfx950 issues at about half the FMA rate (measured), and two XORs), the two
# uniforms (2 shifts, 2 conversions, 2 scalings), Box-Muller (log2, sqrt, sin,
# cos at four slots; 3 products), the AR(1) step and the bridge correction
# (2 + 2 FMAs), the amplitude times x (4) and the Doppler phase (6): 79 slots.
MUL64_SLOTS = 2.0
W_SPK_SLOTS = 10 * (MUL64_SLOTS + 2) + 6 + (4 * 4.0 + 3) + 4 + 4 + 6
# Adjoint sum, per contribution (elevation factors at block centres): the
# facet geometry of the forward (44 FP32 operations, 5 transcendentals: the
# forward listing without taps, weight and deposit), the two tap sums B and
# dB/du from the per-(pulse, first-tap sample) coefficient table (32: the
# fraction and its square, Horner's rule with the derivative for the even
# and odd cubics in y, 5 per real polynomial, and their combination), the
# table itself shared by a block's facets (8 entries per pulse, each 16
# sums and 64 FMAs: 10 per contribution at 64 facets per block), a E and
# B a E (8), the delay and phase terms (6), the range gradient (14), the
# three components of dL/dX (7), the accumulation into dL/dz and dL/dV (4)
# and dL/da (6): 131 FP32 operations and 5 transcendentals.  Staged
# reference reads, the loads of g, loop control and the per-block FP64
# stage prologue are overhead, not counted.
W_ADJ_SLOTS_EL_CONST = 131.0 + 5 * 4.0
# with every pattern factor per facet: two more direction cosines (8), their
# two sines and four more products of the pattern (4)
W_ADJ_SLOTS = W_ADJ_SLOTS_EL_CONST + 12.0 + 2 * 4.0
PEAK_SLOTS = 256 * 128 * 2.4e9         # FP32 lane-operations per second (157.3 TFLOP/s / 2)
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2405_09938_amd", "csrc", f)
                  for f in ("k_forward.hip", "sim_device.h")]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_file(workload_name: str) -> str:
    return os.path.join(PROFILES, f"k_forward_{workload_name.split('_')[0]}_traffic.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=5)
    ap.add_argument("--adj-steps", type=int, default=None,
                    help="forward+adjoint steps timed (default: steps, at most 8 for the "
                         "chunked workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--serial", action="store_true",
                    help="no step pipelining (one kernel at a time, for per-kernel counters)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--tops", type=float, default=0.0,
                    help="steer the transmit antenna in azimuth at this rate (deg/s)")
    ap.add_argument("--rx-exact", action="store_true",
                    help="receiver at each facet's own echo time (eq. 3's r_r(t_r))")
    ap.add_argument("--patterns", action="store_true",
                    help="u-v gridded antenna patterns (129 x 65 nodes per antenna)")
    ap.add_argument("--speckle", action="store_true",
                    help="intra-facet speckle (eq. 7, 10): tau_s 20 ms, f_s +-5.7 Hz per facet")
    ap.add_argument("--fast", type=int, default=0,
                    help="also time the fast mode (Sec. IV.B) with this node spacing n_fast "
                         "(single-scene workloads): speed-up and Doppler-spectrum error")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of a known size (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        # Plain device-to-device copy of 512 MiB, repeated: the HBM counters
        # of one such dispatch must read 512 MiB fetched and 512 MiB written.
        n = 512 * 1024 * 1024 // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(max(1, args.steps)):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 4, "dispatches": max(1, args.steps)}))
        return

    import paper_2405_09938_amd as hs
    import workloads as W

    wl = W.workload(args.workload)
    chunked = bool(wl.chunks)
    if chunked and args.fast:
        print("--fast runs on the single-scene workloads (1-4)", file=sys.stderr)
        sys.exit(2)
    if chunked and (args.speckle or args.rx_exact or args.tops or args.patterns):
        print("the chunked workload runs the plain sum only (no --speckle, --rx-exact, "
              "--tops, --patterns)", file=sys.stderr)
        sys.exit(2)
    if args.rx_exact or args.tops or args.patterns:
        from dataclasses import replace as _replace
        g2 = _replace(wl.geometry, rx_exact=args.rx_exact)
        if args.tops:
            g2 = W.tops_geometry(g2, args.tops)
        if args.patterns:
            g2 = W.gridded_geometry(g2, seed=wl.seed)
        wl = _replace(wl, geometry=g2)
    geom, sea = wl.geometry, wl.sea
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    hs.load()
    sim = hs.Simulator(geom)
    chirp = geom.chirp_T > 0
    C, Np, N = geom.n_channels, geom.n_pulses, geom.n_samples
    stream = torch.cuda.current_stream()
    n_chunks = len(wl.chunks) if chunked else 1
    # contributions of one step: a chunk of the chunked workload, else the scene
    step_facets = (wl.chunks[0][2] * wl.chunks[0][3]) if chunked else wl.n_facets
    contrib = step_facets * Np * C
    if chunked:
        assert all(c[2] * c[3] == step_facets for c in wl.chunks), "chunks of equal size"

    # speckle inputs: one process per facet, Doppler drawn per facet (input,
    # resident in HBM for the whole run)
    spk = W.Speckle(tau_s=W.SPECKLE_TAU_S, seed=wl.seed, first_index=0) if args.speckle else None
    fs_dev = (torch.from_numpy(W.speckle_doppler(wl.n_facets, wl.seed)).to(dev)
              if args.speckle else None)
    side = torch.cuda.Stream(device=dev)     # generation and plan of the next step
    wave = torch.cuda.Stream(device=dev)     # chirp of a single scene beside the next sum
    pipelined = not args.serial

    # resident IQ of the chunked scene: range-compressed (accumulated over the
    # chunks), raw (chirped) and the loss gradient g_rc
    if chunked:
        iq_rc = torch.zeros((C, Np, N), dtype=torch.complex64, device=dev)
        iq_raw = torch.zeros_like(iq_rc) if chirp else iq_rc
        g_rc = torch.zeros_like(iq_rc)
        lines_per_step = (C * Np + n_chunks - 1) // n_chunks

    def line_slice(i):
        a = (i % n_chunks) * lines_per_step
        return slice(a, min(a + lines_per_step, C * Np))

    def prepare(i):
        """Facets and plan of step i (a chunk, or the scene), on the side stream."""
        with torch.cuda.stream(side):
            sub = wl.chunks[i % n_chunks] if chunked else (0, 0, sea.nx, sea.ny)
            f = sim.generate(sea, wl.seed, *sub)
            plan = sim.plan(f["x"], f["y"], wl.block_edge, box=sim.chunk_box(sea, *sub),
                            speckle=args.speckle)
        # the sum reads the facets and the plan's workspace on the main stream
        for v in f.values():
            v.record_stream(stream)
        plan.workspace.record_stream(stream)
        return f, plan

    fwd_ev, adj_ev = [], []

    def fwd_step(i, prep, record=False, overlap=False):
        f, plan = prep
        stream.wait_stream(side)
        if record:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        if chunked:
            rc = sim.forward(plan, f, out=iq_rc, accumulate=True)
        else:
            rc = sim.forward(plan, f, speckle=spk, f_s=fs_dev)
        if record:
            e1.record(stream)
            fwd_ev.append((e0, e1))
        if chunked:
            s = line_slice(i)
            if chirp:
                sim.apply_waveform(iq_rc.view(-1, N)[s], out=iq_raw.view(-1, N)[s])
            out = iq_raw
        elif chirp and overlap:
            wave.wait_stream(stream)
            with torch.cuda.stream(wave):
                out = sim.apply_waveform(rc, out=rc)
            rc.record_stream(wave)
        else:
            out = sim.apply_waveform(rc, out=rc) if chirp else rc
        return f, plan, out

    def run_steps(n, step_fn, label, start=0):
        res = None
        nxt = prepare(start) if pipelined else None
        for i in range(start, start + n):
            cur = nxt if pipelined else prepare(i)
            nxt = None
            res = step_fn(i, cur)
            if pipelined and i + 1 < start + n:
                nxt = prepare(i + 1)
            if chunked:
                torch.cuda.synchronize()
                print(f"  {label} step {i} done", flush=True)
        return res

    print(f"workload {wl.name}: {contrib:.3e} contributions per step"
          + (f" (one chunk of {n_chunks})" if chunked else ""), flush=True)
    if args.warmup:
        run_steps(args.warmup, lambda i, p: fwd_step(i, p, overlap=pipelined), "warmup")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f, plan, out = run_steps(args.steps, lambda i, p: fwd_step(i, p, True, overlap=pipelined),
                             "forward", start=args.warmup)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_s = (t1 - t0) / args.steps
    value = contrib / step_s / 1e9
    kern_ms = sum(a.elapsed_time(b) for a, b in fwd_ev) / len(fwd_ev)
    print(f"forward step {step_s * 1e3:.3f} ms, {value:.2f} G/s; forward sum "
          f"{kern_ms:.3f} ms avg", flush=True)
    el_const = plan.el_const

    fast = None
    if args.fast:
        # fast mode: windows of 64 full-rate pulses every n_fast pulses, the
        # rest synthesized from the gates' Doppler spectra; same pipeline
        fseed = 1000 + wl.seed

        def fast_step(i, prep):
            f2, plan2 = prep
            stream.wait_stream(side)
            rc2 = sim.forward_fast(plan2, f2, args.fast, fseed)
            return sim.apply_waveform(rc2, out=rc2) if chirp else rc2

        if args.warmup:
            run_steps(args.warmup, fast_step, "fast warmup")
        torch.cuda.synchronize()
        tf0 = time.perf_counter()
        run_steps(args.steps, fast_step, "fast", start=args.warmup)
        torch.cuda.synchronize()
        fast_s = (time.perf_counter() - tf0) / args.steps
        # Doppler-spectrum error over the whole dwell: gate-averaged
        # Hann-tapered 64-pulse periodograms (half-overlapping) of the
        # range-compressed lines, fast mode against the full-rate sum
        rc_full = sim.forward(plan, f)
        rc_fast = sim.forward_fast(plan, f, args.fast, fseed)
        m = torch.arange(64, device=dev, dtype=torch.float64)
        hw = (math.sqrt(8.0 / 3.0) * torch.sin(math.pi * (m + 0.5) / 64) ** 2).to(torch.float32)

        def doppler_spectrum(iq):
            segs = iq[:, 64:Np - 64].unfold(1, 64, 32)          # [C, S, N, 64]
            spec = torch.fft.fft(segs * hw, dim=-1).abs() ** 2
            return spec.mean(dim=(0, 1, 2)).double()

        S_full, S_fast = doppler_spectrum(rc_full), doppler_spectrum(rc_fast)
        spec_err = float((S_fast - S_full).abs().sum() / S_full.sum())
        n_win = (Np - 64) // args.fast + 1
        fast = {"n_fast": args.fast, "windows": n_win,
                "computed_pulse_fraction": round(64 * n_win / Np, 4),
                "ms_per_step": round(fast_s * 1e3, 4),
                "value_equivalent": round(contrib / fast_s / 1e9, 3),
                "speedup_vs_full_rate": round(step_s / fast_s, 3),
                "doppler_spectrum_rel_l1": round(spec_err, 4)}
        print(f"fast mode n_fast {args.fast}: step {fast_s * 1e3:.3f} ms, speed-up "
              f"{step_s / fast_s:.2f}x, Doppler spectrum rel L1 {spec_err:.4f}", flush=True)

    fwd_adj = None
    adj_ms = None
    if not args.no_adjoint:
        if chunked:
            def fa_step(i, prep):
                f2, plan2, _ = fwd_step(i, prep)
                s = line_slice(i)
                # loss 1/2 ||raw||^2: g_raw = raw; chirp adjoint of the step's lines
                if chirp:
                    sim.apply_waveform(iq_raw.view(-1, N)[s], out=g_rc.view(-1, N)[s],
                                       adjoint=True)
                else:
                    g_rc.view(-1, N)[s].copy_(iq_raw.view(-1, N)[s])
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                gr = sim.backward(plan2, f2, g_rc, need=("vx", "vy", "vz"))
                e1.record(stream)
                adj_ev.append((e0, e1))
                return gr
        else:
            # target: same scene, velocities perturbed by a 0.1 m/s current
            psi = W.sea_draws(wl.seed)["perturb_heading"]
            with torch.no_grad():
                ft = dict(f)
                ft["vx"] = f["vx"] + 0.1 * math.cos(psi)
                ft["vy"] = f["vy"] + 0.1 * math.sin(psi)
                tgt = sim.forward(plan, ft, speckle=spk, f_s=fs_dev)
                if chirp:
                    tgt = sim.apply_waveform(tgt, out=tgt)

            def fa_step(i, prep):
                f2, plan2, o = fwd_step(i, prep)
                g = 2.0 * (o - tgt)
                if chirp:
                    g = sim.apply_waveform(g, out=g, adjoint=True)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                gr = sim.backward(plan2, f2, g, speckle=spk, f_s=fs_dev)
                e1.record(stream)
                adj_ev.append((e0, e1))
                return gr

        n_adj = args.adj_steps
        if n_adj is None:
            n_adj = min(args.steps, 8) if chunked else args.steps
        if args.warmup:
            run_steps(min(args.warmup, 2), fa_step, "forward+adjoint warmup")
        adj_ev.clear()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        run_steps(n_adj, fa_step, "forward+adjoint")
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        fa_s = (t3 - t2) / n_adj
        adj_ms = sum(a.elapsed_time(b) for a, b in adj_ev) / len(adj_ev)
        fwd_adj = {"value": round(contrib / fa_s / 1e9, 3), "unit": "G contributions/s",
                   "ms_per_step": round(fa_s * 1e3, 4), "steps": n_adj,
                   "adjoint_sum_ms": round(adj_ms, 4)}
        print(f"forward+adjoint step {fa_s * 1e3:.3f} ms, {fwd_adj['value']:.2f} G/s; "
              f"adjoint sum {adj_ms:.3f} ms avg", flush=True)

    if args.patterns:
        el_const = False          # gridded patterns are evaluated per facet
        w_alg = W_ALG_SLOTS_GRID
    else:
        w_alg = W_ALG_SLOTS_EL_CONST if el_const else W_ALG_SLOTS
    if args.speckle:
        w_alg += W_SPK_SLOTS
    achieved = w_alg * contrib / (kern_ms * 1e-3) / 1e12
    peak = PEAK_SLOTS / 1e12
    traffic = None
    valu = None
    tf = traffic_file(wl.name)
    if os.path.exists(tf):
        with open(tf) as fh:
            tr = json.load(fh)
        if (tr.get("kernel_hash") == kernel_hash() and tr.get("workload") == wl.name
                and bool(tr.get("speckle", False)) == args.speckle and not args.rx_exact
                and not args.tops and not args.patterns):
            traffic = tr.get("bytes_per_launch")
            valu = tr.get("valu_insts_per_launch")
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3),
                "unit": "Tslot/s", "frac": round(achieved / peak, 4), "traffic": traffic,
                "kernel": "k_forward", "w_alg_slots_per_contribution": w_alg,
                "elevation_at_block_centres": el_const,
                "contributions_per_launch": contrib, "avg_launch_ms": round(kern_ms, 4)}
    if valu:
        # issued wave64 VALU instructions (rocprof SQ_INSTS_VALU of the same
        # kernel source) against the FP32 issue peak of two per CU per cycle
        # at 2.4 GHz
        roofline["valu_issue_frac"] = round(valu / (256 * 2 * 2.4e9 * kern_ms * 1e-3), 4)
    roofline_adj = None
    if adj_ms is not None and not args.speckle and not args.patterns and not args.tops:
        w_adj = W_ADJ_SLOTS_EL_CONST if el_const else W_ADJ_SLOTS
        a_adj = w_adj * contrib / (adj_ms * 1e-3) / 1e12
        roofline_adj = {"bound": "alu", "achieved": round(a_adj, 3), "peak": round(peak, 3),
                        "unit": "Tslot/s", "frac": round(a_adj / peak, 4), "traffic": None,
                        "kernel": "k_adjoint", "w_alg_slots_per_contribution": w_adj,
                        "contributions_per_launch": contrib,
                        "avg_launch_ms": round(adj_ms, 4)}

    cpu = None
    rel = None
    if not args.no_cpu_baseline:
        import oracle as O
        # bounded sample: the oracle's own scene (same seed and sea draws;
        # workload 5: its first chunk), all facets, pulses from the middle of
        # the dwell until the time budget is spent
        if chunked:
            sub = wl.chunks[0]
            fo = O.as_float32(O.generate_facets(sea, wl.seed, *sub))
            n_fac = sub[2] * sub[3]
        else:
            fo = O.as_float32(O.generate_facets(sea, wl.seed))
            n_fac = wl.n_facets
        fo = {k: v.astype(np.float64) for k, v in fo.items()}
        p_mid = Np // 2
        chunk = 4
        done = 0
        t_cpu = 0.0
        rows = []
        while t_cpu < args.cpu_seconds and done + chunk <= Np // 2:
            p0 = p_mid + done
            ta = time.perf_counter()
            if args.speckle:
                rc = O.forward(geom, fo, p0, chunk, speckle=spk,
                               f_s=W.speckle_doppler(wl.n_facets, wl.seed).astype(np.float64))
            else:
                rc = O.forward(geom, fo, p0, chunk)
            line = O.waveform_fft(geom, rc) if chirp else rc
            t_cpu += time.perf_counter() - ta
            rows.append((p0, line))
            done += chunk
        n_contrib = n_fac * done * C
        cpu = {"value": n_contrib / t_cpu / 1e9, "unit": "G contributions/s",
               "cores": O.num_threads(), "kind": "oracle",
               "sample": f"{n_fac} facets x {done} pulses (from pulse {p_mid}) x "
                         f"{C} ch, FP64 direct sum + FFT waveform, {t_cpu:.1f} s"}
        if chunked:
            # the GPU recomputes the first chunk's lines over the same pulses
            gpu_iq = sim.stream_forward(sea, wl.seed, [wl.chunks[0]], wl.block_edge, p_mid, done)
            if chirp:
                gpu_iq = sim.apply_waveform(gpu_iq, out=gpu_iq)
            rows = [(p0 - p_mid, line) for p0, line in rows]
        else:
            gpu_iq = out
        got = gpu_iq.cpu().numpy()
        num = den = 0.0
        for p0, line in rows:
            d = got[:, p0:p0 + chunk] - line
            num += float(np.sum(np.abs(d) ** 2))
            den += float(np.sum(np.abs(line) ** 2))
        rel = math.sqrt(num / den)
        print(f"oracle: {cpu['value'] * 1e3:.3f} M/s on {cpu['cores']} threads; GPU vs FP64 "
              f"rel-L2 on the sample {rel:.3e}", flush=True)

    res = {
        "metric": "G facet-pulse contributions/s (fwd) at <=1e-4 rel-L2 vs FP64",
        "value": round(value, 3),
        "unit": "G contributions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": ("synthetic (on-device Philox facets, 64-component linear wave sea"
                 + (" + current)" if sea.mode == 1 and any(sea.current) else ")")
                 if sea.mode == 1 else "synthetic (on-device Philox facets, flat sea)"),
        "config": {"workload": wl.name, "facets_per_step": step_facets,
                   "scene_facets": wl.n_facets, "chunks": n_chunks,
                   "step": ("one chunk: generate, plan, sum all pulses and channels into "
                            "the resident IQ, chirp 1/16 of the lines") if chunked
                   else "whole scene: generate, plan, sum, chirp",
                   "pulses": Np, "samples": N, "channels": C, "chirp": chirp,
                   "block_edge_m": wl.block_edge,
                   "speckle": ({"tau_s": W.SPECKLE_TAU_S, "f_s_hz": f"+-{W.SPECKLE_FD_HZ}"}
                               if args.speckle else None),
                   "rx_at_facet_echo_time": args.rx_exact,
                   "tx_steer_deg_s": args.tops or None,
                   "antenna_patterns": "u-v grids 129x65" if args.patterns else "sinc"},
        "fwd_adj": fwd_adj,
        "fast_mode": fast,
        "rel_l2_vs_fp64": rel,
        "roofline": roofline,
        "roofline_adjoint": roofline_adj,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
