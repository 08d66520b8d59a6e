// Fused forward facet sum for gfx950.
//
// Each (channel, pulse) line receives, from every facet, a * F_tx * F_rx * S *
// exp(-j 2 pi f0 R / c) (Sec. III.A eq. 3, Sec. III.B eq. 16) spread around the
// facet's fractional sample u = n_ref + (R - c tau_ref) fs / c by an 8-tap
// Kaiser-windowed sinc (the range slices of eq. 17).
//
// Work decomposition: a work unit is (segment of a range strip, pulse group
// of 64, channel).  A strip holds the blocks whose centres fall in a band of
// S range samples at the reference pulse of the group's band (the plan's
// range-binned sort), so one LDS range window of the band's width W covers
// that band plus a margin and every facet of the strip lands in it.  One
// launch per window width the bands use; a workgroup of K waves takes one
// unit of its width at a time from a work queue (below); wave k sums blocks
// k, k + K, ... of the segment into its own window, facets in pairs (one
// read-modify-write for two facets whose taps start at the same sample on
// every lane).
//   Lane = pulse: every lane handles the same facet
//   (its 32-byte record arrives by two uniform buffer loads) and deposits into
//   its own pulse column of the wave's LDS range window.  Since no other lane
//   or wave touches that column, the deposit is a plain read-modify-write (8 x
//   64-bit reads issued as soon as the sample index is known, 16 FMAs, 8 x
//   64-bit writes) instead of LDS atomics, which serialise per lane on gfx950.
//   The window is stored sample-major ([sample][lane]), so the 64 lanes of one
//   access always fall on distinct bank pairs whatever their sample indices:
//   a lane-major layout conflicts as soon as the lanes' sample indices
//   differ.  At the end the K windows are added in wave order and the sum
//   goes to the unit's own slot of a scratch array with plain stores;
//   k_window_reduce then adds, for every sample, the slots of the strips
//   holding it in strip and segment order, so the result does not depend on
//   the order in which workgroups run and no global atomics are needed.  A
//   contribution whose taps leave the window (only for facets beyond the
//   plan's height and speed bounds) goes straight to global memory.
#include "sim_device.h"
#include "spk_device.h"

namespace hs {

namespace {

// Read-only inputs of the kernel, accessed through the constant address
// space: uniform indices then compile to scalar loads into SGPRs.
template <typename T>
using cptr = const T __attribute__((address_space(4))) *;

__device__ __forceinline__ BlockRec load_block(cptr<BlockRec> p) {
    BlockRec r;
    r.xb = p->xb;
    r.yb = p->yb;
    r.start = p->start;
    r.count = p->count;
    return r;
}

// Facet records are read with vector-memory buffer loads at a uniform
// offset: every lane receives the same 32 bytes in VGPRs.  Scalar loads
// would share the lgkm counter with the LDS deposit, so each wait for the
// deposit's reads would also wait for the next record's scalar-cache miss;
// buffer loads are counted by vmcnt instead.  The resource covers one
// block's records (plus the padding record after the last block), and a
// load past its end returns zeros.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t facet_rsrc(const FacetRec *base, int count) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, 0, (count + 1) * (int)sizeof(FacetRec),
                                             0x00020000);
}

struct FacetV {
    float dx, dy, z, vx, vy, vz, ar, ai;
};

__device__ __forceinline__ FacetV load_facet(__amdgpu_buffer_rsrc_t rs, int j) {
    const auto a = __builtin_amdgcn_raw_buffer_load_b128(rs, 0, j * (int)sizeof(FacetRec), 0);
    const auto b = __builtin_amdgcn_raw_buffer_load_b128(rs, 16, j * (int)sizeof(FacetRec), 0);
    FacetV f;
    f.dx = __uint_as_float(a[0]);
    f.dy = __uint_as_float(a[1]);
    f.z = __uint_as_float(a[2]);
    f.vx = __uint_as_float(a[3]);
    f.vy = __uint_as_float(b[0]);
    f.vz = __uint_as_float(b[1]);
    f.ar = __uint_as_float(b[2]);
    f.ai = __uint_as_float(b[3]);
    return f;
}

// Speckle record (id, f_s) and anchor pair of one facet, also uniform
// buffer loads (zeros past the resource's end).
struct SpkFacet {
    uint32_t id;
    float fs;
    float ygr, ygi, y1r, y1i;   // y_g and y_{g+1}
};

__device__ __forceinline__ SpkFacet load_spk(__amdgpu_buffer_rsrc_t rr, __amdgpu_buffer_rsrc_t ra,
                                             int j, int ng1, int g) {
    const auto r = __builtin_amdgcn_raw_buffer_load_b64(rr, j * (int)sizeof(SpkRec), 0, 0);
    const int off = (j * ng1 + g) * (int)sizeof(float4);
    const auto a = __builtin_amdgcn_raw_buffer_load_b64(ra, off, 0, 0);
    const auto b = __builtin_amdgcn_raw_buffer_load_b64(ra, off + (int)sizeof(float4), 0, 0);
    SpkFacet s;
    s.id = r[0];
    s.fs = __uint_as_float(r[1]);
    s.ygr = __uint_as_float(a[0]);
    s.ygi = __uint_as_float(a[1]);
    s.y1r = __uint_as_float(b[0]);
    s.y1i = __uint_as_float(b[1]);
    return s;
}

template <int WIN>
constexpr int fwd_waves() {
    return hs::fwd_waves(WIN);
}

// SPK: the intra-facet speckle of eq. 7 multiplies each facet's amplitude by
// x(p) and adds f_s t_p cycles to its phase.  Pulse groups are then aligned
// on absolute pulse indices (multiples of 64), so that a wave holds exactly
// one group of the speckle process; lanes before p0 or past the last pulse
// take part in the prefix sum but deposit nothing.
// STR: antenna frames turn with time (steering): per-pulse frames.
// GRD: field patterns from u-v tables (1: on some antennas, 2: on all),
// evaluated per facet (never with ELC).
// One work unit: segment `seg` of a range strip of the band holding pulse
// group `grp`, channel `ch`; accw holds the workgroup's LDS windows.
template <int WIN, bool ELC, bool SPK, bool STR, int GRD>
__device__ __forceinline__ void forward_unit(const FwdArgs &A, float2 *accw, int seg, int grp,
                                             int ch) {
    constexpr int K = fwd_waves<WIN>();
    constexpr int kAcc = 64 * WIN;
    // the wave index, uniform (in an SGPR): block loads stay scalar
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    float2 *acc = accw + wave * kAcc;
    const int poff = SPK ? (A.p0 & 63) : 0;     // lanes before p0 in the first group
    const StripPlan &st = A.st;
    // pulse (relative to p0) of lane 0; grp counts from the pass's first group
    const int gbase = (A.g0 + grp) * A.gstride - poff;
    int pc = A.p0 + gbase + 32;                 // the group's centre pulse
    pc = pc < 0 ? 0 : (pc < A.Np ? pc : A.Np - 1);
    int band = pc / (64 * st.B);
    band = band < st.NB ? band : st.NB - 1;
    const size_t bc = (size_t)band * A.C + ch;
    const cptr<double> bd = (cptr<double>)(st.band + 4 * bc);
    if ((int)bd[3] != WIN) return;   // the band's units run in the launch of its width
    const cptr<int> segoff = (cptr<int>)(st.segoff + bc * (st.NS + 1));
    if (seg >= segoff[st.NS]) return;
    // the segment's strip: the last s with segoff[s] <= seg
    int s_lo = 0, s_hi = st.NS;
    while (s_hi - s_lo > 1) {
        const int mid = (s_lo + s_hi) >> 1;
        if (segoff[mid] <= seg) s_lo = mid;
        else s_hi = mid;
    }
    const int strip = s_lo;
    const cptr<int> soff = (cptr<int>)(st.soff + bc * (st.NS + 1));
    const int q0 = soff[strip] + (seg - segoff[strip]) * st.L;
    const int q1 = soff[strip + 1] < q0 + st.L ? soff[strip + 1] : q0 + st.L;
    const cptr<int> ids = (cptr<int>)(st.ids + bc * st.nbm);
    const cptr<BlockRec> blocks = (cptr<BlockRec>)A.blocks;
    const int lane = (int)(threadIdx.x & 63);
    const int pl = gbase + lane;               // pulse relative to p0, also its output row
    const bool live = pl >= 0 && pl < A.np;
    const int plc = pl < 0 ? 0 : (pl < A.np ? pl : A.np - 1);
    const PulseRec *PR = A.pulses + (size_t)ch * A.Np + A.p0;
    const ChanArgs chn = A.ch[ch];
    const AntArgs &ta = A.ant[chn.tx], &ra = A.ant[chn.rx];
    FacetConsts kc;
    facet_consts(ta, ra, kc);

    // Range window of the strip: its band of samples at the reference
    // pulse, widened by the margin and the taps.
    const int lo = (int)floor(bd[0] + (double)strip * bd[1] - bd[2]) - 3;
    float2 *col = acc + lane;
    for (int i = 0; i < WIN; ++i) col[64 * i] = make_float2(0.f, 0.f);

    const PulseRec &P = PR[plc];
    // antenna frames of this pulse (time-dependent patterns)
    // (float cosines and sines: they scale projections whose float rounding
    // stays below 1e-8 of the direction cosines; boresights are turned
    // only in grazing blocks)
    [[maybe_unused]] float4 rot{1.f, 0.f, 1.f, 0.f};
    if constexpr (STR) {
        rot = float4{(float)P.cst, (float)P.snt, (float)P.csr, (float)P.snr};
        steer_axes(ta, ra, rot.x, rot.y, rot.z, rot.w, kc);
    }
    const double ptx[3] = {P.ptx[0], P.ptx[1], P.ptx[2]};
    const double prx[3] = {P.prx[0], P.prx[1], P.prx[2]};
    const double rref = P.rref;
    const float tf = (float)P.t;
    float *iq_row = A.iq + 2 * ((size_t)ch * A.np + plc) * (size_t)A.N;
    TapV tv;
    tap_all(A.tp, tv);

    // speckle: the lane's pulse, its time split in two floats, the scan weights
    const SpkArgs &S = A.spk;
    [[maybe_unused]] int gabs = 0;
    [[maybe_unused]] uint32_t slot = 0;
    [[maybe_unused]] float thi = 0.f, tlo = 0.f, bk = 0.f, kk = 0.f, b64 = 0.f, l1 = 0.f;
    [[maybe_unused]] SpkScanW sw{};
    if constexpr (SPK) {
        gabs = (A.p0 + gbase) / 64;
        slot = (uint32_t)(64 * gabs + lane + 1);   // the lane draws e_{p + 1}
        thi = (float)P.t;
        tlo = (float)(P.t - (double)thi);
        bk = S.bpow[lane];
        kk = S.gain[lane];
        sw.b1 = to_vgpr(S.b1);
        sw.b2 = to_vgpr(S.b2);
        sw.b4 = to_vgpr(S.b4);
        sw.b8 = to_vgpr(S.b8);
        sw.w15 = ((lane >> 4) & 1) ? S.bpow[(lane & 15) + 1] : 0.0f;
        sw.w31 = lane >= 32 ? S.bpow[lane - 31] : 0.0f;
        b64 = S.b64;
        l1 = S.c1 * S.c1 * 0.69314718055994531f;
    }

    for (int q = q0 + wave; q < q1; q += K) {
        const BlockRec blk = load_block(blocks + ids[q]);
        Refs r;
        // receiver at the block centre's own echo time (optional)
        double prb[3] = {prx[0], prx[1], prx[2]};
        double qr = 1.0;
        if (A.rx_exact)
            rx_echo((double)blk.xb, (double)blk.yb, ptx, prx, rref, A.ch[ch].vr, A.inv_c, prb, qr);
        block_refs<ELC, STR, GRD != 0>((double)blk.xb, (double)blk.yb, ptx, prb, rref, ta, ra, chn.rtrr_mid,
                        A.f0_c, A.fs_c, A.n_ref, live, r, qr, rot.x, rot.y, rot.z, rot.w);
        const bool graze_any = __any(r.graze);
        // the window offset of the first tap rides in the sample fraction, so
        // the floor of the sample position is the window index directly
        r.fb += (float)(r.nb - lo - 3);
        const __amdgpu_buffer_rsrc_t rs = facet_rsrc(A.facets + blk.start, blk.count);
        // speckle records and anchors of the block (unused without speckle)
        const int ng1 = S.n_groups + 1;
        const __amdgpu_buffer_rsrc_t rs_rec = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(S.rec + blk.start), 0, (blk.count + 1) * (int)sizeof(SpkRec), 0x00020000);
        const __amdgpu_buffer_rsrc_t rs_anc = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(S.anch + (size_t)blk.start * ng1), 0,
            (blk.count + 1) * ng1 * (int)sizeof(float4), 0x00020000);
        // A facet's contribution to the lanes' pulses: window index of its
        // first tap, complex weight and tap fraction (sp: its speckle record,
        // unused without speckle).
        struct Dep {
            int n0;            // window index of the first tap
            float wr, wi;      // complex weight (amplitude x phase x gain)
            float f;           // tap fraction (the taps are made at the deposit)
        };
        const auto inside = [](const Dep &d) { return (unsigned)d.n0 <= (unsigned)(WIN - 8); };
        const auto prep = [&](const FacetV &f, [[maybe_unused]] const SpkFacet &sp, Dep &d) {
            float far = f.ar, fai = f.ai, dop = 0.0f;
            if constexpr (SPK) {
                // free path of the group: innovations, prefix sum, end value
                const float2 e = spk_draw(S.key, sp.id, slot, l1);
                float wr = e.x, wi = e.y;
                spk_scan2(wr, wi, sw);
                const float z64r = fmaf(b64, sp.ygr, spk_lane63(wr));
                const float z64i = fmaf(b64, sp.ygi, spk_lane63(wi));
                // x = b^k y_g + (sum up to lane k - 1) + K_k (y_{g+1} - z_64)
                const float xr = fmaf(kk, sp.y1r - z64r, spk_shr1_add(wr, bk * sp.ygr));
                const float xi = fmaf(kk, sp.y1i - z64i, spk_shr1_add(wi, bk * sp.ygi));
                far = fmaf(f.ar, xr, -(f.ai * xi));
                fai = fmaf(f.ar, xi, f.ai * xr);
                // Doppler f_s t_p in cycles, the product split so that its
                // integer part goes without rounding the fraction
                const float dh = sp.fs * thi;
                const float dl = fmaf(sp.fs, tlo, fmaf(sp.fs, thi, -dh));
                dop = __builtin_amdgcn_fractf(dh) + dl;
            }
            Geo g;
            facet_geo<ELC, SPK, STR, GRD>(r, kc, tf, f.dx, f.dy, f.z, f.vx, f.vy, f.vz, graze_any, r.lhi,
                                r.llo, r.fsq, dop, g, &ta, &ra, rot);
            d.n0 = g.fl;
            d.wr = g.amp * fmaf(far, g.cs, -(fai * g.sn));
            d.wi = g.amp * fmaf(far, g.sn, fai * g.cs);
            d.f = g.f;
        };
        // Each lane owns its pulse row, so a deposit is a plain
        // read-modify-write of 8 consecutive complex samples; a lane whose
        // taps leave the window adds zero there and sends them straight to
        // its line (taps inside [0, N)).
        const auto deposit = [&](const Dep &d) {
            const bool inw = inside(d);
            float2 *p = col + 64 * (inw ? d.n0 : 0);
            float2 old[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) old[k] = p[64 * k];
            const float wrl = inw ? d.wr : 0.0f, wil = inw ? d.wi : 0.0f;
            float tap[8];
            taps8(tv, d.f, tap);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                p[64 * k] = make_float2(fmaf(wrl, tap[k], old[k].x), fmaf(wil, tap[k], old[k].y));
            if (!inw && live) {
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int n = d.n0 + lo + k;
                    if (n >= 0 && n < A.N) {
                        unsafeAtomicAdd(iq_row + 2 * n, d.wr * tap[k]);
                        unsafeAtomicAdd(iq_row + 2 * n + 1, d.wi * tap[k]);
                    }
                }
            }
        };
        // Two facets whose taps start at the same window index on every lane
        // (neighbours in a cell mostly do): one read-modify-write for both,
        // with the same additions in the same order as two deposits.
        const auto deposit2 = [&](const Dep &a, const Dep &b) {
            float2 *p = col + 64 * a.n0;
            float2 old[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) old[k] = p[64 * k];
            float ta[8], tb[8];
            taps8(tv, a.f, ta);
            taps8(tv, b.f, tb);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                p[64 * k] = make_float2(fmaf(b.wr, tb[k], fmaf(a.wr, ta[k], old[k].x)),
                                        fmaf(b.wi, tb[k], fmaf(a.wi, ta[k], old[k].y)));
        };
        // Facets in pairs (each pair's taps made and deposited together
        // where they share a window index).  Each record's load is issued as
        // soon as the one before it in its register set is used: with two
        // sets about one facet ahead; with four (kDeep: the wide windows,
        // whose LDS already holds a SIMD to two waves, so registers are
        // there to spare) three facets ahead.
        // (Merging keeps both facets' results live across the second one's
        // geometry: the variants that would lose a wave per SIMD to it, per
        // facet elevation factors without speckle or steering, deposit each
        // facet as soon as it is made.)
        constexpr bool kMerge = ELC || SPK || STR;
        const auto pair_step = [&](FacetV &x, SpkFacet &sx, FacetV &y, SpkFacet &sy, int nx) {
            Dep da, db;
            prep(x, sx, da);
            x = load_facet(rs, nx);
            if constexpr (SPK) sx = load_spk(rs_rec, rs_anc, nx, ng1, gabs);
            if constexpr (!kMerge) deposit(da);
            prep(y, sy, db);
            y = load_facet(rs, nx + 1);
            if constexpr (SPK) sy = load_spk(rs_rec, rs_anc, nx + 1, ng1, gabs);
            if constexpr (kMerge) {
                if (__all(inside(da) && da.n0 == db.n0)) {
                    deposit2(da, db);
                } else {
                    deposit(da);
                    deposit(db);
                }
            } else {
                deposit(db);
            }
        };
        constexpr bool kDeep = WIN >= 32;
        FacetV fa = load_facet(rs, 0), fb = load_facet(rs, 1);
        [[maybe_unused]] SpkFacet sa{}, sb{}, sc{}, sd{};
        if constexpr (SPK) {
            sa = load_spk(rs_rec, rs_anc, 0, ng1, gabs);
            sb = load_spk(rs_rec, rs_anc, 1, ng1, gabs);
        }
        int j = 0;
        if constexpr (kDeep) {
            FacetV fc = load_facet(rs, 2), fd = load_facet(rs, 3);
            if constexpr (SPK) {
                sc = load_spk(rs_rec, rs_anc, 2, ng1, gabs);
                sd = load_spk(rs_rec, rs_anc, 3, ng1, gabs);
            }
            for (; j + 3 < blk.count; j += 4) {
                pair_step(fa, sa, fb, sb, j + 4);
                pair_step(fc, sc, fd, sd, j + 6);
            }
            // one to three facets left: j, j + 1 in (fa, fb), j + 2 in fc
            if (j + 1 < blk.count) {
                pair_step(fa, sa, fb, sb, j + 4);
                j += 2;
                fa = fc;
                sa = sc;
            }
        } else {
            for (; j + 1 < blk.count; j += 2) pair_step(fa, sa, fb, sb, j + 2);
        }
        if (j < blk.count) {
            Dep d;
            prep(fa, sa, d);
            deposit(d);
        }
    }

    // the unit's window to its own slot of the scratch, sample-major like
    // the LDS windows ([sample][pulse row]), plain coalesced stores: the
    // waves' windows added in wave order
    const size_t wslot = ((size_t)ch * A.n_groups + grp) * (size_t)st.seg_max + seg;
    float2 *dst = A.wsum + wslot * 64 * (size_t)A.slot_w;
    __syncthreads();
    for (int e = (int)threadIdx.x; e < 64 * WIN; e += 64 * K) {
        float2 t = accw[e];
#pragma unroll
        for (int k = 1; k < K; ++k) {
            const float2 w = accw[k * kAcc + e];
            t.x += w.x;
            t.y += w.y;
        }
        dst[e] = t;
    }
}

// Persistent workgroups with one work queue per XCD.  Workgroups go to the
// 8 XCDs round-robin by linear index, so workgroup b starts on queue b % 8,
// which holds the segments s with s % 8 == b % 8.  A queue hands out the
// (segment, channel, pulse group) units of a segment band after band (runs
// of B groups, the plan's band length), and within a band channel by
// channel: the units running at one time on an XCD share the segment's
// facet records (the same blocks, or nearly, in neighbouring bands and
// channels) through its L2.  A workgroup whose queue is empty takes units
// from the next queues in turn.  Units of segments a band does not have,
// or of groups past the last, return at once.  Each workgroup leaves after
// one failed take per queue, so every workgroup ends; each unit writes only
// its own window slot, so the result does not depend on who ran it.
// Variants that deposit facets one at a time (no pair merge: per-facet
// elevation factors without speckle or steering) are held to three waves
// per SIMD (168 VGPRs) where the LDS allows three (windows of up to 26
// samples: three workgroups of 53 KB); the others take what their
// registers allow.
template <int WIN, bool ELC, bool SPK, bool STR>
constexpr int fwd_min_waves() {
    return (WIN <= 26 && !(ELC || SPK || STR)) ? 3 : 1;
}

template <int WIN, bool ELC, bool SPK, bool STR, int GRD>
__global__ __launch_bounds__(64 * fwd_waves<WIN>())
__attribute__((amdgpu_waves_per_eu(fwd_min_waves<WIN, ELC, SPK, STR>()))) void k_forward(FwdArgs A) {
    __shared__ float2 acc[fwd_waves<WIN>() * 64 * WIN];
    __shared__ unsigned s_unit;
    const unsigned B = (unsigned)A.st.B, C = (unsigned)A.C, G = (unsigned)A.n_groups;
    const unsigned per_seg = C * ((G + B - 1) / B) * B;
    const unsigned segs = (unsigned)A.st.seg_max;
    for (unsigned k = 0; k < kFwdQueues; ++k) {
        const unsigned q = (blockIdx.x + k) % kFwdQueues;
        const unsigned units = (segs > q ? (segs - q + kFwdQueues - 1) / kFwdQueues : 0u) * per_seg;
        for (;;) {
            __syncthreads();   // the last unit's flush has read the windows
            if (threadIdx.x == 0) s_unit = atomicAdd(A.counter + q, 1u);
            __syncthreads();
            const unsigned u = (unsigned)__builtin_amdgcn_readfirstlane((int)s_unit);
            if (u >= units) break;
            const unsigned j = u / per_seg, rest = u - j * per_seg;
            const unsigned band = rest / (C * B), rem = rest - band * (C * B);
            const unsigned ch = rem / B, grp = band * B + (rem - ch * B);
            if (grp >= G) continue;
            forward_unit<WIN, ELC, SPK, STR, GRD>(A, acc, (int)(q + kFwdQueues * j), (int)grp,
                                                 (int)ch);
        }
    }
}

// One wave per (sample, pulse group, channel), lane = pulse row, over the
// span of sample positions the windows of the group's band can reach: the
// wave gathers, in strip order and within a strip in segment order, the
// windows of the segments of every strip whose window holds the sample (one
// coalesced 512-byte row of each slot) and adds the sums to the 64 lines.
// Window origins follow from the strip index as in the forward kernel, so
// the strips holding a sample are a run of consecutive strips, the same for
// every lane.  Every sample of every line has one writer, and the order of
// the additions is fixed.
__global__ __launch_bounds__(64 * kReduceTile) void k_window_reduce(ReduceArgs A) {
    // consecutive workgroups: consecutive sample tiles of one pulse group, so
    // their partial writes to the same IQ lines meet in the L2
    const int grp = (int)(blockIdx.x / (unsigned)A.n_tiles), ch = blockIdx.y;
    const unsigned tile_id = blockIdx.x - (unsigned)grp * (unsigned)A.n_tiles;
    const int row = (int)(threadIdx.x & 63);
    const int gbase = (A.g0 + grp) * A.gstride - A.poff;
    const int pl = gbase + row;
    const StripPlan &st = A.st;
    int pc = A.p0 + gbase + 32;
    pc = pc < 0 ? 0 : (pc < A.Np ? pc : A.Np - 1);
    int band = pc / (64 * st.B);
    band = band < st.NB ? band : st.NB - 1;
    const size_t bc = (size_t)band * A.C + ch;
    const int *segoff = st.segoff + bc * (st.NS + 1);
    if (segoff[st.NS] == 0) return;
    const double *bd = st.band + 4 * bc;
    const double umin = bd[0], S = bd[1], mg = bd[2];
    // first sample of strip s's window (the forward kernel's expression)
    const auto lo_of = [&](int s) { return (int)floor(umin + (double)s * S - mg) - 3; };
    const int W = (int)bd[3];   // the band's window width (slots are A.win wide)
    const int n = lo_of(0) + (int)tile_id * kReduceTile +
                  __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (n < 0 || n >= A.N) return;
    // s1: the last strip with lo <= n; s0: the first whose window reaches n
    int s1 = (int)floor(((double)n + 3.0 - umin + mg) / S);
    s1 = s1 < 0 ? 0 : (s1 < st.NS ? s1 : st.NS - 1);
    while (s1 + 1 < st.NS && lo_of(s1 + 1) <= n) ++s1;
    while (s1 >= 0 && lo_of(s1) > n) --s1;
    int s0 = s1 + 1;
    while (s0 > 0 && lo_of(s0 - 1) + W > n) --s0;
    const size_t slot0 = ((size_t)ch * A.n_groups + grp) * (size_t)st.seg_max;
    const size_t seg_stride = (size_t)64 * A.win;
    float2 acc = make_float2(0.f, 0.f);
    bool any = false;
    for (int s = s0; s <= s1; ++s) {
        const int a = segoff[s], b = segoff[s + 1];
        if (a == b) continue;
        any = true;
        const float2 *p = A.wsum + (slot0 + a) * seg_stride + (size_t)(n - lo_of(s)) * 64 + row;
#pragma unroll 4
        for (int q = 0; q < b - a; ++q) {
            const float2 v = p[(size_t)q * seg_stride];
            acc.x += v.x;
            acc.y += v.y;
        }
    }
    if (!any || pl < 0 || pl >= A.np) return;
    float2 &o = A.iq[((size_t)ch * A.np + pl) * (size_t)A.N + n];
    o = make_float2(o.x + acc.x, o.y + acc.y);
}

}  // namespace

hipError_t launch_forward(const FwdArgs &a, int C, int win, bool el_const, bool speckle,
                          hipStream_t s) {
    if (a.st.seg_max == 0 || a.np == 0 || a.n_groups == 0) return hipSuccess;
    const unsigned long long B = (unsigned long long)(a.st.B > 0 ? a.st.B : 1);
    const unsigned long long units = (unsigned long long)a.st.seg_max * (unsigned long long)C *
                                     (((unsigned long long)a.n_groups + B - 1) / B * B);
    if (a.st.B <= 0 || units > 0xffffffffULL) return hipErrorInvalidConfiguration;
    // persistent workgroups: 16 waves per compute unit (at least as many as
    // the LDS windows and the registers let run at once)
    static int n_cu = 0;
    if (n_cu == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n_cu <= 0)
            n_cu = 256;
    }
    const auto grid_for = [&](int waves) {
        const unsigned long long cap = (unsigned long long)n_cu * 16ULL / (unsigned long long)waves;
        return dim3((unsigned)(units < cap ? units : cap));
    };
    // gridded patterns are always evaluated per facet (no elevation factor
    // at block centres); a.grid = 2 when every antenna has a table
#define HS_FWD4(W, T)                                                                       \
    if (a.grid == 2) {                                                                      \
        if (speckle) hipLaunchKernelGGL((k_forward<W, false, true, T, 2>), grid_for(fwd_waves<W>()), dim3(64 * fwd_waves<W>()), 0, s, a); \
        else hipLaunchKernelGGL((k_forward<W, false, false, T, 2>), grid_for(fwd_waves<W>()), dim3(64 * fwd_waves<W>()), 0, s, a); \
    } else if (a.grid) {                                                                    \
        if (speckle) hipLaunchKernelGGL((k_forward<W, false, true, T, 1>), grid_for(fwd_waves<W>()), dim3(64 * fwd_waves<W>()), 0, s, a); \
        else hipLaunchKernelGGL((k_forward<W, false, false, T, 1>), grid_for(fwd_waves<W>()), dim3(64 * fwd_waves<W>()), 0, s, a); \
    } else if (speckle) {                                                                   \
        if (el_const) hipLaunchKernelGGL((k_forward<W, true, true, T, 0>), grid_for(fwd_waves<W>()), dim3(64 * fwd_waves<W>()), 0, s, a); \
        else hipLaunchKernelGGL((k_forward<W, false, true, T, 0>), grid_for(fwd_waves<W>()), dim3(64 * fwd_waves<W>()), 0, s, a); \
    } else {                                                                                \
        if (el_const) hipLaunchKernelGGL((k_forward<W, true, false, T, 0>), grid_for(fwd_waves<W>()), dim3(64 * fwd_waves<W>()), 0, s, a); \
        else hipLaunchKernelGGL((k_forward<W, false, false, T, 0>), grid_for(fwd_waves<W>()), dim3(64 * fwd_waves<W>()), 0, s, a); \
    }
#define HS_FWD(W)                                                                           \
    case W:                                                                                 \
        if (a.steer) {                                                                      \
            HS_FWD4(W, true)                                                                \
        } else {                                                                            \
            HS_FWD4(W, false)                                                               \
        }                                                                                   \
        break;
    switch (win) {
        HS_FWD(24)
        HS_FWD(26)
        HS_FWD(32)
        HS_FWD(48)
        HS_FWD(64)
        default: return hipErrorInvalidValue;
    }
#undef HS_FWD
#undef HS_FWD4
    return hipGetLastError();
}

hipError_t launch_window_reduce(const ReduceArgs &a, hipStream_t s) {
    if (a.np == 0 || a.n_groups == 0) return hipSuccess;
    const unsigned long long blocks = (unsigned long long)a.n_groups * (unsigned long long)a.n_tiles;
    if (a.n_tiles <= 0 || blocks > 0xffffffffULL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_window_reduce, dim3((unsigned)blocks, (unsigned)a.C),
                       dim3(64 * kReduceTile), 0, s, a);
    return hipGetLastError();
}

}  // namespace hs
