// Fused forward facet sum for gfx950.
//
// Each (channel, pulse) line receives, from every facet, a * F_tx * F_rx * S *
// exp(-j 2 pi f0 R / c) (Sec. III.A eq. 3, Sec. III.B eq. 16) spread around the
// facet's fractional sample u = n_ref + (R - c tau_ref) fs / c by an 8-tap
// Kaiser-windowed sinc (the range slices of eq. 17).
//
// Work decomposition (one workgroup = one wave):
//   blockIdx.x = (patch of spatial blocks, group of 64 pulses), decoded so
//   that the groups of one patch share an XCD (below); blockIdx.y = channel.
//   Lane = pulse: every lane handles the same facet
//   (its 32-byte record arrives by two uniform buffer loads) and deposits into
//   its own pulse column of an LDS range window.  Since no other lane or wave
//   touches that column, the deposit is a plain read-modify-write (8 x 64-bit
//   reads issued as soon as the sample index is known, 16 FMAs, 8 x 64-bit
//   writes) instead of LDS atomics, which serialise per lane on gfx950.  The
//   window is stored sample-major ([sample][lane]), so the 64 lanes of one
//   access always fall on distinct bank pairs whatever their sample indices:
//   a lane-major layout conflicts as soon as the lanes' sample indices
//   differ.  At the end the window is flushed to the
//   IQ lines with global float atomics, since neighbouring patches overlap in
//   range.  A contribution whose taps leave the window (only for geometries
//   the patch sizing did not foresee) goes straight to global memory.
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

// The flush of windows up to this width goes through a transposed copy in
// LDS, so that one atomic instruction covers contiguous samples of one line.
constexpr int kFlushTransposeMax = 32;

// SPK: the intra-facet speckle of eq. 7 multiplies each facet's amplitude by
// x(p) and adds f_s t_p cycles to its phase.  Pulse groups are then aligned
// on absolute pulse indices (multiples of 64), so that a wave holds exactly
// one group of the speckle process; lanes before p0 or past the last pulse
// take part in the prefix sum but deposit nothing.
// STR: antenna frames turn with time (steering): per-pulse frames.
// GRD: field patterns from u-v tables (1: on some antennas, 2: on all),
// evaluated per facet (never with ELC).
template <int WIN, bool ELC, bool SPK, bool STR, int GRD>
__global__ __launch_bounds__(64) void k_forward(FwdArgs A) {
    // [sample][lane] during the sum; [lane][WIN + 1] for the flush
    constexpr int kAcc = WIN <= kFlushTransposeMax ? 64 * (WIN + 1) : 64 * WIN;
    __shared__ float2 acc[kAcc];

    // Workgroup -> (patch, pulse group).  Workgroups go to the 8 XCDs
    // round-robin by linear index, so index L runs on XCD L % 8.  All pulse
    // groups of one patch get the same L % 8 and consecutive L / 8: they run
    // on one XCD close in time and read the patch's facet records from its
    // L2 instead of HBM.
    const int poff = SPK ? (A.p0 & 63) : 0;     // lanes before p0 in the first group
    const int G = A.n_groups;
    const unsigned L = blockIdx.x, r8 = L >> 3;
    const int grp = (int)(r8 % (unsigned)G);
    const int patch = (int)((r8 / (unsigned)G) * 8u + (L & 7u));
    const int ch = blockIdx.y;
    if (patch >= A.n_patches) return;
    const cptr<int> patch_first = (cptr<int>)A.patch_first;
    const cptr<BlockRec> blocks = (cptr<BlockRec>)A.blocks;
    const int b0 = patch_first[patch], b1 = patch_first[patch + 1];
    if (b0 == b1) return;
    const int lane = threadIdx.x;
    const int gbase = grp * A.gstride - poff;  // pulse (relative to p0) of lane 0
    const int pl = gbase + lane;               // pulse relative to p0, also its output row
    const bool live = pl >= 0 && pl < A.np;
    const int plc = pl < 0 ? 0 : (pl < A.np ? pl : A.np - 1);
    const PulseRec *PR = A.pulses + (size_t)ch * A.Np + A.p0;
    const ChanArgs chn = A.ch[ch];
    const AntArgs &ta = A.ant[chn.tx], &ra = A.ant[chn.rx];
    FacetConsts kc;
    facet_consts(ta, ra, kc);

    // Range window of this (patch, pulse group): sample positions of the
    // patch corners at the group's first and last pulse (lanes 0..7), widened
    // by the halo (facet heights, drift) and the taps.
    int lo;
    {
        double umin = 1e300, umax = -1e300;
        if (lane < 8) {
            const Lattice &L = A.lat;
            const int px = patch % L.npx, py = patch / L.npx;
            const double cx0 = (double)(L.bx0 + (long long)px * L.px);
            const double cy0 = (double)(L.by0 + (long long)py * L.py);
            const double xc = ((lane & 1) ? cx0 + L.px : cx0) * L.edge;
            const double yc = ((lane & 2) ? cy0 + L.py : cy0) * L.edge;
            int pe = gbase + ((lane & 4) ? 63 : 0);
            pe = pe < 0 ? 0 : (pe < A.np ? pe : A.np - 1);
            const PulseRec &Q = PR[pe];
            const double a0 = xc - Q.ptx[0], a1 = yc - Q.ptx[1], a2 = -Q.ptx[2];
            const double c0 = xc - Q.prx[0], c1 = yc - Q.prx[1], c2 = -Q.prx[2];
            const double R = sqrt(a0 * a0 + a1 * a1 + a2 * a2) + sqrt(c0 * c0 + c1 * c1 + c2 * c2);
            umin = umax = A.n_ref + (R - Q.rref) * A.fs_c;
        }
#pragma unroll
        for (int off = 1; off < 8; off <<= 1) {
            umin = fmin(umin, __shfl_xor(umin, off));
            umax = fmax(umax, __shfl_xor(umax, off));
        }
        int l = (int)floor(umin) - A.halo - 3;
        const int h = (int)ceil(umax) + A.halo + 4;
        if (h - l + 1 > WIN) l = ((l + h) >> 1) - WIN / 2;
        lo = __builtin_amdgcn_readfirstlane(l);
    }
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

    for (int b = b0; b < b1; ++b) {
        const BlockRec blk = load_block(blocks + b);
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
        FacetV fn = load_facet(rs, 0);
        // speckle records and anchors of the block (unused without speckle)
        const int ng1 = S.n_groups + 1;
        const __amdgpu_buffer_rsrc_t rs_rec = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(S.rec + blk.start), 0, (blk.count + 1) * (int)sizeof(SpkRec), 0x00020000);
        const __amdgpu_buffer_rsrc_t rs_anc = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(S.anch + (size_t)blk.start * ng1), 0,
            (blk.count + 1) * ng1 * (int)sizeof(float4), 0x00020000);
        [[maybe_unused]] SpkFacet sn{};
        if constexpr (SPK) sn = load_spk(rs_rec, rs_anc, 0, ng1, gabs);
        for (int j = 0; j < blk.count; ++j) {
            const FacetV f = fn;
            fn = load_facet(rs, j + 1);
            float far = f.ar, fai = f.ai, dop = 0.0f;
            if constexpr (SPK) {
                const SpkFacet sp = sn;
                sn = load_spk(rs_rec, rs_anc, j + 1, ng1, gabs);
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
            // Each lane owns its pulse row, so the deposit is a plain
            // read-modify-write of 8 consecutive complex samples.
            const int n0 = g.fl;                  // window index of the first tap
            const bool inw = (unsigned)n0 <= (unsigned)(WIN - 8);
            float2 *p = col + 64 * (inw ? n0 : 0);
            float2 old[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) old[k] = p[64 * k];
            // a lane outside the window adds zero to its row (and goes below)
            const float al = inw ? g.amp : 0.0f;
            const float wrl = al * fmaf(far, g.cs, -(fai * g.sn));
            const float wil = al * fmaf(far, g.sn, fai * g.cs);
            float tap[8];
            taps8(tv, g.f, tap);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                p[64 * k] = make_float2(fmaf(wrl, tap[k], old[k].x), fmaf(wil, tap[k], old[k].y));
            if (!inw && live) {
                const float wr = g.amp * fmaf(far, g.cs, -(fai * g.sn));
                const float wi = g.amp * fmaf(far, g.sn, fai * g.cs);
                // outside the window: straight to the line, taps inside [0, N)
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int n = n0 + lo + k;
                    if (n >= 0 && n < A.N) {
                        unsafeAtomicAdd(iq_row + 2 * n, wr * tap[k]);
                        unsafeAtomicAdd(iq_row + 2 * n + 1, wi * tap[k]);
                    }
                }
            }
        }
    }

    // flush the window into the lines (zeros skipped); neighbouring patches
    // overlap in range, hence the atomics
    if constexpr (WIN <= kFlushTransposeMax) {
        // each lane takes its pulse row into registers, then writes it back
        // lane-major with one pad sample (conflict-free both ways); line p is
        // then flushed by lanes 0 .. 2 WIN - 1, one float each
        float2 v[WIN];
#pragma unroll
        for (int i = 0; i < WIN; ++i) v[i] = col[64 * i];
        float2 *rowp = acc + lane * (WIN + 1);
#pragma unroll
        for (int i = 0; i < WIN; ++i) rowp[i] = v[i];
        const float *accf = reinterpret_cast<const float *>(acc);
        const int n = lo + (lane >> 1);
        const bool lane_in = lane < 2 * WIN && n >= 0 && n < A.N;
        const int rbase = gbase;               // line (relative to p0) of lane 0
        const int pbeg = rbase < 0 ? -rbase : 0;
        const int pend = (A.np - rbase) < 64 ? (A.np - rbase) : 64;
        float *line = A.iq + 2 * ((size_t)ch * A.np * (size_t)A.N) + 2 * (ptrdiff_t)lo + lane;
        for (int p = pbeg; p < pend; ++p) {
            const float x = lane < 2 * WIN ? accf[p * 2 * (WIN + 1) + lane] : 0.0f;
            if (lane_in && x != 0.0f) unsafeAtomicAdd(line + 2 * (size_t)(rbase + p) * A.N, x);
        }
    } else if (live) {
        float *dst = A.iq + 2 * (((size_t)ch * A.np + pl) * (size_t)A.N);
        for (int bin = 0; bin < WIN; ++bin) {
            const int n = lo + bin;
            const float2 v = col[64 * bin];
            if (n < 0 || n >= A.N || (v.x == 0.0f && v.y == 0.0f)) continue;
            unsafeAtomicAdd(dst + 2 * n, v.x);
            unsafeAtomicAdd(dst + 2 * n + 1, v.y);
        }
    }
}

}  // namespace

hipError_t launch_forward(const FwdArgs &a, int C, int win, bool el_const, bool speckle,
                          hipStream_t s) {
    if (a.n_patches == 0 || a.np == 0) return hipSuccess;
    // (patch, pulse group) pairs, patches padded to a multiple of the 8 XCDs;
    // speckle groups are aligned on absolute pulse indices
    const unsigned long long groups = (unsigned long long)a.n_groups;
    const unsigned long long wgs = groups * (((unsigned long long)a.n_patches + 7) / 8 * 8);
    if (wgs > 0xffffffffULL) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)wgs, (unsigned)C);
    // gridded patterns are always evaluated per facet (no elevation factor
    // at block centres); a.grid = 2 when every antenna has a table
#define HS_FWD4(W, T)                                                                       \
    if (a.grid == 2) {                                                                      \
        if (speckle) hipLaunchKernelGGL((k_forward<W, false, true, T, 2>), grid, dim3(64), 0, s, a); \
        else hipLaunchKernelGGL((k_forward<W, false, false, T, 2>), grid, dim3(64), 0, s, a); \
    } else if (a.grid) {                                                                    \
        if (speckle) hipLaunchKernelGGL((k_forward<W, false, true, T, 1>), grid, dim3(64), 0, s, a); \
        else hipLaunchKernelGGL((k_forward<W, false, false, T, 1>), grid, dim3(64), 0, s, a); \
    } else if (speckle) {                                                                   \
        if (el_const) hipLaunchKernelGGL((k_forward<W, true, true, T, 0>), grid, dim3(64), 0, s, a); \
        else hipLaunchKernelGGL((k_forward<W, false, true, T, 0>), grid, dim3(64), 0, s, a); \
    } else {                                                                                \
        if (el_const) hipLaunchKernelGGL((k_forward<W, true, false, T, 0>), grid, dim3(64), 0, s, a); \
        else hipLaunchKernelGGL((k_forward<W, false, false, T, 0>), grid, dim3(64), 0, s, a); \
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
        HS_FWD(32)
        HS_FWD(48)
        HS_FWD(64)
        default: return hipErrorInvalidValue;
    }
#undef HS_FWD
#undef HS_FWD4
    return hipGetLastError();
}

}  // namespace hs
