// Fused forward facet sum for gfx950.
//
// Each (channel, pulse) line receives, from every facet, a * F_tx * F_rx * S *
// exp(-j 2 pi f0 R / c) (Sec. III.A eq. 3, Sec. III.B eq. 16) spread around the
// facet's fractional sample u = n_ref + (R - c tau_ref) fs / c by an 8-tap
// Kaiser-windowed sinc (the range slices of eq. 17).
//
// Work decomposition (one workgroup = 4 waves):
//   blockIdx.x = patch of spatial blocks, blockIdx.y = group of 64 pulses,
//   blockIdx.z = channel.  Lane = pulse: every lane of a wave handles the same
//   facet (its 32-byte record arrives through one scalar load) and deposits
//   into its own pulse row of an LDS range window, so no two lanes of a wave
//   touch the same LDS word.  The four waves take interleaved blocks of the
//   patch and share the window (ds_add_f32).  At the end the window is
//   flushed to the IQ lines with global float atomics, since neighbouring
//   patches overlap in range.  A contribution whose taps leave the window
//   (only for geometries the patch sizing did not foresee) goes straight to
//   global memory.
#include "sim_device.h"

namespace hs {

namespace {

template <int WIN>
__global__ __launch_bounds__(256) void k_forward(FwdArgs A) {
    constexpr int STRIDE = 2 * WIN + 1;     // odd: the 64 rows start in distinct banks
    __shared__ float acc[64 * STRIDE];
    __shared__ int s_lo;

    const int patch = blockIdx.x, grp = blockIdx.y, ch = blockIdx.z;
    const int b0 = A.patch_first[patch], b1 = A.patch_first[patch + 1];
    if (b0 == b1) return;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int pl = grp * 64 + lane;          // pulse relative to p0
    const bool live = pl < A.np;
    const int plc = live ? pl : (A.np - 1);
    const PulseRec *PR = A.pulses + (size_t)ch * A.Np + A.p0;
    const ChanConst &cc = A.ch[ch];

    // Range window of this (patch, pulse group): sample positions of the
    // patch corners at the group's first and last pulse, widened by the halo
    // (facet heights and drift) and the taps.
    if (wave == 0) {
        double umin = 1e300, umax = -1e300;
        if (lane < 8) {
            const Lattice &L = A.lat;
            const int px = patch % L.npx, py = patch / L.npx;
            const double cx0 = (double)(L.bx0 + (long long)px * L.px);
            const double cy0 = (double)(L.by0 + (long long)py * L.py);
            const double xc = ((lane & 1) ? cx0 + L.px : cx0) * L.edge;
            const double yc = ((lane & 2) ? cy0 + L.py : cy0) * L.edge;
            int pe = grp * 64 + ((lane & 4) ? 63 : 0);
            pe = pe < A.np ? pe : A.np - 1;
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
        if (lane == 0) {
            int lo = (int)floor(umin) - A.halo - 3;
            const int hi = (int)ceil(umax) + A.halo + 4;
            if (hi - lo + 1 > WIN) lo = ((lo + hi) >> 1) - WIN / 2;
            s_lo = lo;
        }
    }
    for (int i = threadIdx.x; i < 64 * STRIDE; i += 256) acc[i] = 0.0f;
    __syncthreads();
    const int lo = s_lo;

    const PulseRec &P = PR[plc];
    const double ptx[3] = {P.ptx[0], P.ptx[1], P.ptx[2]};
    const double prx[3] = {P.prx[0], P.prx[1], P.prx[2]};
    const double rref = P.rref;
    const float tf = (float)P.t;
    float *row = acc + lane * STRIDE;
    float *iq_row = A.iq + 2 * ((size_t)ch * A.np + plc) * (size_t)A.N;

    for (int b = b0 + wave; b < b1; b += 4) {
        const BlockRec blk = A.blocks[b];
        Refs r;
        block_refs((double)blk.xb, (double)blk.yb, ptx, prx, rref, cc, A.f0_c, A.fs_c, A.n_ref,
                   live, r);
        const bool graze_any = __any(r.graze);
        const int nb0 = r.nb - lo - 3;
        const int j1 = blk.start + blk.count;
        // the sorted facet array carries one padding record, so the look-ahead
        // load of the next facet is always in bounds
        FacetRec fn = A.facets[blk.start];
        for (int j = blk.start; j < j1; ++j) {
            const FacetRec f = fn;
            fn = A.facets[j + 1];
            Geo g;
            facet_geo(r, cc, tf, f.dx, f.dy, f.z, f.vx, f.vy, f.vz, graze_any, A.linv_hi,
                      A.linv_lo, A.fs_cf, g);
            const float wr = g.amp * fmaf(f.ar, g.cs, -(f.ai * g.sn));
            const float wi = g.amp * fmaf(f.ar, g.sn, f.ai * g.cs);
            float tap[8];
            taps8(A.tp, g.f, tap);
            const int n0 = nb0 + g.fl;            // window index of the first tap
            if ((unsigned)n0 <= (unsigned)(WIN - 8)) {
                float *p = row + 2 * n0;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    __hip_atomic_fetch_add(p + 2 * k, wr * tap[k], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                    __hip_atomic_fetch_add(p + 2 * k + 1, wi * tap[k], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            } else if (live) {
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
    __syncthreads();

    // flush the window into the lines (zeros skipped)
    for (int i = threadIdx.x; i < 64 * WIN; i += 256) {
        const int p = i / WIN, bin = i % WIN;
        const int n = lo + bin;
        const int pp = grp * 64 + p;
        if (pp >= A.np || n < 0 || n >= A.N) continue;
        const float vr = acc[p * STRIDE + 2 * bin], vi = acc[p * STRIDE + 2 * bin + 1];
        if (vr == 0.0f && vi == 0.0f) continue;
        float *dst = A.iq + 2 * (((size_t)ch * A.np + pp) * (size_t)A.N + n);
        unsafeAtomicAdd(dst, vr);
        unsafeAtomicAdd(dst + 1, vi);
    }
}

}  // namespace

hipError_t launch_forward(const FwdArgs &a, int C, hipStream_t s) {
    if (a.n_patches == 0 || a.np == 0) return hipSuccess;
    dim3 grid((unsigned)a.n_patches, (unsigned)((a.np + 63) / 64), (unsigned)C);
    hipLaunchKernelGGL(k_forward<64>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace hs
