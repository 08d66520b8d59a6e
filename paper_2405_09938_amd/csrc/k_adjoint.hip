// Adjoint of the facet sum with respect to facet height, velocity and complex
// amplitude, for gfx950.
//
// With g = dL/dRe(IQ) + j dL/dIm(IQ), one facet's contribution to line (c, p)
// is W h(n - u), W = a T E, T = F_tx F_rx S, E = exp(j phi).  Writing
// B = sum_n conj(g_n) h(n - u) and B_u = sum_n conj(g_n) dh(n - u)/du,
//   dL/da = conj(B T E),
//   dL/dX = Re(B a E) grad T + [Im(B a E) T K0 + Re(B_u a T E) fs/c] grad R,
// with K0 = 2 pi f0 / c and grad R = d_tx + d_rx (unit vectors antenna ->
// facet).  dL/dz = sum_p (dL/dX)_z and dL/dV = sum_p t_p dL/dX (X = X0 + V t_p).
// grad R is the facet's own to first order in its offset e from the block
// centre (d_leg + (e - (e.d_leg) d_leg) / R_leg per leg, which matters at
// airborne ranges where e/R reaches 1e-4); grad T, whose share of dL/dX is
// ~1e-4 at 15 km and ~1e-6 at 850 km, is taken at the block centre, with a
// first-order correction J e (J its Jacobian there, by central differences
// in the stage prologue) where the plan's far-field bound fails (near-field
// geometries, which also evaluate every pattern factor per facet);
// everything else is recomputed exactly as in the forward kernel.
//
// Work decomposition: one wave per spatial block, lane = facet (<= 64 per
// block).  The wave loops over channels and over stages of 32 pulses; per
// stage, lanes 0..31 compute the FP64 block references of one pulse each into
// LDS.  Then, per sub-stage of 8 pulses, the wave builds a table of the two
// tap sums' coefficients as polynomials in the facet's tap fraction, one
// entry per (pulse, first-tap sample) for the 8 first-tap samples around the
// block centre's (lane = entry, from the samples of g under its 8 taps), and
// every lane walks the 8 pulses reading references as LDS broadcasts and its
// own entry: the tap sums B and dB/du cost two short polynomials per facet
// and pulse instead of 8 taps, their derivatives and 32 products.  A facet
// whose taps start outside the table reads g from memory.  Each facet's
// gradient accumulates in registers over all pulses and channels and is
// written once: no atomics, deterministic.
#include "sim_device.h"
#include "spk_device.h"

#ifndef HEEPS_ADJ_SPLIT
#define HEEPS_ADJ_SPLIT 1
#endif

namespace hs {

namespace {

constexpr int kStage = 32;   // pulses per stage
constexpr int kSub = 8;      // pulses per coefficient table (a stage holds four)
constexpr int kNI = 8;       // table intervals per pulse: first tap at window index 0 .. 7

// staged record layout (floats)
enum {
    R_T = 0, R_DTX, R_DTY, R_DTZ, R_GX, R_GY, R_GZ, R_I2RT, R_I2RR, R_PHIB, R_FB, R_NB,
    R_GTAZ, R_GTEL, R_GRAZ, R_GREL, R_IRT, R_IRT2, R_IRR, R_IRR2, R_SB, R_SBT, R_SBR, R_MASK,
    R_DTGX, R_DTGY, R_DTGZ, R_DBT, R_DBR, R_GRAZE, R_I2S,
    R_J0,        // 9 floats: J[i][j] = d(grad T)_i / dx_j at R_J0 + 3 i + j
    R_LHI = 40, R_LLO, R_FSQ,   // q f0/c (two floats), q fs/c
    R_Q,         // q: range-offset factor of the facet's own echo time (1 if off)
    R_TLO        // t_p - float(t_p) (speckle: the Doppler phase)
};

// floats per staged pulse record (a multiple of 4); with steering, four more
// from R_ST0<SPK> on: cos, sin of the Tx and of the Rx steering angle
template <bool SPK>
constexpr int R_ST0 = SPK ? 48 : 44;
template <bool SPK, bool STR>
constexpr int kNRef = R_ST0<SPK> + (STR ? 4 : 0);

// Gradient of one antenna's field pattern at the block centre (FP32 from the
// FP64 geometry): dF/dX = ka sinc'(ka u) sinc(ke v) (az - u d)/R
//                        + ke sinc(ka u) sinc'(ke v) (el - v d)/R.
// GRD: the field of an antenna with a u-v grid from that grid (the others keep
// the sinc); dF/du, dF/dv are its cell slopes (bilinear: piecewise linear
// along each axis).
template <bool STR, int GRD>
__device__ __forceinline__ float ant_grad(const AntArgs &a, double d0, double d1, double d2,
                                          double ir, float *gr, double cs, double sn) {
    const double u0 = d0 * ir, u1 = d1 * ir, u2 = d2 * ir;
    // azimuth axis, turned by the steering angle if STR
    double az[3] = {a.az[0], a.az[1], a.az[2]};
    if constexpr (STR) {
#pragma unroll
        for (int k = 0; k < 3; ++k) az[k] = a.az[k] * cs - a.b[k] * sn;
    }
    const double u = u0 * az[0] + u1 * az[1] + u2 * az[2];
    const double v = u0 * a.el[0] + u1 * a.el[1] + u2 * a.el[2];
    if (GRD == 2 || (GRD != 0 && a.grid)) {   // uniform: the workgroup's channel's antenna
        const float x = (float)(u * a.gidu) - a.gu0, y = (float)(v * a.gidv) - a.gv0;
        const bool in = (x >= 0.0f) & (x < a.gnu1) & (y >= 0.0f) & (y < a.gnv1);
        const float fx = floorf(x), fy = floorf(y);
        const int idx = in ? (int)fy * a.gstride + (int)fx : 0;
        const float4 c = a.grid[idx];
        const float ax = x - fx, ay = y - fy;
        const float d10 = c.y - c.x, d32 = c.w - c.z;
        const float lo = fmaf(ax, d10, c.x), hi = fmaf(ax, d32, c.z);
        const float fu = in ? fmaf(ay, d32 - d10, d10) * (float)a.gidu : 0.0f;
        const float fv = in ? (hi - lo) * (float)a.gidv : 0.0f;
        const float irf = (float)ir;
        const double uu[3] = {u0, u1, u2};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float gu = (float)(az[k] - u * uu[k]) * irf;
            const float gv = (float)(a.el[k] - v * uu[k]) * irf;
            gr[k] = fmaf(fu, gu, fv * gv);
        }
        return in ? fmaf(ay, hi - lo, lo) : 0.0f;
    }
    const float xa = (float)(a.ka * u), xe = (float)(a.ke * v);
    const float su = sinc_f(xa), sv = sinc_f(xe);
    const float dsu = (float)a.ka * dsinc_f(xa), dsv = (float)a.ke * dsinc_f(xe);
    const float irf = (float)ir;
    const double uu[3] = {u0, u1, u2};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float gu = (float)(az[k] - u * uu[k]) * irf;
        const float gv = (float)(a.el[k] - v * uu[k]) * irf;
        gr[k] = dsu * sv * gu + su * dsv * gv;
    }
    return su * sv;
}

// grad T = grad(F_tx F_rx S) at the point (X, Y, Z), S = R_t,mid R_r,mid /
// (R_t R_r) the spreading (without the mask).
template <bool STR, int GRD>
__device__ __forceinline__ void grad_t(const AntArgs &ta, const AntArgs &ra, double rtrr_mid,
                                       double X, double Y, double Z, const double *ptx,
                                       const double *prx, float *out, double cst, double snt,
                                       double csr, double snr) {
    const double dt0 = X - ptx[0], dt1 = Y - ptx[1], dt2 = Z - ptx[2];
    const double dr0 = X - prx[0], dr1 = Y - prx[1], dr2 = Z - prx[2];
    const double irt = 1.0 / sqrt(dt0 * dt0 + dt1 * dt1 + dt2 * dt2);
    const double irr = 1.0 / sqrt(dr0 * dr0 + dr1 * dr1 + dr2 * dr2);
    float gft[3], gfr[3];
    const float ft = ant_grad<STR, GRD>(ta, dt0, dt1, dt2, irt, gft, cst, snt);
    const float fr = ant_grad<STR, GRD>(ra, dr0, dr1, dr2, irr, gfr, csr, snr);
    const double sb = rtrr_mid * irt * irr;
    const double d[3][2] = {{dt0, dr0}, {dt1, dr1}, {dt2, dr2}};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float gs = (float)(-sb * (d[k][0] * irt * irt + d[k][1] * irr * irr));
        out[k] = fr * (float)sb * gft[k] + ft * (float)sb * gfr[k] + ft * fr * gs;
    }
}

// SPK: the facet amplitude carries the intra-facet speckle x(p) and its phase
// the Doppler f_s t_p (eq. 7).  Each lane follows its facet's process pulse by
// pulse: at a group start x = y_g, then z = b z + sqrt(1 - b^2) e_p and
// x = z + K_k D_g with (y_g, D_g) from the preparation pass.
// STR: antenna frames turn with time (steering): the per-pulse angles are
// staged with the references and the facet-part constants rebuilt per pulse.
// GRD: gridded patterns (1: on some antennas, 2: on all), always evaluated
// per facet; ELC then only drops the first-order Jacobian correction of
// grad T (far-field plans, as for the sinc pattern with its elevation
// factors at block centres).
template <bool ELC, bool SPK, bool STR, int GRD>
__global__ __launch_bounds__(64) void k_adjoint(AdjArgs A) {
    constexpr bool kElc = ELC && GRD == 0;   // elevation factors at block centres
    // the stage's references computed two lanes per pulse (Tx and Rx legs)
    constexpr bool kSplit = HEEPS_ADJ_SPLIT && kElc && !STR;
    static_assert(!kSplit || 2 * kStage == 64, "a Tx and an Rx lane per pulse of the stage");
    constexpr int kNR = kNRef<SPK, STR>;
    constexpr int kSt = R_ST0<SPK>;
    __shared__ float4 refs[kStage * kNR / 4];
    // per (pulse of the sub-stage, interval): the coefficients of the tap
    // sum as polynomials in y = s^2, four float4 (see the table build)
    __shared__ float4 ctab[kSub * kNI * 4];

    // Workgroups go to the 8 XCDs round-robin by linear index; XCD x takes
    // the contiguous x-th eighth of the (cell-ordered) blocks, so blocks
    // reading the same range samples of g share that XCD's L2.  The launch
    // covers the plan's bound on the block count; the count itself is read
    // here, and workgroups beyond it return.
    const int nb = *A.n_blocks;
    const unsigned per = ((unsigned)nb + 7u) >> 3;
    if ((blockIdx.x >> 3) >= per) return;
    const long long b = (long long)(blockIdx.x & 7u) * per + (blockIdx.x >> 3);
    if (b >= nb) return;
    const BlockRec blk = A.blocks[b];
    const int lane = threadIdx.x;
    const bool have = lane < blk.count;
    const FacetRec f = A.facets[blk.start + (have ? lane : 0)];
    const double xb = (double)blk.xb, yb = (double)blk.yb;

    float gz_acc = 0.f, gvx = 0.f, gvy = 0.f, gvz = 0.f, gar = 0.f, gai = 0.f;
    float *rf = reinterpret_cast<float *>(refs);

    // speckle: the lane's facet id and Doppler, its anchors, the draw scale
    const SpkArgs &S = A.spk;
    const long long js = blk.start + (have ? lane : 0);
    [[maybe_unused]] SpkRec sr{};
    [[maybe_unused]] const float4 *an = nullptr;
    [[maybe_unused]] float l1 = 0.f;
    if constexpr (SPK) {
        sr = S.rec[js];
        an = S.anch + js * (long long)(S.n_groups + 1);
        l1 = S.c1 * S.c1 * 0.69314718055994531f;
    }

    for (int c = 0; c < A.C; ++c) {
        const ChanArgs chn = A.ch[c];
        const AntArgs &ta = A.ant[chn.tx], &ra = A.ant[chn.rx];
        FacetConsts kc;
        facet_consts(ta, ra, kc);
        const PulseRec *PR = A.pulses + (size_t)c * A.Np + A.p0;
        const float *gline = A.g + 2 * (size_t)c * A.np * (size_t)A.N;
        // speckle state: z holds the free path at the previous pulse; a call
        // starting inside a group first runs the group's path up to there
        [[maybe_unused]] float zr = 0.f, zi = 0.f, dxr = 0.f, dxi = 0.f;
        if constexpr (SPK) {
            const int k0 = A.p0 & 63, g0 = A.p0 >> 6;
            if (k0 != 0) {
                const float4 yd = an[g0];
                zr = yd.x;
                zi = yd.y;
                dxr = yd.z;
                dxi = yd.w;
                for (int k = 1; k < k0; ++k) {
                    const float2 e = spk_draw(S.key, sr.id, (uint32_t)(64 * g0 + k), l1);
                    zr = fmaf(S.b1, zr, e.x);
                    zi = fmaf(S.b1, zi, e.y);
                }
            }
        }
        for (int ps = 0; ps < A.np; ps += kStage) {
            __syncthreads();   // previous stage fully consumed
            // The stage's references, one pulse per lane of the first half:
            // the per-pulse records of the facet loop and grad T at the
            // centre (its Jacobian where the pattern factors are per facet).
            const auto write_refs = [&](const Refs &r, float ft, const float *gft, float fr,
                                        const float *gfr, double qr, const PulseRec &P,
                                        [[maybe_unused]] const double *prb,
                                        [[maybe_unused]] double cst, [[maybe_unused]] double snt,
                                        [[maybe_unused]] double csr, [[maybe_unused]] double snr) {
                float *o = rf + lane * kNR;
                // spreading at the centre (r.sb also carries the sinc normalisation)
                const float sbt = (r.mask != 0.0f || r.graze)
                                      ? (float)(chn.rtrr_mid * (double)r.irt * (double)r.irr)
                                      : 0.0f;
                const float gs[3] = {-sbt * (r.dtx * r.irt + (r.gx - r.dtx) * r.irr),
                                     -sbt * (r.dty * r.irt + (r.gy - r.dty) * r.irr),
                                     -sbt * (r.dtz * r.irt + (r.gz - r.dtz) * r.irr)};
                // grazing blocks keep grad T; each facet's own flag applies below
                const float m = (r.mask != 0.0f || r.graze) ? 1.0f : 0.0f;
                o[R_DTGX] = m * (fr * sbt * gft[0] + ft * sbt * gfr[0] + ft * fr * gs[0]);
                o[R_DTGY] = m * (fr * sbt * gft[1] + ft * sbt * gfr[1] + ft * fr * gs[1]);
                o[R_DTGZ] = m * (fr * sbt * gft[2] + ft * sbt * gfr[2] + ft * fr * gs[2]);
                if constexpr (!ELC) {
                    // Jacobian of grad T at the centre, central differences over
                    // +-0.5 m (one direction at a time to keep registers low)
                    constexpr double h = 0.5;
                    const float s2h = m * (float)(0.5 / h);
#pragma unroll 1
                    for (int j = 0; j < 3; ++j) {
                        const double ox = j == 0 ? h : 0.0, oy = j == 1 ? h : 0.0,
                                     oz = j == 2 ? h : 0.0;
                        float gp[3], gm[3];
                        grad_t<STR, GRD>(ta, ra, chn.rtrr_mid, xb + ox, yb + oy, oz, P.ptx, prb, gp,
                                    cst, snt, csr, snr);
                        grad_t<STR, GRD>(ta, ra, chn.rtrr_mid, xb - ox, yb - oy, -oz, P.ptx, prb, gm,
                                    cst, snt, csr, snr);
                        o[R_J0 + j] = s2h * (gp[0] - gm[0]);
                        o[R_J0 + 3 + j] = s2h * (gp[1] - gm[1]);
                        o[R_J0 + 6 + j] = s2h * (gp[2] - gm[2]);
                    }
                }
                o[R_T] = (float)P.t;
                o[R_LHI] = r.lhi;
                o[R_LLO] = r.llo;
                o[R_FSQ] = r.fsq;
                o[R_Q] = (float)qr;
                if constexpr (STR) {
                    o[kSt] = (float)cst;
                    o[kSt + 1] = (float)snt;
                    o[kSt + 2] = (float)csr;
                    o[kSt + 3] = (float)snr;
                }
                if constexpr (SPK) o[R_TLO] = (float)(P.t - (double)(float)P.t);
                o[R_DTX] = r.dtx; o[R_DTY] = r.dty; o[R_DTZ] = r.dtz;
                o[R_GX] = r.gx; o[R_GY] = r.gy; o[R_GZ] = r.gz;
                o[R_I2RT] = r.i2rt; o[R_I2RR] = r.i2rr; o[R_I2S] = r.i2s;
                o[R_PHIB] = r.phib; o[R_FB] = r.fb;
                o[R_NB] = __int_as_float(r.nb);
                o[R_GTAZ] = r.gtaz; o[R_GTEL] = r.gtel; o[R_GRAZ] = r.graz; o[R_GREL] = r.grel;
                o[R_IRT] = r.irt; o[R_IRT2] = r.irt2; o[R_IRR] = r.irr; o[R_IRR2] = r.irr2;
                o[R_SB] = r.sb; o[R_SBT] = r.sbt; o[R_SBR] = r.sbr; o[R_MASK] = r.mask;
                o[R_DBT] = r.dbt; o[R_DBR] = r.dbr;
                o[R_GRAZE] = __int_as_float(r.graze);
            
            };
            if constexpr (kSplit) {
                // Two lanes per pulse: lanes 0..31 take the Tx leg of pulse
                // lane, lanes 32..63 the Rx leg of pulse lane - 32 (the FP64
                // range, direction and pattern work of a leg), and the Rx
                // leg's results move to the first half, which combines them
                // in the same operations, in the same order, as block_refs.
                const int qp = lane & (kStage - 1);
                const bool rx = lane >= kStage;
                const int pl = ps + qp;
                const bool live = pl < A.np;
                const PulseRec &P = PR[live ? pl : A.np - 1];
                double prb[3] = {P.prx[0], P.prx[1], P.prx[2]};
                double qr = 1.0;
                if (A.rx_exact) rx_echo(xb, yb, P.ptx, P.prx, P.rref, chn.vr, A.inv_c, prb, qr);
                const AntArgs &an = rx ? ra : ta;
                const double *pp = rx ? prb : P.ptx;
                const double d0 = xb - pp[0], d1 = yb - pp[1], d2 = -pp[2];
                const double R = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                const double iR = 1.0 / R;
                const double u0 = d0 * iR, u1 = d1 * iR, u2 = d2 * iR;
                const double dA = d0 * an.az[0] + d1 * an.az[1] + d2 * an.az[2];
                const double dB = d0 * an.b[0] + d1 * an.b[1] + d2 * an.b[2];
                const double dE = d0 * an.el[0] + d1 * an.el[1] + d2 * an.el[2];
                const float gA = (float)(0.5 * an.ka * dA);
                const float gE = (float)(0.5 * an.ke * dE);
                const float y = (float)fabs(0.5 * an.ke * dE * iR) + 1e-9f;
                const float sy = __builtin_amdgcn_sinf(y);
                const double mB = dB * iR;
                float gf[3];
                const float F = ant_grad<false, 0>(an, d0, d1, d2, (double)(float)iR, gf, 1.0, 0.0);
                // the Rx leg's values to the Tx lane of the same pulse
                const double rr = __shfl_down(R, kStage), irr = __shfl_down(iR, kStage);
                const double ur0 = __shfl_down(u0, kStage), ur1 = __shfl_down(u1, kStage);
                const double ur2 = __shfl_down(u2, kStage), mr = __shfl_down(mB, kStage);
                const float dbr = __shfl_down((float)dB, kStage);
                const float graz = __shfl_down(gA, kStage), grel = __shfl_down(gE, kStage);
                const float yr = __shfl_down(y, kStage), syr = __shfl_down(sy, kStage);
                const float fr = __shfl_down(F, kStage);
                float gfr[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) gfr[k] = __shfl_down(gf[k], kStage);
                if (!rx) {
                    const double rt = R, irt = iR, mt = mB;
                    Refs r;
                    r.dtx = (float)u0;
                    r.dty = (float)u1;
                    r.dtz = (float)u2;
                    r.gx = (float)(u0 + ur0);
                    r.gy = (float)(u1 + ur1);
                    r.gz = (float)(u2 + ur2);
                    r.i2rt = (float)(0.5 * irt);
                    r.i2rr = (float)(0.5 * irr);
                    r.i2s = (float)(0.5 * (irt + irr));
                    const double rb = rt + rr;
                    const double cyc = rb * A.f0_c;
                    r.phib = (float)(rint(cyc) - cyc);
                    const double lq = qr * A.f0_c;
                    r.lhi = (float)lq;
                    r.llo = (float)(lq - (double)r.lhi);
                    r.fsq = (float)(qr * A.fs_c);
                    const double ub = A.n_ref + (rb - P.rref) * A.fs_c;
                    const double fl = floor(ub);
                    r.fb = (float)(ub - fl);
                    r.nb = (int)fl;
                    r.gtaz = gA;
                    r.graz = graz;
                    r.gtel = gE;
                    r.grel = grel;
                    r.irt = (float)irt;
                    r.irt2 = (float)(irt * irt);
                    r.irr = (float)irr;
                    r.irr2 = (float)(irr * irr);
                    const double sb = chn.rtrr_mid * irt * irr;
                    r.dbt = (float)dB;
                    r.dbr = dbr;
                    const double margin = 200.0 * (irt > irr ? irt : irr);
                    const bool front = mt > margin && mr > margin;
                    const bool behind = mt < -margin || mr < -margin;
                    r.graze = (live && !front && !behind) ? 1 : 0;
                    r.mask = (live && front) ? 1.0f : 0.0f;
                    const float fe = (sy * syr) * __builtin_amdgcn_rcpf((float)(kTwoPi * kTwoPi) * (y * yr));
                    const double sm = (r.mask != 0.0f || r.graze) ? kInvTwoPi2 * sb * (double)fe : 0.0;
                    r.sb = (float)sm;
                    r.sbt = (float)(sm * irt);
                    r.sbr = (float)(sm * irr);
                    write_refs(r, F, gf, fr, gfr, qr, P, prb, 1.0, 0.0, 1.0, 0.0);
                }
            } else if (lane < kStage) {
                const int pl = ps + lane;
                const bool live = pl < A.np;
                const PulseRec &P = PR[live ? pl : A.np - 1];
                // receiver at the block centre's own echo time (optional)
                double prb[3] = {P.prx[0], P.prx[1], P.prx[2]};
                double qr = 1.0;
                if (A.rx_exact) rx_echo(xb, yb, P.ptx, P.prx, P.rref, chn.vr, A.inv_c, prb, qr);
                [[maybe_unused]] double cst = 1.0, snt = 0.0, csr = 1.0, snr = 0.0;
                if constexpr (STR) {
                    cst = P.cst;
                    snt = P.snt;
                    csr = P.csr;
                    snr = P.snr;
                }
                Refs r;
                block_refs<kElc, STR, GRD != 0>(xb, yb, P.ptx, prb, P.rref, ta, ra, chn.rtrr_mid, A.f0_c,
                                A.fs_c, A.n_ref, live, r, qr, cst, snt, csr, snr);
                // grad T at the centre
                const double dt0 = xb - P.ptx[0], dt1 = yb - P.ptx[1], dt2 = -P.ptx[2];
                const double dr0 = xb - prb[0], dr1 = yb - prb[1], dr2 = -prb[2];
                float gft[3], gfr[3];
                const float ft = ant_grad<STR, GRD>(ta, dt0, dt1, dt2, (double)r.irt, gft, cst, snt);
                const float fr = ant_grad<STR, GRD>(ra, dr0, dr1, dr2, (double)r.irr, gfr, csr, snr);
                write_refs(r, ft, gft, fr, gfr, qr, P, prb, cst, snt, csr, snr);
            }
            __syncthreads();
            // The samples of g under lane (pulse qs + lane / 8, interval
            // w = lane % 8) of a sub-stage's table: nb - 7 + w .. nb + w of
            // that pulse, zero outside the line and past the call's pulses.
            // Loaded one sub-stage ahead (the first at the stage's start).
            const int nq = (A.np - ps) < kStage ? (A.np - ps) : kStage;
            const int w = lane & (kNI - 1);
            float2 gv[8];
            const auto load_g = [&](int qsub) {
                const int qq = qsub + (lane >> 3), pl = ps + qq;
                const int base = __float_as_int(rf[qq * kNR + R_NB]) - 7 + w;
                const float *gl = gline + 2 * (size_t)(pl < A.np ? pl : 0) * A.N;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int n = base + k;
                    gv[k] = (pl < A.np && n >= 0 && n < A.N)
                                ? make_float2(gl[2 * n], gl[2 * n + 1])
                                : make_float2(0.f, 0.f);
                }
            };
            load_g(0);
            for (int qs = 0; qs < nq; qs += kSub) {
                // Coefficient table of the sub-stage's 8 pulses, lane = (pulse,
                // interval w): with G+_j = g[w + 4 + j] + g[w + 3 - j] and
                // G-_j = g[w + 4 + j] - g[w + 3 - j] (the samples under taps
                // j + 4 and 3 - j), the tap sum over the taps' even and odd parts
                // is sum_j G+_j E_j(y) + s sum_j G-_j O_j(y), so its coefficients
                // in y are C_E[m] = sum_j G+_j e_j[m] and C_O[m] =
                // sum_j G-_j o_j[m].
                {
                    float er[4] = {0.f, 0.f, 0.f, 0.f}, ei[4] = {0.f, 0.f, 0.f, 0.f};
                    float orr[4] = {0.f, 0.f, 0.f, 0.f}, oi[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float2 a = gv[4 + j], b = gv[3 - j];
                        const float pr = a.x + b.x, pim = a.y + b.y;
                        const float mr = a.x - b.x, mim = a.y - b.y;
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            er[m] = fmaf(pr, A.tp.e[j][m], er[m]);
                            ei[m] = fmaf(pim, A.tp.e[j][m], ei[m]);
                            orr[m] = fmaf(mr, A.tp.o[j][m], orr[m]);
                            oi[m] = fmaf(mim, A.tp.o[j][m], oi[m]);
                        }
                    }
                    float4 *ct = ctab + lane * 4;
                    ct[0] = make_float4(er[0], ei[0], er[1], ei[1]);
                    ct[1] = make_float4(er[2], ei[2], er[3], ei[3]);
                    ct[2] = make_float4(orr[0], oi[0], orr[1], oi[1]);
                    ct[3] = make_float4(orr[2], oi[2], orr[3], oi[3]);
                }
                __syncthreads();
                if (qs + kSub < nq) load_g(qs + kSub);
                const int qe = (qs + kSub) < nq ? (qs + kSub) : nq;
                for (int q = qs; q < qe; ++q) {
                    const float *o = rf + q * kNR;
                    Refs r;
                    r.dtx = o[R_DTX]; r.dty = o[R_DTY]; r.dtz = o[R_DTZ];
                    r.gx = o[R_GX]; r.gy = o[R_GY]; r.gz = o[R_GZ];
                    r.i2rt = o[R_I2RT]; r.i2rr = o[R_I2RR]; r.i2s = o[R_I2S];
                    r.phib = o[R_PHIB]; r.fb = o[R_FB]; r.nb = __float_as_int(o[R_NB]);
                    r.gtaz = o[R_GTAZ]; r.gtel = o[R_GTEL]; r.graz = o[R_GRAZ]; r.grel = o[R_GREL];
                    r.irt = o[R_IRT]; r.irt2 = o[R_IRT2]; r.irr = o[R_IRR]; r.irr2 = o[R_IRR2];
                    r.sb = o[R_SB]; r.sbt = o[R_SBT]; r.sbr = o[R_SBR]; r.mask = o[R_MASK];
                    r.dbt = o[R_DBT]; r.dbr = o[R_DBR]; r.graze = __float_as_int(o[R_GRAZE]);
                    const float tf = o[R_T];
                    // speckle factor x(p) of this pulse and the Doppler phase (cycles)
                    float xr = 1.0f, xi = 0.0f, dop = 0.0f;
                    if constexpr (SPK) {
                        const int pabs = A.p0 + ps + q, k = pabs & 63;
                        if (k == 0) {
                            const float4 yd = an[pabs >> 6];
                            zr = yd.x;
                            zi = yd.y;
                            dxr = yd.z;
                            dxi = yd.w;
                        } else {
                            const float2 e = spk_draw(S.key, sr.id, (uint32_t)pabs, l1);
                            zr = fmaf(S.b1, zr, e.x);
                            zi = fmaf(S.b1, zi, e.y);
                        }
                        const float K = S.gain[k];
                        xr = fmaf(K, dxr, zr);
                        xi = fmaf(K, dxi, zi);
                        const float dh = sr.fs * tf;
                        const float dl = fmaf(sr.fs, o[R_TLO], fmaf(sr.fs, tf, -dh));
                        dop = __builtin_amdgcn_fractf(dh) + dl;
                    }
                    FacetConsts kq = kc;
                    [[maybe_unused]] float4 rot{1.f, 0.f, 1.f, 0.f};
                    if constexpr (STR) {
                        rot = float4{o[kSt], o[kSt + 1], o[kSt + 2], o[kSt + 3]};
                        steer_axes(ta, ra, rot.x, rot.y, rot.z, rot.w, kq);
                    }
                    Geo g;
                    facet_geo<kElc, SPK, STR, GRD>(r, kq, tf, f.dx, f.dy, f.z, f.vx, f.vy, f.vz,
                                             r.graze != 0, o[R_LHI], o[R_LLO], o[R_FSQ], dop, g, &ta,
                                             &ra, rot);
                    // g at samples floor(u) - 3 .. floor(u) + 4
                    const int w0 = g.fl + 4;            // window index of the first tap
                    float br = 0.f, bi = 0.f, dr = 0.f, di = 0.f;
                    if ((unsigned)w0 < (unsigned)kNI) {
                        // the tap sum B = P_E(y) + s P_O(y) from the table, and
                        // its u-derivative dB/du = 2 dB/ds = 4 s P_E' + 2 P_O +
                        // 4 y P_O' (Horner's rule carrying P and P' together)
                        const float4 *ct = ctab + ((q - qs) * kNI + w0) * 4;
                        const float4 e01 = ct[0], e23 = ct[1], o01 = ct[2], o23 = ct[3];
                        const float sg = fmaf(g.f, 2.0f, -1.0f), y = sg * sg;
                        float per = fmaf(e23.z, y, e23.x), pei = fmaf(e23.w, y, e23.y);
                        float der = fmaf(e23.z, y, per), dei = fmaf(e23.w, y, pei);
                        per = fmaf(per, y, e01.z);
                        pei = fmaf(pei, y, e01.w);
                        der = fmaf(der, y, per);
                        dei = fmaf(dei, y, pei);
                        per = fmaf(per, y, e01.x);
                        pei = fmaf(pei, y, e01.y);
                        float por = fmaf(o23.z, y, o23.x), poi = fmaf(o23.w, y, o23.y);
                        float dor = fmaf(o23.z, y, por), doi = fmaf(o23.w, y, poi);
                        por = fmaf(por, y, o01.z);
                        poi = fmaf(poi, y, o01.w);
                        dor = fmaf(dor, y, por);
                        doi = fmaf(doi, y, poi);
                        por = fmaf(por, y, o01.x);
                        poi = fmaf(poi, y, o01.y);
                        br = fmaf(sg, por, per);
                        bi = fmaf(sg, poi, pei);
                        dr = 2.0f * fmaf(2.0f, fmaf(sg, der, y * dor), por);
                        di = 2.0f * fmaf(2.0f, fmaf(sg, dei, y * doi), poi);
                    } else {
                        TapV tv;
                        tap_all(A.tp, tv);
                        float tap[8], dtap[8];
                        taps_d8(tv, g.f, tap, dtap);
                        const float *gl = gline + 2 * (size_t)(ps + q) * A.N;
#pragma unroll
                        for (int k = 0; k < 8; ++k) {
                            const int n = r.nb + g.fl - 3 + k;
                            if (n >= 0 && n < A.N) {
                                const float vx = gl[2 * n], vy = gl[2 * n + 1];
                                br = fmaf(vx, tap[k], br);
                                bi = fmaf(vy, tap[k], bi);
                                dr = fmaf(vx, dtap[k], dr);
                                di = fmaf(vy, dtap[k], di);
                            }
                        }
                    }
                    bi = -bi;     // B = sum conj(g) h
                    di = -di;     // B_u = sum conj(g) dh/du
                    const float T = g.amp;
                    // a x E (x = 1 without speckle)
                    const float axr = SPK ? fmaf(f.ar, xr, -(f.ai * xi)) : f.ar;
                    const float axi = SPK ? fmaf(f.ar, xi, f.ai * xr) : f.ai;
                    const float aer = fmaf(axr, g.cs, -(axi * g.sn));
                    const float aei = fmaf(axr, g.sn, axi * g.cs);
                    // P = B a E
                    const float pr = fmaf(br, aer, -(bi * aei));
                    const float pi = fmaf(br, aei, bi * aer);
                    // Re(B_u a E) T
                    const float bu = fmaf(dr, aer, -(di * aei)) * T;
                    // grad R carries q with the facet's own echo time
                    const float cR = fmaf(pi * T, A.k0, bu * A.fs_cf) * o[R_Q];
                    // grad R = g (1 - c2) + e (1/R_t + 1/R_r) - d_t (c1 - c2),
                    // c1 = (e.d_t)/R_t, c2 = (e.d_r)/R_r, d_r = g - d_t
                    const float c1 = g.at * r.irt, c2 = g.ar * r.irr;
                    const float s1 = r.irt + r.irr, u1 = 1.0f - c2, w1 = c1 - c2;
                    const float grx = fmaf(g.ex, s1, fmaf(r.gx, u1, -(r.dtx * w1)));
                    const float gry = fmaf(g.ey, s1, fmaf(r.gy, u1, -(r.dty * w1)));
                    const float grz = fmaf(g.ez, s1, fmaf(r.gz, u1, -(r.dtz * w1)));
                    const float pm = pr * g.mf;
                    float tgx = o[R_DTGX], tgy = o[R_DTGY], tgz = o[R_DTGZ];
                    if constexpr (!ELC) {
                        // grad T at the facet, first order in its offset
                        tgx = fmaf(o[R_J0 + 0], g.ex, fmaf(o[R_J0 + 1], g.ey, fmaf(o[R_J0 + 2], g.ez, tgx)));
                        tgy = fmaf(o[R_J0 + 3], g.ex, fmaf(o[R_J0 + 4], g.ey, fmaf(o[R_J0 + 5], g.ez, tgy)));
                        tgz = fmaf(o[R_J0 + 6], g.ex, fmaf(o[R_J0 + 7], g.ey, fmaf(o[R_J0 + 8], g.ez, tgz)));
                    }
                    const float gxv = fmaf(pm, tgx, cR * grx);
                    const float gyv = fmaf(pm, tgy, cR * gry);
                    const float gzv = fmaf(pm, tgz, cR * grz);
                    gz_acc += gzv;
                    gvx = fmaf(tf, gxv, gvx);
                    gvy = fmaf(tf, gyv, gvy);
                    gvz = fmaf(tf, gzv, gvz);
                    // dL/da = conj(B T E x)
                    const float zbr = fmaf(br, g.cs, -(bi * g.sn)), zbi = fmaf(br, g.sn, bi * g.cs);
                    if constexpr (SPK) {
                        gar = fmaf(T, fmaf(zbr, xr, -(zbi * xi)), gar);
                        gai = fmaf(-T, fmaf(zbr, xi, zbi * xr), gai);
                    } else {
                        gar = fmaf(T, zbr, gar);
                        gai = fmaf(-T, zbi, gai);
                    }
                }
                __syncthreads();   // the sub-stage's table fully read
            }
        }
    }

    if (have) {
        const int i = A.perm[blk.start + lane];
        if (A.accumulate) {
            if (A.dz) A.dz[i] += gz_acc;
            if (A.dvx) A.dvx[i] += gvx;
            if (A.dvy) A.dvy[i] += gvy;
            if (A.dvz) A.dvz[i] += gvz;
            if (A.dar) A.dar[i] += gar;
            if (A.dai) A.dai[i] += gai;
        } else {
            if (A.dz) A.dz[i] = gz_acc;
            if (A.dvx) A.dvx[i] = gvx;
            if (A.dvy) A.dvy[i] = gvy;
            if (A.dvz) A.dvz[i] = gvz;
            if (A.dar) A.dar[i] = gar;
            if (A.dai) A.dai[i] = gai;
        }
    }
}

}  // namespace

hipError_t launch_adjoint(const AdjArgs &a, bool el_const, bool speckle, hipStream_t s) {
    if (a.nb_max == 0 || a.np == 0) return hipSuccess;
    const unsigned long long wgs = ((unsigned long long)a.nb_max + 7) / 8 * 8;
    if (wgs > 0xffffffffULL) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)wgs);
#define HS_ADJ(E, S, T) hipLaunchKernelGGL((k_adjoint<E, S, T, 0>), grid, dim3(64), 0, s, a)
#define HS_ADJG(E, S, T)                                                                   \
    do {                                                                                   \
        if (a.grid == 2) hipLaunchKernelGGL((k_adjoint<E, S, T, 2>), grid, dim3(64), 0, s, a); \
        else hipLaunchKernelGGL((k_adjoint<E, S, T, 1>), grid, dim3(64), 0, s, a);        \
    } while (0)
    if (a.grid) {   // gridded patterns: per facet; el_const drops the Jacobian
        if (a.steer) {
            if (speckle) {
                if (el_const) HS_ADJG(true, true, true);
                else HS_ADJG(false, true, true);
            } else {
                if (el_const) HS_ADJG(true, false, true);
                else HS_ADJG(false, false, true);
            }
        } else {
            if (speckle) {
                if (el_const) HS_ADJG(true, true, false);
                else HS_ADJG(false, true, false);
            } else {
                if (el_const) HS_ADJG(true, false, false);
                else HS_ADJG(false, false, false);
            }
        }
    } else if (a.steer) {
        if (speckle) {
            if (el_const) HS_ADJ(true, true, true);
            else HS_ADJ(false, true, true);
        } else {
            if (el_const) HS_ADJ(true, false, true);
            else HS_ADJ(false, false, true);
        }
    } else {
        if (speckle) {
            if (el_const) HS_ADJ(true, true, false);
            else HS_ADJ(false, true, false);
        } else {
            if (el_const) HS_ADJ(true, false, false);
            else HS_ADJ(false, false, false);
        }
    }
#undef HS_ADJ
#undef HS_ADJG
    return hipGetLastError();
}

}  // namespace hs
