// Device-side building blocks shared by the forward and adjoint kernels:
// FP64 per-(block, pulse) references and the FP32 per-facet geometry.
//
// Precision scheme.  The carrier wavelength (5.5 cm) sits against ~1.7e6 m
// of bistatic path, so a facet's range cannot be formed in FP32.  Per
// (block, pulse) the block centre's leg ranges R_b, unit vectors d, phase in
// cycles (integer part removed) and sample position (integer + fraction) are
// computed in FP64.  Per facet only its offset e from the block centre
// (|e| of a few metres: the block half-diagonal, the height and the drift
// V t_p) enters FP32, through the expansion of each leg
//   R - R_b = e.d + (|e|^2 - (e.d)^2) / (2 R_b) + O(|e|^3 / R_b^2),
// whose neglected term is below 1e-8 m for |e| < 30 m.  The phase product
// dR * f0/c uses a two-float split of f0/c and an FMA residual, so the
// integer number of cycles is removed without rounding the large product.
#pragma once

#include "sim_internal.h"

namespace hs {

constexpr float kPiF = 3.14159265358979323846f;
constexpr double kTwoPi = 6.283185307179586476925;
constexpr double kTwoPi4 = kTwoPi * kTwoPi * kTwoPi * kTwoPi;   // (2 pi)^4
constexpr double kInvTwoPi4 = 1.0 / kTwoPi4;
constexpr double kInvTwoPi2 = 1.0 / (kTwoPi * kTwoPi);

// sinc(x) = sin(pi x) / (pi x).  The hardware sine takes revolutions, so
// sin(pi x) = v_sin(x / 2), valid while |x| / 2 <= 256; sim_create keeps
// kappa / beta <= 500 (direction cosines are at most 1).
__device__ __forceinline__ float sinc_f(float x) {
    const float s = __builtin_amdgcn_sinf(0.5f * x);
    const float r = s * __builtin_amdgcn_rcpf(kPiF * x);
    return (fabsf(x) < 1e-6f) ? 1.0f : r;
}

// derivative of sinc: (cos(pi x) - sinc(x)) / x
__device__ __forceinline__ float dsinc_f(float x) {
    const float c = __builtin_amdgcn_cosf(0.5f * x);
    const float r = (c - sinc_f(x)) * __builtin_amdgcn_rcpf(x);
    return (fabsf(x) < 1e-6f) ? 0.0f : r;
}

// One antenna's field for the GRD kernels, in two steps so that the table
// load is in flight while the phase is computed.  fetch: from the projections
// pu, pv of the facet direction (times R) on the antenna's scaled azimuth and
// elevation axes and the first-order 1/R, an antenna with a u-v table gets
// its cell coordinates ((u - u0)/du, (v - v0)/dv; axes scaled to cell units)
// and issues the one 16-byte load of the cell's four corners (cell 0 when
// outside the half-open range [0, nu-1) x [0, nv-1), NaN included); an
// antenna without a table keeps the sinc arguments (axes scaled by
// kappa/(2 beta)).  finish: the bilinear value (0 outside), or the sinc
// product normalised here since GRD spreading terms carry no (2 pi)^k.  The
// branch on the table pointer is uniform (the workgroup's channel's
// antenna); ALL (every antenna of the handle has a table) removes it.
struct GridFetch {
    float4 c;       // cell corners (i,j), (i+1,j), (i,j+1), (i+1,j+1)
    float x, y;     // cell coordinates, or the two sinc arguments
    bool in;
};

template <bool ALL>
__device__ __forceinline__ GridFetch ant_fetch(const AntArgs &a, float pu, float pv, float irf) {
    GridFetch g;
    if (ALL || a.grid) {
        g.x = fmaf(pu, irf, -a.gu0);
        g.y = fmaf(pv, irf, -a.gv0);
        // bitwise tests: no short-circuit branches in the facet loop
        g.in = (g.x >= 0.0f) & (g.x < a.gnu1) & (g.y >= 0.0f) & (g.y < a.gnv1);
        const int idx = g.in ? (int)floorf(g.y) * a.gstride + (int)floorf(g.x) : 0;
        g.c = a.grid[idx];
    } else {
        g.x = fmaf(fabsf(pu), irf, 1e-9f);
        g.y = fmaf(fabsf(pv), irf, 1e-9f);
        g.in = true;
        g.c = float4{0.f, 0.f, 0.f, 0.f};
    }
    return g;
}

template <bool ALL>
__device__ __forceinline__ float ant_finish(const AntArgs &a, const GridFetch &g) {
    if (ALL || a.grid) {
        const float ax = g.x - floorf(g.x), ay = g.y - floorf(g.y);
        const float lo = fmaf(ax, g.c.y - g.c.x, g.c.x);
        const float hi = fmaf(ax, g.c.w - g.c.z, g.c.z);
        return g.in ? fmaf(ay, hi - lo, lo) : 0.0f;
    }
    return (__builtin_amdgcn_sinf(g.x) * __builtin_amdgcn_sinf(g.y)) *
           __builtin_amdgcn_rcpf((float)(kTwoPi * kTwoPi) * (g.x * g.y));
}

// Per-(block, pulse) references of one lane (FP64 -> FP32).
struct Refs {
    float dtx, dty, dtz;            // unit vector Tx -> block centre
    float gx, gy, gz;               // gradient of the bistatic range at the centre
    float i2rt, i2rr;               // 1 / (2 R_b) per leg
    float i2s;                      // i2rt + i2rr
    float phib;                     // -frac(R_b f0 / c): phase of the centre (cycles)
    float fb;                       // fractional part of the centre's sample
    int nb;                         // integer part of the centre's sample
    float gtaz, gtel, graz, grel;   // (kappa/beta)/2 (D . axis) per antenna axis
                                    // (D . axis / du or dv for a gridded antenna)
    float irt, irt2, irr, irr2;     // 1/R_b and 1/R_b^2 per leg
    float sb, sbt, sbr;             // spreading at the centre (and over R per leg),
                                    // times the mask, divided by (2 pi)^4 (not
                                    // with gridded patterns)
    float mask;                     // 1 if the lane's pulse is live and in front
    float dbt, dbr;                 // D . b per leg (grazing blocks only)
    int graze;                      // block straddles an antenna's back plane
    float lhi, llo;                 // q f0/c split in two floats (phase of dR)
    float fsq;                      // q fs/c (sample shift of dR)
};

// Receiver at the echo time of the block centre x_b (eq. 3 takes r_r at the
// reception time): fixed point of c tau = |x_b - P_tx| + |x_b - P_rx(t_p + tau)|
// started from the origin's echo (prx = P_rx(t_p + tau_ref), rref = c
// tau_ref), P_rx moving at vr.  Each step gains a factor ~|vr|/c ~ 3e-5, so
// three leave ~1e-13 m.  A facet at offset e from x_b has its own echo time;
// to first order its range offset is q times the one computed with the
// centre's receiver position, q = 1 / (1 + u_r . vr / c) (u_r: receiver ->
// centre), the neglected terms ~(e/R)(|vr|/c) e < 1e-9 m.
__device__ __forceinline__ void rx_echo(double xb, double yb, const double *ptx,
                                        const double *prx, double rref, const double *vr,
                                        double inv_c, double *pr, double &q) {
    const double a0 = xb - ptx[0], a1 = yb - ptx[1], a2 = -ptx[2];
    const double rt = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
    double dtau = 0.0;
#pragma unroll
    for (int it = 0; it < 3; ++it) {
        const double d0 = xb - (prx[0] + vr[0] * dtau), d1 = yb - (prx[1] + vr[1] * dtau);
        const double d2 = -(prx[2] + vr[2] * dtau);
        dtau = (rt + sqrt(d0 * d0 + d1 * d1 + d2 * d2) - rref) * inv_c;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) pr[k] = prx[k] + vr[k] * dtau;
    const double d0 = xb - pr[0], d1 = yb - pr[1], d2 = -pr[2];
    const double ir = 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    q = 1.0 / (1.0 + (d0 * vr[0] + d1 * vr[1] + d2 * vr[2]) * ir * inv_c);
}

// ELC: the elevation pattern factors of both legs are taken at the block
// centre and folded into the spreading terms (chosen on the host only where
// a bound puts the relative error of that below 1e-6 for every facet).
// GRD: gridded patterns (never with ELC); the spreading terms then carry no
// sinc normalisation and the azimuth/elevation references are in cell units.
template <bool ELC, bool STR = false, bool GRD = false>
__device__ __forceinline__ void block_refs(double xb, double yb, const double *ptx,
                                           const double *prx, double rref, const AntArgs &t,
                                           const AntArgs &q, double rtrr_mid, double f0_c,
                                           double fs_c, double n_ref, bool live, Refs &r,
                                           double qr = 1.0, double cst = 1.0, double snt = 0.0,
                                           double csr = 1.0, double snr = 0.0) {
    const double dt0 = xb - ptx[0], dt1 = yb - ptx[1], dt2 = -ptx[2];
    const double dr0 = xb - prx[0], dr1 = yb - prx[1], dr2 = -prx[2];
    const double rt = sqrt(dt0 * dt0 + dt1 * dt1 + dt2 * dt2);
    const double rr = sqrt(dr0 * dr0 + dr1 * dr1 + dr2 * dr2);
    const double irt = 1.0 / rt, irr = 1.0 / rr;
    const double ut0 = dt0 * irt, ut1 = dt1 * irt, ut2 = dt2 * irt;
    const double ur0 = dr0 * irr, ur1 = dr1 * irr, ur2 = dr2 * irr;
    r.dtx = (float)ut0;
    r.dty = (float)ut1;
    r.dtz = (float)ut2;
    r.gx = (float)(ut0 + ur0);
    r.gy = (float)(ut1 + ur1);
    r.gz = (float)(ut2 + ur2);
    r.i2rt = (float)(0.5 * irt);
    r.i2rr = (float)(0.5 * irr);
    r.i2s = (float)(0.5 * (irt + irr));
    const double rb = rt + rr;
    const double cyc = rb * f0_c;
    r.phib = (float)(rint(cyc) - cyc);
    const double lq = qr * f0_c;
    r.lhi = (float)lq;
    r.llo = (float)(lq - (double)r.lhi);
    r.fsq = (float)(qr * fs_c);
    const double ub = n_ref + (rb - rref) * fs_c;
    const double fl = floor(ub);
    r.fb = (float)(ub - fl);
    r.nb = (int)fl;
    // azimuth axes and boresights turned by the steering angles (cos, sin):
    // az' = az cos - b sin, b' = b cos + az sin (elevation axes unchanged)
    const double dta = dt0 * t.az[0] + dt1 * t.az[1] + dt2 * t.az[2];
    const double dtb = dt0 * t.b[0] + dt1 * t.b[1] + dt2 * t.b[2];
    const double dra = dr0 * q.az[0] + dr1 * q.az[1] + dr2 * q.az[2];
    const double drb = dr0 * q.b[0] + dr1 * q.b[1] + dr2 * q.b[2];
    if constexpr (STR) {
        r.gtaz = (float)(0.5 * t.ka * (dta * cst - dtb * snt));
        r.graz = (float)(0.5 * q.ka * (dra * csr - drb * snr));
    } else {
        r.gtaz = (float)(0.5 * t.ka * dta);
        r.graz = (float)(0.5 * q.ka * dra);
    }
    r.gtel = (float)(0.5 * t.ke * (dt0 * t.el[0] + dt1 * t.el[1] + dt2 * t.el[2]));
    r.grel = (float)(0.5 * q.ke * (dr0 * q.el[0] + dr1 * q.el[1] + dr2 * q.el[2]));
    r.irt = (float)irt;
    r.irt2 = (float)(irt * irt);
    r.irr = (float)irr;
    r.irr2 = (float)(irr * irr);
    const double sb = rtrr_mid * irt * irr;
    const double dbt = STR ? dtb * cst + dta * snt : dtb;
    const double dbr = STR ? drb * csr + dra * snr : drb;
    r.dbt = (float)dbt;
    r.dbr = (float)dbr;
    // Facets lie within ~100 m of the centre, so their direction cosines with a
    // boresight differ from the centre's by < 100 / R; a margin of 200 / R
    // decides whole blocks, the rest is checked facet by facet.
    const double mt = dbt * irt, mr = dbr * irr;
    const double margin = 200.0 * (irt > irr ? irt : irr);
    const bool front = mt > margin && mr > margin;
    const bool behind = mt < -margin || mr < -margin;
    r.graze = (live && !front && !behind) ? 1 : 0;
    r.mask = (live && front) ? 1.0f : 0.0f;
    // the spreading terms carry the mask (grazing lanes are masked per facet)
    // and the 1/(2 pi)^k of the merged sinc product (k = number of factors
    // evaluated per facet), with the elevation factors at the centre in ELC
    double sm = (r.mask != 0.0f || r.graze) ? (GRD ? 1.0 : kInvTwoPi4) * sb : 0.0;
    if constexpr (ELC) {
        const float yt = (float)fabs(0.5 * t.ke * (dt0 * t.el[0] + dt1 * t.el[1] + dt2 * t.el[2]) * irt) + 1e-9f;
        const float yr = (float)fabs(0.5 * q.ke * (dr0 * q.el[0] + dr1 * q.el[1] + dr2 * q.el[2]) * irr) + 1e-9f;
        const float fe = (__builtin_amdgcn_sinf(yt) * __builtin_amdgcn_sinf(yr)) *
                         __builtin_amdgcn_rcpf((float)(kTwoPi * kTwoPi) * (yt * yr));
        sm = (r.mask != 0.0f || r.graze) ? kInvTwoPi2 * sb * (double)fe : 0.0;
    }
    r.sb = (float)sm;
    r.sbt = (float)(sm * irt);
    r.sbr = (float)(sm * irr);
}

// FP32 antenna constants of one channel for the per-facet part.
struct FacetConsts {
    float kta[3], kte[3], kra[3], kre[3];   // (kappa/beta) * axis, Tx and Rx
    float bt[3], br[3];                     // boresights
};

__device__ __forceinline__ void facet_consts(const AntArgs &t, const AntArgs &q,
                                             FacetConsts &k) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        k.kta[i] = t.kaz[i];
        k.kte[i] = t.kel[i];
        k.kra[i] = q.kaz[i];
        k.kre[i] = q.kel[i];
        k.bt[i] = t.b32[i];
        k.br[i] = q.b32[i];
    }
}

// Facet constants for antennas turned by steering angles (cos, sin per leg):
// the azimuth axes az cos - b sin (scaled); the boresights b cos + az sin are
// turned where they are used (facet_geo's back-plane test).
__device__ __forceinline__ void steer_axes(const AntArgs &t, const AntArgs &q, float ct,
                                           float st, float cr, float sr, FacetConsts &k) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        k.kta[i] = fmaf(t.kaz[i], ct, -(t.kb[i] * st));
        k.kra[i] = fmaf(q.kaz[i], cr, -(q.kb[i] * sr));
    }
}

// Per-facet geometry of one (facet, pulse) pair.
struct Geo {
    float mf;            // 1, or 0 for a facet behind an antenna in a straddling block
    float ex, ey, ez;    // offset from the block centre at the pulse time
    float at, ar;        // its projections on the Tx and Rx unit vectors
    float dR;        // bistatic range minus the block centre's
    float sn, cs;    // sin, cos of the carrier phase (2 pi cycles)
    float amp;       // F_tx F_rx S (times the mask)
    float f;         // fractional sample position
    int fl;          // floor(fb + dR fs/c): sample offset from the centre's
};

// ROT: the boresights of cc are the fixed-frame ones and the back-plane test
// (grazing blocks only) turns them by rot = (cos, sin) of the Tx and Rx
// steering angles, with the antennas' FP32 axes (t, q).
// GRD: field patterns from the antennas' u-v grids (t, q), with the direction
// cosines in cell units (per-facet, first order in the offset like the sinc
// arguments); 1: antennas without a table keep the sinc, 2: every antenna
// has a table.
template <bool ELC, bool DOP = false, bool ROT = false, int GRD = 0>
__device__ __forceinline__ void facet_geo(const Refs &r, const FacetConsts &cc, float tf,
                                          float fdx, float fdy, float fz, float fvx, float fvy,
                                          float fvz, bool graze_any, float linv_hi,
                                          float linv_lo, float fs_c, float dop, Geo &o,
                                          const AntArgs *t = nullptr, const AntArgs *q = nullptr,
                                          float4 rot = float4{1.f, 0.f, 1.f, 0.f}) {
    const float ex = fmaf(fvx, tf, fdx);
    const float ey = fmaf(fvy, tf, fdy);
    const float ez = fmaf(fvz, tf, fz);
    const float ee = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
    const float L = fmaf(ez, r.gz, fmaf(ey, r.gy, ex * r.gx));
    const float at = fmaf(ez, r.dtz, fmaf(ey, r.dty, ex * r.dtx));
    const float ar = L - at;
    // second-order terms (|e|^2 - at^2) / (2 R_t) + (|e|^2 - ar^2) / (2 R_r),
    // summed before they meet L
    const float s1 = at * r.i2rt, s2 = ar * r.i2rr;
    const float h2 = fmaf(at, s1, ar * s2);
    const float dR = L + fmaf(ee, r.i2s, -h2);
    [[maybe_unused]] GridFetch gt, gr;
    if constexpr (GRD != 0) {
        static_assert(!ELC, "gridded patterns are evaluated per facet");
        // table cells requested before the phase, used after it
        const float it = fmaf(-at, r.irt2, r.irt), ir = fmaf(-ar, r.irr2, r.irr);
        gt = ant_fetch<GRD == 2>(*t, fmaf(ez, cc.kta[2], fmaf(ey, cc.kta[1], fmaf(ex, cc.kta[0], r.gtaz))),
                       fmaf(ez, cc.kte[2], fmaf(ey, cc.kte[1], fmaf(ex, cc.kte[0], r.gtel))), it);
        gr = ant_fetch<GRD == 2>(*q, fmaf(ez, cc.kra[2], fmaf(ey, cc.kra[1], fmaf(ex, cc.kra[0], r.graz))),
                       fmaf(ez, cc.kre[2], fmaf(ey, cc.kre[1], fmaf(ex, cc.kre[0], r.grel))), ir);
    }
    // phase (cycles) = phib - dR f0/c (+ dop, the intra-facet Doppler of a
    // speckle sum, if DOP), product split so the integer part of the cycle
    // count is removed exactly
    const float hi = dR * linv_hi;
    float lo = fmaf(dR, linv_hi, -hi);
    lo = fmaf(dR, linv_lo, lo);
    float ph = (r.phib - __builtin_amdgcn_fractf(hi)) - lo;
    if constexpr (DOP) ph += dop;
    o.sn = __builtin_amdgcn_sinf(ph);
    o.cs = __builtin_amdgcn_cosf(ph);
    // Antenna field patterns.  With y = kappa u / (2 beta) for each of the four
    // direction cosines (Tx az, el; Rx az, el), sinc(2y) = v_sin(y) / (2 pi y),
    // so F_tx F_rx = prod v_sin(y_k) / ((2 pi)^4 prod y_k): one reciprocal for
    // the four factors, the (2 pi)^4 folded into the spreading terms.  sinc is
    // even, so |y| is used, floored at 1e-9 (sinc(2e-9) = 1 - 7e-18) to keep the
    // product normal and never zero.  1/R per leg to first order in the offset.
    const float irtf = fmaf(-at, r.irt2, r.irt);
    const float irrf = fmaf(-ar, r.irr2, r.irr);
    // spreading R_mid^2 / (R_t R_r), first order in the offsets
    const float s = fmaf(-ar, r.sbr, fmaf(-at, r.sbt, r.sb));
    float amp;
    if constexpr (GRD != 0) {
        amp = (ant_finish<GRD == 2>(*t, gt) * ant_finish<GRD == 2>(*q, gr)) * s;
    } else {
        const float yta = fmaf(fabsf(fmaf(ez, cc.kta[2], fmaf(ey, cc.kta[1], fmaf(ex, cc.kta[0], r.gtaz)))), irtf, 1e-9f);
        const float yra = fmaf(fabsf(fmaf(ez, cc.kra[2], fmaf(ey, cc.kra[1], fmaf(ex, cc.kra[0], r.graz)))), irrf, 1e-9f);
        float sp, yp;
        if constexpr (ELC) {
            sp = __builtin_amdgcn_sinf(yta) * __builtin_amdgcn_sinf(yra);
            yp = yta * yra;
        } else {
            const float yte = fmaf(fabsf(fmaf(ez, cc.kte[2], fmaf(ey, cc.kte[1], fmaf(ex, cc.kte[0], r.gtel)))), irtf, 1e-9f);
            const float yre = fmaf(fabsf(fmaf(ez, cc.kre[2], fmaf(ey, cc.kre[1], fmaf(ex, cc.kre[0], r.grel)))), irrf, 1e-9f);
            sp = (__builtin_amdgcn_sinf(yta) * __builtin_amdgcn_sinf(yte)) *
                 (__builtin_amdgcn_sinf(yra) * __builtin_amdgcn_sinf(yre));
            yp = (yta * yte) * (yra * yre);
        }
        amp = sp * __builtin_amdgcn_rcpf(yp) * s;
    }
    o.mf = 1.0f;
    if (graze_any && r.graze) {
        float bt[3] = {cc.bt[0], cc.bt[1], cc.bt[2]}, br[3] = {cc.br[0], cc.br[1], cc.br[2]};
        if constexpr (ROT) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                bt[i] = fmaf(t->b32[i], rot.x, t->az32[i] * rot.y);
                br[i] = fmaf(q->b32[i], rot.z, q->az32[i] * rot.w);
            }
        }
        const float ct = fmaf(ez, bt[2], fmaf(ey, bt[1], fmaf(ex, bt[0], r.dbt)));
        const float cr = fmaf(ez, br[2], fmaf(ey, br[1], fmaf(ex, br[0], r.dbr)));
        if (!(ct > 0.0f && cr > 0.0f)) {
            amp = 0.0f;
            o.mf = 0.0f;
        }
    }
    o.amp = amp;
    const float uu = fmaf(dR, fs_c, r.fb);
    o.f = __builtin_amdgcn_fractf(uu);
    int fl;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(fl) : "v"(uu));   // floor and convert
    o.fl = fl;
    o.dR = dR;
    o.ex = ex;
    o.ey = ey;
    o.ez = ez;
    o.at = at;
    o.ar = ar;
}

// A uniform value copied into a VGPR (a VALU instruction reads at most one
// SGPR operand on gfx9, so coefficients kept in VGPRs cost no extra moves).
__device__ __forceinline__ float to_vgpr(float x) {
    float r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
    return r;
}

// All tap coefficients held in VGPRs (uniform values).  Frees 32 SGPRs in
// kernels whose scalar registers would otherwise spill, and keeps the tap
// FMAs free of SGPR operands.
struct TapV {
    float e[4][4], o[4][4];
};

__device__ __forceinline__ void tap_all(const TapPoly &tp, TapV &t) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            t.e[j][m] = to_vgpr(tp.e[j][m]);
            t.o[j][m] = to_vgpr(tp.o[j][m]);
        }
}

// The 8 taps at samples floor(u) - 3 .. floor(u) + 4 for fractional part f.
__device__ __forceinline__ void taps8(const TapV &tv, float f, float *tap) {
    const float sg = fmaf(f, 2.0f, -1.0f);
    const float y = sg * sg;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float e = fmaf(fmaf(fmaf(tv.e[j][3], y, tv.e[j][2]), y, tv.e[j][1]), y, tv.e[j][0]);
        const float od =
            sg * fmaf(fmaf(fmaf(tv.o[j][3], y, tv.o[j][2]), y, tv.o[j][1]), y, tv.o[j][0]);
        tap[4 + j] = e + od;
        tap[3 - j] = e - od;
    }
}

// The 8 taps and their derivatives with respect to u, from the same
// coefficients: Horner's rule carries each polynomial and its derivative in y
// together.  With Q_j = E(y) + s O(y), y = s^2, s = 2f - 1 and du = df:
//   dQ_j/du      = 2 (O + 2 y O') + s 4 E'
//   dQ_j(-s)/du  = s 4 E' - 2 (O + 2 y O')
__device__ __forceinline__ void taps_d8(const TapV &tv, float f, float *tap,
                                        float *d) {
    const float sg = fmaf(f, 2.0f, -1.0f);
    const float y = sg * sg;
    const float y2 = y + y, s4 = 4.0f * sg;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float e = fmaf(tv.e[j][3], y, tv.e[j][2]), de = tv.e[j][3];
        de = fmaf(de, y, e);
        e = fmaf(e, y, tv.e[j][1]);
        de = fmaf(de, y, e);
        e = fmaf(e, y, tv.e[j][0]);
        float o = fmaf(tv.o[j][3], y, tv.o[j][2]), dq = tv.o[j][3];
        dq = fmaf(dq, y, o);
        o = fmaf(o, y, tv.o[j][1]);
        dq = fmaf(dq, y, o);
        o = fmaf(o, y, tv.o[j][0]);
        const float so = sg * o;
        tap[4 + j] = e + so;
        tap[3 - j] = e - so;
        const float a = 2.0f * fmaf(y2, dq, o);
        const float b = s4 * de;
        d[4 + j] = a + b;
        d[3 - j] = b - a;
    }
}

}  // namespace hs
