/*
 * FP64 oracle for the HEEPS/MARE facet-sum path (Monnier et al., "Synthetic
 * RAW data generator for ESA HARMONY mission").
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  The product (the HIP
 * library and its Python binding) never links, imports or calls it, and this
 * file shares no code, header, table or constant generator with it.
 *
 * Everything is the plain definition, evaluated directly in double precision
 * with libm: no spatial blocks, no Taylor forms, no reordering.  Where the
 * paper is silent the reading used is stated next to the code.
 *
 * Parity status of each function (see the tests under tests/test_oracle_*):
 *   og_pulse_time, og_pulse_geometry   pinned (closed forms, lone target)
 *   og_kappa, og_gain                  pinned (boresight, 3-dB point)
 *   og_tap                             pinned (numpy.sinc * numpy.i0)
 *   og_forward                         pinned (lone/off-grid target, Doppler
 *                                      of eq. 4, linearity, mpmath brute force)
 *   og_adjoint                         pinned (dot-product test, finite
 *                                      differences of og_forward)
 *   og_chirp, og_waveform[_adjoint]    pinned (numpy FFT convolution, matched
 *                                      filter peak, adjoint identity)
 *   og_philox4x32_10                   pinned bit for bit against rocRAND's
 *                                      header-only engine (an independent
 *                                      implementation) on 56 counters and
 *                                      keys; statistical pins besides
 *   og_generate_facets                 pinned (closed-form moments, dispersion,
 *                                      d(eta)/dt = w, chunk invariance; tiles of
 *                                      eq. 1-2: corner fields, squared weights
 *                                      summing to one, variance kept; CWM:
 *                                      trochoid mean level and excursion,
 *                                      displacement rate = velocity)
 *   steer_ant (time-dependent frames)  pinned (zero rate = stripmap, steered
 *                                      gain = static gain of the facet rotated
 *                                      back about el, back plane, finite
 *                                      differences)
 *   og_echo_time, rx_exact model       pinned (50-digit mpmath root of the echo
 *                                      equation, static-receiver case, lone
 *                                      facet phase/delay shift, finite
 *                                      differences of the implicit gradient)
 *   grid_field (u-v gridded patterns)  pinned (node values, exact on bilinear
 *                                      functions, second-order convergence to
 *                                      the sampled analytic pattern, zero
 *                                      outside, finite differences)
 *   og_speckle_anchors, og_speckle_groups
 *                                      pinned (exact covariance of the
 *                                      construction = the AR(1) law of eq. 10;
 *                                      frozen and white limits)
 *   og_speckle_draw, og_philox2x32_10  bit patterns: parity unpinned;
 *                                      statistical pins (Exp(1) power,
 *                                      uniform angle, avalanche)
 *   og_forward_speckle, og_adjoint_speckle
 *                                      pinned (lone facet closed form of
 *                                      eq. 7, id-keeping split, row slices,
 *                                      eq. 9 autocorrelation, dot-product
 *                                      test, finite differences)
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OG_MAXP 8
#define OG_MAXA 8
#define OG_MAXC 16

typedef struct {
    double c, f0, fs, prf;
    int n_samples, n_pulses, n_ref;
    double kaiser_beta, chirp_bw, chirp_T;
    int n_plat;
    double plat_p0[OG_MAXP][3];
    double plat_v[OG_MAXP][3];
    int n_ant;
    int ant_plat[OG_MAXA];
    double ant_beta_az[OG_MAXA];
    double ant_beta_el[OG_MAXA];
    int n_ch;
    int ch_tx[OG_MAXC];
    int ch_rx[OG_MAXC];
    double ch_off[OG_MAXC][3];
    int rx_exact;   /* 1: receiver at each facet's own echo time (see facet_rx) */
    double ant_steer[OG_MAXA];   /* steering rate about the elevation axis (rad/s) */
    /* u-v gridded field patterns (see gain): NULL = the analytic sinc pattern;
     * else values [nv][nu] (u fastest) at u = u0 + i du, v = v0 + j dv */
    const double *ant_grid[OG_MAXA];
    int ant_gnu[OG_MAXA], ant_gnv[OG_MAXA];
    double ant_gu0[OG_MAXA], ant_gdu[OG_MAXA], ant_gv0[OG_MAXA], ant_gdv[OG_MAXA];
} og_config;

static const double OG_PI = 3.14159265358979323846;

/* Threads an OpenMP region of this library uses. */
int og_num_threads(void) { return omp_get_max_threads(); }

static double dot3(const double *a, const double *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static double norm3(const double *a) { return sqrt(dot3(a, a)); }

/* ---- Pulse timing and platform motion --------------------------------- */

/* Pulse time origin is silent in the paper; reading: centred on the dwell. */
double og_pulse_time(const og_config *g, int p) {
    return ((double)p - 0.5 * (double)(g->n_pulses - 1)) / g->prf;
}

static void plat_pos(const og_config *g, int plat, double t, double *out) {
    for (int k = 0; k < 3; ++k) out[k] = g->plat_p0[plat][k] + g->plat_v[plat][k] * t;
}

/* Tx phase centre: the Tx antenna's platform. */
static void tx_pos(const og_config *g, int ch, double t, double *out) {
    plat_pos(g, g->ant_plat[g->ch_tx[ch]], t, out);
}

/* Rx phase centre: the Rx antenna's platform plus the channel's offset. */
static void rx_pos(const og_config *g, int ch, double t, double *out) {
    plat_pos(g, g->ant_plat[g->ch_rx[ch]], t, out);
    for (int k = 0; k < 3; ++k) out[k] += g->ch_off[ch][k];
}

/*
 * Per-pulse geometry (eq. 3 evaluates r_t at the transmit time and r_r at the
 * reception time).  Reading: Tx at the pulse time t_p; Rx at t_p + tau_ref,
 * where tau_ref is the echo delay of the scene origin O, found as the fixed
 * point of  c*tau = |O - P_tx(t_p)| + |O - P_rx(t_p + tau)|.
 */
void og_pulse_geometry(const og_config *g, int ch, int p, double *t_out,
                       double *ptx, double *prx, double *tau_out) {
    double t = og_pulse_time(g, p);
    tx_pos(g, ch, t, ptx);
    double rt = norm3(ptx);                 /* |O - P_tx|, O = origin */
    double tau = 2.0 * rt / g->c;
    for (int it = 0; it < 50; ++it) {
        rx_pos(g, ch, t + tau, prx);
        double nt = (rt + norm3(prx)) / g->c;
        if (nt == tau) break;
        tau = nt;
    }
    rx_pos(g, ch, t + tau, prx);
    *t_out = t;
    *tau_out = tau;
}

/* ---- Antenna model ---------------------------------------------------- */

static double sinc(double x) {
    if (x == 0.0) return 1.0;
    double px = OG_PI * x;
    return sin(px) / px;
}

/* d sinc / dx */
static double dsinc(double x) {
    if (x == 0.0) return 0.0;
    double px = OG_PI * x;
    return (cos(px) - sin(px) / px) / x;
}

/* kappa such that sinc(kappa/2)^2 = 1/2: the sinc^2 power pattern then has
 * its one-way 3-dB full width equal to beta. */
double og_kappa(void) {
    double lo = 0.0, hi = 1.0, target = sqrt(0.5);
    for (int i = 0; i < 200; ++i) {
        double mid = 0.5 * (lo + hi);
        if (sinc(mid) > target) lo = mid; else hi = mid;
    }
    return lo + hi;  /* 2 * midpoint */
}

/*
 * Antenna frame (reading of "all 3 antennas mechanically point to the same
 * surface target", stripmap, frames fixed over the dwell): boresight b = unit
 * vector from the platform position at t = 0 to O, azimuth axis = along-track
 * x projected orthogonal to b, elevation axis = b x az.
 */
void og_antenna_frame(const og_config *g, int ant, double *b, double *az, double *el) {
    double p[3];
    plat_pos(g, g->ant_plat[ant], 0.0, p);
    double r = norm3(p);
    for (int k = 0; k < 3; ++k) b[k] = -p[k] / r;
    double xh[3] = {1.0, 0.0, 0.0};
    double d = dot3(xh, b);
    for (int k = 0; k < 3; ++k) az[k] = xh[k] - d * b[k];
    double na = norm3(az);
    for (int k = 0; k < 3; ++k) az[k] /= na;
    el[0] = b[1] * az[2] - b[2] * az[1];
    el[1] = b[2] * az[0] - b[0] * az[2];
    el[2] = b[0] * az[1] - b[1] * az[0];
}

/* Per-antenna constants: frame and pattern scale factors. */
typedef struct {
    double b[3], az[3], el[3];
    double ka, ke;            /* kappa / beta_az, kappa / beta_el */
    const double *grid;       /* gridded pattern or NULL (og_config.ant_grid) */
    int gnu, gnv;
    double gu0, gdu, gv0, gdv;
} og_ant;

static void make_ant(const og_config *g, int ant, double kap, og_ant *a) {
    og_antenna_frame(g, ant, a->b, a->az, a->el);
    a->ka = kap / g->ant_beta_az[ant];
    a->ke = kap / g->ant_beta_el[ant];
    a->grid = g->ant_grid[ant];
    a->gnu = g->ant_gnu[ant];
    a->gnv = g->ant_gnv[ant];
    a->gu0 = g->ant_gu0[ant];
    a->gdu = g->ant_gdu[ant];
    a->gv0 = g->ant_gv0[ant];
    a->gdv = g->ant_gdv[ant];
}

/*
 * Gridded field pattern (Sec. III.B: patterns, whatever their source, are
 * converted into u-v grids held in GPU memory).  Reading: a real one-way field
 * gain tabulated over the direction cosines u (azimuth axis) and v (elevation
 * axis), interpolated bilinearly; the table covers the half-open cells
 * [u0, u0 + (nu-1) du) x [v0, v0 + (nv-1) dv) and the field is 0 outside.
 * dFu, dFv receive dF/du, dF/dv (piecewise constant along each axis).
 */
static double grid_field(const og_ant *a, double u, double v, double *dFu, double *dFv) {
    double x = (u - a->gu0) / a->gdu, y = (v - a->gv0) / a->gdv;
    *dFu = *dFv = 0.0;
    if (!(x >= 0.0 && x < a->gnu - 1 && y >= 0.0 && y < a->gnv - 1)) return 0.0;
    int i = (int)floor(x), j = (int)floor(y);
    double fx = x - i, fy = y - j;
    const double *r0 = a->grid + (size_t)j * a->gnu + i, *r1 = r0 + a->gnu;
    double f00 = r0[0], f10 = r0[1], f01 = r1[0], f11 = r1[1];
    *dFu = ((1.0 - fy) * (f10 - f00) + fy * (f11 - f01)) / a->gdu;
    *dFv = ((1.0 - fx) * (f01 - f00) + fx * (f11 - f10)) / a->gdv;
    return (1.0 - fx) * (1.0 - fy) * f00 + fx * (1.0 - fy) * f10 + (1.0 - fx) * fy * f01 +
           fx * fy * f11;
}

/*
 * One-way field pattern of an antenna (eq. 16 weights each facet by the Tx and
 * Rx complex gains).  Reading of "sinc^2 antennas (az, el widths)": sinc^2 is
 * the one-way power pattern with those 3-dB widths, so the field is
 * F = sinc(kappa*u/beta_az) * sinc(kappa*v/beta_el), u, v the direction
 * cosines of the unit vector antenna->facet on the az / el axes; F = 0 behind
 * the antenna.  grad (optional) receives dF/dX.  An antenna with a gridded
 * pattern takes F from its grid instead (grid_field), same back plane.
 */
static double gain(const og_ant *a, const double *pa, const double *x, double *grad) {
    double d[3] = {x[0] - pa[0], x[1] - pa[1], x[2] - pa[2]};
    double r = norm3(d);
    double rh[3] = {d[0] / r, d[1] / r, d[2] / r};
    if (dot3(rh, a->b) <= 0.0) {
        if (grad) grad[0] = grad[1] = grad[2] = 0.0;
        return 0.0;
    }
    double u = dot3(rh, a->az), v = dot3(rh, a->el);
    if (a->grid) {
        double dFu, dFv;
        double F = grid_field(a, u, v, &dFu, &dFv);
        if (grad)
            for (int k = 0; k < 3; ++k)
                grad[k] = dFu * (a->az[k] - u * rh[k]) / r + dFv * (a->el[k] - v * rh[k]) / r;
        return F;
    }
    double su = sinc(a->ka * u), sv = sinc(a->ke * v);
    if (grad) {
        double dsu = a->ka * dsinc(a->ka * u), dsv = a->ke * dsinc(a->ke * v);
        for (int k = 0; k < 3; ++k) {
            double du = (a->az[k] - u * rh[k]) / r;   /* d(rh.az)/dX */
            double dv = (a->el[k] - v * rh[k]) / r;
            grad[k] = dsu * sv * du + su * dsv * dv;
        }
    }
    return su * sv;
}

/* Public single-evaluation form (tests). */
double og_gain(const og_config *g, int ant, const double *pa, const double *x,
               double *grad) {
    og_ant a;
    make_ant(g, ant, og_kappa(), &a);
    return gain(&a, pa, x, grad);
}

/* ---- Range interpolator (deposit into range slices, eq. 17) ----------- */

/* Modified Bessel I0 by its power series. */
static double bessel_i0(double x) {
    double term = 1.0, sum = 1.0, q = 0.25 * x * x;
    for (int k = 1; k < 500; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

/* I1(x)/x by its power series (finite at x = 0). */
static double bessel_i1_over_x(double x) {
    double term = 0.5, sum = 0.5, q = 0.25 * x * x;
    for (int k = 1; k < 500; ++k) {
        term *= q / ((double)k * (double)(k + 1));
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

/*
 * Reading of eq. 17's range slices: instead of a box, each contribution is
 * spread over 8 samples with a Kaiser-windowed sinc of half-width 4:
 * h(t) = sinc(t) * I0(beta*sqrt(1-(t/4)^2)) / I0(beta), |t| <= 4, else 0.
 * i0b = I0(beta).
 */
static double tap(double t, double beta, double i0b) {
    if (fabs(t) > 4.0) return 0.0;
    double s = 1.0 - (t / 4.0) * (t / 4.0);
    if (s < 0.0) s = 0.0;
    return sinc(t) * bessel_i0(beta * sqrt(s)) / i0b;
}

/* dh/dt: sinc'(t) W(t) + sinc(t) W'(t), W'(t) = I1(beta s) beta ds/dt / I0(beta),
 * s = sqrt(1 - (t/4)^2), ds/dt = -t / (16 s). */
static double dtap(double t, double beta, double i0b) {
    if (fabs(t) > 4.0) return 0.0;
    double s2 = 1.0 - (t / 4.0) * (t / 4.0);
    if (s2 < 0.0) s2 = 0.0;
    double s = sqrt(s2);
    double w = bessel_i0(beta * s) / i0b;
    double dw = -bessel_i1_over_x(beta * s) * beta * beta * t / 16.0 / i0b;
    return dsinc(t) * w + sinc(t) * dw;
}

double og_tap(double t, double beta) { return tap(t, beta, bessel_i0(beta)); }
double og_dtap(double t, double beta) { return dtap(t, beta, bessel_i0(beta)); }

/* ---- Per-(channel, pulse) row quantities ------------------------------ */

typedef struct {
    double t, tau, rref;
    double ptx[3], prx[3];
    double rt_mid, rr_mid;
    og_ant at, ar;   /* Tx and Rx antennas of the row's channel, steered */
} og_row;

/* Per-call constants: antenna frames and I0(beta). */
typedef struct {
    og_ant ant[OG_MAXA];
    double i0b;
} og_ctx;

static void make_ctx(const og_config *g, og_ctx *cx) {
    double kap = og_kappa();
    for (int a = 0; a < g->n_ant; ++a) make_ant(g, a, kap, &cx->ant[a]);
    cx->i0b = bessel_i0(g->kaiser_beta);
}

/*
 * Time-dependent antenna patterns (Sec. III.B: time dependent in the TOPSAR
 * modes).  Reading: each antenna's frame turns about its elevation axis at
 * the constant rate ant_steer: with phi = rate * t,
 *   b(t) = b cos(phi) + az sin(phi),  az(t) = az cos(phi) - b sin(phi),
 * el unchanged; the Tx antenna is taken at the pulse time t_p, the Rx antenna
 * at t_p + tau_ref (one state per pulse and channel).
 */
static void steer_ant(const og_ant *a, double phi, og_ant *o) {
    const double c = cos(phi), s = sin(phi);
    *o = *a;
    for (int k = 0; k < 3; ++k) {
        o->b[k] = a->b[k] * c + a->az[k] * s;
        o->az[k] = a->az[k] * c - a->b[k] * s;
    }
}

static void steer_row(const og_config *g, const og_ctx *cx, int ch, og_row *r) {
    const int ta = g->ch_tx[ch], ra = g->ch_rx[ch];
    steer_ant(&cx->ant[ta], g->ant_steer[ta] * r->t, &r->at);
    steer_ant(&cx->ant[ra], g->ant_steer[ra] * (r->t + r->tau), &r->ar);
}

static void make_row(const og_config *g, int ch, int p, og_row *r) {
    og_pulse_geometry(g, ch, p, &r->t, r->ptx, r->prx, &r->tau);
    r->rref = g->c * r->tau;
    double p0[3];
    tx_pos(g, ch, 0.0, p0);
    r->rt_mid = norm3(p0);
    rx_pos(g, ch, 0.0, p0);
    r->rr_mid = norm3(p0);
}

/*
 * Receiver position for the echo of point X (eq. 3 evaluates r_r at the
 * reception time t_r): the fixed point of
 *     c tau = |X - P_tx(t_p)| + |X - P_rx(t_p + tau)|,
 * iterated from tau_ref until it stops changing.  Used when rx_exact is set;
 * otherwise every facet of a row uses P_rx(t_p + tau_ref) (reading: the
 * receiver position of the scene origin's echo).
 */
static double facet_rx(const og_config *g, int ch, const og_row *r, const double *X,
                       double *prx) {
    const double dt[3] = {X[0] - r->ptx[0], X[1] - r->ptx[1], X[2] - r->ptx[2]};
    const double rt = norm3(dt);
    double tau = r->tau;
    for (int it = 0; it < 50; ++it) {
        rx_pos(g, ch, r->t + tau, prx);
        const double dr[3] = {X[0] - prx[0], X[1] - prx[1], X[2] - prx[2]};
        const double nt = (rt + norm3(dr)) / g->c;
        if (nt == tau) break;
        tau = nt;
    }
    rx_pos(g, ch, r->t + tau, prx);
    return tau;
}

/* Echo delay of point X in channel ch, pulse p (rx_exact model). */
double og_echo_time(const og_config *g, int ch, int p, const double *X) {
    og_row r;
    og_pulse_geometry(g, ch, p, &r.t, r.ptx, r.prx, &r.tau);
    double prx[3];
    return facet_rx(g, ch, &r, X, prx);
}

/* Velocity of the receive phase centre of channel ch. */
static void rx_vel(const og_config *g, int ch, double *v) {
    for (int k = 0; k < 3; ++k) v[k] = g->plat_v[g->ant_plat[g->ch_rx[ch]]][k];
}

/*
 * One facet's contribution to one (channel, pulse) row: eq. 3 / eq. 16.
 * Outputs the complex weight W = a * Ftx * Frx * S * exp(j*(phi + dphi)) and
 * the fractional sample position u of the bistatic range in the tracking
 * window (dphi: the intra-facet Doppler phase of eq. 7, 0 without speckle;
 * a then carries the speckle factor x of eq. 7 as well).
 *   X = X0 + V t_p (linear facet motion over the dwell)
 *   R = |X - P_tx| + |X - P_rx|,  phi = -2 pi f0 R / c   (e^{-i K0 (r_t + r_r)})
 *   u = n_ref + (R - c tau_ref) fs / c
 *   S = (R_t,mid R_r,mid) / (R_t R_r)   (1/(r_t r_r) spreading, normalised
 *       to the scene-origin ranges at t = 0; other constants set to 1)
 */
static void contribution(const og_config *g, int ch, const og_row *r,
                         const double *x0, const double *v, double are, double aim,
                         double dphi, double *wre, double *wim, double *u) {
    double X[3];
    for (int k = 0; k < 3; ++k) X[k] = x0[k] + v[k] * r->t;
    double prx[3] = {r->prx[0], r->prx[1], r->prx[2]};
    if (g->rx_exact) facet_rx(g, ch, r, X, prx);
    double dt[3] = {X[0] - r->ptx[0], X[1] - r->ptx[1], X[2] - r->ptx[2]};
    double dr[3] = {X[0] - prx[0], X[1] - prx[1], X[2] - prx[2]};
    double Rt = norm3(dt), Rr = norm3(dr), R = Rt + Rr;
    double ft = gain(&r->at, r->ptx, X, NULL);
    double fr = gain(&r->ar, prx, X, NULL);
    double S = (r->rt_mid * r->rr_mid) / (Rt * Rr);
    double phi = -2.0 * OG_PI * g->f0 * R / g->c + dphi;
    double amp = ft * fr * S;
    double c = cos(phi), s = sin(phi);
    *wre = amp * (are * c - aim * s);
    *wim = amp * (are * s + aim * c);
    *u = (double)g->n_ref + (R - r->rref) * g->fs / g->c;
}

/*
 * Forward sum: iq[c][p - p0][n] (interleaved re, im) for channels 0..n_ch-1,
 * pulses [p0, p0 + np).  Each (c, p) row is independent (parallel, no races).
 * Taps outside [0, N) are dropped.  With xs != NULL, facet i's amplitude at
 * pulse p is a_i x_i(p) (xs[i][p - p0], complex) and its phase gains
 * 2 pi f_s,i t_p: the intra-facet speckle s(t) of eq. 7.
 */
static void forward_impl(const og_config *g, long long nf, const double *x, const double *y,
                         const double *z, const double *vx, const double *vy,
                         const double *vz, const double *are, const double *aim,
                         const double *xs, const double *fs, int p0, int np, double *iq) {
    const int N = g->n_samples;
    const long long rows = (long long)g->n_ch * np;
    memset(iq, 0, sizeof(double) * 2 * (size_t)rows * (size_t)N);
    og_ctx cx;
    make_ctx(g, &cx);
#pragma omp parallel for schedule(dynamic, 1)
    for (long long row = 0; row < rows; ++row) {
        int ch = (int)(row / np), p = p0 + (int)(row % np);
        og_row r;
        make_row(g, ch, p, &r);
        steer_row(g, &cx, ch, &r);
        double *out = iq + 2 * (size_t)row * (size_t)N;
        for (long long i = 0; i < nf; ++i) {
            double X0[3] = {x[i], y[i], z[i]}, V[3] = {vx[i], vy[i], vz[i]};
            double ar = are[i], ai = aim[i], dphi = 0.0;
            if (xs) {
                const double *s = xs + 2 * ((size_t)i * (size_t)np + (size_t)(p - p0));
                ar = are[i] * s[0] - aim[i] * s[1];
                ai = are[i] * s[1] + aim[i] * s[0];
                dphi = fs ? 2.0 * OG_PI * fs[i] * r.t : 0.0;
            }
            double wre, wim, u;
            contribution(g, ch, &r, X0, V, ar, ai, dphi, &wre, &wim, &u);
            long long n0 = (long long)floor(u);
            for (long long n = n0 - 3; n <= n0 + 4; ++n) {
                if (n < 0 || n >= N) continue;
                double h = tap((double)n - u, g->kaiser_beta, cx.i0b);
                out[2 * n] += wre * h;
                out[2 * n + 1] += wim * h;
            }
        }
    }
}

void og_forward(const og_config *g, long long nf, const double *x, const double *y,
                const double *z, const double *vx, const double *vy, const double *vz,
                const double *are, const double *aim, int p0, int np, double *iq) {
    forward_impl(g, nf, x, y, z, vx, vy, vz, are, aim, NULL, NULL, p0, np, iq);
}

/*
 * Adjoint of og_forward with respect to facet height z, velocity V and
 * complex amplitude a.  g_iq holds dL/dRe(IQ) + j dL/dIm(IQ) in the layout of
 * og_forward's output.  Returns dL/dz, dL/dV (components), dL/dRe a and
 * dL/dIm a.  Each facet is independent (parallel, deterministic).
 *
 * With B = sum_n conj(g_n) h(n - u), B' = sum_n conj(g_n) h'(n - u),
 * T = Ftx Frx S, E = exp(j phi), P = B a E:
 *   dL/da       = conj(B T E)
 * (with speckle, a is replaced by a s and dL/da = conj(B T E s), phi
 * including the Doppler phase; s does not depend on z, V or a)
 *   dL/dX       = Re(P) grad T + [Im(P) T K0 - Re(B' a T E) fs/c] grad R
 *   dL/dz       = sum_p (dL/dX)_z,   dL/dV = sum_p t_p dL/dX
 * where grad R = unit(X - P_tx) + unit(X - P_rx), K0 = 2 pi f0 / c (with
 * rx_exact, the implicit-function gradient of the facet's own echo time).
 */
static void adjoint_impl(const og_config *g, long long nf, const double *x, const double *y,
                         const double *z, const double *vx, const double *vy,
                         const double *vz, const double *are, const double *aim,
                         const double *xs, const double *fs, int p0, int np,
                         const double *giq, double *dz, double *dvx, double *dvy,
                         double *dvz, double *dare, double *daim) {
    const int N = g->n_samples;
    const int rows = g->n_ch * np;
    og_ctx cx;
    make_ctx(g, &cx);
    og_row *rw = (og_row *)malloc(sizeof(og_row) * (size_t)rows);
    for (int row = 0; row < rows; ++row) {
        make_row(g, row / np, p0 + row % np, &rw[row]);
        steer_row(g, &cx, row / np, &rw[row]);
    }
    const double K0 = 2.0 * OG_PI * g->f0 / g->c;
#pragma omp parallel for schedule(dynamic, 64)
    for (long long i = 0; i < nf; ++i) {
        double X0[3] = {x[i], y[i], z[i]}, V[3] = {vx[i], vy[i], vz[i]};
        double gz = 0, gv[3] = {0, 0, 0}, gar = 0, gai = 0;
        for (int row = 0; row < rows; ++row) {
            const og_row *r = &rw[row];
            int ch = row / np;
            /* speckle factor of this pulse (1 without speckle) and Doppler phase */
            double sr = 1.0, si = 0.0, dphi = 0.0;
            if (xs) {
                const double *sp = xs + 2 * ((size_t)i * (size_t)np + (size_t)(row % np));
                sr = sp[0];
                si = sp[1];
                dphi = fs ? 2.0 * OG_PI * fs[i] * r->t : 0.0;
            }
            double ar = are[i] * sr - aim[i] * si, ai = are[i] * si + aim[i] * sr;
            double X[3];
            for (int k = 0; k < 3; ++k) X[k] = X0[k] + V[k] * r->t;
            double prx[3] = {r->prx[0], r->prx[1], r->prx[2]};
            if (g->rx_exact) facet_rx(g, ch, r, X, prx);
            double dt[3] = {X[0] - r->ptx[0], X[1] - r->ptx[1], X[2] - r->ptx[2]};
            double dr[3] = {X[0] - prx[0], X[1] - prx[1], X[2] - prx[2]};
            double Rt = norm3(dt), Rr = norm3(dr), R = Rt + Rr;
            double gft[3], gfr[3];
            double ft = gain(&r->at, r->ptx, X, gft);
            double fr = gain(&r->ar, prx, X, gfr);
            double S = (r->rt_mid * r->rr_mid) / (Rt * Rr);
            double T = ft * fr * S;
            double phi = -2.0 * OG_PI * g->f0 * R / g->c + dphi;
            double Er = cos(phi), Ei = sin(phi);
            double u = (double)g->n_ref + (R - r->rref) * g->fs / g->c;
            const double *grow = giq + 2 * (size_t)row * (size_t)N;
            double Br = 0, Bi = 0, Bpr = 0, Bpi = 0;
            long long n0 = (long long)floor(u);
            for (long long n = n0 - 3; n <= n0 + 4; ++n) {
                if (n < 0 || n >= N) continue;
                double h = tap((double)n - u, g->kaiser_beta, cx.i0b);
                double hp = dtap((double)n - u, g->kaiser_beta, cx.i0b);
                /* conj(g_n) = (gr, -gi) */
                Br += grow[2 * n] * h;
                Bi += -grow[2 * n + 1] * h;
                Bpr += grow[2 * n] * hp;
                Bpi += -grow[2 * n + 1] * hp;
            }
            /* Z = B T E s ; grad_a += conj(Z) */
            double Zr0 = T * (Br * Er - Bi * Ei), Zi0 = T * (Br * Ei + Bi * Er);
            double Zr = Zr0 * sr - Zi0 * si, Zi = Zr0 * si + Zi0 * sr;
            gar += Zr;
            gai += -Zi;
            /* P = B a s E */
            double aEr = ar * Er - ai * Ei, aEi = ar * Ei + ai * Er;
            double Pr = Br * aEr - Bi * aEi, Pi = Br * aEi + Bi * aEr;
            /* Re(B' a T E) */
            double BpW = T * (Bpr * aEr - Bpi * aEi);
            double cR = Pi * T * K0 - BpW * g->fs / g->c;
            /* grad R; with the facet's own reception time R is implicit,
             * R = R_t(X) + |X - P_rx(t_p + R/c)|, so grad R = (u_t + u_r) /
             * (1 + u_r.V_rx/c), and a function h(X - P_rx) has the total
             * gradient grad h - grad R (V_rx . grad h)/c */
            double gR[3], vr[3] = {0, 0, 0}, q = 1.0;
            if (g->rx_exact) {
                rx_vel(g, ch, vr);
                q = 1.0 / (1.0 + (dr[0] * vr[0] + dr[1] * vr[1] + dr[2] * vr[2]) / (Rr * g->c));
            }
            for (int k = 0; k < 3; ++k) gR[k] = q * (dt[k] / Rt + dr[k] / Rr);
            double gSr[3];
            for (int k = 0; k < 3; ++k) gSr[k] = dr[k] / (Rr * Rr);
            const double vgfr = (vr[0] * gfr[0] + vr[1] * gfr[1] + vr[2] * gfr[2]) / g->c;
            const double vgsr = (vr[0] * gSr[0] + vr[1] * gSr[1] + vr[2] * gSr[2]) / g->c;
            double gX[3];
            for (int k = 0; k < 3; ++k) {
                double rt_k = dt[k] / Rt;
                double gfr_k = gfr[k] - gR[k] * vgfr;
                double gS = -S * (rt_k / Rt + gSr[k] - gR[k] * vgsr);
                double gT = fr * S * gft[k] + ft * S * gfr_k + ft * fr * gS;
                gX[k] = Pr * gT + cR * gR[k];
            }
            gz += gX[2];
            for (int k = 0; k < 3; ++k) gv[k] += r->t * gX[k];
        }
        dz[i] = gz;
        dvx[i] = gv[0];
        dvy[i] = gv[1];
        dvz[i] = gv[2];
        dare[i] = gar;
        daim[i] = gai;
    }
    free(rw);
}

void og_adjoint(const og_config *g, long long nf, const double *x, const double *y,
                const double *z, const double *vx, const double *vy, const double *vz,
                const double *are, const double *aim, int p0, int np,
                const double *giq, double *dz, double *dvx, double *dvy,
                double *dvz, double *dare, double *daim) {
    adjoint_impl(g, nf, x, y, z, vx, vy, vz, are, aim, NULL, NULL, p0, np, giq, dz, dvx,
                 dvy, dvz, dare, daim);
}

/* ---- Waveform (the impulse response is convolved by the waveform) ------ */

/* Reading: unit-amplitude up-chirp centred on the pulse,
 * chirp[k] = exp(j pi K (k/fs - T/2)^2), k = 0..L-1, L = round(T fs), K = B/T. */
int og_chirp_len(const og_config *g) { return (int)llround(g->chirp_T * g->fs); }

void og_chirp(const og_config *g, double *out) {
    int L = og_chirp_len(g);
    double K = g->chirp_bw / g->chirp_T;
    for (int k = 0; k < L; ++k) {
        double t = (double)k / g->fs - 0.5 * g->chirp_T;
        double ph = OG_PI * K * t * t;
        out[2 * k] = cos(ph);
        out[2 * k + 1] = sin(ph);
    }
}

/* "Same"-mode linear convolution, raw[n] = sum_m rc[m] chirp[n - m + L/2],
 * evaluated directly, line by line. */
void og_waveform(const og_config *g, long long nlines, const double *rc, double *raw) {
    const int N = g->n_samples, L = og_chirp_len(g), h = L / 2;
    double *ch = (double *)malloc(sizeof(double) * 2 * (size_t)L);
    og_chirp(g, ch);
#pragma omp parallel for schedule(dynamic, 1)
    for (long long l = 0; l < nlines; ++l) {
        const double *x = rc + 2 * (size_t)l * N;
        double *y = raw + 2 * (size_t)l * N;
        for (int n = 0; n < N; ++n) {
            double sr = 0, si = 0;
            for (int m = 0; m < N; ++m) {
                int k = n - m + h;
                if (k < 0 || k >= L) continue;
                sr += x[2 * m] * ch[2 * k] - x[2 * m + 1] * ch[2 * k + 1];
                si += x[2 * m] * ch[2 * k + 1] + x[2 * m + 1] * ch[2 * k];
            }
            y[2 * n] = sr;
            y[2 * n + 1] = si;
        }
    }
    free(ch);
}

/* Adjoint of og_waveform: g_rc[m] = sum_n g_raw[n] conj(chirp[n - m + L/2]). */
void og_waveform_adjoint(const og_config *g, long long nlines, const double *graw,
                         double *grc) {
    const int N = g->n_samples, L = og_chirp_len(g), h = L / 2;
    double *ch = (double *)malloc(sizeof(double) * 2 * (size_t)L);
    og_chirp(g, ch);
#pragma omp parallel for schedule(dynamic, 1)
    for (long long l = 0; l < nlines; ++l) {
        const double *x = graw + 2 * (size_t)l * N;
        double *y = grc + 2 * (size_t)l * N;
        for (int m = 0; m < N; ++m) {
            double sr = 0, si = 0;
            for (int n = 0; n < N; ++n) {
                int k = n - m + h;
                if (k < 0 || k >= L) continue;
                sr += x[2 * n] * ch[2 * k] + x[2 * n + 1] * ch[2 * k + 1];
                si += x[2 * n + 1] * ch[2 * k] - x[2 * n] * ch[2 * k + 1];
            }
            y[2 * m] = sr;
            y[2 * m + 1] = si;
        }
    }
    free(ch);
}

/* ---- Counter-based RNG: Philox4x32-10 (Salmon et al., SC'11) ---------- */

/* One Philox round: two 32x32->64 multiplies, the high halves XORed with the
 * other counter words and the key, words permuted. */
static void philox_round(uint32_t *ctr, const uint32_t *key) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)ctr[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)ctr[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ ctr[1] ^ key[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ ctr[3] ^ key[1];
    uint32_t n3 = lo0;
    ctr[0] = n0; ctr[1] = n1; ctr[2] = n2; ctr[3] = n3;
}

void og_philox4x32_10(const uint32_t *ctr_in, const uint32_t *key_in, uint32_t *out) {
    uint32_t ctr[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t key[2] = {key_in[0], key_in[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {               /* Weyl key schedule */
            key[0] += 0x9E3779B9u;
            key[1] += 0xBB67AE85u;
        }
        philox_round(ctr, key);
    }
    memcpy(out, ctr, sizeof(ctr));
}

/* Four standard normals for facet `index`, stream `stream`: Philox output
 * words mapped to (0,1) as (w + 1/2) 2^-32, then two Box-Muller pairs. */
static void normals4(uint64_t seed, uint64_t index, uint32_t stream, double *n) {
    uint32_t ctr[4] = {(uint32_t)index, (uint32_t)(index >> 32), stream, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    og_philox4x32_10(ctr, key, w);
    const double sc = 1.0 / 4294967296.0;
    for (int j = 0; j < 2; ++j) {
        double u1 = ((double)w[2 * j] + 0.5) * sc;
        double u2 = ((double)w[2 * j + 1] + 0.5) * sc;
        double r = sqrt(-2.0 * log(u1));
        n[2 * j] = r * cos(2.0 * OG_PI * u2);
        n[2 * j + 1] = r * sin(2.0 * OG_PI * u2);
    }
}

/* ---- Sea-surface facets (Sec. III: resolved waves move the grid) ------- */

typedef struct {
    int nx, ny;            /* full grid, cell centres centred on O */
    double dx, dy;
    int mode;              /* 0 flat (iid velocities), 1 linear waves + current */
    double sigma_v;
    int n_comp;
    double k_min, k_max, slope, hs, g;
    const double *dirs;    /* [n_comp] propagation directions */
    const double *phases;  /* [n_comp] initial phases */
    double cur[2];         /* uniform current */
    /* mode 2, heterogeneous sea (eq. 1, 2): TL tiles of side tile_L, corner
     * node (i, j) at (tile_x0 + i L, tile_y0 + j L), i <= ntx, j <= nty, each
     * with its own homogeneous field (T2L tile): significant height
     * node_hs[j (ntx+1) + i], directions and phases node_dirs / node_phases
     * [node][n_comp]; k range, slope and g shared */
    int ntx, nty;
    double tile_L, tile_x0, tile_y0;
    const double *node_hs;
    const double *node_dirs;
    const double *node_phases;
    int cwm;               /* Choppy Wave Model horizontal displacement */
} og_sea;

/*
 * Component table (reading of the tile spectrum for a linear surface):
 * wavenumbers log-spaced over [k_min, k_max]; omnidirectional spectrum
 * Psi(k) proportional to k^slope; amplitude A_m = sqrt(2 Psi(k_m) dk_m) with
 * dk_m the local log spacing, scaled so that sum A_m^2 / 2 = (Hs/4)^2;
 * deep-water dispersion omega^2 = g k.
 */
void og_wave_table(const og_sea *s, double *k, double *amp, double *omega) {
    int n = s->n_comp;
    double dl = (n > 1) ? log(s->k_max / s->k_min) / (double)(n - 1) : 1.0;
    double e = 0.0;
    for (int m = 0; m < n; ++m) {
        k[m] = (n > 1) ? s->k_min * exp(dl * (double)m) : s->k_min;
        amp[m] = sqrt(2.0 * pow(k[m], s->slope) * k[m] * dl);
        e += 0.5 * amp[m] * amp[m];
        omega[m] = sqrt(s->g * k[m]);
    }
    double sig = s->hs / 4.0, f = sig / sqrt(e);
    for (int m = 0; m < n; ++m) amp[m] *= f;
}

/*
 * Linear wave field of one homogeneous tile at the point at rest (X, Y),
 * added to D with weight Wt: height eta = sum A cos(theta), theta =
 * k (cos psi X + sin psi Y) + phase; Choppy Wave Model horizontal
 * displacement -sum A (cos psi, sin psi) sin(theta) (Sec. III: grid points
 * follow the orbital motion); velocity = the time derivative of the
 * displacement: sum A omega (cos psi, sin psi) cos(theta) horizontally and
 * sum A omega sin(theta) vertically.
 */
static void wave_field(int n, const double *k, const double *amp, const double *om,
                       const double *dirs, const double *phases, double X, double Y,
                       double *D, double Wt) {
    for (int m = 0; m < n; ++m) {
        double cp = cos(dirs[m]), sp = sin(dirs[m]);
        double th = k[m] * (cp * X + sp * Y) + phases[m];
        double ct = cos(th), st = sin(th);
        D[0] += Wt * amp[m] * ct;
        D[1] -= Wt * amp[m] * cp * st;
        D[2] -= Wt * amp[m] * sp * st;
        D[3] += Wt * amp[m] * om[m] * cp * ct;
        D[4] += Wt * amp[m] * om[m] * sp * ct;
        D[5] += Wt * amp[m] * om[m] * st;
    }
}

/*
 * Facets of the sub-rectangle [ix0, ix0+cnx) x [iy0, iy0+cny), row-major.
 * Global index = iy*nx + ix is the Philox counter, so any chunking of the grid
 * yields the same facets.
 *   a ~ CN(0,1): (n0, n1)/sqrt(2) from stream 0.
 *   mode 0: z = 0, V = sigma_v (n2, n3, n4), n4 from stream 1.
 *   mode 1: z = sum A cos(theta), theta = k (cos psi x + sin psi y) + phase,
 *           horizontal orbital velocity sum A omega (cos psi, sin psi) cos(theta)
 *           plus the current, vertical velocity sum A omega sin(theta)
 *           (= d(eta)/dt at the surface).
 *   mode 2: the heterogeneous surface of eq. 1: in the TL tile holding the
 *           point, the fields of its four corner nodes weighted by eq. 2
 *           (points outside the node lattice use its border tiles).
 *   cwm:    the facet sits at its rest position plus the weighted horizontal
 *           displacement (Choppy Wave Model); z and V as above.
 * out: 8 arrays of cnx*cny doubles: x, y, z, vx, vy, vz, a_re, a_im.
 */
void og_generate_facets(const og_sea *s, uint64_t seed, int ix0, int iy0, int cnx,
                        int cny, double *x, double *y, double *z, double *vx,
                        double *vy, double *vz, double *are, double *aim) {
    int nc = s->n_comp > 0 ? s->n_comp : 1;
    double *k = (double *)malloc(sizeof(double) * nc);
    double *amp = (double *)malloc(sizeof(double) * nc);
    double *om = (double *)malloc(sizeof(double) * nc);
    double *namp = NULL;
    if (s->mode >= 1) og_wave_table(s, k, amp, om);
    if (s->mode == 2) {
        /* each node's amplitudes: the same spectrum shape at its own Hs */
        const int nn = (s->ntx + 1) * (s->nty + 1);
        namp = (double *)malloc(sizeof(double) * (size_t)nn * (size_t)nc);
        og_sea one = *s;
        for (int q = 0; q < nn; ++q) {
            one.hs = s->node_hs[q];
            og_wave_table(&one, k, namp + (size_t)q * (size_t)nc, om);
        }
    }
    long long n = (long long)cnx * cny;
#pragma omp parallel for schedule(static)
    for (long long j = 0; j < n; ++j) {
        int ix = ix0 + (int)(j % cnx), iy = iy0 + (int)(j / cnx);
        uint64_t gidx = (uint64_t)iy * (uint64_t)s->nx + (uint64_t)ix;
        double X = ((double)ix - 0.5 * (double)(s->nx - 1)) * s->dx;
        double Y = ((double)iy - 0.5 * (double)(s->ny - 1)) * s->dy;
        double nr[4];
        normals4(seed, gidx, 0u, nr);
        x[j] = X;
        y[j] = Y;
        are[j] = nr[0] / sqrt(2.0);
        aim[j] = nr[1] / sqrt(2.0);
        if (s->mode == 0) {
            double n2[4];
            normals4(seed, gidx, 1u, n2);
            z[j] = 0.0;
            vx[j] = s->sigma_v * nr[2];
            vy[j] = s->sigma_v * nr[3];
            vz[j] = s->sigma_v * n2[0];
        } else {
            /* displacement and velocity of the point at rest (X, Y): one
             * homogeneous field (mode 1) or the weighted sum of eq. 1 */
            double D[6] = {0, 0, 0, 0, 0, 0};   /* eta, dx, dy, u, v, w */
            if (s->mode == 1) {
                wave_field(s->n_comp, k, amp, om, s->dirs, s->phases, X, Y, D, 1.0);
            } else {
                int ti = (int)floor((X - s->tile_x0) / s->tile_L);
                int tj = (int)floor((Y - s->tile_y0) / s->tile_L);
                if (ti > s->ntx - 1) ti = s->ntx - 1;
                if (tj > s->nty - 1) tj = s->nty - 1;
                if (ti < 0) ti = 0;
                if (tj < 0) tj = 0;
                for (int c = 0; c < 4; ++c) {
                    const int ni = ti + (c & 1), nj = tj + (c >> 1);
                    const double xi = s->tile_x0 + ni * s->tile_L, yi = s->tile_y0 + nj * s->tile_L;
                    /* eq. 2 */
                    const double wx = fabs(xi - X) / s->tile_L, wy = fabs(yi - Y) / s->tile_L;
                    const double Wt = sqrt(fmax(0.0, 1.0 - wx - wy + wx * wy));
                    const int node = nj * (s->ntx + 1) + ni;
                    const double *na = namp + (size_t)node * (size_t)nc;
                    wave_field(s->n_comp, k, na, om, s->node_dirs + (size_t)node * s->n_comp,
                               s->node_phases + (size_t)node * s->n_comp, X, Y, D, Wt);
                }
            }
            x[j] = s->cwm ? X + D[1] : X;
            y[j] = s->cwm ? Y + D[2] : Y;
            z[j] = D[0];
            vx[j] = D[3] + s->cur[0];
            vy[j] = D[4] + s->cur[1];
            vz[j] = D[5];
        }
    }
    free(k);
    free(amp);
    free(om);
    free(namp);
}

/* ---- Intra-facet speckle (Sec. III.A eq. 7, eq. 9, eq. 10) ------------- */
/*
 * Each facet's reflection coefficient carries s(t_p) = x(p) exp(j 2 pi f_s t_p)
 * (eq. 7), with x = R + jI an order-1 autoregressive process over the pulses
 * (eq. 10):  x(p + 1) = b x(p) + sqrt(1 - b^2) e(p + 1),  b = exp(-dt / tau_s),
 * dt = 1 / prf.  Readings: R and I are independent with variance 1/2 each at
 * every pulse and in every innovation e (eq. 10 prints sigma = 1/2, which
 * would make the process decay from its unit initial power; variance 1/2
 * keeps it stationary, E|x|^2 = 1, as eq. 9 requires at t = 0); tau_s is one
 * value per scene (the paper interpolates it, with f_s, from sea-state tables
 * that are not part of this work); f_s is a per-facet input; one process per
 * facet serves every channel.
 *
 * How the random numbers are drawn is not stated.  Reading: the pulses are cut
 * into groups of 64 (absolute pulse index); the process is sampled at the
 * group starts first (anchors, eq. 10 applied over 64 pulses), then inside each
 * group by eq. 10 pulse by pulse from its anchor, the free path being
 * conditioned on the next anchor (Gaussian conditioning on one value):
 *   y_0 = eta_0,   y_g = b^64 y_{g-1} + sqrt(1 - b^128) eta_g,
 *   z_0 = y_g,     z_k = b z_{k-1} + sqrt(1 - b^2) e_{64 g + k},  k = 1..64,
 *   x(64 g + k) = z_k + K_k (y_{g+1} - z_64),   k = 0..63,
 *   K_k = Cov(z_k, z_64 | z_0) / Var(z_64 | z_0) = b^(64-k) (1 - b^2k) / (1 - b^128).
 * x then has exactly the law of the sequential recursion (E[x(p) conj x(q)] =
 * b^|p-q|), and any group can be produced without the others.  Draws are
 * counter based (facet id, slot): the anchor draw eta_g is slot 2^31 + g, the
 * innovation e_p (p >= 1) is slot p.
 */

/* Philox2x32-10 (Salmon et al., SC'11), the two-word member of the family:
 * each round multiplies the first word by 0xD256D193 (32 x 32 -> 64 bits);
 * the new first word is the high half XOR the second word XOR the key, the
 * new second word is the low half; the key grows by 0x9E3779B9 between
 * rounds. */
void og_philox2x32_10(const uint32_t *ctr_in, uint32_t key, uint32_t *out) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) key += 0x9E3779B9u;
        uint64_t prod = (uint64_t)0xD256D193u * (uint64_t)c0;
        uint32_t hi = (uint32_t)(prod >> 32), lo = (uint32_t)prod;
        c0 = hi ^ c1 ^ key;
        c1 = lo;
    }
    out[0] = c0;
    out[1] = c1;
}

/* One complex normal with E|e|^2 = 1 for (id, slot): Philox2x32-10 of
 * counter (id, slot) under key = low ^ high word of the seed gives w0, w1;
 * u1 = (floor(w0 / 2^9) + 1/2) 2^-23 in (0, 1), u2 = floor(w1 / 2^9) 2^-23 in
 * [0, 1) (both exact in float32); Box-Muller: radius sqrt(-ln u1), angle
 * 2 pi u2. */
void og_speckle_draw(uint64_t seed, uint32_t id, uint32_t slot, double *out) {
    uint32_t ctr[2] = {id, slot}, w[2];
    og_philox2x32_10(ctr, (uint32_t)seed ^ (uint32_t)(seed >> 32), w);
    double u1 = ((double)(w[0] >> 9) + 0.5) * (1.0 / 8388608.0);
    double u2 = (double)(w[1] >> 9) * (1.0 / 8388608.0);
    double rho = sqrt(-log(u1));
    out[0] = rho * cos(2.0 * OG_PI * u2);
    out[1] = rho * sin(2.0 * OG_PI * u2);
}

/* b^m with b = exp(-a), a = dt / tau_s >= 0 */
static double spk_pow(double a, int m) { return exp(-a * (double)m); }

/* bridge gain K_k; its limit k / 64 for a = 0 (frozen speckle) */
static double spk_gain(double a, int k) {
    if (a == 0.0) return (double)k / 64.0;
    return spk_pow(a, 64 - k) * expm1(-2.0 * a * (double)k) / expm1(-128.0 * a);
}

/* Anchors y_0 .. y_{ng-1} from the draws eta (complex, interleaved). */
void og_speckle_anchors(double a, int ng, const double *eta, double *y) {
    const double b64 = spk_pow(a, 64), c64 = sqrt(-expm1(-128.0 * a));
    for (int g = 0; g < ng; ++g) {
        if (g == 0) {
            y[0] = eta[0];
            y[1] = eta[1];
        } else {
            y[2 * g] = b64 * y[2 * g - 2] + c64 * eta[2 * g];
            y[2 * g + 1] = b64 * y[2 * g - 1] + c64 * eta[2 * g + 1];
        }
    }
}

/* x at pulses 64 g0 .. 64 g1 - 1 (complex, interleaved) from the anchors
 * y_{g0} .. y_{g1} (g1 - g0 + 1 values) and the innovations
 * e[64 (g - g0) + k - 1] = e_{64 g + k}, k = 1..64. */
void og_speckle_groups(double a, int g0, int g1, const double *y, const double *e, double *x) {
    const double b = spk_pow(a, 1), c = sqrt(-expm1(-2.0 * a));
    for (int g = g0; g < g1; ++g) {
        const int j = g - g0;
        double zr[65], zi[65];
        zr[0] = y[2 * j];
        zi[0] = y[2 * j + 1];
        for (int k = 1; k <= 64; ++k) {
            const double *ek = e + 2 * (64 * (size_t)j + (size_t)(k - 1));
            zr[k] = b * zr[k - 1] + c * ek[0];
            zi[k] = b * zi[k - 1] + c * ek[1];
        }
        const double dr = y[2 * j + 2] - zr[64], di = y[2 * j + 3] - zi[64];
        for (int k = 0; k < 64; ++k) {
            const double K = spk_gain(a, k);
            x[2 * (64 * (size_t)j + k)] = zr[k] + K * dr;
            x[2 * (64 * (size_t)j + k) + 1] = zi[k] + K * di;
        }
    }
}

/* x(p) of facet `id` for absolute pulses [pa, pb) (complex, interleaved),
 * a = dt / tau_s. */
void og_speckle_series(uint64_t seed, uint32_t id, double a, int pa, int pb, double *x) {
    if (pb <= pa) return;
    const int g0 = pa / 64, g1 = (pb - 1) / 64 + 1;
    double *eta = (double *)malloc(sizeof(double) * 2 * (size_t)(g1 + 1));
    double *y = (double *)malloc(sizeof(double) * 2 * (size_t)(g1 + 1));
    double *e = (double *)malloc(sizeof(double) * 2 * 64 * (size_t)(g1 - g0));
    double *xg = (double *)malloc(sizeof(double) * 2 * 64 * (size_t)(g1 - g0));
    for (int g = 0; g <= g1; ++g) og_speckle_draw(seed, id, 0x80000000u + (uint32_t)g, eta + 2 * g);
    og_speckle_anchors(a, g1 + 1, eta, y);
    for (int g = g0; g < g1; ++g)
        for (int k = 1; k <= 64; ++k)
            og_speckle_draw(seed, id, (uint32_t)(64 * g + k),
                            e + 2 * (64 * (size_t)(g - g0) + (size_t)(k - 1)));
    og_speckle_groups(a, g0, g1, y + 2 * g0, e, xg);
    memcpy(x, xg + 2 * (size_t)(pa - 64 * g0), sizeof(double) * 2 * (size_t)(pb - pa));
    free(eta);
    free(y);
    free(e);
    free(xg);
}

/* dt / tau_s; tau_s = +inf freezes the speckle (a = 0) */
static double spk_a(const og_config *g, double tau_s) { return 1.0 / (g->prf * tau_s); }

static double *speckle_table(const og_config *g, long long nf, const uint32_t *ids,
                             double tau_s, uint64_t seed, int p0, int np) {
    double *xs = (double *)malloc(sizeof(double) * 2 * (size_t)nf * (size_t)np);
    const double a = spk_a(g, tau_s);
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < nf; ++i)
        og_speckle_series(seed, ids[i], a, p0, p0 + np, xs + 2 * (size_t)i * (size_t)np);
    return xs;
}

/* og_forward with the intra-facet speckle of eq. 7: facet i uses counter id
 * ids[i] and intra-facet Doppler fs[i] (Hz; NULL = 0). */
void og_forward_speckle(const og_config *g, long long nf, const double *x, const double *y,
                        const double *z, const double *vx, const double *vy,
                        const double *vz, const double *are, const double *aim,
                        const uint32_t *ids, const double *fs, double tau_s, uint64_t seed,
                        int p0, int np, double *iq) {
    double *xs = speckle_table(g, nf, ids, tau_s, seed, p0, np);
    forward_impl(g, nf, x, y, z, vx, vy, vz, are, aim, xs, fs, p0, np, iq);
    free(xs);
}

/* og_adjoint of og_forward_speckle (the speckle is a fixed factor). */
void og_adjoint_speckle(const og_config *g, long long nf, const double *x, const double *y,
                        const double *z, const double *vx, const double *vy,
                        const double *vz, const double *are, const double *aim,
                        const uint32_t *ids, const double *fs, double tau_s, uint64_t seed,
                        int p0, int np, const double *giq, double *dz, double *dvx,
                        double *dvy, double *dvz, double *dare, double *daim) {
    double *xs = speckle_table(g, nf, ids, tau_s, seed, p0, np);
    adjoint_impl(g, nf, x, y, z, vx, vy, vz, are, aim, xs, fs, p0, np, giq, dz, dvx, dvy,
                 dvz, dare, daim);
    free(xs);
}
