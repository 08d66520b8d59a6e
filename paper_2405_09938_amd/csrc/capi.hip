// C ABI of the facet-sum library: argument validation, FP64 host-side
// geometry, the interpolator's polynomial form, the waveform spectrum, the
// facet-set plan (range-binned block sort), and the stream-ordered launches.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sim_internal.h"

// Forward-kernel tuning: smallest LDS range window (samples) and the number
// of work units (strip segments x pulse groups x channels) a launch aims at.
#ifndef HEEPS_WIN_MIN
#define HEEPS_WIN_MIN 24
#endif
#ifndef HEEPS_EL_CONST_TOL
#define HEEPS_EL_CONST_TOL 5e-6
#endif
#ifndef HEEPS_TARGET_UNITS
#define HEEPS_TARGET_UNITS 16384
#endif
// narrowest strips (samples) a band may take to use a narrower window than
// the plan's widest
#ifndef HEEPS_NARROW_S_MIN
#define HEEPS_NARROW_S_MIN 1.0
#endif
// longest segment (blocks): bounds the facet records a work unit streams
#ifndef HEEPS_SEG_MAX_BLOCKS
#define HEEPS_SEG_MAX_BLOCKS 4096
#endif

namespace {

thread_local std::string g_last_error;

constexpr double kPi = 3.14159265358979323846;

#define HS_FAIL(code, msg)          \
    do {                            \
        hs::set_error(msg);         \
        return (code);              \
    } while (0)

#define HS_HIP(call, what)                                                              \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            HS_FAIL(SIM_EHIP, std::string(what) + ": " + hipGetErrorString(e_));        \
    } while (0)

bool finite3(const double *v) {
    return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

double norm3(const double *v) { return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

double sinc(double x) {
    const double px = kPi * x;
    // below 1e-4 the two-term Taylor form is exact in double precision
    if (std::fabs(px) < 1e-4) return 1.0 - px * px / 6.0;
    return std::sin(px) / px;
}

// Modified Bessel function I0 from its integral form, the mean of
// exp(x cos t) over a period: the integrand is smooth and periodic, so the
// trapezoidal rule on 64 equal steps converges geometrically (the error
// terms are I_64(x) and beyond, far below double precision for |x| <= 20).
double bessel_i0(double x) {
    constexpr int n = 64;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += std::exp(x * std::cos(2.0 * kPi * k / n));
    return s / n;
}

// The interpolator h(t) = sinc(t) I0(beta sqrt(1 - (t/4)^2)) / I0(beta),
// zero for |t| > 4: a Kaiser window of half-width 4 over the sinc.
double kaiser_sinc(double t, double beta, double i0b) {
    const double r = 0.25 * t;
    return (r * r <= 1.0) ? sinc(t) * bessel_i0(beta * std::sqrt(1.0 - r * r)) / i0b : 0.0;
}

// Least-squares fit of a degree-3 polynomial in y to samples (y_i, v_i).
void fit3(const std::vector<double> &ys, const std::vector<double> &vs, double c[4]) {
    double A[4][5] = {};
    for (size_t i = 0; i < ys.size(); ++i) {
        double p[4] = {1.0, ys[i], ys[i] * ys[i], ys[i] * ys[i] * ys[i]};
        for (int r = 0; r < 4; ++r) {
            for (int k = 0; k < 4; ++k) A[r][k] += p[r] * p[k];
            A[r][4] += p[r] * vs[i];
        }
    }
    // Gaussian elimination with partial pivoting
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        for (int r = col + 1; r < 4; ++r)
            if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
        if (piv != col)
            for (int k = 0; k < 5; ++k) std::swap(A[col][k], A[piv][k]);
        for (int r = col + 1; r < 4; ++r) {
            const double f = A[r][col] / A[col][col];
            for (int k = col; k < 5; ++k) A[r][k] -= f * A[col][k];
        }
    }
    for (int r = 3; r >= 0; --r) {
        double s = A[r][4];
        for (int k = r + 1; k < 4; ++k) s -= A[r][k] * c[k];
        c[r] = s / A[r][r];
    }
}

double poly3d(const double c[4], double y) { return c[0] + y * (c[1] + y * (c[2] + y * c[3])); }

// Polynomial form of the 8 taps (see TapPoly); returns the max abs error of
// the fitted taps on a dense grid of f.
double fit_taps(double beta, hs::TapPoly &tp) {
    const double i0b = bessel_i0(beta);
    const int K = 256;
    double e[4][4], o[4][4];
    for (int j = 0; j < 4; ++j) {
        const double J = j + 1;
        std::vector<double> ys, ev, ov;
        for (int i = 0; i < K; ++i) {
            const double sg = std::cos(kPi * (i + 0.5) / (2.0 * K));   // in (0, 1)
            const double qp = kaiser_sinc(J - 0.5 - 0.5 * sg, beta, i0b);
            const double qm = kaiser_sinc(J - 0.5 + 0.5 * sg, beta, i0b);
            ys.push_back(sg * sg);
            ev.push_back(0.5 * (qp + qm));
            ov.push_back(0.5 * (qp - qm) / sg);
        }
        fit3(ys, ev, e[j]);
        fit3(ys, ov, o[j]);
        for (int k = 0; k < 4; ++k) {
            tp.e[j][k] = (float)e[j][k];
            tp.o[j][k] = (float)o[j][k];
        }
    }
    double err = 0.0;
    for (int i = 0; i <= 2000; ++i) {
        const double f = std::min(i / 2000.0, 1.0 - 1e-12);
        const double sg = 2.0 * f - 1.0, y = sg * sg;
        for (int j = 0; j < 4; ++j) {
            const double J = j + 1;
            const double ep = poly3d(e[j], y), op = sg * poly3d(o[j], y);
            err = std::max(err, std::fabs(ep + op - kaiser_sinc(J - f, beta, i0b)));
            err = std::max(err, std::fabs(ep - op - kaiser_sinc(1.0 - J - f, beta, i0b)));
        }
    }
    return err;
}

// kappa with sinc(kappa / 2)^2 = 1/2: Newton's method on
// sinc(x) - 1/sqrt(2), whose root lies near 0.443 (sinc decreases there),
// with d sinc / dx = (cos(pi x) - sinc(x)) / x; kappa = 2 x.
double half_power_kappa() {
    const double target = std::sqrt(0.5);
    double x = 0.45;
    for (int i = 0; i < 50; ++i) {
        const double sx = sinc(x);
        const double dx = (sx - target) / ((std::cos(kPi * x) - sx) / x);
        x -= dx;
        if (std::fabs(dx) < 1e-17) break;
    }
    return 2.0 * x;
}

void plat_pos(const sim_handle *h, int plat, double t, double *out) {
    const sim_traj &p = h->plats[plat];
    for (int k = 0; k < 3; ++k) out[k] = p.p0[k] + p.v[k] * t;
}

void tx_pos(const sim_handle *h, int ch, double t, double *out) {
    plat_pos(h, h->ants[h->chans[ch].tx_antenna].platform, t, out);
}

void rx_pos(const sim_handle *h, int ch, double t, double *out) {
    plat_pos(h, h->ants[h->chans[ch].rx_antenna].platform, t, out);
    for (int k = 0; k < 3; ++k) out[k] += h->chans[ch].pc_offset[k];
}

// Stripmap antenna frame pointing at O from the platform position at t = 0.
void antenna_frame(const sim_handle *h, int a, hs::AntArgs &ac) {
    double p[3];
    plat_pos(h, h->ants[a].platform, 0.0, p);
    const double r = norm3(p);
    for (int k = 0; k < 3; ++k) ac.b[k] = -p[k] / r;
    const double d = ac.b[0];   // x . b
    double az[3] = {1.0 - d * ac.b[0], -d * ac.b[1], -d * ac.b[2]};
    const double na = norm3(az);
    for (int k = 0; k < 3; ++k) ac.az[k] = az[k] / na;
    ac.el[0] = ac.b[1] * ac.az[2] - ac.b[2] * ac.az[1];
    ac.el[1] = ac.b[2] * ac.az[0] - ac.b[0] * ac.az[2];
    ac.el[2] = ac.b[0] * ac.az[1] - ac.b[1] * ac.az[0];
    ac.ka = h->kappa / h->ants[a].beta_az;
    ac.ke = h->kappa / h->ants[a].beta_el;
    ac.steer = h->ants[a].steer_rate;
    for (int k = 0; k < 3; ++k) {
        ac.kaz[k] = (float)(0.5 * ac.ka * ac.az[k]);
        ac.kel[k] = (float)(0.5 * ac.ke * ac.el[k]);
        ac.b32[k] = (float)ac.b[k];
        ac.kb[k] = (float)(0.5 * ac.ka * ac.b[k]);
        ac.az32[k] = (float)ac.az[k];
    }
    ac.pad = 0.0f;
    const sim_antenna &an = h->ants[a];
    ac.grid = nullptr;   // device cells, set when the tables are uploaded
    ac.gidu = ac.gidv = 0.0;
    ac.gu0 = ac.gv0 = ac.gnu1 = ac.gnv1 = 0.0f;
    ac.gstride = 0;
    ac.pad2 = 0;
    if (an.pattern) {
        // direction cosines in cell units: the scaled axes become axis / du
        ac.gidu = 1.0 / an.pattern_du;
        ac.gidv = 1.0 / an.pattern_dv;
        ac.ka = 2.0 * ac.gidu;
        ac.ke = 2.0 * ac.gidv;
        for (int k = 0; k < 3; ++k) {
            ac.kaz[k] = (float)(ac.az[k] * ac.gidu);
            ac.kel[k] = (float)(ac.el[k] * ac.gidv);
            ac.kb[k] = (float)(ac.b[k] * ac.gidu);
        }
        ac.gu0 = (float)(an.pattern_u0 * ac.gidu);
        ac.gv0 = (float)(an.pattern_v0 * ac.gidv);
        ac.gnu1 = (float)(an.pattern_nu - 1);
        ac.gnv1 = (float)(an.pattern_nv - 1);
        ac.gstride = an.pattern_nu - 1;
    }
}

template <typename T>
hipError_t dalloc(T **p, size_t count) {
    return hipMalloc((void **)p, sizeof(T) * (count > 0 ? count : 1));
}

// Bound on the relative error of taking each antenna's elevation pattern
// factor sinc(kappa v / beta_el) at the block centre instead of per facet.
// Over the scene rectangle (z = 0) and the first, middle and last pulses,
// x = kappa v / beta_el spans [x_lo, x_hi] and the range is at least R_min;
// a facet within e_max of its block centre moves x by at most
// dx = (kappa / beta_el) e_max / R_min.  The first-order error is then at
// most dx max|sinc'| / min sinc over [x_lo - dx, x_hi + dx], plus the
// second-order term dx^2 max|sinc''| / 2 / min sinc (|sinc''| <= pi^2 / 3).
// Returns +inf when the interval reaches |x| >= 0.9 (near the first null).
// An antenna with a u-v table is bounded through its nominal elevation width
// (the sinc of that width stands for its beam; the bound then only decides
// whether the adjoint drops its first-order gain-gradient correction).
double elevation_bound(const sim_handle *h, const double box[4], double e_max) {
    double worst = 0.0;
    const double xs[3] = {box[0], 0.5 * (box[0] + box[1]), box[1]};
    const double ys[3] = {box[2], 0.5 * (box[2] + box[3]), box[3]};
    const int ps[3] = {0, h->Np / 2, h->Np - 1};
    for (int ch = 0; ch < h->C; ++ch)
        for (int leg = 0; leg < 2; ++leg) {
            const int ai = leg == 0 ? h->chc[ch].tx : h->chc[ch].rx;
            const hs::AntArgs &a = h->antc[ai];
            const double ke = h->kappa / h->ants[ai].beta_el;   // the sinc's, grid or not
            double x_lo = 1e300, x_hi = -1e300, r_min = 1e300;
            for (int pi = 0; pi < 3; ++pi) {
                const hs::PulseRec &r = h->pulses_h[(size_t)ch * h->Np + ps[pi]];
                const double *P = leg == 0 ? r.ptx : r.prx;
                for (double xv : xs)
                    for (double yv : ys) {
                        const double d[3] = {xv - P[0], yv - P[1], -P[2]};
                        const double R = norm3(d);
                        const double x = ke * (d[0] * a.el[0] + d[1] * a.el[1] + d[2] * a.el[2]) / R;
                        x_lo = std::min(x_lo, x);
                        x_hi = std::max(x_hi, x);
                        r_min = std::min(r_min, R);
                    }
            }
            const double dx = ke * e_max / r_min;
            const double lo = x_lo - dx - 0.1 * (x_hi - x_lo), hi = x_hi + dx + 0.1 * (x_hi - x_lo);
            if (std::max(std::fabs(lo), std::fabs(hi)) >= 0.9)
                return std::numeric_limits<double>::infinity();
            double max_d = 0.0, min_f = 1.0;
            for (int k = 0; k <= 2000; ++k) {
                const double x = lo + (hi - lo) * k / 2000.0;
                const double px = M_PI * x;
                const double f = std::fabs(px) < 1e-8 ? 1.0 : std::sin(px) / px;
                const double df = std::fabs(x) < 1e-8 ? 0.0 : (std::cos(px) - f) / x;
                max_d = std::max(max_d, std::fabs(df));
                min_f = std::min(min_f, f);
            }
            // |sinc''| <= pi^2 / 3 bounds how much sinc' moves between samples
            max_d += M_PI * M_PI / 3.0 * (hi - lo) / 2000.0;
            const double b = (dx * max_d + 0.5 * dx * dx * M_PI * M_PI / 3.0) / min_f;
            worst = std::max(worst, b);
        }
    return worst;
}

void release_handle(sim_handle *h) {
    if (h->pulses_d) (void)hipFree(h->pulses_d);
    if (h->chirp_spec_d) (void)hipFree(h->chirp_spec_d);
    if (h->twiddle_d) (void)hipFree(h->twiddle_d);
    for (float4 *p : h->pat_d)
        if (p) (void)hipFree(p);
    delete h;
}

// Scratch of sim_stream_forward_noalloc: a fixed device array, one copy per
// GPU, held until the process ends.  Host code never passes its name to a
// kernel or a copy (on the host the name stands for no device address): its
// address on each device comes from hipGetSymbolAddress, taken once per
// device by the set-up of the first handle initialised there.
static __device__ __align__(256) unsigned char scratch[SIM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on the current device d (set-up: called with d current).
int scratch_setup(int d) {
    if (d < 0 || d >= kMaxDevices) HS_FAIL(SIM_EUNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[d]) return SIM_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        HS_FAIL(SIM_EHIP, std::string("scratch address: ") + hipGetErrorString(e));
    g_scratch_ptr[d] = ptr;
    return SIM_OK;
}

void *scratch_on(int d) {
    if (d < 0 || d >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[d];
}

// Device tables are uploaded on the first call that needs the GPU, on the
// device current at that time; later calls must run on the same device.
int ensure_device(sim_handle *h) {
    int d = -1;
    if (hipGetDevice(&d) != hipSuccess) HS_FAIL(SIM_EHIP, "no HIP device");
    if (h->uploaded) {
        if (d != h->device)
            HS_FAIL(SIM_EINVAL, "current HIP device differs from the handle's device");
        return SIM_OK;
    }
    h->device = d;
    hipError_t e = dalloc(&h->pulses_d, h->pulses_h.size());
    if (e == hipSuccess)
        e = hipMemcpy(h->pulses_d, h->pulses_h.data(), sizeof(hs::PulseRec) * h->pulses_h.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && h->fft_len > 0) {
        e = dalloc(&h->chirp_spec_d, h->spec_h.size());
        if (e == hipSuccess)
            e = hipMemcpy(h->chirp_spec_d, h->spec_h.data(), sizeof(float) * h->spec_h.size(),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess) e = dalloc(&h->twiddle_d, h->tw_h.size());
        if (e == hipSuccess)
            e = hipMemcpy(h->twiddle_d, h->tw_h.data(), sizeof(float) * h->tw_h.size(),
                          hipMemcpyHostToDevice);
    }
    // gridded patterns as cells of four corners (one 16-byte load per lookup)
    for (size_t a = 0; a < h->ants.size() && e == hipSuccess; ++a) {
        const sim_antenna &an = h->ants[a];
        if (!an.pattern) continue;
        const int nu = an.pattern_nu, nv = an.pattern_nv;
        std::vector<float4> cells((size_t)(nu - 1) * (size_t)(nv - 1));
        const float *g = h->pat_h[a].data();
        for (int j = 0; j + 1 < nv; ++j)
            for (int i = 0; i + 1 < nu; ++i) {
                const float *r0 = g + (size_t)j * nu + i, *r1 = r0 + nu;
                cells[(size_t)j * (nu - 1) + i] = make_float4(r0[0], r0[1], r1[0], r1[1]);
            }
        e = dalloc(&h->pat_d[a], cells.size());
        if (e == hipSuccess)
            e = hipMemcpy(h->pat_d[a], cells.data(), sizeof(float4) * cells.size(),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess) h->antc[a].grid = h->pat_d[a];
    }
    if (e != hipSuccess) {
        HS_FAIL(e == hipErrorOutOfMemory ? SIM_ENOMEM : SIM_EHIP,
                std::string("device table upload: ") + hipGetErrorString(e));
    }
    if (int rc = scratch_setup(d)) return rc;
    h->uploaded = true;
    return SIM_OK;
}

int facets_ok(const sim_facets *f, long long n) {
    if (!f) HS_FAIL(SIM_EINVAL, "facets is NULL");
    if (f->n != n) HS_FAIL(SIM_EINVAL, "facets->n differs from the plan's facet count");
    if (!f->x || !f->y || !f->z || !f->vx || !f->vy || !f->vz || !f->a_re || !f->a_im)
        HS_FAIL(SIM_EINVAL, "a facet array pointer is NULL");
    return SIM_OK;
}

}  // namespace

namespace hs {
void set_error(const std::string &msg) { g_last_error = msg; }
}  // namespace hs

extern "C" {

const char *sim_last_error(void) { return g_last_error.c_str(); }

int sim_create(const sim_config *cfg, sim_handle **out) {
    if (!cfg || !out) HS_FAIL(SIM_EINVAL, "cfg or out is NULL");
    *out = nullptr;
    const double c = cfg->c > 0 ? cfg->c : 299792458.0;
    if (!(cfg->f0 > 0) || !(cfg->fs > 0) || !(cfg->prf > 0) || !std::isfinite(cfg->f0) ||
        !std::isfinite(cfg->fs) || !std::isfinite(cfg->prf) || !std::isfinite(c))
        HS_FAIL(SIM_EINVAL, "f0, fs, prf and c must be finite and positive");
    if (cfg->n_samples < 2 || cfg->n_samples > 65536)
        HS_FAIL(SIM_EINVAL, "n_samples must be in [2, 65536]");
    if (cfg->n_pulses < 1 || cfg->n_pulses > (1 << 24))
        HS_FAIL(SIM_EINVAL, "n_pulses must be in [1, 2^24]");
    if (!(cfg->kaiser_beta >= 0) || cfg->kaiser_beta > 20)
        HS_FAIL(SIM_EINVAL, "kaiser_beta must be in [0, 20]");
    if (cfg->n_ref >= cfg->n_samples) HS_FAIL(SIM_EINVAL, "n_ref must be < n_samples");
    if (!(cfg->chirp_T >= 0) || !std::isfinite(cfg->chirp_T) || !std::isfinite(cfg->chirp_bw))
        HS_FAIL(SIM_EINVAL, "chirp_T must be >= 0 and finite");
    if (cfg->n_platforms < 1 || cfg->n_platforms > SIM_MAX_PLATFORMS || !cfg->platforms)
        HS_FAIL(SIM_EINVAL, "need 1..8 platforms");
    if (cfg->n_antennas < 1 || cfg->n_antennas > SIM_MAX_ANTENNAS || !cfg->antennas)
        HS_FAIL(SIM_EINVAL, "need 1..8 antennas");
    if (cfg->n_channels < 1 || cfg->n_channels > SIM_MAX_CHANNELS || !cfg->channels)
        HS_FAIL(SIM_EINVAL, "need 1..16 channels");
    for (int i = 0; i < cfg->n_platforms; ++i)
        if (!finite3(cfg->platforms[i].p0) || !finite3(cfg->platforms[i].v))
            HS_FAIL(SIM_EINVAL, "platform trajectory is not finite");
    for (int i = 0; i < cfg->n_antennas; ++i) {
        const sim_antenna &a = cfg->antennas[i];
        if (a.platform < 0 || a.platform >= cfg->n_platforms)
            HS_FAIL(SIM_EINVAL, "antenna platform index out of range");
        if (!(a.beta_az > 0) || !(a.beta_el > 0) || !std::isfinite(a.beta_az) ||
            !std::isfinite(a.beta_el))
            HS_FAIL(SIM_EINVAL, "antenna widths must be finite and positive");
        double p[3];
        for (int k = 0; k < 3; ++k) p[k] = cfg->platforms[a.platform].p0[k];
        const double r = norm3(p);
        if (!(r > 0)) HS_FAIL(SIM_EINVAL, "an antenna's platform sits on the scene origin");
        if (std::fabs(p[0]) / r > 1.0 - 1e-9)
            HS_FAIL(SIM_EINVAL, "boresight parallel to the along-track axis");
        if (a.pattern) {
            if (a.pattern_nu < 2 || a.pattern_nv < 2 ||
                (long long)(a.pattern_nu - 1) * (a.pattern_nv - 1) > (1LL << 24))
                HS_FAIL(SIM_EINVAL, "pattern grid needs 2..(2^24 cells) nodes per axis");
            if (!(a.pattern_du > 0) || !(a.pattern_dv > 0) || !std::isfinite(a.pattern_du) ||
                !std::isfinite(a.pattern_dv) || !std::isfinite(a.pattern_u0) ||
                !std::isfinite(a.pattern_v0))
                HS_FAIL(SIM_EINVAL, "pattern grid origin and steps must be finite, steps > 0");
            // cell coordinates u/du - u0/du are FP32: at most 2^14 cells from
            // u = 0 anywhere on the table keeps their rounding below 1e-3 cell
            const double ue = a.pattern_u0 + (a.pattern_nu - 1) * a.pattern_du;
            const double ve = a.pattern_v0 + (a.pattern_nv - 1) * a.pattern_dv;
            if (std::max(std::fabs(a.pattern_u0), std::fabs(ue)) > 16384.0 * a.pattern_du ||
                std::max(std::fabs(a.pattern_v0), std::fabs(ve)) > 16384.0 * a.pattern_dv)
                HS_FAIL(SIM_EUNSUPPORTED, "pattern grid reaches more than 2^14 cells from u, v = 0");
            const long long nn = (long long)a.pattern_nu * a.pattern_nv;
            for (long long k = 0; k < nn; ++k)
                if (!std::isfinite(a.pattern[k]))
                    HS_FAIL(SIM_EINVAL, "pattern values must be finite");
        }
    }
    for (int i = 0; i < cfg->n_channels; ++i) {
        const sim_channel &ch = cfg->channels[i];
        if (ch.tx_antenna < 0 || ch.tx_antenna >= cfg->n_antennas || ch.rx_antenna < 0 ||
            ch.rx_antenna >= cfg->n_antennas)
            HS_FAIL(SIM_EINVAL, "channel antenna index out of range");
        if (!finite3(ch.pc_offset)) HS_FAIL(SIM_EINVAL, "phase-centre offset is not finite");
    }

    sim_handle *h = new (std::nothrow) sim_handle();
    if (!h) HS_FAIL(SIM_ENOMEM, "host allocation failed");
    h->c = c;
    h->f0 = cfg->f0;
    h->fs = cfg->fs;
    h->prf = cfg->prf;
    h->N = cfg->n_samples;
    h->Np = cfg->n_pulses;
    h->n_ref = cfg->n_ref < 0 ? cfg->n_samples / 2 : cfg->n_ref;
    h->beta = cfg->kaiser_beta;
    h->chirp_bw = cfg->chirp_bw;
    h->chirp_T = cfg->chirp_T;
    h->plats.assign(cfg->platforms, cfg->platforms + cfg->n_platforms);
    h->ants.assign(cfg->antennas, cfg->antennas + cfg->n_antennas);
    h->chans.assign(cfg->channels, cfg->channels + cfg->n_channels);
    h->C = cfg->n_channels;
    h->rx_exact = cfg->rx_exact ? 1 : 0;
    h->kappa = half_power_kappa();

    h->steer = 0;
    for (const sim_antenna &an : h->ants) {
        if (!std::isfinite(an.steer_rate)) {
            delete h;
            HS_FAIL(SIM_EINVAL, "antenna steer_rate must be finite");
        }
        if (an.steer_rate != 0.0) h->steer = 1;
    }
    h->pat_h.resize(h->ants.size());
    h->pat_d.assign(h->ants.size(), nullptr);
    size_t n_grid = 0;
    for (size_t a = 0; a < h->ants.size(); ++a) {
        sim_antenna &an = h->ants[a];
        if (an.pattern) {
            h->pat_h[a].assign(an.pattern,
                               an.pattern + (size_t)an.pattern_nu * (size_t)an.pattern_nv);
            an.pattern = h->pat_h[a].data();   // the caller's array is not kept
            ++n_grid;
        }
    }
    h->grid = n_grid == 0 ? 0 : (n_grid == h->ants.size() ? 2 : 1);
    h->antc.resize(h->ants.size());
    for (size_t a = 0; a < h->ants.size(); ++a) {
        antenna_frame(h, (int)a, h->antc[a]);
        if (!h->ants[a].pattern && (h->antc[a].ka > 500.0 || h->antc[a].ke > 500.0)) {
            delete h;
            HS_FAIL(SIM_EUNSUPPORTED, "antenna 3-dB width below kappa/500 rad is not supported");
        }
    }
    h->chc.resize(h->C);
    for (int ch = 0; ch < h->C; ++ch) {
        hs::ChanArgs &cc = h->chc[ch];
        cc.tx = h->chans[ch].tx_antenna;
        cc.rx = h->chans[ch].rx_antenna;
        double pt[3], pr[3];
        tx_pos(h, ch, 0.0, pt);
        rx_pos(h, ch, 0.0, pr);
        cc.rtrr_mid = norm3(pt) * norm3(pr);
        const sim_traj &rt = h->plats[h->ants[cc.rx].platform];
        for (int k = 0; k < 3; ++k) cc.vr[k] = rt.v[k];
    }
    // per (channel, pulse) geometry: echo delay of O by fixed-point iteration
    h->pulses_h.resize((size_t)h->C * h->Np);
    for (int ch = 0; ch < h->C; ++ch) {
        for (int p = 0; p < h->Np; ++p) {
            hs::PulseRec &r = h->pulses_h[(size_t)ch * h->Np + p];
            r.t = ((double)p - 0.5 * (double)(h->Np - 1)) / h->prf;
            tx_pos(h, ch, r.t, r.ptx);
            const double rt = norm3(r.ptx);
            double tau = 2.0 * rt / c;
            for (int it = 0; it < 60; ++it) {
                rx_pos(h, ch, r.t + tau, r.prx);
                const double nt = (rt + norm3(r.prx)) / c;
                if (nt == tau) break;
                tau = nt;
            }
            rx_pos(h, ch, r.t + tau, r.prx);
            r.rref = c * tau;
            // steering angles (time-dependent antenna frames)
            const double at = h->ants[h->chans[ch].tx_antenna].steer_rate * r.t;
            const double ar = h->ants[h->chans[ch].rx_antenna].steer_rate * (r.t + tau);
            r.cst = std::cos(at);
            r.snt = std::sin(at);
            r.csr = std::cos(ar);
            r.snr = std::sin(ar);
            if (!std::isfinite(r.rref) || !(rt > 0)) {
                delete h;
                HS_FAIL(SIM_EINVAL, "pulse geometry is not finite");
            }
        }
    }
    h->tap_fit_err = fit_taps(h->beta, h->tp);

    // waveform spectrum S = FFT_M(chirp) / M and twiddles, FP64 on the host
    h->chirp_len = 0;
    h->fft_len = 0;
    std::vector<float> &spec = h->spec_h, &tw = h->tw_h;
    if (h->chirp_T > 0) {
        const long long L = std::llround(h->chirp_T * h->fs);
        if (L < 1) {
            delete h;
            HS_FAIL(SIM_EINVAL, "chirp shorter than one sample");
        }
        long long M = 256;
        while (M < (long long)h->N + L - 1) M <<= 1;
        h->chirp_len = (int)L;
        if (M <= 16384) {
            h->fft_len = (int)M;
            std::vector<double> wr(M), wi(M);
            for (long long m = 0; m < M; ++m) {
                const double a = -2.0 * kPi * (double)m / (double)M;
                wr[m] = std::cos(a);
                wi[m] = std::sin(a);
            }
            const double K = h->chirp_bw / h->chirp_T;
            std::vector<double> cr(L), ci(L);
            for (long long k = 0; k < L; ++k) {
                const double t = (double)k / h->fs - 0.5 * h->chirp_T;
                const double ph = kPi * K * t * t;
                cr[k] = std::cos(ph);
                ci[k] = std::sin(ph);
            }
            spec.resize(2 * M);
            tw.resize(2 * M);
            for (long long m = 0; m < M; ++m) {
                double sr = 0.0, si = 0.0;
                for (long long k = 0; k < L; ++k) {
                    const long long q = (m * k) % M;
                    sr += cr[k] * wr[q] - ci[k] * wi[q];
                    si += cr[k] * wi[q] + ci[k] * wr[q];
                }
                spec[2 * m] = (float)(sr / (double)M);
                spec[2 * m + 1] = (float)(si / (double)M);
                tw[2 * m] = (float)wr[m];
                tw[2 * m + 1] = (float)wi[m];
            }
        }
    }

    *out = h;
    return SIM_OK;
}

void sim_destroy(sim_handle *h) {
    if (!h) return;
    release_handle(h);
}

int sim_pulse_info(const sim_handle *h, int ch, int p0, int np, double *t, double *tau_ref) {
    if (!h) HS_FAIL(SIM_EINVAL, "handle is NULL");
    if (ch < 0 || ch >= h->C) HS_FAIL(SIM_EINVAL, "channel out of range");
    if (p0 < 0 || np < 0 || (long long)p0 + np > h->Np) HS_FAIL(SIM_EINVAL, "pulse range");
    for (int i = 0; i < np; ++i) {
        const hs::PulseRec &r = h->pulses_h[(size_t)ch * h->Np + p0 + i];
        if (t) t[i] = r.t;
        if (tau_ref) tau_ref[i] = r.rref / h->c;
    }
    return SIM_OK;
}

int sim_waveform_info(const sim_handle *h, int *chirp_len, int *fft_len) {
    if (!h) HS_FAIL(SIM_EINVAL, "handle is NULL");
    if (chirp_len) *chirp_len = h->chirp_len;
    if (fft_len) *fft_len = h->fft_len;
    return SIM_OK;
}

// ---- plan (range-binned block sort) in a caller-owned workspace ------------

// Host-side shape of a plan: the block lattice over the scene rectangle, the
// range strips of every band and channel, the window of the forward kernel,
// the elevation-factor mode, and the sizes the workspace must hold.
struct PlanGeom {
    hs::Lattice L;
    long long n_keys, nb_max;
    int win;
    int NB, B, NS, L_seg, seg_max, ng_max;
    int ng_slots;                // pulse groups the window slots hold (<= ng_max)
    int win_mask;                // window widths the bands use (hs::win_bit)
    std::vector<double> band;    // [NB][C][3]: umin, S, margin
    double el_bound;
    bool el_const;
    double zlim, vlim;           // bounds on |z| and |V| (the box's or the defaults)
};

static int box_ok(const sim_box *box) {
    if (!box) HS_FAIL(SIM_EINVAL, "box is NULL");
    if (!std::isfinite(box->x_min) || !std::isfinite(box->x_max) || !std::isfinite(box->y_min) ||
        !std::isfinite(box->y_max) || !(box->x_min <= box->x_max) || !(box->y_min <= box->y_max))
        HS_FAIL(SIM_EINVAL, "box must be finite with x_min <= x_max and y_min <= y_max");
    if (!(box->z_max >= 0) || !(box->v_max >= 0) || !std::isfinite(box->z_max) ||
        !std::isfinite(box->v_max))
        HS_FAIL(SIM_EINVAL, "box z_max and v_max must be finite and >= 0");
    return SIM_OK;
}

// The plan's bounds on |z| (m) and |V| (m/s): the box's, or the defaults.
static double z_limit(const sim_box *box) { return box->z_max > 0 ? box->z_max : 4.0; }
static double v_limit(const sim_box *box) { return box->v_max > 0 ? box->v_max : 2.5; }

// Sample position u = n_ref + (|X - P_tx| + |X - P_rx| - c tau_ref) fs / c of
// the point (x, y, 0) at pulse p of channel ch, and the bistatic range
// gradient there (unit vectors from the antennas to the point, summed).
static double sample_pos(const sim_handle *h, int ch, int p, double x, double y, double *g) {
    const hs::PulseRec &r = h->pulses_h[(size_t)ch * h->Np + p];
    const double dt[3] = {x - r.ptx[0], y - r.ptx[1], -r.ptx[2]};
    const double dr[3] = {x - r.prx[0], y - r.prx[1], -r.prx[2]};
    const double nt = norm3(dt), nr = norm3(dr);
    if (g)
        for (int k = 0; k < 3; ++k) g[k] = dt[k] / nt + dr[k] / nr;
    return (double)h->n_ref + (nt + nr - r.rref) * h->fs / h->c;
}

// Range strips of the forward sum.  Bands of B pulse groups; per band and
// channel, over a 17 x 17 grid of the lattice's block centres (z = 0):
// umin, umax of the centres' sample positions at the band's reference pulse
// (plus a curvature slack of 0.05 sample, far above the grid's error of
// ~1e-3 for ranges of tens of km and spacings up to km); the migration M,
// the largest |u(p) - u(p_ref)| over the band's pulses widened by half a
// group on each side (a call's groups need not start on a group boundary:
// a unit takes the band of its group's centre pulse, so its 64 lanes reach
// at most 32 pulses before the band and 31 after it);
// the halo of facet heights (up to the plan's z bound, 4 m by default) and
// drift (its speed bound, 2.5 m/s by default, over the band's largest |t|)
// along the range gradient; E, half a block diagonal along its
// horizontal part.  margin = M + halo + E + 0.5, and the strip width
// S = W - 2 margin - 9 keeps every tap of the strip's facets inside a window
// of W samples.  W (the widest window of the plan) is the smallest
// instantiated width for which some band length leaves S >= 4 in every
// band; each band then takes its own narrowest width (strip_geometry).
struct BandStats {
    std::vector<double> umin, umax, margin;   // [NB][C]
};

static void band_stats(const sim_handle *h, const hs::Lattice &L, int B, int NB, double zlim,
                       double vlim, BandStats &bs) {
    const int K = 17;
    const double x0 = ((double)L.bx0 + 0.5) * L.edge, x1 = ((double)(L.bx0 + L.nbx) - 0.5) * L.edge;
    const double y0 = ((double)L.by0 + 0.5) * L.edge, y1 = ((double)(L.by0 + L.nby) - 0.5) * L.edge;
    const double bins = h->fs / h->c;
    bs.umin.assign((size_t)NB * h->C, 0.0);
    bs.umax.assign((size_t)NB * h->C, 0.0);
    bs.margin.assign((size_t)NB * h->C, 0.0);
    for (int b = 0; b < NB; ++b) {
        const int pref = std::min(b * B * 64 + B * 32, h->Np - 1);
        const int pa = std::max(0, b * B * 64 - 32);
        const int pb = std::min(h->Np - 1, (b + 1) * B * 64 + 31);
        const int pt[5] = {pa, (3 * pa + pb) / 4, (pa + pb) / 2, (pa + 3 * pb) / 4, pb};
        for (int ch = 0; ch < h->C; ++ch) {
            double lo = 1e300, hi = -1e300, m = 0.0, gz = 0.0, gn = 0.0, gh = 0.0;
            for (int i = 0; i < K; ++i)
                for (int j = 0; j < K; ++j) {
                    const double x = x0 + (x1 - x0) * i / (K - 1), y = y0 + (y1 - y0) * j / (K - 1);
                    double g[3];
                    const double u = sample_pos(h, ch, pref, x, y, g);
                    lo = std::min(lo, u);
                    hi = std::max(hi, u);
                    gh = std::max(gh, std::hypot(g[0], g[1]));
                    for (int q = 0; q < 5; ++q) {
                        double g2[3];
                        m = std::max(m, std::fabs(sample_pos(h, ch, pt[q], x, y, g2) - u));
                        gz = std::max(gz, std::fabs(g2[2]));
                        gn = std::max(gn, norm3(g2));
                        gh = std::max(gh, std::hypot(g2[0], g2[1]));
                    }
                }
            const double ta = std::fabs(h->pulses_h[(size_t)ch * h->Np + pa].t);
            const double tb = std::fabs(h->pulses_h[(size_t)ch * h->Np + pb].t);
            const size_t k = (size_t)b * h->C + ch;
            const double halo = (zlim * gz + vlim * std::max(ta, tb) * gn) * bins;
            const double E = 0.5 * std::sqrt(2.0) * L.edge * gh * bins;
            bs.umin[k] = lo - 0.05;
            bs.umax[k] = hi + 0.05;
            bs.margin[k] = m + halo + E + 0.5;
        }
    }
}

static int strip_geometry(const sim_handle *h, PlanGeom &G) {
    const hs::Lattice &L = G.L;
    const int NG = (h->Np + 63) / 64;
    G.ng_max = NG + 1;
    G.ng_slots = G.ng_max;
    // candidate band lengths, longest first
    std::vector<int> Bs;
    for (int b = 1; b < NG; b *= 4) Bs.push_back(b);
    Bs.push_back(NG);
    std::sort(Bs.rbegin(), Bs.rend());
    const int wins[5] = {24, 26, 32, 48, 64};
    // per band and channel the narrowest window (at most wmax) leaving
    // strips of HEEPS_NARROW_S_MIN samples: bands near the middle of the
    // dwell, with little drift, take narrower windows, so more waves share a
    // compute unit (narrower strips cost more work units and window slots)
    const auto narrowest = [&](const BandStats &st, size_t k, int wmax) {
        for (int w : wins)
            if (w >= HEEPS_WIN_MIN && w < wmax &&
                w - 2.0 * st.margin[k] - 9.0 >= HEEPS_NARROW_S_MIN)
                return w;
        return wmax;
    };
    // relative cost of a band-channel by window width (measured per band
    // on the 9.6 s dwell: 32 samples 1.15x the 24-sample time; 26 samples
    // keep three workgroups of four waves per compute unit like 24; the
    // one-wave 48 and 64 estimated from their occupancy)
    const auto width_cost = [](int w) {
        return w <= 24 ? 1.0 : (w <= 26 ? 1.02 : (w <= 32 ? 1.15 : (w <= 48 ? 1.6 : 2.0)));
    };
    BandStats bs;
    bool found = false;
    // band statistics by band length, made once (they do not depend on w)
    std::vector<BandStats> stats(Bs.size());
    std::vector<bool> have(Bs.size(), false);
    for (int w : wins) {
        if (w < HEEPS_WIN_MIN) continue;
        // the band lengths leaving S >= 4 at width w; of these the one whose
        // per-band widths cost least, the longest on a tie (a strip's blocks
        // stay the same for all groups of its band, which share their facet
        // records through the L2)
        double best = 1e300;
        for (size_t bi = 0; bi < Bs.size(); ++bi) {
            const int B = Bs[bi];
            const int NB = (NG + B - 1) / B;
            if (!have[bi]) {
                band_stats(h, L, B, NB, G.zlim, G.vlim, stats[bi]);
                have[bi] = true;
            }
            const BandStats &cand = stats[bi];
            double smin = 1e300;
            for (double mg : cand.margin) smin = std::min(smin, w - 2.0 * mg - 9.0);
            if (smin < 4.0) continue;
            double cost = 0.0;
            for (size_t k = 0; k < cand.margin.size(); ++k)
                cost += width_cost(narrowest(cand, k, w));
            cost /= (double)cand.margin.size();
            if (cost < best - 1e-9) {
                best = cost;
                G.win = w;
                G.B = B;
                G.NB = NB;
                bs = cand;
                found = true;
            }
            // every band at the narrowest width: no shorter band does better
            if (best <= width_cost(std::max(24, HEEPS_WIN_MIN)) + 1e-9) break;
        }
        if (found) break;
    }
    if (!found) {   // far outside the workloads' geometries: narrowest strips
        G.win = 64;
        G.B = 1;
        G.NB = NG;
        band_stats(h, L, G.B, G.NB, G.zlim, G.vlim, bs);
    }
    G.band.assign((size_t)4 * G.NB * h->C, 0.0);
    G.NS = 1;
    G.win_mask = 0;
    for (size_t k = 0; k < bs.umin.size(); ++k) {
        const int wk = found ? narrowest(bs, k, G.win) : G.win;
        double S = std::max(1.0, wk - 2.0 * bs.margin[k] - 9.0);
        // at most kStripMax strips: wider ones (facets may then leave the
        // window and take the global path)
        S = std::max(S, (bs.umax[k] - bs.umin[k]) / 8000.0);
        G.band[4 * k] = bs.umin[k];
        G.band[4 * k + 1] = S;
        G.band[4 * k + 2] = bs.margin[k];
        G.band[4 * k + 3] = (double)wk;
        G.win_mask |= hs::win_bit(wk);
        G.NS = std::max(G.NS, (int)std::floor((bs.umax[k] - bs.umin[k]) / S) + 1);
    }
    // segments: enough work units to fill the GPU, long enough to amortise
    // the window flush
    const long long per_band = std::max(1LL, (long long)HEEPS_TARGET_UNITS / ((long long)NG * h->C));
    long long Ls = std::min((long long)HEEPS_SEG_MAX_BLOCKS,
                            std::max(16LL, (G.nb_max / 2 + per_band - 1) / per_band));
    // a multiple of every window's wave count (4 or 1)
    G.L_seg = (int)((Ls + 3) / 4 * 4);
    G.seg_max = G.NS + (int)((G.nb_max + G.L_seg - 1) / G.L_seg);
    return SIM_OK;
}

static int plan_geometry(const sim_handle *h, long long n, const sim_box *bx, double block_edge,
                         PlanGeom &G) {
    if (n < 1 || n >= (1LL << 31) - 64) HS_FAIL(SIM_EINVAL, "facet count must be in [1, 2^31 - 64)");
    if (!(block_edge > 0) || block_edge > 64) HS_FAIL(SIM_EINVAL, "block_edge must be in (0, 64]");
    if (int rc = box_ok(bx)) return rc;
    const double box[4] = {bx->x_min, bx->x_max, bx->y_min, bx->y_max};
    hs::Lattice &L = G.L;
    L.edge = block_edge;
    const double fx0 = std::floor(box[0] / block_edge), fx1 = std::floor(box[1] / block_edge);
    const double fy0 = std::floor(box[2] / block_edge), fy1 = std::floor(box[3] / block_edge);
    if (fx1 - fx0 + 1 > (double)(1 << 28) || fy1 - fy0 + 1 > (double)(1 << 28) ||
        (fx1 - fx0 + 1) * (fy1 - fy0 + 1) > (double)(1LL << 28))
        HS_FAIL(SIM_EUNSUPPORTED, "facet lattice exceeds 2^28 cells");
    L.bx0 = (long long)fx0;
    L.by0 = (long long)fy0;
    L.nbx = (int)(fx1 - fx0) + 1;
    L.nby = (int)(fy1 - fy0) + 1;

    G.n_keys = (long long)L.nbx * L.nby;
    // a cell of c facets makes ceil(c / 64) blocks: at most one per non-empty
    // cell plus one per 64 facets
    G.nb_max = std::min(n, G.n_keys) + n / 64;
    G.zlim = z_limit(bx);
    G.vlim = v_limit(bx);
    if (int rc = strip_geometry(h, G)) return rc;
    const double tmax = 0.5 * (double)(h->Np - 1) / h->prf;
    // facets lie within half a block diagonal of their block centre, moved by
    // heights up to zlim and drift at up to vlim over the dwell (as the halo)
    G.el_bound = elevation_bound(h, box, 0.5 * std::sqrt(2.0) * block_edge + G.zlim + G.vlim * tmax);
    G.el_const = G.el_bound <= HEEPS_EL_CONST_TOL;
    return SIM_OK;
}

// Byte offsets of a plan's buffers in its workspace (each 256-byte aligned).
struct PlanLayout {
    size_t perm, sorted, blocks, count, offset, nblk, blk_offset, scan_tmp, misc;
    size_t band, ids, skey, scount, soff, segoff, wsum;
    size_t spk, anch, total;
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static PlanLayout plan_layout(const PlanGeom &G, long long n, int flags, int Np) {
    PlanLayout Y{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    const size_t nk = (size_t)G.n_keys;
    Y.perm = take(sizeof(int) * (size_t)n);
    // the sort's keys and ranks (8 bytes per facet) live in the first part of
    // `sorted` until the first gather overwrites it
    Y.sorted = take(sizeof(hs::FacetRec) * ((size_t)n + 1));
    Y.blocks = take(sizeof(hs::BlockRec) * (size_t)std::max(1LL, G.nb_max));
    Y.count = take(sizeof(int) * nk);
    Y.offset = take(sizeof(int) * (nk + 1));
    Y.nblk = take(sizeof(int) * nk);
    Y.blk_offset = take(sizeof(int) * (nk + 1));
    Y.scan_tmp = take(sizeof(int) * (size_t)hs::scan_tmp_len(G.n_keys));
    Y.misc = take(256);
    const size_t bcn = G.band.size() / 4;   // bands x channels
    const size_t nbm = (size_t)std::max(1LL, G.nb_max);
    Y.band = take(sizeof(double) * G.band.size());
    Y.ids = take(sizeof(int) * bcn * nbm);
    Y.skey = take(sizeof(int) * bcn * nbm);
    Y.scount = take(sizeof(int) * bcn * ((size_t)G.NS + 1));
    Y.soff = take(sizeof(int) * bcn * ((size_t)G.NS + 1));
    Y.segoff = take(sizeof(int) * bcn * ((size_t)G.NS + 1));
    const size_t units = bcn / (size_t)G.NB * (size_t)G.ng_slots * (size_t)G.seg_max;
    Y.wsum = take(sizeof(float2) * units * 64 * (size_t)G.win);
    if (flags & SIM_PLAN_SPECKLE) {
        const size_t groups = (size_t)((Np + 63) / 64) + 1;
        Y.spk = take(sizeof(hs::SpkRec) * ((size_t)n + 1));
        Y.anch = take(sizeof(float4) * ((size_t)n + 1) * groups);
    }
    Y.total = o;
    return Y;
}

static int workspace_ok(const void *ws, size_t ws_bytes, size_t need) {
    if (!ws) HS_FAIL(SIM_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws & 255u) != 0) HS_FAIL(SIM_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
        HS_FAIL(SIM_EINVAL, "workspace too small: " + std::to_string(need) + " bytes needed, " +
                                std::to_string(ws_bytes) + " given");
    return SIM_OK;
}

// Builds the plan of facets (x, y) in the workspace `ws` (laid out by Y):
// counting sort by cell (each cell's facets then in ascending index), blocks
// of at most 64 facets, and the range strips of every band and channel.
// Everything is enqueued on s; nothing is read back.
static int plan_build(const sim_handle *h, const float *x, const float *y, long long n,
                      const PlanGeom &G, const PlanLayout &Y, int flags, char *ws, hipStream_t s,
                      sim_plan &P) {
    P.h = h;
    P.n = n;
    P.nb_max = G.nb_max;
    P.flags = flags;
    P.lat = G.L;
    P.win = G.win;
    P.el_const = G.el_const;
    P.el_bound = G.el_bound;
    P.stream = s;
    P.perm = (int *)(ws + Y.perm);
    P.sorted = (hs::FacetRec *)(ws + Y.sorted);
    P.blocks = (hs::BlockRec *)(ws + Y.blocks);
    int *count = (int *)(ws + Y.count), *offset = (int *)(ws + Y.offset);
    int *nblk = (int *)(ws + Y.nblk), *blk_offset = (int *)(ws + Y.blk_offset);
    int *scan_tmp = (int *)(ws + Y.scan_tmp);
    int *keys = (int *)(ws + Y.sorted);
    int *rank = keys + n;
    P.n_blocks = blk_offset + G.n_keys;
    P.n_outside = (unsigned *)(ws + Y.misc);
    P.counter = (unsigned *)(ws + Y.misc + 64);
    P.beyond = (unsigned *)(ws + Y.misc + 128);
    P.zlim = G.zlim;
    P.vlim = G.vlim;
    hs::StripPlan &st = P.st;
    st.band = (const double *)(ws + Y.band);
    st.ids = (int *)(ws + Y.ids);
    st.soff = (int *)(ws + Y.soff);
    st.segoff = (int *)(ws + Y.segoff);
    st.NB = G.NB;
    st.B = G.B;
    st.NS = G.NS;
    st.nbm = (int)std::max(1LL, G.nb_max);
    st.L = G.L_seg;
    st.seg_max = G.seg_max;
    P.wsum = (float2 *)(ws + Y.wsum);
    P.ng_slots = G.ng_slots;
    P.win_mask = G.win_mask;
    // sample span of any band's windows, in tiles of the window reduction
    {
        long long span = 1;
        for (size_t k = 0; k + 3 < G.band.size(); k += 4) {
            const double umin = G.band[k], S = G.band[k + 1], mg = G.band[k + 2];
            const long long lo0 = (long long)std::floor(umin - mg);
            const long long lo1 = (long long)std::floor(umin + (double)(G.NS - 1) * S - mg);
            span = std::max(span, lo1 - lo0 + (long long)G.band[k + 3]);
        }
        P.span_tiles = (int)((span + hs::kReduceTile - 1) / hs::kReduceTile);
    }
    P.spk = (flags & SIM_PLAN_SPECKLE) ? (hs::SpkRec *)(ws + Y.spk) : nullptr;
    P.anch = (flags & SIM_PLAN_SPECKLE) ? (float4 *)(ws + Y.anch) : nullptr;
    const long long stl = hs::scan_tmp_len(G.n_keys);
    const long long nk = G.n_keys;
    hipError_t e = hipSuccess;
    if ((e = hs::launch_fill_zero((float *)count, nk, s)) != hipSuccess ||
        (e = hs::launch_fill_zero((float *)P.n_outside, 64, s)) != hipSuccess ||   // misc counters
        (e = hs::launch_cell_keys(x, y, n, G.L, keys, rank, count, P.n_outside, s)) !=
            hipSuccess ||
        (e = hs::launch_exclusive_scan(count, offset, nk, scan_tmp, stl, s)) != hipSuccess ||
        (e = hs::launch_scatter(keys, rank, offset, n, P.perm, s)) != hipSuccess ||
        (e = hs::launch_fill_zero((float *)(P.sorted + n), 8, s)) != hipSuccess ||
        (e = hs::launch_block_counts(count, nk, nblk, s)) != hipSuccess ||
        (e = hs::launch_exclusive_scan(nblk, blk_offset, nk, scan_tmp, stl, s)) != hipSuccess ||
        (e = hs::launch_make_blocks(count, offset, blk_offset, nk, G.L, P.blocks, s)) !=
            hipSuccess ||
        (e = hs::launch_cell_sort(count, offset, nk, P.perm, s)) != hipSuccess ||
        (e = hs::launch_upload((double *)(ws + Y.band), G.band.data(), (long long)G.band.size(),
                               s)) != hipSuccess ||
        (e = hs::launch_strips(st, h->pulses_d, P.blocks, P.n_blocks, h->Np, h->C,
                               (double)h->n_ref, h->fs / h->c, (int *)(ws + Y.skey),
                               (int *)(ws + Y.scount), s)) != hipSuccess)
        HS_FAIL(SIM_EHIP, std::string("plan: ") + hipGetErrorString(e));
    return SIM_OK;
}

int sim_device_init(sim_handle *h) {
    if (!h) HS_FAIL(SIM_EINVAL, "handle is NULL");
    return ensure_device(h);
}

int sim_workspace_size(const sim_handle *h, long long n, const sim_box *box, double block_edge,
                       int flags, size_t *bytes) {
    if (!h || !bytes) HS_FAIL(SIM_EINVAL, "handle or bytes is NULL");
    if (flags & ~SIM_PLAN_SPECKLE) HS_FAIL(SIM_EINVAL, "unknown plan flags");
    PlanGeom G;
    if (int rc = plan_geometry(h, n, box, block_edge, G)) return rc;
    *bytes = plan_layout(G, n, flags, h->Np).total;
    return SIM_OK;
}

int sim_plan_geometry(const sim_handle *h, long long n, const sim_box *box, double block_edge,
                      int *win, int *n_bands, int *band_groups, int *n_strips, int *seg_len,
                      int *seg_max, double *bands, int *band_win) {
    if (!h) HS_FAIL(SIM_EINVAL, "handle is NULL");
    PlanGeom G;
    if (int rc = plan_geometry(h, n, box, block_edge, G)) return rc;
    if (win) *win = G.win;
    if (n_bands) *n_bands = G.NB;
    if (band_groups) *band_groups = G.B;
    if (n_strips) *n_strips = G.NS;
    if (seg_len) *seg_len = G.L_seg;
    if (seg_max) *seg_max = G.seg_max;
    for (size_t k = 0; k + 3 < G.band.size(); k += 4) {
        if (bands)
            for (int j = 0; j < 3; ++j) bands[3 * (k / 4) + j] = G.band[k + j];
        if (band_win) band_win[k / 4] = (int)G.band[k + 3];
    }
    return SIM_OK;
}

int sim_plan_create(sim_handle *h, const float *x, const float *y, long long n,
                    const sim_box *box, double block_edge, int flags, void *workspace,
                    size_t workspace_bytes, void *stream, sim_plan **out) {
    if (!h || !out) HS_FAIL(SIM_EINVAL, "handle or out is NULL");
    *out = nullptr;
    if (!x || !y) HS_FAIL(SIM_EINVAL, "x or y is NULL");
    if (flags & ~SIM_PLAN_SPECKLE) HS_FAIL(SIM_EINVAL, "unknown plan flags");
    PlanGeom G;
    if (int rc = plan_geometry(h, n, box, block_edge, G)) return rc;
    const PlanLayout Y = plan_layout(G, n, flags, h->Np);
    if (int rc = workspace_ok(workspace, workspace_bytes, Y.total)) return rc;
    if (int rc = ensure_device(h)) return rc;
    sim_plan *P = new (std::nothrow) sim_plan();
    if (!P) HS_FAIL(SIM_ENOMEM, "host allocation failed");
    if (int rc = plan_build(h, x, y, n, G, Y, flags, (char *)workspace, (hipStream_t)stream, *P)) {
        delete P;
        return rc;
    }
    *out = P;
    return SIM_OK;
}

void sim_plan_destroy(sim_plan *P) { delete P; }

int sim_plan_info(const sim_plan *P, long long *n_facets, long long *n_blocks,
                  long long *n_strips, long long *n_outside) {
    if (!P) HS_FAIL(SIM_EINVAL, "plan is NULL");
    if (n_facets) *n_facets = P->n;
    if (n_strips) *n_strips = P->st.NS;
    if (n_blocks || n_outside) {
        int nb = 0;
        unsigned no = 0;
        HS_HIP(hipMemcpyAsync(&nb, P->n_blocks, sizeof(int), hipMemcpyDeviceToHost, P->stream),
               "plan info read");
        HS_HIP(hipMemcpyAsync(&no, P->n_outside, sizeof(unsigned), hipMemcpyDeviceToHost,
                              P->stream),
               "plan info read");
        HS_HIP(hipStreamSynchronize(P->stream), "plan info sync");
        if (n_blocks) *n_blocks = nb;
        if (n_outside) *n_outside = no;
    }
    return SIM_OK;
}

int sim_plan_beyond(const sim_plan *P, void *stream, long long *n_beyond) {
    if (!P || !n_beyond) HS_FAIL(SIM_EINVAL, "plan or n_beyond is NULL");
    unsigned v = 0;
    hipStream_t s = (hipStream_t)stream;
    HS_HIP(hipMemcpyAsync(&v, P->beyond, sizeof(unsigned), hipMemcpyDeviceToHost, s),
           "plan beyond read");
    HS_HIP(hipStreamSynchronize(s), "plan beyond sync");
    *n_beyond = v;
    return SIM_OK;
}

int sim_plan_mode(const sim_plan *P, int *el_const, double *el_bound) {
    if (!P) HS_FAIL(SIM_EINVAL, "plan is NULL");
    if (el_const) *el_const = P->el_const ? 1 : 0;
    if (el_bound) *el_bound = P->el_bound;
    return SIM_OK;
}

// Validation of a sea description (before any device work).
static int sea_ok(const sim_sea *sea) {
    if (sea->mode < 0 || sea->mode > 2) HS_FAIL(SIM_EINVAL, "sea mode must be 0, 1 or 2");
    if (sea->mode == 0) return SIM_OK;
    const int nc = sea->n_comp;
    if (nc < 1 || nc > 4096) HS_FAIL(SIM_EINVAL, "wave modes need 1..4096 components");
    if (!(sea->k_min > 0) || !(sea->k_max >= sea->k_min) || !(sea->g > 0))
        HS_FAIL(SIM_EINVAL, "bad wave spectrum parameters");
    if (sea->mode == 1) {
        if (!sea->dirs || !sea->phases || !(sea->hs >= 0))
            HS_FAIL(SIM_EINVAL, "mode 1 needs dirs, phases and hs >= 0");
        return SIM_OK;
    }
    if (sea->ntx < 1 || sea->nty < 1 || !(sea->tile_L > 0) || !sea->node_hs ||
        !sea->node_dirs || !sea->node_phases)
        HS_FAIL(SIM_EINVAL, "mode 2 needs ntx, nty >= 1, tile_L > 0 and node arrays");
    const long long nodes = (long long)(sea->ntx + 1) * (sea->nty + 1);
    if (nodes * nc > (1LL << 22)) HS_FAIL(SIM_EINVAL, "too many node components");
    // the lattice must cover the grid
    const double hx = 0.5 * (sea->nx - 1) * sea->dx, hy = 0.5 * (sea->ny - 1) * sea->dy;
    if (!(sea->tile_x0 <= -hx) || !(sea->tile_y0 <= -hy) ||
        !(sea->tile_x0 + sea->ntx * sea->tile_L >= hx) ||
        !(sea->tile_y0 + sea->nty * sea->tile_L >= hy))
        HS_FAIL(SIM_EINVAL, "mode 2: the tile lattice does not cover the grid");
    for (long long q = 0; q < nodes; ++q)
        if (!(sea->node_hs[q] >= 0)) HS_FAIL(SIM_EINVAL, "mode 2: node_hs must be >= 0");
    return SIM_OK;
}

// Wave-component table of a sea (one homogeneous field in mode 1, one per
// lattice node in mode 2), rows (k, A, omega, cos psi, sin psi, phase):
// wavenumbers log-spaced on [k_min, k_max]; A_m^2 = 2 Psi(k_m) dk_m with
// Psi ~ k^slope and dk_m = k_m dlnk, scaled so sum A_m^2 / 2 = (hs/4)^2 per
// field; omega^2 = g k (deep water).  Empty for mode 0.  Parameters checked
// by sea_ok.
static void sea_table(const sim_sea *sea, std::vector<double> &tab) {
    tab.clear();
    if (sea->mode < 1) return;
    const int nc = sea->n_comp;
    int nodes = 1;
    const double *hs_of = &sea->hs;
    const double *dirs = sea->dirs, *phases = sea->phases;
    if (sea->mode == 2) {
        nodes = (sea->ntx + 1) * (sea->nty + 1);
        hs_of = sea->node_hs;
        dirs = sea->node_dirs;
        phases = sea->node_phases;
    }
    tab.assign((size_t)6 * nc * nodes, 0.0);
    const double dl = nc > 1 ? std::log(sea->k_max / sea->k_min) / (nc - 1) : 1.0;
    for (int q = 0; q < nodes; ++q) {
        double energy = 0.0;
        double *tq = &tab[(size_t)6 * nc * q];
        for (int m = 0; m < nc; ++m) {
            const double k = nc > 1 ? sea->k_min * std::exp(dl * m) : sea->k_min;
            const double A = std::sqrt(2.0 * std::pow(k, sea->slope) * k * dl);
            energy += 0.5 * A * A;
            double *t = tq + 6 * m;
            t[0] = k;
            t[1] = A;
            t[2] = std::sqrt(sea->g * k);
            t[3] = std::cos(dirs[(size_t)q * nc + m]);
            t[4] = std::sin(dirs[(size_t)q * nc + m]);
            t[5] = phases[(size_t)q * nc + m];
        }
        const double scale = energy > 0 ? (hs_of[q] / 4.0) / std::sqrt(energy) : 0.0;
        for (int m = 0; m < nc; ++m) tq[6 * m + 1] *= scale;
    }
}

static int grid_ok(const sim_sea *sea, int ix0, int iy0, int cnx, int cny) {
    if (sea->nx < 1 || sea->ny < 1 || !(sea->dx > 0) || !(sea->dy > 0))
        HS_FAIL(SIM_EINVAL, "grid size and spacing must be positive");
    if (ix0 < 0 || iy0 < 0 || cnx < 0 || cny < 0 || (long long)ix0 + cnx > sea->nx ||
        (long long)iy0 + cny > sea->ny)
        HS_FAIL(SIM_EINVAL, "sub-rectangle outside the grid");
    return SIM_OK;
}

// Rectangle holding every facet of a grid sub-rectangle: its cell centres,
// widened by the largest Choppy Wave Model displacement (the sum of a
// field's amplitudes, twice that for the four weighted fields of mode 2,
// whose weights add up to at most 2) and by a rounding margin.
static void chunk_box(const sim_sea *sea, const std::vector<double> &tab, int ix0, int iy0,
                      int cnx, int cny, sim_box *box) {
    const double cx = 0.5 * (double)(sea->nx - 1), cy = 0.5 * (double)(sea->ny - 1);
    double x0 = ((double)ix0 - cx) * sea->dx, x1 = ((double)(ix0 + cnx - 1) - cx) * sea->dx;
    double y0 = ((double)iy0 - cy) * sea->dy, y1 = ((double)(iy0 + cny - 1) - cy) * sea->dy;
    double shift = 0.0;
    if (sea->cwm && sea->mode >= 1 && !tab.empty()) {
        const size_t rows = tab.size() / 6, nc = (size_t)sea->n_comp;
        for (size_t q = 0; q < rows / nc; ++q) {
            double s = 0.0;
            for (size_t m = 0; m < nc; ++m) s += std::fabs(tab[6 * (q * nc + m) + 1]);
            shift = std::max(shift, s);
        }
        if (sea->mode == 2) shift *= 2.0;
    }
    const double mx = 1e-3 + 1e-6 * std::max(std::max(std::fabs(x0), std::fabs(x1)),
                                             std::max(std::fabs(y0), std::fabs(y1)));
    box->x_min = x0 - shift - mx;
    box->x_max = x1 + shift + mx;
    box->y_min = y0 - shift - mx;
    box->y_max = y1 + shift + mx;
    // heights and speeds: per field at most sum A and sum A omega (each
    // component's velocity has magnitude A omega), weights adding up to at
    // most 2 in mode 2, plus the current; a flat sea's Gaussian speeds
    // exceed 6 sigma_v with probability below 1e-7
    double zs = 0.0, vs = 0.0;
    if (sea->mode >= 1 && !tab.empty()) {
        const size_t rows = tab.size() / 6, nc = (size_t)sea->n_comp;
        for (size_t q = 0; q < rows / nc; ++q) {
            double a = 0.0, aw = 0.0;
            for (size_t m = 0; m < nc; ++m) {
                const double *t = &tab[6 * (q * nc + m)];
                a += std::fabs(t[1]);
                aw += std::fabs(t[1]) * t[2];
            }
            zs = std::max(zs, a);
            vs = std::max(vs, aw);
        }
        if (sea->mode == 2) {
            zs *= 2.0;
            vs *= 2.0;
        }
        vs += std::hypot(sea->current[0], sea->current[1]);
    } else {
        vs = 6.0 * sea->sigma_v;
    }
    // float32 rounding of the generated values, and never 0 (the default)
    box->z_max = std::max(1e-3, zs * (1.0 + 1e-5) + 1e-6);
    box->v_max = std::max(1e-3, vs * (1.0 + 1e-5) + 1e-6);
}

// Launch of the generator for a sub-rectangle, its sea table already on the
// device (tab_d; NULL in mode 0).
static int generate_launch(const sim_sea *sea, unsigned long long seed, int ix0, int iy0,
                           int cnx, int cny, const sim_facets_out *out, const double *tab_d,
                           hipStream_t s) {
    hs::GenArgs a{};
    a.nx = sea->nx;
    a.ny = sea->ny;
    a.dx = sea->dx;
    a.dy = sea->dy;
    a.mode = sea->mode;
    a.sigma_v = sea->sigma_v;
    a.seed = seed;
    a.ix0 = ix0;
    a.iy0 = iy0;
    a.cnx = cnx;
    a.cny = cny;
    a.out = *out;
    a.cur0 = sea->current[0];
    a.cur1 = sea->current[1];
    a.n_comp = sea->mode >= 1 ? sea->n_comp : 0;
    a.cwm = sea->cwm ? 1 : 0;
    a.tab = tab_d;
    if (sea->mode == 2) {
        a.ntx = sea->ntx;
        a.nty = sea->nty;
        a.tile_L = sea->tile_L;
        a.tile_x0 = sea->tile_x0;
        a.tile_y0 = sea->tile_y0;
    }
    HS_HIP(hs::launch_generate(a, s), "generate launch");
    return SIM_OK;
}

int sim_sea_table_size(const sim_sea *sea, size_t *bytes) {
    if (!sea || !bytes) HS_FAIL(SIM_EINVAL, "sea or bytes is NULL");
    if (int rc = sea_ok(sea)) return rc;
    long long nodes = sea->mode == 2 ? (long long)(sea->ntx + 1) * (sea->nty + 1) : 1;
    *bytes = sea->mode >= 1 ? align256(sizeof(double) * 6 * (size_t)sea->n_comp * (size_t)nodes)
                            : 0;
    return SIM_OK;
}

int sim_chunk_box(const sim_sea *sea, int ix0, int iy0, int cnx, int cny, sim_box *box) {
    if (!sea || !box) HS_FAIL(SIM_EINVAL, "sea or box is NULL");
    if (int rc = grid_ok(sea, ix0, iy0, cnx, cny)) return rc;
    if (cnx < 1 || cny < 1) HS_FAIL(SIM_EINVAL, "empty sub-rectangle");
    if (int rc = sea_ok(sea)) return rc;
    std::vector<double> tab;
    sea_table(sea, tab);
    chunk_box(sea, tab, ix0, iy0, cnx, cny, box);
    return SIM_OK;
}

int sim_generate_facets(sim_handle *h, const sim_sea *sea, unsigned long long seed, int ix0,
                        int iy0, int cnx, int cny, const sim_facets_out *out, void *workspace,
                        size_t workspace_bytes, void *stream) {
    if (!h || !sea || !out) HS_FAIL(SIM_EINVAL, "handle, sea or out is NULL");
    if (int rc = grid_ok(sea, ix0, iy0, cnx, cny)) return rc;
    if (out->n != (long long)cnx * cny) HS_FAIL(SIM_EINVAL, "out->n must equal cnx*cny");
    if (out->n > 0 && (!out->x || !out->y || !out->z || !out->vx || !out->vy || !out->vz ||
                       !out->a_re || !out->a_im))
        HS_FAIL(SIM_EINVAL, "an output array pointer is NULL");
    if (int rc = sea_ok(sea)) return rc;
    size_t need = 0;
    if (int rc = sim_sea_table_size(sea, &need)) return rc;
    if (need > 0)
        if (int rc = workspace_ok(workspace, workspace_bytes, need)) return rc;
    if (int rc = ensure_device(h)) return rc;
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> &tab = h->gen_tab_h;
    sea_table(sea, tab);
    double *tab_d = need > 0 ? (double *)workspace : nullptr;
    if (tab_d) HS_HIP(hs::launch_upload(tab_d, tab.data(), (long long)tab.size(), s), "sea table");
    return generate_launch(sea, seed, ix0, iy0, cnx, cny, out, tab_d, s);
}

// ---- intra-facet speckle (Sec. III.A eq. 7, eq. 10) ------------------------

static int speckle_ok(const sim_handle *h, const sim_speckle *sp) {
    if (!sp) return SIM_OK;
    if (!(sp->tau_s > 0.0)) HS_FAIL(SIM_EINVAL, "speckle tau_s must be > 0 (or +inf)");
    if (sp->first_index < 0) HS_FAIL(SIM_EINVAL, "speckle first_index < 0");
    (void)h;
    return SIM_OK;
}

// Host constants of the speckle process for one call (FP64, then float):
// b = exp(-a), a = 1 / (prf tau_s) (0 for tau_s = inf), the powers b^m, the
// bridge gains K_k = b^(64-k) (1 - b^2k) / (1 - b^128) (k / 64 at a = 0) and
// the innovation scales sqrt(1 - b^2), sqrt(1 - b^128); then the per-facet
// records and anchors of the groups the pulse range covers.
// chunk: (ix0, iy0, cnx, cny) of a generated chunk of a grid grid_nx wide, whose
// facets take ids and Doppler by grid index; NULL for a caller's facet set.
static int speckle_prepare(const sim_handle *h, const sim_plan *P, const sim_speckle *sp,
                           int p0, int np,
                           bool with_d, const int *chunk, int grid_nx, hipStream_t s,
                           hs::SpkArgs &k) {
    const double a = std::isinf(sp->tau_s) ? 0.0 : 1.0 / (h->prf * sp->tau_s);
    for (int m = 0; m <= 64; ++m) k.bpow[m] = (float)std::exp(-a * m);
    for (int j = 0; j < 64; ++j)
        k.gain[j] = a == 0.0 ? (float)(j / 64.0)
                             : (float)(std::exp(-a * (64 - j)) * std::expm1(-2.0 * a * j) /
                                       std::expm1(-128.0 * a));
    k.b1 = k.bpow[1];
    k.b2 = k.bpow[2];
    k.b4 = k.bpow[4];
    k.b8 = k.bpow[8];
    k.b64 = k.bpow[64];
    k.c1 = (float)std::sqrt(-std::expm1(-2.0 * a));
    k.c64 = (float)std::sqrt(-std::expm1(-128.0 * a));
    k.key = (uint32_t)sp->seed ^ (uint32_t)(sp->seed >> 32);
    k.n_groups = (h->Np + 63) / 64;
    const long long n = P->n;
    if (!P->spk || !P->anch)
        HS_FAIL(SIM_EINVAL, "the plan was made without SIM_PLAN_SPECKLE (no speckle space)");
    k.rec = P->spk;
    k.anch = P->anch;
    hs::SpkPrep pp{};
    pp.n = n;
    pp.perm = P->perm;
    pp.fs = sp->f_s;
    pp.first_index = sp->first_index;
    pp.g_lo = p0 >> 6;
    pp.g_hi = (p0 + np - 1) >> 6;
    pp.with_d = with_d;
    if (chunk) {
        pp.grid_nx = grid_nx;
        pp.sub_x0 = chunk[0];
        pp.sub_y0 = chunk[1];
        pp.sub_nx = chunk[2];
    }
    HS_HIP(hs::launch_speckle_prep(pp, k, P->spk, P->anch, s), "speckle preparation");
    return SIM_OK;
}

// Gather of the facet records and launch of the forward sum over n_groups
// groups of 64 pulses starting gstride pulses apart from p0 (pulse p0 + j
// writes row j of iq, np rows per channel); the IQ rows already hold what the
// sum is added to.
static int forward_launch(const sim_handle *h, const sim_plan *P, const sim_facets *f,
                          const sim_speckle *sp, int p0, int np, int n_groups, int gstride,
                          float *iq, hipStream_t s, const int *chunk, int grid_nx) {
    HS_HIP(hs::launch_gather(*f, P->perm, P->blocks, P->n_blocks, P->nb_max, P->sorted,
                             (float)(P->zlim * (1.0 + 1e-6)), (float)(P->vlim * (1.0 + 1e-6)),
                             P->beyond, s),
           "gather");
    hs::FwdArgs a{};
    if (sp)
        if (int rc = speckle_prepare(h, P, sp, p0, np, false, chunk, grid_nx, s, a.spk))
            return rc;
    if (P->ng_slots < 1) HS_FAIL(SIM_EINVAL, "the plan has no window slots");
    a.facets = P->sorted;
    a.blocks = P->blocks;
    a.st = P->st;
    a.wsum = P->wsum;
    a.counter = P->counter;
    a.pulses = h->pulses_d;
    a.iq = iq;
    for (size_t i = 0; i < h->antc.size(); ++i) a.ant[i] = h->antc[i];
    for (int i = 0; i < h->C; ++i) a.ch[i] = h->chc[i];
    a.tp = h->tp;
    a.f0_c = h->f0 / h->c;
    a.fs_c = h->fs / h->c;
    a.n_ref = (double)h->n_ref;
    a.linv_hi = (float)a.f0_c;
    a.linv_lo = (float)(a.f0_c - (double)a.linv_hi);
    a.fs_cf = (float)a.fs_c;
    a.N = h->N;
    a.Np = h->Np;
    a.p0 = p0;
    a.np = np;
    a.n_groups = n_groups;
    a.gstride = gstride;
    a.C = h->C;
    a.rx_exact = h->rx_exact;
    a.steer = h->steer;
    a.grid = h->grid;
    a.inv_c = 1.0 / h->c;
    hs::ReduceArgs r{};
    r.st = P->st;
    r.wsum = P->wsum;
    r.iq = reinterpret_cast<float2 *>(iq);
    r.C = h->C;
    r.N = h->N;
    r.Np = h->Np;
    r.p0 = p0;
    r.np = np;
    r.gstride = gstride;
    r.poff = sp ? (p0 & 63) : 0;
    r.win = P->win;
    r.n_tiles = P->span_tiles;
    // the pulse groups in passes of as many as the window slots hold (one
    // pass unless the plan was laid out for fewer groups), each summed and
    // reduced before the next reuses the slots
    a.slot_w = P->win;
    for (int g0 = 0; g0 < n_groups; g0 += P->ng_slots) {
        const int ng = std::min(P->ng_slots, n_groups - g0);
        a.g0 = r.g0 = g0;
        a.n_groups = r.n_groups = ng;
        // one launch per window width the bands use (each takes the units
        // of its own bands)
        for (int w : {24, 26, 32, 48, 64}) {
            if (!(P->win_mask & hs::win_bit(w))) continue;
            HS_HIP(hs::launch_fill_zero((float *)P->counter, hs::kFwdQueues, s), "work queues");
            HS_HIP(hs::launch_forward(a, h->C, w, P->el_const && !h->grid, sp != nullptr, s),
                   "forward");
        }
        HS_HIP(hs::launch_window_reduce(r, s), "window reduce");
    }
    return SIM_OK;
}

static int forward_common(sim_handle *h, sim_plan *P, const sim_facets *f,
                          const sim_speckle *sp, int p0, int np, float *iq, int accumulate,
                          void *stream, const int *chunk = nullptr, int grid_nx = 0) {
    if (!h || !P) HS_FAIL(SIM_EINVAL, "handle or plan is NULL");
    if (P->h != h) HS_FAIL(SIM_EINVAL, "plan belongs to another handle");
    if (int rc = facets_ok(f, P->n)) return rc;
    if (p0 < 0 || np < 0 || (long long)p0 + np > h->Np) HS_FAIL(SIM_EINVAL, "pulse range");
    if (int rc = speckle_ok(h, sp)) return rc;
    if (sp && !(P->flags & SIM_PLAN_SPECKLE))
        HS_FAIL(SIM_EINVAL, "the plan was made without SIM_PLAN_SPECKLE (no speckle space)");
    if (np == 0) return SIM_OK;   // nothing to write (an empty IQ may have a NULL pointer)
    if (!iq) HS_FAIL(SIM_EINVAL, "iq is NULL");
    if (int rc = ensure_device(h)) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (!accumulate)
        HS_HIP(hs::launch_fill_zero(iq, 2LL * h->C * np * h->N, s), "zero iq");
    // speckle groups are aligned on absolute pulse indices
    const int poff = sp ? (p0 & 63) : 0;
    return forward_launch(h, P, f, sp, p0, np, (poff + np + 63) / 64, 64, iq, s, chunk, grid_nx);
}

// ---- fast mode (Sec. IV.B) ----------------------------------------------------

struct FastLayout {
    int K, L_s, log_L;
    size_t x_bytes;
};

static int fast_layout(const sim_handle *h, int n_fast, FastLayout &F) {
    if (n_fast < 64 || n_fast > 1024) HS_FAIL(SIM_EINVAL, "n_fast must be in [64, 1024]");
    if (h->Np < 64) HS_FAIL(SIM_EINVAL, "the fast mode needs at least 64 pulses");
    F.K = (h->Np - 64) / n_fast + 1;
    F.L_s = 1;
    F.log_L = 0;
    while (F.L_s < 2 * n_fast + 64) {
        F.L_s <<= 1;
        ++F.log_L;
    }
    F.x_bytes = align256(sizeof(float) * 2 * (size_t)h->C * F.K * 64 * (size_t)h->N);
    return SIM_OK;
}

int sim_fast_workspace_size(const sim_handle *h, int n_fast, size_t *bytes) {
    if (!h || !bytes) HS_FAIL(SIM_EINVAL, "handle or bytes is NULL");
    FastLayout F;
    if (int rc = fast_layout(h, n_fast, F)) return rc;
    *bytes = F.x_bytes;
    return SIM_OK;
}

int sim_forward_fast(sim_handle *h, sim_plan *P, const sim_facets *f, int n_fast,
                     unsigned long long seed, float *iq, void *workspace, size_t workspace_bytes,
                     void *stream) {
    if (!h || !P) HS_FAIL(SIM_EINVAL, "handle or plan is NULL");
    if (P->h != h) HS_FAIL(SIM_EINVAL, "plan belongs to another handle");
    if (int rc = facets_ok(f, P->n)) return rc;
    FastLayout F;
    if (int rc = fast_layout(h, n_fast, F)) return rc;
    if (!iq) HS_FAIL(SIM_EINVAL, "iq is NULL");
    if (int rc = workspace_ok(workspace, workspace_bytes, F.x_bytes)) return rc;
    if (int rc = ensure_device(h)) return rc;
    hipStream_t s = (hipStream_t)stream;
    HS_HIP(hs::launch_fill_zero(iq, 2LL * h->C * h->Np * h->N, s), "zero iq");
    // the windows: K groups of 64 pulses, n_fast apart, into their own rows
    if (int rc = forward_launch(h, P, f, nullptr, 0, h->Np, F.K, n_fast, iq, s, nullptr, 0))
        return rc;
    hs::FastArgs a{};
    a.iq = reinterpret_cast<float2 *>(iq);
    a.X = reinterpret_cast<float2 *>(workspace);
    a.C = h->C;
    a.Np = h->Np;
    a.N = h->N;
    a.n_fast = n_fast;
    a.K = F.K;
    a.L_s = F.L_s;
    a.log_L = F.log_L;
    a.seed = seed;
    HS_HIP(hs::launch_fast(a, s), "fast mode");
    return SIM_OK;
}

int sim_forward(sim_handle *h, sim_plan *P, const sim_facets *f, int p0, int np, float *iq,
                int accumulate, void *stream) {
    return forward_common(h, P, f, nullptr, p0, np, iq, accumulate, stream);
}

int sim_forward_speckle(sim_handle *h, sim_plan *P, const sim_facets *f,
                        const sim_speckle *speckle, int p0, int np, float *iq, int accumulate,
                        void *stream) {
    if (!speckle) HS_FAIL(SIM_EINVAL, "speckle is NULL");
    return forward_common(h, P, f, speckle, p0, np, iq, accumulate, stream);
}

static int backward_common(sim_handle *h, sim_plan *P, const sim_facets *f,
                           const sim_speckle *sp, int p0, int np, const float *g,
                           const sim_facet_grads *gr, int accumulate, void *stream,
                           const int *chunk = nullptr, int grid_nx = 0) {
    if (!h || !P) HS_FAIL(SIM_EINVAL, "handle or plan is NULL");
    if (P->h != h) HS_FAIL(SIM_EINVAL, "plan belongs to another handle");
    if (int rc = facets_ok(f, P->n)) return rc;
    if (p0 < 0 || np < 0 || (long long)p0 + np > h->Np) HS_FAIL(SIM_EINVAL, "pulse range");
    if (!gr) HS_FAIL(SIM_EINVAL, "grads is NULL");
    if (!g && np > 0) HS_FAIL(SIM_EINVAL, "g is NULL");
    if (gr->n != P->n) HS_FAIL(SIM_EINVAL, "grads->n differs from the plan's facet count");
    if (int rc = speckle_ok(h, sp)) return rc;
    if (sp && !(P->flags & SIM_PLAN_SPECKLE))
        HS_FAIL(SIM_EINVAL, "the plan was made without SIM_PLAN_SPECKLE (no speckle space)");
    if (int rc = ensure_device(h)) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (np == 0) {
        if (!accumulate) {
            float *outs[6] = {gr->dz, gr->dvx, gr->dvy, gr->dvz, gr->da_re, gr->da_im};
            for (float *o : outs)
                if (o) HS_HIP(hs::launch_fill_zero(o, P->n, s), "zero grads");
        }
        return SIM_OK;
    }
    HS_HIP(hs::launch_gather(*f, P->perm, P->blocks, P->n_blocks, P->nb_max, P->sorted,
                             (float)(P->zlim * (1.0 + 1e-6)), (float)(P->vlim * (1.0 + 1e-6)),
                             P->beyond, s),
           "gather");
    hs::AdjArgs a{};
    if (sp)
        if (int rc = speckle_prepare(h, P, sp, p0, np, true, chunk, grid_nx, s, a.spk))
            return rc;
    a.facets = P->sorted;
    a.blocks = P->blocks;
    a.perm = P->perm;
    a.pulses = h->pulses_d;
    for (size_t i = 0; i < h->antc.size(); ++i) a.ant[i] = h->antc[i];
    for (int i = 0; i < h->C; ++i) a.ch[i] = h->chc[i];
    a.g = g;
    a.dz = gr->dz;
    a.dvx = gr->dvx;
    a.dvy = gr->dvy;
    a.dvz = gr->dvz;
    a.dar = gr->da_re;
    a.dai = gr->da_im;
    a.tp = h->tp;
    a.f0_c = h->f0 / h->c;
    a.fs_c = h->fs / h->c;
    a.n_ref = (double)h->n_ref;
    a.linv_hi = (float)a.f0_c;
    a.linv_lo = (float)(a.f0_c - (double)a.linv_hi);
    a.fs_cf = (float)a.fs_c;
    a.k0 = (float)(2.0 * kPi * a.f0_c);
    a.N = h->N;
    a.Np = h->Np;
    a.p0 = p0;
    a.np = np;
    a.C = h->C;
    a.n_blocks = P->n_blocks;
    a.nb_max = P->nb_max;
    a.accumulate = accumulate ? 1 : 0;
    a.rx_exact = h->rx_exact;
    a.steer = h->steer;
    a.inv_c = 1.0 / h->c;
    a.grid = h->grid;
    // (with gridded patterns the plan's far-field mode only drops the
    // adjoint's Jacobian correction; the patterns stay per facet)
    HS_HIP(hs::launch_adjoint(a, P->el_const, sp != nullptr, s), "adjoint");
    return SIM_OK;
}

int sim_backward(sim_handle *h, sim_plan *P, const sim_facets *f, int p0, int np,
                 const float *g, const sim_facet_grads *gr, int accumulate, void *stream) {
    return backward_common(h, P, f, nullptr, p0, np, g, gr, accumulate, stream);
}

int sim_backward_speckle(sim_handle *h, sim_plan *P, const sim_facets *f,
                         const sim_speckle *speckle, int p0, int np, const float *g,
                         const sim_facet_grads *gr, int accumulate, void *stream) {
    if (!speckle) HS_FAIL(SIM_EINVAL, "speckle is NULL");
    return backward_common(h, P, f, speckle, p0, np, g, gr, accumulate, stream);
}

static int waveform_common(sim_handle *h, const float *in, float *out, long long n_lines,
                           void *stream, int adjoint) {
    if (!h) HS_FAIL(SIM_EINVAL, "handle is NULL");
    if (h->chirp_len == 0) HS_FAIL(SIM_EUNSUPPORTED, "the handle has no waveform (chirp_T = 0)");
    if (h->fft_len == 0) HS_FAIL(SIM_EUNSUPPORTED, "waveform FFT longer than 16384");
    if (n_lines < 0) HS_FAIL(SIM_EINVAL, "n_lines < 0");
    if (n_lines > 0 && (!in || !out)) HS_FAIL(SIM_EINVAL, "in or out is NULL");
    if (n_lines > (1LL << 31)) HS_FAIL(SIM_EINVAL, "too many lines");
    if (int rc = ensure_device(h)) return rc;
    HS_HIP(hs::launch_waveform(in, out, n_lines, h->N, h->fft_len, h->chirp_len / 2,
                               h->chirp_spec_d, h->twiddle_d, adjoint, (hipStream_t)stream),
           "waveform");
    return SIM_OK;
}

int sim_apply_waveform(sim_handle *h, const float *iq_rc, float *iq_raw, long long n_lines,
                       void *stream) {
    return waveform_common(h, iq_rc, iq_raw, n_lines, stream, 0);
}

int sim_apply_waveform_adjoint(sim_handle *h, const float *g_raw, float *g_rc,
                               long long n_lines, void *stream) {
    return waveform_common(h, g_raw, g_rc, n_lines, stream, 1);
}

}  // extern "C"

namespace {

int check_chunks(const sim_sea *sea, const int *chunks, int n_chunks, long long *max_n) {
    if (!sea || !chunks || n_chunks < 1) HS_FAIL(SIM_EINVAL, "sea, chunks and n_chunks >= 1 needed");
    long long m = 0;
    for (int k = 0; k < n_chunks; ++k) {
        const int *c = chunks + 4 * k;
        if (c[0] < 0 || c[1] < 0 || c[2] < 1 || c[3] < 1 || (long long)c[0] + c[2] > sea->nx ||
            (long long)c[1] + c[3] > sea->ny)
            HS_FAIL(SIM_EINVAL, "chunk outside the grid or empty");
        m = std::max(m, (long long)c[2] * c[3]);
    }
    *max_n = m;
    return SIM_OK;
}

sim_facets as_in(const sim_facets_out &o) {
    sim_facets f;
    f.n = o.n;
    f.x = o.x; f.y = o.y; f.z = o.z; f.vx = o.vx; f.vy = o.vy; f.vz = o.vz;
    f.a_re = o.a_re; f.a_im = o.a_im;
    return f;
}

}  // namespace

extern "C" {

// Workspace of a streamed call: the sea table, one chunk's facets (8 float32
// arrays of the largest chunk) and the plan of the largest chunk layout.
struct StreamLayout {
    size_t tab = 0, facets = 0, facet_stride = 0, plan = 0, total = 0;
    long long max_n = 0;
    std::vector<PlanGeom> geom;     // per chunk
    std::vector<PlanLayout> lay;    // per chunk
};

// Layouts of the chunks' plans with window slots for at most ng_cap pulse
// groups, and the offsets and total of the streamed workspace.
static void stream_relayout(const sim_handle *h, const int *chunks, int n_chunks, int flags,
                            int ng_cap, long long max_n, size_t tab_doubles, StreamLayout &Y) {
    size_t plan_bytes = 0;
    for (int k = 0; k < n_chunks; ++k) {
        const int *c = chunks + 4 * k;
        Y.geom[k].ng_slots = std::max(1, std::min(Y.geom[k].ng_max, ng_cap));
        Y.lay[k] = plan_layout(Y.geom[k], (long long)c[2] * c[3], flags, h->Np);
        plan_bytes = std::max(plan_bytes, Y.lay[k].total);
    }
    Y.tab = 0;
    Y.facets = align256(sizeof(double) * tab_doubles);
    Y.facet_stride = align256(sizeof(float) * (size_t)max_n);
    Y.plan = Y.facets + 8 * Y.facet_stride;
    Y.total = Y.plan + plan_bytes;
}

static int stream_layout(const sim_handle *h, const sim_sea *sea, const int *chunks,
                         int n_chunks, double block_edge, int flags,
                         const std::vector<double> &tab, StreamLayout &Y,
                         int ng_cap = 1 << 30) {
    long long max_n = 0;
    if (int rc = check_chunks(sea, chunks, n_chunks, &max_n)) return rc;
    Y.geom.resize(n_chunks);
    Y.lay.resize(n_chunks);
    for (int k = 0; k < n_chunks; ++k) {
        const int *c = chunks + 4 * k;
        sim_box box;
        chunk_box(sea, tab, c[0], c[1], c[2], c[3], &box);
        const long long n = (long long)c[2] * c[3];
        if (int rc = plan_geometry(h, n, &box, block_edge, Y.geom[k])) return rc;
    }
    Y.max_n = max_n;
    stream_relayout(h, chunks, n_chunks, flags, ng_cap, max_n, tab.size(), Y);
    return SIM_OK;
}

static sim_facets_out chunk_facets(char *ws, const StreamLayout &Y, long long n) {
    sim_facets_out o;
    o.n = n;
    float *q[8];
    for (int k = 0; k < 8; ++k) q[k] = (float *)(ws + Y.facets + (size_t)k * Y.facet_stride);
    o.x = q[0]; o.y = q[1]; o.z = q[2]; o.vx = q[3]; o.vy = q[4]; o.vz = q[5];
    o.a_re = q[6]; o.a_im = q[7];
    return o;
}

int sim_stream_workspace_size(const sim_handle *h, const sim_sea *sea, const int *chunks,
                              int n_chunks, double block_edge, int flags, size_t *bytes) {
    if (!h || !bytes) HS_FAIL(SIM_EINVAL, "handle or bytes is NULL");
    if (flags & ~SIM_PLAN_SPECKLE) HS_FAIL(SIM_EINVAL, "unknown plan flags");
    if (!sea) HS_FAIL(SIM_EINVAL, "sea is NULL");
    if (int rc = sea_ok(sea)) return rc;
    std::vector<double> tab;
    sea_table(sea, tab);
    StreamLayout Y;
    if (int rc = stream_layout(h, sea, chunks, n_chunks, block_edge, flags, tab, Y)) return rc;
    *bytes = Y.total;
    return SIM_OK;
}

// Checks, lays out the workspace and uploads the sea table of a streamed call.
static int stream_setup(sim_handle *h, const sim_sea *sea, const int *chunks, int n_chunks,
                        double block_edge, const sim_speckle *sp, int p0, int np, void *ws,
                        size_t ws_bytes, hipStream_t s, StreamLayout &Y, int ng_cap = 1 << 30) {
    if (!h) HS_FAIL(SIM_EINVAL, "handle is NULL");
    if (!sea) HS_FAIL(SIM_EINVAL, "sea is NULL");
    long long max_n = 0;
    if (int rc = check_chunks(sea, chunks, n_chunks, &max_n)) return rc;
    if (p0 < 0 || np < 0 || (long long)p0 + np > h->Np) HS_FAIL(SIM_EINVAL, "pulse range");
    if (int rc = speckle_ok(h, sp)) return rc;
    if (int rc = sea_ok(sea)) return rc;
    std::vector<double> &tab = h->gen_tab_h;
    sea_table(sea, tab);
    const int flags = sp ? SIM_PLAN_SPECKLE : 0;
    if (int rc = stream_layout(h, sea, chunks, n_chunks, block_edge, flags, tab, Y, ng_cap))
        return rc;
    if (int rc = workspace_ok(ws, ws_bytes, Y.total)) return rc;
    if (int rc = ensure_device(h)) return rc;
    if (!tab.empty())
        HS_HIP(hs::launch_upload((double *)((char *)ws + Y.tab), tab.data(), (long long)tab.size(),
                                 s),
               "sea table");
    return SIM_OK;
}

static int stream_forward_common(sim_handle *h, const sim_sea *sea, unsigned long long seed,
                                 const int *chunks, int n_chunks, double block_edge,
                                 const sim_speckle *sp, int p0, int np, float *iq,
                                 int accumulate, void *ws, size_t ws_bytes, void *stream,
                                 int ng_cap = 1 << 30) {
    if (!iq) HS_FAIL(SIM_EINVAL, "iq is NULL");
    hipStream_t s = (hipStream_t)stream;
    StreamLayout Y;
    if (int rc = stream_setup(h, sea, chunks, n_chunks, block_edge, sp, p0, np, ws, ws_bytes, s,
                              Y, ng_cap))
        return rc;
    char *w = (char *)ws;
    const double *tab_d = sea->mode >= 1 ? (const double *)(w + Y.tab) : nullptr;
    if (!accumulate) HS_HIP(hs::launch_fill_zero(iq, 2LL * h->C * np * h->N, s), "zero iq");
    const int flags = sp ? SIM_PLAN_SPECKLE : 0;
    for (int k = 0; k < n_chunks; ++k) {
        const int *c = chunks + 4 * k;
        const long long n = (long long)c[2] * c[3];
        const sim_facets_out o = chunk_facets(w, Y, n);
        if (int rc = generate_launch(sea, seed, c[0], c[1], c[2], c[3], &o, tab_d, s)) return rc;
        sim_plan P;
        if (int rc = plan_build(h, o.x, o.y, n, Y.geom[k], Y.lay[k], flags, w + Y.plan, s, P))
            return rc;
        const sim_facets f = as_in(o);
        if (int rc = forward_common(h, &P, &f, sp, p0, np, iq, 1, stream, c, sea->nx)) return rc;
    }
    return SIM_OK;
}

int sim_stream_forward(sim_handle *h, const sim_sea *sea, unsigned long long seed,
                       const int *chunks, int n_chunks, double block_edge, int p0, int np,
                       float *iq, int accumulate, void *workspace, size_t workspace_bytes,
                       void *stream) {
    return stream_forward_common(h, sea, seed, chunks, n_chunks, block_edge, nullptr, p0, np,
                                 iq, accumulate, workspace, workspace_bytes, stream);
}

int sim_stream_forward_speckle(sim_handle *h, const sim_sea *sea, unsigned long long seed,
                               const int *chunks, int n_chunks, double block_edge,
                               const sim_speckle *speckle, int p0, int np, float *iq,
                               int accumulate, void *workspace, size_t workspace_bytes,
                               void *stream) {
    if (!speckle) HS_FAIL(SIM_EINVAL, "speckle is NULL");
    return stream_forward_common(h, sea, seed, chunks, n_chunks, block_edge, speckle, p0, np,
                                 iq, accumulate, workspace, workspace_bytes, stream);
}

static int stream_backward_common(sim_handle *h, const sim_sea *sea, unsigned long long seed,
                                  const int *chunks, int n_chunks, double block_edge,
                                  const sim_speckle *sp, int p0, int np, const float *g,
                                  float *dvx, float *dvy, float *dvz, void *ws, size_t ws_bytes,
                                  void *stream) {
    if (!g) HS_FAIL(SIM_EINVAL, "g is NULL");
    hipStream_t s = (hipStream_t)stream;
    StreamLayout Y;
    if (int rc = stream_setup(h, sea, chunks, n_chunks, block_edge, sp, p0, np, ws, ws_bytes, s,
                              Y))
        return rc;
    char *w = (char *)ws;
    const double *tab_d = sea->mode >= 1 ? (const double *)(w + Y.tab) : nullptr;
    const int flags = sp ? SIM_PLAN_SPECKLE : 0;
    long long off = 0;
    for (int k = 0; k < n_chunks; ++k) {
        const int *c = chunks + 4 * k;
        const long long n = (long long)c[2] * c[3];
        const sim_facets_out o = chunk_facets(w, Y, n);
        if (int rc = generate_launch(sea, seed, c[0], c[1], c[2], c[3], &o, tab_d, s)) return rc;
        sim_plan P;
        if (int rc = plan_build(h, o.x, o.y, n, Y.geom[k], Y.lay[k], flags, w + Y.plan, s, P))
            return rc;
        const sim_facets f = as_in(o);
        sim_facet_grads gr;
        gr.n = n;
        gr.dz = nullptr;
        gr.dvx = dvx ? dvx + off : nullptr;
        gr.dvy = dvy ? dvy + off : nullptr;
        gr.dvz = dvz ? dvz + off : nullptr;
        gr.da_re = nullptr;
        gr.da_im = nullptr;
        if (int rc = backward_common(h, &P, &f, sp, p0, np, g, &gr, 0, stream, c, sea->nx))
            return rc;
        off += n;
    }
    return SIM_OK;
}

int sim_stream_backward(sim_handle *h, const sim_sea *sea, unsigned long long seed,
                        const int *chunks, int n_chunks, double block_edge, int p0, int np,
                        const float *g, float *dvx, float *dvy, float *dvz, void *workspace,
                        size_t workspace_bytes, void *stream) {
    return stream_backward_common(h, sea, seed, chunks, n_chunks, block_edge, nullptr, p0, np,
                                  g, dvx, dvy, dvz, workspace, workspace_bytes, stream);
}

int sim_stream_backward_speckle(sim_handle *h, const sim_sea *sea, unsigned long long seed,
                                const int *chunks, int n_chunks, double block_edge,
                                const sim_speckle *speckle, int p0, int np, const float *g,
                                float *dvx, float *dvy, float *dvz, void *workspace,
                                size_t workspace_bytes, void *stream) {
    if (!speckle) HS_FAIL(SIM_EINVAL, "speckle is NULL");
    return stream_backward_common(h, sea, seed, chunks, n_chunks, block_edge, speckle, p0, np,
                                  g, dvx, dvy, dvz, workspace, workspace_bytes, stream);
}

int sim_stream_forward_noalloc(sim_handle *h, const sim_sea *sea, unsigned long long seed,
                               const int *chunks, int n_chunks, double block_edge, int p0,
                               int np, float *iq, int accumulate, void *stream) {
    if (!h) HS_FAIL(SIM_EINVAL, "handle is NULL");
    if (!sea) HS_FAIL(SIM_EINVAL, "sea is NULL");
    if (int rc = sea_ok(sea)) return rc;
    std::vector<double> tab;
    sea_table(sea, tab);
    StreamLayout Y;
    if (int rc = stream_layout(h, sea, chunks, n_chunks, block_edge, 0, tab, Y)) return rc;
    // window slots for as many pulse groups as fit (the sum then runs in
    // passes of that many groups); refused if one group does not fit
    int ng_cap = 1 << 30;
    if (Y.total > SIM_NOALLOC_SCRATCH_BYTES) {
        int lo = 0, hi = 0;
        for (const PlanGeom &G : Y.geom) hi = std::max(hi, G.ng_max);
        while (lo < hi) {   // largest cap in [1, hi] that fits; lo = 0: none
            const int mid = (lo + hi + 1) / 2;
            stream_relayout(h, chunks, n_chunks, 0, mid, Y.max_n, tab.size(), Y);
            if (Y.total <= SIM_NOALLOC_SCRATCH_BYTES) lo = mid;
            else hi = mid - 1;
        }
        stream_relayout(h, chunks, n_chunks, 0, std::max(lo, 1), Y.max_n, tab.size(), Y);
        if (lo == 0 || Y.total > SIM_NOALLOC_SCRATCH_BYTES)
            HS_FAIL(SIM_EINVAL, "the call needs " + std::to_string(Y.total) +
                                    " bytes of scratch with one pulse group per pass, beyond "
                                    "the fixed " +
                                    std::to_string((unsigned long long)SIM_NOALLOC_SCRATCH_BYTES) +
                                    " (use smaller chunks, or sim_stream_forward with a workspace)");
        ng_cap = lo;
    }
    if (!h->uploaded)
        HS_FAIL(SIM_EINVAL, "sim_stream_forward_noalloc needs sim_device_init first "
                            "(it uploads the handle's tables, which allocates)");
    int d = -1;
    if (hipGetDevice(&d) != hipSuccess) HS_FAIL(SIM_EHIP, "no HIP device");
    void *ptr = scratch_on(d);
    if (!ptr) HS_FAIL(SIM_EINVAL, "no scratch address on this device: call sim_device_init here");
    return stream_forward_common(h, sea, seed, chunks, n_chunks, block_edge, nullptr, p0, np, iq,
                                 accumulate, ptr, SIM_NOALLOC_SCRATCH_BYTES, stream, ng_cap);
}

}  // extern "C"
