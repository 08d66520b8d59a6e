// Internal types and launcher declarations of the facet-sum library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "heeps_sim.h"

namespace hs {

// Per (channel, pulse) FP64 geometry, indexed by the global pulse index.
struct PulseRec {
    double t;        // pulse time t_p (s)
    double ptx[3];   // Tx phase centre at t_p
    double prx[3];   // Rx phase centre at t_p + tau_ref
    double rref;     // c * tau_ref: bistatic range of O
    double cst, snt; // cos, sin of the Tx antenna's steering angle at t_p
    double csr, snr; // cos, sin of the Rx antenna's steering angle at t_p + tau_ref
};

// Sorted facet copy, one record per facet in block order (32 bytes, so one
// scalar load brings a whole facet into SGPRs).  (dx, dy) = position minus the
// block centre, exact in float32.
struct alignas(32) FacetRec {
    float dx, dy, z;
    float vx, vy, vz;
    float ar, ai;
};

// Spatial block: exact float32 centre (the FP64 reference point of its
// facets) and the range [start, start + count) of its facets, count <= 64.
struct alignas(16) BlockRec {
    float xb, yb;
    int start, count;
};

// Interpolator in polynomial form.  With sigma = 2f - 1 (f the fractional
// sample position) the tap of offset j in {1,2,3,4} is
//   Q_j(sigma) = E_j(sigma^2) + sigma O_j(sigma^2)  (samples floor(u)+j),
// and its mirror (samples floor(u)+1-j) is Q_j(-sigma).
// Horner order: c[0] + y (c[1] + y (c[2] + y c[3])).
struct TapPoly {
    float e[4][4];
    float o[4][4];
};

// Lattice of spatial blocks: cell (cx, cy) covers [(bx0 + cx) B, (bx0 + cx + 1) B)
// x [(by0 + cy) B, ...), key cy nbx + cx.
struct Lattice {
    double edge;            // block edge B (m)
    long long bx0, by0;     // lattice origin in cells
    int nbx, nby;           // cells along x, y
};

// Range strips of the forward sum.  Pulse groups (64 pulses, absolute index
// p / 64) form bands of B groups.  For band b and channel c, a block belongs
// to strip floor((u - umin) / S), u its centre's sample position at the
// band's reference pulse min(64 B b + 32 B, Np - 1), and its facets reach the
// samples [umin + s S - margin, umin + (s + 1) S + margin) of every pulse of
// the band (margin: the centre's migration over the band, the facets'
// offsets from it, heights and drift).  Each strip's blocks are listed in
// block order and cut into segments of at most L blocks.
// Bit of a window width in a plan's mask of the widths its bands use.
constexpr int win_bit(int W) {
    return W <= 24 ? 1 : (W <= 26 ? 16 : (W <= 32 ? 2 : (W <= 48 ? 4 : 8)));
}

struct StripPlan {
    const double *band;         // [NB][C][4]: umin, S, margin (samples), window width W
    int *ids;                   // [NB][C][nbm]: block ids, strip after strip
    int *soff;                  // [NB][C][NS + 1]: first list position per strip; [NS] total
    int *segoff;                // [NB][C][NS + 1]: first segment per strip; [NS] total
    int NB, B, NS;              // bands, groups per band, strips per band and channel
    int nbm;                    // list stride (the plan's bound on blocks)
    int L;                      // blocks per segment
    int seg_max;                // bound on the segments of a band and channel
};

// Per-antenna constants, passed inside the kernel arguments (constant
// address space, so uniform reads become scalar loads).
struct AntArgs {
    double az[3], el[3], b[3];  // frame at t = 0
    double ka, ke;              // kappa / beta_az, kappa / beta_el
    double steer;               // rate of turn about el (rad/s), 0 = fixed frame
    float kaz[3], kel[3];       // (kappa/beta)/2 * axis, FP32, for the facet part
    float b32[3];               // boresight, FP32
    float kb[3];                // (kappa/beta_az)/2 * boresight, FP32 (steering)
    float az32[3];              // azimuth axis, FP32 (steering)
    float pad;
    // u-v gridded field pattern (NULL = the analytic sinc pattern).  With a
    // grid, ka = 2/du and ke = 2/dv, so the facet part's scaled direction
    // cosines come out in cell units.
    const float4 *grid;         // [nv-1][nu-1] cells: corners (i,j), (i+1,j), (i,j+1), (i+1,j+1)
    double gidu, gidv;          // 1/du, 1/dv
    float gu0, gv0;             // u0/du, v0/dv
    float gnu1, gnv1;           // nu - 1, nv - 1
    int gstride;                // nu - 1 (cells per row)
    int pad2;
};

struct ChanArgs {
    int tx, rx;                 // antenna indices
    double rtrr_mid;            // R_t,mid * R_r,mid
    double vr[3];               // velocity of the receive phase centre
};

// Intra-facet speckle (Sec. III.A eq. 7, eq. 10).  Per sorted facet: the
// counter id of its draws and its intra-facet Doppler f_s (Hz).
struct alignas(8) SpkRec {
    uint32_t id;
    float fs;
};

// Speckle constants of one call, b = exp(-1 / (prf tau_s)).
struct SpkArgs {
    const SpkRec *rec;          // [n + 1] sorted order (last one zero)
    const float4 *anch;         // [n + 1][n_groups + 1]: (y_g, D_g) per absolute group g
    int n_groups;               // ceil(Np / 64)
    uint32_t key;               // Philox2x32-10 key
    float b1, b2, b4, b8, b64;  // b^m
    float c1, c64;              // sqrt(1 - b^2), sqrt(1 - b^128)
    float bpow[65];             // b^m, m = 0..64
    float gain[64];             // bridge gains K_k = b^(64-k) (1 - b^2k) / (1 - b^128)
};

// Arguments of the fused forward kernel.
// forward work queues: one per XCD of the MI355X
constexpr unsigned kFwdQueues = 8;

// Waves of a forward workgroup for an LDS window of W samples: each wave
// sums every K-th block of a segment into a window of its own, and the
// windows are added at the end of the unit.  Four waves, one per SIMD, for
// windows of up to 32 samples (48 or 64 KB of LDS per workgroup); a
// workgroup of three waves would put two of its waves on one SIMD and make
// the others wait at the unit's end (measured 10 % slower on the 32-sample
// window).  Wider windows: one wave.  Segments are a multiple of K blocks.
constexpr int fwd_waves(int W) { return W <= 32 ? 4 : 1; }

struct FwdArgs {
    const FacetRec *facets;
    const BlockRec *blocks;
    StripPlan st;               // range strips (work units: strip segments)
    float2 *wsum;               // [C][n_groups][seg_max][64][WIN] window of each work unit
    unsigned *counter;          // [kFwdQueues] work-queue counters, zero at launch
    int g0;                     // first pulse group of this pass (units carry groups from 0)
    int slot_w;                 // window samples per slot (the plan's widest window)
    const PulseRec *pulses;     // [C][Np]
    float *iq;                  // [C][np][N] complex64 interleaved
    AntArgs ant[SIM_MAX_ANTENNAS];
    ChanArgs ch[SIM_MAX_CHANNELS];
    TapPoly tp;
    double f0_c, fs_c, n_ref;   // f0/c, fs/c, reference sample
    float linv_hi, linv_lo;     // f0/c split so that linv_hi + linv_lo ~ f0/c
    float fs_cf;                // fs/c in float
    int N, Np, p0, np;
    int n_groups;               // pulse groups of 64 lanes in the launch
    int gstride;                // pulses between the starts of consecutive groups (64:
                                // contiguous; the fast mode's node spacing otherwise)
    int C;
    int rx_exact;               // receiver at each facet's own echo time
    int steer;                  // some antenna frame turns with time
    int grid;                   // 0: no gridded pattern, 1: some antennas, 2: all
    double inv_c;               // 1 / c
    SpkArgs spk;                // speckle variant only
};

// Arguments of the fixed-order sum of the forward windows into the lines.
// samples per workgroup of the window reduction (one wave each)
constexpr int kReduceTile = 4;

struct ReduceArgs {
    StripPlan st;
    const float2 *wsum;
    float2 *iq;                 // [C][np][N]
    int C, N, Np, p0, np;
    int n_groups, gstride, poff, win;   // win: window samples per slot
    int n_tiles;                // sample tiles (kReduceTile) per line: the plan's span_tiles
    int g0;                     // first pulse group of this pass
};

// Arguments of the adjoint kernel.
struct AdjArgs {
    const FacetRec *facets;
    const BlockRec *blocks;
    const int *perm;            // sorted position -> original facet index
    const PulseRec *pulses;
    const float *g;             // [C][np][N] complex64 interleaved
    float *dz, *dvx, *dvy, *dvz, *dar, *dai;
    AntArgs ant[SIM_MAX_ANTENNAS];
    ChanArgs ch[SIM_MAX_CHANNELS];
    TapPoly tp;
    double f0_c, fs_c, n_ref;
    float linv_hi, linv_lo, fs_cf, k0;
    int N, Np, p0, np, C;
    const int *n_blocks;        // device: number of blocks (the plan's block count)
    long long nb_max;           // host bound on it (the launch covers this many)
    int accumulate;
    int rx_exact;               // receiver at each facet's own echo time
    int steer;                  // some antenna frame turns with time
    int grid;                   // 0: no gridded pattern, 1: some antennas, 2: all
    double inv_c;               // 1 / c
    SpkArgs spk;                // speckle variant only
};

// kernel arguments travel in the 4 KiB kernarg segment
static_assert(sizeof(FwdArgs) <= 4096 && sizeof(AdjArgs) <= 4096, "kernel arguments too large");

}  // namespace hs

// ---- opaque handle / plan --------------------------------------------------

struct sim_handle {
    // configuration
    double c, f0, fs, prf;
    int N, Np, n_ref;
    double beta;
    double chirp_bw, chirp_T;
    std::vector<sim_traj> plats;
    std::vector<sim_antenna> ants;
    std::vector<sim_channel> chans;
    int C;
    int rx_exact;
    int steer;                  // some antenna has a nonzero steering rate
    int grid;                   // 0: no gridded pattern, 1: some antennas, 2: all
    std::vector<std::vector<float>> pat_h;   // per antenna: host copy of its grid (or empty)
    std::vector<float4 *> pat_d;             // per antenna: device cells (or NULL)
    // derived on the host in FP64
    double kappa;
    std::vector<hs::AntArgs> antc;
    std::vector<hs::ChanArgs> chc;
    std::vector<hs::PulseRec> pulses_h;     // [C][Np]
    hs::TapPoly tp;
    double tap_fit_err;
    int chirp_len, fft_len;
    std::vector<float> spec_h, tw_h;    // waveform spectrum and twiddles (host copies)
    bool uploaded = false;              // device tables exist (on `device`)
    int device = -1;
    // device tables
    hs::PulseRec *pulses_d = nullptr;
    float *chirp_spec_d = nullptr;      // [M] complex64: FFT_M(chirp) / M
    float *twiddle_d = nullptr;         // [M] complex64: exp(-2 pi i m / M)
    std::vector<double> gen_tab_h;       // host scratch for sea tables
};

struct sim_plan {
    const sim_handle *h;
    long long n;                 // facets
    long long nb_max;            // bound on the block count (size of `blocks`)
    int flags;                   // SIM_PLAN_* flags the workspace was laid out for
    hs::Lattice lat;
    int win;                     // widest LDS range window of the bands (the slot width)
    int win_mask = 0;            // window widths the bands use (win_bit)
    bool el_const = false;       // elevation factors taken at block centres
    double el_bound = 0.0;       // bound on the relative error of doing so
    hipStream_t stream = nullptr;   // stream the plan was built on
    // every buffer lies in the caller's workspace
    int *perm = nullptr;         // [n] sorted position -> facet index
    hs::BlockRec *blocks = nullptr;     // [nb_max], the first *n_blocks valid
    const int *n_blocks = nullptr;      // device: block count
    unsigned *n_outside = nullptr;      // device: facets outside the plan's box
    unsigned *counter = nullptr;        // device: the forward's work-queue counters
    unsigned *beyond = nullptr;         // device: facets of the last call beyond zlim, vlim
    double zlim = 4.0, vlim = 2.5;      // bounds on |z| and |V| the plan was sized for
    hs::StripPlan st{};          // range strips
    float2 *wsum = nullptr;      // forward windows, for ng_slots pulse groups at a time
    int span_tiles = 0;          // tiles of kReduceTile samples covering any band's windows
    int ng_slots = 0;
    hs::FacetRec *sorted = nullptr;     // [n + 1] scratch refreshed by each call
    hs::SpkRec *spk = nullptr;          // [n + 1] speckle records (SIM_PLAN_SPECKLE)
    float4 *anch = nullptr;             // [n + 1][ceil(Np/64) + 1] speckle anchors
};

// ---- launchers (each returns hipError_t of the launch) --------------------
namespace hs {

void set_error(const std::string &msg);

hipError_t launch_fill_zero(float *p, long long n_floats, hipStream_t s);

// Plan construction kernels.
hipError_t launch_cell_keys(const float *x, const float *y, long long n, const Lattice &L,
                            int *keys, int *rank, int *count, unsigned *outside, hipStream_t s);
hipError_t launch_exclusive_scan(const int *in, int *out, long long n, int *tmp,
                                 long long tmp_len, hipStream_t s);
long long scan_tmp_len(long long n);
hipError_t launch_scatter(const int *keys, const int *rank, const int *offset, long long n,
                          int *perm, hipStream_t s);
hipError_t launch_block_counts(const int *count, long long n_keys, int *nblk, hipStream_t s);
hipError_t launch_make_blocks(const int *count, const int *offset, const int *blk_offset,
                              long long n_keys, const Lattice &L, BlockRec *blocks,
                              hipStream_t s);
hipError_t launch_cell_sort(const int *count, const int *offset, long long n_keys, int *perm,
                            hipStream_t s);
hipError_t launch_strips(const StripPlan &sp, const PulseRec *pulses, const BlockRec *blocks,
                         const int *n_blocks, int Np, int C, double n_ref, double fs_c, int *skey,
                         int *scount, hipStream_t s);
// Gather into the sorted records; counts into *beyond (zeroed here) the
// facets with |z| > zlim or |V| > vlim.
hipError_t launch_gather(const sim_facets &f, const int *perm, const BlockRec *blocks,
                         const int *n_blocks, long long nb_max, FacetRec *sorted, float zlim,
                         float vlim, unsigned *beyond, hipStream_t s);
// Copies n doubles from host memory to device memory through kernel
// arguments (stream-ordered, no pinned buffer and no host wait).
hipError_t launch_upload(double *dst, const double *src, long long n, hipStream_t s);

// Speckle records and anchors of the sorted facets for absolute pulse groups
// [g_lo, g_hi] (anchors g_lo .. g_hi + 1; with_d adds D_g = y_{g+1} - z_64).
struct SpkPrep {
    long long n;
    const int *perm;
    const float *fs;            // caller's order, NULL = 0
    long long first_index;
    int g_lo, g_hi;
    bool with_d;
    // grid mapping of a generated chunk (sub_nx > 0): facet i of the chunk
    // (row-major in its sub-rectangle) is grid point
    // (sub_y0 + i / sub_nx) * grid_nx + sub_x0 + i % sub_nx, which gives its
    // id (first_index + that index) and indexes fs
    int grid_nx, sub_x0, sub_y0, sub_nx;
};
hipError_t launch_speckle_prep(const SpkPrep &p, const SpkArgs &k, SpkRec *rec, float4 *anch,
                               hipStream_t s);

// Hot path.
hipError_t launch_forward(const FwdArgs &a, int C, int win, bool el_const, bool speckle,
                          hipStream_t s);
// Sums the forward windows into the lines in a fixed order (after
// launch_forward on the same stream).
hipError_t launch_window_reduce(const ReduceArgs &a, hipStream_t s);
hipError_t launch_adjoint(const AdjArgs &a, bool el_const, bool speckle, hipStream_t s);
// (the adjoint picks its reception-time variant from a.rx_exact)
hipError_t launch_waveform(const float *in, float *out, long long n_lines, int N, int M,
                           int shift, const float *spec, const float *tw, int adjoint,
                           hipStream_t s);

// Fast mode (Sec. IV.B): window spectra and synthesis of the pulses between
// the windows of 64 full-rate pulses that start every n_fast pulses.
struct FastArgs {
    float2 *iq;                 // [C][Np][N]: window rows hold the full-rate sum
    float2 *X;                  // [C][K][64][N] tapered window spectra
    int C, Np, N;
    int n_fast, K;              // node spacing, number of windows
    int L_s, log_L;             // synthesis length (power of two) and its log2
    unsigned long long seed;
};
size_t fast_synth_lds_bytes(int L_s, int n_fast);
hipError_t launch_fast(const FastArgs &a, hipStream_t s);

// Facet generation.
struct GenArgs {
    int nx, ny;
    double dx, dy;
    int mode;
    double sigma_v;
    int n_comp;
    const double *tab;          // [nodes][n_comp][6]: k, A, omega, cos psi, sin psi, phase
    double cur0, cur1;
    int ntx, nty;               // mode 2: tiles; nodes (ntx + 1) x (nty + 1)
    double tile_L, tile_x0, tile_y0;
    int cwm;                    // horizontal displacement of the facets
    unsigned long long seed;
    int ix0, iy0, cnx, cny;
    sim_facets_out out;
};
hipError_t launch_generate(const GenArgs &a, hipStream_t s);

}  // namespace hs
