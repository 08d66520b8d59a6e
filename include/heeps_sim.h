/*
 * heeps_sim.h -- C ABI of the MI355X (gfx950) facet-sum raw-data generator.
 *
 * The library computes the hot path of a SAR/ATI raw-data generator of the
 * HEEPS/MARE kind (Monnier et al., "Synthetic RAW data generator for ESA
 * HARMONY mission"): for every pulse and receive channel, the coherent sum
 * over independent moving sea-surface facets of their complex amplitudes,
 * weighted by the transmit and receive antenna patterns, with the two-way
 * bistatic phase and 1/(r_t r_r) spreading (Sec. III.A eq. 3, Sec. III.B
 * eq. 16), deposited into range slices of the received line (eq. 17) and
 * convolved with the waveform (the paragraph after eq. 17).  It also provides
 * the adjoint of that sum with respect to facet height, velocity and complex
 * amplitude, and on-device generation of facets on a regular grid (Sec. III,
 * resolved linear waves; scene generated where and when it is sensed, Sec. II.B).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Frame: flat local Cartesian frame (metres), scene origin O = (0,0,0).
 *  - Pulse p (0-based over the whole acquisition of n_pulses pulses) is
 *    transmitted at t_p = (p - (n_pulses-1)/2) / prf seconds.
 *  - A facet is (x, y, z, vx, vy, vz, a_re, a_im) in float32: position at
 *    t = 0, constant velocity (its position at pulse p is X0 + V t_p), and
 *    complex amplitude a.
 *  - Tx position at t_p; Rx phase centre at t_p + tau_ref(p, c), where
 *    tau_ref is the echo delay of O (fixed point of
 *    c tau = |O - P_tx(t_p)| + |O - P_rx(t_p + tau)|).
 *  - Range-compressed sample n of line (c, p) sits at delay
 *    tau_ref(p, c) + (n - n_ref) / fs.  A facet with bistatic range R
 *    contributes W * h(n - u) to samples n = floor(u)-3 .. floor(u)+4 inside
 *    [0, N), with u = n_ref + (R - c tau_ref) fs / c, h the Kaiser-windowed
 *    sinc of half-width 4, and
 *    W = a * F_tx * F_rx * (R_t,mid R_r,mid / (R_t R_r)) * exp(-j 2 pi f0 R / c),
 *    F the one-way field patterns sinc(kappa u/beta_az) sinc(kappa v/beta_el)
 *    (sinc^2 power pattern with 3-dB widths beta), R_.,mid the ranges of O at
 *    t = 0.
 *  - Complex buffers are interleaved float32 (re, im) = complex64.
 *    IQ layout: [channel][pulse - p0][sample], row-major, N samples per line.
 *  - Gradient convention: g = dL/dRe(IQ) + j dL/dIm(IQ) for a real loss L
 *    (PyTorch's convention for complex tensors).
 *  - Device pointers are HIP device memory on the current device; host
 *    pointers are marked "host".  The caller owns every buffer passed in.
 *  - `stream` is a hipStream_t (NULL = default stream).  Every entry point
 *    that takes a stream is asynchronous on it unless stated otherwise.
 *  - Return value: SIM_OK (0) or a negative SIM_E* code; arguments are
 *    validated before anything is written or launched.  sim_last_error()
 *    returns a thread-local message describing the last failure.
 *  - Device memory: the caller owns every buffer, workspaces included
 *    (sim_workspace_size, sim_sea_table_size, sim_stream_workspace_size give
 *    their sizes; a workspace is 256-byte aligned device memory).  The
 *    library itself holds only the handle's constant tables (per-pulse
 *    geometry, waveform spectrum, pattern grids), uploaded once by
 *    sim_device_init.  No other entry point allocates device memory or waits
 *    for the device, except the queries marked "synchronises".
 *  - Calls that use the same handle from several host threads at once, or
 *    that overlap on the device through one workspace (a plan's sorted facet
 *    copy is rewritten by every sum over the plan), race; serialise them
 *    (one stream per plan or workspace).
 */
#ifndef HEEPS_SIM_H
#define HEEPS_SIM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIM_OK 0
#define SIM_EINVAL (-1)        /* bad argument (null pointer, size, range, NaN geometry) */
#define SIM_ENOMEM (-2)        /* device or host allocation failed */
#define SIM_EHIP (-3)          /* HIP runtime / launch failure */
#define SIM_EUNSUPPORTED (-4)  /* valid but unsupported request (e.g. too many cells) */

#define SIM_MAX_PLATFORMS 8
#define SIM_MAX_ANTENNAS 8
#define SIM_MAX_CHANNELS 16

typedef struct sim_handle sim_handle;   /* opaque, owned by the library */
typedef struct sim_plan sim_plan;       /* opaque host descriptor, owned by the library;
                                           its device buffers are the caller's workspace */

/* Plan flag: the workspace also holds the intra-facet speckle records and
 * anchors (needed by sim_forward_speckle / sim_backward_speckle). */
#define SIM_PLAN_SPECKLE 1

/* Scene rectangle (metres) that every facet position (x, y) of a plan lies
 * in, and the plan's bounds on the facets' heights and speeds: z_max, the
 * largest |z| (metres), and v_max, the largest |V| (m/s).  A zero bound
 * takes the default (4 m, 2.5 m/s).  The bounds size the forward sum's
 * range windows (the drift V t over the dwell) and decide whether antenna
 * elevation factors may be taken at block centres (sim_plan_mode);
 * sim_chunk_box derives them from a sea state.  A facet beyond them is
 * still summed exactly (its taps outside a window go straight to the IQ
 * lines), but the elevation-factor bound no longer covers it:
 * sim_plan_beyond counts such facets. */
typedef struct {
    double x_min, x_max, y_min, y_max;
    double z_max, v_max;
} sim_box;

/* Straight-line trajectory: position p0 (m) at t = 0, constant velocity v (m/s). */
typedef struct {
    double p0[3];
    double v[3];
} sim_traj;

/*
 * Antenna on a platform: one-way 3-dB widths (radians) of its sinc^2 power
 * pattern.  Frame (stripmap, fixed over the dwell, all antennas pointing at
 * the same surface target as in Sec. I / Fig. 1): boresight b from the
 * platform position at t = 0 to O, azimuth axis = x projected orthogonal to
 * b, elevation axis = b x az.  Facets behind the antenna (r.b <= 0) get 0.
 */
typedef struct {
    int platform;
    double beta_az;
    double beta_el;
    /* Time-dependent pattern (TOPS-like azimuth steering, Sec. III.B): the
     * frame turns about the elevation axis at this rate (rad/s), angle
     * rate * t, so b(t) = b cos + az sin, az(t) = az cos - b sin; a transmit
     * antenna at the pulse time, a receive antenna at t_p + tau_ref.  0 =
     * fixed frame. */
    double steer_rate;
    /* u-v gridded field pattern (Sec. III.B: patterns, whatever their source,
     * become u-v grids in GPU memory), or NULL for the sinc pattern above.
     * Host float32 [pattern_nv][pattern_nu] (u fastest), the real one-way
     * field gain at direction cosines u = u0 + i du on the azimuth axis and
     * v = v0 + j dv on the elevation axis (the turned axes when steered);
     * bilinear between nodes, 0 outside [u0, u0 + (nu-1) du) x
     * [v0, v0 + (nv-1) dv) and behind the antenna.  sim_create copies it
     * (the caller's array may be freed afterwards).  nu, nv >= 2,
     * (nu-1)(nv-1) <= 2^24, du, dv > 0, all values finite, else SIM_EINVAL;
     * |u| <= 2^14 du and |v| <= 2^14 dv over the whole table (cell
     * coordinates are FP32), else SIM_EUNSUPPORTED.
     * A handle with any gridded antenna evaluates every pattern per facet
     * (no elevation factor at block centres); sim_plan_mode's far-field mode
     * then only drops the adjoint's first-order correction of the gain
     * gradient across a block. */
    const float *pattern;
    int pattern_nu, pattern_nv;
    double pattern_u0, pattern_du, pattern_v0, pattern_dv;
} sim_antenna;

/* Channel: transmit antenna, receive antenna and the receive phase-centre
 * offset (m) from the receiving platform's position (eq. 16's channels). */
typedef struct {
    int tx_antenna;
    int rx_antenna;
    double pc_offset[3];
} sim_channel;

/* Acquisition, instrument and waveform description (Sec. II.B inputs). */
typedef struct {
    double c;            /* propagation speed (m/s); 0 selects 299792458 */
    double f0;           /* carrier frequency (Hz) */
    double fs;           /* range sampling rate (Hz) */
    double prf;          /* pulse repetition frequency (Hz) */
    int n_samples;       /* N, samples per range line (2..65536) */
    int n_pulses;        /* total pulses of the acquisition */
    int n_ref;           /* reference sample of the window; < 0 selects N/2 */
    double kaiser_beta;  /* Kaiser beta of the 8-tap interpolator (0..20) */
    double chirp_bw;     /* chirp bandwidth (Hz) */
    double chirp_T;      /* chirp duration (s); 0 disables the waveform step */
    int n_platforms;
    const sim_traj *platforms;      /* host, [n_platforms] */
    int n_antennas;
    const sim_antenna *antennas;    /* host, [n_antennas] */
    int n_channels;
    const sim_channel *channels;    /* host, [n_channels] */
    /* Receiver position (eq. 3 evaluates r_r at the reception time t_r):
     * 0 = one position per pulse and channel, at the echo time of O;
     * 1 = at each facet's own echo time, the fixed point of
     *     c tau = |X - P_tx(t_p)| + |X - P_rx(t_p + tau)|
     * (solved in FP64 per spatial block and pulse, first order in the
     * facet's offset from the block centre, error < 1e-9 m). */
    int rx_exact;
} sim_config;

/* Facets, structure of arrays, device float32 [n] each. */
typedef struct {
    long long n;
    const float *x, *y, *z, *vx, *vy, *vz, *a_re, *a_im;
} sim_facets;

/* Output facets of the generator, device float32 [n] each. */
typedef struct {
    long long n;
    float *x, *y, *z, *vx, *vy, *vz, *a_re, *a_im;
} sim_facets_out;

/* Facet gradients, device float32 [n] each; a NULL member is not computed. */
typedef struct {
    long long n;
    float *dz, *dvx, *dvy, *dvz, *da_re, *da_im;
} sim_facet_grads;

/*
 * Sea surface for on-device facet generation on a grid of nx x ny cells of
 * dx x dy metres centred on O (cell centres x = (ix - (nx-1)/2) dx, grid index
 * iy*nx + ix).
 *  mode 0: flat sea, z = 0, velocities N(0, sigma_v^2) per axis.
 *  mode 1: n_comp linear wave components (Sec. III, resolved waves of a
 *          homogeneous tile without the choppy-wave option): wavenumbers
 *          log-spaced on [k_min, k_max], spectrum ~ k^slope, amplitudes
 *          scaled to significant height hs, deep-water dispersion with
 *          gravity g; directions and phases are given (host arrays); the
 *          facet moves with the first-order orbital velocity plus `current`.
 *  mode 2: heterogeneous sea (Sec. III eq. 1, 2): the plane is cut into
 *          square TL tiles of side tile_L whose corners form a lattice of
 *          (ntx + 1) x (nty + 1) nodes, node (i, j) at (tile_x0 + i tile_L,
 *          tile_y0 + j tile_L), index j (ntx + 1) + i.  Each node carries its
 *          own homogeneous field as in mode 1 (a T2L tile: significant height
 *          node_hs[node], directions node_dirs[node][m], phases
 *          node_phases[node][m]; k range, slope and g shared).  A facet sums
 *          the fields of the four corners of its TL tile with weights
 *          W = sqrt((1 - |x_i - x| / L)(1 - |y_i - y| / L)).  The lattice
 *          must cover the whole grid.
 *  cwm:    (modes 1, 2) Choppy Wave Model: each facet is moved from its
 *          grid point by the horizontal displacement
 *          -sum A (cos psi, sin psi) sin(theta); z and V are those of the
 *          point at rest (the facets follow the orbital motion).
 *  Complex amplitudes are CN(0, 1) in every mode.
 */
typedef struct {
    int nx, ny;
    double dx, dy;
    int mode;
    double sigma_v;
    int n_comp;
    double k_min, k_max, slope, hs, g;
    const double *dirs;     /* host, [n_comp] propagation directions (rad) */
    const double *phases;   /* host, [n_comp] initial phases (rad) */
    double current[2];      /* uniform surface current (m/s) */
    int ntx, nty;           /* mode 2: TL tiles along x, y */
    double tile_L, tile_x0, tile_y0;   /* mode 2: tile side (m), lattice origin (m) */
    const double *node_hs;       /* mode 2, host [(ntx+1)(nty+1)] */
    const double *node_dirs;     /* mode 2, host [(ntx+1)(nty+1)][n_comp] (rad) */
    const double *node_phases;   /* mode 2, host [(ntx+1)(nty+1)][n_comp] (rad) */
    int cwm;                /* 1: Choppy Wave Model horizontal displacement */
} sim_sea;

/*
 * Create a simulator: validates `cfg` and derives in FP64 on the host the
 * per-(channel, pulse) geometry (t_p, P_tx, tau_ref, P_rx), antenna frames,
 * the interpolator's polynomial form and, if chirp_T > 0, the waveform
 * spectrum.  Host only (a handle may be created without a GPU).
 * out: receives the handle (freed by sim_destroy).
 * Errors: SIM_EINVAL, SIM_ENOMEM, SIM_EUNSUPPORTED (antenna width below
 * kappa/500 rad).
 */
int sim_create(const sim_config *cfg, sim_handle **out);

/*
 * Upload the handle's constant tables (per-pulse geometry, waveform spectrum
 * and twiddles, pattern grids) to the current HIP device: the one set-up
 * step that allocates device memory and synchronises.  Every later call on
 * the handle must run with that device current.  A device call made before
 * it performs it implicitly.  Repeated calls do nothing.
 * Errors: SIM_EINVAL (NULL, or another device current than the first call's),
 * SIM_ENOMEM, SIM_EHIP.
 */
int sim_device_init(sim_handle *h);

/* Release a handle and its device tables (waits for the device).  NULL is
 * ignored.  Plans of the handle must not be used afterwards (destroying them
 * is still allowed). */
void sim_destroy(sim_handle *h);

/* Thread-local text of the last error ("" if none). */
const char *sim_last_error(void);

/*
 * Per-pulse window metadata (the raw data are output with their timing,
 * after eq. 17): for channel ch and pulses [p0, p0+np), host outputs t[np]
 * (pulse times, s) and tau_ref[np] (echo delay of O, s); sample n of that
 * line is at delay tau_ref + (n - n_ref)/fs.  Either pointer may be NULL.
 */
int sim_pulse_info(const sim_handle *h, int ch, int p0, int np, double *t,
                   double *tau_ref);

/* Waveform length L and FFT size M used by sim_apply_waveform (0 if none). */
int sim_waveform_info(const sim_handle *h, int *chirp_len, int *fft_len);

/*
 * Bytes of device workspace for the plan of up to n facets whose positions
 * lie in `box` (host), with lattice cells of block_edge metres and the given
 * SIM_PLAN_* flags (see sim_plan_create).  Host only.
 * Errors: SIM_EINVAL (NULL handle or bytes, n outside [1, 2^31 - 64),
 * block_edge outside (0, 64], box not finite or empty in a direction,
 * unknown flags), SIM_EUNSUPPORTED (lattice larger than 2^28 cells).
 */
int sim_workspace_size(const sim_handle *h, long long n, const sim_box *box, double block_edge,
                       int flags, size_t *bytes);

/*
 * Plan a facet set (the range-binned block sort of the sum, eq. 17's range
 * slices gathered per tile as in Sec. IV.A/B): facets are binned into
 * spatial blocks (cells of block_edge x block_edge metres of a lattice
 * covering `box`, at most 64 facets per block, a cell's facets in ascending
 * index; each block carries an exact float32 centre used as its FP64
 * reference point), and for every band of pulse groups and every channel
 * the blocks are binned by the sample position of their centre into range
 * strips, listed in block order and cut into segments (sim_plan_geometry
 * reports the bands, strips and segments); the forward sum gives each
 * (segment, pulse group, channel) its own window and adds the windows in a
 * fixed order, so its result does not depend on scheduling.  Cells of more
 * than 1024 facets keep the order of an atomically ranked scatter, so sums
 * over such cells may differ in the last bits from run to run.  Everything
 * is written into
 * `workspace` (caller-owned device memory, 256-byte aligned, at least
 * sim_workspace_size bytes; it must stay allocated and untouched while the
 * plan is used).  Depends only on x, y (device float32 [n]).  block_edge in
 * (0, 64] metres; 8 suits 1 m grids.  flags: 0, or SIM_PLAN_SPECKLE to make
 * room for the intra-facet speckle.  Asynchronous on `stream`: no allocation
 * and no wait.  A facet outside `box` is placed in the nearest edge cell:
 * it is still summed, but its offset from that block's centre may exceed
 * what the FP32 precision scheme is bounded for; sim_plan_info counts such
 * facets.  out receives a host descriptor (freed by sim_plan_destroy).
 * Errors: as sim_workspace_size, and SIM_EINVAL for NULL x, y or out, a
 * NULL, misaligned or too small workspace; SIM_EHIP.
 */
int sim_plan_create(sim_handle *h, const float *x, const float *y, long long n,
                    const sim_box *box, double block_edge, int flags, void *workspace,
                    size_t workspace_bytes, void *stream, sim_plan **out);

/*
 * Host outputs (host only, nothing allocated): the range-strip geometry a
 * plan of these arguments would take.  win: the widest LDS window of the
 * forward kernel (samples); n_bands bands of band_groups pulse groups;
 * n_strips: strips per band and channel (a bound); seg_len: blocks per work
 * unit; seg_max: bound on the work units of a band and channel; bands (NULL
 * to skip): host double [n_bands][n_channels][3] = (umin, S, margin): a
 * block whose centre sits at sample position u at the band's reference pulse
 * (64 band_groups b + 32 band_groups, capped at n_pulses - 1) is in strip
 * floor((u - umin) / S), and the forward sum assumes its facets' taps within
 * [umin + s S - margin - 3, umin + (s + 1) S + margin + 4] at every pulse of
 * the band (facets within half a block diagonal of the centre, heights and
 * speeds within the box's bounds); band_win (NULL to skip): host int
 * [n_bands][n_channels], the band's window width W (the window of strip s
 * covers W samples from floor(umin + s S - margin) - 3; at most win).
 * Errors as sim_workspace_size.
 */
int sim_plan_geometry(const sim_handle *h, long long n, const sim_box *box, double block_edge,
                      int *win, int *n_bands, int *band_groups, int *n_strips, int *seg_len,
                      int *seg_max, double *bands, int *band_win);

/* Release a plan's host descriptor.  NULL is ignored.  Touches no device
 * memory: the workspace stays the caller's. */
void sim_plan_destroy(sim_plan *plan);

/* Host outputs: number of facets, blocks, range strips per band and channel
 * (a bound; strips the scene does not reach hold no block) and facets
 * outside the plan's box.  n_blocks and n_outside are read back from the
 * device: synchronises the stream the plan was created on (NULL pointers
 * skip them, and then nothing waits). */
int sim_plan_info(const sim_plan *plan, long long *n_facets, long long *n_blocks,
                  long long *n_strips, long long *n_outside);

/* Host output: the facets of the last sim_forward or sim_backward call on
 * this plan (made on `stream`) whose |z| or |V| exceeds the bounds of the
 * plan's box (z_max, v_max); counted by the gather kernel of every call.
 * Synchronises `stream`.  Errors: SIM_EINVAL (NULL plan or output),
 * SIM_EHIP. */
int sim_plan_beyond(const sim_plan *plan, void *stream, long long *n_beyond);

/*
 * Host outputs: the plan's evaluation mode of the antenna elevation factors
 * (Sec. III.B eq. 16 gains).  The field pattern of each antenna is the
 * product of an azimuth and an elevation sinc factor.  When *el_const = 1
 * the forward and adjoint sums take both legs' elevation factors at each
 * block centre (per pulse) instead of per facet: sim_plan_create chooses
 * this only when its bound on the relative error of doing so, *el_bound,
 * is at most 5e-6 for every facet within reach of its block centre (half a
 * block diagonal plus the box's z_max of height and v_max of drift over the
 * dwell).
 * Otherwise *el_const = 0 and every factor is evaluated per facet.
 * Either output pointer may be NULL.  Errors: SIM_EINVAL (NULL plan).
 */
int sim_plan_mode(const sim_plan *plan, int *el_const, double *el_bound);

/* Bytes of device workspace sim_generate_facets needs for `sea` (its wave
 * component table; 0 for a flat sea).  Host only.  Errors: SIM_EINVAL. */
int sim_sea_table_size(const sim_sea *sea, size_t *bytes);

/* Host output: a rectangle holding every facet sim_generate_facets makes for
 * the grid sub-rectangle [ix0, ix0+cnx) x [iy0, iy0+cny) of `sea` (cell
 * centres widened by the largest Choppy Wave Model displacement and a
 * rounding margin), with bounds on the facets' heights and speeds: the sum
 * of a field's amplitudes and the sum of amplitude x angular frequency plus
 * the current's speed (twice the sums in mode 2, whose four weights add up
 * to at most 2); in mode 0, z_max = 1 mm (flat) and v_max = 6 sigma_v (a
 * speed exceeded with probability below 1e-7 per facet).  The box to plan such
 * facets with.  Host only.  Errors: SIM_EINVAL (empty or outside
 * sub-rectangle, bad sea). */
int sim_chunk_box(const sim_sea *sea, int ix0, int iy0, int cnx, int cny, sim_box *box);

/*
 * Generate facets of the grid sub-rectangle [ix0, ix0+cnx) x [iy0, iy0+cny)
 * of `sea` (row-major in the sub-rectangle).  Random draws use Philox4x32-10
 * keyed by `seed` with the global grid index as counter, so any chunking of
 * the grid yields the same facets.  out->n must equal cnx*cny.  The sea's
 * wave table is written into `workspace` (device, 256-byte aligned, at least
 * sim_sea_table_size bytes; may be NULL for a flat sea) through the kernel
 * arguments of small copy launches: asynchronous on `stream`, no allocation,
 * no wait.  The workspace must stay allocated until the generation has run.
 * Errors: SIM_EINVAL (NULL arguments, sub-rectangle outside the grid, bad
 * sea description: unknown mode, missing arrays, bad spectrum, a tile
 * lattice that does not cover the grid, negative heights; NULL, misaligned
 * or too small workspace), checked before any device work; SIM_EHIP.
 */
int sim_generate_facets(sim_handle *h, const sim_sea *sea, unsigned long long seed,
                        int ix0, int iy0, int cnx, int cny, const sim_facets_out *out,
                        void *workspace, size_t workspace_bytes, void *stream);

/*
 * Forward facet sum (eq. 3/16 summed into range slices, eq. 17) for pulses
 * [p0, p0+np) of every channel, into iq_rc (device complex64
 * [n_channels][np][N]).  accumulate = 0 overwrites iq_rc, 1 adds to it.
 * `facets` must be the facet set `plan` was made from (same n, same x, y);
 * z, V and a may change between calls.  Rewrites the plan's sorted facet
 * copy in its workspace; asynchronous on `stream`, no allocation, no wait.
 */
int sim_forward(sim_handle *h, sim_plan *plan, const sim_facets *facets, int p0,
                int np, float *iq_rc, int accumulate, void *stream);

/*
 * Intra-facet speckle (Sec. III.A eq. 7 and eq. 10).  Each facet's amplitude
 * at pulse p is multiplied by s(t_p) = x(p) exp(j 2 pi f_s t_p), where x is a
 * complex order-1 autoregressive process over the pulses with unit power and
 * correlation b^|p - q|, b = exp(-1 / (prf tau_s)) (real and imaginary parts
 * N(0, 1/2) each; one process per facet, shared by all channels).  Random
 * draws are Philox2x32-10 with key = low ^ high word of `seed` and counter
 * (facet id, slot), facet id = first_index + i for facet i of the arrays
 * (mod 2^32): so a scene split into several facet sets draws the same
 * speckle when each set passes its own first_index.  The process is sampled
 * at every 64th absolute pulse (anchors, eq. 10 over 64 pulses; slot 2^31 + g)
 * and pulse by pulse in between (eq. 10; slot p), each 64-pulse stretch
 * conditioned on its closing anchor, which keeps the law of the recursion;
 * so any pulse sub-range gives the rows of the full range.
 */
typedef struct {
    double tau_s;              /* correlation time (s), > 0; +inf freezes x */
    unsigned long long seed;
    long long first_index;     /* id of facet 0, >= 0 */
    const float *f_s;          /* device float32 [n] intra-facet Doppler (Hz); NULL = 0 */
} sim_speckle;

/*
 * sim_forward with the intra-facet speckle `speckle` (same arguments
 * otherwise).  The plan must have been made with SIM_PLAN_SPECKLE: its
 * workspace then holds (n + 1) * 8 bytes of speckle records and
 * (n + 1) * 16 * (ceil(n_pulses / 64) + 1) bytes of anchors.
 * Errors as sim_forward, and SIM_EINVAL for a NULL speckle, tau_s <= 0 or NaN,
 * first_index < 0, or a plan without SIM_PLAN_SPECKLE.
 */
int sim_forward_speckle(sim_handle *h, sim_plan *plan, const sim_facets *facets,
                        const sim_speckle *speckle, int p0, int np, float *iq_rc,
                        int accumulate, void *stream);

/*
 * Convolve n_lines range lines with the chirp (the waveform convolution that
 * follows eq. 17): raw[n] = sum_m rc[m] chirp[n - m + L/2],
 * chirp[k] = exp(j pi (B/T) (k/fs - T/2)^2), k < L = round(T fs), by
 * zero-padded FFT of size M = 2^ceil(log2(N + L - 1)).  Device complex64
 * [n_lines][N] in and out; in-place (iq_raw == iq_rc) is allowed.
 * SIM_EUNSUPPORTED if the handle has no waveform or M > 16384.
 */
int sim_apply_waveform(sim_handle *h, const float *iq_rc, float *iq_raw,
                       long long n_lines, void *stream);

/* Adjoint of sim_apply_waveform: g_rc[m] = sum_n g_raw[n] conj(chirp[n - m + L/2]). */
int sim_apply_waveform_adjoint(sim_handle *h, const float *g_raw, float *g_rc,
                               long long n_lines, void *stream);

/*
 * Adjoint of sim_forward: given g_rc = dL/dRe(IQ_rc) + j dL/dIm(IQ_rc)
 * (device complex64 [n_channels][np][N]) writes, per facet in the original
 * order, dL/dz, dL/dV (= sum_p t_p dL/dX) and dL/dRe(a), dL/dIm(a)
 * (device float32 [n]; NULL members skipped).  Facet geometry is recomputed,
 * not stored.  accumulate = 1 adds to the outputs.
 */
int sim_backward(sim_handle *h, sim_plan *plan, const sim_facets *facets, int p0,
                 int np, const float *g_rc, const sim_facet_grads *grads,
                 int accumulate, void *stream);

/* Adjoint of sim_forward_speckle (the speckle factor does not depend on z,
 * V or a; dL/da = conj(sum B T E s) as for sim_backward).  Arguments and
 * errors as sim_backward and sim_forward_speckle. */
int sim_backward_speckle(sim_handle *h, sim_plan *plan, const sim_facets *facets,
                         const sim_speckle *speckle, int p0, int np, const float *g_rc,
                         const sim_facet_grads *grads, int accumulate, void *stream);

/*
 * Bytes of device workspace of the streamed calls below for the given sea,
 * chunks and block_edge (flags: SIM_PLAN_SPECKLE for the speckle variants):
 * the sea table, the facets of the largest chunk (32 bytes per facet) and
 * the largest chunk's plan (sim_workspace_size over sim_chunk_box).  Host
 * only.  Errors as sim_workspace_size and sim_chunk_box.
 */
int sim_stream_workspace_size(const sim_handle *h, const sim_sea *sea, const int *chunks,
                              int n_chunks, double block_edge, int flags, size_t *bytes);

/*
 * Streamed forward over a large generated scene (the paper processes the scene
 * as a sequence of tile batches on the GPU, Sec. IV.B, and generates it where
 * and when it is sensed, Sec. II.B): for each grid chunk k, given host
 * chunks[4k..4k+3] = (ix0, iy0, cnx, cny), the library generates the chunk's
 * facets (as sim_generate_facets), plans them with `block_edge` over their
 * sim_chunk_box (as sim_plan_create) and adds their sum for pulses
 * [p0, p0+np) into iq_rc (device complex64 [n_channels][np][N]);
 * accumulate = 0 clears iq_rc first.  Facets and plans live in `workspace`
 * (caller-owned device memory, 256-byte aligned, at least
 * sim_stream_workspace_size(..., flags = 0) bytes), reused chunk after chunk
 * in stream order: asynchronous on `stream`, no allocation, no wait.
 */
int sim_stream_forward(sim_handle *h, const sim_sea *sea, unsigned long long seed,
                       const int *chunks, int n_chunks, double block_edge, int p0, int np,
                       float *iq_rc, int accumulate, void *workspace, size_t workspace_bytes,
                       void *stream);

/*
 * Adjoint of sim_stream_forward with respect to the facet velocities: for
 * each chunk the facets are regenerated and replanned (geometry recomputed,
 * nothing stored), and dL/dvx, dL/dvy, dL/dvz are written (device float32,
 * chunk after chunk, each chunk row-major in its sub-rectangle; total length
 * sum of cnx*cny).  NULL outputs are skipped.  g_rc as in sim_backward;
 * workspace as sim_stream_forward.
 */
int sim_stream_backward(sim_handle *h, const sim_sea *sea, unsigned long long seed,
                        const int *chunks, int n_chunks, double block_edge, int p0, int np,
                        const float *g_rc, float *dvx, float *dvy, float *dvz, void *workspace,
                        size_t workspace_bytes, void *stream);

/*
 * sim_stream_forward with the intra-facet speckle (Sec. III.A eq. 7 and
 * eq. 10, as sim_forward_speckle) over a generated scene: the facet at grid
 * point (ix, iy) takes the id speckle->first_index + iy * nx + ix (nx =
 * sea->nx), whatever chunk it falls in, and speckle->f_s, if not NULL, is
 * indexed the same way (device float32 [sea->nx * sea->ny], Hz).  So any
 * split of the grid into chunks gives the speckle of the whole scene.  The
 * workspace is sized with flags = SIM_PLAN_SPECKLE.
 * Errors as sim_stream_forward and sim_forward_speckle.
 */
int sim_stream_forward_speckle(sim_handle *h, const sim_sea *sea, unsigned long long seed,
                               const int *chunks, int n_chunks, double block_edge,
                               const sim_speckle *speckle, int p0, int np, float *iq_rc,
                               int accumulate, void *workspace, size_t workspace_bytes,
                               void *stream);

/* Adjoint of sim_stream_forward_speckle with respect to the facet velocities
 * (outputs as sim_stream_backward, speckle and workspace as
 * sim_stream_forward_speckle). */
int sim_stream_backward_speckle(sim_handle *h, const sim_sea *sea, unsigned long long seed,
                                const int *chunks, int n_chunks, double block_edge,
                                const sim_speckle *speckle, int p0, int np, const float *g_rc,
                                float *dvx, float *dvy, float *dvz, void *workspace,
                                size_t workspace_bytes, void *stream);

/*
 * Fast mode (Sec. IV.B, the fast-mode paragraph): the Doppler spectrum of
 * every range gate is estimated at PRF / n_fast, and the pulses in between
 * are generated by inverse FFT and linear combination, as the heterogeneous
 * sea of eq. 1-2 but in one dimension (slow time).  Windows of 64 full-rate
 * pulses start every n_fast pulses (s_k = k n_fast, k < K =
 * floor((n_pulses - 64) / n_fast) + 1); their rows of iq_rc are the facet sum
 * of sim_forward.  Node k sits at p_k = s_k + 32.  Per gate and node, the
 * window's Hann-tapered DFT X (taper sqrt(8/3) sin^2(pi (m + 1/2) / 64))
 * gives the power |X|^2 / 64^2 per window bin; on L_s bins (L_s the power
 * of two >= 2 n_fast + 64) the node's signal takes that power interpolated
 * linearly and scaled by 64 / L_s, the argument of the interpolated
 * X_c conj(X_0) as its phase relative to channel 0, and a bin phase
 * 2 pi (w + 1/2) 2^-32 with w word (bin mod 4) of Philox4x32-10 keyed by
 * `seed`, counter (bin / 4, gate, k, 0x46415354), shared by the channels;
 * its inverse DFT g_k(tau) is taken at tau = p - p_k.  A pulse p between
 * windows, with p_k < p < p_{k+1} and d = (p - p_k) / n_fast, gets
 * sqrt(1 - d) g_k + sqrt(d) g_{k+1} (after the last node: g_{K-1}).
 * n_fast in [64, 1024] (n_fast = 64 leaves no pulse out: the plain sum).
 * sim_fast_workspace_size gives the workspace (the window spectra,
 * 8 * C * K * 64 * N bytes); iq_rc is device complex64
 * [n_channels][n_pulses][N], overwritten.  Asynchronous, no allocation, no
 * wait.  Errors: as sim_forward, SIM_EINVAL for n_fast outside [64, 1024],
 * fewer than 64 pulses, or a NULL, misaligned or too small workspace.
 */
int sim_fast_workspace_size(const sim_handle *h, int n_fast, size_t *bytes);
int sim_forward_fast(sim_handle *h, sim_plan *plan, const sim_facets *facets, int n_fast,
                     unsigned long long seed, float *iq_rc, void *workspace,
                     size_t workspace_bytes, void *stream);

/* Bytes of the fixed device scratch of sim_stream_forward_noalloc (96 MiB
 * per GPU, held from the library's load until the process ends). */
#define SIM_NOALLOC_SCRATCH_BYTES (96ull << 20)

/*
 * sim_stream_forward without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the chunk facets, the sea table and the
 * plans live in a fixed device array of SIM_NOALLOC_SCRATCH_BYTES per GPU
 * instead of a caller workspace.  Same arguments, results and stream
 * semantics as sim_stream_forward; it never allocates and never waits.
 * The handle must have been initialised on this device by sim_device_init
 * (the one call that allocates).  Every call on one GPU shares that GPU's
 * array and leaves its contents behind (everything the call needs zeroed is
 * cleared on its stream): calls that overlap on one GPU race, so serialise
 * them (one stream, or events between streams).  When the call's workspace
 * (sim_stream_workspace_size with flags 0: the sea table, 32 bytes per facet
 * of the largest chunk and its plan, whose window slots grow with the pulse
 * groups and channels) exceeds the scratch, the plans hold window slots for
 * as many pulse groups as fit and the sum runs in passes over the groups:
 * the same bits, more launches.
 * Errors: as sim_stream_forward; SIM_EINVAL if the call does not fit even
 * with slots for one pulse group (about 1e6 facets per chunk over 16384
 * pulses and 3 channels) or the handle was not initialised here.
 */
int sim_stream_forward_noalloc(sim_handle *h, const sim_sea *sea, unsigned long long seed,
                               const int *chunks, int n_chunks, double block_edge, int p0,
                               int np, float *iq_rc, int accumulate, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HEEPS_SIM_H */
