/*
 * inkjet_lbm.h -- C ABI of the MI355X (gfx950) binary-fluid lattice Boltzmann
 * library for inkjet droplet formation.
 *
 * Method: He, Yang, Qin, Wen & Zhang, "The roles of wettability and surface
 * tension in droplet formation during inkjet printing", arXiv:1702.04487.
 *   - mean density n and order parameter phi (Methods, Eqs. 1 and 7);
 *   - D2Q9 distributions f with BGK collision and the forcing of Eq. 4,
 *     equilibrium Eqs. 5-6, streaming Eq. 3;
 *   - D2Q5 distributions g with the modified streaming of Eq. 8 and the
 *     equilibrium of Eqs. 9-10;
 *   - the interfacial force mu_phi grad(phi) from neighbour gradients and the
 *     pulsed +/-/idle body force of Results, "Actuation modeling" (Fig. 1);
 *   - periodic left/right, "fully developed" top/bottom rows and wetting
 *     walls with a set contact angle (Results, "Reproducing the experiment").
 *
 * Conventions shared by every entry point:
 *   - Lattice x in [0,nx) (periodic), y in [0,ny) (jet direction).  Every
 *     field array the caller passes or receives is row-major [ny][nx]
 *     (index y*nx + x), float32 unless stated otherwise.
 *   - Distribution arrays exchanged with the caller are [9][ny][nx] (f) and
 *     [5][ny][nx] (g) with velocities c_0=(0,0) c_1=(1,0) c_2=(0,1)
 *     c_3=(-1,0) c_4=(0,-1) c_5=(1,1) c_6=(-1,1) c_7=(-1,-1) c_8=(1,-1).
 *   - "device" pointers are HIP device memory on the current device; "host"
 *     pointers are ordinary process memory.  The library never frees memory
 *     it did not allocate.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Device work is enqueued on it and is asynchronous unless the entry
 *     point says it synchronises.
 *   - Every call returns an ij_status.  On failure the handle keeps a text
 *     message (ij_last_error); no exception crosses the ABI.  A handle must
 *     not be used from two threads at once.
 */
#ifndef INKJET_LBM_H
#define INKJET_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IJ_OK = 0,
    IJ_ERR_INVALID_ARG = -1, /* bad parameter, size or geometry; nothing changed */
    IJ_ERR_OOM = -2,         /* device allocation failed */
    IJ_ERR_DEVICE = -3,      /* a HIP call failed (message has the HIP error) */
    IJ_ERR_UNSTABLE = -4,    /* a diagnostics sample saw NaN, n <= 0 or |u| > u_limit */
    IJ_ERR_STATE = -5        /* call out of order (e.g. step before init) */
} ij_status;

enum { IJ_BC_PERIODIC = 0, IJ_BC_OPEN = 1 };
enum { IJ_FLUID = 0, IJ_WALL_INNER = 1, IJ_WALL_OUTER = 2 };

/* Simulation parameters (all fields 8 bytes wide).  Lattice units. */
typedef struct ij_params {
    int64_t nx, ny;            /* lattice size, nx >= 3, ny >= 3 */
    int64_t bc_y;              /* IJ_BC_PERIODIC or IJ_BC_OPEN ("fully developed"
                                  top and bottom rows, Results) */
    int64_t force_rows;        /* body force acts on fluid nodes with y < force_rows */
    int64_t t_pos, t_neg, t_idle; /* pulse durations in steps (Fig. 1) */
    int64_t periodic_pulse;    /* nonzero: repeat the pulse with period t_pos+t_neg+t_idle */
    int64_t nozzle_x0, nozzle_w, nozzle_len; /* nozzle channel; nozzle_w = 0: none */
    int64_t diag_row0;         /* first row of the droplet diagnostics (nozzle exit) */
    int64_t diag_every;        /* ij_step samples diagnostics every K steps (0: never) */
    double rho_ink, rho_amb;   /* bulk densities: phi* = (rho_ink-rho_amb)/2, n0 = mean */
    double sigma, width;       /* surface tension and interface width W */
    double gamma;              /* mobility parameter Gamma of Eq. 10 */
    double tau_ink, tau_amb;   /* relaxation time of f in ink / ambient (Eq. 4) */
    double tau_phi;            /* relaxation time of g (Eq. 8), q = 1/(tau_phi+1/2) */
    double theta_inner, theta_outer; /* contact angles (degrees, through the ink) of
                                        wall classes IJ_WALL_INNER / IJ_WALL_OUTER */
    double f_pos, f_neg;       /* magnitudes of the positive / negative force pulses */
    double u_limit;            /* stability guard on max |u| (<= 0: 0.3) */
} ij_params;

/* One diagnostics sample (Results: breakup time, drop velocity). */
typedef struct ij_sample {
    int64_t step;
    double mass_n, mass_phi;   /* sum of n and of phi over fluid nodes */
    double mom_x, mom_y;       /* sum over fluid nodes of sum_i c_i f_i */
    double max_u;              /* max |u| over fluid nodes */
    int64_t nan_count;         /* fluid nodes with a non-finite n, phi or u, or
                                  with n <= 0 (the stability guard's count) */
    int64_t n_detached;        /* detached ink segments (rows >= diag_row0) */
    int64_t largest_count;     /* ink nodes (phi > 0) of the largest one */
    double largest_uy;         /* sum of u_y over those nodes */
    int64_t largest_top;       /* its highest row (-1: none) */
    int64_t largest_bottom;    /* its lowest row (-1: none) */
    double head_uy, tail_uy;   /* mean u_y of its ink in its top / bottom ceil(W)
                                  rows: the head and tail velocities of Fig. 3 */
} ij_sample;

/* Summary of the samples recorded so far. */
typedef struct ij_diag {
    int64_t step;              /* current time step */
    int64_t n_samples;
    int64_t breakup_step;      /* first sample with a detached drop, -1: none */
    double v_drop;             /* mean drop velocity over [t_b+1000, t_b+3000] (NaN: none) */
    int64_t vol_drop;          /* ink nodes of the drop at t_b+2000 */
    int64_t satellite;         /* >= 2 detached drops at t_b+2000 */
    int64_t unstable_step;     /* first sample failing the guard, -1: none */
    ij_sample last;            /* the latest sample */
    int64_t drop_len;          /* rows spanned by the largest drop at t_b: the
                                  drop and its filament at breakup (Fig. 4) */
} ij_diag;

typedef struct ij_sim ij_sim;

/* Fill *p with the 64x256 nozzle defaults (density 1.0/0.1, tau 1, theta 90,
 * sigma 0.01, W 4, Gamma 1, no pulse). */
ij_status ij_params_default(ij_params *p);

/* Validate *p, derive the model constants (phi*, n0, beta, kappa, q, wetting
 * offsets) and allocate device memory on the current device: two
 * distribution buffers unless ij_attach_buffers follows, the wall mask
 * (nozzle of nozzle_x0/w/len, or all fluid), scratch fields and the
 * diagnostics ring.  *out receives the handle.  On failure *out is NULL and
 * ij_last_error(NULL) describes the error. */
ij_status ij_create(const ij_params *p, ij_sim **out);

/* Release everything the library allocated.  NULL is allowed. */
void ij_destroy(ij_sim *s);

/* Text of the last error of the handle (or of the last failed create when
 * s is NULL).  Valid until the next call on the handle. */
const char *ij_last_error(const ij_sim *s);

/* Bytes of ONE distribution buffer for the given parameters: for each
 * lattice row, 14 rows of floats with a 64-float aligned pitch (9 f, 5 g:
 * the populations of one lattice row are stored together) followed by one
 * row of 16-bit words (low-order part of g_0). */
ij_status ij_required_bytes(const ij_params *p, size_t *bytes);

/* Use caller-owned device buffers (each >= ij_required_bytes, 256-byte
 * aligned) instead of library allocations.  Ownership stays with the caller;
 * they must outlive the handle.  Invalidates the current state (init again). */
ij_status ij_attach_buffers(ij_sim *s, void *pdf_a, void *pdf_b, size_t bytes_each);

/* Replace the wall mask: host array of ny*nx bytes, IJ_FLUID / IJ_WALL_INNER /
 * IJ_WALL_OUTER.  With open rows, a fluid node of the bottom (top) row must
 * have fluid directly above (below) it.  Invalidates the state. */
ij_status ij_set_wall(ij_sim *s, const uint8_t *wall_host);

/* ij_set_wall from a mask on the host (on_device = 0) or on the device
 * (on_device != 0: device array of ny*nx bytes, copied to the host for the
 * wall analysis; synchronises the device).  Same classes, checks and
 * effect as ij_set_wall (geometry of the nozzle: "Reproducing the
 * experiment", wall classes of the two contact angles). */
ij_status ij_set_solid_mask(ij_sim *s, const uint8_t *mask, int32_t on_device);

/* Initial state from a signed distance d (device, [ny][nx], positive inside
 * the ink): phi = phi* tanh(2 d / W), n = n0, u = 0, f = f_eq, g = g_eq
 * (Eqs. 5-6, 9-10) with mu from this phi including the wetting ghosts.
 * Sets t = 0 and clears the diagnostics. */
ij_status ij_init_distance(ij_sim *s, const float *d_dev, void *stream);

/* As ij_init_distance from phi itself (device, [ny][nx]) and an optional
 * velocity (device arrays, NULL = 0). */
ij_status ij_init_phi(ij_sim *s, const float *phi_dev, const float *ux_dev,
                      const float *uy_dev, void *stream);

/* Nozzle default: ink fills the rows y < nozzle_len (flat meniscus half a
 * node above the last nozzle row). */
ij_status ij_init_default(ij_sim *s, void *stream);

/* Advance nsteps time steps (Eqs. 3-4 and 8 with the boundary rules), each a
 * fused collide-stream launch; samples diagnostics every diag_every steps.
 * Asynchronous.  Returns IJ_ERR_UNSTABLE without stepping once a checked
 * sample has failed the guard (see ij_check). */
ij_status ij_step(ij_sim *s, int64_t nsteps, void *stream);

/* Same update as ij_step through the unfused reference kernels (phi and
 * wetting ghosts written to a field, then one node per thread).  Slower;
 * exists to cross-check the fused kernel. */
ij_status ij_step_reference(ij_sim *s, int64_t nsteps, void *stream);

/* Current time step. */
int64_t ij_time(const ij_sim *s);

/* Moments at the current step into caller device arrays [ny][nx] (NULL to
 * skip): n, phi = sum g, and u = (sum c f + F/2)/n with the force of the
 * current step.  Solid nodes receive 0. */
ij_status ij_get_moments(ij_sim *s, float *n_dev, float *phi_dev, float *ux_dev,
                         float *uy_dev, void *stream);

/* Distributions of the current step into caller device arrays f [9][ny][nx]
 * and g [5][ny][nx]; solid nodes carry no populations and read as 0. */
ij_status ij_get_state(ij_sim *s, float *f_dev, float *g_dev, void *stream);

/* Overwrite the distributions (same layout; entries at solid nodes are
 * ignored) and the step counter. */
ij_status ij_set_state(ij_sim *s, const float *f_dev, const float *g_dev, int64_t t,
                       void *stream);

/* Checkpoint and bit-exact resume of the state the update works on (Eqs. 3
 * and 8 advance f and g alone; the pulse phase of Fig. 1 follows from the
 * step counter).  The blob is a 64-byte header (magic "IJSTATE3", lattice
 * size, row pitch, step counter, a hash of the wall mask, payload size)
 * followed by the current distribution buffer exactly as the kernels store
 * it: the shifted f, the g and the 16-bit remainder of
 * g_0.  ij_state_bytes gives its size (64 + ij_required_bytes).
 * ij_save_state writes it to caller host memory of at least that size.
 * ij_load_state restores it into a handle with the same lattice size and
 * wall mask (IJ_ERR_INVALID_ARG otherwise, nothing changed), sets the step
 * counter, and clears the recorded diagnostics samples and the stability
 * flag.  Steps after a load are bit for bit those of the run that saved.
 * Both synchronise the stream; the blob may be reused on return. */
ij_status ij_state_bytes(const ij_sim *s, size_t *bytes);
ij_status ij_save_state(ij_sim *s, void *blob_host, size_t bytes, void *stream);
ij_status ij_load_state(ij_sim *s, const void *blob_host, size_t bytes, void *stream);

/* Record one diagnostics sample at the current step (asynchronous): sums of
 * n, phi and momentum, max |u|, the guard's count of bad nodes, and the per-row ink
 * profile of rows >= diag_row0 split into segments. */
ij_status ij_diag_sample(ij_sim *s, void *stream);

/* Per-row ink count and summed u_y of the latest sample into host arrays of
 * ny entries (rows below diag_row0 are 0).  Synchronises the stream. */
ij_status ij_get_row_profile(ij_sim *s, int64_t *count_host, double *uy_host, void *stream);

/* Copy up to cap recorded samples (oldest first) into host memory; *count
 * receives the number recorded.  Synchronises the stream. */
ij_status ij_get_samples(ij_sim *s, ij_sample *out_host, int64_t cap, int64_t *count,
                         void *stream);

/* Breakup step, drop velocity and volume, satellite flag and the latest
 * sample.  Synchronises the stream. */
ij_status ij_get_diagnostics(ij_sim *s, ij_diag *out, void *stream);

/* Synchronise and check every sample recorded so far against the guard
 * (non-finite values, a density n <= 0, or max |u| > u_limit): IJ_OK or
 * IJ_ERR_UNSTABLE. */
ij_status ij_check(ij_sim *s, void *stream);

/* Derived constants: out[0..7] = phi*, n0, beta, kappa, q, inner and outer
 * wetting offsets 2 Omega phi_star / W, mobility Gamma q (q tau_phi - 1/2). */
ij_status ij_derived(const ij_sim *s, double out[8]);

/* Autotuner: time trial_steps (2..10000) fused steps for each candidate
 * tile shape (1, 2, 4 waves x 1, 8, 16, 32, 64 rows), keep the fastest, and
 * restore the distributions (the step counter does not move).  Outputs may
 * be NULL.  Synchronises the stream. */
ij_status ij_autotune(ij_sim *s, int32_t trial_steps, void *stream, int32_t *waves_x, int32_t *rows_per_block,
                      double *ms_per_step);

/* Tile shape of the fused collide-stream kernels: waves across x per
 * workgroup (1, 2 or 4) and rows per workgroup (1..1024).  With 1 row the
 * rows away from walls and open rows are updated without a walk (one wave
 * per 64 columns of a row); with more, each workgroup walks its block of
 * rows.  The default is 4 waves (256 columns) by 1 row.  0 keeps the
 * current value.  Results do not depend on the tile shape (bit for bit). */
ij_status ij_set_tiling(ij_sim *s, int32_t waves_x, int32_t rows_per_block);

/* ------------------------------------------------------------------ batches
 *
 * A batch steps many independent lattices (a parameter sweep over contact
 * angle, surface tension and pulse, with lattices of different sizes) as
 * one: each launch of the step covers the tiles of every case, and the steps
 * between two diagnostics samples can replay as one captured graph.  Every
 * case is an ij_sim owned by the batch: set it up, initialise it and read it
 * back with the single-lattice calls on the handle from ij_batch_case; it is
 * stepped only by ij_batch_step (ij_step, ij_step_reference,
 * ij_set_tiling and ij_attach_buffers on it return IJ_ERR_STATE, and
 * ij_destroy on it does nothing).  The update of each case is the same, bit
 * for bit, as stepping it alone; a case whose diagnostics sample fails the
 * stability guard is frozen on the device and reports the step
 * (ij_get_diagnostics on its handle) while the others go on.
 */
typedef struct ij_batch ij_batch;

/* n cases (1..65535), each validated as by ij_create (a nozzle from its
 * nozzle_* fields, or no wall); every case must have the same diag_every.
 * On failure *out is NULL and ij_batch_last_error(NULL) has the reason. */
ij_status ij_batch_create(const ij_params *cases, int32_t n, ij_batch **out);

/* Frees the batch and every case handle, after waiting for all work on the
 * device (a step without graphs runs on the caller's stream). */
void ij_batch_destroy(ij_batch *b);

const char *ij_batch_last_error(const ij_batch *b);

/* Number of cases, or -1 for NULL. */
int32_t ij_batch_size(const ij_batch *b);

/* Borrowed handle of case i (valid until ij_batch_destroy). */
ij_status ij_batch_case(ij_batch *b, int32_t i, ij_sim **out);

/* Step counter shared by the cases. */
int64_t ij_batch_time(const ij_batch *b);

/* Advance every case nsteps steps (Eqs. 3-10 with each case's pulse; a
 * diagnostics sample of every case before each step whose index is a
 * multiple of diag_every).  Every case must be initialised and at the same
 * step (all cases re-initialised count as step 0).  Asynchronous; it
 * synchronises only when a case's sample store fills up. */
ij_status ij_batch_step(ij_batch *b, int64_t nsteps, void *stream);

/* Replay the steps as captured graphs of about steps_per_graph steps
 * (rounded to a multiple of 2 and of diag_every); 0 (default) launches each
 * kernel.  Results are the same either way. */
ij_status ij_batch_set_graph(ij_batch *b, int32_t steps_per_graph);

/* Tile shape of every case: waves across x per workgroup (1, 2 or 4), rows
 * per workgroup (1..1024); mixed_strips: nonzero gives the columns past a
 * case's last full strip of 64 * waves_x to 64-column strips (a second,
 * one-wave launch) instead of a partly idle full-width strip; persistent:
 * nonzero runs as many workgroups as are resident at once, each over a
 * contiguous run of tiles, zero one workgroup per tile.  With one row per
 * workgroup the plain rows go to pieces of 64 columns, one per wave and
 * waves_x per workgroup.  Default (4, 1, 0, 1). */
ij_status ij_batch_set_tiling(ij_batch *b, int32_t waves_x, int32_t rows_per_block, int32_t mixed_strips,
                              int32_t persistent);
ij_status ij_batch_get_tiling(const ij_batch *b, int32_t *waves_x, int32_t *rows_per_block,
                              int32_t *mixed_strips, int32_t *persistent);

/* Autotuner: time trial_steps steps (2..10000) of the batch for each
 * candidate tile shape (waves 1, 2, 4 x rows 32, 64, with and without mixed
 * strips, persistent or not) and keep the fastest; the state of every case is restored
 * afterwards (the step counter does not move).  Results are cached for the
 * process by the cases' sizes and walls: a cached shape is applied without
 * timing (*ms_per_step = -1).  Outputs may be NULL.  Synchronises the
 * stream. */
ij_status ij_batch_autotune(ij_batch *b, int32_t trial_steps, void *stream, int32_t *waves_x,
                            int32_t *rows_per_block, int32_t *mixed_strips, int32_t *persistent,
                            double *ms_per_step);

/* --------------------------------------------------------------- surrogate
 *
 * An ensemble of small networks that predict the droplet outputs of a case
 * (Results: breakup time and drop velocity, Figs. 4-7; drop volume and the
 * satellite flag) from its seven inputs, so that a sweep can skip the
 * lattice run where the members agree.  Each member is a multilayer
 * perceptron 7 -> 128 -> 128 -> 4 with GELU (z Phi(z)), trained with Adam on
 * float32 master weights; every product runs on the matrix cores in bfloat16
 * with float32 accumulation.
 *
 * Inputs x (float32 [n][7]): contact angle (deg), surface tension sigma, f_pos,
 * f_neg, t_pos, t_neg, t_idle; the network sees (x - x_mean) / x_std.
 * Targets y (float32 [n][4]): breakup step, drop velocity, drop volume (the
 * first three learned as (y - y_mean) / y_std with a squared-error loss) and
 * the satellite flag in {0, 1} (logistic loss on the fourth output).
 * Loss per minibatch of S rows: mean over rows of (1/3) sum of the three
 * squared errors plus the logistic loss.
 * Packed parameters of one member (float64, ij_mlp_param_count() = 18052
 * values): W1 [128][7], b1 [128], W2 [128][128], b2 [128], W3 [4][128], b3 [4].
 */
typedef struct ij_mlp ij_mlp;

/* n_members (1..64) members with zero parameters and unit scaling. */
ij_status ij_mlp_create(int32_t n_members, ij_mlp **out);

/* n_members members with seeded initial parameters: parameter j (packed
 * layout below) of member k is -a + 2a u_j, a = 1/sqrt(fan_in of its
 * layer) (7, 128, 128), u_j = (x_j >> 11) / 2^53 with x_j output j + 1 of
 * SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) started at seed + 1000 k;
 * stored as float like ij_mlp_set_weights.  Unit scaling, Adam moments
 * zero.  Synchronises the device; *out is NULL on failure. */
ij_status ij_mlp_create_seeded(int32_t n_members, uint64_t seed, ij_mlp **out);
void ij_mlp_destroy(ij_mlp *m);
const char *ij_mlp_last_error(const ij_mlp *m);
int32_t ij_mlp_param_count(void);

/* Parameters of one member from / to a host array in the packed layout;
 * setting them resets that member's Adam moments and the step count.
 * Synchronise the device. */
ij_status ij_mlp_set_weights(ij_mlp *m, int32_t member, const double *packed);
ij_status ij_mlp_get_weights(ij_mlp *m, int32_t member, double *packed);

/* Input and target scaling (host arrays of 7, 7, 3, 3; std > 0). */
ij_status ij_mlp_set_scaling(ij_mlp *m, const double *x_mean, const double *x_std, const double *y_mean,
                             const double *y_std);

/* Loss and its gradient with respect to every parameter, for every member,
 * over rows 0..n-1 (1..1024) of the device arrays x, y: grad (host,
 * [n_members][18052] packed), loss (host, [n_members], may be NULL).
 * Synchronises the stream. */
ij_status ij_mlp_gradients(ij_mlp *m, const float *x_dev, const float *y_dev, int32_t n, double *grad,
                           double *loss, void *stream);

/* `steps` Adam steps (b1 0.9, b2 0.999, eps 1e-8, learning rate lr) of every
 * member; member k's step s uses rows idx[k][s][0..batch) (device int32,
 * [n_members][steps][batch], clamped to [0, n_rows)) of x, y; batch
 * 1..1024.  loss (device [n_members][steps], may be NULL) gets each step's
 * minibatch loss before its update.  Asynchronous. */
ij_status ij_mlp_train(ij_mlp *m, const float *x_dev, const float *y_dev, int32_t n_rows, const int32_t *idx_dev,
                       int32_t steps, int32_t batch, float lr, float *loss_dev, void *stream);

/* Ensemble prediction for n queries (device x [n][7]): mean and spread
 * (standard deviation over the members) of each output (device [n][4]:
 * breakup step, drop velocity, drop volume in target units, and the
 * satellite probability); members (device [n_members][n][4]) optional.
 * Without members the per-member outputs go to a buffer of the handle,
 * allocated (hipMalloc) on the first call that needs it larger.
 * Asynchronous. */
ij_status ij_mlp_predict(ij_mlp *m, const float *x_dev, int64_t n, float *mean_dev, float *spread_dev,
                         float *members_dev, void *stream);

/* ij_mlp_predict (mean and spread) for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same kernels and results, bit for bit; the per-member
 * outputs go to a fixed 8 MiB array the library holds on every device it
 * runs on (until the process ends), whose address is looked up once per
 * device on the first call.  The call allocates and frees nothing.
 * Limits: n * n_members <= 524288 (131072 queries for 4 members), else
 * IJ_ERR_INVALID_ARG; mean_dev and spread_dev are required; the current
 * device must be the one the handle was created on (IJ_ERR_STATE).  Every
 * call on a device shares that device's array: calls that overlap on one
 * device (other streams, threads or handles) race and must be ordered by
 * the caller.  Asynchronous. */
ij_status ij_mlp_predict_noalloc(ij_mlp *m, const float *x_dev, int64_t n, float *mean_dev, float *spread_dev,
                                 void *stream);

/* ------------------------------------------------------------------------
 * Three-dimensional lattice (round nozzles).
 *
 * The update of the two-dimensional entry points written on D3Q19 (f) and
 * D3Q7 (g): Methods, Eqs. 1-10, with the pulse of Fig. 1 and the wetting
 * walls of "Reproducing the experiment".  Every closure and boundary rule
 * is the two-dimensional one carried to three dimensions:
 *   f equilibrium w_i [A_i + n (3 c.u + 9/2 (c.u)^2 - 3/2 u^2)], A_i = 3p off
 *   rest, A_0 = 3n - 6p at rest, p = n/3 + phi mu (Eqs. 5-6);
 *   g equilibrium g_0 = phi - 3 Gamma mu, g_i = Gamma mu/2 + phi c_i.u/(2q)
 *   (Eqs. 9-10); gradient and Laplacian over the 18 D3Q19 neighbours; the
 *   wetting ghost averages the fluid axis neighbours (else the 12 edge
 *   neighbours).  Summed along one axis D3Q19 has the D2Q9 weights, so a
 *   state that does not vary along z evolves as the two-dimensional update.
 *
 * Axes: x in [0,nx) periodic (width), y in [0,ny) the jet direction
 * (periodic or open rows), z in [0,nz) periodic (depth).  Every field array
 * the caller passes or receives is [ny][nz][nx] (index (y*nz + z)*nx + x).
 * Velocities: 0 rest; 1..6 = +x, +y, -x, -y, +z, -z (D3Q7 = 0..6);
 * 7..10 = (1,1,0) (-1,1,0) (-1,-1,0) (1,-1,0); 11..14 = (1,0,1) (-1,0,1)
 * (-1,0,-1) (1,0,-1); 15..18 = (0,1,1) (0,-1,1) (0,-1,-1) (0,1,-1).
 * Distribution arrays exchanged with the caller are [19][ny][nz][nx] (f)
 * and [7][ny][nz][nx] (g).  Error handling, streams and ownership follow the
 * conventions at the top of this file.
 * ------------------------------------------------------------------------ */
typedef struct ij3_params {
    int64_t nx, ny, nz;        /* lattice size, each >= 3 */
    int64_t bc_y;              /* IJ_BC_PERIODIC or IJ_BC_OPEN (rows y = 0 and ny-1) */
    int64_t force_rows;        /* body force along +y on fluid nodes with y < force_rows */
    int64_t t_pos, t_neg, t_idle, periodic_pulse; /* pulse of Fig. 1, in steps */
    double rho_ink, rho_amb, sigma, width, gamma;
    double tau_ink, tau_amb, tau_phi;
    double theta_inner, theta_outer; /* contact angles of wall classes 1 and 2 (degrees) */
    double f_pos, f_neg;
} ij3_params;

typedef struct ij3_sim ij3_sim;

/* Validate *p and allocate, on the current device, two distribution buffers
 * (26 floats per node: the 19 f and 7 g rows of each lattice row (y, z) are
 * stored one after the other, row pitch nx rounded up to 64; then a 16-bit
 * plane with the low-order part of g_0), the
 * phi field (double) and the wall mask from `wall` (host, [ny][nz][nx]
 * bytes, IJ_FLUID / IJ_WALL_INNER / IJ_WALL_OUTER; NULL: all fluid).  With
 * open rows, a fluid node of row 0 (ny-1) must have fluid directly above
 * (below) it.  *out is NULL on failure; ij3_last_error(NULL) says why. */
ij_status ij3_create(const ij3_params *p, const uint8_t *wall, ij3_sim **out);
void ij3_destroy(ij3_sim *s);
const char *ij3_last_error(const ij3_sim *s);

/* Initial state at t = 0: phi from src (device float [ny][nz][nx]; with
 * from_distance != 0 src is a signed distance d to the ink, positive inside,
 * and phi = phi* tanh(2d/W)); n = n0; velocity from ux, uy, uz (device, NULL
 * = 0); f = f_eq and g = g_eq with mu from phi and its wetting ghosts.
 * Asynchronous. */
ij_status ij3_init(ij3_sim *s, const float *src_dev, int32_t from_distance, const float *ux_dev,
                   const float *uy_dev, const float *uz_dev, void *stream);

/* nsteps time steps (Eqs. 3, 4, 8): the wetting ghosts, then one fused
 * launch that forms phi from g, collides and pushes, then the open rows.
 * Asynchronous. */
ij_status ij3_step(ij3_sim *s, int64_t nsteps, void *stream);
int64_t ij3_time(const ij3_sim *s);

/* n, phi, u of the current state into device float arrays [ny][nz][nx]
 * (NULL = skip; solid nodes read 0).  Asynchronous. */
ij_status ij3_get_moments(ij3_sim *s, float *n_dev, float *phi_dev, float *ux_dev, float *uy_dev,
                          float *uz_dev, void *stream);

/* Distributions to / from device float arrays [19][ny][nz][nx] and
 * [7][ny][nz][nx] (solid nodes read 0 and are not written).  set_state also
 * sets the step counter.  Asynchronous. */
ij_status ij3_get_state(ij3_sim *s, float *f_dev, float *g_dev, void *stream);
ij_status ij3_set_state(ij3_sim *s, const float *f_dev, const float *g_dev, int64_t t, void *stream);

/* Checkpoint and bit-exact resume, as ij_state_bytes / ij_save_state /
 * ij_load_state for the three-dimensional lattice: a 64-byte header (magic
 * "IJ3STAT1", lattice size, row pitch, step counter, wall hash, payload
 * size) and the current buffer as stored (shifted f, g, the g_0 remainder
 * plane).  A load needs the same lattice size and wall mask.  Both
 * synchronise the stream. */
ij_status ij3_state_bytes(const ij3_sim *s, size_t *bytes);
ij_status ij3_save_state(ij3_sim *s, void *blob_host, size_t bytes, void *stream);
ij_status ij3_load_state(ij3_sim *s, const void *blob_host, size_t bytes, void *stream);

/* Droplet segments of a sample (Results: breakup time and drop velocity,
 * Figs. 3-4): the rows y >= row0 split into maximal runs of rows with ink;
 * the run that starts at row0 is attached to the nozzle and every other run
 * with at least a_min ink nodes is a detached drop. */
typedef struct ij3_drops {
    int64_t n_detached;        /* detached drops */
    int64_t largest_count;     /* ink nodes (phi > 0) of the largest (the lowest on a tie) */
    double largest_uy;         /* sum of u_y over them */
    int64_t largest_top;       /* its highest row (-1: none) */
    int64_t largest_bottom;    /* its lowest row (-1: none) */
    double head_uy, tail_uy;   /* mean u_y of its ink in its top / bottom `band` rows */
} ij3_drops;

/* Diagnostic sums of the current state (Results: mass, momentum, breakup):
 * rec (host, 7 doubles) = {sum n, sum phi, sum c_x f, sum c_y f, sum c_z f,
 * max |u|, fluid nodes with a non-finite n, phi or u or with n <= 0}; for each row y
 * (an x-z slice) with y >= row0, row_count[y] (host int64) = fluid nodes
 * with phi > 0 and row_uy[y] (host double) = the sum of their u_y (0 below
 * row0; either pointer may be NULL).  With drops (host, may be NULL) the
 * droplet segments of the sample, for a_min >= 1 and band >= 1.  Sums
 * accumulate in double in a fixed order.  Synchronises the stream. */
ij_status ij3_sample(ij3_sim *s, int64_t row0, double *rec, int64_t *row_count, double *row_uy, int64_t a_min,
                     int64_t band, ij3_drops *drops, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* INKJET_LBM_H */
