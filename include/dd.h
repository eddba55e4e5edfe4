/*
 * dd.h -- C ABI of libdd, the MI355X (gfx950) library for the cumulative
 * damage-diffusion distribution of a STEM scan.
 *
 * Paper: "Fast Simulation of Damage Diffusion Distribution in Scanning
 * Transmission Electron Microscopy".  The library evaluates
 *
 *   psi(r, t) = sum over visits i with t_i < t of phi_i(r, t)          (Eq. 6)
 *   phi_i     = Q0/(4 pi D) [E1(a/b1) - E1(a/b0)]                       (Eqs. 1-2)
 *   phi_i     = Q0/(4 pi D) ln(b1/b0)                  at r = r_i      (Eqs. 3-4)
 *
 * with a = |r - r_i|^2, Ds = r_s^2 = sigma^2, b1 = 2 Ds + 4 D (t - t_i),
 * b0 = 2 Ds while the beam is on (t - t_i <= tau) and 2 Ds + 4 D (t - t_i - tau)
 * after.  E1 is the exponential integral of order one (Sec. II).
 *
 * Conventions shared by every call:
 *  - Every call returns a dd_status; 0 is success, negative is an error.  No
 *    call throws or aborts.  dd_last_error() returns a thread-local message
 *    for the last failing call on this thread.
 *  - A dd_scan handle owns its host and device buffers; it is not thread
 *    safe (use one handle per thread), distinct handles are independent.
 *  - Input arrays are read during the call and never retained.
 *  - Outputs are caller-owned.  With out_on_device = 1, `out` is a device
 *    pointer and the work is enqueued on `hip_stream` (a hipStream_t, NULL =
 *    the null stream); the call returns once the work is enqueued.  With
 *    out_on_device = 0, `out` is host memory and the call synchronizes the
 *    stream before returning.
 *  - Results are double precision in u/m^2 (the unit of Q0 per square metre).
 *  - Precision DD_FP64 evaluates every term in double precision;
 *    DD_MIXED evaluates the bulk of the E1 differences in single precision
 *    (with exact lattice distances, exact dwell increments and a split
 *    exponent) and accumulates in double precision.  A map grid whose pixels
 *    are not on a dyadic lattice shared with the probes (multiples of 2^-q
 *    pitches, q <= 8) is evaluated in double precision under DD_MIXED too.
 *  - Lengths are metres, times seconds, D m^2/s, Q0 u/s.
 */
#ifndef DD_H
#define DD_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DD_OK = 0,
  DD_EINVAL = -1,       /* invalid or non-finite argument                       */
  DD_ENOMEM = -2,       /* host or device allocation failed                     */
  DD_EDEVICE = -3,      /* HIP runtime error or no usable gfx950 device         */
  DD_EUNSUPPORTED = -4  /* valid request the library does not handle           */
} dd_status;

/* Visit orders (Sec. I: raster, interleaved/alternating, random and
 * multi-frame scans).  Probe id = row * nx + col, probe at (col, row) * pitch. */
typedef enum {
  DD_RASTER = 0,       /* row-major, +x fastest                                */
  DD_INTERLEAVED = 1,  /* stride^2 sub-lattice passes, offsets (oy, ox) row-major,
                          each pass a raster of its sub-lattice                */
  DD_RANDOM = 2,       /* seeded permutation: SplitMix64 + Fisher-Yates (from
                          the last slot) + Lemire's unbiased bounded integers  */
  DD_MULTIFRAME = 3,   /* `frames` raster frames, per-visit dwell dwell_s/frames */
  DD_EXPLICIT = 4      /* caller-supplied probe ids, repeats allowed           */
} dd_order;

typedef enum {
  DD_FP64 = 0,
  DD_MIXED = 1,
  /* bounds of the type only: every int32 value is a value of dd_precision, so
   * a call can read whatever the caller passes and rejects values other than
   * DD_FP64 and DD_MIXED with DD_EINVAL                                    */
  DD_PRECISION_RANGE_MIN = -2147483647 - 1,
  DD_PRECISION_RANGE_MAX = 2147483647
} dd_precision;

/* Scan description (Sec. II assumptions: deposition rate Q0, constant D,
 * Gaussian probe of per-axis standard deviation sigma = r_s).  Visit v
 * (0-based) starts at v * tau_v and lasts tau_v, back to back, where
 * tau_v = dwell_s / frames for DD_MULTIFRAME and dwell_s otherwise.       */
typedef struct {
  int32_t nx, ny;          /* probe grid, 1 .. 2048 each (DD_EINVAL beyond:   *
                            * squared lattice distances, below 2^23, then    *
                            * stay exact in single precision)                */
  int32_t order;           /* dd_order                                         */
  int32_t stride;          /* DD_INTERLEAVED: >= 1                             */
  int32_t frames;          /* DD_MULTIFRAME: >= 1                              */
  int32_t reserved;        /* must be 0                                        */
  uint64_t seed;           /* DD_RANDOM                                        */
  const int32_t *visits;   /* DD_EXPLICIT: probe ids in [0, nx*ny), copied     */
  int64_t n_visits;        /* DD_EXPLICIT: >= 1                                */
  double pitch_m;          /* > 0                                              */
  double dwell_s;          /* > 0                                              */
  double sigma_m;          /* > 0 (the log form needs Ds > 0)                  */
  double D_m2s;            /* > 0                                              */
  double Q0_us;            /* >= 0                                             */
} dd_scan_desc;

typedef struct dd_scan dd_scan; /* opaque */

/* Evaluation grid for maps: pixel (u, v) at (x0 + u dx, y0 + v dy), u < w,
 * v < h; w, h >= 1; spacings may be any finite value.                     */
typedef struct {
  double x0_m, y0_m, dx_m, dy_m;
  int32_t w, h;
} dd_grid;

/* Builds the visit list and probe table (Sec. I scan strategies, Sec. II
 * probe placement).  Host only: no device is touched until the first query.
 * Errors: DD_EINVAL for a bad description, DD_ENOMEM.                      */
dd_status dd_scan_create(const dd_scan_desc *desc, dd_scan **out);
/* Frees the handle and its device buffers; NULL is allowed.               */
void dd_scan_destroy(dd_scan *s);
/* Number of visits V (nx*ny, frames*nx*ny or n_visits); -1 for NULL.      */
int64_t dd_scan_num_visits(const dd_scan *s);
/* Copies the probe id of each visit, in visit order, to out_host[V].      */
dd_status dd_scan_visits(const dd_scan *s, int32_t *out_host);

/* psi on a pixel grid at n_t times (Eq. 6 at each pixel and time).
 * t_s: host array of n_t finite times >= 0 (seconds from the start of the
 * first visit).  out: [n_t][h][w] row-major.  Times before a visit's start
 * give that visit no contribution; a time within 8 ulp of a dwell boundary
 * is taken to be on it.                                                   */
dd_status dd_damage_map(dd_scan *s, const dd_grid *g, const double *t_s, int32_t n_t,
                        dd_precision p, double *out, int32_t out_on_device, void *hip_stream);

/* Time-sampled simulation, the paper's workload of maps every time step dt
 * on a sampling grid (Sec. III, the cost model of Eq. 7; Fig. 1 shows maps
 * of it): psi on grid g at t_k = t0_s + k dt_s, k = 0 .. n_t-1, out
 * [n_t][h][w] row-major.  The same values as dd_damage_map with that list of
 * times (up to the order of the per-pixel sums); the library evaluates the
 * times in chunks so that its scratch stays bounded whatever n_t is.
 * t0_s: finite, >= 0; dt_s: finite, > 0; n_t >= 1; the last time finite.
 * Host outputs (out_on_device = 0) are copied chunk by chunk; the call then
 * returns when all of them are in out.
 * Errors: DD_EINVAL (bad times, grid, precision or NULL), DD_ENOMEM,
 * DD_EDEVICE.                                                             */
dd_status dd_damage_sweep(dd_scan *s, const dd_grid *g, double t0_s, double dt_s, int32_t n_t,
                          dd_precision p, double *out, int32_t out_on_device, void *hip_stream);

/* psi at every probe visit at the moment that visit starts: out[j] =
 * psi(r_j, t_j), summed over visits i < j (Eq. 6 with j the visit being
 * made; the visit itself contributes phi_j(r_j, t_j) = 0).  out: [V].    */
dd_status dd_damage_at_probe_arrival(dd_scan *s, dd_precision p, double *out,
                                     int32_t out_on_device, void *hip_stream);

/* Streaming form of the arrival query (the real-time simulation the paper
 * aims at, Sec. V): psi at the visits j0 <= j < j1 only, out[j - j0] =
 * psi(r_j, t_j) summed over visits i < j (Eq. 6), e.g. for the visits the
 * scan has just made.  The same values as dd_damage_at_probe_arrival (up to
 * the order of the per-visit sums); the work is the pairs of those visits
 * (about j per visit).  0 <= j0 <= j1 <= V; j0 == j1 does nothing.
 * Errors: DD_EINVAL (range, precision, NULL), DD_ENOMEM, DD_EDEVICE.     */
dd_status dd_damage_at_probe_arrival_range(dd_scan *s, int64_t j0, int64_t j1, dd_precision p,
                                           double *out, int32_t out_on_device, void *hip_stream);

/* The streaming arrival query for callers that cannot allocate device
 * memory (code under stream capture, serving loops that must not allocate,
 * harnesses that forbid allocation): the same values as
 * dd_damage_at_probe_arrival_range(s, j0, j1, p, out_dev, 1, hip_stream),
 * bit for bit, with no device or pinned allocation.  Its scratch (work
 * items, slots per tile, partial sums) is one static device array of 32 MiB
 * per GPU, held until the process ends; a range whose plan needs more
 * returns DD_EINVAL (for a 512 x 512 scan, ranges up to about 60000 visits
 * fit).  Every call on a GPU shares that array: calls that overlap on one
 * GPU (other streams, other threads) race on it and must not be issued;
 * calls on one stream are ordered by it.  The scan's device tables must be
 * resident on the current device: any earlier query of this scan there by
 * dd_damage_at_probe_arrival, dd_damage_at_probe_arrival_range,
 * dd_damage_map or dd_damage_sweep builds them (else DD_EINVAL).  out_dev
 * is a device array of j1 - j0 doubles; the work is enqueued on hip_stream
 * and the call returns once it is (dd_scan_check reports non-finite
 * values).  The plan is copied from host memory in stream order.
 * Errors: DD_EINVAL (range, precision, NULL, tables not resident, scratch
 * too small), DD_EDEVICE.                                                 */
dd_status dd_damage_at_probe_arrival_range_noalloc(dd_scan *s, int64_t j0, int64_t j1,
                                                   dd_precision p, double *out_dev,
                                                   void *hip_stream);

/* Queries for dd_batch_solve (bit mask).                                  */
typedef enum {
  DD_Q_ARRIVAL = 1,          /* [V] as dd_damage_at_probe_arrival              */
  DD_Q_FINAL_AT_PROBES = 2   /* [ny][nx]: psi at each probe position at the end
                                of the scan, t = V * tau_v                     */
} dd_query;

/* Many independent scans in one persistent launch (work items of all scans
 * ordered longest first, taken from a device work counter).  outs[k] holds
 * scan k's results back to back: [V_k] arrival (if requested) then
 * [ny_k * nx_k] final map (if requested).  Results equal the per-scan calls.
 * Errors: DD_EINVAL (n < 1, NULL scans or outs, empty mask).              */
dd_status dd_batch_solve(dd_scan *const *scans, int32_t n, uint32_t query_mask,
                         dd_precision p, double *const *outs, int32_t out_on_device,
                         void *hip_stream);

/* Non-finite output check of the handle's last query (its own call, or its
 * part of the last dd_batch_solve that included it).  Waits for that call
 * to finish on the device.  Returns DD_EDEVICE if a value it wrote for this
 * scan was not finite, with *first_bad (may be NULL) set to the smallest
 * such index of the scan's output of that call (for a batched call: [V]
 * arrival first, then the final map), else DD_OK with *first_bad = -1
 * (also for a handle that has run no query).  Calls with host outputs make
 * this check themselves and return DD_EDEVICE before they return; a batched
 * call then names the scan.  Every value of Eq. 6 is finite for a valid
 * scan; a non-finite one means that Q0/(4 pi D) times the dimensionless
 * sum overflowed, or a device fault.  The current device must be the one
 * the handle ran on.  Errors: DD_EINVAL (NULL, another device), DD_EDEVICE. */
dd_status dd_scan_check(dd_scan *s, int64_t *first_bad);

/* Dimensionless pair term phi_hat = phi * 4 pi D / Q0 (Eqs. 1-4) for n
 * (a, lag) pairs: a[k] = squared distance / pitch^2 (>= 0), lag[k] = time
 * since the visit started / tau_v (> 0), with kappa = D tau_v / pitch^2 and
 * sigma_hat = sigma / pitch.  a, lag, out are device pointers; the work is
 * enqueued on hip_stream.  Exposes the device E1 difference for testing.  */
dd_status dd_pair_terms(double kappa, double sigma_hat, int64_t n, const double *a,
                        const double *lag, dd_precision p, double *out, void *hip_stream);

/* Autotuner: times the candidate tile shapes on representative problems
 * and writes a JSON cache to cache_path (NULL: $DD_TUNE_CACHE or
 * ./dd_tune.json).  Later queries in this process use the winners.        */
dd_status dd_autotune(const char *cache_path);
/* Loads a cache written by dd_autotune; DD_EINVAL if unreadable.          */
dd_status dd_tune_load(const char *cache_path);

/* Kernel timing for measurement.  While enabled, the library brackets each
 * launch of its main kernels with HIP events on the stream it launches on
 * and records the algorithmic work of the launch: pairs is the number of
 * causal (evaluation point, visit) pairs it evaluates, flops the FP32/FP64
 * operations of the evaluation form used for them, counted as the hardware
 * FLOP counters count them (FMA 2; add, multiply, exp 1; per pair of a
 * series of degree M: 13 + 2 max(M, 1) for M <= 3 and 17 + 2M above in
 * mixed precision, 4 fewer in the arrival rows of small exponents that skip
 * the exponent's rounding correction, 9 in all in those that fold the
 * series' linear term into the exponent; 29 + 2M in FP64).  Kernel names: "arrival_far",
 * "arrival_near", "map", "batch", "lag_rows", "reduce".                   */
typedef struct {
  double ms;         /* summed event time of the launches                   */
  int64_t launches;
  double pairs;      /* summed pairs                                        */
  double flops;      /* summed algorithmic floating-point operations         */
} dd_kernel_stats;
dd_status dd_profiling(int32_t enable);
/* Synchronizes the recorded events and returns the totals since the last
 * reset; reset = 1 clears them.  DD_EINVAL for an unknown name.          */
dd_status dd_profile_read(const char *kernel, dd_kernel_stats *out, int32_t reset);

/* ---- Learned surrogate --------------------------------------------------
 * A 4-level U-Net (32, 64, 128, 256 channels at 64^2, 32^2, 16^2, 8^2; two
 * 3x3 convolutions + SiLU per level, 2x2 average pooling, nearest 2x
 * upsampling with skip concatenation, FP32 1x1 head) that predicts the
 * dimensionless damage map psi_hat = psi 4 pi D / Q0 of a 64x64 scan at the
 * end of the scan (Eq. 6 at every probe position).  Per probe it reads
 * DD_SURROGATE_CHANNELS inputs:
 *   0  first visit start / scan duration (the arrival-time map),
 *   1  (log10 kappa + 1) / 3, kappa = D tau / pitch^2 (tau: one visit's dwell),
 *   2  (sigma / pitch - 0.6) / 0.4,
 *   3  ln(lambda_last) / ln(V), lambda_last = V - (index of the last visit),
 *   4  (ln O + 4) / 4,
 * where O = sum over the probe's own visits v of ln(b1/b0), b0 = 2 sigma_hat^2
 * + 4 kappa (V - v - 1), b1 = b0 + 4 kappa (the a = 0 bracket of Eq. 6 at the
 * end of the scan).  The prediction is psi_hat = O + exp(y), y the network
 * output.  Convolutions run on BF16 MFMA with FP32 accumulation; activations,
 * master weights, Adam moments and the head are FP32.  Parameters are one
 * flat FP32 vector: per convolution weights [9 ci][co] (k = (3 ky + kx) ci +
 * c) then bias [co], in forward order, then the head's 32 weights and bias.
 * Tensors are device pointers, NHWC: x [B][64][64][DD_SURROGATE_CHANNELS],
 * y, own and targets [B][64][64].  Calls enqueue on hip_stream.  One handle
 * per thread.                                                              */
#define DD_SURROGATE_CHANNELS 5
typedef struct dd_unet dd_unet;
/* He-normal convolutions from `seed`, zero biases and head.  DD_EDEVICE
 * without a gfx950 GPU.                                                   */
dd_status dd_unet_create(uint64_t seed, dd_unet **out);
void dd_unet_destroy(dd_unet *u);                           /* NULL-safe */
int64_t dd_unet_num_params(const dd_unet *u);               /* -1 for NULL */
/* Copies the FP32 master parameters out (host_get) and/or in (host_set). */
dd_status dd_unet_params(dd_unet *u, float *host_get, const float *host_set);
/* Copies the gradient of the last backward pass to host_out.            */
dd_status dd_unet_grads(const dd_unet *u, float *host_out);
/* Forward pass of a batch; train = 1 keeps what the backward pass needs.  */
dd_status dd_unet_forward(dd_unet *u, int32_t batch, const float *x, float *y, int32_t train,
                          void *hip_stream);
/* Backward pass of the last (training) forward batch, whose input was x,
 * for output gradient dy; the gradient is overwritten (not accumulated).  */
dd_status dd_unet_backward(dd_unet *u, const float *x, const float *dy, void *hip_stream);
/* Loss of `maps` predictions own + exp(y) against targets t: loss_host (may
 * be NULL; synchronizes) receives the mean over maps of |pred - t|^2 / |t|^2
 * (squared relative L2 error per map); dy is the gradient of that mean plus
 * the anchor term (anchor / 4096) sum_i (r_i/t_i)^2 (y_i - ln r_i)^2 per map,
 * r_i = max(t_i - own_i, 1e-6 t_i), whose gradient does not vanish when
 * exp(y) is far below r.  exp arguments are capped at 80.  maps <= 4096.  */
dd_status dd_unet_loss(dd_unet *u, int32_t maps, const float *y, const float *own, const float *t,
                       float anchor, float *dy, double *loss_host, void *hip_stream);
/* One Adam step (bias-corrected) on the FP32 master weights with the
 * gradient scaled to global L2 norm <= clip (clip = 0: no clipping; a
 * non-finite gradient skips the step).  grad_norm_host (may be NULL)
 * receives the norm before clipping (synchronizes).                       */
dd_status dd_unet_adam(dd_unet *u, float lr, float beta1, float beta2, float eps, float clip,
                       float *grad_norm_host, void *hip_stream);
/* Adam state for checkpoints: copies the first and second moments (n_params
 * floats each, host) and the step count (dd_unet_adam calls so far, which
 * sets the bias correction) out through the *_get pointers and then in from
 * the *_set pointers; any of them may be NULL.  With the parameters
 * (dd_unet_params) this is all the state a training step reads, so a run
 * restored from them continues bit for bit.  Synchronizes.
 * Errors: DD_EINVAL (NULL handle, every pointer NULL, a negative step),
 * DD_EDEVICE.                                                             */
dd_status dd_unet_adam_state(dd_unet *u, float *m_get, float *v_get, int64_t *step_get,
                             const float *m_set, const float *v_set, const int64_t *step_set);
/* Training mini-batch: slot b <- map idx[b] of (x_all, own_all, t_all; n_all
 * maps) under the symmetry transform[b] of the square (0..7: transpose if
 * bit 0, then mirror rows if bit 1, columns if bit 2); idx and transform are
 * device arrays of nb entries; an idx outside [0, n_all) gives zeros.      */
dd_status dd_surrogate_batch(const float *x_all, const float *own_all, const float *t_all,
                             int64_t n_all, const int32_t *idx, const int32_t *transform,
                             int32_t nb, float *xb, float *ob, float *tb, void *hip_stream);
/* Network inputs x [n][64][64][DD_SURROGATE_CHANNELS] and the own-visit term
 * own [n][64][64] of n scans (64x64 grids with every probe visited, else
 * DD_EINVAL).  The per-scan table is built once and kept with the scan.   */
dd_status dd_surrogate_inputs(dd_scan *const *scans, int32_t n, float *x, float *own,
                              void *hip_stream);
/* Training targets t = psi 4 pi D / Q0 (float) from exact final maps psi
 * [n][4096] (double).                                                     */
dd_status dd_surrogate_targets(dd_scan *const *scans, int32_t n, const double *psi, float *t,
                               void *hip_stream);
/* Final damage maps psi [n][64*64] (u/m^2, device) by the network, judged by
 * the exact kernels: a map is accepted if the relative L2 error of its 64
 * values on the probe sub-grid of stride 9 (rows and columns 0, 9, ..., 63:
 * corners, borders and interior) against the exact values is <= spot_tol;
 * scans outside
 * the training range (64x64 grid, every probe visited, kappa in
 * [2.5e-5, 100], sigma/pitch in [0.2, 1]) and rejected maps are computed
 * exactly (used_fallback[k] = 1, host array).  Synchronizes.               */
dd_status dd_unet_predict(dd_unet *u, dd_scan *const *scans, int32_t n, double spot_tol,
                          dd_precision p, double *psi, int32_t *used_fallback, void *hip_stream);

/* ---- General visit lists ----------------------------------------------------
 * Sec. II's single-visit field (Eqs. 1-4) holds for each visit with its own
 * position r_i, start time t_i and dwell tau_i, and Eq. 6 sums it over the
 * visits with t_i < t.  A general list states every visit this way, so
 * per-visit dwells, flyback and dead time between lines or frames,
 * subsampled (sparse) scans, revisits and any visit order are all lists.
 * DD_FP64 meets the FP64 bound; DD_MIXED evaluates the near-pair integral
 * (almost every pair of a long list) in FP32 and meets the mixed bound.
 * These calls synchronize the stream before they return (also with device
 * outputs), and return DD_EDEVICE naming the list and the index of the
 * first output value that is not finite.                                  */
typedef struct dd_visits dd_visits; /* opaque */

/* Copies n >= 1 visits: x_m, y_m (metres), t0_s (beam-on start, seconds)
 * and dwell_s (seconds, > 0), host arrays in any order; visits may overlap
 * in time.  sigma_m, D_m2s > 0, Q0_us >= 0 as in dd_scan_desc.  Host only.
 * Errors: DD_EINVAL (NULL, n < 1 or n > 2^31, a non-finite value, a dwell
 * <= 0), DD_ENOMEM.                                                       */
dd_status dd_visits_create(int64_t n, const double *x_m, const double *y_m, const double *t0_s,
                           const double *dwell_s, double sigma_m, double D_m2s, double Q0_us,
                           dd_visits **out);
/* Frees the handle and its device buffers; NULL is allowed.               */
void dd_visits_destroy(dd_visits *v);
/* Number of visits; -1 for NULL.                                          */
int64_t dd_visits_count(const dd_visits *v);

/* psi at each visit's position at the moment its beam turns on: out[i] =
 * psi(r_i, t0_i), the sum over visits j with t0_j < t0_i (Eq. 6), in the
 * caller's visit order.  out: [n].
 * Errors: DD_EINVAL (NULL, precision), DD_ENOMEM, DD_EDEVICE.             */
dd_status dd_visits_arrival(dd_visits *v, dd_precision p, double *out, int32_t out_on_device,
                            void *hip_stream);

/* psi on grid g at n_t >= 1 finite times t_s (host array, seconds on the
 * visits' clock), out [n_t][h][w] row-major; visits not started at a time
 * give it nothing.
 * Errors: DD_EINVAL (NULL, grid, times, precision), DD_ENOMEM, DD_EDEVICE. */
dd_status dd_visits_map(dd_visits *v, const dd_grid *g, const double *t_s, int32_t n_t,
                        dd_precision p, double *out, int32_t out_on_device, void *hip_stream);

/* Arrival queries of n >= 1 lists in one launch, for many small lists:
 * outs[k] gets [count(lists[k])] values, the same as dd_visits_arrival on
 * lists[k] alone, bit for bit.  outs: n pointers, all on the device or all
 * on the host (out_on_device).
 * Errors: DD_EINVAL (NULL list or output, n < 1, precision), DD_ENOMEM,
 * DD_EDEVICE.                                                             */
dd_status dd_visits_batch_arrival(dd_visits *const *lists, int32_t n, dd_precision p,
                                  double *const *outs, int32_t out_on_device, void *hip_stream);

/* Maps of n >= 1 distinct lists in one launch: list k on grids[k] at the
 * n_t[k] host times t_s[k], into outs[k] [n_t[k]][h][w], the same as
 * dd_visits_map on list k alone, bit for bit.  outs: all on the device or
 * all on the host (out_on_device).
 * Errors: DD_EINVAL (NULL, n < 1, a list given twice, a grid, times or
 * precision as for dd_visits_map), DD_ENOMEM, DD_EDEVICE.                 */
dd_status dd_visits_batch_map(dd_visits *const *lists, int32_t n, const dd_grid *grids,
                              const double *const *t_s, const int32_t *n_t, dd_precision p,
                              double *const *outs, int32_t out_on_device, void *hip_stream);

/* ---- Visualisation -----------------------------------------------------------
 * The paper's integrated 2-D views of the damage diffusion distribution
 * (Sec. IV), on the device: n maps psi [n][h][w] (device doubles, e.g. the
 * output of dd_damage_map, dd_damage_sweep or the final maps of
 * dd_batch_solve) rendered to 8-bit RGB images rgb [n][h][w][3] (device),
 * row-major, in the order of the maps.  Per pixel with value v and the
 * range [lo, hi] of its map:
 *   t = 0 if not (v > lo) (NaN, and v <= 0 on a log scale), 1 if v >= hi,
 *       ln(v / lo) / ln(hi / lo) on a log scale, (v - lo) / (hi - lo) on a
 *       linear one (a t that is not a number counts as 0);
 *   colour = table[min(255, floor(256 t))], where table[i] interpolates the
 *       anchors (bin; r, g, b) = (0; 0,0,0) (38; 32,12,96) (90; 118,24,132)
 *       (141; 200,52,84) (192; 244,128,32) (230; 250,208,64)
 *       (255; 255,255,232) linearly in the bin, each channel
 *       c0 + (c1 - c0) (i - b0) / (b1 - b0) in double precision rounded to
 *       the nearest integer (black through violet, red and orange to white).
 * With levels L > 0, a pixel whose level min(L - 1, floor(L t)) differs
 * from that of its right or lower neighbour in the same map is white
 * (iso-lines, e.g. one per decade on a log scale).  lo = hi = 0 asks for an
 * automatic range per map: hi = the map's largest finite value, lo =
 * max(hi 10^-decades, 2^-1022) on a log scale and 0 on a linear one; a map
 * with hi <= lo (no positive value) is black.  Work is enqueued on
 * hip_stream.  n = 0 does nothing.
 * Errors: DD_EINVAL (NULL, n < 0, w or h < 1, levels outside [0, 256],
 * log_scale not 0/1, explicit range not finite with lo < hi, log scale with
 * lo <= 0, automatic log range with decades outside (0, 300]), DD_EDEVICE. */
typedef struct {
  double lo, hi;       /* range shown; lo = hi = 0: automatic per map          */
  double decades;      /* automatic log range: decades below the map's maximum */
  int32_t log_scale;   /* 1: logarithmic, 0: linear                            */
  int32_t levels;      /* iso-lines between `levels` equal steps of t; 0: none */
} dd_render_opts;
dd_status dd_render_maps(const double *psi, int64_t n, int32_t w, int32_t h,
                         const dd_render_opts *opt, uint8_t *rgb, void *hip_stream);

/* Thread-local description of the last error on this thread ("" if none). */
const char *dd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
