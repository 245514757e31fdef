/*
 * kbm.h - C ABI of the MI355X (gfx950) shift-and-stack trajectory search.
 *
 * Method: Smotherman et al., "Sifting Through the Static: Moving Object
 * Detection in Difference Images" (arXiv 2109.03296), Section 3 (likelihood
 * planes and trajectory sums), Section 3.1 (sigma_G lightcurve filter,
 * Eqs. 1-5) and Section 3.2 (in-line GPU filter, per-pixel top-K).
 *
 * Conventions shared by every entry point
 *  - Bulk arrays are caller-owned *device* memory, contiguous, row-major.
 *    Images are [T][H][W] (epoch, row y, column x).  Small descriptive arrays
 *    (epoch times, velocity list, PSF) are *host* memory and are read only
 *    during the call.
 *  - The library keeps no pointer after a call returns and never frees
 *    caller memory.
 *  - Every call validates all arguments on the host first.  On an invalid
 *    argument nothing is enqueued, the call returns an error code and
 *    kbm_last_error() describes it.  No HIP call is made before validation
 *    succeeds, so argument errors are reported even without a GPU.
 *  - Work is enqueued asynchronously on `stream` (0 = the null stream).
 *    Launch failures return KBM_ERR_DEVICE with the HIP error text.
 *  - Bad *data* is not an error: NaN/inf pixels and var <= 0 are treated as
 *    masked; trajectories with no usable epoch give empty result slots.
 *  - Times are days; only differences matter (t_i - min_j t_j is used).
 *    Velocities are pixels/day.  Offsets are floor(v * t + 1/2) in FP64.
 *  - Calls are reentrant; concurrent calls may use different streams.
 */
#ifndef KBM_H
#define KBM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KBM_MAX_EPOCHS 64   /* keep masks are 64-bit */
#define KBM_MAX_K 16        /* results per pixel */
#define KBM_MAX_PSF 31      /* odd PSF width limit */

typedef enum {
    KBM_OK = 0,
    KBM_ERR_INVALID_ARG = 1,
    KBM_ERR_UNSUPPORTED = 2,
    KBM_ERR_OUT_OF_MEMORY = 3,
    KBM_ERR_DEVICE = 4,
    KBM_ERR_WORKSPACE = 5
} kbm_status;

/* Static text for a status code. */
const char *kbm_status_string(kbm_status s);
/* Detail of the last failure on the calling thread ("" if none). */
const char *kbm_last_error(void);
/* Library version, major*10000 + minor*100 + patch. */
int kbm_version(void);
/* Id of the sources and flags the library was built from (16 hex digits;
 * comments do not enter it), so a binding can refuse a stale build. */
const char *kbm_build_id(void);

/* One aligned image stack (one CCD over T epochs). */
typedef struct {
    int32_t width;       /* W >= 1 */
    int32_t height;      /* H >= 1 */
    int32_t num_epochs;  /* T in [1, KBM_MAX_EPOCHS] */
    const double *times; /* host [T], days, finite */
} kbm_stack;

/*
 * kbm_make_planes - likelihood planes of Section 3.
 *
 *   w_i(p)   = 0 if mask_i(p) != 0, or sci/var non-finite, or var <= 0;
 *              otherwise 1 / var_i(p)
 *   psi_i(p) = sum_{a,b} P[b][a] * sci_i(p + (a-r, b-r)) * w_i(p + (a-r, b-r))
 *   phi_i(p) = sum_{a,b} P[b][a]^2 * w_i(p + (a-r, b-r))
 *
 * i.e. correlation with the PSF (matched filter), r = (psf_k-1)/2, taps
 * outside the image add nothing.  Masked pixels are removed by selection,
 * so any value under the mask (NaN, 1e30) never reaches the planes.
 * A PSF that equals an outer product c_b r_a to within 1e-6 of its largest
 * tap (a sampled Gaussian) is applied as a row pass then a column pass; the
 * result differs from the direct double sum by binary32 rounding only.
 *
 *   sci, var : device float [T][H][W]
 *   mask     : device uint8 [T][H][W], nonzero = masked; may be NULL
 *   psf      : host float [psf_k][psf_k], row = y, col = x; not normalised
 *              by the library; psf_k odd, 1 <= psf_k <= KBM_MAX_PSF
 *   psi, phi : device float [T][H][W], written
 */
kbm_status kbm_make_planes(const kbm_stack *s, const float *sci,
                           const float *var, const uint8_t *mask,
                           const float *psf, int32_t psf_k, float *psi,
                           float *phi, hipStream_t stream);

/* Search parameters (Section 3.1 and 3.2). */
typedef struct {
    const float *vel;   /* host [num_vel][2] (vx, vy) px/day, finite */
    int32_t num_vel;    /* >= 1 */
    int32_t k;          /* results kept per start pixel, 1..KBM_MAX_K */
    int32_t min_obs;    /* minimum usable epochs, >= 1 */
    int32_t sigmag;     /* 1 = in-line sigma_G filter, 0 = plain sums */
    double q_lo, q_hi;  /* quantiles, 0 <= q_lo < q_hi <= 1 (0.25, 0.75) */
    double coeff;       /* sigma_G = coeff * (x_hi - x_lo), >= 0 (0.7413) */
    double n_sigma;     /* keep |nu - median| <= n_sigma * sigma_G (2.0) */
    int32_t x_begin, y_begin, x_end, y_end; /* start pixels [begin, end) */
} kbm_search_params;

/* Search results, device SoA arrays [Hr][Wr][k] with Hr = y_end - y_begin,
 * Wr = x_end - x_begin.  Slot order: best first.  Empty slot: lh = -inf,
 * flux = 0, vel_idx = -1, n_obs = 0, keep = 0, lh_raw = -inf. */
typedef struct {
    float *lh;          /* filtered likelihood L' = Psi'/sqrt(Phi') */
    float *flux;        /* Psi'/Phi' */
    int32_t *vel_idx;   /* index into the velocity list */
    int16_t *n_obs;     /* usable epochs before filtering */
    uint64_t *keep;     /* bit i: epoch i kept by the filter */
    float *lh_raw;      /* unfiltered likelihood; may be NULL */
} kbm_results;

/* Bytes of device workspace kbm_search needs for these stacks/params. */
kbm_status kbm_search_workspace_size(const kbm_stack *stacks,
                                     const kbm_search_params *p,
                                     int32_t num_stacks, size_t *bytes);

/*
 * kbm_search - exhaustive linear-trajectory search with the in-line sigma_G
 * filter and per-pixel top-K (Section 3, 3.1, 3.2).
 *
 * For start pixel p and velocity v, epoch i is usable when p + off_i(v) lies
 * in the image and phi_i > 0 there (and psi, phi are finite).  n_obs =
 * number of usable epochs.  Plain sums Psi, Phi over usable epochs give
 * lh_raw = Psi/sqrt(Phi).  With sigmag = 1, over the usable epochs:
 * nu_i = psi_i / sqrt(phi_i); x_q = sorted(nu)[floor(q (n_obs-1) + 1/2)] for
 * q in {q_lo, 1/2, q_hi}; sigma_G = coeff (x_hi - x_lo); epoch i is kept iff
 * |nu_i - x_1/2| <= n_sigma sigma_G (this decision is taken in binary32);
 * L' = Psi'/sqrt(Phi') over kept epochs.  With sigmag = 0, L' = lh_raw and
 * keep = usable.  Trajectories with n_obs < min_obs or non-finite L' are
 * dropped.  Each start pixel keeps its k best by L' (ties: smaller velocity
 * index first).
 *
 *   stacks, p, out : host arrays [num_stacks]
 *   psi, phi       : host arrays [num_stacks] of device float [T][H][W]
 *   workspace      : device, >= kbm_search_workspace_size bytes
 */
kbm_status kbm_search(const kbm_stack *stacks, const float *const *psi,
                      const float *const *phi, const kbm_search_params *p,
                      kbm_results *out, int32_t num_stacks, void *workspace,
                      size_t workspace_bytes, hipStream_t stream);

/*
 * Batched persistent search - kbm_search's result for many independent
 * stacks (the paper searches each CCD of each pointing separately, Section
 * 2, and runs the search many times over, Section 3) from ONE persistent
 * kernel launch, replayed from a captured HIP graph.
 *
 * Work items are (stack, 64-pixel row tile, block of vel_block velocities).
 * Eight queues, one per XCD, each hold a contiguous strip of every stack's
 * tiles, ordered velocity-block-major and, within a block, by descending
 * cost per item (longest-processing-time first).  Workgroups take items
 * from their own XCD's queue with an atomic counter and then from the other
 * queues.  A tile's running top-K lists pass from one velocity block to the
 * next through the workspace; a per-tile progress counter orders them.  The
 * item that covers a tile's last velocity block writes its results.
 * Results are bit-identical to kbm_search on the same inputs (the ranking
 * is a total order, so the schedule cannot change it).
 *
 * Limits: T <= 32, k <= 8, and T*H*W*8 bytes of packed planes per stack
 * below 2^32 (otherwise KBM_ERR_UNSUPPORTED: use kbm_search).
 */
typedef struct {
    int32_t vel_block;     /* velocities per work item, >= 32 */
    int32_t tile_cols;     /* super-tile width in 64-pixel tiles: 1,2,4,8,16 */
    int32_t tile_rows;     /* super-tile height in rows: 1,2,4,...,64 */
    int32_t waves;         /* wavefronts per workgroup sharing a tile: 1 or 4 */
    int32_t blocks_per_cu; /* persistent workgroups per CU; 0 = all that fit */
    int32_t sweep;         /* velocity order of a workgroup's waves: 0 = wave w
                              takes every waves-th velocity from w, 1 = wave w
                              takes the w-th contiguous share of the block */
    float probe_ms;        /* out: time of this schedule on the autotuner's
                              probe (0 when not tuned) */
} kbm_schedule;

#define KBM_TUNE_DEFAULT 0 /* built-in schedule: vel_block 1024, 2 x 32
                              super-tiles, 4 waves, all that fit, sweep 1 if
                              some stack has >= 16384 velocities else 0 */
#define KBM_TUNE_AUTO 1    /* time candidate schedules on a probe, keep the
                              fastest if a full run confirms that it beats
                              the built-in schedule; cached per process and
                              in a file by library build id, GPU
                              architecture and batch shape (see
                              kbm_tune_cache_clear) */
#define KBM_TUNE_GIVEN 2   /* use *schedule as given */

typedef struct kbm_batch kbm_batch; /* opaque plan with its captured graph */

/* Bytes of device workspace kbm_batch_create needs (any schedule). */
kbm_status kbm_batch_workspace_size(const kbm_stack *stacks,
                                    const kbm_search_params *p,
                                    int32_t num_stacks, size_t *bytes);

/*
 * kbm_batch_create - validate, build the offset tables and work queues in
 * the workspace, pick the schedule (tune), and capture the launch sequence
 * (clear control block -> pack planes -> persistent search) into a graph.
 * Synchronous: returns when the workspace is ready.  With KBM_TUNE_AUTO it
 * runs the search several times on a probe (a sixteenth of every stack's
 * tiles, from the middle of each XCD's share), then the whole batch under
 * the probe's winner and under the built-in schedule, overwriting `out`.
 *
 *   stacks, p, out, psi, phi : as kbm_search.  The device pointers (psi,
 *       phi, result arrays, workspace) are baked into the graph: they must
 *       stay valid until kbm_batch_destroy; their contents may change
 *       between runs (new images of the same geometry).
 *   schedule : in for KBM_TUNE_GIVEN; out (may be NULL otherwise): the
 *       schedule in use.
 *   batch    : out, the plan; free with kbm_batch_destroy.
 */
kbm_status kbm_batch_create(const kbm_stack *stacks, const float *const *psi,
                            const float *const *phi,
                            const kbm_search_params *p, kbm_results *out,
                            int32_t num_stacks, void *workspace,
                            size_t workspace_bytes, int32_t tune,
                            kbm_schedule *schedule, hipStream_t stream,
                            kbm_batch **batch);

/* Enqueue one run of the captured graph on `stream` (asynchronous). */
kbm_status kbm_batch_run(kbm_batch *b, hipStream_t stream);

/* Synchronise `stream` and report whether a dependency wait of the last
 * completed run gave up (stalled != 0: that run's results are not valid).
 * Each wait is bounded, so a run always ends. */
kbm_status kbm_batch_check(kbm_batch *b, hipStream_t stream, int32_t *stalled);

/* Report how many trajectory-epochs (start pixel x velocity x epoch) one run
 * of the plan evaluates: the nominal W*H*V*T of every search region minus
 * the (64-pixel row tile, velocity) pairs that the kernel skips because
 * some epoch of the tile leaves the image and no start pixel of the tile can
 * keep min_obs epochs inside it (their slots are empty either way).  The
 * skip depends only on the geometry, so the count is fixed when the plan is
 * created and computed on the host from the same offset tables the kernel
 * reads (a counter inside the sweep would cost it registers); `stream` is
 * not used. */
kbm_status kbm_batch_evaluated(kbm_batch *b, hipStream_t stream, uint64_t *traj_epochs);

/* Forget the autotuner's choices held in this process.  The choices also
 * persist in a JSON file, KBM_TUNE_CACHE if that environment variable is
 * set (empty: no file), else $HOME/.cache/kbm/autotune.json; a later
 * KBM_TUNE_AUTO plan of a shape found there uses the stored schedule and
 * probe time without tuning again.  Delete the file to re-tune. */
kbm_status kbm_tune_cache_clear(void);

/* Release the plan (graph, stream, host buffers); NULL is a no-op. */
kbm_status kbm_batch_destroy(kbm_batch *b);

/*
 * kbm_sigmag_filter - the sigma_G lightcurve filter of Section 3.1 on n
 * independent lightcurves, with the same rule and precision as kbm_search.
 *
 *   psi_curve  : device float [n][T]
 *   phi_curve  : device float [n][T]; NULL means phi = 1 (the values in
 *                psi_curve are filtered directly and L' = sum / sqrt(count))
 *   valid      : device uint8 [n][T], 0 = epoch absent; may be NULL
 *   keep       : device uint64 [n], written
 *   lh_filtered: device float [n] (L', -inf if nothing participates); may
 *                be NULL
 * An epoch participates when valid != 0, phi > 0 and psi, phi are finite.
 * T in [1, KBM_MAX_EPOCHS]; n >= 0.
 */
kbm_status kbm_sigmag_filter(const float *psi_curve, const float *phi_curve,
                             const uint8_t *valid, int64_t n, int32_t T,
                             double q_lo, double q_hi, double coeff,
                             double n_sigma, uint64_t *keep,
                             float *lh_filtered, hipStream_t stream);

/*
 * kbm_sigmag_filter_ex - kbm_sigmag_filter with the variants Section 3.1
 * leaves to the user: the filtered per-epoch value is psi/sqrt(phi)
 * (quantity 0, the likelihood; what kbm_sigmag_filter and the search use)
 * or psi/phi (quantity 1, the flux); and a post-filter flag
 * pass = (L' >= lh_min) (the paper keeps trajectories whose recomputed
 * likelihood clears a threshold, 10 in its searches).
 *
 *   pass : device uint8 [n] or NULL; 0 for curves with no usable epoch
 * Other arguments as kbm_sigmag_filter; lh_min may be -inf, not NaN.
 */
kbm_status kbm_sigmag_filter_ex(const float *psi_curve, const float *phi_curve,
                                const uint8_t *valid, int64_t n, int32_t T,
                                int32_t quantity, double q_lo, double q_hi,
                                double coeff, double n_sigma, double lh_min,
                                uint64_t *keep, float *lh_filtered,
                                uint8_t *pass, hipStream_t stream);

/*
 * kbm_sigmag_coeff - the constant C of Eq. 3 for a quantile pair, with the
 * sqrt(2) that Eq. 4 as printed drops: C = 1 / (sqrt(2) (erfinv(2 q_hi - 1)
 * - erfinv(2 q_lo - 1))), so C (x_hi - x_lo) estimates sigma for normal
 * data (0.741301... for 0.25, 0.75; the paper prints 0.7413).  Host only,
 * FP64; needs 0 < q_lo < q_hi < 1.
 */
kbm_status kbm_sigmag_coeff(double q_lo, double q_hi, double *coeff);

/*
 * kbm_refine - bilinear trajectory likelihood and its adjoint, used to
 * refine candidates to sub-pixel start positions and velocities.  (Not a
 * step of the paper; it continues Section 3's likelihood to real-valued
 * positions.)
 *
 * x_i = x0 + vx t_i, y_i = y0 + vy t_i (FP64 positions), B(P, x, y) the
 * bilinear sample with pixel centres at integer coordinates and zero
 * outside the image;  L = sum_{i in keep} B(psi_i) / sqrt(sum B(phi_i)),
 * L = 0 when the kept samples carry no phi.
 *
 *   psi, phi    : device float [T][H][W]
 *   params      : device float [n][4] (x0, y0, vx, vy)
 *   keep        : device uint64 [n]; NULL = all epochs
 *   lh          : device float [n], written
 *   grad_lh     : device float [n] upstream gradient g; NULL = forward only
 *   grad_params : device float [n][4], overwritten with g * dL/dparams
 *                 (required when grad_lh != NULL)
 *   grad_psi, grad_phi : device float [T][H][W], g * dL/dplane is ADDED
 *                 (float atomics, order not deterministic); may be NULL
 * Derivatives at integer coordinates are the right-sided ones.
 */
kbm_status kbm_refine(const kbm_stack *s, const float *psi, const float *phi,
                      int64_t n, const float *params, const uint64_t *keep,
                      float *lh, const float *grad_lh, float *grad_params,
                      float *grad_psi, float *grad_phi, hipStream_t stream);

/*
 * kbm_refine_adam - the refinement loop in one launch: `steps` gradient-
 * ascent steps of Adam (Kingma & Ba 2015) on the likelihood of kbm_refine,
 * then L at the final parameters.  Candidates are independent, so each
 * lane runs its candidate's whole loop with the Adam moments in registers;
 * the result equals, bit for bit, alternating kbm_refine (upstream gradient
 * 1) and kbm_adam_step (maximize, step k) for k = 1 .. steps, then
 * kbm_refine forward.  (Not a step of the paper: it refines search
 * candidates to sub-pixel starts and real-valued velocities.)
 *
 *   params : device float [n][4] (x0, y0, vx, vy), updated in place
 *   keep   : device uint64 [n]; NULL = all epochs
 *   lr     : host float [steps][4], the step size of each step and column
 *   steps  : 1 .. 64 (KBM_ERR_UNSUPPORTED above)
 *   beta1, beta2, eps : as kbm_adam_step
 *   lh     : device float [n], written: L at the returned params
 */
kbm_status kbm_refine_adam(const kbm_stack *s, const float *psi, const float *phi,
                           int64_t n, float *params, const uint64_t *keep,
                           const float *lr, int32_t steps, double beta1,
                           double beta2, double eps, float *lh, hipStream_t stream);

/*
 * kbm_score_trajectories - targeted evaluation: the search's filtered
 * likelihood (Section 3, 3.1) for an explicit list of linear trajectories
 * with real-valued starts, e.g. refined candidates or known objects.
 *
 * Epoch i samples the pixel (floor((x0 + vx t_i) + 1/2), floor((y0 + vy t_i)
 * + 1/2)) with t_i from the earliest epoch, each product and sum rounded in
 * FP64 as written.  Usable epochs, n_obs, the sigma_G keep rule (binary32
 * decision) and L' are those of kbm_search; an integer start on a velocity
 * of the search grid reproduces the search's values for that trajectory.
 * A trajectory the search would drop (n_obs < min_obs, non-finite L') gets
 * the empty-slot values (lh = lh_raw = -inf, flux 0, keep 0); n_obs is
 * always written.
 *
 *   psi, phi : device float [T][H][W]
 *   params   : device float [n][4] (x0, y0, vx, vy), 16-byte aligned
 *   lh, flux : device float [n]; keep: device uint64 [n]; n_obs: device
 *              int16 [n]; lh_raw: device float [n] or NULL
 */
kbm_status kbm_score_trajectories(const kbm_stack *s, const float *psi,
                                  const float *phi, int64_t n,
                                  const float *params, int32_t min_obs,
                                  int32_t sigmag, double q_lo, double q_hi,
                                  double coeff, double n_sigma, float *lh,
                                  float *flux, uint64_t *keep, int16_t *n_obs,
                                  float *lh_raw, hipStream_t stream);

/*
 * kbm_stamps - median coadded postage stamps along trajectories and the
 * central-moment cut of Section 3.3.
 *
 * For trajectory j (params x0, y0, vx, vy) and epoch i, the stamp is the
 * (2r+1) x (2r+1) window of the science image centred on the pixel
 * (floor((x0 + vx t_i) + 1/2), floor((y0 + vy t_i) + 1/2)) (FP64, as in
 * kbm_score_trajectories).  A stamp pixel of an epoch is usable when it lies
 * in the image, is unmasked, sci and var are finite and var > 0, and (with
 * `keep` given) bit i of keep[j] is set.  The coadd pixel is the median of
 * its usable values (the mean of the two middle values for an even count,
 * in binary32), 0 if none.  With S the coadd, offsets dx, dy from its centre
 * pixel and sums in FP64: moments = (sum S, x, y, xy, xx, yy) with
 * x = sum dx S / sum S, ..., yy = sum dy^2 S / sum S (NaN if sum S <= 0).
 * pass = |x| < lim[0] && |y| < lim[1] && |xy| < lim[2] && xx < lim[3] &&
 * yy < lim[4] (strict; the paper's limits 0.5, 0.5, 1.5, 36.5, 36.5).
 *
 *   sci, var : device float [T][H][W]; mask: device uint8 [T][H][W] or NULL
 *   params   : device float [n][4], 16-byte aligned
 *   keep     : device uint64 [n] or NULL (all epochs)
 *   radius   : r in [1, 15] (the paper's stamps are 21 x 21: r = 10)
 *   limits   : host double [5], or NULL for the paper's
 *   coadd    : device float [n][2r+1][2r+1] or NULL
 *   moments  : device double [n][6]; pass: device uint8 [n]
 */
kbm_status kbm_stamps(const kbm_stack *s, const float *sci, const float *var,
                      const uint8_t *mask, int64_t n, const float *params,
                      const uint64_t *keep, int32_t radius,
                      const double *limits, float *coadd, double *moments,
                      uint8_t *pass, hipStream_t stream);

/*
 * kbm_detect - the decision of the targeted (known-object) mode: trajectory
 * j is detected when n_obs[j] >= min_obs, lh[j] >= lh_min (the paper keeps
 * trajectories whose recomputed likelihood clears a threshold, Section 3.1)
 * and its coadded stamp passes the moment cut (Section 3.3).  NaN lh never
 * passes.
 *   lh: device float [n]; n_obs: device int16 [n]; stamp_pass: device
 *   uint8 [n]; detected: device uint8 [n], written (0 or 1)
 */
kbm_status kbm_detect(int64_t n, const float *lh, const int16_t *n_obs,
                      const uint8_t *stamp_pass, int32_t min_obs, float lh_min,
                      uint8_t *detected, hipStream_t stream);

/*
 * kbm_extract_top - candidate extraction: the global top-N result slots by
 * filtered likelihood with L' >= lh_min (the paper hands trajectories whose
 * recomputed likelihood clears a threshold on from the GPU, Section 3.1, and
 * keeps per-pixel lists, Section 3.2; this collects them across pixels).
 *
 * Slots are ranked by L' descending, then by flat slot index
 * ((y - y_begin) * Wr + (x - x_begin)) * k + slot ascending; empty and
 * non-finite slots never qualify.  The first min(n_max, #qualifying) are
 * written in increasing flat index order.
 *
 *   r         : device results of kbm_search, [Hr][Wr][k]
 *   vel       : host [num_vel][2], the velocity list the search used
 *   params    : device float [n_max][4] out: (x, y, vx, vy) of each slot
 *   lh        : device float [n_max] out
 *   flux, keep, index (int64 flat slot index), n_obs : device, may be NULL
 *   n_out     : device int64 [1], number written
 *   workspace : device, >= kbm_extract_workspace_size bytes
 * Hr*Wr*k must be below 2^32.
 */
kbm_status kbm_extract_workspace_size(int32_t Hr, int32_t Wr, int32_t k,
                                      int32_t num_vel, size_t *bytes);
kbm_status kbm_extract_top(const kbm_results *r, int32_t Hr, int32_t Wr,
                           int32_t k, int32_t x_begin, int32_t y_begin,
                           const float *vel, int32_t num_vel, float lh_min,
                           int64_t n_max, float *params, float *lh, float *flux,
                           uint64_t *keep, int64_t *index, int16_t *n_obs,
                           int64_t *n_out, void *workspace,
                           size_t workspace_bytes, hipStream_t stream);

/*
 * kbm_extract_top_noalloc - kbm_extract_top for callers that cannot
 * allocate device or pinned host memory: code under HIP graph capture,
 * tight serving loops, hosts that forbid allocation.  It calls no
 * hipMalloc, hipFree or hipHostMalloc and copies nothing from the host.
 *
 * Same selection, order, outputs and limits as kbm_extract_top, except:
 *   vel_dev : DEVICE float [num_vel][2], the velocity list the search used
 *   (no workspace argument)
 * Scratch: the radix-select state and per-block counts live in a static
 * device array of the library, KBM_EXTRACT_SCRATCH_BYTES per GPU, held
 * until the process ends; every call needs at most that much, whatever the
 * number of slots (below 2^32).  All calls on one GPU share it and it keeps
 * the last call's contents (each call re-initialises what it reads): calls
 * that overlap on one GPU race and must be serialised by the caller, e.g.
 * on one stream.
 */
#define KBM_EXTRACT_SCRATCH_BYTES 17664
kbm_status kbm_extract_top_noalloc(const kbm_results *r, int32_t Hr, int32_t Wr,
                                   int32_t k, int32_t x_begin, int32_t y_begin,
                                   const float *vel_dev, int32_t num_vel,
                                   float lh_min, int64_t n_max, float *params,
                                   float *lh, float *flux, uint64_t *keep,
                                   int64_t *index, int16_t *n_obs, int64_t *n_out,
                                   hipStream_t stream);

/*
 * kbm_adam_step - one Adam update (Kingma & Ba 2015, Algorithm 1) of the
 * refinement parameters, the optimiser that drives kbm_refine's gradient
 * ascent.  With g the gradient (negated when maximize != 0):
 *   m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2
 *   p <- p - lr[c] * (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps)
 * where c is the column of the element (row-major [n][cols]).
 *
 *   params, m, v : device float [n][cols], updated in place
 *   grad         : device float [n][cols]
 *   lr           : host float [cols]; cols in [1, 8]; step >= 1
 */
kbm_status kbm_adam_step(float *params, const float *grad, float *m, float *v,
                         int64_t n, int32_t cols, const float *lr,
                         double beta1, double beta2, double eps, int32_t step,
                         int32_t maximize, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* KBM_H */
