/*
 * tno_search.h -- C ABI of the MI355X matched-filter trajectory search.
 *
 * Method (Ganapathi, arXiv:2209.09848, Sec. 3.2 "Matched Filter", eq. 4, and
 * Sec. 3.3 "Interpreting Scores"): for every candidate constant-velocity
 * trajectory j and every start pixel (x0, y0), the matched filter is the
 * trajectory line convolved with the pixel response function (PRF); applying
 * it is the dot product of filter and residual data, which estimates the
 * object's total flux; the bank's maximum gives the most likely trajectory;
 * scores above a threshold are candidates.  With the Gaussian noise model of
 * Sec. 3.2 (per-pixel sigma, bright pixels clipped), the maximum-likelihood
 * form is
 *
 *   ivar(y,x)  = 1/sigma(y,x)^2  (0 where sigma is <= 0 or not finite, and
 *                                 0 off the image)
 *   D          = v_j * (t_k - t_ref)   (per axis, FP64)
 *   i = floor(D + 1/2), f = D - i      (anchor, sub-pixel phase)
 *   W_jk(a,b)  = g(a; f_y) g(b; f_x), g the unit-sum Gaussian PRF profile
 *   nu   = sum_k sum_ab W_jk(a,b) R_k(y0+i_y+a, x0+i_x+b) ivar(...)
 *   Lam  = sum_k sum_ab W_jk(a,b)^2 ivar(...)
 *   SNR  = nu / sqrt(Lam),  flux = nu / Lam   (0 where Lam == 0)
 *
 * Coordinates: x = column, y = row, pixel centres at integers.  All 2-D
 * arrays are row-major [H][W]; the residual stack is [T][H][W].
 *
 * Calls on one handle are serialised internally; tno_search_destroy must not
 * race other calls on the same handle.  No C++ exception crosses this ABI.
 * On any error the out-parameters (handle, ticket) are not written and no
 * output buffer is touched.
 */
#ifndef TNO_SEARCH_H
#define TNO_SEARCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define TNO_OK 0
#define TNO_PENDING 1          /* poll only: work not finished yet */
#define TNO_E_INVAL (-1)       /* bad argument (message says which) */
#define TNO_E_NOMEM (-2)       /* footprint can never fit the HBM budget, or allocation failed
                                  with nothing in flight */
#define TNO_E_BUSY (-3)        /* in-flight limit or budget full right now, or allocation failed
                                  while requests are in flight; retry later */
#define TNO_E_DEVICE (-4)      /* HIP runtime or kernel error */
#define TNO_E_TICKET (-5)      /* unknown ticket, or already collected */
#define TNO_E_CANCELLED (-6)   /* request cancelled */
#define TNO_E_INTERNAL (-7)    /* internal invariant broken */

/* ---------------------------------------------------------------- enums */
/* Storage type of the residual stack. */
#define TNO_F32 0
#define TNO_BF16 1             /* bfloat16 codes, per-tile power-of-two scales */
#define TNO_F16 2              /* IEEE binary16 codes, per-tile scales */
#define TNO_FP8_E4M3 3         /* OCP E4M3 "fn" codes, per-tile scales */

/* PRF model (Sec. 2: PRF; Sec. 3.2: filter = trajectory line (x) PRF). */
#define TNO_PRF_GAUSS_SAMPLED 0     /* exp(-(b-f)^2 / (2 s^2)) at pixel centres */
#define TNO_PRF_GAUSS_INTEGRATED 1  /* Gaussian integrated over each pixel */
#define TNO_PRF_TABLE 2             /* caller's tabulated PRF (Sec. 2: the share of a point
                                       source's flux each pixel records), not separable in
                                       general; read at the sub-pixel phase by bilinear
                                       interpolation (see tno_prf) */

/* Largest oversampling of a tabulated PRF. */
#define TNO_MAX_TABLE_Q 64

/* Side of the square quantisation tiles of the reduced-precision stacks. */
#define TNO_QTILE 64

/* tno_config.flags */
#define TNO_CFG_GRAPHS 1u           /* run each request's kernels and device copies as one HIP
                                       graph: captured at submit, used to update an executable
                                       graph of the same structure left by an earlier request
                                       (instantiated the first time), then launched; the phase
                                       times of tno_result are 0 in this mode.  Needs an own
                                       stream pool or a non-default stream. */
#define TNO_CFG_AUTOTUNE 2u         /* time the search's tile shapes and trajectory blocks on the
                                       first request of each shape class; keep the fastest */
#define TNO_CFG_BATCH 4u            /* continuous batching: the search of every admitted request
                                       is cut into chunks of its (tile, trajectory) work items;
                                       steps -- single launches whose block ranges serve the
                                       chunks of several requests -- run on two search streams,
                                       at most two steps queued at a time, so a request admitted
                                       while others run joins the next step.  Each request's
                                       preparation and reductions run on its pool stream.
                                       Results are bit-identical to unbatched requests.  Needs
                                       the own stream pool (stream NULL) and excludes GRAPHS;
                                       steps are formed whenever submit or poll is called, so
                                       the caller's thread must not stall: combine with
                                       TNO_CFG_RESERVE. */

#define TNO_CFG_RESERVE 8u          /* reserve the whole HBM budget at create as one device block
                                       and carve every request's arena and resident stack from it:
                                       no device allocation or free after create (a large one can
                                       hold the calling thread for hundreds of ms, which stalls
                                       batched steps, launched from submit and poll).  Other users
                                       of the GPU see the budget as taken.  TNO_E_NOMEM from create
                                       if the block cannot be had. */

/* tno_request.flags */
#define TNO_REQ_DEVICE_PTRS 1u      /* every input and output pointer is device memory */
#define TNO_REQ_VALIDATE 2u         /* also scan inputs for non-finite values */
#define TNO_REQ_STAGE_FP32 4u       /* reduced-precision residuals: decode them into a
                                       zero-padded FP32 copy (about T*(H+2P)*(W+2P)*4 bytes,
                                       P the largest trail shift, up to 512) before the search,
                                       which then runs faster.  Without this flag, stamps of
                                       side 1, 3 and 5 with W % 4 == 0 and H*W*4 < 2^31 read
                                       the codes in place (decoded, scaled and weighted while
                                       each window is staged): no copy, a slower search.
                                       FP32 residuals are always staged. */

/* Largest stamp side accepted (odd). */
#define TNO_MAX_STAMP 15

/* ---------------------------------------------------------------- types */
typedef struct tno_search tno_search;   /* opaque handle */

typedef struct {
    int32_t device;              /* HIP device ordinal */
    int32_t max_inflight;        /* tickets admitted at once (<= 0: 64) */
    uint64_t hbm_budget_bytes;   /* device bytes the handle may hold (0: 90% of the memory
                                    free at create; a caller that allocates device memory
                                    after creating the handle passes a budget that leaves
                                    room for it and for the HIP runtime's own needs) */
    uint32_t flags;              /* TNO_CFG_* */
    uint32_t reserved;           /* must be 0 */
    void *stream;                /* hipStream_t to run on, or NULL for an own stream */
    const char *tune_cache_path; /* text tuning cache read at create and rewritten after each
                                    tuning (one line per arch and shape class), or NULL */
    uint64_t slab_bytes;         /* device bytes of one trajectory slab (0: 4 GiB).  A request
                                    searches its trajectories in slabs, consecutive runs of its
                                    velocity-sorted search order: the FP64 normaliser (8 bytes
                                    per start pixel and trajectory) and the slab's SNR and flux
                                    maps (4 bytes each) exist for one slab at a time; the bank
                                    maximum, per-trajectory peaks and top-k are merged slab
                                    after slab, and maps the caller asked for receive each
                                    slab's rows.  A slab holds at least one trajectory.
                                    Results do not depend on it. */
} tno_config;

/* Stamp weights of frame k (Sec. 3.2): with phase (f_y, f_x) in [-1/2, 1/2)
 * of the trail position, pixel (a, b) of the stamp, a, b = -h..h, weighs
 *   Gaussian kinds:  g(a - f_y) g(b - f_x), each 1-D profile scaled to unit sum;
 *   TNO_PRF_TABLE:   P(a - f_y, b - f_x), as given (no renormalisation), where
 *                    P is `table` [n][n], n = (S+1)*table_q + 1, row-major with
 *                    rows along y, sampling offsets u = -(h+1) + i/table_q
 *                    (i = 0..n-1) from the source, read between samples by
 *                    bilinear interpolation (FP64).  Values are used as given;
 *                    non-finite entries make non-finite scores. */
typedef struct {
    int32_t kind;                /* TNO_PRF_* */
    int32_t stamp;               /* odd side S of the S x S stamp, 1..TNO_MAX_STAMP */
    double sigma_px;             /* Gaussian sigma in pixels, > 0 (ignored for TNO_PRF_TABLE) */
    const double *table;         /* TNO_PRF_TABLE: [n][n] samples as above (copied at submit;
                                    host memory unless TNO_REQ_DEVICE_PTRS); else ignored */
    int32_t table_q;             /* TNO_PRF_TABLE: samples per pixel, 1..TNO_MAX_TABLE_Q */
    int32_t reserved;            /* must be 0 */
} tno_prf;

typedef struct {
    int32_t height, width;       /* H, W > 0 */
    int32_t n_frames;            /* T > 0 */
    int32_t dtype;               /* TNO_F32 / TNO_BF16 / TNO_F16 / TNO_FP8_E4M3 */
    const void *residuals;       /* [T][H][W] of dtype (float, or uint16/uint8 codes); NULL to
                                    search the stack resident under stack_key */
    const float *tile_scales;    /* [T][ceil(H/64)][ceil(W/64)]: value = code * scale;
                                    required with residuals unless dtype == TNO_F32 */
    const float *sigma;          /* [H][W] per-pixel noise sigma; required with residuals
                                    (a resident stack keeps its own) */
    const double *times;         /* [T] frame times, any finite values (gaps allowed) */
    double t_ref;                /* reference time of the start pixel; NaN: times[0] */
    tno_prf prf;
    int32_t n_traj;              /* J >= 1 */
    int32_t top_k;               /* candidates wanted, 0..TNO_MAX_TOPK */
    const double *velocities;    /* [J][2] = (vx, vy) in pixels per unit of `times` */
    const double *jitter;        /* [T][2] = (theta_x, theta_y): pointing jitter of each frame
                                    in pixels (Sec. 2.1, 3.1), added to the trail position of
                                    every trajectory in that frame: v*(t_k - t_ref) + theta_k;
                                    finite, |theta| <= 256; NULL: none */
    int32_t sig_box;             /* 0: no significance map; else the odd side of the square
                                    window (e.g. 255) over which the local standard deviation
                                    of the best-score map is taken (Sec. 3.3) */
    float sig_threshold;         /* detections: significance >= this (e.g. 3 or 5) */
    uint64_t stack_key;          /* 0, or a key: with residuals, the library keeps a device copy
                                    of residuals, scales and sigma under the key (evicted least
                                    recently used when the budget needs room); with NULL
                                    residuals the resident copy is searched (TNO_E_INVAL if the
                                    key is not resident or has another shape or dtype) */
    uint32_t flags;              /* TNO_REQ_* */
    uint32_t reserved;           /* must be 0 */
} tno_request;

#define TNO_MAX_TOPK 1024

typedef struct {
    float snr, flux;
    int32_t y, x;                /* start pixel of the trajectory's best score */
} tno_peak;

typedef struct {
    float snr, flux;
    int32_t traj, y, x;
} tno_candidate;

/* A detection of the Sec. 3.3 significance test: the pixel's best score over
 * the bank in units of the local standard deviation of the best-score map. */
typedef struct {
    float significance, snr, flux;
    int32_t traj, y, x;
} tno_detection;

#define TNO_MAX_DETECTIONS 1024

/* Outputs; every pointer may be NULL (= not produced).  Host or device memory
 * according to TNO_REQ_DEVICE_PTRS.  Caller-owned; written only between a
 * successful submit and the ticket's terminal poll. */
typedef struct {
    float *snr;                  /* [J][H][W]; NULL: never held whole on the device (each
                                    trajectory slab's rows only, see slab_bytes) */
    float *flux;                 /* [J][H][W]; NULL: likewise */
    float *best_snr;             /* [H][W] max over the bank, ties to the lowest j */
    int32_t *best_traj;          /* [H][W] arg-max j */
    tno_peak *traj_max;          /* [J] per-trajectory max, ties to the smallest y*W+x */
    tno_candidate *topk;         /* [top_k] SNR descending, then j*H*W+y*W+x ascending */
    float *significance;         /* [H][W] best_snr / local std over sig_box x sig_box
                                    (0 where the std is 0); needs sig_box > 0 */
    tno_detection *detections;   /* [max_detections] pixels with significance >=
                                    sig_threshold, significance descending then y*W+x
                                    ascending; needs sig_box > 0 */
    int32_t max_detections;      /* capacity of detections, 0..TNO_MAX_DETECTIONS */
    int32_t reserved;            /* must be 0 */
} tno_outputs;

typedef struct {
    int32_t status;              /* TNO_OK or a TNO_E_* code */
    int32_t n_topk;              /* candidates written (min(top_k, J*H*W)) */
    int32_t n_detections;        /* detections written (<= max_detections) */
    int32_t n_above;             /* pixels with significance >= sig_threshold */
    uint64_t updates;            /* J*H*W*T (trajectory x pixel x frame terms) */
    double queue_ms;             /* total_ms - device_ms (host staging, queueing, polling) */
    double device_ms;            /* device start -> device end (HIP events) */
    double total_ms;             /* submit -> completion seen by poll */
    /* device time per phase (HIP events on the request's stream): */
    double prep_ms;              /* ivar and the inverse-variance-weighted stack */
    double table_ms;             /* FP64 offset/PRF table and trail kernels */
    double lambda_ms;            /* FP64 normaliser */
    double search_ms;            /* numerator gather-stencil + SNR/flux epilogue */
    double reduce_ms;            /* bank maximum, per-trajectory maximum, top-k, copies */
    char message[160];           /* human-readable detail for errors */
} tno_result;

/* ---------------------------------------------------------------- calls */

/* Create a search handle on cfg->device.  Returns TNO_OK and writes
 * *out_handle, or TNO_E_INVAL (NULL args, reserved != 0), TNO_E_DEVICE (no
 * such device / HIP failure).  The handle owns its device memory. */
int tno_search_create(const tno_config *cfg, tno_search **out_handle);

/* Enqueue one search (Sec. 3.2 eq. 4 over the whole trajectory bank, then the
 * Sec. 3.2/3.3 reductions).  Host inputs are fully read before the call
 * returns; with TNO_REQ_DEVICE_PTRS inputs are borrowed until the terminal
 * poll and must stay unmodified.  Returns TNO_OK and writes *out_ticket, or
 * TNO_E_INVAL / TNO_E_NOMEM / TNO_E_BUSY / TNO_E_DEVICE; on error nothing is
 * enqueued.  tno_search_last_error() holds the message of a refusal.  A device
 * allocation that fails (memory held outside the handle) first frees the
 * handle's cached blocks, then its idle resident stacks, least recently used
 * first. */
int tno_search_submit(tno_search *h, const tno_request *req, const tno_outputs *out,
                      uint64_t *out_ticket);

/* Wait up to timeout_ms (0: just test, < 0: forever) for a ticket.  Returns
 * TNO_PENDING if not finished (out_result untouched), else the terminal status,
 * filling *out_result; the ticket is then retired (a second poll gives
 * TNO_E_TICKET). */
int tno_search_poll(tno_search *h, uint64_t ticket, int32_t timeout_ms, tno_result *out_result);

/* Cancel pending work, free every device buffer, destroy the handle.
 * Tickets still live are cancelled (nothing is copied back to host outputs;
 * work already enqueued drains first).  destroy(NULL) is a no-op. */
void tno_search_destroy(tno_search *h);

/* Cancel a live ticket: its results are discarded.  Work already enqueued on
 * the device runs to completion (device outputs may hold partial results);
 * nothing is copied to host outputs.  The ticket's terminal poll then returns
 * TNO_E_CANCELLED and releases its memory.  Returns TNO_OK, TNO_E_INVAL (NULL
 * handle) or TNO_E_TICKET (unknown or collected ticket). */
int tno_search_cancel(tno_search *h, uint64_t ticket);

/* Memory and queue state of a handle (monitoring; not part of the method). */
typedef struct {
    uint64_t budget_bytes;       /* HBM budget of the handle */
    uint64_t in_use_bytes;       /* device bytes charged to live requests and resident stacks */
    uint64_t held_bytes;         /* recomputed sum of those blocks' sizes (equals in_use_bytes) */
    uint64_t cached_bytes;       /* device blocks kept for reuse (in_use + cached <= budget) */
    uint64_t device_allocs;      /* fresh device allocations attempted */
    int32_t inflight;            /* tickets not yet collected */
    int32_t resident_stacks;     /* stacks kept under a stack_key */
    uint64_t batch_steps;        /* TNO_CFG_BATCH: search steps launched so far */
    uint64_t batch_items;        /* TNO_CFG_BATCH: work items those steps covered */
    uint64_t batch_shared;       /* TNO_CFG_BATCH: steps that served more than one request */
    uint64_t reserved[1];
} tno_stats;

/* Fill *out with the handle's state.  Returns TNO_OK or TNO_E_INVAL. */
int tno_search_stats(tno_search *h, tno_stats *out);

/* Quantise an FP32 residual stack into reduced-precision codes with one
 * power-of-two scale per frame and 64x64 tile (the precision form's storage;
 * the paper states no precision).  For tile amax > 0 the scale is
 * s = 2^(ceil(log2 amax) - E), E = 8 for TNO_FP8_E4M3 and 15 for TNO_BF16 /
 * TNO_F16, else s = 1; codes hold round-to-nearest-even R/s (E4M3 saturates at
 * 448), so code * s is exact in FP32.  All pointers are device memory:
 * residuals [T][H][W] float, codes [T][H][W] (uint16 or uint8), tile_scales
 * [T][ceil(H/64)][ceil(W/64)] float.  Enqueued on `stream` (a hipStream_t, or
 * NULL for the null stream); returns TNO_OK, TNO_E_INVAL or TNO_E_DEVICE. */
int tno_quantize(int32_t n_frames, int32_t height, int32_t width, int32_t dtype,
                 const float *residuals, void *codes, float *tile_scales, void *stream);

/* ---------------------------------------------------------------- background re-fit */

/* The per-pixel re-fit that turns raw frames into the residual stack and
 * noise map the search reads (Sec. 3.1 eq. 1-3, Sec. 3.2 noise model).
 *
 * Per pixel, y_t = D_t - U(S_t): the raw frame minus the fixed low-resolution
 * scattered light upsampled bilinearly (grid point (a, b) at pixel
 * ((a + 1/2) H/sl_height - 1/2, (b + 1/2) W/sl_width - 1/2), edge values
 * beyond the outermost points).  y is regressed on the basis
 * x_t = (1, tx, ty, tx^2, ty^2, tx ty) of the frame's jitter (tx, ty); the one
 * Gram matrix inverse serves every pixel.  The Huber loss of eq. 3 is
 * minimised by a least-squares start and `iterations` rounds of least squares
 * on pseudo-data X beta + clip(y - X beta, -delta, delta).  beta = (B, B_x,
 * B_y, B_xx, B_yy, B_xy).  Noise model: pixels with B > bright_threshold are
 * masked (residuals 0, sigma 0); sigma0 is the rms of the other pixels'
 * residuals, then `sigma_rounds` times the rms of those within clip_sigma *
 * sigma0; residual samples beyond clip_sigma * sigma0 are set to 0.
 * Arithmetic is FP64; residuals are stored as FP32. */
typedef struct {
    int32_t height, width;       /* H, W > 0 */
    int32_t n_frames;            /* T >= 6 */
    int32_t sl_height, sl_width; /* scattered-light grid, >= 1 with `scattered`; else ignored */
    const float *data;           /* [T][H][W] raw frames D_t */
    const float *scattered;      /* [T][sl_height][sl_width] fixed scattered light (finite), or NULL */
    const double *jitter;        /* [T][2] = (tx, ty) pixels, finite, not degenerate (the
                                    basis must have full rank: TNO_E_INVAL otherwise) */
    double delta;                /* Huber threshold delta_0 in data units, > 0 (inf: least squares) */
    double bright_threshold;     /* mask pixels whose B exceeds this (inf: none; not NaN) */
    double clip_sigma;           /* kappa > 0 of the sigma rounds and the transient clip (inf: none) */
    int32_t iterations;          /* clip-and-solve rounds after the least-squares start, 0..1000 */
    int32_t sigma_rounds;        /* clipped re-estimates of sigma0, 0..100 */
    uint32_t flags;              /* must be 0: every pointer is device memory */
    uint32_t reserved;           /* must be 0 */
} tno_refit_request;

typedef struct {
    float *residuals;            /* [T][H][W] residual stack for the search (device) */
    float *sigma;                /* [H][W] sigma0, 0 at masked pixels (device) */
    double *coeffs;              /* [6][H][W] beta (device), or NULL */
    double sigma0;               /* written: the common noise sigma */
    int64_t n_clipped;           /* written: residual samples set to 0 by the clip */
    int64_t n_masked;            /* written: bright pixels */
    double device_ms;            /* written: device time of the re-fit (HIP events) */
} tno_refit_outputs;

/* Run the re-fit on `stream` (hipStream_t, NULL: the default stream) and wait
 * for it.  Allocates and frees its own scratch (the per-pixel coefficients
 * when coeffs is NULL, and a few KB of partial sums).  Returns TNO_OK,
 * TNO_E_INVAL (bad arguments, non-finite jitter, singular basis), TNO_E_NOMEM
 * or TNO_E_DEVICE; tno_search_last_error() holds the message of a refusal. */
int tno_refit(const tno_refit_request *req, tno_refit_outputs *out, void *stream);

/* ---------------------------------------------------------------- host-only helpers */

/* Check a request and outputs without touching a GPU (the same checks submit
 * makes).  Returns TNO_OK or TNO_E_INVAL; writes a message of up to len bytes
 * to msg if msg is not NULL. */
int tno_search_validate(const tno_request *req, const tno_outputs *out, char *msg, int32_t len);

/* Device bytes a request needs while in flight (inputs staged on the device,
 * internal buffers, outputs produced internally).  0 if the request is invalid. */
uint64_t tno_search_footprint(const tno_request *req, const tno_outputs *out);

/* Size of the fixed working array of tno_search_run_scratch (per GPU). */
#define TNO_SCRATCH_BYTES (128ull << 20)

/* For callers that cannot allocate device memory (code running under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the search
 * of tno_search_submit + tno_search_poll as one synchronous call on `stream`
 * (hipStream_t, NULL = the default stream) of the current device, with every
 * intermediate buffer (staged stack, ivar maps, offset/weight table, trail
 * kernels, normaliser and SNR/flux maps of a trajectory slab, tile keys,
 * top-k state; slabs here hold at most TNO_SCRATCH_BYTES / 4 bytes, so a
 * large bank runs in more slabs) placed in a fixed TNO_SCRATCH_BYTES array that the library's
 * code object holds on each GPU it runs on, until the process ends.  No
 * handle, no hipMalloc/hipFree and no allocating library call; the small
 * inputs the plan needs (times, velocities, jitter) are read back to host
 * memory, as tno_search_submit does.
 *   req, out: as for tno_search_submit; TNO_REQ_DEVICE_PTRS is required, the
 *             residuals are given (no stack_key), outputs are device memory.
 *   out_result: filled on return (status, n_topk, updates, total_ms; the
 *             per-phase times are 0).
 * Returns TNO_OK; TNO_E_INVAL for an invalid request (as tno_search_validate)
 * or without TNO_REQ_DEVICE_PTRS / with a stack_key; TNO_E_NOMEM when the
 * request's working memory (with those slabs) exceeds TNO_SCRATCH_BYTES;
 * TNO_E_DEVICE on a HIP error.  Calls on one GPU
 * share its array: the library serialises the calls of one process on a GPU
 * (a lock held for the whole call), and every buffer a search needs cleared is
 * cleared by its kernels; calls from several processes each hold their own
 * array.  Outputs are complete when the call returns. */
int tno_search_run_scratch(const tno_request *req, const tno_outputs *out, void *stream,
                           tno_result *out_result);

/* Message of the last refused call on this thread (empty if none). */
const char *tno_search_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TNO_SEARCH_H */
