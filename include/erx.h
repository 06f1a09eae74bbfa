/*
 * erx.h - C ABI of the MI355X (gfx950) ERX anomaly-detector library.
 *
 * ERX (exponentially moving RX) scores every pixel of each incoming scan line
 * X_t in R^{p x b} (p pixels, b bands) by its Mahalanobis distance from a
 * background whose mean and covariance are exponential moving averages over
 * the lines seen so far:
 *
 *   mu_hat_t = (1/p) sum_i x_i,  K_hat_t = 1/(p-1) sum_i (x_i-mu_hat)(x_i-mu_hat)^T
 *                                                    (paper Sec. III-C, Eqs. (18)-(19))
 *   mu_t = (1-a) mu_{t-1} + a mu_hat_t,  K_t = (1-a) K_{t-1} + a K_hat_t
 *       with the first line's statistics as the initial background
 *                                                    (Sec. III-C, Eqs. (20)-(21))
 *   L_t L_t^T = K_t + eps I,  L_t m_i = x_i - mu_t,  delta_i = sqrt(m_i . m_i)
 *                                                    (Sec. III-D, Eqs. (22)-(23))
 *   delta_N,i = (delta_i - mean(delta)) / std(delta) (Sec. III-E, Eq. (24))
 *
 * Each line is scored with the background after its own update.  The sparse
 * random projection of Sec. III-B is not applied (every band is kept).
 *
 * Conventions for every entry point:
 *   - Line buffers are row-major [n][pixels][bands], band index fastest.
 *     They may be host or device pointers (detected with
 *     hipPointerGetAttributes); host buffers may be reused as soon as the call
 *     returns, device buffers must stay valid until the handle's stream has
 *     executed the work (erx_synchronize, or any blocking call).
 *   - The caller owns every buffer it passes; the library owns its handle,
 *     the device-resident detector state and all scratch memory.
 *   - Functions return ERX_OK (0) or a negative ERX_E* code and set a
 *     thread-local message readable with erx_last_error().  Argument errors
 *     (ERX_EINVAL) are detected before any work is enqueued, so the detector
 *     state is unchanged.
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef ERX_H
#define ERX_H

#include <stddef.h>

#ifndef ERX_API
#define ERX_API __attribute__((visibility("default")))
#endif

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ERX_OK = 0,
    ERX_EINVAL = -1,  /* invalid argument; nothing was enqueued */
    ERX_ENOMEM = -2,  /* device or host allocation failed */
    ERX_EDEVICE = -3, /* a HIP runtime call failed */
    ERX_ENOTPD = -4,  /* returned by erx_scores* when at least one line of the last push had
                         a regularised covariance that is not positive definite (possible only
                         with ridge 0); those lines' scores are NaN, the others are valid */
    ERX_ESTATE = -5   /* e.g. scores requested before any push */
};

/* storage type of the input lines */
enum { ERX_F32 = 0, ERX_F16 = 1, ERX_U16 = 2 /* raw counts u, value u * 2^-16 */ };

/* arithmetic of the per-line Gram (covariance) contraction */
enum {
    ERX_GRAM_FP32 = 0, /* FP32 matrix cores, FP32 partials per <=64-pixel chunk, FP64 sums */
    ERX_GRAM_BF16 = 1, /* BF16 inputs on the matrix cores, FP32 accumulate */
    ERX_GRAM_FP16 = 2, /* FP16 inputs on the matrix cores, FP32 accumulate */
    ERX_GRAM_SPLIT16 = 3 /* FP16 matrix cores with each value, scaled by a per-band power of two,
                            split into two FP16 halves (three products, FP32 partials per 64
                            pixels, FP64 sums): FP32-class accuracy.  A 64x64 block of the Gram
                            whose values exceed the split's range (128 times the first 64
                            pixels' spread, or a band constant over them) is recomputed in FP32 */
};

/* arithmetic of the score product L^{-1}(x - mu) (Sec. III-D) */
enum {
    ERX_SCORE_SPLIT16 = 0, /* default: operands scaled by powers of two and split into two FP16
                              halves, three FP16 matrix-core products per tile with FP32
                              accumulation (FP32-class accuracy); lines whose residuals span
                              more than the split can hold are scored again in FP32 */
    ERX_SCORE_FP32 = 1     /* FP32 matrix cores */
};

typedef struct erx_ctx erx_ctx;

typedef struct erx_config {
    int bands;       /* b >= 1 (at most ERX_MAX_BANDS) */
    int pixels;      /* p >= 2 (the line covariance divides by p-1) */
    float momentum;  /* a in (0, 1]; the paper's default is 0.1 */
    float ridge;     /* eps >= 0 added to the covariance diagonal; default 1e-5 */
    int warmup;      /* lines flagged as warm-up buffer (paper: 99); scores are still computed,
                        only the labels of erx_labels are forced to 0 for them */
    int dtype;       /* ERX_F32 / ERX_F16 / ERX_U16 */
    int precision;   /* ERX_GRAM_* */
    double fp64_cond_threshold; /* 0 (default): every line is factored in FP64.  > 0: lines are
                                   factored in FP32 and those whose 1-norm condition estimate of
                                   K_t + eps I exceeds this (or that meet a non-positive pivot) are
                                   re-factored in FP64; +inf: FP32 only, and a line that
                                   meets a non-positive pivot is reported not positive
                                   definite (ERX_ENOTPD, NaN scores) */
    int normalise;   /* 1: also produce line-normalised scores (erx_scores_normalised) */
    int block_lines; /* lines per device pass (scratch is sized for it); default 2048 */
    int scan_lines;  /* lines per segment of the chunked moving-average scan; default 64 */
    int cond_estimate; /* 1-norm condition estimate per line: -1 (default) only when it decides
                          the FP64 re-factor (0 < threshold < inf), 0 never, 1 always */
    int score_arith;   /* ERX_SCORE_SPLIT16 (default) or ERX_SCORE_FP32 */
    int srp_dims;      /* 0 (default): every band is kept.  d in [1, ERX_SRP_MAX_DIMS]: each line is
                          first projected to d dimensions with the sparse random projection of
                          Sec. III-B (the paper's default is 5) and the detector runs on the
                          projected lines: state, statistics and scores are those of Z_t = X_t W */
    unsigned long long srp_seed; /* seed of the projection weights (erx_srp_matrix) */
    int background;    /* ERX_BG_EMA (default): the moving averages of Sec. III-C.  ERX_BG_IMC: the
                          paper's "No EMAs" ablation (Sec. IV-D): every pixel of every line seen so
                          far weighs equally; the background of line t is the mean and the sample
                          covariance (divisor N - 1) of the N = t * pixels pooled pixels (the batch
                          Welford update), plus the ridge; momentum is then unused */
    int state_fp32;    /* 0 (default): the moving-average state, the per-line statistics and the
                          scan carries are stored in FP64.  1: they are stored in FP32 (half the
                          device memory and traffic of the statistics; the averaging recurrence of
                          Eqs. (20)-(21) is still evaluated in FP64 and each stored value is rounded
                          once).  erx_get_state / erx_set_state convert; not with ERX_BG_IMC */
    int score_tiles;   /* tile shape of the split-FP16 score kernel: 16-pixel tiles per wave, 1 or 2;
                          0 (default): 1 above 192 bands (where two would spill registers), else 2.
                          Results do not depend on it; erx_autotune chooses it */
    int gram_macro;    /* bands per macro tile (one workgroup's block of the Gram) of the split-FP16
                          Gram: 64 or 128; 0 (default): 128 from 65 bands on, else 64.  128-band
                          macro tiles split each element into its FP16 halves half as often at
                          224 bands.  Results do not depend on it: both write the same values,
                          except that a 128-band block the split cannot hold (a band constant
                          over the first 64 pixels, or a value beyond the scale's headroom) is
                          recomputed in FP32 as the four 64-band blocks it covers */
} erx_config;

enum { ERX_BG_EMA = 0, ERX_BG_IMC = 1 };

#define ERX_SRP_MAX_DIMS 32

#define ERX_MAX_BANDS 304

/* Fill *cfg with defaults: ridge 1e-5, warmup 0, F32 input, split-FP16 Gram,
 * threshold 0 (FP64 factorisation), no normalisation, block_lines 2048,
 * scan_lines 64, cond_estimate -1, split-FP16 score. */
ERX_API void erx_config_default(erx_config *cfg, int bands, int pixels, float momentum);

/* The sparse random projection W in R^{bands x dims} of Sec. III-B, as a detector with
 * srp_dims = dims and srp_seed = seed uses it: w_ij = sqrt(s/dims) * (+1 with probability
 * 1/(2s), 0 with 1 - 1/s, -1 with 1/(2s)), s = sqrt(bands), so about dims * sqrt(bands)
 * weights are non-zero.  The draws are SplitMix64 outputs (the published generator, as a
 * counter): weight (i, j) takes output k = i * dims + j + 1 from state seed, as the
 * uniform (u >> 11) * 2^-53.  W: host buffer [bands][dims], row-major.  Host only (no
 * device work); ERX_EINVAL for bands outside [1, ERX_MAX_BANDS] or dims outside
 * [1, ERX_SRP_MAX_DIMS]. */
ERX_API int erx_srp_matrix(int bands, int dims, unsigned long long seed, float *W);

/* Create a detector on the current HIP device.  Returns NULL on error
 * (erx_last_error says why).  erx_create uses the defaults above. */
ERX_API erx_ctx *erx_create(int bands, int pixels, float momentum);
ERX_API erx_ctx *erx_create_ex(const erx_config *cfg);

/* Run the handle's later work on a caller-provided hipStream_t (NULL is the
 * device's default stream).  Until this is called the handle uses a stream of
 * its own.  The stream must outlive its use by the handle. */
ERX_API int erx_set_stream(erx_ctx *h, void *hip_stream);

/* Absorb and score n >= 1 lines (Sec. III, one line at a time, in order).
 * erx_push_lines takes FP32 lines; erx_push_lines_ex takes the configured
 * dtype.  Stream-ordered: returns once the work is enqueued (host input is
 * staged before return). */
ERX_API int erx_push_lines(erx_ctx *h, const float *lines, int n);
ERX_API int erx_push_lines_ex(erx_ctx *h, const void *lines, int n);

/* Scores of the last push, [n][pixels] FP32 distances delta.  erx_scores
 * copies to host memory and blocks; erx_scores_device copies into a device
 * buffer on the handle's stream without blocking. */
ERX_API int erx_scores(erx_ctx *h, float *out);
ERX_API int erx_scores_device(erx_ctx *h, float *dev_out);

/* Line-normalised scores of the last push (needs cfg.normalise = 1). */
ERX_API int erx_scores_normalised(erx_ctx *h, float *out);

/* Labels y = [delta_N >= tau] of the last push as bytes [n][pixels] (Sec. III-E,
 * Eq. (25)); warm-up lines give 0.  Needs cfg.normalise = 1.  Host output. */
ERX_API int erx_labels(erx_ctx *h, float tau, unsigned char *out);

/* Detector state: number of lines absorbed, background mean [b] and full
 * symmetric covariance [b*b] (FP64, host buffers), with b = srp_dims for a detector
 * that projects its lines (Sec. III-B).  erx_set_state with t = 0
 * resets the detector; the next line initialises the background. */
ERX_API int erx_get_state(erx_ctx *h, long long *t, double *mu, double *K);
ERX_API int erx_set_state(erx_ctx *h, long long t, const double *mu, const double *K);

typedef struct erx_stats_t {
    long long lines;          /* lines absorbed */
    long long fp64_refactors; /* lines re-factored in FP64 */
    long long notpd;          /* lines whose covariance was not positive definite */
    double max_cond;          /* largest 1-norm condition estimate seen */
} erx_stats_t;
ERX_API int erx_stats(erx_ctx *h, erx_stats_t *out);

/* Per-line diagnostics of the last push (host buffers of n entries, either may
 * be NULL): condition estimate and status bits (1 = FP64 re-factor requested,
 * 2 = re-factored in FP64, 4 = not positive definite). */
ERX_API int erx_line_info(erx_ctx *h, float *cond, int *flags);

/* Kernel timing: when enabled, every kernel launch of the handle is bracketed
 * by HIP events on the handle's stream.  erx_profile_read waits for the
 * stream, writes up to max entries (kernel name, launches, total
 * milliseconds) in a fixed kernel order, returns the number of entries and
 * clears the record. */
typedef struct erx_kernel_time {
    char name[32];
    long long launches;
    double total_ms;
} erx_kernel_time;
ERX_API int erx_profile_enable(erx_ctx *h, int on);
ERX_API int erx_profile_read(erx_ctx *h, erx_kernel_time *out, int max);

/* ------------------------------------------------------------------------
 * Many independent streams.  Each stream is its own detector (Sec. III applied
 * to that stream alone) with its own band count, pixel count and momentum;
 * ridge, input dtype, precision options, scan segment and pass capacity come
 * from `common` (its bands / pixels / momentum fields are ignored).  A push
 * gives every stream zero or more new lines; the library processes them in
 * device passes that mix lines of all streams with the same number of
 * 16-band tiles (longest work first), and can replay passes of identical
 * shape from captured HIP graphs.  Line buffers of a batch must be device
 * memory.
 * ------------------------------------------------------------------------ */
typedef struct erx_batch erx_batch;
ERX_API erx_batch *erx_batch_create(int nstreams, const int *bands, const int *pixels, const float *momentum,
                                    const erx_config *common);
/* Order the batch's work after / before the caller's hipStream_t (NULL is the default stream);
 * the batch itself runs on a stream of its own so that its passes can be captured. */
ERX_API int erx_batch_set_stream(erx_batch *bt, void *hip_stream);
/* lines[s]: device buffer [nlines[s]][pixels[s]][bands[s]] (ignored when nlines[s] == 0) */
ERX_API int erx_batch_push(erx_batch *bt, const void *const *lines, const int *nlines);
/* out[s]: buffer of nlines[s] * pixels[s] floats (host or device) receiving the scores of
 * stream s's lines of the last push, or NULL to skip stream s; blocks.  ERX_ENOTPD as for
 * erx_scores. */
ERX_API int erx_batch_scores(erx_batch *bt, float *const *out);
ERX_API int erx_batch_get_state(erx_batch *bt, int stream, long long *t, double *mu, double *K);
ERX_API int erx_batch_stats(erx_batch *bt, erx_stats_t *out);
/* 1 (default): capture passes in HIP graphs and replay them; 0: launch every kernel */
ERX_API int erx_batch_use_graphs(erx_batch *bt, int on);
/* Streams with at most 16 bands can run on a fused path: one workgroup per stream walks the
 * stream's lines in order with the moving-average state on chip (no per-line statistics in
 * device memory, no scan), the Gram from FP64 differences and products and every line
 * factored in FP64, whatever the configured precision.  The line is held in LDS (one read
 * from device memory, the next line's loads in flight meanwhile) when every line of the
 * push is at most 40960 bytes and starts on a 16-byte boundary; otherwise each tile is
 * streamed from device memory twice.  mode 1: use it for every such stream; 2: the same
 * but always streamed; 0: never; -1 (default): when at least 32 such streams are in the
 * batch.  Results agree with the general path to rounding.  A batch made with state_fp32 = 1
 * never takes it (the fused path keeps an FP64 state).  ERX_EINVAL for another mode. */
ERX_API int erx_batch_small_path(erx_batch *bt, int mode);
ERX_API int erx_batch_synchronize(erx_batch *bt);
ERX_API void erx_batch_destroy(erx_batch *bt);

/* ---------------------------------------------------------------------------------------
 * Autotuning of launch settings (a project addition; the paper has none).  For one
 * workload shape - a configuration plus the number of identical streams sharing it - the
 * tuner runs every candidate setting on synthetic lines of that shape (values in
 * [0.25, 0.75), independent bands) through the entry points above, times each with HIP
 * events on a stream of its own, and returns the fastest.  Candidates: for one stream,
 * lines per device pass (block_lines 512..8192) x scan segment (scan_lines 32, 64, 128);
 * for a batch, pass capacity (1024, 4096, 16384) and, when bands <= 16, the small-band
 * path mode (erx_batch_small_path 0, 1, 2); with the split-FP16 score, each also x the
 * score kernel's tile shape (score_tiles 1, 2); with the split-FP16 Gram above 64 bands,
 * each also x the Gram's macro tile (gram_macro 64, 128).  No candidate changes what is computed:
 * pass and segment lengths only regroup the FP64 moving-average updates (scores agree with
 * an untuned handle's to 1e-6 relative), the tile shapes change no product, and the
 * small-band modes agree with the general path as erx_batch_small_path states.  The timings are those of well-conditioned
 * backgrounds (no FP64 re-factor triggered).
 * ------------------------------------------------------------------------------------- */
typedef struct erx_tune_result {
    int block_lines;    /* erx_config.block_lines to use */
    int scan_lines;     /* erx_config.scan_lines to use */
    int small_path;     /* erx_batch_small_path mode to use; -1 for a single stream */
    int candidates;     /* settings timed by this call; 0 when the result came from the cache */
    double us_per_line; /* measured microseconds per line (per stream line for a batch) */
    int score_tiles;    /* erx_config.score_tiles to use */
    int gram_macro;     /* erx_config.gram_macro to use */
} erx_tune_result;
/* cfg: the workload (its block_lines and scan_lines are ignored); nstreams >= 1 (1: a
 * detector made with erx_create_ex, more: a batch of that many streams of cfg's shape);
 * cache_path: a JSON file {"erx_tune": 1, "entries": [...]} that is read first (an entry
 * for the same bands, pixels, dtype, precision, fp64_cond_threshold, normalise, score_arith,
 * state_fp32 and nstreams is returned without timing) and updated with a new result, or NULL.  Uses the
 * current HIP device and allocates the synthetic input (at most 4 GiB) for the duration
 * of the call.  ERX_EINVAL for invalid arguments or an unreadable cache file (nothing is
 * timed), ERX_ENOMEM / ERX_EDEVICE on device failures. */
ERX_API int erx_autotune(const erx_config *cfg, int nstreams, const char *cache_path, erx_tune_result *out);
/* Cache lookup only (no device work): ERX_OK with *out filled when cache_path holds an
 * entry for (cfg, nstreams), ERX_ESTATE when it holds none (or the file does not exist),
 * ERX_EINVAL for invalid arguments or a file that is not a tuning cache. */
ERX_API int erx_tune_lookup(const erx_config *cfg, int nstreams, const char *cache_path, erx_tune_result *out);

/* ---------------------------------------------------------------------------------------
 * Learned band-projection surrogate (a stated change to the method, the learned analogue of
 * the sparse random projection of Sec. III-B).  For b-band FP32 lines:
 *     z = W x + c (ERX_SURR_K outputs),  u = L_z^{-1} (z - mu_z) with (mu_z, L_z) the ERX
 *     statistics of the z stream (same momentum, first-line initialisation, ridge 1e-5),
 *     o = w2 . relu(A1 u + a1) + c2 (ERX_SURR_HIDDEN hidden units),  score = ||u|| exp(o).
 * Parameters are one flat FP32 vector (the master copy; every forward pass uses FP16 copies
 * of the weights W, A1 and w2, refreshed at every change, and the FP32 biases), laid out as
 * W [K][b] row-major, c [K], A1 [HIDDEN][K] row-major, a1 [HIDDEN], w2 [HIDDEN], c2:
 * erx_surrogate_num_params() floats.  Scoring lines of at most 1024 pixels is one fused
 * kernel per call (a workgroup per line; the moving average passes between lines through a
 * decoupled look-back); longer lines take a staged path with the same results.
 * A handle owns its device memory and its own stream; calls block until done.
 * --------------------------------------------------------------------------------------- */
#define ERX_SURR_K 16
#define ERX_SURR_HIDDEN 64
typedef struct erx_surr erx_surr;
/* NULL on error (bands outside [1, ERX_MAX_BANDS], no memory).  seed: initial parameters. */
ERX_API erx_surr *erx_surrogate_create(int bands, unsigned long long seed);
ERX_API int erx_surrogate_num_params(const erx_surr *net);
/* host arrays of erx_surrogate_num_params() floats; set also resets the Adam moments */
ERX_API int erx_surrogate_set_params(erx_surr *net, const float *params);
ERX_API int erx_surrogate_get_params(const erx_surr *net, float *params);
/* Surrogate scores of n lines [n][pixels][bands] (device FP32) of a stream scored from its
 * first line into out [n][pixels] (device FP32).  ERX_EDEVICE if a look-back wait of the
 * fused kernel did not complete (its lines are then NaN). */
ERX_API int erx_surrogate_scores(erx_surr *net, const float *lines, int n, int pixels, float momentum,
                                 float *out);
/* One training step on n consecutive lines (device FP32 [n][pixels][bands]) of a stream
 * scored from its first line, against targets [n][pixels] (device FP32, the plain-ERX
 * scores of the same lines): loss = mean w (log score - log target)^2, w = clamp(target^2 /
 * bands, 1, 100) (a background pixel's squared distance averages the band count, so pixels
 * plain ERX scores far above the background weigh more), with the z-stream statistics held
 * fixed; the gradient is kept (erx_surrogate_grads) and, for lr > 0, one
 * Adam step (beta 0.9 / 0.999, eps 1e-8) is taken.  *loss receives the loss before the step.
 * The loss and the gradient are summed in a fixed order: a step is reproducible. */
ERX_API int erx_surrogate_train_step(erx_surr *net, const float *lines, const float *targets, int n,
                                     int pixels, float momentum, float lr, float *loss);
/* gradient of the last training step, host array of erx_surrogate_num_params() floats */
ERX_API int erx_surrogate_grads(const erx_surr *net, float *grads);
ERX_API void erx_surrogate_destroy(erx_surr *net);

/* A stream scored by the surrogate and checked against plain ERX: line t with (t+1) %
 * check_every == 0 is also scored by plain ERX and by the surrogate, each on a state that
 * sees only those lines (momentum 1 - (1 - momentum)^check_every); the drift of a check is
 * the median over the line's pixels of |log surrogate - log plain| of those two scores.
 * After two consecutive checks with drift above drift_threshold the stream switches to
 * plain ERX (re-initialised from the next line) for good.  The plain-ERX detector used after
 * a switch is allocated at creation (256 lines per pass), so a switch allocates nothing.
 * The detector keeps a pointer to net, which must outlive it. */
typedef struct erx_sdet erx_sdet;
ERX_API erx_sdet *erx_surrogate_detector_create(erx_surr *net, int pixels, float momentum,
                                                float drift_threshold, int check_every);
/* lines: device FP32 [n][pixels][bands]; blocks at every check line */
ERX_API int erx_surrogate_detector_push(erx_sdet *sd, const float *lines, int n);
/* out: n_last * pixels floats, host or device */
ERX_API int erx_surrogate_detector_scores(erx_sdet *sd, float *out);
/* active: 1 while the surrogate scores; checks / drifts: counts; switched_at: first line
 * scored by plain ERX after the switch, or -1 */
ERX_API int erx_surrogate_detector_status(const erx_sdet *sd, int *active, long long *checks,
                                          long long *drifts, long long *switched_at);
/* Drift of the last check and the mean and largest drift over all checks so far (a NaN
 * drift is the largest); ERX_ESTATE before the first check.  Used to set drift_threshold
 * from the checks of in-distribution streams. */
ERX_API int erx_surrogate_detector_drift_stats(const erx_sdet *sd, float *last, float *mean, float *max);
ERX_API void erx_surrogate_detector_destroy(erx_sdet *sd);

/* ---------------------------------------------------------------------------------------
 * Allocation-free push, for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It computes what
 * erx_create_ex + erx_push_lines_ex + erx_scores_device compute for one stream (same
 * kernels, same results), with no handle: the caller owns the lines, the scores and the
 * stream's moving-average state, and the library's intermediate buffers (per-line
 * statistics, scan carries, inverse factors) live in one static device array of
 * ERX_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends.  No hipMalloc, hipFree or
 * allocating library routine is called; the first call on a device looks up the array's
 * address once (hipGetSymbolAddress), so make one call on each device before capturing.
 *
 *   cfg      as for erx_create_ex; normalise, srp_dims and state_fp32 must be 0 and the
 *            background ERX_BG_EMA.  block_lines caps the lines per
 *            device pass; the scratch caps it further (152 lines at 224 bands, 84 at
 *            304 with scan_lines 64), and longer pushes run in several passes.
 *   state    device buffer of E = 256*NT*(NT+1)/2 + 16*NT doubles, NT = ceil(bands/16): the
 *            background after the stream's last line, in the library's packed layout
 *            (opaque).  Read and rewritten by the call; with t0 = 0 its contents are ignored.
 *   t0       lines the stream absorbed before this call (0: the first line initialises the
 *            background); the caller adds n after each call.
 *   lines    device buffer [n][pixels][bands] in cfg->dtype, aligned to its element size.
 *   out      device buffer [n][pixels] FP32 receiving the distances delta.
 *   hip_stream  stream the work is enqueued on (NULL: the default stream).  Returns once
 *            enqueued and never waits for the device.
 *
 * Errors: ERX_EINVAL for invalid arguments (bands beyond ERX_MAX_BANDS, the largest size the
 * scratch is laid out for; pixels < 2; n < 1; normalise = 1; state_fp32 = 1; a buffer that is not device
 * memory ...), with nothing enqueued; ERX_EDEVICE when the scratch address cannot be found
 * or a launch fails.  Lines whose covariance is not positive definite get NaN scores and
 * are not reported (that would need a wait).  Every call on a GPU shares that GPU's scratch
 * and it keeps the last call's contents: calls that overlap on one GPU (different streams,
 * several threads) race and must be serialised, e.g. on one stream. */
#define ERX_NOALLOC_SCRATCH_BYTES (48u << 20)
ERX_API int erx_push_lines_noalloc(const erx_config *cfg, double *state, long long t0, const void *lines, int n,
                                   float *out, void *hip_stream);

/* ---------------------------------------------------------------------------------------
 * Detection metrics of Sec. IV-C for scored pixels with ground truth.  TPR(tau) and
 * FPR(tau) are the fractions of anomalies and of background pixels scoring >= tau
 * (Eqs. (26)-(27)); the ROC curve visits every distinct score as a threshold and auc is
 * its area (the fraction of (anomaly, background) pairs ranked correctly, ties counting
 * one half).  auc_tpr_tau and auc_fpr_tau are the areas under TPR(tau) and FPR(tau) for
 * tau in [0, 1] with the scores min-max normalised over the evaluated pixels (0 when all
 * are equal); auc_td = (auc + auc_tpr_tau) / 2 and auc_bs = (auc - auc_fpr_tau + 1) / 2
 * (Eqs. (28)-(29)).  Pixels whose score is not finite are left out and counted.
 * --------------------------------------------------------------------------------------- */
typedef struct erx_detection_metrics_t {
    double auc, auc_tpr_tau, auc_fpr_tau, auc_td, auc_bs;
    long long positives;  /* anomalies evaluated */
    long long negatives;  /* background pixels evaluated */
    long long excluded;   /* pixels with a non-finite score */
} erx_detection_metrics_t;
/* scores: device FP32 [n]; truth: device bytes [n], non-zero = anomaly; n >= 2.  Runs on
 * hip_stream (NULL: the default stream), allocates a sort buffer of the smaller class for
 * the call and blocks until the result is in *out.  ERX_EINVAL for host buffers, or when
 * no anomaly or no background pixel has a finite score; ERX_EDEVICE on device failures. */
ERX_API int erx_detection_metrics(const float *scores, const unsigned char *truth, long long n, void *hip_stream,
                                  erx_detection_metrics_t *out);

/* ---------------------------------------------------------------------------------------
 * RX Baseline, the reference detector the paper compares ERX with (Sec. IV-B): a rolling
 * buffer holds the last `window` lines (the paper: 99); the mean and the covariance
 * (divisor n, the RX definition of Sec. II-A) of all pixels in the buffer, plus cfg->ridge
 * on the diagonal (0 gives the RX definition; the ERX default 1e-5 is kept if not changed),
 * score the buffer's centre line.  The window ending at stream line t (0-based) scores
 * line t - (window - 1) / 2; the first window is complete once `window` lines arrived, so
 * the first (window - 1) / 2 lines are never scored, and the last (window - 1) / 2 lines
 * are scored only by later pushes.  cfg: bands, pixels, ridge, dtype, precision,
 * fp64_cond_threshold, cond_estimate, score_arith, block_lines and scan_lines as for
 * erx_create_ex (momentum is unused; srp_dims, normalise and state_fp32 must be 0: the window
 * statistics are differences of running sums, kept in FP64).  window: odd, >= 1.
 * --------------------------------------------------------------------------------------- */
typedef struct erx_rxb erx_rxb;
ERX_API erx_rxb *erx_rxb_create(const erx_config *cfg, int window);
/* lines: device buffer [n][pixels][bands] in cfg->dtype; stream-ordered */
ERX_API int erx_rxb_push(erx_rxb *r, const void *lines, int n);
/* Scores of the centre lines whose windows the last push completed: *nlines lines
 * [nlines][pixels] from stream line *first_line on (-1 and 0 when none) into out (host or
 * device, may be NULL to query the count); blocks. */
ERX_API int erx_rxb_scores(erx_rxb *r, float *out, long long *first_line, int *nlines);
ERX_API void erx_rxb_destroy(erx_rxb *r);

/* Wait for all work enqueued on the handle's stream. */
ERX_API int erx_synchronize(erx_ctx *h);

ERX_API void erx_destroy(erx_ctx *h);

/* Thread-local description of the last error (never NULL). */
ERX_API const char *erx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ERX_H */
