/*
 * chamfer.h -- C ABI of libchamfer, a gfx950 (MI355X) implementation of the
 * near-linear (1 +- eps) Chamfer-distance estimator of Bakshi, Indyk,
 * Jayaram, Silwal and Waingarten, "A Near-Linear Time Algorithm for the
 * Chamfer Distance" (NeurIPS 2023), and of the exact brute-force Chamfer
 * distance it speeds up.
 *
 *   CH(A, B) = sum_{a in A} min_{b in B} d(a, b),  d = l1 or l2, NOT squared
 *   (definition of CH in the introduction and the footnote to it).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Point sets are DEVICE pointers to row-major, contiguous float32 arrays
 *   [n, d] (row p at X + p*d).  Every other array argument is a device
 *   pointer too, unless marked "host".  The caller owns all memory,
 *   including the workspace `ws` (size from chamfer_workspace_bytes); the
 *   library never allocates or frees device memory.  It keeps no state
 *   between calls, with two exceptions: a server (chamfer_server_create)
 *   owns its arena and lanes until chamfer_server_destroy, and
 *   chamfer_retrieve creates three side streams per device on its first
 *   call there and keeps them until the process ends.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *   work is enqueued on it asynchronously; the caller synchronises.  Output
 *   buffers are valid once the stream has reached the end of the call.
 * - Return value: CHAMFER_OK, or a negative chamfer_status for an argument
 *   error (checked on the host before anything is launched) or a failed HIP
 *   launch.  Data-dependent errors (a NaN or Inf coordinate) cannot be seen
 *   on the host without a synchronisation; they are reported through the
 *   optional device status word and make the floating outputs NaN.
 * - Calls on one stream with one workspace must not overlap; calls with
 *   distinct workspaces may run concurrently on distinct streams.
 * - Graph capture: chamfer_exact, chamfer_nn_min, crude_nn and
 *   chamfer_estimate with l1 (or with uniform sampling) enqueue kernels
 *   only, with no host synchronisation, and may be captured into a HIP
 *   graph.  An l2 call that hashes (crude_nn, chamfer_hash_keys,
 *   chamfer_estimate with importance sampling) uploads the embedding
 *   matrix, drawn on the host for this seed, from a host buffer that the
 *   next call overwrites: a replay would read whatever that buffer then
 *   holds.  Such calls return CHAMFER_EINVAL when `stream` is capturing.
 * - Results are deterministic: the same arguments give bit-identical outputs
 *   on every run, whatever the launch configuration (no floating-point
 *   atomics; integer atomics only for min/max, whose result is order-free).
 */
#ifndef CHAMFER_H
#define CHAMFER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum chamfer_metric { CHAMFER_L1 = 1, CHAMFER_L2 = 2 };

enum chamfer_status {
    CHAMFER_OK = 0,
    CHAMFER_EINVAL = -1,      /* bad argument (host check, nothing launched)   */
    CHAMFER_EWORKSPACE = -2,  /* ws NULL or ws_bytes < chamfer_workspace_bytes */
    CHAMFER_EHIP = -3,        /* a HIP launch or runtime call failed           */
    CHAMFER_ENONFINITE = -4,  /* device status: an input coordinate is NaN/Inf */
    CHAMFER_ETOOLARGE = -5    /* chamfer_estimate_noalloc: the call needs more
                                 workspace than CHAMFER_STATIC_SCRATCH_BYTES */
};

enum chamfer_precision {
    CHAMFER_FP32 = 0,  /* exact canonical float32 arg-mins (l2: certified    *
                        * candidates from bf16-split MFMA tiles)             */
    CHAMFER_BF16 = 1,  /* l2 distance tiles on bf16 MFMA + float32 re-rank    */
    CHAMFER_FP8 = 2    /* l2 distance tiles on fp8-e4m3 MFMA + float32 re-rank*/
};

/* How chamfer_estimate draws its T points of A (the uniform-vs-importance
 * paragraph of the algorithm overview). */
enum chamfer_sampling {
    CHAMFER_IMPORTANCE = 0,  /* proportional to the CrudeNN distances D_a      */
    CHAMFER_UNIFORM = 1      /* uniform over A (the baseline): the same steps
                                with every D_a = 1, so eta = (n_A/T) sum of
                                the sampled nearest-neighbour distances; no
                                CrudeNN and no tables                          */
};

/* Tunables; pass NULL for all defaults.  Zero fields take their default. */
typedef struct chamfer_opts {
    int32_t n_scales;   /* L grid scales; 0 => ceil(log2(max(n_A,n_B)/eps))   */
    int32_t embed_dim;  /* l2 only: embedding dimension k_e; 0 => 32          */
    int32_t precision;  /* enum chamfer_precision; 0 => CHAMFER_FP32          */
    int32_t window;     /* W points retrieved per point of A by CrudeNN, 1..32;
                           0 => 1 (the first colliding point)                  */
    int32_t reps;       /* k independent LSH structures, 1..64; 0 => 1       */
    int32_t sampling;   /* enum chamfer_sampling; 0 => importance             */
    int32_t reduction;  /* enum chamfer_reduction_mode, chamfer_estimate only;
                           0 => none                                          */
} chamfer_opts;

/* Reduction to bounded aspect ratio before the estimate (the lemma on
 * reducing to poly(n/eps) aspect ratio and its proof in the appendix). */
enum chamfer_reduction_mode {
    CHAMFER_REDUCE_NONE = 0,
    CHAMFER_REDUCE_PARTITION = 1, /* crude bounds, coarse partition, sum of parts */
    CHAMFER_REDUCE_PAD = 2        /* the same, on copies with appended coordinates */
};

/* Optional device outputs of chamfer_estimate; any field may be NULL. */
typedef struct chamfer_aux {
    int32_t *sample_idx;   /* [T] sampled rows x_l of A                         */
    float *sample_min;     /* [T] min_b d(x_l, b), float32                      */
    int32_t *sample_nn;    /* [T] the b attaining it (lowest index on ties)     */
    double *D;             /* [1] normaliser D = sum_a D_a (= W * 2^-s)         */
    uint64_t *W;           /* [1] fixed-point total of the weights              */
    int32_t *s;            /* [1] fixed-point exponent (w_a = ceil(D_a 2^s))    */
    int32_t *status;       /* [1] CHAMFER_OK or CHAMFER_ENONFINITE              */
    float *crude_D;        /* [n_A] D_a from CrudeNN (1 with uniform sampling)  */
    int32_t *crude_nn;     /* [n_A] the b with D_a = d(a, b) (-1 if uniform)    */
    int32_t *crude_scale;  /* [n_A] first colliding scale, L if none (-1 if
                              uniform)                                          */
    /* Host array of CHAMFER_STAGE_EVENTS hipEvent_t (as void*), or NULL.  When
     * set, event i is recorded on the stream at stage boundary i: 0 start,
     * 1 calibration and tables done, 2 B bucketed, 3 CrudeNN done (D_a),
     * 4 weights and draws done, 5 exact pass over the draws done, 6 end.
     * Stage 4->5 is the nearest-neighbour pass over the draws: for l2 with
     * 12 <= d <= 256 the BF16 split table of the draws, the matrix-core
     * record kernel, the per-draw resolve kernel and, when B's chunks are
     * longer than 512 rows, the rescan kernel (B's split table is written
     * in stage 1->2 by the kernel that hashes B, or in stage 4->5 for the
     * uniform-sampling baseline); otherwise one vector-ALU kernel. */
    void **stage_events;
} chamfer_aux;

#define CHAMFER_STAGE_EVENTS 7

/*
 * Workspace bytes sufficient for any entry point below called with these
 * sizes and options (T = 0 means the default sample count; for
 * chamfer_nn_min, n_A is n_x).  With eps outside (0, 1) the size covers only
 * chamfer_exact and chamfer_nn_min.  Returns 0 for invalid sizes/options.
 */
size_t chamfer_workspace_bytes(int64_t n_A, int64_t n_B, int32_t d, int32_t metric,
                               double eps, int64_t T, const chamfer_opts *opts);

/*
 * Reduction to bounded aspect ratio (lemma on the reduction to poly(n/eps)
 * aspect ratio; its proof in the appendix), the steps of
 * chamfer_aspect_reduce:
 *  1. a p-stable direction g (l1: Cauchy, l2: Gaussian entries; Philox
 *     purpose 4, counter (j, 0)), drawn on the host in double precision;
 *  2. projections p_x = <x, g> in double (fused multiply-adds, coordinates
 *     ascending);
 *  3. t_a = min_b |p_a - p_b| (1-D nearest neighbour: B's projections
 *     sorted, a binary search per a), M = max_a t_a and ch1 = sum_a t_a, the
 *     1-D Chamfer distance (a poly(n)-approximation of CH);
 *  4. with n = max(n_A, n_B), lA = ceil(log2 n_A), lB, ln likewise,
 *     k_hi = lA + ln, k_lo = lA + lB + ln and e_M = floor(log2 M):
 *     eta_lo = 2^(e_M - k_hi) <= CH(A, B) <= eta_hi = 2^(e_M + 1 + lA + k_lo)
 *     with probability >= 1 - 2/n; the partition side 2^e_part with
 *     e_part = log2(eta_hi / eta_lo) + ln + log2(eta_hi) (>= c n eta_hi);
 *     m padding coordinates of value +-q, q = eps eta_lo / (2 n m), where m
 *     is at least 3 ln, rounded up so that d + m is the next of 16, 32, 64,
 *     128 (a multiple of 16 above 128);
 *     M = 0 (every a on a b in projection) is "degenerate": no partition,
 *     q = 0;
 *  5. partition keys: the grid hash of side 2^e_part on the hashed
 *     coordinates (x - lo for l1, the l2 -> l1 embedding for l2; shifts and
 *     multipliers from Philox purpose 5, counter (k, 0)), cells computed in
 *     double: ceil(ldexp(y, -e_part) + z'), clamped to +-2^62 (0 for NaN),
 *     key = (sum_k cell_k M_k mod 2^64) >> 1; one_part = every key of A and
 *     B equal;
 *  6. padded copies (if asked): row i followed by m values +-q, the sign of
 *     value j being bit j mod 64 of word j / 64 of the Philox block
 *     (i, side, 6) (side 0 for A, 1 for B; a set bit gives -q).
 *   info_out  [1] chamfer_reduction (device).
 *   t_out     [n_A] double (device) or NULL.
 *   keys_A_out [n_A], keys_B_out [n_B] uint64 (device) or NULL.
 *   A_pad_out [n_A, d + m], B_pad_out [n_B, d + m] float (device) or NULL;
 *   m = chamfer_pad_dims(n_A, n_B, d).
 * Asynchronous on `stream`.  Workspace: chamfer_reduce_workspace_bytes.
 * Errors: EINVAL if n_A < 1, n_B < 1, d < 1, metric not 1/2, eps not in
 * (0, 1) or a bad embedding dimension; EWORKSPACE; EHIP.
 */
typedef struct chamfer_reduction {
    double ch1;          /* sum_a t_a */
    double max_t;        /* M = max_a t_a */
    double eta_lo;       /* lower bound of CH(A, B) (a power of two) */
    double eta_hi;       /* upper bound of CH(A, B) (a power of two) */
    int32_t e_M;         /* floor(log2 M) */
    int32_t e_part;      /* partition cells have side 2^e_part */
    int32_t pad_dims;    /* m */
    float pad_value;     /* q */
    int32_t degenerate;  /* M == 0 (or not finite): no partition, q = 0 */
    int32_t one_part;    /* every partition key of A and B is the same */
} chamfer_reduction;

int32_t chamfer_pad_dims(int64_t n_A, int64_t n_B, int32_t d);
size_t chamfer_reduce_workspace_bytes(int64_t n_A, int64_t n_B, int32_t d, int32_t metric,
                                      const chamfer_opts *opts);
int chamfer_aspect_reduce(const float *A, const float *B, int64_t n_A, int64_t n_B, int32_t d,
                          int32_t metric, double eps, uint64_t seed, const chamfer_opts *opts,
                          chamfer_reduction *info_out, double *t_out, uint64_t *keys_A_out,
                          uint64_t *keys_B_out, float *A_pad_out, float *B_pad_out, void *ws,
                          size_t ws_bytes, void *stream);

/*
 * Exact Chamfer distance by brute force (definition of CH in the
 * introduction; the O(d n^2) baseline the paper compares against).
 *   ch_out     [1] double: sum_a m_a, summed in double precision.
 *   rowmin_out [n_A] float or NULL: m_a = min_b d(a, b) in float32.
 *   rownn_out  [n_A] int32 or NULL: the b attaining m_a.
 * With precision FP32 (the default), m_a and its arg-min are the canonical
 * float32 values: accumulator over k ascending (l1: acc + |a_k - b_k|, l2:
 * fma(t, t, acc) with t = a_k - b_k, then a correctly rounded square root),
 * minimised over b with ties to the lower index.  BF16/FP8 (l2 only) rank
 * candidates with low-precision tiles and re-rank the best ones in float32;
 * their results carry a stated error instead.
 * Errors: EINVAL if d < 1, metric not 1/2, n_A < 0, n_B < 1, or rows exceed
 * the int32 index range; EWORKSPACE; EHIP.
 */
int chamfer_exact(const float *A, const float *B, int64_t n_A, int64_t n_B, int32_t d,
                  int32_t metric, double *ch_out, float *rowmin_out, int32_t *rownn_out,
                  const chamfer_opts *opts, void *ws, size_t ws_bytes, void *stream);

/*
 * CrudeNN (the CrudeNN figure): for every a in A an upper bound
 * D_a >= min_b d(a, b).  L randomly shifted grids with sides
 * r_i = 2^(e_top - (L-1-i)), i = 0 finest, where 2^e_top is the smallest
 * power of two >= sum_k (max_k - min_k) over A u B.  l2 points are first
 * mapped to l1 by a Gaussian embedding with k_e rows (appendix theorem on
 * embedding l2 into l1).  D_a = d(a, b) for the lowest-index b sharing a's
 * bucket at the first scale where any b does; if none does, b = 0.
 *   D_out [n_A] float (canonical float32 distance), nn_out [n_A] int32,
 *   scale_out [n_A] int32 or NULL (the scale, L when no scale collided).
 * Randomness: Philox4x64-10 with key (seed, 0) and counter
 * (c0, c1, purpose, 0); shifts and multipliers use purpose 1 with
 * (c0, c1) = (coordinate, scale), the embedding purpose 2 with
 * (row * d + column, 0).  The same seed gives the same output.
 * Errors: as chamfer_exact, plus EINVAL unless 0 < eps < 1, or if opts
 * request more than 64 scales or a bad embedding dimension.
 */
int crude_nn(const float *A, const float *B, int64_t n_A, int64_t n_B, int32_t d,
             int32_t metric, double eps, uint64_t seed, float *D_out, int32_t *nn_out,
             int32_t *scale_out, const chamfer_opts *opts, void *ws, size_t ws_bytes,
             void *stream);

/*
 * Chamfer-Estimate (the Chamfer-Estimate figure): CrudeNN, then T i.i.d.
 * draws x_l ~ D_a / D, then eta = (1/T) sum_l (D / D_{x_l}) min_b d(x_l, b).
 * The distribution is held in 64-bit fixed point: s = 47 - ceil(log2 n_A) -
 * e_max (max_a D_a in [2^(e_max-1), 2^e_max)), w_a = ceil(D_a 2^s), W = sum
 * w_a, and eta uses W / w_{x_l}, which keeps it exactly unbiased.  Draws
 * use Lemire's bounded integers on Philox4x64-10.  T = 0 selects
 * T = ceil(ceil(log2 n_A) / eps^2).  eta = 0 if n_A = 0 or every D_a = 0.
 *   eta_out [1] double (device).  aux: optional extra outputs (see above).
 * opts.reduction = CHAMFER_REDUCE_PARTITION / _PAD runs the reduction above
 * first (with _PAD the estimate runs on the padded copies, d + m
 * coordinates, d + m <= 2048): if the partition is degenerate, has one
 * part, or leaves a part of A without points of B (probability <= 1/n), the
 * estimate is the plain one of the (padded) sets; otherwise it is the sum,
 * in ascending key order, of the estimates of the parts (rows in ascending
 * order, the same eps, T, seed and options).  aux must then be NULL, and
 * the call synchronises the stream (the host reads the partition; with
 * several parts it also returns only after the parts' estimates).
 * Errors: as crude_nn, plus EINVAL if T < 0.
 */
int chamfer_estimate(const float *A, const float *B, int64_t n_A, int64_t n_B, int32_t d,
                     int32_t metric, double eps, int64_t T, uint64_t seed, double *eta_out,
                     chamfer_aux *aux, const chamfer_opts *opts, void *ws, size_t ws_bytes,
                     void *stream);

/*
 * chamfer_estimate without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The workspace is a static
 * device array of CHAMFER_STATIC_SCRATCH_BYTES (64 MiB) that the library
 * holds on each device it runs on until the process ends; its address is
 * looked up once per device on the first call there.  The call allocates
 * nothing: arguments, outputs and results are exactly those of
 * chamfer_estimate with ws = that array.  The array keeps the last call's
 * contents; nothing in it needs to start at zero (every region the
 * estimate reads is written earlier in the same call).  All calls on one
 * device share the one array, so calls that overlap on a device (on
 * different streams, or from different host threads) race and give wrong
 * results: serialise them.  opts.reduction must be CHAMFER_REDUCE_NONE.
 * Errors: as chamfer_estimate, plus CHAMFER_ETOOLARGE when
 * chamfer_workspace_bytes(n_A, n_B, d, metric, eps, T, opts) exceeds
 * CHAMFER_STATIC_SCRATCH_BYTES (about 30,000 x 30,000 points at d = 128, or
 * 65,000 x 65,000 at d = 3, with the default options), checked before any
 * launch.
 */
#define CHAMFER_STATIC_SCRATCH_BYTES (64u << 20)
int chamfer_estimate_noalloc(const float *A, const float *B, int64_t n_A, int64_t n_B,
                             int32_t d, int32_t metric, double eps, int64_t T, uint64_t seed,
                             double *eta_out, chamfer_aux *aux, const chamfer_opts *opts,
                             void *stream);

/*
 * The bucket keys CrudeNN joins on, for inspection and testing (appendix
 * lemma on the grid hash at every scale).  For scale i and point x with
 * hashed coordinates y (l1: y_k = x_k - lo_k; l2: the embedding of x - lo):
 *   cell_k = ceilf(ldexpf(y_k, -e_i) + z'_ik) + 0.0f,
 *   key    = (sum_k bits(cell_k) * M_ik mod 2^64) >> 1.
 *   keys_A_out [L][n_A] uint64, keys_B_out [L][n_B] uint64 (either may be
 *   NULL), e_top_out [1] int32 or NULL.
 * Errors: as crude_nn.
 */
int chamfer_hash_keys(const float *A, const float *B, int64_t n_A, int64_t n_B, int32_t d,
                      int32_t metric, double eps, uint64_t seed, uint64_t *keys_A_out,
                      uint64_t *keys_B_out, int32_t *e_top_out, const chamfer_opts *opts,
                      void *ws, size_t ws_bytes, void *stream);

/*
 * Exact nearest neighbour of selected rows (step 3 of the Chamfer-Estimate
 * figure; also the inner loop of chamfer_exact).  Query q is row rows[q] of
 * X (or row q when rows is NULL), q < n_x; B has n_B rows.
 *   min_out [n_x] float, arg_out [n_x] int32 (either may be NULL): canonical
 *   float32 min and arg-min as in chamfer_exact.
 * Errors: as chamfer_exact (n_x < 0 is EINVAL).
 */
int chamfer_nn_min(const float *X, const int32_t *rows, int64_t n_x, const float *B,
                   int64_t n_B, int32_t d, int32_t metric, float *min_out, int32_t *arg_out,
                   const chamfer_opts *opts, void *ws, size_t ws_bytes, void *stream);

/*
 * Serving: continuous batching of chamfer_estimate requests (importance
 * sampling, the Chamfer-Estimate figure, run for many independent pairs).
 *
 * A server owns one device arena of arena_bytes, allocated once by
 * chamfer_server_create, and `lanes` (1..16) batch lanes, each with its own
 * stream (default priority), a device batch descriptor and pinned staging.
 * chamfer_server_submit queues a request (host side only; a request with
 * n_A == 0 is finished at once with eta = 0).  chamfer_server_progress never
 * blocks: it retires finished batches, which frees their lanes and arena
 * blocks at once, and while a lane is free forms the next batch.  The first
 * of the 9 oldest queued requests whose footprint (its two point sets and
 * its workspace, chamfer_workspace_bytes) fits the arena sets the batch's
 * class: (d, metric, embed_dim, precision, where precision counts as FP32
 * if the low-precision pass does not apply).  When that request is the
 * oldest, up to 64 requests of the same class among the 256 oldest that fit
 * the arena join it.  Inputs are copied in on the lane's stream and the
 * batch runs as ONE replay of a HIP graph captured once per lane and class,
 * in which each stage of the estimator is a single persistent-grid launch
 * over every request of the batch.  chamfer_server_results drains finished
 * requests (members of one batch share admit_s).  A request's host arrays A,
 * B (row-major float32; pinned memory makes the copy-in asynchronous) must
 * stay valid until its result is drained.  Results are bit-identical to a
 * direct chamfer_estimate call with the same arguments.  Requires d <= 2048
 * and the single-structure CrudeNN (opts.window and opts.reps 0 or 1).
 * A server is not thread-safe: call it from one host thread.
 * Errors: EINVAL for bad arguments (as chamfer_estimate, or d > 2048),
 * EWORKSPACE if a request can never fit the arena, EHIP for runtime
 * failures (a failed request is also reported through its result's status).
 */
typedef struct chamfer_server chamfer_server;

typedef struct chamfer_request {
    const float *A, *B;  /* host [n_A, d], [n_B, d] */
    int64_t n_A, n_B;
    int32_t d, metric;
    double eps;
    int64_t T;           /* 0 => default */
    uint64_t seed;
    chamfer_opts opts;
} chamfer_request;

typedef struct chamfer_result {
    uint64_t id;         /* as returned by chamfer_server_submit */
    int32_t status;      /* CHAMFER_OK, CHAMFER_ENONFINITE or a launch error */
    int32_t s;           /* fixed-point exponent */
    double eta;          /* the estimate */
    double D;            /* normaliser */
    uint64_t W;
    double submit_s, admit_s, done_s;  /* host steady-clock seconds */
    size_t footprint;    /* arena bytes the request held */
} chamfer_result;

typedef struct chamfer_server_stat {
    int64_t queued;
    int32_t in_flight;   /* requests admitted and not yet finished */
    int32_t lanes_busy;
    size_t arena_bytes, arena_used, arena_peak;
    int64_t batches;     /* batches launched */
    int64_t batched;     /* requests launched in those batches */
    int64_t graphs;      /* graphs instantiated (one per lane and class) */
    int64_t stalls;      /* admissions that found a free lane but no room in the arena */
} chamfer_server_stat;

int chamfer_server_create(size_t arena_bytes, int32_t lanes, chamfer_server **out);
/* Capture and instantiate, on every lane, the graph of the class of requests
 * with this d, metric, embed_dim (0 = default) and precision, so that the
 * first such request does not pay for it.  Optional. */
int chamfer_server_warm(chamfer_server *srv, int32_t d, int32_t metric, int32_t embed_dim,
                        int32_t precision);
int chamfer_server_submit(chamfer_server *srv, const chamfer_request *req, uint64_t *id_out);
int chamfer_server_progress(chamfer_server *srv); /* returns requests finished */
int chamfer_server_results(chamfer_server *srv, chamfer_result *out, int32_t max);
int chamfer_server_stats(const chamfer_server *srv, chamfer_server_stat *out);
int chamfer_server_destroy(chamfer_server *srv);

/*
 * Symmetric forms, CH(A, B) + CH(B, A) (the small-scale experiments).
 * out[0] = the sum, out[1] = the A->B value, out[2] = the B->A value
 * (device doubles).  The estimate runs chamfer_estimate in both directions
 * with the same eps, T (0 => each direction's default), seed and opts; the
 * exact form runs chamfer_exact both ways.  Both need n_A, n_B >= 1 and one
 * workspace of at least the larger of chamfer_workspace_bytes(n_A, n_B, ...)
 * and chamfer_workspace_bytes(n_B, n_A, ...) (eps = 0 for the exact form);
 * the two directions run one after the other on `stream`.  Errors as the
 * one-directional calls; a NaN in either direction makes the sum NaN.
 */
int chamfer_estimate_symmetric(const float *A, const float *B, int64_t n_A, int64_t n_B,
                               int32_t d, int32_t metric, double eps, int64_t T, uint64_t seed,
                               double *eta_out, const chamfer_opts *opts, void *ws,
                               size_t ws_bytes, void *stream);
int chamfer_exact_symmetric(const float *A, const float *B, int64_t n_A, int64_t n_B, int32_t d,
                            int32_t metric, double *ch_out, const chamfer_opts *opts, void *ws,
                            size_t ws_bytes, void *stream);

/*
 * One-vs-many retrieval (the downstream experiment of the experiments
 * section: the nearest cloud to A under CH(A, B) + CH(B, A)).  Bs holds m
 * clouds back to back (device, row-major float32); offsets (host, m + 1
 * entries, offsets[0] = 0, strictly increasing) gives cloud i as rows
 * offsets[i] .. offsets[i+1]-1.  For every cloud the symmetric estimate
 * eta(A, B_i) + eta(B_i, A) is computed (both directions with eps, T, seed
 * and opts; the jobs run up to 256 at a time through the batched estimator
 * stages) into est_out (device double[m], may be NULL); the k clouds with
 * the smallest estimates (ties to the lower index) are then re-ranked by
 * their exact symmetric CH (always float32, whatever opts.precision):
 * top_out (host int32[k]) gets their indices in
 * ascending order of exact CH (ties to the lower index) and top_ch_out
 * (host double[k]) the values.  opts.window, reps and sampling must be the
 * defaults; d <= 2048; every cloud non-empty.  The workspace needs
 * chamfer_retrieve_workspace_bytes (one estimator workspace sized for the
 * largest cloud per job of a batch, 256 jobs or as many as fit 4 GiB, plus
 * small tables; 0 on invalid arguments).  Synchronous: returns after the
 * stream has drained.  Errors as chamfer_estimate; a cloud with a NaN/Inf
 * coordinate gets a NaN estimate and ranks last.
 */
size_t chamfer_retrieve_workspace_bytes(int64_t n_A, const int64_t *offsets, int32_t m,
                                        int32_t d, int32_t metric, double eps, int64_t T,
                                        const chamfer_opts *opts);
int chamfer_retrieve(const float *A, int64_t n_A, const float *Bs, const int64_t *offsets,
                     int32_t m, int32_t d, int32_t metric, double eps, int64_t T, uint64_t seed,
                     int32_t k, const chamfer_opts *opts, double *est_out, int32_t *top_out,
                     double *top_ch_out, void *ws, size_t ws_bytes, void *stream);

/* Host helpers (no device work). */
int64_t chamfer_default_samples(int64_t n_A, double eps);            /* T default */
int32_t chamfer_default_scales(int64_t n_A, int64_t n_B, double eps); /* L default */
/* The l2 -> l1 embedding matrix chamfer_estimate uses for `seed`, into host
 * memory, [k_e][d] int8: Zq_jk = clamp(rint(32 g_jk), -127, 127), g_jk the
 * standard Gaussians of Philox purpose 2, counter (j d + k, 0), by
 * Box-Muller.  The hashed coordinates of a point x are
 * y_j = (float)((sum_k Zq_jk u_k) 2^(e_top - 24) / (sqrt(2/pi) k_e 32)),
 * u_k = floor(min((x_k - lo_k) 2^(24 - e_top), 2^24 - 1)), the integer sum
 * exact: the Gaussian embedding of the appendix theorem on quantised
 * coordinates. */
int chamfer_embedding_matrix(uint64_t seed, int32_t d, int32_t embed_dim, int8_t *Z_host);
const char *chamfer_strerror(int status);
/* The bound E of the l2 exact pass's certificate (the exact pass of
 * chamfer_exact, chamfer_nn_min and chamfer_estimate for l2 with
 * 12 <= d <= 256, FP32 precision): for a query x with float32 |x|^2 = xn2
 * and rows b with float32 |b|^2 <= b2max, the matrix-core score of every b
 * is within E of |b|^2 - 2 x.b, assuming the matrix cores add each product
 * to their float32 accumulator with one rounding to nearest.  terms = 3
 * (the estimator's draws, batches below 16384 queries) or 4 (larger
 * batches).  Returns -1 for d outside 1..256 or other terms. */
double chamfer_split_score_bound(int32_t d, int32_t terms, float xn2, float b2max);

#ifdef __cplusplus
}
#endif

#endif /* CHAMFER_H */
