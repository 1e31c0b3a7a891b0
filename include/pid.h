/*
 * pid.h -- C ABI of the MI355X (gfx950) Probabilistic Inclusion Depth library.
 *
 * The library computes, for an ensemble of N fuzzy contours given as
 * membership probabilities on M grid points, the Probabilistic Inclusion Depth
 * (PID) and its linear-time variant PID-mean, together with ranks.
 *
 * Notation (paper sections in parentheses):
 *   u_i(x) in [0,1]        membership probability of member i at point x (Sec. 3.2)
 *   w_x >= 0               volume of the cell of point x; 1 on uniform grids (Sec. 3.4)
 *   m_i = sum_x w_x u_i(x) mass of member i (Sec. 3.2)
 *   u <_p v = sum_x w u v / sum_x w u, and 0 when m(u) = 0
 *                           probabilistic inclusion operator (Sec. 3.2, Eqs.
 *                           expectation_form / prob_contain; Sec. 3.4 weighted form)
 *   PID:  IN_in(i) = (1/N) sum_j u_i <_p u_j,  IN_out(i) = (1/N) sum_j u_j <_p u_i,
 *         depth = min(IN_in, IN_out)            (Sec. 3.2, Eq. pid; the sums include j = i)
 *   PID-mean: ubar = (1/N) sum_i u_i; IN_in = u_i <_p ubar, IN_out = ubar <_p u_i,
 *         depth = min                             (Sec. 4.1)
 *   Fuzzy contour of a scalar field f with isovalue ~ N(c, sigma^2):
 *         u = Phi(side * (f - c) / sigma)          (Sec. 3.5, isovalue distribution)
 *   Rank: 0 = deepest; equal depths are ordered by the lower member index
 *         (ranking by depth, Sec. 5.1).
 *
 * Conventions of every call:
 *   - All array pointers are DEVICE pointers owned by the caller; the library
 *     never frees or keeps them.  The depth calls allocate no device memory:
 *     the caller passes a workspace of at least pid_workspace_size() bytes.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = the default
 *     stream).  Outputs are valid after that stream is synchronised.  Inputs
 *     are never modified.
 *   - Every call returns a pid_status.  Shape, dtype, pointer and scheme errors
 *     are detected on the host before anything is launched; the text of the
 *     last error of the calling thread is returned by pid_last_error().
 *   - Results are deterministic: the same inputs, shapes and scheme give
 *     bitwise identical outputs on the same device, whatever else runs.
 */
#ifndef PID_H_
#define PID_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PID_OK = 0,
  PID_ERR_INVALID_ARG = 1,          /* bad shape, null pointer, bad enum value        */
  PID_ERR_UNSUPPORTED = 2,          /* valid request this library does not implement  */
  PID_ERR_WORKSPACE_TOO_SMALL = 3,  /* ws_bytes < pid_workspace_size()                */
  PID_ERR_DEVICE = 4,               /* a HIP runtime call failed                      */
  PID_ERR_VALUE_RANGE = 5,          /* PID_FLAG_VALIDATE found a value out of range   */
  PID_ERR_OVER_BUDGET = 6,          /* serving: request larger than the whole arena   */
  PID_ERR_CANCELLED = 7,            /* serving: server stopped before the request ran */
  PID_ERR_INTERNAL = 8
} pid_status;

/* Element type of the stored ensemble. */
typedef enum {
  PID_F64 = 0, PID_F32 = 1, PID_F16 = 2, PID_BF16 = 3,
  PID_U8 = 4,  /* binary masks: every value must be 0 or 1 */
  PID_B1 = 5   /* bit-packed binary masks: point x of row i is bit (i*ld + x) mod 32 of
                  32-bit word (i*ld + x) / 32 (little-endian, so bit x mod 8 of byte x / 8 of
                  the row); ld (in points) a multiple of 32, data 4-byte aligned; bits past m
                  are ignored.  Taken by pid_mean (exact integers, no weights, PID_ISO_NONE)
                  and produced from U8 masks by pid_pack_bits; the other calls return
                  PID_ERR_UNSUPPORTED for it */
} pid_dtype;

/* How stored values become membership probabilities (Sec. 3.5, 3.6, 6.3). */
typedef enum {
  PID_ISO_NONE = 0,      /* values already are probabilities in [0,1] (soft masks)          */
  PID_ISO_GAUSSIAN = 1,  /* scalar field, isovalue ~ N(c, sigma^2): u = Phi(side*(f-c)/sigma) */
  PID_ISO_STEP = 2,      /* scalar field, sharp isovalue: u = 1 iff side*(f-c) > 0, else 0   */
  PID_ISO_RAMP = 3,      /* scalar field, isovalue uniform on [c - sigma, c + sigma] (Sec. 3.5):
                            u = P(isovalue < f) = clamp(1/2 + side*(f-c)/(2 sigma), 0, 1)     */
  PID_ISO_TENT = 4,      /* level-centred map (Sec. 3.6): u = max(0, 1 - |f - c| / sigma):
                            1 at the level c, falling linearly to 0 at distance sigma      */
  PID_ISO_DENSITY = 5    /* normalised density (Sec. 6.3): u = clamp(f / c, 0, 1), c > 0 the
                            normalising density (e.g. the ensemble's largest density,
                            pid_field_max)                                                  */
} pid_iso_kind;

/* Arithmetic of the all-pairs numerators G_ij = sum_x w u_i u_j. */
typedef enum {
  PID_GEMM_AUTO = 0,        /* I8 for unweighted binary input, F64 for F64 input, else F16    */
  PID_GEMM_F64 = 1,         /* FP64 vector FMA                                                */
  PID_GEMM_F32 = 2,         /* FP32 vector FMA (plain FP32 comparator)                        */
  PID_GEMM_F16 = 3,         /* FP16 MFMA, FP32 accumulation (inputs rounded to FP16 once)     */
  PID_GEMM_BF16 = 4,        /* BF16 MFMA, FP32 accumulation (inputs rounded to BF16 once)     */
  PID_GEMM_BF16_SPLIT = 5,  /* BF16 MFMA on hi/lo split inputs, three products, FP32 acc.     */
  PID_GEMM_I8 = 6           /* INT8 MFMA, INT32 accumulation: binary masks, no weights; exact */
} pid_gemm;

/* Flags of pid_ensemble.flags. */
#define PID_FLAG_VALIDATE 1u  /* check values first (probabilities in [0,1], U8 in {0,1},
                                 finite fields, weights finite and >= 0); the call then
                                 synchronises `stream` and returns PID_ERR_VALUE_RANGE
                                 without computing anything if a check fails.  Without
                                 it the values are trusted: one out of range (a NaN field
                                 value, say) gives unspecified depths, not an error     */

/* The ensemble: N members x M grid points, member-major.  Element (i, x) is at
 * data[i * ld + x] (ld >= M, in elements).  Rows whose byte address is a
 * multiple of 16 take the vectorised path; others are read element by element.
 * weights: M floats (w_x >= 0), or NULL for a uniform grid (w = 1). */
typedef struct {
  int64_t n;
  int64_t m;
  int64_t ld;
  int32_t dtype;    /* pid_dtype */
  uint32_t flags;   /* PID_FLAG_* */
  const void* data;
  const float* weights;
} pid_ensemble;

/* Isovalue model.  side = +1: f > c is inside (p = Phi((f - c)/sigma));
 * side = -1: f < c is inside (the sublevel set of Sec. 3.1 Eq. 2).  side
 * must be +1 or -1 for GAUSSIAN, STEP and RAMP and is ignored by TENT and
 * DENSITY.  sigma (GAUSSIAN: standard deviation; RAMP: half-width of the
 * isovalue interval; TENT: fall-off width) must be finite and > 0 there;
 * c must be finite, and > 0 for DENSITY.  RAMP, TENT and DENSITY take
 * F64, F32 or F16 fields (PID_ERR_UNSUPPORTED otherwise). */
typedef struct {
  int32_t kind;     /* pid_iso_kind */
  int32_t side;     /* +1 or -1 */
  double c;
  double sigma;
} pid_iso;

/* Outputs (device pointers; any may be NULL to skip it).
 *   inclusion: N x N row-major, inclusion[i*N + j] = u_i <_p u_j (all-pairs only)
 *   mass, in_in, in_out, depth: N doubles; rank, order: N int32
 *   (rank[i] = position of member i, 0 = deepest; order[k] = member at position k). */
typedef struct {
  double* inclusion;
  double* mass;
  double* in_in;
  double* in_out;
  double* depth;
  int32_t* rank;
  int32_t* order;
} pid_out;

/* Bytes of device workspace needed by pid_all_pairs (variant 0), pid_mean
 * (variant 1), pid_both (variant 2), pid_pairs_depths (variant 3; gemm is
 * ignored) or pid_mean_weighted (variant 4; gemm is ignored) for this
 * ensemble, isovalue model and
 * scheme.  The size depends on n, m, dtype, iso kind, weights (NULL or not)
 * and scheme only.  iso may be NULL (= PID_ISO_NONE). */
pid_status pid_workspace_size(const pid_ensemble* ens, const pid_iso* iso, int variant,
                              int gemm, size_t* bytes);

/* All-pairs PID (Sec. 3.2 Eq. pid with the weighted sums of Sec. 3.4).
 * The numerators G_ij are one symmetric Gram product of the N x M membership
 * matrix (scaled by sqrt(w)) computed with `gemm`; masses, ratios and depths are
 * FP64.  Fuzzy extraction (iso) is applied to each value as it is loaded.
 * PID_GEMM_I8 (and AUTO on unweighted U8 / STEP input) is exact: G and m are
 * integers and depths are bitwise reproducible from them (IN_in = S_i/(N m_i)
 * with S_i = sum_j G_ij; IN_out = (sum over ascending j of G_ij/m_j) / N). */
pid_status pid_all_pairs(const pid_ensemble* ens, const pid_iso* iso, int gemm,
                         const pid_out* out, void* workspace, size_t ws_bytes, void* stream);

/* All-pairs PID depths (Sec. 3.2 Eq. pid with the weighted sums of Sec. 3.4)
 * without the N x N inclusion matrix, in O(N M) work: by linearity,
 *   IN_in(i)  = S_i / (N m_i),  S_i = sum_x w u_i(x) s(x),  s = sum_j u_j,
 *   IN_out(i) = (1/N) sum_j G_ji / m_j = (1/N) sum_x w u_i(x) t(x),
 *   t(x) = sum_j u_j(x) / m_j  (members with m_j = 0 contribute 0),
 * so three streaming passes replace the Gram product: the PID-mean pass
 * (masses, IN_in), t into the workspace, and the row sums B_i = sum_x w u_i t
 * (IN_out = B_i / N).  FP32 sums inside a tile and in t, FP64 across tiles
 * (FP64 for FP64 input); binary input uses the same soft arithmetic for t and
 * B (IN_in stays exact).  out->inclusion is ignored; the other fields as
 * pid_all_pairs.  Workspace: pid_workspace_size(variant 3).  For large N, where
 * the Gram product's N^2 M work dominates, this reads the masks three times
 * instead (four beyond 256 members, where the PID-mean pass itself takes a
 * column-sum read and a row-sum read). */
pid_status pid_pairs_depths(const pid_ensemble* ens, const pid_iso* iso, const pid_out* out,
                            void* workspace, size_t ws_bytes, void* stream);

/* PID-mean (Sec. 4.1): one streaming pass over the ensemble computes, for
 * every member, m_i and A_i = sum_x w u_i(x) s(x) with s(x) = sum_j u_j(x);
 * then IN_in = A_i / (N m_i), IN_out = A_i / sum_k m_k.  FP32 inside a point
 * tile, FP64 across tiles; exact integers for unweighted binary input.
 * out->inclusion is ignored. */
pid_status pid_mean(const pid_ensemble* ens, const pid_iso* iso, const pid_out* out,
                    void* workspace, size_t ws_bytes, void* stream);

/* PID-mean against a reliability-weighted mean contour (Sec. 4.1, the
 * optional weighting of the point-wise mean): with member weights r_j >= 0
 * (member_w: N device doubles, not all 0; the library reads them, the caller
 * owns them), ubar = sum_j r_j u_j / R with R = sum_j r_j, IN_in = u_i <_p ubar
 * = A_i / (R m_i) and IN_out = ubar <_p u_i = A_i / sum_j r_j m_j, where
 * A_i = sum_x w u_i(x) sum_j r_j u_j(x).  Two streaming passes: the weighted
 * column sums into the workspace, then m_i and A_i.  FP32 sums inside a tile
 * (FP64 for FP64 input), FP64 across tiles; binary input takes the same soft
 * arithmetic.  R <= 0 gives zero depths.  out->inclusion is ignored; the
 * other outputs as pid_mean.  Workspace: pid_workspace_size(variant 4).
 * Unit weights give the values of pid_mean within its tolerance. */
pid_status pid_mean_weighted(const pid_ensemble* ens, const pid_iso* iso, const double* member_w,
                             const pid_out* out, void* workspace, size_t ws_bytes, void* stream);

/* Packs U8 0/1 masks (ens: dtype PID_U8, any row stride) into PID_B1 rows:
 * row i of `out` (device, 4-byte aligned) starts at 32-bit word i * out_ld / 32,
 * out_ld (in points) a multiple of 32 and >= m; the words past the last one
 * that holds points are left untouched.  A nonzero byte counts as 1.  One
 * launch, asynchronous on `stream`.  Bit-packed masks hold one bit per point,
 * an eighth of the U8 bytes, for the binary ensembles of Sec. 5.2 and 6.2. */
pid_status pid_pack_bits(const pid_ensemble* ens, void* out, int64_t out_ld, void* stream);

/* Largest stored value of the ensemble (values that are NaN are skipped; NaN
 * if every value is), written as one double to the device pointer max_out
 * (8-byte aligned): e.g. the normalising density c of PID_ISO_DENSITY (Sec.
 * 6.3), read back by the caller before the depth call.  Exact; one streaming
 * pass, asynchronous on `stream`.  Weights and flags are ignored. */
pid_status pid_field_max(const pid_ensemble* ens, double* max_out, void* stream);

/* All-pairs PID and PID-mean of one ensemble (Sec. 3.2 with the weighted
 * sums of Sec. 3.4, and Sec. 4.1) from one all-pairs pass.  pairs_out as
 * pid_all_pairs with `gemm` (bitwise the same results).  The PID-mean
 * numerators are the Gram row sums: A_i = sum_x w u_i(x) s(x) with
 * s = sum_j u_j equals S_i = sum_j G_ij, so mean_out gets IN_in = S_i/(N m_i)
 * (the all-pairs IN_in: the recall identity of Sec. 4.1) and
 * IN_out = S_i / sum_k m_k (sum_k m_k by a fixed tree), with the masses of the
 * same pass.  mean_out therefore has the accuracy of the `gemm` scheme:
 * bitwise the oracle's integer forms for PID_GEMM_I8, within the mixed
 * precision tolerance for FP16/BF16 (pid_mean keeps its FP32/FP64 sums).
 * Workspace: pid_workspace_size(variant 2) (that of variant 0 plus room for
 * a second depth array).  Errors as pid_all_pairs; both output structs are
 * required (their fields may be NULL). */
pid_status pid_both(const pid_ensemble* ens, const pid_iso* iso, int gemm, const pid_out* pairs_out,
                    const pid_out* mean_out, void* workspace, size_t ws_bytes, void* stream);

/* pid_both without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  The workspace is a fixed array of
 * PID_STATIC_SCRATCH_BYTES in the library's device code: one copy per GPU,
 * allocated when the library's code is loaded on that GPU and held until the
 * process ends; the call itself allocates nothing.  Outputs, results and
 * errors as pid_both; PID_ERR_UNSUPPORTED when the call's workspace
 * (pid_workspace_size, variant 2) exceeds the array.  Every call on one GPU
 * uses the same array, so calls on one GPU must not overlap: two calls on
 * different streams, or from different threads, without an ordering between
 * them race on it. */
#define PID_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
pid_status pid_both_static(const pid_ensemble* ens, const pid_iso* iso, int gemm, const pid_out* pairs_out,
                           const pid_out* mean_out, void* stream);

/* Fuzzy-contour extraction alone (Sec. 3.5): writes u = model(value) for the
 * N x M ensemble into `u_out` (dense N x M, row stride M) as float (out_dtype
 * PID_F32) or double (PID_F64); Phi by erfcf for float output and erfc for
 * double output. */
pid_status pid_extract(const pid_ensemble* ens, const pid_iso* iso, void* u_out, int out_dtype,
                       void* stream);

/* Contour-boxplot bands of a ranked ensemble (the depth -> percentile ->
 * boxplot pipeline of Sec. 1; the envelopes of Sec. 6 / 6.1).  Each member
 * is binarised after extraction (iso, as above): a point is inside when
 * u >= threshold (0.5 for soft masks, 0.02 for normalised densities in the
 * paper's examples), the decision taken in FP64.  `order` (device, int32,
 * at least k_outer entries) lists members deepest first, as pid_rank's
 * order; the median is order[0], the inner band the k_inner deepest, the
 * outer band the k_outer deepest (e.g. ceil(N/2) and N for the 50 % and
 * 100 % groups), 1 <= k_inner <= k_outer <= N.  `out` (device, M bytes,
 * owned by the caller) receives per point the bits
 *   1 median inside, 2 union of the inner band, 4 intersection of the inner
 *   band, 8 union of the outer band, 16 intersection of the outer band,
 *   128 some order entry among the first k_outer was outside 0..N-1 (such an
 *   entry is skipped, never read through).
 * Ensemble weights are ignored.  Reads k_outer rows of M values once; one
 * launch, asynchronous on `stream`.  PID_ERR_INVALID_ARG on NULL pointers,
 * bad k or a non-finite threshold. */
pid_status pid_bands(const pid_ensemble* ens, const pid_iso* iso, const int32_t* order, int64_t k_inner,
                     int64_t k_outer, double threshold, uint8_t* out, void* stream);

/* Ranks from depths (device arrays of n): rank 0 = deepest, ties by index. */
pid_status pid_rank(const double* depth, int64_t n, int32_t* rank, int32_t* order, void* stream);

/* ---------------------------------------------------------------------------
 * Serving: requests of uneven ensemble and grid size, admitted by device-memory
 * footprint and run concurrently (continuous batching).  The workload is one
 * depth call per request (Sec. 3.2 Eq. pid with Sec. 3.4, or Sec. 4.1).
 *
 * The server owns no device memory of its own: `arena` is a caller-allocated
 * device buffer of `arena_bytes` from which each admitted request's workspace
 * is carved.  A request waits in the admission queue until (a) one of
 * `max_slots` execution slots (HIP streams) is free, (b) its workspace fits in
 * the arena (first fit) and (c) its footprint -- the bytes of its stored
 * ensemble, weights and outputs plus its workspace -- keeps the footprint of
 * all running requests within the budget set by pid_server_set_budget (no
 * budget by default).  Queued requests are taken in arrival order; one that
 * does not fit yet is passed over by later ones until it has waited 50 ms,
 * after which nothing starts ahead of it.  The ensemble and output buffers
 * of a request stay owned by the caller and must stay valid until the
 * request completes.  Results of a request are bitwise identical to the same
 * request run alone through pid_all_pairs / pid_mean / pid_pairs_depths.
 * ------------------------------------------------------------------------- */
typedef struct pid_server pid_server;

typedef struct {
  int32_t variant;   /* 0 = all-pairs, 1 = PID-mean, 3 = all-pairs depths without the matrix */
  int32_t gemm;      /* pid_gemm (all-pairs only)   */
  pid_ensemble ens;
  pid_iso iso;
  pid_out out;
  /* Optional hipEvent_t (NULL: none).  The request's kernels run on the
   * server's own streams; when set, its slot stream waits for this event
   * (hipStreamWaitEvent at admission) before them, so inputs that the
   * caller's stream is still producing are complete when read.  The event
   * must stay valid until the request has started. */
  void* ready;
} pid_request;

pid_status pid_server_create(int device, void* arena, size_t arena_bytes, int max_slots,
                             pid_server** server);
/* Footprint budget in bytes (0 = none).  A request whose footprint alone
 * exceeds it is refused by pid_submit with PID_ERR_OVER_BUDGET. */
pid_status pid_server_set_budget(pid_server* server, size_t footprint_bytes);
/* Non-blocking: validates the request, queues it and returns a ticket.
 * PID_ERR_OVER_BUDGET when its workspace exceeds the arena or its footprint
 * the budget; PID_ERR_CANCELLED once the server is stopping. */
pid_status pid_submit(pid_server* server, const pid_request* req, uint64_t* ticket);
/* done = 1 once the request finished; result = its status (PID_OK or an
 * error).  After a failed request, pid_last_error() of the calling thread
 * holds the request's error text. */
pid_status pid_poll(pid_server* server, uint64_t ticket, int* done, pid_status* result);
/* Blocks until the request finished; result and error text as pid_poll. */
pid_status pid_wait(pid_server* server, uint64_t ticket, pid_status* result);
/* Seconds on the server's clock (pid_server_clock): submission, admission
 * (start of its launch) and the moment the scheduler saw it complete. */
pid_status pid_request_times(pid_server* server, uint64_t ticket, double* t_submit,
                             double* t_start, double* t_done);
/* Start and end of the request's work on the device, in milliseconds after
 * the server's creation, from timing events recorded on its slot stream
 * before its first and after its last kernel.  PID_ERR_INVALID_ARG unless the
 * request completed with PID_OK. */
pid_status pid_request_device_times(pid_server* server, uint64_t ticket, double* start_ms,
                                    double* end_ms);
/* The server's clock: seconds since creation (a monotonic clock). */
pid_status pid_server_clock(pid_server* server, double* now_s);
/* Forget a finished request (its ticket becomes unknown).  A server keeps
 * every ticket's record until it is released or the server is destroyed.
 * PID_ERR_INVALID_ARG for unknown or unfinished tickets. */
pid_status pid_release(pid_server* server, uint64_t ticket);
/* Stops admitting, lets running requests finish, cancels queued ones
 * (PID_ERR_CANCELLED), joins the scheduler thread and frees host resources. */
pid_status pid_server_destroy(pid_server* server);

/* Per-kernel timing (diagnostics for benchmarks).  When on, every kernel the
 * library launches is bracketed by a pair of HIP events recorded on its
 * stream.  pid_timing_enable() clears the accumulated times (and waits for
 * pending events); pid_timing_get() waits for the pending events and returns
 * the total milliseconds and launch count of one kernel: "gram" (all-pairs
 * numerators), "gram_reduce", "pairs_finish" (inclusion rows, depths and,
 * after a fused pass, the PID-mean ratios), "pidmean" (the streaming PID-mean
 * pass), "pidmean_colsum", "pidmean_finalize", "rank", "extract", "bands".  Unknown
 * names report 0. */
pid_status pid_timing_enable(int on);
pid_status pid_timing_get(const char* kernel, double* total_ms, int64_t* launches);
/* Restrict timing to a comma-separated list of the kernel names above (so
 * that a benchmark brackets only the kernel it reports); NULL or "" times
 * every kernel again.  Takes effect for launches after the call. */
pid_status pid_timing_select(const char* names);
/* Bracket only every `every`-th launch of each timed kernel (launches 0,
 * every, 2*every, ... counted per kernel name since the last enable or
 * sample call), so that a benchmark can measure a kernel's duration inside
 * its timed loop while paying the events' cost on a fraction of the
 * launches; pid_timing_get() then counts the bracketed launches only.
 * 1 (the default) brackets all.  PID_ERR_INVALID_ARG outside 1..2^20. */
pid_status pid_timing_sample(int every);

/* Diagnostics. */
const char* pid_status_string(pid_status s);
const char* pid_last_error(void);   /* thread-local text of the last failed call */
int pid_abi_version(void);          /* 3 */

#ifdef __cplusplus
}
#endif
#endif /* PID_H_ */
