/*
 * tac.h -- C ABI of libtac, the MI355X (gfx950) token-aware clustering library.
 *
 * The library computes the index-build path of Token-Aware Clustering
 * (Sect. 2.1 of the paper): group token vectors by token id, give every token a
 * centroid budget from its frequency and spread (Phases 1-4), run Lloyd's
 * k-means independently inside every token's vectors, and compress the
 * normalised residuals with product quantisation (Sect. 2.1, "Residuals
 * Compression"; M = 32 subspaces of 8-bit codes in Sect. 3.1).
 *
 * Conventions shared by every call
 *  - Pointers ending in _d are device pointers (HIP device memory of the
 *    context's device); pointers ending in _h are host pointers.  Arrays are
 *    dense and row-major; vectors are float32 rows of d = 128 values.
 *  - The caller owns every input and output buffer.  The context owns only its
 *    workspace, which grows on demand.  A workspace that has to grow is
 *    replaced, and the replaced allocation stays until tac_ctx_destroy, so a
 *    HIP graph captured earlier keeps addressing valid memory; every
 *    allocation the context holds counts towards max_workspace_bytes.  No
 *    call keeps a caller pointer after it returns.
 *  - Every call except tac_budget, tac_init_centroids, tac_assign_stats and
 *    tac_gather only enqueues work on the context's HIP stream and returns;
 *    the caller keeps buffers alive until that stream has finished the work.
 *    These calls may be captured into a HIP graph once one eager call of the
 *    same sizes has grown the workspace (growth is refused during capture).
 *  - Arguments are checked on the host before anything is launched; on any
 *    error nothing is enqueued and the call returns a negative status, with a
 *    message in tac_last_error().  No call aborts or throws.
 *  - Results are deterministic: the same inputs give bitwise-identical
 *    outputs, independent of launch shapes and of what else is in a batch.
 *  - Assignments and PQ codes are the argmin of a canonical FP32 squared
 *    distance over the candidate set, lowest index on equal values:
 *        acc = 0; for i in 0..d-1: t = x_i - c_i; acc = acc + t*t
 *    with every operation rounded to float32 and no fused multiply-add.
 *    Matrix-core screens only nominate candidates; a rigorous error bound
 *    certifies that no other candidate can win, else the vector is rescored
 *    exhaustively.  TAC_FP32, TAC_BF16 and TAC_F16 therefore return identical argmins.
 *  - One context per host thread, or external locking.
 */
#ifndef TAC_H
#define TAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tac_ctx_s* tac_ctx;

typedef enum {
    TAC_OK = 0,
    TAC_E_INVAL = -1,       /* bad argument (sizes, NULL, d != 128, ...) */
    TAC_E_INFEASIBLE = -2,  /* no budget satisfies the bounds for this K */
    TAC_E_NOMEM = -3,       /* workspace would exceed max_workspace_bytes, or growth during capture */
    TAC_E_HIP = -4,         /* a HIP runtime call failed; the HIP error string is in tac_last_error() */
    TAC_E_UNSEEN_TOKEN = -5 /* a token with vectors has no centroids (reported by tac_assign_stats) */
} tac_status;

typedef enum {
    TAC_FP32 = 0,  /* FP32 matrix-core screen (v_mfma_f32_16x16x4f32) */
    TAC_BF16 = 1,  /* BF16 matrix-core screen, FP32 accumulation: x.c from three BF16
                      products of hi/lo splits (v_mfma_f32_16x16x32_bf16) */
    TAC_F16 = 2    /* FP16 matrix-core screen, FP32 accumulation: x.c from one FP16
                      product per coordinate (v_mfma_f32_16x16x32_f16); the certificate
                      bounds both operands' rounding by their measured norms */
} tac_precision;

typedef enum {
    TAC_THETA_FILL_THEN_RELAX = 0, /* fill up to the theta caps, then relax theta to n_j */
    TAC_THETA_SOFT = 1             /* drop theta from the start when the caps cannot hold B */
} tac_theta_policy;

/* Budget parameters (Sect. 2.1, Phases 1-3; values of Sect. 3.1: 128, 256, 4, 39). */
typedef struct {
    int64_t mu;            /* micro tokens: n < mu get 1 centroid */
    int64_t tau;           /* small tokens: mu <= n < tau get 2; n >= tau are active */
    int64_t eps;           /* floor: every active token gets at least eps */
    double theta;          /* cap: n_j / kappa_j >= theta (theta <= 0: no cap) */
    int32_t theta_policy;  /* tac_theta_policy */
} tac_budget_params;

/* Counters of the last tac_assign on a context (see tac_assign_stats). */
typedef struct {
    int64_t rows;          /* rows assigned */
    int64_t screened;      /* rows decided by a matrix-core screen plus certificate */
    int64_t fallback;      /* screened rows whose certificate failed -> exhaustive rescoring */
    int64_t unassigned;    /* rows whose token has no centroid (assign = -1) */
} tac_assign_counters;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  The context's device
 * allocations (current and replaced workspaces) stay within
 * max_workspace_bytes (0 = no limit).  The context also owns a second stream
 * (default priority) on which tac_assign runs its split-route kernel; every
 * call forks it from and joins it back to the context's stream with events, so
 * callers only ever order work on the context's stream.  On success *out holds
 * the context. */
tac_status tac_ctx_create(int device, void* hip_stream, size_t max_workspace_bytes, tac_ctx* out);

/* Switch the stream later calls enqueue on.  The caller orders it after any
 * work still in flight on the previous stream that uses the workspace. */
tac_status tac_ctx_set_stream(tac_ctx ctx, void* hip_stream);

/* Kernel timing (measurement aid).  When enabled, each entry point records HIP
 * events on the context's stream around its dominant kernel, one slot each:
 *  TAC_SLOT_ASSIGN  the persistent assignment kernel of tac_assign
 *  TAC_SLOT_UPDATE  the centroid-mean kernels of tac_update (flags + means)
 *  TAC_SLOT_ENCODE  the fused residual + PQ encode kernel of pq_encode
 * tac_kernel_ms waits for the slot's stop event and returns the elapsed time of
 * its last recording (TAC_E_INVAL if never recorded).  Keep timing disabled
 * while capturing a graph. */
#define TAC_KERNEL_SLOTS 3
enum { TAC_SLOT_ASSIGN = 0, TAC_SLOT_UPDATE = 1, TAC_SLOT_ENCODE = 2 };
tac_status tac_ctx_enable_timing(tac_ctx ctx, int enable);
tac_status tac_kernel_ms(tac_ctx ctx, int slot, float* ms);

/* Launch tuning of tac_assign, chosen per workload by measurement
 * (paper_2604_28142_amd/autotune.py).  Results do not depend on it.
 *  direct_max_kappa  tokens with at most this many centroids (0..16) skip the
 *                    matrix-core screen and compute every canonical distance;
 *                    tokens without centroids always take that route (default 4)
 *  heavy_kappa       tokens with at least this many centroids are scheduled
 *                    first in the persistent work queue (default 1024)
 *  groups_per_cu     persistent work-groups per compute unit; 0 = as many as
 *                    fit (default 0)
 *  tile_blocks       the 16-bit screens' tile shape: column blocks of 16 rows
 *                    per wave, so a work item is 64 * tile_blocks rows of one
 *                    token; 3, 4 or 5 (each is compiled), 0 = the default of
 *                    the occupancy (3 at two work-groups per CU, 5 at one).
 *                    The FP32 screen keeps its 512-row items.
 *  waves_per_simd    the 16-bit screens' occupancy: 1 = one 256-thread
 *                    work-group per compute unit (a wave per SIMD, the whole
 *                    register file, 32 KiB centroid stages); 2 = two of them
 *                    (two waves per SIMD, half of each, 16 KiB stages), whose
 *                    tile is 3 column blocks (tile_blocks must then be 0 or 3);
 *                    0 = two, unless tile_blocks is 4 or 5 (default 0).  The
 *                    FP32 screen ignores it. */
typedef struct {
    int32_t direct_max_kappa;
    int32_t heavy_kappa;
    int32_t groups_per_cu;
    int32_t tile_blocks;
    int32_t waves_per_simd;
} tac_tuning;
tac_status tac_ctx_set_tuning(tac_ctx ctx, const tac_tuning* tuning);
tac_status tac_ctx_get_tuning(tac_ctx ctx, tac_tuning* tuning);

/* Declare centroids unchanging (a resident index, as in the encode service):
 * their squared norms, norm bounds and 16-bit staging rows, which tac_assign
 * otherwise recomputes from all K centroids on every call, are prepared once
 * here for this precision.  Later tac_assign calls on this context with
 * exactly this (C_d, K, precision) use them; any other call prepares its own
 * as before.  The caller must not change C_d's contents while the
 * declaration stands.  C_d = NULL clears it.  The prepared buffer (about
 * 516 bytes per centroid for TAC_BF16, 260 for TAC_F16, 4 for TAC_FP32) is
 * held until the context is destroyed, also after clearing, because a graph
 * captured on the context may address it.  Not allowed during stream
 * capture.  Synchronous (later calls may use another stream). */
tac_status tac_ctx_set_static_centroids(tac_ctx ctx, const float* C_d, int64_t K, int32_t precision);

/* Wait for the context's stream, then free the workspace and the context. */
void tac_ctx_destroy(tac_ctx ctx);

/* Message of the last non-OK status returned on this host thread ("" if none). */
const char* tac_last_error(void);

/* Group by token and budget (Sect. 2.1, Phases 1-4).  Synchronous.
 *  x_d      [N, d] float32 token vectors; tok_d [N] int32 token ids in [0, T).
 *  K        total number of centroids (sum of kappa).
 *  params   NULL = the defaults of Sect. 3.1 (128, 256, 4, 39, fill-then-relax).
 *  spread_override_h  [T] float64 or NULL: when given, the budget uses these
 *           spreads instead of the ones computed on the GPU (spread_h still
 *           receives the GPU values).
 * Outputs (each may be NULL unless noted):
 *  perm_d   [N] int32: sorted row i is input row perm_d[i]; segments ascend by
 *           token id and keep input order inside a token (stable).  Required.
 *  xs_d     [N, d] float32: the token-sorted rows x[perm].
 *  seg_off_d/_h [T+1] int64: token j owns sorted rows [seg_off[j], seg_off[j+1]).
 *  count_h  [T] int64 vectors per token;  spread_h [T] float64 spread
 *           s_j = (1/n_j) sum ||x - mean_j||^2 (two-pass, float64).
 *  kappa_h  [T] int64 centroids per token (sum = K).
 *  cent_off_d/_h [T+1] int64: token j owns centroids [cent_off[j], cent_off[j+1]).
 * Errors: TAC_E_INVAL for token ids outside [0, T) or bad sizes,
 * TAC_E_INFEASIBLE when K is below the tail plus eps per active token or above
 * the number of active vectors. */
tac_status tac_budget(tac_ctx ctx, const float* x_d, const int32_t* tok_d, int64_t N, int32_t d,
                      int32_t T, int64_t K, const tac_budget_params* params,
                      const double* spread_override_h, int32_t* perm_d, float* xs_d,
                      int64_t* seg_off_d, int64_t* seg_off_h, int64_t* count_h, double* spread_h,
                      int64_t* kappa_h, int64_t* cent_off_d, int64_t* cent_off_h);

/* The budget alone (Phases 1-4 of Sect. 2.1) from per-token statistics, on the
 * host: counts_h [T] int64 vectors per token, spread_h [T] float64 spreads.
 * kappa_h [T] int64 output (sum = K); tier2_h (nullable) receives the number
 * of units placed after the theta caps were relaxed.  This is the budget
 * tac_budget applies after computing the statistics on the GPU; it needs no
 * device.  Errors as for tac_budget. */
tac_status tac_budget_from_stats(const int64_t* counts_h, const double* spread_h, int32_t T, int64_t K,
                                 const tac_budget_params* params, int64_t* kappa_h, int64_t* tier2_h);

/* Seeded initial centroids (the paper states none): centroid k of token j is
 * sorted row seg_off[j] + picks_d[k], with picks_d[k] in [0, n_j).
 * picks_d [K] int32; C_d [K, d] float32 output.  Synchronous (validates picks). */
tac_status tac_init_centroids(tac_ctx ctx, const float* xs_d, const int64_t* seg_off_d,
                              const int64_t* cent_off_d, int32_t T, int32_t d,
                              const int32_t* picks_d, int64_t K, float* C_d);

/* Assignment step of per-token Lloyd (Sect. 2.1): every row goes to the
 * nearest centroid of its own token (canonical FP32 distance, lowest index on
 * ties).  Asynchronous.
 * Segments are given either by seg_off_d (rows of x_d token-sorted) or by tok_d
 * (rows in any order, grouped internally; the serving path); exactly one of
 * the two is non-NULL.
 *  C_d [K, d] float32 centroids, cent_off_d [T+1] int64.
 *  assign_d [N] int32 output: global centroid id, or -1 for a row whose token
 *           has no centroid (or, with tok_d, an id outside [0, T)).
 *  dist_d   [N] float32 output or NULL: canonical distance to that centroid.
 *  inertia_d device float64 scalar or NULL: sum of dist over assigned rows,
 *           summed in float64 in a fixed order (within-cluster sum of squares).
 * With TAC_BF16 and TAC_F16, a token of at most 8,192 rows and at least 2,048
 * centroids (a serving batch's frequent token; a clustering budget gives such
 * a kappa_j only to tokens with far more rows) is screened as (row tile,
 * 1,024-centroid chunk) work items of a second launch across the device, each
 * chunk's exact minimum merged per row; the results are the same as on every
 * other route.  The workspace holds one 12-byte slot per such row. */
tac_status tac_assign(tac_ctx ctx, const float* x_d, const int64_t* seg_off_d, const int32_t* tok_d,
                      int64_t N, int32_t d, int32_t T, const float* C_d, const int64_t* cent_off_d,
                      int64_t K, int32_t precision, int32_t* assign_d, float* dist_d,
                      double* inertia_d);

/* tac_assign without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops that must not call
 * hipMalloc).  Same arguments, results and errors as tac_assign; the results
 * are bitwise those of tac_assign.  Its workspace is one fixed 64 MiB scratch
 * array per device inside the library (held by every device the library runs
 * on until the process ends) instead of the context's arena, so a call whose
 * workspace would exceed 64 MiB returns TAC_E_NOMEM without launching
 * anything.  The need grows with N (about 60 bytes per row on the serving
 * path), T (about 50 bytes per token) and, unless the centroids were prepared
 * with tac_ctx_set_static_centroids for this (C_d, K, precision), with K
 * (4 bytes per centroid in FP32, 516 in BF16, 260 in FP16): a serving batch
 * of 100k rows over 30,522 tokens against prepared centroids needs about
 * 10 MB.  Every call on a device shares that device's scratch: calls that
 * overlap on one device (other streams, other contexts, other threads) race
 * and must be serialised by the caller.  The scratch keeps the last call's
 * contents; every part a kernel reads is written earlier in the same call. */
tac_status tac_assign_noalloc(tac_ctx ctx, const float* x_d, const int64_t* seg_off_d, const int32_t* tok_d,
                              int64_t N, int32_t d, int32_t T, const float* C_d, const int64_t* cent_off_d,
                              int64_t K, int32_t precision, int32_t* assign_d, float* dist_d,
                              double* inertia_d);

/* Device workspace, in bytes, that tac_assign takes on this context for a call
 * of N rows over T tokens and K centroids at `precision`, with token ids
 * (with_tok != 0: the serving path) or token-sorted rows, with or without a
 * dist_d output (with_dist), given the centroids the context has prepared
 * (tac_ctx_set_static_centroids) for that precision.  For callers that budget
 * device memory (an encode service admitting batches by memory).  Host-only:
 * launches nothing.  TAC_E_INVAL for NULL arguments or sizes out of range. */
tac_status tac_assign_workspace_bytes(tac_ctx ctx, int64_t N, int32_t T, const float* C_d, int64_t K,
                                      int32_t precision, int with_tok, int with_dist, size_t* bytes);

/* Counters of the last tac_assign on this context.  Synchronises the stream. */
tac_status tac_assign_stats(tac_ctx ctx, tac_assign_counters* out);

/* Update step of Lloyd (Sect. 2.1): each centroid becomes the mean of the rows
 * assigned to it; a centroid with no rows keeps C_old.  Asynchronous.
 *  xs_d [N, d] token-sorted rows; seg_off_d [T+1]; assign_d [N] (rows with -1
 *  are ignored); C_old_d, C_new_d [K, d] float32 (may not alias);
 *  count_d [K] int64 output or NULL.
 * Sums run in a fixed order: compensated float32 for tokens with at most
 * 65,536 rows, float64 above; the mean is rounded to float32. */
tac_status tac_update(tac_ctx ctx, const float* xs_d, const int64_t* seg_off_d, int32_t T, int64_t N,
                      int32_t d, const int32_t* assign_d, const float* C_old_d, int64_t K,
                      float* C_new_d, int64_t* count_d);

/* Residuals (Sect. 2.1, "Residuals Compression"): for i < n, with
 * row = rows_d ? rows_d[i] : i, r = x[row] - C[assign[row]], rho = ||r||,
 * u = r / rho (u = 0 when rho = 0; normalize = 0 keeps u = r).  Asynchronous.
 *  R_d [n, d] float32 output; rnorm_d [n] float32 output or NULL.
 *  rows_d [n] int64 or NULL.  Rows with assign -1 give u = 0, rho = 0. */
tac_status tac_residuals(tac_ctx ctx, const float* x_d, const int32_t* assign_d, const float* C_d,
                         int64_t K, const int64_t* rows_d, int64_t n, int32_t d, int normalize,
                         float* R_d, float* rnorm_d);

/* PQ codebook training (Sect. 3.1: M subspaces, 8-bit codes): `iters` Lloyd
 * iterations per subspace on the rows R_d [n, d], subspace m = coordinates
 * [m*d/M, (m+1)*d/M).  init_d and codebooks_d are [M, ksub, d/M] float32
 * (may alias).  Empty codes keep their value.  Asynchronous.
 * Requires d % M == 0, d/M == 4, ksub <= 256. */
tac_status pq_train(tac_ctx ctx, const float* R_d, int64_t n, int32_t d, int32_t M, int32_t ksub,
                    int32_t iters, const float* init_d, float* codebooks_d);

/* Residual + normalise + PQ encode, fused (Sect. 2.1): codes_d [n, M] uint8,
 * code m = argmin over the ksub codes of the canonical distance between the
 * subvector m of u and the code vector.  rnorm_d [n] float32 or NULL.
 * assign_d [n] int32 (the row's centroid; -1 gives codes 0 and rho 0).
 * normalize = 0 encodes r itself.  Asynchronous. */
tac_status pq_encode(tac_ctx ctx, const float* x_d, const int32_t* assign_d, const float* C_d,
                     int64_t K, int64_t n, int32_t d, const float* codebooks_d, int32_t M,
                     int32_t ksub, int normalize, uint8_t* codes_d, float* rnorm_d);

/* Inverted lists (Sect. 2.2, "Index Structure"): every centroid keeps the ids
 * of the documents whose tokens are assigned to it.  assign_d [N] int32 (the
 * token's centroid; outside [0, K) enters no list), doc_d [N] int32 (the
 * token's document; outside [0, D) enters no list), in any order.  Output:
 * list_off_d [K + 1] int64 and list_docs_d (capacity N int32); list k is
 * list_docs_d[list_off_d[k] .. list_off_d[k + 1]), each document id once, in
 * increasing order; list_off_d[K] is the number of entries.  The caller owns
 * all buffers; the workspace grows by about 40 bytes per token.  Asynchronous;
 * TAC_E_INVAL on bad sizes or NULL pointers. */
tac_status tac_ivf_build(tac_ctx ctx, const int32_t* assign_d, const int32_t* doc_d, int64_t N, int64_t K,
                         int64_t D, int64_t* list_off_d, int32_t* list_docs_d);

/* Document layout (Sect. 2.2, "Document Layout"): per document, the centroid
 * ids of all of its tokens contiguously, followed by all of their PQ codes.
 * The tokens of document d are rows doc_off_d[d] .. doc_off_d[d + 1] - 1
 * (doc_off_d [D + 1] int64, non-decreasing from 0 to N); assign_d [N] int32,
 * codes_d [N, M] uint8.  Output layout_d [N * (4 + M)] uint8: document d
 * occupies bytes [doc_off_d[d] * (4 + M), doc_off_d[d + 1] * (4 + M)): its
 * centroid ids as 4-byte little-endian integers, then its codes in token
 * order (M per token).  Offsets outside [0, N] are clamped, so a malformed
 * doc_off_d never addresses memory outside the layout (the affected documents'
 * bytes are then unspecified).  Asynchronous; TAC_E_INVAL on bad sizes. */
tac_status tac_doc_layout(tac_ctx ctx, const int32_t* assign_d, const uint8_t* codes_d, int32_t M,
                          const int64_t* doc_off_d, int64_t D, int64_t N, uint8_t* layout_d);

/* Gather phase of retrieval (Sect. 2.2, "Gather Phase: Centroid-based
 * Document Scoring"): for each of the B queries,
 *  1. every query token q_i takes the kc centroids of largest <q_i, c_j>
 *     (exactly: the paper's HNSW graph approximates this set; ties go to the
 *     lower centroid id);
 *  2. s_i(d) = the largest <q_i, c_j> over those centroids whose inverted list
 *     holds document d;
 *  3. S(q, d) = sum_i s_i(d) over the tokens that reach d;
 * and returns the kd documents of largest S, ties to the lower document id.
 *  Q_d         [B, nq, d] float32 (1 <= nq <= 1024), C_d [K, d] float32 (d = 128);
 *  list_off_d  [K + 1] int64, list_docs_d [list_off_d[K]] int32: the inverted
 *              lists of tac_ivf_build, document ids in [0, D);
 *  cand_d      [B, kd] int32 and score_d [B, kd] float32 (output): documents by
 *              S descending; unused slots hold (-1, -inf).
 * 1 <= kc <= 256, 1 <= kd <= 4096.  Similarities are FP32 products with FP32
 * accumulation on the matrix cores and S adds them in float64 in token order,
 * so repeated calls give identical results.  The workspace holds at most 4 GiB
 * of similarities plus 36 bytes per visited list entry.  Synchronous (the
 * call returns after its work has completed on the context's stream); not for
 * graph capture.  TAC_E_INVAL on bad sizes or NULL pointers; list offsets must
 * be non-decreasing within list_docs_d. */
tac_status tac_gather(tac_ctx ctx, const float* Q_d, int64_t B, int32_t nq, int32_t d, const float* C_d, int64_t K,
                      const int64_t* list_off_d, const int32_t* list_docs_d, int64_t D, int32_t kc, int32_t kd,
                      int32_t* cand_d, float* score_d);

/* Proximity graph over the centroids, the gather's centroid search (Sect.
 * 2.2, "Index Structure": the paper builds an HNSW graph over the centroids,
 * with M = 32 neighbours, Sect. 3).  Row i of nbr_d [K, 64] int32 (output)
 * holds the 32 centroids of largest <c_i, c_j>, j != i (largest first, lower
 * id on ties: exact, from float32 products on the matrix cores), then up to
 * 32 reverse edges: the centroids whose own 32 list i and that i does not
 * list, largest similarity first, lower id on ties; -1 fills the rest.
 * C_d [K, d] float32, d = 128, 2 <= K < 2^31.  Asynchronous.  The workspace
 * holds up to 4 GiB of similarities plus about 260 bytes per centroid. */
tac_status tac_graph_build(tac_ctx ctx, const float* C_d, int64_t K, int32_t d, int32_t* nbr_d);

/* Centroid search on that graph (step 1 of the gather, approximate like the
 * paper's HNSW search): for each of the R query-token rows of Q_d [R, d],
 * the ef router centroids (entry_d [nentry]: distinct centroid ids, e.g. one
 * per token segment) of largest similarity start a beam of ef entries; the
 * best entry not yet expanded is expanded (its listed and reverse neighbours
 * scored once each) until every entry is, and the kc best entries are the
 * result: top_id_d [R, kc] int32 and top_sim_d [R, kc] float32 (output, best
 * first, (-1, -inf) where fewer), similarities being float32 dot products in a
 * fixed order.  1 <= kc <= ef <= 64 (the paper takes ef_s = 1.5 kappa_c).
 * Deterministic; asynchronous.  TAC_E_INVAL on bad sizes or NULL pointers. */
tac_status tac_graph_search(tac_ctx ctx, const float* Q_d, int64_t R, int32_t d, const float* C_d, int64_t K,
                            const int32_t* nbr_d, const int32_t* entry_d, int64_t nentry, int32_t ef, int32_t kc,
                            int32_t* top_id_d, float* top_sim_d);

/* Step 1 of the gather, exact (as tac_gather): top_id_d [R, kc] int32 and
 * top_sim_d [R, kc] float32 (output) hold, per query-token row of Q_d [R, d],
 * the kc centroids of largest <q, c> (float32 matrix-core products; ties to the
 * lower id; (-1, -inf) where K < kc).  1 <= kc <= 256.  Asynchronous; the
 * workspace holds up to 4 GiB of similarities. */
tac_status tac_centroid_topk(tac_ctx ctx, const float* Q_d, int64_t R, int32_t d, const float* C_d, int64_t K,
                             int32_t kc, int32_t* top_id_d, float* top_sim_d);

/* Steps 2-4 of the gather (as tac_gather) for B queries of nq tokens whose
 * top-kc centroid lists are given: top_id_d [B, nq, kc] int32 (-1 for an
 * empty slot, ids < K) with top_sim_d [B, nq, kc] float32, e.g. from
 * tac_graph_search.  Same inverted lists and outputs as tac_gather.
 * Synchronous; not for graph capture. */
tac_status tac_gather_lists(tac_ctx ctx, const int32_t* top_id_d, const float* top_sim_d, int64_t B, int32_t nq,
                            int32_t kc, const int64_t* list_off_d, const int32_t* list_docs_d, int64_t K, int64_t D,
                            int32_t kd, int32_t* cand_d, float* score_d);

/* Refine phase of retrieval (Sect. 2.2, "Refine Phase: PQ-Optimized MaxSim
 * Computation"): the MaxSim score of each candidate document for its query,
 *   S(q, d) = sum_i max_{t in d} <q_i, c_{a_t} + rho_t * u_t>,
 * with u_t the concatenation of the codewords codebooks[m][code_{t,m}] (the
 * decoded normalised residual, Sect. 2.1 "Residuals Compression").
 *  Q_d         [B, nq, d] float32: B queries of nq tokens (1 <= nq <= 32, B <= 65535);
 *  C_d         [K, d] float32 centroids; codebooks_d [M, ksub, d / M] float32
 *              (d = 128, M = 32, 1 <= ksub <= 256);
 *  layout_d    the document layout of tac_doc_layout for the same M (4-byte
 *              aligned), doc_off_d [D + 1] int64 its token offsets (N tokens);
 *  rnorm_d     [N] float32: rho of token t of document d is rnorm_d[doc_off_d[d] + t];
 *  cand_d      [B, nc] int32: the candidate documents of each query (repeats allowed);
 *  scores_d    [B, nc] float32 output, scores_d[b * nc + j] for cand_d[b * nc + j].
 * Tokens whose centroid id is outside [0, K) are skipped; a document with no
 * remaining token scores -inf; a candidate id outside [0, D) scores NaN;
 * offsets outside [0, N] are clamped and codes at or above ksub read codeword
 * ksub - 1, so malformed inputs never address memory outside the buffers.
 * FP32 products and FP32 accumulation on the matrix cores, in a fixed order:
 * repeated calls give identical scores.  The caller owns every buffer; no
 * workspace.  Asynchronous; TAC_E_INVAL on bad sizes, NULL pointers or a
 * misaligned layout. */
tac_status tac_maxsim(tac_ctx ctx, const float* Q_d, int64_t B, int32_t nq, int32_t d, const float* C_d,
                      int64_t K, const float* codebooks_d, int32_t M, int32_t ksub, const uint8_t* layout_d,
                      const int64_t* doc_off_d, int64_t D, int64_t N, const float* rnorm_d,
                      const int32_t* cand_d, int64_t nc, float* scores_d);

#ifdef __cplusplus
}
#endif

#endif /* TAC_H */
