/*
 * cfsim.h - C ABI of the CFG-pair coupled-similarity library (MI355X, gfx950).
 *
 * Method: Lim, Norris & Malony, "A Similarity Measure for GPU Kernel Subgraph
 * Matching" (arXiv 1707.02423).  Two control-flow graphs are compared through
 * their transition-probability matrices (Section 3, Background, "Transition
 * probability") by the IsoRank solution of their Kronecker operator (Table 1,
 * row "Iso"; Section 4.2, Pairwise Comparison), after an optional bilinear
 * resize to a common size (Section 4, Methodology; Section 4.1, Bilinear
 * Interpolation).
 *
 * What every entry point computes, for a pair (A, B) with n_A and n_B nodes:
 *   S_0 = 1/sqrt(n_A n_B) (n_B x n_A, row i = node of B, column j = node of A)
 *   Y_k = B S_k A^T + B^T S_k A,   S_{k+1} = Y_k / ||Y_k||_F
 *   at even k: delta_k = ||S_k - S_{k-2}||_F; stop when delta_k < tol or
 *   k = max_iter; return S_k.  Greedy matching on S (value descending, then
 *   row-major flat index ascending), score = sum of matched entries.
 *   margin = min over the greedy picks (i, j) of 1 - q / S_ij, q the largest
 *   entry of row i or column j that was still free when (i, j) was picked
 *   (+inf if no pick has such a rival; 0 for a pick below the smallest
 *   normal number of the arithmetic type).  Every S here is non-negative,
 *   so rounding errors are relative per entry: when every entry of another
 *   S' differs from S by a relative amount below 0.5 * margin, S' has the
 *   same greedy matching as S.
 *
 * Conventions for every entry point:
 *   - Pointers documented "device" must point to device memory (or memory
 *     the device can access); "host" pointers are read on the host before
 *     the call returns.  The caller owns every buffer; the library allocates
 *     no device memory in these calls (the context owns only cached launch
 *     graphs).
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *     asynchronously; outputs are valid after the stream is synchronised.
 *   - Return values: CFSIM_OK or a negative cfsim_status.  Argument errors
 *     are detected on the host before any HIP call and leave all outputs
 *     untouched; cfsim_last_error() then describes the problem.  Per-pair
 *     conditions are not call errors: they are bits of cfsim_pair_result.status.
 *   - One context per host thread; calls on one context must not overlap.
 */
#ifndef CFSIM_H
#define CFSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CFSIM_OK = 0,
    CFSIM_E_INVALID_ARG = -1,   /* NULL pointer, bad size, bad option value   */
    CFSIM_E_BAD_GRAPH = -2,     /* inconsistent graph description              */
    CFSIM_E_NONFINITE = -3,     /* a jump count is NaN or infinite (host check) */
    CFSIM_E_NEGWEIGHT = -4,     /* a jump count is negative (host check)        */
    CFSIM_E_WORKSPACE = -5,     /* workspace smaller than the *_workspace_size */
    CFSIM_E_UNSUPPORTED = -6,   /* valid request this build does not serve     */
    CFSIM_E_HIP = -7            /* a HIP runtime call failed                   */
} cfsim_status;

/* Arithmetic type of S. */
enum { CFSIM_F64 = 0, CFSIM_F32 = 1 };
/* Scale-to-common-size step (Section 4 and Section 4.1). */
enum { CFSIM_RESIZE_NONE = 0, CFSIM_RESIZE_BILINEAR = 1 };

/* Per-pair status bits (cfsim_pair_result.status). */
#define CFSIM_CONVERGED     1u  /* an even-step delta fell below tol          */
#define CFSIM_HIT_MAX_ITER  2u  /* stopped at max_iter                         */
#define CFSIM_DEGENERATE    4u  /* A or B has no positive weight: S = S_0      */
#define CFSIM_INVALID_INPUT 8u  /* pair skipped (bad index or size over limit) */
#define CFSIM_NEAR_TIE      16u /* margin <= tie_tol: the greedy matching may
                                   change under perturbations of that size  */
#define CFSIM_FP64_FINAL    32u /* an FP32 near-tie pair computed again in FP64
                                   (CFSIM_FLAG_FP64_FINAL); its outputs are
                                   the FP64 results                           */

/* Option flags (cfsim_options.flags). */
#define CFSIM_FLAG_FP64_FINAL 1u /* FP32 calls of cfsim_score / cfsim_score_batch
                                    (no resize): every pair whose FP32 result is
                                    CFSIM_NEAR_TIE is iterated again in FP64 on
                                    the device, and its score, matching, S_out
                                    (rounded to FP32), nu, delta, margin, iters
                                    and status are replaced by the FP64 ones   */

#define CFSIM_FLAG_MFMA_BF16 2u  /* cfsim_score_large, FP32, no resize: the
                                    operator products run as block-sparse
                                    BF16 matrix-core products with FP32
                                    accumulation (32 x 32 blocks of A, B and S
                                    rounded to BF16; Y, norms, the even-step
                                    test and the matching in FP32/FP64).  A
                                    graph with more nonzero 32 x 32 blocks than
                                    twice the largest node count of the set
                                    gives its pair CFSIM_INVALID_INPUT.  The
                                    results are not gated against FP64: their
                                    error is of the order of BF16 rounding
                                    (Table 1 "Iso" with dense padded tiles)   */

/* Pack error bits written by cfsim_pack into *err_flags. */
#define CFSIM_PACK_BAD_INDEX 1  /* a jump endpoint outside [0, n_g): dropped   */
#define CFSIM_PACK_NONFINITE 2  /* a count is NaN or infinite: weight set to 0 */
#define CFSIM_PACK_NEGATIVE  4  /* a count is negative: weight set to 0        */

typedef struct {
    int32_t dtype;      /* CFSIM_F64 or CFSIM_F32                                  */
    int32_t max_iter;   /* K_max >= 1: maximum number of updates                   */
    double tol;         /* stopping threshold on delta (>= 0; 0 = never converge)  */
    int32_t resize;     /* CFSIM_RESIZE_NONE or CFSIM_RESIZE_BILINEAR              */
    uint32_t flags;     /* 0 or CFSIM_FLAG_FP64_FINAL                              */
    double tie_tol;     /* NEAR_TIE threshold on the relative greedy margin (>= 0,
                           finite); 0 selects the default of the arithmetic type:
                           1e-12 for FP64, 2e-5 for FP32 (twice the largest
                           relative per-entry FP32 error measured at 200 updates) */
} cfsim_options;

/* Result of one pair (device memory, 40 bytes). */
typedef struct {
    double score;       /* sum of S over the greedy matching                       */
    double nu;          /* ||Y|| of the last update (tends to the spectral radius) */
    double delta;       /* last even-step ||S_k - S_{k-2}||_F (inf if none)        */
    double margin;      /* relative greedy margin (see above; NaN if skipped)      */
    int32_t iters;      /* number of updates applied (0 if degenerate)             */
    uint32_t status;    /* CFSIM_* status bits                                     */
} cfsim_pair_result;

/*
 * One graph: transition-probability matrix P (P[u][v] = weight of jump u->v)
 * in CSR (successor lists) and CSC (predecessor lists) form.  n, nnz are host
 * values; all arrays are device memory with 0-based local indices.
 *   row_ptr[n+1], col[nnz], w[nnz]   successors of u: col[row_ptr[u]..row_ptr[u+1])
 *   col_ptr[n+1], row[nnz], eid[nnz] predecessors of v: row[col_ptr[v]..], with
 *                                    weight w[eid[t]] (eid = CSR position)
 * cfsim_pack produces this layout; rows are sorted by column, columns by row.
 */
typedef struct {
    int32_t n, nnz;
    const int32_t* row_ptr;
    const int32_t* col;
    const double* w;
    const int32_t* col_ptr;
    const int32_t* row;
    const int32_t* eid;
} cfsim_graph;

/*
 * A packed set of graphs (device arrays; counts are host values).
 * Graph g owns nodes [node_off[g], node_off[g+1]) and edges
 * [edge_off[g], edge_off[g+1]); its row_ptr/col_ptr slices start at
 * node_off[g] + g and hold n_g + 1 local offsets.  max_nodes is an upper
 * bound of every n_g (used to size launches and workspaces).
 */
typedef struct {
    int32_t n_graphs, max_nodes;
    int64_t total_nodes, total_edges;
    const int64_t* node_off;   /* [n_graphs+1] */
    const int64_t* edge_off;   /* [n_graphs+1] */
    const int32_t* row_ptr;    /* [total_nodes + n_graphs] */
    const int32_t* col;        /* [total_edges] */
    const double* w;           /* [total_edges] */
    const int32_t* col_ptr;    /* [total_nodes + n_graphs] */
    const int32_t* row;        /* [total_edges] */
    const int32_t* eid;        /* [total_edges], local CSR position */
} cfsim_graph_set;

typedef struct cfsim_context cfsim_context;

/* Thread-local description of the last error on this thread ("" if none). */
const char* cfsim_last_error(void);
/* Library version string. */
const char* cfsim_version(void);

/* Create a context bound to HIP device `device` (queries its properties). */
cfsim_status cfsim_context_create(cfsim_context** out, int device);
/* Destroy a context and its cached launch graphs (NULL is a no-op). */
void cfsim_context_destroy(cfsim_context* ctx);

/*
 * Host validation of jump lists before a1 (all pointers are host memory):
 * node_off[n_graphs+1], edge_off[n_graphs+1] (non-decreasing, starting at
 * 0), src/dst/count[edge_off[n_graphs]].  Returns CFSIM_E_BAD_GRAPH for
 * offsets that decrease or a graph with no node, or a jump endpoint outside
 * [0, n_g); CFSIM_E_NONFINITE for a NaN or infinite count; CFSIM_E_NEGWEIGHT
 * for a negative count (the first offending jump is named by
 * cfsim_last_error()); CFSIM_OK otherwise.  Makes no HIP call.
 */
cfsim_status cfsim_check_jumps(int32_t n_graphs, const int64_t* node_off, const int64_t* edge_off,
                               const int32_t* src, const int32_t* dst, const double* count);

/*
 * Step a1 - transition probabilities (Section 3, Background, "Transition
 * probability"):
 * build a graph set from jump lists with execution counts.  For graph g the
 * jumps are src/dst/count[edge_off[g] .. edge_off[g+1]) with local node ids;
 * w = count / (sum of counts of the same source); a row with zero total
 * (the STOP node) stays zero.  Repeated jumps stay separate entries.
 * Inputs node_off, edge_off, src, dst, count and outputs row_ptr .. eid,
 * err_flags (one int32, overwritten) are device memory; ws is a device
 * workspace of at least cfsim_pack_workspace_size() bytes.
 */
size_t cfsim_pack_workspace_size(int32_t n_graphs, int64_t total_nodes, int64_t total_edges);
cfsim_status cfsim_pack(cfsim_context* ctx, int32_t n_graphs, int64_t total_nodes, int64_t total_edges,
                        const int64_t* node_off, const int64_t* edge_off,
                        const int32_t* src, const int32_t* dst, const double* count,
                        int32_t* row_ptr, int32_t* col, double* w,
                        int32_t* col_ptr, int32_t* row, int32_t* eid, int32_t* err_flags,
                        void* ws, size_t ws_bytes, void* stream);

/*
 * Steps a2-a7 for one pair (plain path, one launch): S_out (n_B x n_A
 * row-major, opt->dtype; or n_M x n_M, n_M = max(n_A, n_B), when resized),
 * match_out[n_B] (or [n_M]) and res[1] are device memory; S_out and
 * match_out may be NULL.  With opt->resize = CFSIM_RESIZE_BILINEAR
 * (Section 4 and Section 4.1: the smaller transition matrix X becomes
 * R X R^T with the order-1 interpolation R from its m nodes to n_M points
 * at p (m - 1) / (n_M - 1)) a pair of unequal sizes runs in the resized
 * mode of an LDS kernel when one holds it (one launch: the operator in
 * factored form at n_M x m, then S at n_M x n_M), else on the tiled path of
 * cfsim_score_large (a short launch sequence; n_M <= 8192 and max_iter <=
 * 4096); a pair of equal sizes needs no scaling and runs as without resize.
 */
size_t cfsim_score_workspace_size(const cfsim_context* ctx, int32_t n_a, int32_t n_b,
                                  const cfsim_options* opt);
cfsim_status cfsim_score(cfsim_context* ctx, const cfsim_graph* A, const cfsim_graph* B,
                         const cfsim_options* opt, void* S_out, int32_t* match_out,
                         cfsim_pair_result* res, void* ws, size_t ws_bytes, void* stream);

/*
 * cfsim_score without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments (minus ws,
 * ws_bytes), kernels, outputs and per-pair semantics as cfsim_score; the
 * workspace is a static device array of CFSIM_NOALLOC_SCRATCH_BYTES that
 * each GPU holds until the process ends (its address is taken once per
 * device by cfsim_context_create).  The call allocates nothing: a pair whose
 * cfsim_score_workspace_size exceeds CFSIM_NOALLOC_SCRATCH_BYTES (FP64
 * beyond about 1,000 x 1,000 nodes, FP32 beyond about 1,400 x 1,400; less
 * when resized or with CFSIM_FLAG_FP64_FINAL) returns CFSIM_E_UNSUPPORTED
 * before any HIP call.  Every call on one GPU shares that GPU's scratch and
 * leaves it holding its own intermediate data (the kernels initialise
 * everything they read): calls that overlap on one GPU (several streams or
 * host threads) race, so serialise them.
 */
#define CFSIM_NOALLOC_SCRATCH_BYTES (16 << 20)
cfsim_status cfsim_score_noalloc(cfsim_context* ctx, const cfsim_graph* A, const cfsim_graph* B,
                                 const cfsim_options* opt, void* S_out, int32_t* match_out,
                                 cfsim_pair_result* res, void* stream);

/*
 * Steps a2-a8 for many pairs (batched path): pair p compares A = graph
 * pair_a[p] with B = graph pair_b[p] of `set`.  The pairs are planned on the
 * device (size buckets, longest first) and run by persistent workgroups
 * pulling from a device work queue; the launches are captured once into a
 * HIP graph cached in the context and replayed while the arguments repeat.
 * Device buffers: pair_a/pair_b[n_pairs], res[n_pairs]; optional (NULL to
 * skip): match with match_off[n_pairs] (element offset of pair p's n_B
 * entries), S_out with S_off[n_pairs] (element offset of pair p's S).
 * Resized calls (opt->resize = CFSIM_RESIZE_BILINEAR): S and match of pair p
 * have n_M x n_M and n_M entries, n_M = max(n_A, n_B).  The LDS kernels run
 * every pair they hold in a resized mode (the operator in factored form at
 * n_M x min(n_A, n_B), with the larger graph on the rows, expanded to
 * n_M x n_M for the matching); the others run on the tiled path of
 * cfsim_score_large in the same call.
 */
size_t cfsim_batch_workspace_size(const cfsim_context* ctx, const cfsim_graph_set* set,
                                  int64_t n_pairs, const cfsim_options* opt);
cfsim_status cfsim_score_batch(cfsim_context* ctx, const cfsim_graph_set* set,
                               const int32_t* pair_a, const int32_t* pair_b, int64_t n_pairs,
                               const cfsim_options* opt, cfsim_pair_result* res,
                               int32_t* match, const int64_t* match_off,
                               void* S_out, const int64_t* S_off,
                               void* ws, size_t ws_bytes, void* stream);

/*
 * Step a9 - large pairs (the Table 1 "Iso" operator at hundreds to
 * thousands of nodes): same arguments, outputs and per-pair semantics as
 * cfsim_score_batch, for pairs whose lists do not fit the batched kernels
 * (those report CFSIM_INVALID_INPUT there).  The iterates live in the
 * workspace (HBM); every update is one launch over the tiles of all pairs of
 * the call, followed by a per-pair reduction launch; the whole sequence
 * (about 2 * max_iter launches, 3 * max_iter with resize) is captured once
 * into a HIP graph cached in the context.  This tiled path also serves every resized pair (opt->resize =
 * CFSIM_RESIZE_BILINEAR) of cfsim_score and cfsim_score_batch.  Limits:
 * graphs of at most 8192 nodes (set->max_nodes), max_iter at most 4096;
 * otherwise CFSIM_E_UNSUPPORTED.  ws is a device workspace of
 * cfsim_large_workspace_size() bytes, about 4 (6 with resize) * n_pairs *
 * max_nodes^2 elements of opt->dtype.
 */
size_t cfsim_large_workspace_size(const cfsim_context* ctx, const cfsim_graph_set* set,
                                  int64_t n_pairs, const cfsim_options* opt);
cfsim_status cfsim_score_large(cfsim_context* ctx, const cfsim_graph_set* set,
                               const int32_t* pair_a, const int32_t* pair_b, int64_t n_pairs,
                               const cfsim_options* opt, cfsim_pair_result* res,
                               int32_t* match, const int64_t* match_off,
                               void* S_out, const int64_t* S_off,
                               void* ws, size_t ws_bytes, void* stream);

/*
 * Batch schedule and kernel timing (observability of the batched path).
 * Every pair of a batch runs in one of CFSIM_NUM_BUCKETS buckets: 0..4 are
 * the LDS-resident pair kernels in increasing size, 5 the global-memory pair
 * kernel, 6 the pairs no kernel takes (they get CFSIM_INVALID_INPUT; in a
 * resized call, the pairs left to the tiled path).
 *   cfsim_batch_buckets: writes the bucket cfsim_score_batch would give each
 *     pair to bucket[n_pairs] (device int32), on `stream`.  Same argument
 *     rules as cfsim_score_batch; no workspace.
 *   cfsim_bucket_kernel: the name of the kernel serving `bucket` for `dtype`
 *     (static string, as profilers print it without namespace and argument
 *     list); "" for bucket 6 or an out-of-range argument.
 *   cfsim_context_set_timing: with on != 0, later cfsim_score_batch calls
 *     launch without the cached graph and record a HIP event pair on the
 *     caller's stream around each bucket's kernel (the bucket kernels run one
 *     after another on that stream, as in the graph).  on = 0 returns to
 *     graph replays.
 *   cfsim_batch_timings: waits for the last timed call and writes each
 *     bucket kernel's duration in milliseconds to ms[CFSIM_NUM_BUCKETS]
 *     (host).  CFSIM_E_INVALID_ARG if no timed call was made.
 */
#define CFSIM_NUM_BUCKETS 7
cfsim_status cfsim_batch_buckets(cfsim_context* ctx, const cfsim_graph_set* set, const int32_t* pair_a,
                                 const int32_t* pair_b, int64_t n_pairs, const cfsim_options* opt,
                                 int32_t* bucket, void* stream);
const char* cfsim_bucket_kernel(int32_t bucket, int32_t dtype);
cfsim_status cfsim_context_set_timing(cfsim_context* ctx, int32_t on);
cfsim_status cfsim_batch_timings(cfsim_context* ctx, float* ms);

/*
 * Batch plan tuning (step a8).  The batched path runs each pair on the first
 * LDS kernel (bucket 0..4, in increasing size) that holds it.  A tune table
 * of CFSIM_TUNE_CLASSES entries per arithmetic type may send the pairs of a
 * class to a larger LDS kernel; classes group pairs by half octaves of
 * n_A * n_B (cfsim_tune_class; class c holds 2 log2(n_A n_B) in [c, c+1),
 * the last class everything above).  Entry -1 keeps the first kernel that
 * holds the pair; an entry b in 0..4 is used when b is larger than that
 * kernel and b holds the pair.  The table is a host array; it is copied into
 * the context and every later cfsim_score_batch / cfsim_batch_buckets call
 * of that dtype plans with it (a changed table invalidates the cached launch
 * graph).  cfsim_context_set_tune with table NULL restores the default.
 * Tables are produced by the autotuner of the Python package, which times
 * every candidate kernel per class with HIP events and caches the fastest.
 * Errors: CFSIM_E_INVALID_ARG for a NULL context, a bad dtype, n other than
 * CFSIM_TUNE_CLASSES or an entry outside -1..4.
 */
#define CFSIM_TUNE_CLASSES 32
int32_t cfsim_tune_class(int32_t n_a, int32_t n_b);
cfsim_status cfsim_context_set_tune(cfsim_context* ctx, int32_t dtype, const int32_t* table, int32_t n);
cfsim_status cfsim_context_get_tune(const cfsim_context* ctx, int32_t dtype, int32_t* table, int32_t n);

/*
 * Step a10 - reverse mode: d(sum_p grad_score[p] * score_p) / d(w), added to
 * grad_w[total_edges] (device, FP64, CSR order of `set`; not cleared).  The
 * matching and the update count of each pair are held fixed (the
 * almost-everywhere derivative): fwd[p].iters and match (at match_off[p])
 * must come from the forward call with the same set, pairs and options.
 * The reverse walks segments of checkpoint_every updates backwards, each
 * recomputed from its first iterate: S_0, or the forward's checkpoints when
 * ckpt / ckpt_off are given (from cfsim_score_batch_ckpt with the same
 * checkpoint_every; both NULL: the forward is recomputed here first, S stored
 * every checkpoint_every updates).
 * Degenerate pairs contribute zero.  pair_status[n_pairs] (device, may be
 * NULL) receives 0, or CFSIM_INVALID_INPUT for a pair that was skipped (bad
 * ids, or lists too long for the kernel).  Graphs shared between pairs
 * accumulate with FP64 atomics (summation order not fixed).  ws is a device
 * workspace of cfsim_backward_workspace_size() bytes.
 */
size_t cfsim_backward_workspace_size(const cfsim_context* ctx, const cfsim_graph_set* set, int64_t n_pairs,
                                     const cfsim_options* opt, int32_t checkpoint_every);
cfsim_status cfsim_score_backward(cfsim_context* ctx, const cfsim_graph_set* set, const int32_t* pair_a,
                                  const int32_t* pair_b, int64_t n_pairs, const cfsim_options* opt,
                                  const cfsim_pair_result* fwd, const int32_t* match, const int64_t* match_off,
                                  const double* grad_score, double* grad_w, int32_t* pair_status,
                                  int32_t checkpoint_every, const void* ckpt, const int64_t* ckpt_off,
                                  void* ws, size_t ws_bytes, void* stream);

/*
 * cfsim_score_batch that also leaves the forward checkpoints the reverse
 * mode starts its segments from (so cfsim_score_backward need not recompute
 * the forward): pair p's S_k for k = c * checkpoint_every, c = 1, 2, ...,
 * k < the pair's update count, at ckpt + ckpt_off[p] + (c - 1) n_A n_B
 * elements of opt->dtype, n_B x n_A row-major.  The caller sizes pair p's
 * area as (max_iter / checkpoint_every) n_A n_B elements (device memory,
 * owned by the caller; entries past the update count are not written).
 * Pass the same ckpt, ckpt_off and checkpoint_every to cfsim_score_backward.
 * Same arguments and results as cfsim_score_batch otherwise.  Errors as
 * cfsim_score_batch, plus CFSIM_E_INVALID_ARG for checkpoint_every < 1 or a
 * NULL ckpt / ckpt_off, CFSIM_E_UNSUPPORTED with resize or
 * CFSIM_FLAG_FP64_FINAL.
 */
cfsim_status cfsim_score_batch_ckpt(cfsim_context* ctx, const cfsim_graph_set* set,
                                    const int32_t* pair_a, const int32_t* pair_b, int64_t n_pairs,
                                    const cfsim_options* opt, cfsim_pair_result* res,
                                    int32_t* match, const int64_t* match_off,
                                    void* S_out, const int64_t* S_off, void* ckpt, const int64_t* ckpt_off,
                                    int32_t checkpoint_every, void* ws, size_t ws_bytes, void* stream);

/*
 * The damped IsoRank measure of many pairs: Table 1, row "Iso", in its full
 * form (I - alpha Q x P) x = (1 - alpha) E, with IsoRank's normalisation of
 * the product-graph operator (Section 4.2, Pairwise Comparison; Table 1).
 * For pair p (A = graph pair_a[p], B = graph pair_b[p] of `set`):
 *   M = B (x) A + B^T (x) A^T on the row-major vec of X (n_B x n_A), the
 *   operator of the undamped measure; M_hat = M D^-1 with D the column sums
 *   of M, d_uv = c^B_u c^A_v + r^B_u r^A_v (c: column sums, r: row sums of
 *   the transition matrices), a zero column staying zero;
 *   E = the uniform 1/(n_A n_B) (prior = NULL), or pair p's prior
 *   (n_B x n_A row-major FP64 at prior + prior_off[p], device memory,
 *   finite and non-negative with a positive sum) divided by its sum;
 *   x_0 = E, x_k = alpha M_hat x_{k-1} + (1 - alpha) E, stopped at the first
 *   k with delta = ||x_k - x_{k-1}||_1 < opt->tol or at k = opt->max_iter
 *   (the update contracts by alpha in the 1-norm, so ||x_k - x*||_1 <=
 *   alpha delta / (1 - alpha) for the solution x*);
 *   S = x_k / ||x_k||_F; greedy matching, score and margin as for the
 *   undamped measure (see the top of this file).
 * res[p]: score, nu = ||x_k||_F, delta, margin, iters = k, status
 * (CONVERGED or HIT_MAX_ITER, NEAR_TIE, FP64_FINAL; INVALID_INPUT for a bad
 * index, a pair no kernel holds, or a prior that is negative, non-finite or
 * all zero).  0 <= alpha < 1 (alpha = 0 returns the prior).  Same buffers,
 * workspace (cfsim_batch_workspace_size), schedule, kernels' shapes and
 * CFSIM_FLAG_FP64_FINAL pass as cfsim_score_batch, whose pairs the damped
 * kernels take bucket by bucket.  Errors as cfsim_score_batch, plus
 * CFSIM_E_INVALID_ARG for alpha outside [0, 1) or only one of prior /
 * prior_off given, and CFSIM_E_UNSUPPORTED with resize.
 */
cfsim_status cfsim_score_damped(cfsim_context* ctx, const cfsim_graph_set* set, const int32_t* pair_a,
                                const int32_t* pair_b, int64_t n_pairs, const cfsim_options* opt, double alpha,
                                const double* prior, const int64_t* prior_off, cfsim_pair_result* res,
                                int32_t* match, const int64_t* match_off, void* S_out, const int64_t* S_off,
                                void* ws, size_t ws_bytes, void* stream);

/*
 * Step a11 - ranking of a query against a database: the k best scores.
 * scores[i * stride] for i in [0, n) (device; stride 4 reads the score field
 * of a cfsim_pair_result array).  Larger score first, ties to the lower
 * index, NaN (invalid pairs) ranks as -infinity.  idx_out[k] and score_out[k]
 * (device) receive the indices and scores; entries past n get index -1 and
 * score -infinity.  1 <= k <= 1024; ws is a device workspace of
 * cfsim_topk_workspace_size(n, k) bytes.
 */
size_t cfsim_topk_workspace_size(int64_t n, int32_t k);
cfsim_status cfsim_topk(cfsim_context* ctx, const double* scores, int64_t n, int64_t stride, int32_t k,
                        int32_t* idx_out, double* score_out, void* ws, size_t ws_bytes, void* stream);

/*
 * Table 1's elementwise distances of many pairs (Section 4.2, Pairwise
 * Comparison), computed on the pair's two transition matrices once both are
 * at the common size M = max(n_A, n_B) (Section 4 and Section 4.1: the
 * smaller matrix X becomes R X R^T with the order-1 interpolation R of the
 * resize option above; the larger one is kept; equal sizes are compared as
 * they are).  With x and y the two M x M matrices read as vectors, d = x - y:
 *   out[5 q + CFSIM_DIST_EUCLIDEAN] = sqrt(sum d^2)
 *   out[5 q + CFSIM_DIST_MANHATTAN] = sum |d|
 *   out[5 q + CFSIM_DIST_MINKOWSKI] = (sum |d|^p)^(1/p)
 *   out[5 q + CFSIM_DIST_JACCARD]   = sum d^2 / (sum x^2 + sum y^2 - sum x y)
 *                                     (0 when x = y = 0)
 *   out[5 q + CFSIM_DIST_COSINE]    = 1 - sum x y / (||x|| ||y||)
 *                                     (NaN when x or y is 0)
 * All five are symmetric, so which graph of the pair is A does not matter.
 * Pair q compares graphs pair_a[q] and pair_b[q] of `set`; a pair with an
 * index outside [0, n_graphs), or a graph above set->max_nodes, gets five
 * NaN.  Device buffers: pair_a and
 * pair_b [n_pairs], out [5 n_pairs] (FP64), ws of
 * cfsim_distances_workspace_size() bytes.  p is the Minkowski order (the
 * paper gives none; 3 is the usual choice): finite and >= 1, else
 * CFSIM_E_INVALID_ARG.  Sums are FP64; the scaled matrices are never stored
 * (each entry is evaluated from the CSR rows), so set->max_nodes may be up
 * to 32,768.  Results do not depend on the launch shape.
 */
#define CFSIM_NUM_DISTANCES 5
enum {
    CFSIM_DIST_EUCLIDEAN = 0,
    CFSIM_DIST_MANHATTAN = 1,
    CFSIM_DIST_MINKOWSKI = 2,
    CFSIM_DIST_JACCARD = 3,
    CFSIM_DIST_COSINE = 4
};
size_t cfsim_distances_workspace_size(const cfsim_graph_set* set, int64_t n_pairs);
cfsim_status cfsim_distances(cfsim_context* ctx, const cfsim_graph_set* set, const int32_t* pair_a,
                             const int32_t* pair_b, int64_t n_pairs, double p, double* out, void* ws,
                             size_t ws_bytes, void* stream);

/*
 * Optimal-assignment matching of similarity matrices: the other reading of
 * how the IsoRank solution is reduced to matched node pairs (Section 4.2,
 * Pairwise Comparison; the paper fixes no extraction rule).  For matrix q
 * (S of n_rows[q] x n_cols[q], row-major, opt dtype CFSIM_F64 or CFSIM_F32,
 * at S + S_off[q] elements; e.g. the S_out of cfsim_score_batch or
 * cfsim_score_damped with its S_off, n_rows = n_B, n_cols = n_A) it finds
 * the matching of min(n_rows, n_cols) pairs with the largest total sum S_ij
 * (the linear assignment problem) by the Hungarian method with
 * shortest augmenting paths and FP64 potentials; ties take the smallest
 * column index at every step, so the result is deterministic.
 *   match[match_off[q] + i] = column of row i, or -1 (rows beyond the
 *   matching when n_rows > n_cols); score[q] = the matched total (FP64).
 * A matrix with a non-finite entry, or a dimension outside [1, max_dim],
 * gets score NaN and every row -1.  Device buffers: S, S_off, n_rows,
 * n_cols, score [n_pairs]; match and match_off may both be NULL.  max_dim
 * (host) bounds every dimension and sizes the LDS state of a matrix:
 * 1 <= max_dim <= 4096, else CFSIM_E_INVALID_ARG / CFSIM_E_UNSUPPORTED.
 * Work per matrix: O(n^2 m) in the worst case, n = min and m = max of its
 * dimensions.  No workspace.
 */
cfsim_status cfsim_assign(cfsim_context* ctx, int32_t dtype, const void* S, const int64_t* S_off,
                          const int32_t* n_rows, const int32_t* n_cols, int64_t n_pairs, int32_t max_dim,
                          int32_t* match, const int64_t* match_off, double* score, void* stream);

/*
 * Ward's minimum-variance clustering (Section 6.2, Clustering of Kernels):
 * X is n_obs x n_feat row-major FP64 (device), one feature vector per
 * observation (e.g. each graph's row of an all-pairs score or distance
 * matrix).  Initial distances are squared Euclidean, d_ij = ||X_i - X_j||^2
 * (features added in order); each of the n_obs - 1 merges joins the pair of
 * current clusters with the smallest distance (ties: the pair of smaller
 * slots, slot i < j, the merged cluster taking slot i), and distances to
 * the merged cluster follow the Lance-Williams recurrence of Ward's method:
 *   d(k, i u j) = ((n_i + n_k) d_ki + (n_j + n_k) d_kj - n_k d_ij)
 *                 / (n_i + n_j + n_k),
 * so a merge height is twice the increase in within-cluster variance
 * (scipy's Ward heights are its square root).  Z (device, (n_obs - 1) x 4
 * FP64, row-major) receives the usual linkage layout: row s =
 * [id_a, id_b, height, size], id_a < id_b, observations numbered
 * 0..n_obs-1 and the cluster of step s numbered n_obs + s.  A non-finite
 * feature makes every entry of Z NaN.  FP64 arithmetic without fused
 * multiply-adds, in the order above: the result is reproducible bit for bit.
 * ws: device workspace of cfsim_ward_workspace_size(n_obs) bytes (the
 * n_obs x n_obs distances).  1 <= n_obs <= 4096 (more: CFSIM_E_UNSUPPORTED),
 * n_feat >= 1; n_obs = 1 writes nothing.
 */
size_t cfsim_ward_workspace_size(int32_t n_obs);
cfsim_status cfsim_ward(cfsim_context* ctx, const double* X, int32_t n_obs, int32_t n_feat, double* Z, void* ws,
                        size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* CFSIM_H */
