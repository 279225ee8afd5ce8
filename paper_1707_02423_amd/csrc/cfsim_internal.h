// Internal declarations shared by the HIP translation units of libcfsim.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cfsim.h"

namespace cfsim {

constexpr int kWave = 64;

// ---------------------------------------------------------------- graphs
// Device pointers of one graph in the packed layout described in cfsim.h.
struct GraphRef {
    int n, nnz;
    const int32_t* rp;   // [n+1] successor offsets
    const int32_t* ci;   // [nnz] successor ids
    const double* w;     // [nnz] weights (CSR order)
    const int32_t* cp;   // [n+1] predecessor offsets
    const int32_t* ri;   // [nnz] predecessor ids
    const int32_t* eid;  // [nnz] CSR position of each CSC entry
};

struct SetRef {
    const int64_t* node_off;
    const int64_t* edge_off;
    const int32_t* rp;
    const int32_t* ci;
    const double* w;
    const int32_t* cp;
    const int32_t* ri;
    const int32_t* eid;
    int n_graphs;
};

__host__ __device__ inline GraphRef graph_of(const SetRef& s, int g) {
    GraphRef r;
    int64_t n0 = s.node_off[g], n1 = s.node_off[g + 1];
    int64_t e0 = s.edge_off[g], e1 = s.edge_off[g + 1];
    r.n = (int)(n1 - n0);
    r.nnz = (int)(e1 - e0);
    r.rp = s.rp + n0 + g;
    r.cp = s.cp + n0 + g;
    r.ci = s.ci + e0;
    r.w = s.w + e0;
    r.ri = s.ri + e0;
    r.eid = s.eid + e0;
    return r;
}

// ---------------------------------------------------------------- scale to a common size
// The order-1 interpolation matrix R (M x m) of Section 4.1 and G = R^T R,
// used by the tiled path and by the LDS kernels' resized mode.
// Interpolation from m to M points at p (m - 1) / (M - 1): row p of R holds
// 1 - f at column r0 and f at column r1 (one entry 1 when r0 = r1).
struct Interp {
    int r0, r1;
    double f;
};
__host__ __device__ inline Interp interp_at(int p, int m, int M) {
    Interp q;
    if (M <= 1) {
        q.r0 = q.r1 = 0;
        q.f = 0.0;
        return q;
    }
    const long long num = (long long)p * (m - 1);
    q.r0 = (int)(num / (M - 1));
    q.f = (double)(num - (long long)q.r0 * (M - 1)) / (double)(M - 1);
    q.r1 = q.r0 + 1 < m ? q.r0 + 1 : m - 1;
    return q;
}

// First and last p with r0(p) = u.
__host__ __device__ inline void interp_rows(int u, int m, int M, int* plo, int* phi) {
    if (m <= 1) {
        *plo = 0;
        *phi = M - 1;
        return;
    }
    const long long a = (long long)u * (M - 1), b = (long long)(u + 1) * (M - 1);
    *plo = (int)((a + (m - 2)) / (m - 1));
    *phi = u == m - 1 ? M - 1 : (int)((b + (m - 2)) / (m - 1)) - 1;
}

// G = R^T R at column u: diagonal d and the coupling e = G[u][u+1].
__host__ __device__ inline void gram_entries(int u, int m, int M, double* d, double* e) {
    double dd = 0.0, ee = 0.0;
    int lo, hi;
    interp_rows(u, m, M, &lo, &hi);
    for (int p = lo; p <= hi; ++p) {
        const Interp q = interp_at(p, m, M);
        if (q.r1 == q.r0) {
            dd += 1.0;  // (1 - f + f)^2 with a single entry
        } else {
            dd += (1.0 - q.f) * (1.0 - q.f);
            ee += (1.0 - q.f) * q.f;
        }
    }
    if (u > 0) {
        interp_rows(u - 1, m, M, &lo, &hi);
        for (int p = lo; p <= hi; ++p) {
            const Interp q = interp_at(p, m, M);
            if (q.r1 == u && q.r0 != q.r1) dd += q.f * q.f;
        }
    }
    *d = dd;
    *e = ee;
}

// ---------------------------------------------------------------- pair shape
// The kernels store S in a "compute orientation": rows are the nodes of the
// R graph (handled wave-uniformly), columns the nodes of the C graph (one lane
// per column, in 64-column chunks).  R = B, C = A keeps S as n_B x n_A; the
// swapped choice (R = A, C = B) stores S^T.  Wave w owns rows w, w + NW, ...
struct PairShape {
    int swap;    // 1: stored matrix is S^T (rows = A, columns = B)
    int nR, nC;  // stored rows / columns
    int nchunk;  // ceil(nC / 64)
    int rows;    // rows per wave, ceil(nR / NW)
};

// Kernel-variant table of the LDS-resident pair kernel.
struct Variant {
    int nt;         // threads per workgroup
    int nch;        // max 64-column chunks (lane lists held in VGPRs)
    int lds_bytes;  // dynamic LDS per workgroup
};

constexpr int kNumVariants = 5;
// Larger variants serve larger pairs; a pair runs on the first that fits.
__host__ __device__ inline Variant variant_info(int v, int esize) {
    switch (v) {
        case 0: return Variant{64, esize == 8 ? 1 : 2, 16 * 1024};
        case 1: return Variant{256, esize == 8 ? 2 : 4, 40 * 1024};
        case 2: return Variant{512, 2, 78 * 1024};
        case 3: return Variant{1024, 2, 159 * 1024};
        default: return Variant{1024, 4, 159 * 1024};
    }
}

__host__ __device__ inline size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

__host__ __device__ inline PairShape make_shape(int nA, int nB, int swap, int NW) {
    PairShape s;
    s.swap = swap;
    s.nR = swap ? nA : nB;
    s.nC = swap ? nB : nA;
    s.nchunk = (s.nC + 63) / 64;
    s.rows = (s.nR + NW - 1) / NW;
    return s;
}

// Bytes of one inline R-row record (see RowRec in pair.hip).
__host__ __device__ inline size_t rowrec_bytes(int esize) { return esize == 8 ? 80 : 64; }

// Bytes of the staged graph lists of one pair (both kernels keep them in LDS).
// Layout: row records [nR] | row starts int2 [nR] | R succ, pred edges [nnzR]
//         | C columns int4 [nC] | C succ, pred edges [nnzC]
//         | rstate, rbest [nR] | cstate, cbest [nC]
__host__ __device__ inline size_t lds_lists_bytes(int nR, int nC, int nnzR, int nnzC, int esize) {
    const size_t edge = (esize == 8) ? 16 : 8;
    size_t b = align16((size_t)nR * rowrec_bytes(esize)) + align16((size_t)nR * 8);
    b += 2 * align16((size_t)nnzR * edge);
    b += align16((size_t)nC * 16) + 2 * align16((size_t)nnzC * edge);
    b += 2 * align16((size_t)nR * 4);
    b += 2 * align16((size_t)nC * 4);
    return b;
}

// Bytes of dynamic LDS one pair needs in the LDS-resident kernel:
// S_cur, S_next [nR*nC] followed by the lists.
__host__ __device__ inline size_t lds_pair_bytes(const PairShape& s, int nnzR, int nnzC, int esize) {
    return 2 * align16((size_t)s.nR * s.nC * esize) + lds_lists_bytes(s.nR, s.nC, nnzR, nnzC, esize);
}

// The global-memory kernel: one workgroup per pair, S_cur and S_next in a
// workspace slot of `slot_elems` elements each; lists in LDS.
constexpr int kGlobalThreads = 512;
constexpr int kGlobalLds = 78 * 1024;

// Orientation that fills 64-lane chunks better (ties keep S as n_B x n_A).
__host__ __device__ inline int preferred_swap(int nA, int nB) {
    const int cA = (nA + 63) / 64, cB = (nB + 63) / 64;
    return ((long long)nB * cA > (long long)nA * cB) ? 1 : 0;
}

__host__ __device__ inline bool global_fits(int nA, int nB, int nnzA, int nnzB, int esize, long long slot_elems,
                                            PairShape* out) {
    const PairShape s = make_shape(nA, nB, preferred_swap(nA, nB), kGlobalThreads / 64);
    const int nnzR = s.swap ? nnzA : nnzB, nnzC = s.swap ? nnzB : nnzA;
    if ((long long)nA * nB > slot_elems) return false;
    if (lds_lists_bytes(s.nR, s.nC, nnzR, nnzC, esize) > (size_t)kGlobalLds) return false;
    *out = s;
    return true;
}

// Orientation choice: prefer the one that fills 64-lane chunks better; take
// the other if only it fits the variant.  Returns false if neither fits.
__host__ __device__ inline bool choose_shape(int nA, int nB, int nnzA, int nnzB, int variant, int esize,
                                             PairShape* out) {
    const Variant v = variant_info(variant, esize);
    const int NW = v.nt / 64;
    const int pref = preferred_swap(nA, nB);
    for (int k = 0; k < 2; ++k) {
        const int swap = k == 0 ? pref : 1 - pref;
        const PairShape s = make_shape(nA, nB, swap, NW);
        const int nnzR = swap ? nnzA : nnzB;
        const int nnzC = swap ? nnzB : nnzA;
        if (s.nchunk <= v.nch &&
            lds_pair_bytes(s, nnzR, nnzC, esize) <= (size_t)v.lds_bytes) {
            *out = s;
            return true;
        }
    }
    return false;
}

// Resized mode of the LDS kernels (pairs of unequal sizes, M = the larger
// node count, m = the smaller): the iteration keeps U_even, V_a, V_b (M x m
// each) and the lists of the larger graph's rows and the smaller graph's
// columns; the matching then needs S and S^T at M x M and a fresh set of
// matching arrays.  The larger graph always takes the rows.
__host__ __device__ inline size_t resized_iter_bytes(int M, int m, int nnzR, int nnzC, int esize) {
    return 3 * align16((size_t)M * m * esize) + lds_lists_bytes(M, m, nnzR, nnzC, esize);
}
__host__ __device__ inline size_t resized_match_bytes(int M, int esize) {
    return 2 * align16((size_t)M * M * esize) + lds_lists_bytes(M, M, 0, 0, esize);
}
// Resized pairs beyond every LDS variant: one 512-thread workgroup per pair
// with U_even, V_a, V_b (and then S, S^T) in a global-memory slot of
// 3 * align16(slot_elems * esize) bytes, slot_elems = min(max_nodes, 256)^2,
// the lists in LDS; the smaller graph at most two 64-column chunks.
constexpr int kResizedGlobalMax = 256;
__host__ __device__ inline long long resized_slot_elems(int max_nodes) {
    const long long n = max_nodes < kResizedGlobalMax ? max_nodes : kResizedGlobalMax;
    return n * n;
}
__host__ __device__ inline size_t resized_slot_bytes(long long slot_elems, int esize) {
    return 3 * align16((size_t)slot_elems * esize);
}
__host__ __device__ inline bool resized_global_fits(int M, int m, int nnzR, int nnzC, int esize, long long slot_elems) {
    return m <= 2 * 64 && (long long)M * M <= slot_elems &&
           lds_lists_bytes(M, m, nnzR, nnzC, esize) <= (size_t)kGlobalLds &&
           lds_lists_bytes(M, M, 0, 0, esize) <= (size_t)kGlobalLds;
}
__host__ __device__ inline bool resized_fits(int M, int m, int nnzR, int nnzC, int variant, int esize) {
    const Variant v = variant_info(variant, esize);
    if ((m + 63) / 64 > v.nch) return false;
    const size_t it = resized_iter_bytes(M, m, nnzR, nnzC, esize), mt = resized_match_bytes(M, esize);
    return (it > mt ? it : mt) <= (size_t)v.lds_bytes;
}

// ---------------------------------------------------------------- launch descriptors
struct PairJob {
    // pairs: either one explicit pair (single = 1) or pairs of a graph set
    int single;
    GraphRef ga, gb;
    SetRef set;
    const int32_t* pair_a;
    const int32_t* pair_b;
    // schedule: items [bounds[0], bounds[1]) of `order`, pulled through `queue`
    const int32_t* order;
    const int32_t* bounds;
    int32_t* queue;
    // options
    int max_iter;
    double tol;
    double tie_tol;     // NEAR_TIE threshold on the relative greedy margin
    // FP64 pass over the near-tie pairs of an FP32 call: a pair runs only if
    // its FP32 result carries NEAR_TIE; S_out is FP32; status gets FP64_FINAL
    int refine;
    // outputs
    cfsim_pair_result* res;
    int32_t* match;
    const int64_t* match_off;
    void* S_out;
    const int64_t* S_off;
    int variant;
    // Global kernel: gridDim.x slots of S_cur, S_next (2 * slot_elems
    // elements each); unused by the LDS kernels.
    void* gws;
    long long slot_elems;
    // Forward checkpoints for the reverse mode (NULL: none): pair p's S_k for
    // k = c * ckpt_every (c = 1, 2, ...) at ckpt + ckpt_off[p] + (c - 1) n_A n_B,
    // n_B x n_A row-major, in the arithmetic type
    void* ckpt;
    const int64_t* ckpt_off;
    int ckpt_every;
    // Scale to a common size (resize = 1): pairs of unequal sizes run the
    // resized operator in factored form (rows: the larger graph, M nodes;
    // columns: the smaller one, m nodes; see iterate_resized)
    int resize;
    // Damped measure (damped = 1): the fixed point of x = alpha M_hat x +
    // (1 - alpha) E with M_hat the operator with unit column sums and E the
    // prior (NULL: uniform; else pair p's n_B x n_A FP64 prior at
    // prior + prior_off[p], scaled to unit sum on the device)
    int damped;
    double alpha;
    const double* prior;
    const int64_t* prior_off;
};

// Plan: assign every pair a bucket and order each bucket longest first.
// Buckets 0..kNumVariants-1 are the LDS variants, kNumVariants the
// global-memory kernel, kNumVariants+1 the pairs no kernel can take (bad
// graph ids, empty graphs, lists too long for LDS).  Writes order[n_pairs],
// bounds[2*kBuckets] and zeroes queues[kBuckets].
constexpr int kBucketGlobal = kNumVariants;
constexpr int kBucketInvalid = kNumVariants + 1;
constexpr int kBuckets = kNumVariants + 2;
static_assert(kBuckets == CFSIM_NUM_BUCKETS, "bucket count of the C ABI");
// Tune classes of the batch plan: pairs grouped by 2 log2(n_A n_B) (half
// octaves of S's entry count); a tuned table may send a class to a larger
// LDS variant than the first one that holds it.
constexpr int kTuneClasses = CFSIM_TUNE_CLASSES;
__host__ __device__ inline int tune_class(int nA, int nB) {
    const double a = (double)(nA > 1 ? nA : 1) * (double)(nB > 1 ? nB : 1);
    int c = (int)(2.0 * log2(a));
    return c < 0 ? 0 : (c >= kTuneClasses ? kTuneClasses - 1 : c);
}

struct PlanJob {
    SetRef set;
    const int32_t* pair_a;
    const int32_t* pair_b;
    int64_t n_pairs;
    // if set: only pairs whose result here carries NEAR_TIE (and not
    // INVALID_INPUT) are planned; the others are left out of every bucket
    const cfsim_pair_result* filter;
    int esize;
    long long slot_elems;
    int32_t* order;
    int32_t* bounds;
    int32_t* queues;
    // LDS variant per tune class (-1: the first variant that holds the pair)
    int8_t tune[kTuneClasses];
    // resized mode: pairs of unequal sizes are planned on their resized LDS
    // footprint; pairs no LDS kernel holds are left to the tiled path
    int resize;
};

// Host-side launchers (return hipError_t as int).
// variant in [0, kNumVariants): LDS kernel; kBucketGlobal: global-memory
// kernel; kBucketInvalid: marks the bucket's pairs invalid.
int launch_pair_lds(int variant, int dtype, const PairJob& job, int grid, hipStream_t stream);
int launch_plan(const PlanJob& job, hipStream_t stream);
int launch_buckets(const PlanJob& job, int32_t* bucket, hipStream_t stream);  // bucket of every pair
const char* bucket_kernel_name(int bucket, int dtype);
int set_kernel_attributes();
int occupancy_of(int variant, int dtype, int* blocks);  // variant may be kBucketGlobal

struct PackJob {
    int n_graphs;
    const int64_t* node_off;
    const int64_t* edge_off;
    const int32_t* src;
    const int32_t* dst;
    const double* count;
    int32_t* rp;
    int32_t* ci;
    double* w;
    int32_t* cp;
    int32_t* ri;
    int32_t* eid;
    int32_t* err;
    int32_t* cursor;   // [total_nodes] workspace
    int32_t* eorig;    // [total_edges] workspace
    int32_t* csrpos;   // [total_edges] workspace
};
int launch_pack(const PackJob& job, hipStream_t stream);

// Large pairs (large.hip): per-pair state and the launch descriptor.
struct LargeState {
    int nA, nB;
    int rz;              // scaled to a common size (resize requested and n_A != n_B)
    int swap;            // state rows are A's nodes (rows = B's otherwise)
    int nR, nC;          // state shape: n_B x n_A, or M x m when resized
    int M;               // common size when resized
    int ntiles;          // tiles of the state (128 rows x 64 columns)
    int active;          // still iterating
    unsigned status;     // CFSIM_* bits once decided
    int final_step;      // k of the returned iterate
    double nu, delta;    // reported norm and last even-step change
    double nu_k[4];      // nu_k of the iterate held in buffer k % 4 (1 for S_0)
};

struct LargeJob {
    // if set: only pairs whose result here carries CFSIM_INVALID_INPUT run
    // (the rest were scored by the LDS kernels and keep their results)
    const cfsim_pair_result* filter;
    int single;          // one explicit pair (ga, gb) instead of pairs of a set
    GraphRef ga, gb;
    SetRef set;
    const int32_t* pair_a;
    const int32_t* pair_b;
    int n_pairs;
    int max_nodes;
    int max_iter;
    double tol;
    double tie_tol;      // NEAR_TIE threshold on the relative greedy margin
    int resize;          // CFSIM_RESIZE_BILINEAR
    cfsim_pair_result* res;
    int32_t* match;
    const int64_t* match_off;
    void* S_out;
    const int64_t* S_off;
    // workspace
    LargeState* st;      // [n_pairs]
    long long* tile_off; // [n_pairs + 1]
    int* tile_pair;      // [tiles] pair of each tile
    double* part_nu;     // [tiles] squared-norm partials of Y
    double* part_delta;  // [tiles] squared partials of S_{k-1} - S_{k-3}
    void* bufs;          // [n_pairs][nslots][slot_elems]: 4 rotating iterates (+ V, S when resized)
    int nslots;
    long long slot_elems;
    void* recs;          // [n_pairs][2][max_nodes] node records: rows of the row graph, columns of the column graph
    // BF16 MFMA tile products (CFSIM_FLAG_MFMA_BF16; plain FP32 pairs only)
    int mfma;
    int mf_nb, mf_cap;   // 32-node blocks per side of the largest graph; stored blocks per graph
    long long mf_idx_stride;
    int* mf_idx;         // [n_pairs][2][mf_idx_stride] block lists of the row graph (0) and column graph (1)
    uint4* mf_tiles;     // [n_pairs][2][mf_cap][2][128] nonzero 32 x 32 blocks, row-major and transposed
    uint4* mf_blocks;    // [n_pairs][3][mf_nb^2][128] Y_{k-1}, T1^T, T2^T as BF16 blocks
};

constexpr int kLargeMaxNodes = 8192;  // bound of the finish kernel's LDS matching state
constexpr int kMfmaMaxBlocks = kLargeMaxNodes / 32;  // 32-node blocks of the largest graph
// Stored 32 x 32 blocks per graph on the MFMA variant: all of them, at most
// twice the node count (a graph of out-degree <= 2 never has more).
__host__ __device__ inline int mfma_block_cap(int max_nodes) {
    const long long nb = (max_nodes + 31) / 32;
    const long long all = nb * nb, two_n = 2ll * max_nodes;
    return (int)(all < two_n ? all : two_n);
}
__host__ __device__ inline long long mfma_idx_stride(int max_nodes) {
    return 2ll * ((max_nodes + 31) / 32 + 1) + 3ll * mfma_block_cap(max_nodes);
}
int launch_mfma_prep(const LargeJob& job, hipStream_t stream);
int launch_mfma_update(const LargeJob& job, int k, int grid, hipStream_t stream);
// Bytes of one node record of the tiled path (first 2 successors, 3 predecessors).
__host__ __device__ inline size_t large_rec_bytes(int esize) { return esize == 8 ? 80 : 48; }
__host__ __device__ inline long long large_tiles(int n) { return (long long)((n + 127) / 128) * ((n + 63) / 64); }
int large_step_grid(int num_cus);
int set_large_attributes();
int launch_large(int dtype, const LargeJob& job, int grid, hipStream_t stream);

// Adjoint (adjoint.hip).
long long backward_slot_bytes(int max_iter, int ckpt, long long slot_elems, int esize);
int backward_grid(int num_cus);
int launch_backward(int dtype, const SetRef& set, const int32_t* pair_a, const int32_t* pair_b, int n_pairs,
                    const cfsim_pair_result* fwd, const int32_t* match, const int64_t* match_off,
                    const double* grad_score, double* grad_w, int32_t* pair_status, int ckpt,
                    const void* fck, const int64_t* fck_off, int max_iter,
                    void* ws, long long slot_elems, int grid, hipStream_t stream);

// Top-k (topk.hip).
long long topk_blocks(long long n);
int topk_max_k();
size_t topk_stage2_lds(long long n, int k);
int launch_topk(const double* scores, long long n, long long stride, int k, int32_t* idx_out, double* score_out,
                void* ws, hipStream_t stream);

// Elementwise distances (distances.hip).  A pair of common size M is cut into
// row chunks of dist_rows(M) rows: about kDistEntries entries per chunk, at
// most kDistMaxTasks chunks per pair.
constexpr int kDistEntries = 2048;
constexpr int kDistMaxTasks = 64;
constexpr int kDistSums = 6;
__host__ __device__ inline int dist_rows(int M) {
    int r = (M + kDistMaxTasks - 1) / kDistMaxTasks;
    const int by_entries = kDistEntries / M;
    if (by_entries > r) r = by_entries;
    if (r < 1) r = 1;
    return r < M ? r : M;
}
__host__ __device__ inline int dist_tasks(int M) {
    const int r = dist_rows(M);
    return (M + r - 1) / r;
}
long long dist_tasks_bound(int max_nodes);
int dist_grid(int num_cus);
int launch_distances(const SetRef& set, int max_nodes, const int32_t* pa, const int32_t* pb, int n_pairs, double p,
                     double* out, int64_t* task_off, double* part, int grid, hipStream_t stream);

// Optimal-assignment matching (assign.hip): LDS bytes of one workgroup for
// matrices of at most max_dim rows and columns.
constexpr int kAssignMaxDim = 4096;
size_t assign_lds_bytes(int max_dim);
int launch_assign(int dtype, const void* S, const int64_t* S_off, const int32_t* n_rows, const int32_t* n_cols,
                  int n_pairs, int max_dim, int32_t* match, const int64_t* match_off, double* score, int grid,
                  hipStream_t stream);

// Ward's clustering (ward.hip): distances into D (n x n FP64), then the merges.
constexpr int kWardMaxObs = 4096;
int launch_ward(const double* X, int n, int f, double* Z, double* D, hipStream_t stream);

}  // namespace cfsim
