// Host side of the C ABI declared in include/cfsim.h: argument validation
// (always before any HIP call), the context, workspace carving, the batch
// plan / persistent launches, and the HIP-graph cache of the batched path.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "cfsim_internal.h"

// Device scratch of cfsim_score_noalloc: the workspace of cfsim_score, held
// by every GPU the library runs on until the process ends.  In host code
// `scratch` only names the symbol; its device address comes from
// hipGetSymbolAddress (once per device, at context creation) and only that
// address is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[CFSIM_NOALLOC_SCRATCH_BYTES];

struct cfsim_context {
    int device = 0;
    int num_cus = 0;
    int grid[2][cfsim::kBucketGlobal + 1] = {};  // persistent grid per [dtype][LDS variant | global]
    hipStream_t cap = nullptr;              // capture stream of the cached graphs
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<unsigned char> key;         // arguments the cached graph was built for
    hipGraph_t large_graph = nullptr;       // cached graph of the large-pair sequence
    hipGraphExec_t large_exec = nullptr;
    std::vector<unsigned char> large_key;
    int timing = 0;                         // eager launches with per-bucket event pairs
    int timed = 0;                          // a timed call has been enqueued
    hipEvent_t t0[cfsim::kBuckets] = {};
    hipEvent_t t1[cfsim::kBuckets] = {};
    void* scratch = nullptr;                // this device's copy of `scratch`
    int8_t tune[2][cfsim::kTuneClasses];    // batch plan: LDS variant per tune class, [F64, F32]
};

namespace {

thread_local std::string g_err;

// Device address of `scratch` per device, taken once per device.
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxScratchDevices] = {};

// With `device` current: its address of `scratch` (NULL for device ids past
// the table).  Returns a HIP error code.
int scratch_address(int device, void** out) {
    *out = nullptr;
    if (device >= kMaxScratchDevices) return 0;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        const int e = (int)hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != 0) return e;
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return 0;
}

cfsim_status fail(cfsim_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

cfsim_status ok() {
    g_err.clear();
    return CFSIM_OK;
}

cfsim_status hip_fail(int e, const char* what) {
    return fail(CFSIM_E_HIP, "%s: %s", what, hipGetErrorString((hipError_t)e));
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

cfsim_status check_options(const cfsim_options* o) {
    if (!o) return fail(CFSIM_E_INVALID_ARG, "options pointer is NULL");
    if (o->dtype != CFSIM_F64 && o->dtype != CFSIM_F32)
        return fail(CFSIM_E_INVALID_ARG, "dtype must be CFSIM_F64 or CFSIM_F32 (got %d)", o->dtype);
    if (o->max_iter < 1) return fail(CFSIM_E_INVALID_ARG, "max_iter must be >= 1 (got %d)", o->max_iter);
    if (!(o->tol >= 0.0) || !std::isfinite(o->tol))
        return fail(CFSIM_E_INVALID_ARG, "tol must be finite and >= 0");
    if (o->resize != CFSIM_RESIZE_NONE && o->resize != CFSIM_RESIZE_BILINEAR)
        return fail(CFSIM_E_INVALID_ARG, "resize must be CFSIM_RESIZE_NONE or CFSIM_RESIZE_BILINEAR");
    const uint32_t known = CFSIM_FLAG_FP64_FINAL | CFSIM_FLAG_MFMA_BF16;
    if ((o->flags & ~known) != 0) return fail(CFSIM_E_INVALID_ARG, "flags: unknown bits %#x", o->flags & ~known);
    if ((o->flags & CFSIM_FLAG_FP64_FINAL) && o->dtype != CFSIM_F32)
        return fail(CFSIM_E_INVALID_ARG, "CFSIM_FLAG_FP64_FINAL applies to FP32 calls only");
    if ((o->flags & CFSIM_FLAG_MFMA_BF16) && (o->dtype != CFSIM_F32 || o->resize != CFSIM_RESIZE_NONE))
        return fail(CFSIM_E_INVALID_ARG, "CFSIM_FLAG_MFMA_BF16 applies to FP32 calls without resize only");
    if ((o->flags & CFSIM_FLAG_MFMA_BF16) && (o->flags & CFSIM_FLAG_FP64_FINAL))
        return fail(CFSIM_E_INVALID_ARG, "CFSIM_FLAG_MFMA_BF16 and CFSIM_FLAG_FP64_FINAL exclude each other");
    if (!(o->tie_tol >= 0.0) || !std::isfinite(o->tie_tol))
        return fail(CFSIM_E_INVALID_ARG, "tie_tol must be finite and >= 0");
    return CFSIM_OK;
}

// NEAR_TIE threshold of a call in arithmetic type `dtype`: the option, or
// the type's default (twice the largest relative per-entry error against
// FP64 measured on the all-pairs workload for FP32; the C9-style floor for
// FP64).
double tie_tol_of(const cfsim_options* o, int dtype) {
    if (o->tie_tol > 0.0 && dtype == o->dtype) return o->tie_tol;
    return dtype == CFSIM_F64 ? 1e-12 : 2e-5;
}

bool fp64_final(const cfsim_options* o) { return (o->flags & CFSIM_FLAG_FP64_FINAL) != 0; }
bool mfma_bf16(const cfsim_options* o) { return (o->flags & CFSIM_FLAG_MFMA_BF16) != 0; }

// The BF16 matrix-core variant is an option of cfsim_score_large only.
cfsim_status check_no_mfma(const cfsim_options* o) {
    if (mfma_bf16(o)) return fail(CFSIM_E_UNSUPPORTED, "CFSIM_FLAG_MFMA_BF16 applies to cfsim_score_large only");
    return CFSIM_OK;
}

// The tiled path (large pairs, resize) has no FP64 pass.
cfsim_status check_no_fp64_final(const cfsim_options* o) {
    if (fp64_final(o)) return fail(CFSIM_E_UNSUPPORTED, "CFSIM_FLAG_FP64_FINAL on the tiled path (large pairs, resize)");
    return CFSIM_OK;
}

cfsim_status check_graph(const cfsim_graph* g, const char* name) {
    if (!g) return fail(CFSIM_E_INVALID_ARG, "graph %s is NULL", name);
    if (g->n < 1) return fail(CFSIM_E_BAD_GRAPH, "graph %s: n must be >= 1 (got %d)", name, g->n);
    if (g->nnz < 0) return fail(CFSIM_E_BAD_GRAPH, "graph %s: nnz must be >= 0", name);
    if (!g->row_ptr || !g->col_ptr) return fail(CFSIM_E_INVALID_ARG, "graph %s: row_ptr/col_ptr is NULL", name);
    if (g->nnz > 0 && (!g->col || !g->w || !g->row || !g->eid))
        return fail(CFSIM_E_INVALID_ARG, "graph %s: an edge array is NULL", name);
    return CFSIM_OK;
}

cfsim_status check_set(const cfsim_graph_set* s) {
    if (!s) return fail(CFSIM_E_INVALID_ARG, "graph set is NULL");
    if (s->n_graphs < 1) return fail(CFSIM_E_BAD_GRAPH, "graph set: n_graphs must be >= 1");
    if (s->max_nodes < 1) return fail(CFSIM_E_BAD_GRAPH, "graph set: max_nodes must be >= 1");
    if (s->total_nodes < s->n_graphs || s->total_edges < 0)
        return fail(CFSIM_E_BAD_GRAPH, "graph set: bad total_nodes/total_edges");
    if (!s->node_off || !s->edge_off || !s->row_ptr || !s->col_ptr)
        return fail(CFSIM_E_INVALID_ARG, "graph set: an offset array is NULL");
    if (s->total_edges > 0 && (!s->col || !s->w || !s->row || !s->eid))
        return fail(CFSIM_E_INVALID_ARG, "graph set: an edge array is NULL");
    return CFSIM_OK;
}

cfsim::GraphRef ref_of(const cfsim_graph* g) {
    cfsim::GraphRef r;
    r.n = g->n;
    r.nnz = g->nnz;
    r.rp = g->row_ptr;
    r.ci = g->col;
    r.w = g->w;
    r.cp = g->col_ptr;
    r.ri = g->row;
    r.eid = g->eid;
    return r;
}

cfsim::SetRef ref_of(const cfsim_graph_set* s) {
    cfsim::SetRef r;
    r.node_off = s->node_off;
    r.edge_off = s->edge_off;
    r.rp = s->row_ptr;
    r.ci = s->col;
    r.w = s->w;
    r.cp = s->col_ptr;
    r.ri = s->row;
    r.eid = s->eid;
    r.n_graphs = s->n_graphs;
    return r;
}

int dtype_index(int dtype) { return dtype == CFSIM_F64 ? 0 : 1; }
int esize_of(int dtype) { return dtype == CFSIM_F64 ? 8 : 4; }

// Workgroups per CU the LDS budget of a kernel allows (an upper bound of the
// persistent grid, used to size workspaces before a context exists).
int lds_blocks_per_cu(int v, int esize) {
    const int lds = v == cfsim::kBucketGlobal ? cfsim::kGlobalLds : cfsim::variant_info(v, esize).lds_bytes;
    const int nt = v == cfsim::kBucketGlobal ? cfsim::kGlobalThreads : cfsim::variant_info(v, esize).nt;
    const int by_lds = (160 * 1024) / (lds + 1024);
    const int by_waves = (4 * 4) / (nt / 64 > 0 ? nt / 64 : 1);  // 4 waves per SIMD
    const int b = by_lds < by_waves ? by_lds : by_waves;
    return b > 0 ? b : 1;
}

int num_cus_of(const cfsim_context* ctx) { return ctx && ctx->num_cus > 0 ? ctx->num_cus : 256; }

// Elements of one global-kernel slot (each of the two iterate buffers).
long long global_slot_elems(int max_nodes) { return (long long)max_nodes * (long long)max_nodes; }

// Batch workspace: order[n_pairs] | bounds[2*kBuckets] | queues[kBuckets]
//   | global kernel: grid slots of 2 * global_slot_elems (the LDS variants
//     keep both iterates in LDS and need no slots)
struct BatchWs {
    int32_t* order;
    int32_t* bounds;
    int32_t* queues;
    void* slots[cfsim::kBucketGlobal + 1];
};
size_t slot_bytes(const cfsim_context* ctx, int v, int esize, int max_nodes) {
    const size_t wgs = (size_t)num_cus_of(ctx) * (size_t)lds_blocks_per_cu(v, esize);
    if (v == cfsim::kBucketGlobal) return align256(wgs * 2 * (size_t)global_slot_elems(max_nodes) * esize);
    return 0;
}
// esize: the largest arithmetic type of the call (8 with the FP64 pass).
size_t batch_ws_bytes(const cfsim_context* ctx, int64_t n_pairs, int esize, int max_nodes) {
    size_t b = align256((size_t)n_pairs * 4) + align256(2 * cfsim::kBuckets * 4) + align256(cfsim::kBuckets * 4);
    for (int v = 0; v <= cfsim::kBucketGlobal; ++v) b += slot_bytes(ctx, v, esize, max_nodes);
    return b;
}
// Global-memory slots of the resized mode's global kernel (one per workgroup).
size_t resized_slots_bytes(const cfsim_context* ctx, int esize, int max_nodes) {
    const size_t wgs = (size_t)num_cus_of(ctx) * (size_t)lds_blocks_per_cu(cfsim::kBucketGlobal, esize);
    return align256(wgs * cfsim::resized_slot_bytes(cfsim::resized_slot_elems(max_nodes), esize));
}
// The schedule part of the batch workspace alone (order, bounds, queues).
size_t sched_ws_bytes(int64_t n_pairs) {
    return align256((size_t)n_pairs * 4) + align256(2 * cfsim::kBuckets * 4) + align256(cfsim::kBuckets * 4);
}
BatchWs carve_sched(void* ws, int64_t n_pairs) {
    unsigned char* p = static_cast<unsigned char*>(ws);
    BatchWs b;
    b.order = reinterpret_cast<int32_t*>(p);
    p += align256((size_t)n_pairs * 4);
    b.bounds = reinterpret_cast<int32_t*>(p);
    p += align256(2 * cfsim::kBuckets * 4);
    b.queues = reinterpret_cast<int32_t*>(p);
    for (int v = 0; v <= cfsim::kBucketGlobal; ++v) b.slots[v] = nullptr;
    return b;
}
BatchWs carve_batch(const cfsim_context* ctx, void* ws, int64_t n_pairs, int esize, int max_nodes) {
    unsigned char* p = static_cast<unsigned char*>(ws);
    BatchWs b;
    b.order = reinterpret_cast<int32_t*>(p);
    p += align256((size_t)n_pairs * 4);
    b.bounds = reinterpret_cast<int32_t*>(p);
    p += align256(2 * cfsim::kBuckets * 4);
    b.queues = reinterpret_cast<int32_t*>(p);
    p += align256(cfsim::kBuckets * 4);
    for (int v = 0; v <= cfsim::kBucketGlobal; ++v) {
        b.slots[v] = p;
        p += slot_bytes(ctx, v, esize, max_nodes);
    }
    return b;
}

template <typename X>
void append_key(std::vector<unsigned char>& k, const X& x) {
    const unsigned char* p = reinterpret_cast<const unsigned char*>(&x);
    k.insert(k.end(), p, p + sizeof(X));
}

// Large-pair (tiled) workspace: state[n_pairs] | tile_off[n_pairs + 1]
//   | part_nu, part_delta, tile_pair [n_pairs * large_tiles(max_nodes)]
//   | node records [n_pairs][2][max_nodes]
//   | nslots iterate slots of max_nodes^2 per pair (4, or 6 when resized)
int large_nslots(const cfsim_options* o) { return o->resize == CFSIM_RESIZE_BILINEAR ? 6 : 4; }

size_t large_ws_bytes(int64_t n_pairs, int max_nodes, int esize, int nslots) {
    const size_t tiles = (size_t)n_pairs * (size_t)cfsim::large_tiles(max_nodes);
    return align256((size_t)n_pairs * sizeof(cfsim::LargeState)) + align256((size_t)(n_pairs + 1) * 8) +
           2 * align256(tiles * 8) + align256(tiles * 4) +
           align256((size_t)n_pairs * 2 * max_nodes * cfsim::large_rec_bytes(esize)) +
           align256((size_t)n_pairs * nslots * (size_t)global_slot_elems(max_nodes) * (size_t)esize);
}

// MFMA variant, after the tiled-path workspace: block lists [n_pairs][2][idx
// stride] | stored blocks [n_pairs][2][cap][2] | BF16 blocks [n_pairs][3][nb^2]
// (2 KiB per 32 x 32 block).
size_t mfma_ws_bytes(int64_t n_pairs, int max_nodes) {
    const size_t nb = (size_t)(max_nodes + 31) / 32;
    return align256((size_t)n_pairs * 2 * (size_t)cfsim::mfma_idx_stride(max_nodes) * 4) +
           align256((size_t)n_pairs * 2 * (size_t)cfsim::mfma_block_cap(max_nodes) * 2 * 2048) +
           align256((size_t)n_pairs * 3 * nb * nb * 2048);
}

// Options, outputs and workspace of a tiled-path launch (pairs filled by the caller).
cfsim::LargeJob large_job(const cfsim_options* opt, int64_t n_pairs, int max_nodes, cfsim_pair_result* res,
                          int32_t* match, const int64_t* match_off, void* S_out, const int64_t* S_off, void* ws) {
    cfsim::LargeJob J{};
    J.n_pairs = (int)n_pairs;
    J.max_nodes = max_nodes;
    J.max_iter = opt->max_iter;
    J.tol = opt->tol;
    J.tie_tol = tie_tol_of(opt, opt->dtype);
    J.resize = opt->resize == CFSIM_RESIZE_BILINEAR;
    J.res = res;
    J.match = match;
    J.match_off = match_off;
    J.S_out = S_out;
    J.S_off = S_off;
    unsigned char* p = static_cast<unsigned char*>(ws);
    const size_t tiles = (size_t)n_pairs * (size_t)cfsim::large_tiles(max_nodes);
    J.st = reinterpret_cast<cfsim::LargeState*>(p);
    p += align256((size_t)n_pairs * sizeof(cfsim::LargeState));
    J.tile_off = reinterpret_cast<long long*>(p);
    p += align256((size_t)(n_pairs + 1) * 8);
    J.part_nu = reinterpret_cast<double*>(p);
    p += align256(tiles * 8);
    J.part_delta = reinterpret_cast<double*>(p);
    p += align256(tiles * 8);
    J.tile_pair = reinterpret_cast<int*>(p);
    p += align256(tiles * 4);
    J.recs = p;
    p += align256((size_t)n_pairs * 2 * max_nodes * cfsim::large_rec_bytes(esize_of(opt->dtype)));
    J.bufs = p;
    J.nslots = large_nslots(opt);
    J.slot_elems = global_slot_elems(max_nodes);
    p += align256((size_t)n_pairs * J.nslots * (size_t)J.slot_elems * (size_t)esize_of(opt->dtype));
    if (mfma_bf16(opt)) {
        const size_t nb = (size_t)(max_nodes + 31) / 32;
        J.mfma = 1;
        J.mf_nb = (int)nb;
        J.mf_cap = cfsim::mfma_block_cap(max_nodes);
        J.mf_idx_stride = cfsim::mfma_idx_stride(max_nodes);
        J.mf_idx = reinterpret_cast<int*>(p);
        p += align256((size_t)n_pairs * 2 * (size_t)J.mf_idx_stride * 4);
        J.mf_tiles = reinterpret_cast<uint4*>(p);
        p += align256((size_t)n_pairs * 2 * (size_t)J.mf_cap * 2 * 2048);
        J.mf_blocks = reinterpret_cast<uint4*>(p);
    }
    return J;
}

// Replays the graph cached in (graph, exec, cached_key) when `key` matches,
// else captures `enqueue` on the context's capture stream first.
template <typename F>
cfsim_status replay_or_capture(cfsim_context* ctx, hipGraph_t* graph, hipGraphExec_t* exec,
                               std::vector<unsigned char>* cached_key, const std::vector<unsigned char>& key,
                               hipStream_t st, F enqueue) {
    int e;
    if (!*exec || key != *cached_key) {
        if (*exec) {
            (void)hipGraphExecDestroy(*exec);
            *exec = nullptr;
        }
        if (*graph) {
            (void)hipGraphDestroy(*graph);
            *graph = nullptr;
        }
        cached_key->clear();
        if ((e = (int)hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal)) != 0)
            return hip_fail(e, "hipStreamBeginCapture");
        const int le = enqueue(ctx->cap);
        hipGraph_t g = nullptr;
        e = (int)hipStreamEndCapture(ctx->cap, &g);
        if (le != 0) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(le, "launch during capture");
        }
        if (e != 0) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t x = nullptr;
        if ((e = (int)hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != 0) {
            (void)hipGraphDestroy(g);
            return hip_fail(e, "hipGraphInstantiate");
        }
        *graph = g;
        *exec = x;
        *cached_key = key;
    }
    if ((e = (int)hipGraphLaunch(*exec, st)) != 0) return hip_fail(e, "hipGraphLaunch");
    return ok();
}

bool graphs_disabled() {
    const char* nog = getenv("CFSIM_NO_GRAPH");
    return nog && nog[0] == '1';
}

std::vector<unsigned char> set_call_key(const cfsim_context* ctx, const cfsim_graph_set* set,
                                        const int32_t* pair_a, const int32_t* pair_b,
                                        int64_t n_pairs, const cfsim_options* opt, cfsim_pair_result* res,
                                        int32_t* match, const int64_t* match_off, void* S_out,
                                        const int64_t* S_off, void* ws) {
    std::vector<unsigned char> key;
    append_key(key, ctx->tune);
    append_key(key, *set);
    append_key(key, pair_a);
    append_key(key, pair_b);
    append_key(key, n_pairs);
    append_key(key, *opt);
    append_key(key, res);
    append_key(key, match);
    append_key(key, match_off);
    append_key(key, S_out);
    append_key(key, S_off);
    append_key(key, ws);
    return key;
}

// Limits of the tiled path (LDS of its matching state, graph length).
cfsim_status check_large_limits(int max_nodes, const cfsim_options* opt) {
    if (max_nodes > cfsim::kLargeMaxNodes)
        return fail(CFSIM_E_UNSUPPORTED, "graphs above %d nodes on the tiled path (large pairs, resize)",
                    cfsim::kLargeMaxNodes);
    if (opt->max_iter > 4096) return fail(CFSIM_E_UNSUPPORTED, "max_iter above 4096 on the tiled path");
    return CFSIM_OK;
}

}  // namespace

extern "C" {

const char* cfsim_last_error(void) { return g_err.c_str(); }

const char* cfsim_version(void) { return "cfsim 0.1.0 gfx950"; }

cfsim_status cfsim_context_create(cfsim_context** out, int device) {
    if (!out) return fail(CFSIM_E_INVALID_ARG, "out pointer is NULL");
    *out = nullptr;
    int count = 0;
    int e = (int)hipGetDeviceCount(&count);
    if (e != 0) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return fail(CFSIM_E_INVALID_ARG, "device %d out of range [0,%d)", device, count);
    if ((e = (int)hipSetDevice(device)) != 0) return hip_fail(e, "hipSetDevice");
    cfsim_context* ctx = new cfsim_context();
    ctx->device = device;
    memset(ctx->tune, -1, sizeof(ctx->tune));
    if ((e = (int)hipDeviceGetAttribute(&ctx->num_cus, hipDeviceAttributeMultiprocessorCount, device)) != 0) {
        delete ctx;
        return hip_fail(e, "hipDeviceGetAttribute");
    }
    if ((e = cfsim::set_kernel_attributes()) != 0 || (e = cfsim::set_large_attributes()) != 0) {
        delete ctx;
        return hip_fail(e, "hipFuncSetAttribute");
    }
    for (int d = 0; d < 2; ++d) {
        for (int v = 0; v <= cfsim::kBucketGlobal; ++v) {
            int blocks = 0;
            if ((e = cfsim::occupancy_of(v, d == 0 ? CFSIM_F64 : CFSIM_F32, &blocks)) != 0) {
                delete ctx;
                return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
            }
            const int cap = lds_blocks_per_cu(v, d == 0 ? 8 : 4);
            blocks = blocks < 1 ? 1 : (blocks > cap ? cap : blocks);
            ctx->grid[d][v] = ctx->num_cus * blocks;
        }
    }
    if ((e = scratch_address(device, &ctx->scratch)) != 0) {
        delete ctx;
        return hip_fail(e, "hipGetSymbolAddress(scratch)");
    }
    if ((e = (int)hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking)) != 0) {
        delete ctx;
        return hip_fail(e, "hipStreamCreateWithFlags");
    }
    *out = ctx;
    return ok();
}

void cfsim_context_destroy(cfsim_context* ctx) {
    if (!ctx) return;
    if (ctx->exec) (void)hipGraphExecDestroy(ctx->exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->large_exec) (void)hipGraphExecDestroy(ctx->large_exec);
    if (ctx->large_graph) (void)hipGraphDestroy(ctx->large_graph);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    for (int v = 0; v < cfsim::kBuckets; ++v) {
        if (ctx->t0[v]) (void)hipEventDestroy(ctx->t0[v]);
        if (ctx->t1[v]) (void)hipEventDestroy(ctx->t1[v]);
    }
    delete ctx;
}

// ------------------------------------------------------------------ host check of jump lists
cfsim_status cfsim_check_jumps(int32_t n_graphs, const int64_t* node_off, const int64_t* edge_off,
                               const int32_t* src, const int32_t* dst, const double* count) {
    if (n_graphs < 0) return fail(CFSIM_E_INVALID_ARG, "n_graphs must be >= 0");
    if (!node_off || !edge_off) return fail(CFSIM_E_INVALID_ARG, "node_off or edge_off is NULL");
    if (node_off[0] != 0 || edge_off[0] != 0) return fail(CFSIM_E_BAD_GRAPH, "node_off[0] and edge_off[0] must be 0");
    for (int32_t g = 0; g < n_graphs; ++g) {
        if (node_off[g + 1] <= node_off[g])
            return fail(CFSIM_E_BAD_GRAPH, "graph %d: node_off must increase (every graph has a node)", g);
        if (edge_off[g + 1] < edge_off[g]) return fail(CFSIM_E_BAD_GRAPH, "graph %d: edge_off decreases", g);
    }
    if (edge_off[n_graphs] > 0 && (!src || !dst || !count))
        return fail(CFSIM_E_INVALID_ARG, "src, dst or count is NULL");
    for (int32_t g = 0; g < n_graphs; ++g) {
        const int64_t n = node_off[g + 1] - node_off[g];
        for (int64_t t = edge_off[g]; t < edge_off[g + 1]; ++t) {
            if (src[t] < 0 || src[t] >= n || dst[t] < 0 || dst[t] >= n)
                return fail(CFSIM_E_BAD_GRAPH, "graph %d, jump %lld: endpoint (%d, %d) outside [0, %lld)", g,
                            (long long)(t - edge_off[g]), src[t], dst[t], (long long)n);
            if (!std::isfinite(count[t]))
                return fail(CFSIM_E_NONFINITE, "graph %d, jump %lld: count is not finite", g,
                            (long long)(t - edge_off[g]));
            if (count[t] < 0.0)
                return fail(CFSIM_E_NEGWEIGHT, "graph %d, jump %lld: negative count %g", g,
                            (long long)(t - edge_off[g]), count[t]);
        }
    }
    return ok();
}

// ------------------------------------------------------------------ pack (a1)
size_t cfsim_pack_workspace_size(int32_t n_graphs, int64_t total_nodes, int64_t total_edges) {
    (void)n_graphs;
    if (total_nodes < 0 || total_edges < 0) return 0;
    return align256((size_t)total_nodes * 4) + 2 * align256((size_t)total_edges * 4);
}

cfsim_status cfsim_pack(cfsim_context* ctx, int32_t n_graphs, int64_t total_nodes, int64_t total_edges,
                        const int64_t* node_off, const int64_t* edge_off, const int32_t* src, const int32_t* dst,
                        const double* count, int32_t* row_ptr, int32_t* col, double* w, int32_t* col_ptr,
                        int32_t* row, int32_t* eid, int32_t* err_flags, void* ws, size_t ws_bytes, void* stream) {
    if (n_graphs < 0) return fail(CFSIM_E_INVALID_ARG, "n_graphs must be >= 0");
    if (total_nodes < 0 || total_edges < 0) return fail(CFSIM_E_INVALID_ARG, "totals must be >= 0");
    if (total_nodes > INT32_MAX || total_edges > INT32_MAX)
        return fail(CFSIM_E_UNSUPPORTED, "more than 2^31-1 nodes or edges in one set");
    if (!node_off || !edge_off || !row_ptr || !col_ptr || !err_flags)
        return fail(CFSIM_E_INVALID_ARG, "an offset or output array is NULL");
    if (total_edges > 0 && (!src || !dst || !count || !col || !w || !row || !eid))
        return fail(CFSIM_E_INVALID_ARG, "an edge array is NULL");
    const size_t need = cfsim_pack_workspace_size(n_graphs, total_nodes, total_edges);
    if (ws_bytes < need || (need > 0 && !ws))
        return fail(CFSIM_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if (!ctx) return fail(CFSIM_E_INVALID_ARG, "context is NULL");
    unsigned char* p = static_cast<unsigned char*>(ws);
    cfsim::PackJob job;
    job.n_graphs = n_graphs;
    job.node_off = node_off;
    job.edge_off = edge_off;
    job.src = src;
    job.dst = dst;
    job.count = count;
    job.rp = row_ptr;
    job.ci = col;
    job.w = w;
    job.cp = col_ptr;
    job.ri = row;
    job.eid = eid;
    job.err = err_flags;
    job.cursor = reinterpret_cast<int32_t*>(p);
    p += align256((size_t)total_nodes * 4);
    job.eorig = reinterpret_cast<int32_t*>(p);
    p += align256((size_t)total_edges * 4);
    job.csrpos = reinterpret_cast<int32_t*>(p);
    int e = (int)hipSetDevice(ctx->device);
    if (e != 0) return hip_fail(e, "hipSetDevice");
    e = cfsim::launch_pack(job, static_cast<hipStream_t>(stream));
    if (e != 0) return hip_fail(e, "pack launch");
    return ok();
}

// ------------------------------------------------------------------ plain pair (a2-a7)
// One pair alone is latency-bound: every update ends in a workgroup barrier,
// so more waves (fewer rows per wave) shorten it.  The plain path takes the
// smaller of the 512- and 1024-thread kernels that holds the pair with at
// most two rows per wave, else the 1024-thread two-chunk kernel if it holds
// the pair, else the first LDS kernel that does, else the global-memory
// kernel; -1 if none can take it.  (Measured on one MI355X: a 12 x 16 pair
// 292 us on the 512-thread kernel against 763 us on the one-wave kernel.)
static int plain_variant(int nA, int nB, int nnzA, int nnzB, int esize, cfsim::PairShape* sh) {
    int first = -1;
    for (int v = 0; v < cfsim::kNumVariants && first < 0; ++v)
        if (cfsim::choose_shape(nA, nB, nnzA, nnzB, v, esize, sh)) first = v;
    if (first < 0) {
        if (cfsim::global_fits(nA, nB, nnzA, nnzB, esize, (long long)nA * nB, sh)) return cfsim::kBucketGlobal;
        return -1;
    }
    cfsim::PairShape s;
    for (int v = first > 2 ? first : 2; v <= 3; ++v)
        if (cfsim::choose_shape(nA, nB, nnzA, nnzB, v, esize, &s) && cfsim::variant_info(v, esize).nt / 32 >= s.nR) {
            *sh = s;
            return v;
        }
    if (first <= 3 && cfsim::choose_shape(nA, nB, nnzA, nnzB, 3, esize, &s)) {
        *sh = s;
        return 3;
    }
    return first;
}

size_t cfsim_score_workspace_size(const cfsim_context* ctx, int32_t n_a, int32_t n_b, const cfsim_options* opt) {
    (void)ctx;
    if (n_a < 1 || n_b < 1 || !opt) return 0;
    const size_t esize = fp64_final(opt) ? 8 : esize_of(opt->dtype);
    if (opt->resize == CFSIM_RESIZE_BILINEAR) return large_ws_bytes(1, n_a > n_b ? n_a : n_b, (int)esize, 6);
    // the two iterate buffers of the global kernel (the LDS kernels need none)
    return align256(2 * (size_t)n_a * (size_t)n_b * esize);
}

cfsim_status cfsim_score(cfsim_context* ctx, const cfsim_graph* A, const cfsim_graph* B, const cfsim_options* opt,
                         void* S_out, int32_t* match_out, cfsim_pair_result* res, void* ws, size_t ws_bytes,
                         void* stream) {
    cfsim_status s;
    if ((s = check_graph(A, "A")) != CFSIM_OK) return s;
    if ((s = check_graph(B, "B")) != CFSIM_OK) return s;
    if ((s = check_options(opt)) != CFSIM_OK) return s;
    if ((s = check_no_mfma(opt)) != CFSIM_OK) return s;
    if (!res) return fail(CFSIM_E_INVALID_ARG, "res is NULL");
    const int esize = esize_of(opt->dtype);
    if (opt->resize == CFSIM_RESIZE_BILINEAR && A->n == B->n && fp64_final(opt))
        return check_no_fp64_final(opt);
    if (opt->resize == CFSIM_RESIZE_BILINEAR && A->n != B->n) {
        // scaled pairs: the resized mode of an LDS kernel when one holds the
        // pair (one launch), else the tiled path (the same factored operator);
        // equal sizes need no scaling and take the plain path below
        const int M = A->n > B->n ? A->n : B->n;
        if ((s = check_no_fp64_final(opt)) != CFSIM_OK) return s;
        if ((s = check_large_limits(M, opt)) != CFSIM_OK) return s;
        const size_t need = cfsim_score_workspace_size(ctx, A->n, B->n, opt);
        if (ws_bytes < need || !ws)
            return fail(CFSIM_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
        if (!ctx) return fail(CFSIM_E_INVALID_ARG, "context is NULL");
        {
            const bool a_larger = A->n > B->n;
            const int m = a_larger ? B->n : A->n;
            const int nnzL = a_larger ? A->nnz : B->nnz, nnzX = a_larger ? B->nnz : A->nnz;
            // the widest workgroup first: a lone pair waits on a barrier every update
            int v = -1;
            for (int c : {3, 4, 2, 1, 0})
                if (v < 0 && cfsim::resized_fits(M, m, nnzL, nnzX, c, esize)) v = c;
            if (v >= 0) {
                cfsim::PairJob job{};
                job.single = 1;
                job.ga = ref_of(A);
                job.gb = ref_of(B);
                job.max_iter = opt->max_iter;
                job.tol = opt->tol;
                job.tie_tol = tie_tol_of(opt, opt->dtype);
                job.res = res;
                job.match = match_out;
                job.S_out = S_out;
                job.variant = v;
                job.resize = 1;
                int e = (int)hipSetDevice(ctx->device);
                if (e != 0) return hip_fail(e, "hipSetDevice");
                e = cfsim::launch_pair_lds(v, opt->dtype, job, 1, static_cast<hipStream_t>(stream));
                if (e != 0) return hip_fail(e, "resized pair kernel launch");
                return ok();
            }
        }
        cfsim::LargeJob J = large_job(opt, 1, M, res, match_out, nullptr, S_out, nullptr, ws);
        J.single = 1;
        J.ga = ref_of(A);
        J.gb = ref_of(B);
        int e = (int)hipSetDevice(ctx->device);
        if (e != 0) return hip_fail(e, "hipSetDevice");
        e = cfsim::launch_large(opt->dtype, J, cfsim::large_step_grid(num_cus_of(ctx)),
                                static_cast<hipStream_t>(stream));
        if (e != 0) return hip_fail(e, "tiled-path launch");
        return ok();
    }
    cfsim::PairShape sh;
    const int variant = plain_variant(A->n, B->n, A->nnz, B->nnz, esize, &sh);
    if (variant < 0)
        return fail(CFSIM_E_UNSUPPORTED, "pair %d x %d: its graph lists do not fit the kernels' LDS", B->n, A->n);
    const size_t need = cfsim_score_workspace_size(ctx, A->n, B->n, opt);
    if (ws_bytes < need || !ws) return fail(CFSIM_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if (!ctx) return fail(CFSIM_E_INVALID_ARG, "context is NULL");
    // FP64 pass (near-tie FP32 result): the first FP64 kernel that holds the pair
    int variant64 = -1;
    if (fp64_final(opt)) {
        cfsim::PairShape sh64;
        variant64 = plain_variant(A->n, B->n, A->nnz, B->nnz, 8, &sh64);
    }
    cfsim::PairJob job{};
    job.single = 1;
    job.ga = ref_of(A);
    job.gb = ref_of(B);
    job.max_iter = opt->max_iter;
    job.tol = opt->tol;
    job.tie_tol = tie_tol_of(opt, opt->dtype);
    job.res = res;
    job.match = match_out;
    job.S_out = S_out;
    job.variant = variant;
    job.gws = ws;
    job.slot_elems = (long long)A->n * B->n;
    int e = (int)hipSetDevice(ctx->device);
    if (e != 0) return hip_fail(e, "hipSetDevice");
    hipStream_t st = static_cast<hipStream_t>(stream);
    e = cfsim::launch_pair_lds(variant, opt->dtype, job, 1, st);
    if (e != 0) return hip_fail(e, "pair kernel launch");
    if (variant64 >= 0) {  // runs only if the FP32 result is a near tie (decided on the device)
        job.refine = 1;
        job.variant = variant64;
        job.tie_tol = tie_tol_of(opt, CFSIM_F64);
        e = cfsim::launch_pair_lds(variant64, CFSIM_F64, job, 1, st);
        if (e != 0) return hip_fail(e, "FP64 pass launch");
    }
    return ok();
}

cfsim_status cfsim_score_noalloc(cfsim_context* ctx, const cfsim_graph* A, const cfsim_graph* B,
                                 const cfsim_options* opt, void* S_out, int32_t* match_out, cfsim_pair_result* res,
                                 void* stream) {
    cfsim_status s;
    if ((s = check_graph(A, "A")) != CFSIM_OK) return s;
    if ((s = check_graph(B, "B")) != CFSIM_OK) return s;
    if ((s = check_options(opt)) != CFSIM_OK) return s;
    if (!res) return fail(CFSIM_E_INVALID_ARG, "res is NULL");
    if (!ctx) return fail(CFSIM_E_INVALID_ARG, "context is NULL");
    const size_t need = cfsim_score_workspace_size(ctx, A->n, B->n, opt);
    if (need > (size_t)CFSIM_NOALLOC_SCRATCH_BYTES)
        return fail(CFSIM_E_UNSUPPORTED, "pair %d x %d needs %zu bytes of scratch; the static scratch holds %zu",
                    B->n, A->n, need, (size_t)CFSIM_NOALLOC_SCRATCH_BYTES);
    if (!ctx->scratch) return fail(CFSIM_E_UNSUPPORTED, "no static scratch on device %d", ctx->device);
    return cfsim_score(ctx, A, B, opt, S_out, match_out, res, ctx->scratch, (size_t)CFSIM_NOALLOC_SCRATCH_BYTES,
                       stream);
}

// ------------------------------------------------------------------ batch (a2-a8)
size_t cfsim_batch_workspace_size(const cfsim_context* ctx, const cfsim_graph_set* set, int64_t n_pairs,
                                  const cfsim_options* opt) {
    if (n_pairs < 0 || !set || !opt || set->max_nodes < 1) return 0;
    if (opt->resize == CFSIM_RESIZE_BILINEAR) {
        if (set->max_nodes > cfsim::kLargeMaxNodes) return 0;
        // the tiled path's workspace, then the LDS kernels' schedule
        return large_ws_bytes(n_pairs > 0 ? n_pairs : 1, set->max_nodes, esize_of(opt->dtype), 6) +
               sched_ws_bytes(n_pairs) + resized_slots_bytes(ctx, esize_of(opt->dtype), set->max_nodes);
    }
    return batch_ws_bytes(ctx, n_pairs, fp64_final(opt) ? 8 : esize_of(opt->dtype), set->max_nodes);
}

// Plan and bucket kernels of one pass of the batched path on `st`: dtype is
// the pass's arithmetic type; filter (the FP32 results) restricts the FP64
// pass of an FP32 call to its near-tie pairs.
// Forward checkpoints requested by cfsim_score_batch_ckpt (none: ptr NULL).
struct CkptOut {
    void* ptr;
    const int64_t* off;
    int every;
};

// The damped measure of cfsim_score_damped (on = 0: the undamped iteration).
struct Damping {
    int on;
    double alpha;
    const double* prior;
    const int64_t* prior_off;
};

static int enqueue_pass(cfsim_context* ctx, const cfsim_graph_set* set, const int32_t* pair_a, const int32_t* pair_b,
                        int64_t n_pairs, const cfsim_options* opt, int dtype, const cfsim_pair_result* filter,
                        cfsim_pair_result* res, int32_t* match, const int64_t* match_off, void* S_out,
                        const int64_t* S_off, const BatchWs& b, hipStream_t st, bool timed, const CkptOut& ck,
                        const Damping& dm, int resize = 0) {
    const int esize = esize_of(dtype);
    cfsim::PlanJob plan{};
    plan.set = ref_of(set);
    plan.pair_a = pair_a;
    plan.pair_b = pair_b;
    plan.n_pairs = n_pairs;
    plan.filter = filter;
    plan.esize = esize;
    plan.slot_elems = resize ? cfsim::resized_slot_elems(set->max_nodes) : global_slot_elems(set->max_nodes);
    plan.order = b.order;
    plan.bounds = b.bounds;
    plan.queues = b.queues;
    memcpy(plan.tune, ctx->tune[dtype_index(dtype)], sizeof(plan.tune));
    plan.resize = resize;
    int e = cfsim::launch_plan(plan, st);
    if (e != 0) return e;
    cfsim::PairJob job{};
    job.single = 0;
    job.set = ref_of(set);
    job.pair_a = pair_a;
    job.pair_b = pair_b;
    job.order = b.order;
    job.max_iter = opt->max_iter;
    job.tol = opt->tol;
    job.tie_tol = tie_tol_of(opt, dtype);
    job.refine = filter != nullptr;
    job.res = res;
    job.match = match;
    job.match_off = match_off;
    job.S_out = S_out;
    job.S_off = S_off;
    job.ckpt = ck.ptr;
    job.ckpt_off = ck.off;
    job.ckpt_every = ck.every;
    job.resize = resize;
    job.damped = dm.on;
    job.alpha = dm.alpha;
    job.prior = dm.prior;
    job.prior_off = dm.prior_off;
    const int d = dtype_index(dtype);
    // The bucket kernels run one after another on the caller's stream, each
    // with the whole device: a bucket's persistent grid drains its queue
    // longest pair first, so its tail is about one pair long.
    for (int v = 0; v < cfsim::kBuckets; ++v) {
        if (filter && v == cfsim::kBucketInvalid) continue;  // the FP64 pass leaves no pair invalid
        job.bounds = b.bounds + 2 * v;
        job.queue = b.queues + v;
        job.variant = v;
        int grid = 1;
        if (v < cfsim::kNumVariants) {
            job.gws = nullptr;  // both iterates stay in LDS
            job.slot_elems = 0;
            grid = ctx->grid[d][v];
        } else if (v == cfsim::kBucketGlobal) {
            job.gws = b.slots[v];
            job.slot_elems = resize ? cfsim::resized_slot_elems(set->max_nodes) : global_slot_elems(set->max_nodes);
            grid = ctx->grid[d][v];
        }
        if (timed && (e = (int)hipEventRecord(ctx->t0[v], st)) != 0) return e;
        if ((e = cfsim::launch_pair_lds(v, dtype, job, grid, st)) != 0) return e;
        if (timed && (e = (int)hipEventRecord(ctx->t1[v], st)) != 0) return e;
    }
    (void)esize;
    return 0;
}

static int enqueue_batch(cfsim_context* ctx, const cfsim_graph_set* set, const int32_t* pair_a,
                         const int32_t* pair_b, int64_t n_pairs, const cfsim_options* opt, cfsim_pair_result* res,
                         int32_t* match, const int64_t* match_off, void* S_out, const int64_t* S_off, void* ws,
                         hipStream_t st, bool timed, const CkptOut& ck, const Damping& dm) {
    const int esize = fp64_final(opt) ? 8 : esize_of(opt->dtype);
    const BatchWs b = carve_batch(ctx, ws, n_pairs, esize, set->max_nodes);
    int e = enqueue_pass(ctx, set, pair_a, pair_b, n_pairs, opt, opt->dtype, nullptr, res, match, match_off, S_out,
                         S_off, b, st, timed, ck, dm);
    if (e != 0 || !fp64_final(opt)) return e;
    // FP64 pass over the pairs whose FP32 result is a near tie (the schedule
    // arrays are reused: the stream orders the passes)
    return enqueue_pass(ctx, set, pair_a, pair_b, n_pairs, opt, CFSIM_F64, res, res, match, match_off, S_out, S_off, b,
                        st, false, CkptOut{nullptr, nullptr, 0}, dm);
}

static int enqueue_large(cfsim_context* ctx, const cfsim_graph_set* set, const int32_t* pair_a,
                         const int32_t* pair_b, int64_t n_pairs, const cfsim_options* opt, cfsim_pair_result* res,
                         int32_t* match, const int64_t* match_off, void* S_out, const int64_t* S_off, void* ws,
                         hipStream_t st) {
    cfsim::LargeJob J = large_job(opt, n_pairs, set->max_nodes, res, match, match_off, S_out, S_off, ws);
    J.set = ref_of(set);
    J.pair_a = pair_a;
    J.pair_b = pair_b;
    return cfsim::launch_large(opt->dtype, J, cfsim::large_step_grid(num_cus_of(ctx)), st);
}

// Resized batch: the LDS kernels in their resized mode take every pair they
// hold; the tiled path then runs the pairs they left invalid (pairs too large
// for LDS, and pairs with bad ids, which it marks invalid itself).
static int enqueue_resized(cfsim_context* ctx, const cfsim_graph_set* set, const int32_t* pair_a,
                           const int32_t* pair_b, int64_t n_pairs, const cfsim_options* opt, cfsim_pair_result* res,
                           int32_t* match, const int64_t* match_off, void* S_out, const int64_t* S_off, void* ws,
                           hipStream_t st) {
    const size_t lb = large_ws_bytes(n_pairs, set->max_nodes, esize_of(opt->dtype), 6);
    BatchWs b = carve_sched(static_cast<unsigned char*>(ws) + lb, n_pairs);
    b.slots[cfsim::kBucketGlobal] = static_cast<unsigned char*>(ws) + lb + sched_ws_bytes(n_pairs);
    int e = enqueue_pass(ctx, set, pair_a, pair_b, n_pairs, opt, opt->dtype, nullptr, res, match, match_off, S_out,
                         S_off, b, st, false, CkptOut{nullptr, nullptr, 0}, Damping{0, 0.0, nullptr, nullptr}, 1);
    if (e != 0) return e;
    cfsim::LargeJob J = large_job(opt, n_pairs, set->max_nodes, res, match, match_off, S_out, S_off, ws);
    J.set = ref_of(set);
    J.pair_a = pair_a;
    J.pair_b = pair_b;
    J.filter = res;
    return cfsim::launch_large(opt->dtype, J, cfsim::large_step_grid(num_cus_of(ctx)), st);
}

// The tiled path over the pairs of a set (large pairs; every pair when resized).
static cfsim_status run_large(cfsim_context* ctx, const cfsim_graph_set* set, const int32_t* pair_a,
                              const int32_t* pair_b, int64_t n_pairs, const cfsim_options* opt,
                              cfsim_pair_result* res, int32_t* match, const int64_t* match_off, void* S_out,
                              const int64_t* S_off, void* ws, hipStream_t st) {
    if (graphs_disabled()) {
        const int e = enqueue_large(ctx, set, pair_a, pair_b, n_pairs, opt, res, match, match_off, S_out, S_off, ws,
                                    st);
        if (e != 0) return hip_fail(e, "tiled-path launch");
        return ok();
    }
    const auto key = set_call_key(ctx, set, pair_a, pair_b, n_pairs, opt, res, match, match_off, S_out, S_off, ws);
    return replay_or_capture(ctx, &ctx->large_graph, &ctx->large_exec, &ctx->large_key, key, st, [&](hipStream_t cs) {
        return enqueue_large(ctx, set, pair_a, pair_b, n_pairs, opt, res, match, match_off, S_out, S_off, ws, cs);
    });
}

static cfsim_status score_batch(cfsim_context* ctx, const cfsim_graph_set* set, const int32_t* pair_a,
                                const int32_t* pair_b, int64_t n_pairs, const cfsim_options* opt,
                                cfsim_pair_result* res, int32_t* match, const int64_t* match_off, void* S_out,
                                const int64_t* S_off, const CkptOut& ck, const Damping& dm, void* ws,
                                size_t ws_bytes, void* stream) {
    cfsim_status s;
    if ((s = check_set(set)) != CFSIM_OK) return s;
    if ((s = check_options(opt)) != CFSIM_OK) return s;
    if ((s = check_no_mfma(opt)) != CFSIM_OK) return s;
    if (n_pairs < 0) return fail(CFSIM_E_INVALID_ARG, "n_pairs must be >= 0");
    if (n_pairs > INT32_MAX) return fail(CFSIM_E_UNSUPPORTED, "more than 2^31-1 pairs in one call");
    if (n_pairs > 0 && (!pair_a || !pair_b || !res))
        return fail(CFSIM_E_INVALID_ARG, "pair_a, pair_b or res is NULL");
    if ((match == nullptr) != (match_off == nullptr))
        return fail(CFSIM_E_INVALID_ARG, "match and match_off must both be given or both be NULL");
    if ((S_out == nullptr) != (S_off == nullptr))
        return fail(CFSIM_E_INVALID_ARG, "S_out and S_off must both be given or both be NULL");
    if (set->max_nodes > 65536) return fail(CFSIM_E_UNSUPPORTED, "max_nodes above 65536");
    const bool resize = opt->resize == CFSIM_RESIZE_BILINEAR;
    if (resize && (s = check_no_fp64_final(opt)) != CFSIM_OK) return s;
    if (resize && (s = check_large_limits(set->max_nodes, opt)) != CFSIM_OK) return s;
    const size_t need = cfsim_batch_workspace_size(ctx, set, n_pairs, opt);
    if (ws_bytes < need || !ws) return fail(CFSIM_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if (!ctx) return fail(CFSIM_E_INVALID_ARG, "context is NULL");
    if (n_pairs == 0) return ok();
    int e = (int)hipSetDevice(ctx->device);
    if (e != 0) return hip_fail(e, "hipSetDevice");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (resize) {
        // the resized operator in factored form: LDS kernels, the rest on the tiled path
        ctx->timed = 0;
        if (ctx->timing || graphs_disabled()) {
            e = enqueue_resized(ctx, set, pair_a, pair_b, n_pairs, opt, res, match, match_off, S_out, S_off, ws, st);
            if (e != 0) return hip_fail(e, "resized batch launch");
            return ok();
        }
        auto key = set_call_key(ctx, set, pair_a, pair_b, n_pairs, opt, res, match, match_off, S_out, S_off, ws);
        return replay_or_capture(ctx, &ctx->graph, &ctx->exec, &ctx->key, key, st, [&](hipStream_t cs) {
            return enqueue_resized(ctx, set, pair_a, pair_b, n_pairs, opt, res, match, match_off, S_out, S_off, ws,
                                   cs);
        });
    }
    if (ctx->timing || graphs_disabled()) {
        e = enqueue_batch(ctx, set, pair_a, pair_b, n_pairs, opt, res, match, match_off, S_out, S_off, ws, st,
                          ctx->timing != 0, ck, dm);
        if (e != 0) return hip_fail(e, "batch launch");
        if (ctx->timing) ctx->timed = 1;
        return ok();
    }
    auto key = set_call_key(ctx, set, pair_a, pair_b, n_pairs, opt, res, match, match_off, S_out, S_off, ws);
    append_key(key, ck.ptr);
    append_key(key, ck.off);
    append_key(key, ck.every);
    append_key(key, dm.on);
    append_key(key, dm.alpha);
    append_key(key, dm.prior);
    append_key(key, dm.prior_off);
    return replay_or_capture(ctx, &ctx->graph, &ctx->exec, &ctx->key, key, st, [&](hipStream_t cs) {
        return enqueue_batch(ctx, set, pair_a, pair_b, n_pairs, opt, res, match, match_off, S_out, S_off, ws, cs,
                             false, ck, dm);
    });
}

cfsim_status cfsim_score_batch(cfsim_context* ctx, const cfsim_graph_set* set, const int32_t* pair_a,
                               const int32_t* pair_b, int64_t n_pairs, const cfsim_options* opt,
                               cfsim_pair_result* res, int32_t* match, const int64_t* match_off, void* S_out,
                               const int64_t* S_off, void* ws, size_t ws_bytes, void* stream) {
    return score_batch(ctx, set, pair_a, pair_b, n_pairs, opt, res, match, match_off, S_out, S_off,
                       CkptOut{nullptr, nullptr, 0}, Damping{0, 0.0, nullptr, nullptr}, ws, ws_bytes, stream);
}

cfsim_status cfsim_score_damped(cfsim_context* ctx, const cfsim_graph_set* set, const int32_t* pair_a,
                                const int32_t* pair_b, int64_t n_pairs, const cfsim_options* opt, double alpha,
                                const double* prior, const int64_t* prior_off, cfsim_pair_result* res,
                                int32_t* match, const int64_t* match_off, void* S_out, const int64_t* S_off, void* ws,
                                size_t ws_bytes, void* stream) {
    if (!(alpha >= 0.0 && alpha < 1.0)) return fail(CFSIM_E_INVALID_ARG, "alpha must lie in [0, 1)");
    if ((prior == nullptr) != (prior_off == nullptr))
        return fail(CFSIM_E_INVALID_ARG, "prior and prior_off must both be given or both be NULL");
    if (opt && opt->resize != CFSIM_RESIZE_NONE)
        return fail(CFSIM_E_UNSUPPORTED, "the damped measure runs on the unscaled operator only");
    return score_batch(ctx, set, pair_a, pair_b, n_pairs, opt, res, match, match_off, S_out, S_off,
                       CkptOut{nullptr, nullptr, 0}, Damping{1, alpha, prior, prior_off}, ws, ws_bytes, stream);
}

cfsim_status cfsim_score_batch_ckpt(cfsim_context* ctx, const cfsim_graph_set* set, const int32_t* pair_a,
                                    const int32_t* pair_b, int64_t n_pairs, const cfsim_options* opt,
                                    cfsim_pair_result* res, int32_t* match, const int64_t* match_off, void* S_out,
                                    const int64_t* S_off, void* ckpt, const int64_t* ckpt_off,
                                    int32_t checkpoint_every, void* ws, size_t ws_bytes, void* stream) {
    if (checkpoint_every < 1) return fail(CFSIM_E_INVALID_ARG, "checkpoint_every must be >= 1");
    if (n_pairs > 0 && (!ckpt || !ckpt_off)) return fail(CFSIM_E_INVALID_ARG, "ckpt or ckpt_off is NULL");
    if (opt && opt->resize == CFSIM_RESIZE_BILINEAR)
        return fail(CFSIM_E_UNSUPPORTED, "forward checkpoints on the unscaled operator only");
    if (opt && fp64_final(opt))
        return fail(CFSIM_E_UNSUPPORTED, "forward checkpoints with CFSIM_FLAG_FP64_FINAL");
    return score_batch(ctx, set, pair_a, pair_b, n_pairs, opt, res, match, match_off, S_out, S_off,
                       CkptOut{ckpt, ckpt_off, checkpoint_every}, Damping{0, 0.0, nullptr, nullptr}, ws, ws_bytes,
                       stream);
}

cfsim_status cfsim_batch_buckets(cfsim_context* ctx, const cfsim_graph_set* set, const int32_t* pair_a,
                                 const int32_t* pair_b, int64_t n_pairs, const cfsim_options* opt, int32_t* bucket,
                                 void* stream) {
    cfsim_status s;
    if ((s = check_set(set)) != CFSIM_OK) return s;
    if ((s = check_options(opt)) != CFSIM_OK) return s;
    if ((s = check_no_mfma(opt)) != CFSIM_OK) return s;
    if (n_pairs < 0) return fail(CFSIM_E_INVALID_ARG, "n_pairs must be >= 0");
    if (n_pairs > INT32_MAX) return fail(CFSIM_E_UNSUPPORTED, "more than 2^31-1 pairs in one call");
    if (n_pairs > 0 && (!pair_a || !pair_b || !bucket))
        return fail(CFSIM_E_INVALID_ARG, "pair_a, pair_b or bucket is NULL");
    if (set->max_nodes > 65536) return fail(CFSIM_E_UNSUPPORTED, "max_nodes above 65536");
    if (!ctx) return fail(CFSIM_E_INVALID_ARG, "context is NULL");
    if (n_pairs == 0) return ok();
    int e = (int)hipSetDevice(ctx->device);
    if (e != 0) return hip_fail(e, "hipSetDevice");
    cfsim::PlanJob plan{};
    plan.set = ref_of(set);
    memcpy(plan.tune, ctx->tune[dtype_index(opt->dtype)], sizeof(plan.tune));
    plan.pair_a = pair_a;
    plan.pair_b = pair_b;
    plan.n_pairs = n_pairs;
    plan.esize = esize_of(opt->dtype);
    plan.slot_elems = global_slot_elems(set->max_nodes);
    plan.resize = opt->resize == CFSIM_RESIZE_BILINEAR ? 1 : 0;
    e = cfsim::launch_buckets(plan, bucket, static_cast<hipStream_t>(stream));
    if (e != 0) return hip_fail(e, "bucket launch");
    return ok();
}

int32_t cfsim_tune_class(int32_t n_a, int32_t n_b) { return cfsim::tune_class(n_a, n_b); }

cfsim_status cfsim_context_set_tune(cfsim_context* ctx, int32_t dtype, const int32_t* table, int32_t n) {
    if (!ctx) return fail(CFSIM_E_INVALID_ARG, "context is NULL");
    if (dtype != CFSIM_F64 && dtype != CFSIM_F32) return fail(CFSIM_E_INVALID_ARG, "dtype must be CFSIM_F64 or CFSIM_F32");
    if (n != cfsim::kTuneClasses) return fail(CFSIM_E_INVALID_ARG, "table needs %d entries (got %d)", cfsim::kTuneClasses, n);
    if (!table) {
        memset(ctx->tune[dtype_index(dtype)], -1, cfsim::kTuneClasses);
        return ok();
    }
    for (int c = 0; c < n; ++c)
        if (table[c] < -1 || table[c] >= cfsim::kNumVariants)
            return fail(CFSIM_E_INVALID_ARG, "table[%d] = %d: must be -1 or an LDS bucket 0..%d", c, table[c],
                        cfsim::kNumVariants - 1);
    for (int c = 0; c < n; ++c) ctx->tune[dtype_index(dtype)][c] = (int8_t)table[c];
    return ok();
}

cfsim_status cfsim_context_get_tune(const cfsim_context* ctx, int32_t dtype, int32_t* table, int32_t n) {
    if (!ctx || !table) return fail(CFSIM_E_INVALID_ARG, "context or table is NULL");
    if (dtype != CFSIM_F64 && dtype != CFSIM_F32) return fail(CFSIM_E_INVALID_ARG, "dtype must be CFSIM_F64 or CFSIM_F32");
    if (n != cfsim::kTuneClasses) return fail(CFSIM_E_INVALID_ARG, "table needs %d entries (got %d)", cfsim::kTuneClasses, n);
    for (int c = 0; c < n; ++c) table[c] = ctx->tune[dtype_index(dtype)][c];
    return ok();
}

const char* cfsim_bucket_kernel(int32_t bucket, int32_t dtype) { return cfsim::bucket_kernel_name(bucket, dtype); }

cfsim_status cfsim_context_set_timing(cfsim_context* ctx, int32_t on) {
    if (!ctx) return fail(CFSIM_E_INVALID_ARG, "context is NULL");
    if (on && !ctx->t0[0]) {
        int e = (int)hipSetDevice(ctx->device);
        for (int v = 0; v < cfsim::kBuckets && e == 0; ++v) {
            e = (int)hipEventCreate(&ctx->t0[v]);
            if (e == 0) e = (int)hipEventCreate(&ctx->t1[v]);
        }
        if (e != 0) return hip_fail(e, "hipEventCreate");
    }
    ctx->timing = on != 0;
    return ok();
}

cfsim_status cfsim_batch_timings(cfsim_context* ctx, float* ms) {
    if (!ctx || !ms) return fail(CFSIM_E_INVALID_ARG, "context or ms is NULL");
    if (!ctx->timed) return fail(CFSIM_E_INVALID_ARG, "no timed cfsim_score_batch call was made");
    int e = (int)hipSetDevice(ctx->device);
    if (e != 0) return hip_fail(e, "hipSetDevice");
    for (int v = 0; v < cfsim::kBuckets; ++v) {
        if ((e = (int)hipEventSynchronize(ctx->t1[v])) != 0) return hip_fail(e, "hipEventSynchronize");
        float t = 0.0f;
        if ((e = (int)hipEventElapsedTime(&t, ctx->t0[v], ctx->t1[v])) != 0) return hip_fail(e, "hipEventElapsedTime");
        ms[v] = t;
    }
    return ok();
}

// ------------------------------------------------------------------ large pairs (a9)
size_t cfsim_large_workspace_size(const cfsim_context* ctx, const cfsim_graph_set* set, int64_t n_pairs,
                                  const cfsim_options* opt) {
    (void)ctx;
    if (n_pairs < 1 || !set || !opt || set->max_nodes < 1 || set->max_nodes > cfsim::kLargeMaxNodes) return 0;
    size_t b = large_ws_bytes(n_pairs, set->max_nodes, esize_of(opt->dtype), large_nslots(opt));
    if (mfma_bf16(opt)) b += mfma_ws_bytes(n_pairs, set->max_nodes);
    return b;
}

cfsim_status cfsim_score_large(cfsim_context* ctx, const cfsim_graph_set* set, const int32_t* pair_a,
                               const int32_t* pair_b, int64_t n_pairs, const cfsim_options* opt,
                               cfsim_pair_result* res, int32_t* match, const int64_t* match_off, void* S_out,
                               const int64_t* S_off, void* ws, size_t ws_bytes, void* stream) {
    cfsim_status s;
    if ((s = check_set(set)) != CFSIM_OK) return s;
    if ((s = check_options(opt)) != CFSIM_OK) return s;
    if (n_pairs < 0) return fail(CFSIM_E_INVALID_ARG, "n_pairs must be >= 0");
    if (n_pairs > INT32_MAX) return fail(CFSIM_E_UNSUPPORTED, "more than 2^31-1 pairs in one call");
    if (n_pairs > 0 && (!pair_a || !pair_b || !res))
        return fail(CFSIM_E_INVALID_ARG, "pair_a, pair_b or res is NULL");
    if ((match == nullptr) != (match_off == nullptr))
        return fail(CFSIM_E_INVALID_ARG, "match and match_off must both be given or both be NULL");
    if ((S_out == nullptr) != (S_off == nullptr))
        return fail(CFSIM_E_INVALID_ARG, "S_out and S_off must both be given or both be NULL");
    if ((s = check_no_fp64_final(opt)) != CFSIM_OK) return s;
    if ((s = check_large_limits(set->max_nodes, opt)) != CFSIM_OK) return s;
    if (n_pairs == 0) {
        if (!ctx) return fail(CFSIM_E_INVALID_ARG, "context is NULL");
        return ok();
    }
    const size_t need = cfsim_large_workspace_size(ctx, set, n_pairs, opt);
    if (ws_bytes < need || !ws) return fail(CFSIM_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if (!ctx) return fail(CFSIM_E_INVALID_ARG, "context is NULL");
    int e = (int)hipSetDevice(ctx->device);
    if (e != 0) return hip_fail(e, "hipSetDevice");
    return run_large(ctx, set, pair_a, pair_b, n_pairs, opt, res, match, match_off, S_out, S_off, ws,
                     static_cast<hipStream_t>(stream));
}

// ------------------------------------------------------------------ adjoint (a10)
size_t cfsim_backward_workspace_size(const cfsim_context* ctx, const cfsim_graph_set* set, int64_t n_pairs,
                                     const cfsim_options* opt, int32_t checkpoint_every) {
    (void)n_pairs;
    if (!set || !opt || set->max_nodes < 1 || checkpoint_every < 1 || opt->max_iter < 1) return 0;
    const long long slot = global_slot_elems(set->max_nodes);
    return 256 + (size_t)cfsim::backward_grid(num_cus_of(ctx)) *
                     (size_t)cfsim::backward_slot_bytes(opt->max_iter, checkpoint_every, slot, esize_of(opt->dtype));
}

cfsim_status cfsim_score_backward(cfsim_context* ctx, const cfsim_graph_set* set, const int32_t* pair_a,
                                  const int32_t* pair_b, int64_t n_pairs, const cfsim_options* opt,
                                  const cfsim_pair_result* fwd, const int32_t* match, const int64_t* match_off,
                                  const double* grad_score, double* grad_w, int32_t* pair_status,
                                  int32_t checkpoint_every, const void* ckpt, const int64_t* ckpt_off, void* ws,
                                  size_t ws_bytes, void* stream) {
    cfsim_status s;
    if ((s = check_set(set)) != CFSIM_OK) return s;
    if ((s = check_options(opt)) != CFSIM_OK) return s;
    if ((s = check_no_mfma(opt)) != CFSIM_OK) return s;
    if (n_pairs < 0) return fail(CFSIM_E_INVALID_ARG, "n_pairs must be >= 0");
    if (n_pairs > INT32_MAX) return fail(CFSIM_E_UNSUPPORTED, "more than 2^31-1 pairs in one call");
    if (checkpoint_every < 1) return fail(CFSIM_E_INVALID_ARG, "checkpoint_every must be >= 1");
    if (opt->resize == CFSIM_RESIZE_BILINEAR)
        return fail(CFSIM_E_UNSUPPORTED, "the reverse mode runs on the unscaled operator only");
    if (fp64_final(opt))
        return fail(CFSIM_E_UNSUPPORTED, "the reverse mode has no FP64 pass (CFSIM_FLAG_FP64_FINAL)");
    if (n_pairs > 0 && (!pair_a || !pair_b || !fwd || !match || !match_off || !grad_score || !grad_w))
        return fail(CFSIM_E_INVALID_ARG, "a pair, forward-result, matching or gradient array is NULL");
    if (set->max_nodes > 65536) return fail(CFSIM_E_UNSUPPORTED, "max_nodes above 65536");
    if ((ckpt == nullptr) != (ckpt_off == nullptr))
        return fail(CFSIM_E_INVALID_ARG, "ckpt and ckpt_off must both be given or both be NULL");
    const size_t need = cfsim_backward_workspace_size(ctx, set, n_pairs, opt, checkpoint_every);
    if (ws_bytes < need || !ws) return fail(CFSIM_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if (!ctx) return fail(CFSIM_E_INVALID_ARG, "context is NULL");
    if (n_pairs == 0) return ok();
    int e = (int)hipSetDevice(ctx->device);
    if (e != 0) return hip_fail(e, "hipSetDevice");
    e = cfsim::launch_backward(opt->dtype, ref_of(set), pair_a, pair_b, (int)n_pairs, fwd, match, match_off,
                               grad_score, grad_w, pair_status, checkpoint_every, ckpt, ckpt_off, opt->max_iter, ws,
                               global_slot_elems(set->max_nodes), cfsim::backward_grid(ctx->num_cus),
                               static_cast<hipStream_t>(stream));
    if (e != 0) return hip_fail(e, "backward launch");
    return ok();
}

// ------------------------------------------------------------------ top-k (a11)
size_t cfsim_topk_workspace_size(int64_t n, int32_t k) {
    if (n < 1 || k < 1) return 0;
    return align256((size_t)cfsim::topk_blocks(n) * (size_t)k * 16);
}

cfsim_status cfsim_topk(cfsim_context* ctx, const double* scores, int64_t n, int64_t stride, int32_t k,
                        int32_t* idx_out, double* score_out, void* ws, size_t ws_bytes, void* stream) {
    if (n < 1) return fail(CFSIM_E_INVALID_ARG, "n must be >= 1");
    if (n > INT32_MAX) return fail(CFSIM_E_UNSUPPORTED, "more than 2^31-1 scores");
    if (stride < 1) return fail(CFSIM_E_INVALID_ARG, "stride must be >= 1");
    if (k < 1 || k > cfsim::topk_max_k()) return fail(CFSIM_E_INVALID_ARG, "k must be in [1, %d]", cfsim::topk_max_k());
    if (!scores || !idx_out || !score_out) return fail(CFSIM_E_INVALID_ARG, "scores, idx_out or score_out is NULL");
    if (cfsim::topk_stage2_lds(n, k) > 159 * 1024)
        return fail(CFSIM_E_UNSUPPORTED, "n * k too large for the two-stage selection");
    const size_t need = cfsim_topk_workspace_size(n, k);
    if (ws_bytes < need || !ws) return fail(CFSIM_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if (!ctx) return fail(CFSIM_E_INVALID_ARG, "context is NULL");
    int e = (int)hipSetDevice(ctx->device);
    if (e != 0) return hip_fail(e, "hipSetDevice");
    e = cfsim::launch_topk(scores, n, stride, k, idx_out, score_out, ws, static_cast<hipStream_t>(stream));
    if (e != 0) return hip_fail(e, "top-k launch");
    return ok();
}

// ------------------------------------------------------------------ elementwise distances (Table 1)
size_t cfsim_distances_workspace_size(const cfsim_graph_set* set, int64_t n_pairs) {
    if (!set || set->max_nodes < 1 || set->max_nodes > 32768 || n_pairs < 1) return 0;
    return align256((size_t)(n_pairs + 1) * 8) +
           align256((size_t)n_pairs * (size_t)cfsim::dist_tasks_bound(set->max_nodes) * cfsim::kDistSums * 8);
}

cfsim_status cfsim_distances(cfsim_context* ctx, const cfsim_graph_set* set, const int32_t* pair_a,
                             const int32_t* pair_b, int64_t n_pairs, double p, double* out, void* ws,
                             size_t ws_bytes, void* stream) {
    cfsim_status s;
    if ((s = check_set(set)) != CFSIM_OK) return s;
    if (n_pairs < 0) return fail(CFSIM_E_INVALID_ARG, "n_pairs must be >= 0");
    if (n_pairs > INT32_MAX - 1) return fail(CFSIM_E_UNSUPPORTED, "more than 2^31-2 pairs in one call");
    if (!(p >= 1.0) || !std::isfinite(p)) return fail(CFSIM_E_INVALID_ARG, "the Minkowski order must be finite and >= 1");
    if (set->max_nodes > 32768) return fail(CFSIM_E_UNSUPPORTED, "max_nodes above 32768");
    if (n_pairs > 0 && (!pair_a || !pair_b || !out)) return fail(CFSIM_E_INVALID_ARG, "pair_a, pair_b or out is NULL");
    if (!ctx) return fail(CFSIM_E_INVALID_ARG, "context is NULL");
    if (n_pairs == 0) return ok();
    const size_t need = cfsim_distances_workspace_size(set, n_pairs);
    if (ws_bytes < need || !ws) return fail(CFSIM_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    int e = (int)hipSetDevice(ctx->device);
    if (e != 0) return hip_fail(e, "hipSetDevice");
    unsigned char* base = static_cast<unsigned char*>(ws);
    int64_t* task_off = reinterpret_cast<int64_t*>(base);
    double* part = reinterpret_cast<double*>(base + align256((size_t)(n_pairs + 1) * 8));
    e = cfsim::launch_distances(ref_of(set), set->max_nodes, pair_a, pair_b, (int)n_pairs, p, out, task_off, part,
                                cfsim::dist_grid(num_cus_of(ctx)), static_cast<hipStream_t>(stream));
    if (e != 0) return hip_fail(e, "distance launch");
    return ok();
}

}  // extern "C"

// ------------------------------------------------------------------ optimal-assignment matching
cfsim_status cfsim_assign(cfsim_context* ctx, int32_t dtype, const void* S, const int64_t* S_off,
                          const int32_t* n_rows, const int32_t* n_cols, int64_t n_pairs, int32_t max_dim,
                          int32_t* match, const int64_t* match_off, double* score, void* stream) {
    if (dtype != CFSIM_F64 && dtype != CFSIM_F32) return fail(CFSIM_E_INVALID_ARG, "dtype must be CFSIM_F64 or CFSIM_F32");
    if (n_pairs < 0) return fail(CFSIM_E_INVALID_ARG, "n_pairs must be >= 0");
    if (n_pairs > INT32_MAX) return fail(CFSIM_E_UNSUPPORTED, "more than 2^31-1 matrices in one call");
    if (max_dim < 1) return fail(CFSIM_E_INVALID_ARG, "max_dim must be >= 1");
    if (max_dim > cfsim::kAssignMaxDim)
        return fail(CFSIM_E_UNSUPPORTED, "max_dim above %d (the LDS state of one matrix)", cfsim::kAssignMaxDim);
    if (n_pairs > 0 && (!S || !S_off || !n_rows || !n_cols || !score))
        return fail(CFSIM_E_INVALID_ARG, "S, S_off, n_rows, n_cols or score is NULL");
    if ((match == nullptr) != (match_off == nullptr))
        return fail(CFSIM_E_INVALID_ARG, "match and match_off must both be given or both be NULL");
    if (!ctx) return fail(CFSIM_E_INVALID_ARG, "context is NULL");
    if (n_pairs == 0) return ok();
    int e = (int)hipSetDevice(ctx->device);
    if (e != 0) return hip_fail(e, "hipSetDevice");
    const int64_t cap = (int64_t)num_cus_of(ctx) * 32;
    const int grid = (int)(n_pairs < cap ? n_pairs : cap);
    e = cfsim::launch_assign(dtype, S, S_off, n_rows, n_cols, (int)n_pairs, max_dim, match, match_off, score, grid,
                             static_cast<hipStream_t>(stream));
    if (e != 0) return hip_fail(e, "assignment launch");
    return ok();
}

// ------------------------------------------------------------------ Ward's clustering (Section 6.2)
size_t cfsim_ward_workspace_size(int32_t n_obs) {
    if (n_obs < 1 || n_obs > cfsim::kWardMaxObs) return 0;
    return align256((size_t)n_obs * (size_t)n_obs * sizeof(double));
}

cfsim_status cfsim_ward(cfsim_context* ctx, const double* X, int32_t n_obs, int32_t n_feat, double* Z, void* ws,
                        size_t ws_bytes, void* stream) {
    if (n_obs < 1) return fail(CFSIM_E_INVALID_ARG, "n_obs must be >= 1");
    if (n_feat < 1) return fail(CFSIM_E_INVALID_ARG, "n_feat must be >= 1");
    if (n_obs > cfsim::kWardMaxObs)
        return fail(CFSIM_E_UNSUPPORTED, "more than %d observations (the merge state of one workgroup)",
                    cfsim::kWardMaxObs);
    if (!X || (n_obs > 1 && !Z)) return fail(CFSIM_E_INVALID_ARG, "X or Z is NULL");
    const size_t need = cfsim_ward_workspace_size(n_obs);
    if (!ws || ws_bytes < need) return fail(CFSIM_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if (!ctx) return fail(CFSIM_E_INVALID_ARG, "context is NULL");
    if (n_obs == 1) return ok();
    int e = (int)hipSetDevice(ctx->device);
    if (e != 0) return hip_fail(e, "hipSetDevice");
    e = cfsim::launch_ward(X, n_obs, n_feat, Z, static_cast<double*>(ws), static_cast<hipStream_t>(stream));
    if (e != 0) return hip_fail(e, "Ward launch");
    return ok();
}
