// Step a1: transition-probability matrices of a set of CFGs (paper Section 3,
// "Transition probability": P[u][v] = Pr(v | u), each non-empty row sums to 1).
//
// One workgroup per graph builds, from the graph's jump list with execution
// counts, the CSR (successor lists, rows sorted by target then by input
// position) and the CSC (predecessor lists, sorted by source then input
// position) and the row-normalised weights.  Everything is deterministic:
// atomics only count, and every list is sorted afterwards.
#include "cfsim_internal.h"

namespace cfsim {

namespace {

constexpr int kPackThreads = 256;

// In-place exclusive scan of a[0..n) (global memory) by one workgroup.
__device__ void block_exclusive_scan(int32_t* a, int n, int32_t* lds) {
    const int tid = threadIdx.x;
    int carry = 0;
    for (int base = 0; base < n; base += kPackThreads) {
        const int i = base + tid;
        const int v = (i < n) ? a[i] : 0;
        lds[tid] = v;
        __syncthreads();
        for (int off = 1; off < kPackThreads; off <<= 1) {
            const int t = (tid >= off) ? lds[tid - off] : 0;
            __syncthreads();
            lds[tid] += t;
            __syncthreads();
        }
        if (i < n) a[i] = carry + lds[tid] - v;
        const int total = lds[kPackThreads - 1];
        __syncthreads();
        carry += total;
    }
}

// Sort keys[b..e) ascending by (keys, tie) with insertion sort; `tie` moves along.
__device__ void sort_pairs(int32_t* keys, int32_t* tie, int b, int e) {
    for (int p = b + 1; p < e; ++p) {
        const int k = keys[p], t = tie[p];
        int q = p - 1;
        while (q >= b && (keys[q] > k || (keys[q] == k && tie[q] > t))) {
            keys[q + 1] = keys[q];
            tie[q + 1] = tie[q];
            --q;
        }
        keys[q + 1] = k;
        tie[q + 1] = t;
    }
}

__global__ void pack_init_kernel(int32_t* err) { *err = 0; }

__global__ __launch_bounds__(kPackThreads) void pack_kernel(PackJob J) {
    __shared__ int32_t lds[kPackThreads];
    __shared__ int32_t s_err;
    const int tid = threadIdx.x;
    const int g = blockIdx.x;
    const int64_t n0 = J.node_off[g], e0 = J.edge_off[g];
    const int n = (int)(J.node_off[g + 1] - n0);
    const int m = (int)(J.edge_off[g + 1] - e0);
    int32_t* rp = J.rp + n0 + g;
    int32_t* cp = J.cp + n0 + g;
    const int32_t* src = J.src + e0;
    const int32_t* dst = J.dst + e0;
    const double* cnt = J.count + e0;
    int32_t* ci = J.ci + e0;
    double* w = J.w + e0;
    int32_t* ri = J.ri + e0;
    int32_t* eid = J.eid + e0;
    int32_t* cur = J.cursor + n0;
    int32_t* eo = J.eorig + e0;
    int32_t* pos = J.csrpos + e0;

    if (tid == 0) s_err = 0;
    for (int i = tid; i <= n; i += kPackThreads) {
        rp[i] = 0;
        cp[i] = 0;
    }
    for (int i = tid; i < n; i += kPackThreads) cur[i] = 0;
    __syncthreads();

    int err = 0;
    // degree histograms (counts are order independent)
    for (int e = tid; e < m; e += kPackThreads) {
        const int u = src[e], v = dst[e];
        if (u < 0 || u >= n || v < 0 || v >= n) {
            err |= CFSIM_PACK_BAD_INDEX;
            continue;
        }
        atomicAdd(&rp[u], 1);
        atomicAdd(&cp[v], 1);
    }
    __syncthreads();
    block_exclusive_scan(rp, n + 1, lds);
    block_exclusive_scan(cp, n + 1, lds);
    __syncthreads();

    // CSR scatter, then per-row sort by (target, input position)
    for (int e = tid; e < m; e += kPackThreads) {
        const int u = src[e], v = dst[e];
        if (u < 0 || u >= n || v < 0 || v >= n) continue;
        const int p = rp[u] + atomicAdd(&cur[u], 1);
        ci[p] = v;
        eo[p] = e;
    }
    __syncthreads();
    for (int u = tid; u < n; u += kPackThreads) {
        const int b = rp[u], en = rp[u + 1];
        sort_pairs(ci, eo, b, en);
        double sum = 0.0;
        for (int p = b; p < en; ++p) {
            double c = cnt[eo[p]];
            if (!isfinite(c)) {
                err |= CFSIM_PACK_NONFINITE;
                c = 0.0;
            } else if (c < 0.0) {
                err |= CFSIM_PACK_NEGATIVE;
                c = 0.0;
            }
            sum += c;
        }
        for (int p = b; p < en; ++p) {
            double c = cnt[eo[p]];
            if (!isfinite(c) || c < 0.0) c = 0.0;
            w[p] = (sum > 0.0) ? c / sum : 0.0;
            pos[eo[p]] = p;
        }
        cur[u] = 0;
    }
    __syncthreads();

    // CSC scatter (eid temporarily holds the input position)
    for (int e = tid; e < m; e += kPackThreads) {
        const int u = src[e], v = dst[e];
        if (u < 0 || u >= n || v < 0 || v >= n) continue;
        const int p = cp[v] + atomicAdd(&cur[v], 1);
        ri[p] = u;
        eid[p] = e;
    }
    __syncthreads();
    for (int v = tid; v < n; v += kPackThreads) {
        const int b = cp[v], en = cp[v + 1];
        sort_pairs(ri, eid, b, en);
        for (int p = b; p < en; ++p) eid[p] = pos[eid[p]];
    }
    // slots of dropped jumps (bad ids) stay inert
    const int kept = rp[n];
    for (int p = kept + tid; p < m; p += kPackThreads) {
        ci[p] = 0;
        w[p] = 0.0;
        ri[p] = 0;
        eid[p] = 0;
    }
    if (err) atomicOr(&s_err, err);
    __syncthreads();
    if (tid == 0 && s_err) atomicOr(J.err, s_err);
}

}  // namespace

int launch_pack(const PackJob& job, hipStream_t stream) {
    hipLaunchKernelGGL(pack_init_kernel, dim3(1), dim3(1), 0, stream, job.err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || job.n_graphs == 0) return (int)e;
    hipLaunchKernelGGL(pack_kernel, dim3(job.n_graphs), dim3(kPackThreads), 0, stream, job);
    return (int)hipGetLastError();
}

}  // namespace cfsim
