// The five elementwise distances of Table 1 (Euclidean, Manhattan,
// Minkowski, Jaccard, Cosine) between the two transition matrices of a pair
// once both are at the common size M = max(n_A, n_B) (Section 4 and
// Section 4.1: the smaller matrix X, m x m, becomes R X R^T with the order-1
// interpolation R from its m nodes to M points at p (m - 1) / (M - 1); the
// larger matrix L is kept).
//
// No scaled matrix is ever stored.  Entry (i, j) of the scaled matrix is
//   y_ij = sum_a R_ia sum_b X_ab R_jb
// with at most two nonzero R_ia (rows a0(i), a0(i) + 1) and two R_jb, so
// each entry is a few reads of two CSR rows of X; x_ij is one CSR row of L.
// A pair's M rows are cut into at most kDistMaxTasks row chunks of about
// kDistEntries entries; one wave evaluates one chunk (lanes over columns,
// the chunk's rows in order) and writes six FP64 partial sums:
//   sum |d|, sum d^2, sum |d|^p, sum x^2, sum y^2, sum x y   (d = x - y).
// Three launches: a one-workgroup plan (chunk counts and their exclusive
// scan), the persistent chunk kernel, and a per-pair finish that adds the
// chunk partials in chunk order (the result does not depend on the grid).
#include <math.h>

#include "cfsim_internal.h"

namespace cfsim {

namespace {

constexpr int kPlanThreads = 1024;
constexpr int kWorkThreads = 256;
constexpr int kWorkWaves = kWorkThreads / kWave;
constexpr int kFinishThreads = 256;

__device__ inline bool pair_sizes(const SetRef& s, const int32_t* pa, const int32_t* pb, int q, int& ga, int& gb) {
    ga = pa[q];
    gb = pb[q];
    return ga >= 0 && ga < s.n_graphs && gb >= 0 && gb < s.n_graphs;
}

__device__ inline long long wave_scan_incl(long long v, int lane) {
    for (int o = 1; o < kWave; o <<= 1) {
        const long long u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
    }
    return v;
}

// Chunk counts T_q (0 for a pair with a graph index out of range or a graph
// above the set's max_nodes, whose chunks the workspace does not hold) and
// task_off[q] = T_0 + ... + T_{q-1}, task_off[n_pairs] = total.
__global__ __launch_bounds__(kPlanThreads) void dist_plan(SetRef set, const int32_t* pa, const int32_t* pb,
                                                          int n_pairs, int max_nodes, int64_t* task_off) {
    __shared__ long long wsum[kPlanThreads / kWave];
    __shared__ long long carry;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n_pairs; base += kPlanThreads) {
        const int q = base + tid;
        long long T = 0;
        int ga, gb;
        if (q < n_pairs && pair_sizes(set, pa, pb, q, ga, gb)) {
            const int nA = (int)(set.node_off[ga + 1] - set.node_off[ga]);
            const int nB = (int)(set.node_off[gb + 1] - set.node_off[gb]);
            const int M = nA > nB ? nA : nB;
            if (M <= max_nodes) T = dist_tasks(M);
        }
        const long long incl = wave_scan_incl(T, lane);
        if (lane == kWave - 1) wsum[wave] = incl;
        __syncthreads();
        long long before = carry;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (q < n_pairs) task_off[q] = before + incl - T;
        __syncthreads();
        if (tid == kPlanThreads - 1) carry = before + incl;
        __syncthreads();
    }
    if (tid == 0) task_off[n_pairs] = carry;
}

// Sum of X[a][b] R[j][b] over row a of X (repeated columns add up): R[j]
// has (1 - f) at column c0 and f at c1.  The row bounds are wave-uniform, so
// the column ids and weights are scalar loads shared by the wave; each lane
// compares them with its own c0, c1.
__device__ inline double interp_row(const int32_t* ci, const double* w, int t0, int t1, int c0, int c1, double f) {
    double s = 0.0;
    for (int t = t0; t < t1; ++t) {
        const int b = ci[t];
        const double v = w[t];
        s += b == c0 ? (1.0 - f) * v : (b == c1 ? f * v : 0.0);
    }
    return s;
}

// One chunk = rows [r0, r1) of one pair.  Lanes own columns j = jb + lane of
// a 64-column block (the column interpolation is computed once per block);
// the rows of the chunk are walked in order, wave-uniform, so every read of
// the CSR arrays is a scalar load shared by the wave.
template <bool P3>
__global__ __launch_bounds__(kWorkThreads) void dist_work(SetRef set, const int32_t* pa, const int32_t* pb,
                                                          int n_pairs, const int64_t* task_off, double p,
                                                          double* __restrict__ part) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const long long total = task_off[n_pairs];
    const long long stride = (long long)gridDim.x * kWorkWaves;
    for (long long t = (long long)blockIdx.x * kWorkWaves + wave; t < total; t += stride) {
        // The pair of chunk t: the last q with task_off[q] <= t (its T_q > 0).
        int lo = 0, hi = n_pairs;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (task_off[mid] <= t)
                lo = mid;
            else
                hi = mid;
        }
        const int q = lo;
        const int slot = (int)(t - task_off[q]);
        int ga, gb;
        pair_sizes(set, pa, pb, q, ga, gb);
        const GraphRef A = graph_of(set, ga), B = graph_of(set, gb);
        const GraphRef& L = A.n >= B.n ? A : B;
        const GraphRef& X = A.n >= B.n ? B : A;
        const int M = L.n, m = X.n;
        const int rows = dist_rows(M);
        const int r0 = slot * rows;
        const int r1 = r0 + rows < M ? r0 + rows : M;
        // Interpolation positions p (m - 1) / (M - 1) as quotient and
        // remainder of p (m - 1) by (M - 1); all zero when M = 1.
        const unsigned den = M > 1 ? (unsigned)(M - 1) : 1u;
        const unsigned mul = M > 1 ? (unsigned)(m - 1) : 0u;
        const double inv = 1.0 / (double)den;
        const unsigned num0 = (unsigned)r0 * mul;
        const int a00 = (int)(num0 / den);
        const unsigned rem00 = num0 - (unsigned)a00 * den;

        double s1 = 0.0, s2 = 0.0, sp = 0.0, sxx = 0.0, syy = 0.0, sxy = 0.0;
        for (int jb = 0; jb < M; jb += kWave) {
            const int j = jb + lane;
            const bool on = j < M;
            const unsigned numj = on ? (unsigned)j * mul : 0u;
            const int c0 = (int)(numj / den);
            const int c1 = c0 + 1 < m ? c0 + 1 : m - 1;
            const double fj = (double)(numj - (unsigned)c0 * den) * inv;
            const int jj = on ? j : -1;   // an idle lane matches no column
            int a0 = a00;
            unsigned rem = rem00;
            for (int i = r0; i < r1; ++i) {
                const int a1 = a0 + 1 < m ? a0 + 1 : m - 1;
                const double fi = (double)rem * inv;
                double x = 0.0;
                for (int e = L.rp[i], ee = L.rp[i + 1]; e < ee; ++e) x += L.ci[e] == jj ? L.w[e] : 0.0;
                double y = (1.0 - fi) * interp_row(X.ci, X.w, X.rp[a0], X.rp[a0 + 1], c0, c1, fj);
                if (rem != 0u) y += fi * interp_row(X.ci, X.w, X.rp[a1], X.rp[a1 + 1], c0, c1, fj);
                if (!on) y = 0.0;
                const double d = x - y;
                const double ad = fabs(d);
                s1 += ad;
                s2 += d * d;
                if (P3)
                    sp += ad * ad * ad;
                else if (ad != 0.0)
                    sp += pow(ad, p);
                sxx += x * x;
                syy += y * y;
                sxy += x * y;
                rem += mul;   // m <= M: the quotient grows by at most one per row
                if (rem >= den) {
                    rem -= den;
                    ++a0;
                }
            }
        }
        for (int o = kWave / 2; o > 0; o >>= 1) {
            s1 += __shfl_xor(s1, o, kWave);
            s2 += __shfl_xor(s2, o, kWave);
            sp += __shfl_xor(sp, o, kWave);
            sxx += __shfl_xor(sxx, o, kWave);
            syy += __shfl_xor(syy, o, kWave);
            sxy += __shfl_xor(sxy, o, kWave);
        }
        if (lane == 0) {
            double* o = part + t * kDistSums;
            o[0] = s1;
            o[1] = s2;
            o[2] = sp;
            o[3] = sxx;
            o[4] = syy;
            o[5] = sxy;
        }
    }
}

__global__ __launch_bounds__(kFinishThreads) void dist_finish(int n_pairs, const int64_t* task_off,
                                                              const double* part, double p, double* out) {
    const int q = blockIdx.x * kFinishThreads + threadIdx.x;
    if (q >= n_pairs) return;
    double* o = out + (long long)q * CFSIM_NUM_DISTANCES;
    const long long t0 = task_off[q], t1 = task_off[q + 1];
    if (t1 == t0) {
        for (int k = 0; k < CFSIM_NUM_DISTANCES; ++k) o[k] = __builtin_nan("");
        return;
    }
    double s[kDistSums] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (long long t = t0; t < t1; ++t)
        for (int k = 0; k < kDistSums; ++k) s[k] += part[t * kDistSums + k];
    const double denom = s[3] + s[4] - s[5];
    o[CFSIM_DIST_EUCLIDEAN] = sqrt(s[1]);
    o[CFSIM_DIST_MANHATTAN] = s[0];
    o[CFSIM_DIST_MINKOWSKI] = pow(s[2], 1.0 / p);
    o[CFSIM_DIST_JACCARD] = denom > 0.0 ? s[1] / denom : 0.0;
    o[CFSIM_DIST_COSINE] = s[3] > 0.0 && s[4] > 0.0 ? 1.0 - s[5] / (sqrt(s[3]) * sqrt(s[4])) : __builtin_nan("");
}

}  // namespace

long long dist_tasks_bound(int max_nodes) {
    long long best = 1;
    for (int M = 1; M <= max_nodes; ++M) {
        const long long T = dist_tasks(M);
        if (T > best) best = T;
    }
    return best;
}

int dist_grid(int num_cus) { return num_cus * 8; }

int launch_distances(const SetRef& set, int max_nodes, const int32_t* pa, const int32_t* pb, int n_pairs, double p,
                     double* out, int64_t* task_off, double* part, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(dist_plan, dim3(1), dim3(kPlanThreads), 0, stream, set, pa, pb, n_pairs, max_nodes, task_off);
    if (p == 3.0)
        hipLaunchKernelGGL(dist_work<true>, dim3(grid), dim3(kWorkThreads), 0, stream, set, pa, pb, n_pairs,
                           (const int64_t*)task_off, p, part);
    else
        hipLaunchKernelGGL(dist_work<false>, dim3(grid), dim3(kWorkThreads), 0, stream, set, pa, pb, n_pairs,
                           (const int64_t*)task_off, p, part);
    hipLaunchKernelGGL(dist_finish, dim3((n_pairs + kFinishThreads - 1) / kFinishThreads), dim3(kFinishThreads), 0,
                       stream, n_pairs, (const int64_t*)task_off, (const double*)part, p, out);
    return (int)hipGetLastError();
}

}  // namespace cfsim
