// Optimal-assignment matching of similarity matrices: for each S (n_rows x
// n_cols) the matching of min(n_rows, n_cols) pairs with the largest total
// sum S_ij, by the Hungarian method in its shortest-augmenting-path form
// (row potentials u, column potentials v).  With the cost C = -S, transposed
// when S has more rows than columns so that C is n x m with n <= m, rows of C
// are inserted one at a time: a Dijkstra tree over the columns grows on the
// reduced costs C[i][j] - u[i] - v[j] until it reaches a free column; each
// step shifts the potentials by the smallest slack of the tree, and the
// matching is then flipped along the path.  Ties go to the smallest column.
//
// Work mapping: one wave per matrix (64-thread workgroups, one matrix after
// another from a grid-stride loop); lanes own columns j = 1 + lane, 65 + lane,
// ...; the tree's state (potentials, slacks, back pointers, tree marks, the
// column -> row matching) lives in LDS, sized by the call's largest
// dimension.  A step reads one row of C (a contiguous row of S, or a strided
// column when transposed) and ends with one wave argmin, so an insertion
// costs (tree steps) x (m / 64) lane iterations.  All arithmetic is FP64 in
// the order the method states it, so the result does not depend on the launch.
#include <limits.h>
#include <math.h>

#include "cfsim_internal.h"
#include "pair_device.h"

namespace cfsim {

namespace {

using namespace dev;

constexpr int kAssignThreads = kWave;

struct AssignJob {
    const void* S;
    const int64_t* S_off;
    const int32_t* n_rows;
    const int32_t* n_cols;
    int n_pairs;
    int max_dim;
    int32_t* match;
    const int64_t* match_off;
    double* score;
};

// C[r][c] of the cost matrix (rows of C = columns of S when transposed); the
// row stride of S is its column count in both cases.
template <typename T>
__device__ inline double cost_at(const T* S, long long ld, bool tr, int r, int c) {
    return -(double)(tr ? S[(long long)c * ld + r] : S[(long long)r * ld + c]);
}

template <typename T>
__global__ __launch_bounds__(kAssignThreads) void assign_kernel(AssignJob J) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = J.max_dim + 1;
    double* u = reinterpret_cast<double*>(smem);  // [n + 1] row potentials
    double* v = u + L;                            // [m + 1] column potentials
    double* minv = v + L;                         // [m + 1] slack of each column
    int* col_row = reinterpret_cast<int*>(minv + L);  // [m + 1] row on column j (1-based, 0 free)
    int* way = col_row + L;                       // [m + 1] previous column on the tree path
    int* used = way + L;                          // [m + 1] column in the tree
    const int lane = threadIdx.x;
    const double inf = __builtin_inf();
    for (int p = blockIdx.x; p < J.n_pairs; p += gridDim.x) {
        const int nr = J.n_rows[p], nc = J.n_cols[p];
        const int64_t mo = J.match ? J.match_off[p] : 0;
        const bool dims_ok = nr >= 1 && nc >= 1 && nr <= J.max_dim && nc <= J.max_dim;
        const T* S = reinterpret_cast<const T*>(J.S) + (dims_ok ? J.S_off[p] : 0);
        int bad = !dims_ok;
        if (dims_ok)
            for (long long t = lane; t < (long long)nr * nc; t += kWave) bad |= !isfinite((double)S[t]);
        if (__ballot(bad) != 0) {  // every lane takes this exit
            if (J.match && nr >= 1)
                for (int r = lane; r < nr; r += kWave) J.match[mo + r] = -1;
            if (lane == 0) J.score[p] = __builtin_nan("");
            continue;
        }
        const bool tr = nr > nc;
        const int n = tr ? nc : nr, m = tr ? nr : nc;
        for (int j = lane; j <= m; j += kWave) {
            v[j] = 0.0;
            col_row[j] = 0;
            way[j] = 0;
        }
        for (int i = lane; i <= n; i += kWave) u[i] = 0.0;
        __syncthreads();
        // set if a step finds no column (only possible when reduced costs
        // overflow): the matrix is then reported like a non-finite one
        bool failed = false;
        for (int i = 1; i <= n && !failed; ++i) {
            for (int j = lane; j <= m; j += kWave) {
                minv[j] = inf;
                used[j] = 0;
            }
            if (lane == 0) col_row[0] = i;
            int j0 = 0;
            __syncthreads();
            for (;;) {
                if (lane == 0) used[j0] = 1;
                __syncthreads();
                const int i0 = uni(col_row[j0]);
                const double ui0 = u[i0];
                double bv = -inf;  // best -slack of the lane (argmax of -slack = argmin of slack)
                int bk = INT_MAX, bc = 0;
                for (int j = 1 + lane; j <= m; j += kWave) {
                    if (used[j]) continue;
                    const double cur = cost_at<T>(S, nc, tr, i0 - 1, j - 1) - ui0 - v[j];
                    double mj = minv[j];
                    if (cur < mj) {
                        mj = cur;
                        minv[j] = cur;
                        way[j] = j0;
                    }
                    if (better(-mj, j, bv, bk)) {
                        bv = -mj;
                        bk = j;
                    }
                }
                wave_argmax(bv, bk, bc);
                const double delta = -bv;
                const int j1 = bk;
                if (j1 < 1 || j1 > m) {
                    failed = true;
                    break;
                }
                for (int j = lane; j <= m; j += kWave) {
                    if (used[j]) {
                        u[col_row[j]] += delta;
                        v[j] -= delta;
                    } else {
                        minv[j] -= delta;
                    }
                }
                __syncthreads();
                j0 = j1;
                if (uni(col_row[j0]) == 0) break;
            }
            if (failed) break;
            if (lane == 0) {  // flip the matching along the path back to the root column
                while (j0 != 0) {
                    const int j1 = way[j0];
                    col_row[j0] = col_row[j1];
                    j0 = j1;
                }
            }
            __syncthreads();
        }
        if (failed) {
            if (J.match)
                for (int r = lane; r < nr; r += kWave) J.match[mo + r] = -1;
            if (lane == 0) J.score[p] = __builtin_nan("");
            __syncthreads();
            continue;
        }
        // rows of S -> columns of S (way[] is free now and holds it)
        int* row_match = way;
        for (int r = lane; r < nr; r += kWave) row_match[r] = -1;
        __syncthreads();
        for (int j = 1 + lane; j <= m; j += kWave) {
            const int r = col_row[j];
            if (r == 0) continue;
            if (tr)
                row_match[j - 1] = r - 1;
            else
                row_match[r - 1] = j - 1;
        }
        __syncthreads();
        double sc = 0.0;
        for (int r = lane; r < nr; r += kWave) {
            const int c = row_match[r];
            if (c >= 0) sc += (double)S[(long long)r * nc + c];
            if (J.match) J.match[mo + r] = c;
        }
        sc = wave_sum(sc);
        if (lane == 0) J.score[p] = sc;
        __syncthreads();  // the LDS state is reset by the next matrix
    }
}

}  // namespace

size_t assign_lds_bytes(int max_dim) { return (size_t)(max_dim + 1) * (3 * sizeof(double) + 3 * sizeof(int)); }

int launch_assign(int dtype, const void* S, const int64_t* S_off, const int32_t* n_rows, const int32_t* n_cols,
                  int n_pairs, int max_dim, int32_t* match, const int64_t* match_off, double* score, int grid,
                  hipStream_t stream) {
    AssignJob J{S, S_off, n_rows, n_cols, n_pairs, max_dim, match, match_off, score};
    const void* k = dtype == CFSIM_F64 ? reinterpret_cast<const void*>(&assign_kernel<double>)
                                       : reinterpret_cast<const void*>(&assign_kernel<float>);
    const size_t lds = assign_lds_bytes(max_dim);
    int e = (int)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != 0) return e;
    void* args[] = {&J};
    return (int)hipLaunchKernel(k, dim3(grid), dim3(kAssignThreads), args, lds, stream);
}

}  // namespace cfsim
