// Ward's minimum-variance clustering (Section 6.2, "Clustering of Kernels")
// of n observations with f features each: squared Euclidean distances
// d_ij = ||X_i - X_j||^2, then n - 1 merges, each of the pair of current
// clusters with the smallest distance (ties: smaller slot pair), the merged
// cluster's distances following the Lance-Williams recurrence of Ward's method
// on squared distances,
//   d(k, i u j) = ((n_i + n_k) d_ki + (n_j + n_k) d_kj - n_k d_ij) / (n_i + n_j + n_k).
//
// Two kernels.  ward_distances fills the n x n matrix in the workspace (16 x 16
// pairs per workgroup, features staged through LDS 32 at a time, each sum
// taken in feature order).  ward_merge is one 1024-thread workgroup that keeps
// every slot's nearest neighbour (distance, index) in LDS: a merge step is a
// block argmin over the slots' cached neighbours, the recurrence for the
// merged slot's row and column (one thread per slot), and the neighbour
// refresh: slots whose neighbour was one of the merged pair (and the merged
// slot) rescan their rows, one wave per row; every other slot only compares
// its cached neighbour with the merged slot.  Under the tie rule the cached
// minimum over slots is the same pair the definition picks by scanning all
// pairs.  Arithmetic is FP64 without fused multiply-adds, in the order the
// definition states it, so heights are reproducible to the last bit.
#include <limits.h>
#include <math.h>

#include "cfsim_internal.h"
#include "pair_device.h"

namespace cfsim {

namespace {

using namespace dev;

constexpr int kDistTile = 16;
constexpr int kFeatTile = 32;
constexpr int kMergeThreads = 1024;
constexpr int kMergeWaves = kMergeThreads / kWave;

#pragma clang fp contract(off)

__global__ __launch_bounds__(kDistTile * kDistTile) void ward_distances(const double* __restrict__ X, int n, int f,
                                                                        double* __restrict__ D) {
    __shared__ double xi[kDistTile][kFeatTile + 1];
    __shared__ double xj[kDistTile][kFeatTile + 1];
    const int tx = threadIdx.x % kDistTile, ty = threadIdx.x / kDistTile;
    const int i0 = blockIdx.y * kDistTile, j0 = blockIdx.x * kDistTile;
    const int i = i0 + ty, j = j0 + tx;
    double d = 0.0;
    for (int k0 = 0; k0 < f; k0 += kFeatTile) {
        for (int t = threadIdx.x; t < kDistTile * kFeatTile; t += kDistTile * kDistTile) {
            const int r = t / kFeatTile, k = k0 + t % kFeatTile;
            const double a = (i0 + r < n && k < f) ? X[(long long)(i0 + r) * f + k] : 0.0;
            const double b = (j0 + r < n && k < f) ? X[(long long)(j0 + r) * f + k] : 0.0;
            xi[r][t % kFeatTile] = a;
            xj[r][t % kFeatTile] = b;
        }
        __syncthreads();
        const int kn = f - k0 < kFeatTile ? f - k0 : kFeatTile;
        for (int k = 0; k < kn; ++k) {
            const double t = xi[ty][k] - xj[tx][k];
            d = d + t * t;
        }
        __syncthreads();
    }
    if (i < n && j < n) D[(long long)i * n + j] = d;
}

// Distance from slot k to the union of slots i and j.
__device__ inline double ward_update(double dki, double dkj, double dij, double ni, double nj, double nk) {
    return ((ni + nk) * dki + (nj + nk) * dkj - nk * dij) / (ni + nj + nk);
}

// Nearest active slot of row k (smallest distance, then smallest index) by one
// wave; (inf, INT_MAX) if no other slot is active.
__device__ inline void row_nearest(const double* D, int n, int k, const int* active, double& bd, int& bj) {
    double v = -__builtin_inf();
    int key = INT_MAX, c = 0;
    const double* row = D + (long long)k * n;
    for (int j = threadIdx.x % kWave; j < n; j += kWave) {
        if (j == k || !active[j]) continue;
        const double x = -row[j];
        if (better(x, j, v, key)) {
            v = x;
            key = j;
        }
    }
    wave_argmax(v, key, c);
    bd = -v;
    bj = key;
}

__global__ __launch_bounds__(kMergeThreads) void ward_merge(const double* X, int f, double* D, int n, double* Z) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* nnd = reinterpret_cast<double*>(smem);  // [n] distance to the nearest active slot
    double* size = nnd + n;                         // [n] observations in the slot's cluster
    double* ident = size + n;                       // [n] cluster number of the slot
    int* nn = reinterpret_cast<int*>(ident + n);    // [n] nearest active slot
    int* active = nn + n;                           // [n]
    int* todo = active + n;                         // [n] slots to rescan
    __shared__ double wv[kMergeWaves];
    __shared__ int wk[kMergeWaves];
    __shared__ int ntodo;
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    int nonfinite = 0;
    for (long long t = tid; t < (long long)n * f; t += kMergeThreads) nonfinite |= !isfinite(X[t]);
    if (__syncthreads_or(nonfinite)) {  // a non-finite feature: every row of the linkage is NaN
        for (long long t = tid; t < 4ll * (n - 1); t += kMergeThreads) Z[t] = __builtin_nan("");
        return;
    }
    for (int k = tid; k < n; k += kMergeThreads) {
        size[k] = 1.0;
        ident[k] = (double)k;
        active[k] = 1;
    }
    __syncthreads();
    for (int k = wave; k < n; k += kMergeWaves) {
        double bd;
        int bj;
        row_nearest(D, n, k, active, bd, bj);
        if (lane == 0) {
            nnd[k] = bd;
            nn[k] = bj;
        }
    }
    __syncthreads();
    for (int s = 0; s < n - 1; ++s) {
        // the active slot with the nearest neighbour (distance, then slot)
        double v = -__builtin_inf();
        int key = INT_MAX, c = 0;
        for (int k = tid; k < n; k += kMergeThreads)
            if (active[k] && better(-nnd[k], k, v, key)) {
                v = -nnd[k];
                key = k;
            }
        wave_argmax(v, key, c);
        if (lane == 0) {
            wv[wave] = v;
            wk[wave] = key;
        }
        __syncthreads();
        v = wv[0];
        key = wk[0];
        for (int w = 1; w < kMergeWaves; ++w)
            if (better(wv[w], wk[w], v, key)) {
                v = wv[w];
                key = wk[w];
            }
        const int r = key, q = nn[r];
        const int i = r < q ? r : q, j = r < q ? q : r;
        const double dij = -v;
        const double ni = size[i], nj = size[j];
        if (tid == 0) {
            const double a = ident[i], b = ident[j];
            Z[4ll * s + 0] = a < b ? a : b;
            Z[4ll * s + 1] = a < b ? b : a;
            Z[4ll * s + 2] = dij;
            Z[4ll * s + 3] = ni + nj;
            ntodo = 0;
        }
        for (int k = tid; k < n; k += kMergeThreads) {
            if (!active[k] || k == i || k == j) continue;
            const double d = ward_update(D[(long long)k * n + i], D[(long long)k * n + j], dij, ni, nj, size[k]);
            D[(long long)k * n + i] = d;
            D[(long long)i * n + k] = d;
        }
        __syncthreads();
        if (tid == 0) {
            size[i] = ni + nj;
            active[j] = 0;
            ident[i] = (double)(n + s);
        }
        __syncthreads();
        for (int k = tid; k < n; k += kMergeThreads) {
            if (!active[k]) continue;
            if (k == i || nn[k] == i || nn[k] == j) {
                todo[atomicAdd(&ntodo, 1)] = k;
            } else {
                const double d = D[(long long)k * n + i];
                if (d < nnd[k] || (d == nnd[k] && i < nn[k])) {
                    nnd[k] = d;
                    nn[k] = i;
                }
            }
        }
        __syncthreads();
        const int nt = ntodo;
        for (int t = wave; t < nt; t += kMergeWaves) {
            const int k = todo[t];
            double bd;
            int bj;
            row_nearest(D, n, k, active, bd, bj);
            if (lane == 0) {
                nnd[k] = bd;
                nn[k] = bj;
            }
        }
        __syncthreads();
    }
}

}  // namespace

size_t ward_merge_lds(int n) { return (size_t)n * (3 * sizeof(double) + 3 * sizeof(int)); }

int launch_ward(const double* X, int n, int f, double* Z, double* D, hipStream_t stream) {
    const int tiles = (n + kDistTile - 1) / kDistTile;
    hipLaunchKernelGGL(ward_distances, dim3(tiles, tiles), dim3(kDistTile * kDistTile), 0, stream, X, n, f, D);
    int e = (int)hipGetLastError();
    if (e != 0) return e;
    const size_t lds = ward_merge_lds(n);
    if ((e = (int)hipFuncSetAttribute(reinterpret_cast<const void*>(&ward_merge),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != 0)
        return e;
    hipLaunchKernelGGL(ward_merge, dim3(1), dim3(kMergeThreads), lds, stream, X, f, D, n, Z);
    return (int)hipGetLastError();
}

}  // namespace cfsim
