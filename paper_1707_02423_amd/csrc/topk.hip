// Step a11: the k best scores of a batch (query-vs-database ranking).
//
// Order: larger score first, ties to the lower index; NaN (invalid pairs)
// counts as -infinity.  Two launches: every block selects the k best of its
// contiguous range by k rounds of a block-wide argmax over an LDS copy, then
// one block selects the k best of the blocks' candidates the same way.
#include <float.h>
#include <limits.h>

#include "cfsim_internal.h"

namespace cfsim {

namespace {

constexpr int kTopkThreads = 1024;
constexpr int kTopkRange = 4096;  // elements per first-stage block

__device__ inline bool tk_better(double v, long long i, double bv, long long bi) {
    return v > bv || (v == bv && i < bi);
}

__device__ inline void tk_wave_argmax(double& v, long long& i, int& slot) {
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(v, o, kWave);
        const long long oi = __shfl_xor(i, o, kWave);
        const int os = __shfl_xor(slot, o, kWave);
        if (tk_better(ov, oi, v, i)) {
            v = ov;
            i = oi;
            slot = os;
        }
    }
}

// k rounds of argmax over vals/ids[0..m) in LDS; picked slots become -inf
// with index LLONG_MAX.  Results go to out_v/out_i[0..k).
__device__ void select_k(double* vals, long long* ids, int m, int k, double* out_v, long long* out_i,
                         double* wv, long long* wi, int* ws) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    constexpr int NW = kTopkThreads / kWave;
    for (int r = 0; r < k; ++r) {
        double bv = -__builtin_inf();
        long long bi = LLONG_MAX;
        int bs = -1;
        for (int t = tid; t < m; t += kTopkThreads) {
            if (tk_better(vals[t], ids[t], bv, bi)) {
                bv = vals[t];
                bi = ids[t];
                bs = t;
            }
        }
        tk_wave_argmax(bv, bi, bs);
        if (lane == 0) {
            wv[wave] = bv;
            wi[wave] = bi;
            ws[wave] = bs;
        }
        __syncthreads();
        if (tid == 0) {
            double v = wv[0];
            long long i = wi[0];
            int sl = ws[0];
            for (int w = 1; w < NW; ++w)
                if (tk_better(wv[w], wi[w], v, i)) {
                    v = wv[w];
                    i = wi[w];
                    sl = ws[w];
                }
            out_v[r] = v;
            out_i[r] = i;
            if (sl >= 0) {
                vals[sl] = -__builtin_inf();
                ids[sl] = LLONG_MAX;
            }
        }
        __syncthreads();
    }
}

struct TopkJob {
    const double* scores;
    long long n, stride;
    int k;
    double* cand_v;     // [blocks * k]
    long long* cand_i;  // [blocks * k]
    int32_t* idx_out;
    double* score_out;
};

__global__ __launch_bounds__(kTopkThreads) void topk_stage1(TopkJob J) {
    __shared__ double vals[kTopkRange];
    __shared__ long long ids[kTopkRange];
    __shared__ double wv[kTopkThreads / kWave];
    __shared__ long long wi[kTopkThreads / kWave];
    __shared__ int ws[kTopkThreads / kWave];
    const long long base = (long long)blockIdx.x * kTopkRange;
    const long long rem = J.n - base;
    const int m = rem < kTopkRange ? (int)rem : kTopkRange;
    for (int t = threadIdx.x; t < m; t += kTopkThreads) {
        double v = J.scores[(base + t) * J.stride];
        if (v != v) v = -__builtin_inf();
        vals[t] = v;
        ids[t] = base + t;
    }
    __syncthreads();
    const int kk = J.k < m ? J.k : m;
    select_k(vals, ids, m, kk, J.cand_v + (long long)blockIdx.x * J.k, J.cand_i + (long long)blockIdx.x * J.k, wv, wi,
             ws);
    // blocks with fewer than k elements pad their candidate list
    for (int r = kk + threadIdx.x; r < J.k; r += kTopkThreads) {
        J.cand_v[(long long)blockIdx.x * J.k + r] = -__builtin_inf();
        J.cand_i[(long long)blockIdx.x * J.k + r] = LLONG_MAX;
    }
}

__global__ __launch_bounds__(kTopkThreads) void topk_stage2(TopkJob J, int m) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* vals = reinterpret_cast<double*>(smem);
    long long* ids = reinterpret_cast<long long*>(smem + (size_t)m * 8);
    __shared__ double wv[kTopkThreads / kWave];
    __shared__ long long wi[kTopkThreads / kWave];
    __shared__ int ws[kTopkThreads / kWave];
    __shared__ double out_v[1024];
    __shared__ long long out_i[1024];
    for (int t = threadIdx.x; t < m; t += kTopkThreads) {
        vals[t] = J.cand_v[t];
        ids[t] = J.cand_i[t];
    }
    __syncthreads();
    select_k(vals, ids, m, J.k, out_v, out_i, wv, wi, ws);
    for (int r = threadIdx.x; r < J.k; r += kTopkThreads) {
        J.score_out[r] = out_v[r];
        J.idx_out[r] = out_i[r] == LLONG_MAX ? -1 : (int32_t)out_i[r];
    }
}

}  // namespace

long long topk_blocks(long long n) { return (n + kTopkRange - 1) / kTopkRange; }

int topk_max_k() { return 1024; }

size_t topk_stage2_lds(long long n, int k) { return (size_t)topk_blocks(n) * k * 16; }

int launch_topk(const double* scores, long long n, long long stride, int k, int32_t* idx_out, double* score_out,
                void* ws, hipStream_t stream) {
    TopkJob J;
    J.scores = scores;
    J.n = n;
    J.stride = stride;
    J.k = k;
    const long long blocks = topk_blocks(n);
    J.cand_v = static_cast<double*>(ws);
    J.cand_i = reinterpret_cast<long long*>(static_cast<unsigned char*>(ws) + (size_t)blocks * k * 8);
    J.idx_out = idx_out;
    J.score_out = score_out;
    hipLaunchKernelGGL(topk_stage1, dim3((unsigned)blocks), dim3(kTopkThreads), 0, stream, J);
    int e = (int)hipGetLastError();
    if (e != 0) return e;
    const int m = (int)(blocks * k);
    const size_t lds = (size_t)m * 16;
    if (lds > 64 * 1024) {
        e = (int)hipFuncSetAttribute(reinterpret_cast<const void*>(&topk_stage2),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != 0) return e;
    }
    hipLaunchKernelGGL(topk_stage2, dim3(1), dim3(kTopkThreads), lds, stream, J, m);
    return (int)hipGetLastError();
}

}  // namespace cfsim
