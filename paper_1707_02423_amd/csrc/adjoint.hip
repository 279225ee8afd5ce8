// Step a10: reverse mode through the coupled iteration.
//
// Forward (per pair, K = the forward's update count, matching held fixed):
//   Y_k = M S_k = B S_k A^T + B^T S_k A,  nu_k = ||Y_k||,  S_{k+1} = Y_k / nu_k,
//   score = <G, S_K> with G the indicator of the matching.
// Reverse, from Gbar = g_score * G:
//   Ybar = (Gbar - S_{k+1} <S_{k+1}, Gbar>) / nu_k
//   d w_A[p->q] += sum_{(i->u) in B} w_iu (Ybar[i][p] S_k[u][q] + S_k[i][p] Ybar[u][q])
//   d w_B[i->u] += sum_{(p->q) in A} w_pq (Ybar[i][p] S_k[u][q] + S_k[i][p] Ybar[u][q])
//   Gbar = M Ybar
// (the two edge sums are the entries of Ybar^T B S_k + S_k^T B Ybar and of
// Ybar A S_k^T + S_k A Ybar^T on the edges).  The forward is recomputed with S
// stored every `ckpt` updates; each segment is recomputed from its checkpoint
// before it is walked backwards.  One workgroup per pair; S, Ybar and Gbar
// live in a workspace slot (L2-resident), lists and gradient accumulators in
// LDS; gradients are added to grad_w with FP64 atomics (graphs may be shared).
#include "cfsim_internal.h"
#include "pair_device.h"

namespace cfsim {

namespace {

using namespace dev;

constexpr int kBwdThreads = 512;
constexpr int kBwdLds = 78 * 1024;
constexpr int kAChunks = 8;  // A edges held by the lanes (64 per chunk) in the lane-parallel edge sums

template <typename T>
__device__ inline T* slot_buf(T* base, long long slot_elems, int b) {
    return base + (size_t)b * (size_t)slot_elems;
}

// dst = scale * M src over all entries (R = B rows, C = A columns); returns
// sum of dst^2 (FP64, fixed order, same value in every thread).
template <typename T>
__device__ double apply_M(const T* src, T* dst, T scale, const PairShape& sh, const Lists<T>& G, double* red) {
    constexpr int NW = kBwdThreads / kWave;
    const int wave = uni((int)threadIdx.x / kWave);
    const int nR = sh.nR, nC = sh.nC, esz = (int)sizeof(T), rowb = nC * esz;
    const unsigned char* Sb = reinterpret_cast<const unsigned char*>(src);
    double nu2 = 0.0;
    for (int ch = 0; ch < sh.nchunk; ++ch) {
        LaneList<T> L[1];
        int col[1];
        bool cv[1];
        uint64_t ovf[1];
        lane_setup(G, ch, nC, L[0], col[0], cv[0], ovf[0]);
        for (int i = wave; i < nR; i += NW) {
            const RowRec<T> rr = G.rec[i];
            T y[1];
            update_row<T, 1>(Sb, rowb, i, rr, G, L, ovf, ovf[0] != 0, col, cv, y, ch);
            const T v = y[0] * scale;
            if (cv[0]) {
                dst[(long long)i * nC + col[0]] = v;
                nu2 += (double)v * (double)v;
            }
        }
    }
    return block_sum<NW>(nu2, red);
}

struct BwdJob {
    SetRef set;
    const int32_t* pair_a;
    const int32_t* pair_b;
    int n_pairs;
    const cfsim_pair_result* fwd;
    const int32_t* match;
    const int64_t* match_off;
    const double* grad_score;
    double* grad_w;
    int32_t* pair_status;  // optional: 0 done, CFSIM_INVALID_INPUT skipped
    int ckpt, max_iter;
    const void* fck;       // forward checkpoints (NULL: the forward is recomputed here)
    const int64_t* fck_off;
    void* ws;              // gridDim.x slots of slot_bytes
    long long slot_elems, slot_bytes;
    int32_t* queue;
};

__host__ __device__ inline int n_ckpt(int max_iter, int ckpt) { return max_iter / ckpt + 1; }

template <typename T>
__device__ void backward_pair(const BwdJob& J, int p, unsigned char* smem, double* red) {
    constexpr int NT = kBwdThreads;
    constexpr int NW = NT / kWave;
    const int tid = threadIdx.x;
    int32_t st = CFSIM_INVALID_INPUT;
    const int ga = J.pair_a[p], gb = J.pair_b[p];
    const cfsim_pair_result fr = J.fwd[p];
    const int K = fr.iters;
    bool ok = ga >= 0 && ga < J.set.n_graphs && gb >= 0 && gb < J.set.n_graphs && K >= 0 && K <= J.max_iter &&
              !(fr.status & CFSIM_INVALID_INPUT);
    GraphRef A{}, B{};
    PairShape sh{};
    size_t lists_bytes = 0;
    if (ok) {
        A = graph_of(J.set, ga);
        B = graph_of(J.set, gb);
        sh = make_shape(A.n, B.n, 0, NW);  // S kept as n_B x n_A: R = B, C = A
        lists_bytes = lds_lists_bytes(sh.nR, sh.nC, B.nnz, A.nnz, (int)sizeof(T));
        ok = A.n >= 1 && B.n >= 1 && (long long)A.n * B.n <= J.slot_elems &&
             lists_bytes + align16((size_t)(A.nnz + B.nnz) * 8) + align16((size_t)(A.nnz + B.nnz) * 4) <=
                 (size_t)kBwdLds;
    }
    if (!ok) {
        if (tid == 0 && J.pair_status) J.pair_status[p] = st;
        return;
    }
    st = 0;
    const double gs = J.grad_score[p];
    if ((fr.status & CFSIM_DEGENERATE) || K == 0 || gs == 0.0) {  // no dependence on the weights
        if (tid == 0 && J.pair_status) J.pair_status[p] = st;
        return;
    }
    const int nR = sh.nR, nC = sh.nC;  // nR = n_B, nC = n_A
    const long long E = (long long)nR * nC;
    const Lists<T> G = carve_lists<T>(smem, nR, nC, B.nnz, A.nnz);
    double* gA = reinterpret_cast<double*>(smem + lists_bytes);
    double* gB = gA + A.nnz;
    int* srcA = reinterpret_cast<int*>(smem + lists_bytes + align16((size_t)(A.nnz + B.nnz) * 8));
    int* srcB = srcA + A.nnz;
    const size_t scratch_off = lists_bytes + align16((size_t)(A.nnz + B.nnz) * 8) + align16((size_t)(A.nnz + B.nnz) * 4);
    const size_t scratch_bytes = (size_t)NW * kAChunks * kWave * sizeof(T);

    // workspace slot: checkpoints | segment (ckpt+1) | Ybar | Gbar | nu[max_iter]
    T* base = reinterpret_cast<T*>(static_cast<unsigned char*>(J.ws) + (size_t)blockIdx.x * J.slot_bytes);
    const int nck = n_ckpt(J.max_iter, J.ckpt);
    T* ck = base;
    T* seg = slot_buf(base, J.slot_elems, nck);
    T* Ybar = slot_buf(base, J.slot_elems, nck + J.ckpt + 1);
    T* Gbar = slot_buf(base, J.slot_elems, nck + J.ckpt + 2);
    double* nus = reinterpret_cast<double*>(slot_buf(base, J.slot_elems, nck + J.ckpt + 3));

    const T s0 = T(1.0 / sqrt((double)nR * (double)nC));
    (void)stage_pair<T, NT>(B, A, nR, nC, G, ck, s0);
    // edges kept by the packer (slots of dropped jumps, if any, follow them)
    const int keptA = uni(A.rp[A.n]), keptB = uni(B.rp[B.n]);
    for (int t = tid; t < A.nnz; t += NT) gA[t] = 0.0;
    for (int t = tid; t < B.nnz; t += NT) gB[t] = 0.0;
    for (int r = tid; r < A.n; r += NT)
        for (int t = A.rp[r]; t < A.rp[r + 1]; ++t) srcA[t] = r;
    for (int r = tid; r < B.n; r += NT)
        for (int t = B.rp[r]; t < B.rp[r + 1]; ++t) srcB[t] = r;
    __syncthreads();

    // ---- forward with checkpoints: S_0 = ck[0], S_{c * ckpt} = ck[c] (only
    // when the forward call left none: then its checkpoints are read below)
    const T* fwd_ck = J.fck ? reinterpret_cast<const T*>(J.fck) + J.fck_off[p] : nullptr;
    if (!fwd_ck) {
        const T* cur = ck;
        for (int k = 0; k < K; ++k) {
            T* dst = slot_buf(seg, J.slot_elems, k & 1);
            const double nu2 = apply_M(cur, dst, T(1), sh, G, red + (k & 1) * NW);
            const double nu = sqrt(nu2);
            if (tid == 0) nus[k] = nu;
            const T inv = T(1.0 / nu);
            const bool store = ((k + 1) % J.ckpt == 0) && (k + 1 < K);
            T* cdst = slot_buf(ck, J.slot_elems, (k + 1) / J.ckpt);
            for (long long t = tid; t < E; t += NT) {
                const T v = dst[t] * inv;
                dst[t] = v;
                if (store) cdst[t] = v;
            }
            __syncthreads();
            cur = dst;
        }
    }

    // ---- edge sums with lanes over A edges need a per-wave scratch of their
    // per-step partials (at most kAChunks * 64 A edges; otherwise the
    // thread-per-edge loops below)
    const int wave = uni(tid / kWave);
    const int nchA = (keptA + kWave - 1) / kWave;
    T* part = reinterpret_cast<T*>(smem + scratch_off);
    const bool lane_edges = nchA <= kAChunks && scratch_off + scratch_bytes <= (size_t)kBwdLds;

    // ---- reverse: Gbar = g * indicator(matching)
    const int64_t mo = J.match_off ? J.match_off[p] : 0;
    for (long long t = tid; t < E; t += NT) Gbar[t] = T(0);
    __syncthreads();
    for (int i = tid; i < nR; i += NT) {
        const int j = J.match[mo + i];
        if (j >= 0 && j < nC) Gbar[(long long)i * nC + j] = T(gs);
    }
    __syncthreads();
    for (int s0i = ((K - 1) / J.ckpt) * J.ckpt; s0i >= 0; s0i -= J.ckpt) {
        const int s1 = min(s0i + J.ckpt, K);
        // recompute S_{s0i+1 .. s1} into seg[1 ..] from the segment's first
        // iterate (S_0, or a checkpoint), with nu_k of every update
        const T* Sfirst = (s0i == 0 || !fwd_ck) ? slot_buf(ck, J.slot_elems, s0i / J.ckpt)
                                                : fwd_ck + (long long)(s0i / J.ckpt - 1) * E;
        for (int k = s0i; k < s1; ++k) {
            const T* src = k == s0i ? Sfirst : slot_buf(seg, J.slot_elems, k - s0i);
            T* dst = slot_buf(seg, J.slot_elems, k + 1 - s0i);
            const double nu = sqrt(apply_M(src, dst, T(1), sh, G, red + (k & 1) * NW));
            if (tid == 0) nus[k] = nu;
            const T inv = T(1.0 / nu);
            for (long long t = tid; t < E; t += NT) dst[t] *= inv;
            __syncthreads();
        }
        for (int k = s1 - 1; k >= s0i; --k) {
            const T* Sk = k == s0i ? Sfirst : slot_buf(seg, J.slot_elems, k - s0i);
            const T* Sk1 = slot_buf(seg, J.slot_elems, k + 1 - s0i);
            double dot = 0.0;
            for (long long t = tid; t < E; t += NT) dot += (double)Sk1[t] * (double)Gbar[t];
            dot = block_sum<NW>(dot, red + 2 * NW);
            const T a = T(dot);
            const T invnu = T(1.0 / nus[k]);  // written by thread 0 before a barrier of the recompute
            for (long long t = tid; t < E; t += NT) Ybar[t] = (Gbar[t] - a * Sk1[t]) * invnu;
            __syncthreads();
            // edge gradients: every pair of a B edge f = (i -> u) and an A edge
            // e = (p -> q) has the summand c = Ybar[i][p] S[u][q] + S[i][p] Ybar[u][q];
            // dA[e] += w_f c and dB[f] += w_e c
            if (lane_edges) {
                // wave w: B edges f = w, w + NW, ...; lane l: A edges e = l + 64 ch;
                // dB[f] is a wave sum, dA[e] the waves' partials summed in wave order
                const int lane = tid & (kWave - 1);
                int ep[kAChunks], eq[kAChunks];
                T ew[kAChunks], accA[kAChunks];
#pragma unroll
                for (int ch = 0; ch < kAChunks; ++ch) {
                    const int e = ch * kWave + lane;
                    const bool has = e < keptA;  // absent edges read entry 0 with weight 0
                    ep[ch] = has ? srcA[e] : 0;
                    eq[ch] = has ? A.ci[e] : 0;
                    ew[ch] = has ? T(A.w[e]) : T(0);
                    accA[ch] = T(0);
                }
                for (int f = wave; f < keptB; f += NW) {
                    const int i = uni(srcB[f]), u = uni(B.ci[f]);
                    const T wf = T(B.w[f]);
                    const T* Yi = Ybar + (long long)i * nC;
                    const T* Yu = Ybar + (long long)u * nC;
                    const T* Si = Sk + (long long)i * nC;
                    const T* Su = Sk + (long long)u * nC;
                    T pb = T(0);
#pragma unroll
                    for (int ch = 0; ch < kAChunks; ++ch) {
                        if (ch < nchA) {
                            const T c = Yi[ep[ch]] * Su[eq[ch]] + Si[ep[ch]] * Yu[eq[ch]];
                            accA[ch] = fma_t(wf, c, accA[ch]);
                            pb = fma_t(ew[ch], c, pb);
                        }
                    }
                    const double sb = wave_sum((double)pb);
                    if (lane == 0) gB[f] += sb;
                }
#pragma unroll
                for (int ch = 0; ch < kAChunks; ++ch)
                    if (ch < nchA) part[(wave * kAChunks + ch) * kWave + lane] = accA[ch];
                __syncthreads();
                for (int e = tid; e < keptA; e += NT) {
                    double a = 0.0;
                    for (int w = 0; w < NW; ++w) a += (double)part[(w * kAChunks + e / kWave) * kWave + (e % kWave)];
                    gA[e] += a;
                }
            } else for (int e = tid; e < keptA; e += NT) {
                const int pa = srcA[e], qa = A.ci[e];
                T acc = T(0);
                for (int f = 0; f < keptB; ++f) {
                    const int i = srcB[f], u = B.ci[f];
                    const T c = Ybar[(long long)i * nC + pa] * Sk[(long long)u * nC + qa] +
                                Sk[(long long)i * nC + pa] * Ybar[(long long)u * nC + qa];
                    acc = fma_t(T(B.w[f]), c, acc);
                }
                gA[e] += (double)acc;
            }
            if (!lane_edges) for (int f = tid; f < keptB; f += NT) {
                const int i = srcB[f], u = B.ci[f];
                T acc = T(0);
                for (int e = 0; e < keptA; ++e) {
                    const int pa = srcA[e], qa = A.ci[e];
                    const T c = Ybar[(long long)i * nC + pa] * Sk[(long long)u * nC + qa] +
                                Sk[(long long)i * nC + pa] * Ybar[(long long)u * nC + qa];
                    acc = fma_t(T(A.w[e]), c, acc);
                }
                gB[f] += (double)acc;
            }
            __syncthreads();  // gB of this step complete; Ybar and Gbar are rewritten next
            // Gbar = M Ybar
            (void)apply_M(Ybar, Gbar, T(1), sh, G, red + (k & 1) * NW);
        }
    }
    const int64_t ea = J.set.edge_off[ga], eb = J.set.edge_off[gb];
    for (int e = tid; e < keptA; e += NT) atomicAdd(J.grad_w + ea + e, gA[e]);
    for (int f = tid; f < keptB; f += NT) atomicAdd(J.grad_w + eb + f, gB[f]);
    if (tid == 0 && J.pair_status) J.pair_status[p] = st;
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kBwdThreads) __attribute__((amdgpu_waves_per_eu(4)))
void backward_kernel(BwdJob J) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[4 * (kBwdThreads / kWave)];
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(J.queue, 1);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= J.n_pairs) break;
        backward_pair<T>(J, item, smem, red);
    }
}

__global__ void zero_kernel(int32_t* q) { *q = 0; }

}  // namespace

long long backward_slot_bytes(int max_iter, int ckpt, long long slot_elems, int esize) {
    const long long bufs = n_ckpt(max_iter, ckpt) + ckpt + 3;
    const long long b = bufs * slot_elems * esize + (long long)(max_iter + 1) * 8;
    return (b + 255) & ~255ll;
}

int backward_grid(int num_cus) { return num_cus * 2; }

int launch_backward(int dtype, const SetRef& set, const int32_t* pair_a, const int32_t* pair_b, int n_pairs,
                    const cfsim_pair_result* fwd, const int32_t* match, const int64_t* match_off,
                    const double* grad_score, double* grad_w, int32_t* pair_status, int ckpt,
                    const void* fck, const int64_t* fck_off, int max_iter,
                    void* ws, long long slot_elems, int grid, hipStream_t stream) {
    BwdJob J;
    J.set = set;
    J.pair_a = pair_a;
    J.pair_b = pair_b;
    J.n_pairs = n_pairs;
    J.fwd = fwd;
    J.match = match;
    J.match_off = match_off;
    J.grad_score = grad_score;
    J.grad_w = grad_w;
    J.pair_status = pair_status;
    J.ckpt = ckpt;
    J.max_iter = max_iter;
    J.fck = fck;
    J.fck_off = fck_off;
    const int esize = dtype == CFSIM_F64 ? 8 : 4;
    J.slot_elems = slot_elems;
    J.slot_bytes = backward_slot_bytes(max_iter, ckpt, slot_elems, esize);
    // queue counter in front of the slots
    J.queue = static_cast<int32_t*>(ws);
    J.ws = static_cast<unsigned char*>(ws) + 256;
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(1), 0, stream, J.queue);
    int e = (int)hipGetLastError();
    if (e != 0) return e;
    const void* f = dtype == CFSIM_F64 ? reinterpret_cast<const void*>(&backward_kernel<double>)
                                       : reinterpret_cast<const void*>(&backward_kernel<float>);
    e = (int)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kBwdLds);
    if (e != 0) return e;
    void* args[] = {&J};
    return (int)hipLaunchKernel(f, dim3(grid), dim3(kBwdThreads), args, kBwdLds, stream);
}

}  // namespace cfsim
