// Step a9: large pairs (hundreds to thousands of nodes per graph).
//
// S no longer fits a workgroup's LDS, so every update is one grid-wide launch
// over tiles of all pairs of the call, with S in HBM (the MI355X last-level
// cache holds a pair's working set).  The host captures the sequence
//   large_init, large_scan, large_step(k) for k = 1 .. max_iter + 1, large_finish
// into one HIP graph.  Per pair four buffers rotate: launch k reads
// Y_{k-1} (with the scale sigma_{k-1} = 1 / nu_{k-1} folded into the update,
// so no separate normalisation pass runs) and writes the un-normalised
// Y_k = M S_{k-1}.  The even-step change delta_{k-1} = ||S_{k-1} - S_{k-3}||
// is accumulated by the odd launch k, which is the first one that knows both
// scales.  The last workgroup to finish a pair's tiles in a launch (counted
// with a device-scope atomic) reduces the pair's per-tile FP64 partials in
// tile order, so the reductions are deterministic.  Launch max_iter + 1 only
// computes the final even-step change.  large_finish rescales the final
// iterate in place and runs the greedy matching with one workgroup per pair.
#include "cfsim_internal.h"
#include "pair_device.h"

namespace cfsim {

namespace {

using dev::better;
using dev::uni;
using dev::wave_argmax;
using dev::wave_sum;

constexpr int kTileRows = 32;                   // rows of Y per tile
constexpr int kStepThreads = 256;               // 4 waves, 8 rows each
constexpr int kRowsPerWave = kTileRows / (kStepThreads / kWave);
constexpr int kFinishThreads = 1024;
constexpr int kLS = 2;                          // successors per lane column in registers
constexpr int kLP = 3;                          // predecessors per lane column in registers

__device__ inline int tiles_of(int nA, int nB) { return ((nB + kTileRows - 1) / kTileRows) * ((nA + 63) / 64); }
static_assert(kTileRows == 32, "large_tiles() in cfsim_internal.h assumes 32-row tiles");

// Pair p's buffer b (0..3) of slot_elems elements.
template <typename T>
__device__ inline T* buf_of(const LargeJob& J, int p, int b) {
    return reinterpret_cast<T*>(J.bufs) + ((long long)p * 4 + b) * J.slot_elems;
}

__device__ inline int pair_of_tile(const LargeJob& J, long long t) {
    int lo = 0, hi = J.n_pairs;  // largest p with tile_off[p] <= t
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (J.tile_off[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------- set-up
// One workgroup per pair: validity, degeneracy, tile count, initial state.
__global__ __launch_bounds__(256) void large_init(LargeJob J) {
    const int p = blockIdx.x;
    __shared__ int pos[2];
    const int ga = J.pair_a[p], gb = J.pair_b[p];
    LargeState* s = J.st + p;
    const bool ok_ids = ga >= 0 && ga < J.set.n_graphs && gb >= 0 && gb < J.set.n_graphs;
    int nA = 0, nB = 0;
    GraphRef A{}, B{};
    if (ok_ids) {
        A = graph_of(J.set, ga);
        B = graph_of(J.set, gb);
        nA = A.n;
        nB = B.n;
    }
    const bool ok = ok_ids && nA >= 1 && nB >= 1 && (long long)nA * nB <= J.slot_elems && nA <= J.max_nodes &&
                    nB <= J.max_nodes;
    if (threadIdx.x < 2) pos[threadIdx.x] = 0;
    __syncthreads();
    if (ok) {
        for (int e = threadIdx.x; e < A.nnz; e += 256)
            if (A.w[e] > 0.0) pos[0] = 1;
        for (int e = threadIdx.x; e < B.nnz; e += 256)
            if (B.w[e] > 0.0) pos[1] = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s->nA = nA;
        s->nB = nB;
        s->ntiles = ok ? tiles_of(nA, nB) : 0;
        s->active = (ok && pos[0] && pos[1]) ? 1 : 0;
        s->status = !ok ? CFSIM_INVALID_INPUT : (s->active ? 0u : (unsigned)CFSIM_DEGENERATE);
        s->final_step = 0;
        s->nu = 0.0;
        s->delta = __builtin_inf();
        for (int b = 0; b < 4; ++b) s->nu_k[b] = 1.0;
        J.done[p] = 0;
    }
}

// Exclusive scan of the pairs' tile counts (one workgroup).
__global__ __launch_bounds__(1024) void large_scan(LargeJob J) {
    __shared__ long long part[1024];
    const int tid = threadIdx.x;
    const int per = (J.n_pairs + 1023) / 1024;
    const int lo = min(tid * per, J.n_pairs), hi = min(lo + per, J.n_pairs);
    long long sum = 0;
    for (int p = lo; p < hi; ++p) sum += J.st[p].ntiles;
    part[tid] = sum;
    __syncthreads();
    if (tid == 0) {
        long long run = 0;
        for (int i = 0; i < 1024; ++i) {
            const long long t = part[i];
            part[i] = run;
            run += t;
        }
        J.tile_off[J.n_pairs] = run;
    }
    __syncthreads();
    long long run = part[tid];
    for (int p = lo; p < hi; ++p) {
        J.tile_off[p] = run;
        run += J.st[p].ntiles;
    }
}

// ---------------------------------------------------------------- one update
// Launch k (1 .. max_iter): Y_k = M (Y_{k-1} / nu_{k-1}) into buffer k % 4
// (S_0 is the constant 1/sqrt(n_A n_B)); at odd k >= 3 also the partial
// squares of S_{k-1} - S_{k-3}.  Launch max_iter + 1 computes only the latter.
template <typename T>
__global__ __launch_bounds__(kStepThreads) void large_step(LargeJob J, int k) {
    __shared__ double red[2][kStepThreads / kWave];
    __shared__ int last_flag;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const bool compute = k <= J.max_iter;
    const bool want_delta = (k & 1) && k >= 3;
    const long long total = J.tile_off[J.n_pairs];
    // XCD-aware order: workgroups are dealt to the 8 XCDs round-robin, so the
    // workgroups of one XCD take one contiguous range of tiles (neighbouring
    // row strips of one pair share S rows through that XCD's L2).
    const int G = gridDim.x;
    const int xcd = blockIdx.x & 7, per_xcd = G >> 3, y = blockIdx.x >> 3;
    const long long lo = total * xcd / 8, hi = total * (xcd + 1) / 8;
    for (long long t = lo + y; t < hi; t += per_xcd) {
        const int p = uni(pair_of_tile(J, t));
        LargeState* s = J.st + p;
        if (!uni(s->active)) continue;
        const int nA = s->nA, nB = s->nB;
        const int lt = (int)(t - J.tile_off[p]);
        const int nct = (nA + 63) / 64;
        const int r0 = (lt / nct) * kTileRows, c0 = (lt % nct) * 64;
        const GraphRef A = graph_of(J.set, J.pair_a[p]);
        const GraphRef B = graph_of(J.set, J.pair_b[p]);
        const int j = c0 + lane;
        const bool colv = j < nA;
        const T* src = buf_of<T>(J, p, (k - 1) & 3);
        T* dst = buf_of<T>(J, p, k & 3);
        const T* old = buf_of<T>(J, p, (k - 3) & 3);
        const T c0v = T(1.0 / sqrt((double)nA * (double)nB));
        const T sig = T(1.0 / s->nu_k[(k - 1) & 3]);     // sigma_{k-1} (1 for S_0)
        const T sig3 = T(1.0 / s->nu_k[(k - 3) & 3]);    // sigma_{k-3}
        const bool first = k == 1;                        // S_0 is the constant
        const bool old_is_s0 = k == 3;
        // the lane column's neighbour lists in A (padding has zero weight)
        int sv[kLS], pv[kLP];
        T sw[kLS], pw[kLP];
        int ns = 0, np = 0, sb = 0, pb = 0;
        if (colv) {
            sb = A.rp[j];
            ns = A.rp[j + 1] - sb;
            pb = A.cp[j];
            np = A.cp[j + 1] - pb;
        }
#pragma unroll
        for (int q = 0; q < kLS; ++q) {
            sv[q] = q < ns ? A.ci[sb + q] : 0;
            sw[q] = q < ns ? T(A.w[sb + q]) : T(0);
        }
#pragma unroll
        for (int q = 0; q < kLP; ++q) {
            pv[q] = q < np ? A.ri[pb + q] : 0;
            pw[q] = q < np ? T(A.w[A.eid[pb + q]]) : T(0);
        }
        const bool ovf = uni(dev::wave_max(max(ns - kLS, np - kLP))) > 0;
        double nu2 = 0.0, d2 = 0.0;
        for (int rr = 0; rr < kRowsPerWave; ++rr) {
            const int i = r0 + wave * kRowsPerWave + rr;
            if (i >= nB) break;
            if (compute) {
                T acc = T(0);
                if (first) {
                    // S_0 constant: Y_1[i][j] = c0 (outdeg_w_B(i) outdeg_w_A(j) + indeg_w_B(i) indeg_w_A(j))
                    T ra = T(0), rb = T(0), qa = T(0), qb = T(0);
                    for (int e = 0; e < ns; ++e) ra += T(A.w[sb + e]);
                    for (int e = 0; e < np; ++e) qa += T(A.w[A.eid[pb + e]]);
                    for (int e = B.rp[i]; e < B.rp[i + 1]; ++e) rb += T(B.w[e]);
                    for (int e = B.cp[i]; e < B.cp[i + 1]; ++e) qb += T(B.w[B.eid[e]]);
                    acc = c0v * (rb * ra + qb * qa);
                } else {
                    const int e1 = uni(B.rp[i + 1]);
                    for (int e = uni(B.rp[i]); e < e1; ++e) {
                        const int u = uni(B.ci[e]);
                        const T wu = T(B.w[e]);
                        const T* row = src + (long long)u * nA;
                        T in = T(0);
#pragma unroll
                        for (int q = 0; q < kLS; ++q) in = dev::fma_t(sw[q], row[sv[q]], in);
                        if (ovf)
                            for (int q = kLS; q < ns; ++q) in = dev::fma_t(T(A.w[sb + q]), row[A.ci[sb + q]], in);
                        acc = dev::fma_t(wu, in, acc);
                    }
                    const int f1 = uni(B.cp[i + 1]);
                    for (int e = uni(B.cp[i]); e < f1; ++e) {
                        const int u = uni(B.ri[e]);
                        const T wu = T(B.w[uni(B.eid[e])]);
                        const T* row = src + (long long)u * nA;
                        T in = T(0);
#pragma unroll
                        for (int q = 0; q < kLP; ++q) in = dev::fma_t(pw[q], row[pv[q]], in);
                        if (ovf)
                            for (int q = kLP; q < np; ++q)
                                in = dev::fma_t(T(A.w[A.eid[pb + q]]), row[A.ri[pb + q]], in);
                        acc = dev::fma_t(wu, in, acc);
                    }
                    acc *= sig;
                }
                if (colv) {
                    dst[(long long)i * nA + j] = acc;
                    nu2 += (double)acc * (double)acc;
                }
            }
            if (want_delta && colv) {
                const long long o = (long long)i * nA + j;
                const T a = T(src[o] * sig);                        // S_{k-1}
                const T b = old_is_s0 ? c0v : T(old[o] * sig3);     // S_{k-3}
                const double d = (double)a - (double)b;
                d2 += d * d;
            }
        }
        // per-tile partials (fixed order: waves, then lanes)
        nu2 = wave_sum(nu2);
        d2 = wave_sum(d2);
        if (lane == 0) {
            red[0][wave] = nu2;
            red[1][wave] = d2;
        }
        __syncthreads();
        if (tid == 0) {
            double a = 0.0, b = 0.0;
            for (int w = 0; w < kStepThreads / kWave; ++w) {
                a += red[0][w];
                b += red[1][w];
            }
            J.part_nu[t] = a;
            J.part_delta[t] = b;
            __threadfence();
            const int prev = atomicAdd(J.done + p, 1);
            last_flag = prev == s->ntiles - 1;
        }
        __syncthreads();
        if (last_flag) {
            // the pair's last tile of this launch: reduce its partials in tile order
            __threadfence();
            const long long t0 = J.tile_off[p], nt = s->ntiles;
            double a = 0.0, b = 0.0;
            for (long long q = tid; q < nt; q += kStepThreads) {
                a += J.part_nu[t0 + q];
                b += J.part_delta[t0 + q];
            }
            a = wave_sum(a);
            b = wave_sum(b);
            __syncthreads();
            if (lane == 0) {
                red[0][wave] = a;
                red[1][wave] = b;
            }
            __syncthreads();
            if (tid == 0) {
                double nu2s = 0.0, d2s = 0.0;
                for (int w = 0; w < kStepThreads / kWave; ++w) {
                    nu2s += red[0][w];
                    d2s += red[1][w];
                }
                J.done[p] = 0;
                bool stop = false;
                if (want_delta) {
                    const double delta = sqrt(d2s);
                    s->delta = delta;
                    if (delta < J.tol) {   // converged at the even step k - 1
                        s->final_step = k - 1;
                        s->nu = s->nu_k[(k - 1) & 3];
                        s->status = CFSIM_CONVERGED;
                        stop = true;
                    }
                }
                if (!stop && compute) {
                    const double nu = sqrt(nu2s);
                    s->nu_k[k & 3] = nu;
                    if (k == J.max_iter && (k & 1)) {  // odd max_iter: no change test at k
                        s->final_step = k;
                        s->nu = nu;
                        s->status = CFSIM_HIT_MAX_ITER;
                        stop = true;
                    }
                }
                if (!stop && !compute) {               // launch max_iter + 1
                    s->final_step = J.max_iter;
                    s->nu = s->nu_k[J.max_iter & 3];
                    s->status = CFSIM_HIT_MAX_ITER;
                    stop = true;
                }
                if (stop) s->active = 0;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- finish
// One workgroup per pair: rescale the final iterate in place (S_f = Y_f /
// nu_f, or S_0 for a degenerate pair), greedy matching, outputs.
template <typename T>
__global__ __launch_bounds__(kFinishThreads) void large_finish(LargeJob J) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NW = kFinishThreads / kWave;
    __shared__ double red[NW];
    __shared__ int s_count;
    const int p = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = uni(tid / kWave);
    const LargeState* s = J.st + p;
    cfsim_pair_result* res = J.res + p;
    if (s->status & CFSIM_INVALID_INPUT) {
        if (tid == 0) dev::write_invalid(res);
        return;
    }
    const int nA = s->nA, nB = s->nB;
    const int f = s->final_step;
    T* S = buf_of<T>(J, p, f & 3);
    const long long total = (long long)nA * nB;
    if (f == 0) {
        const T c0v = T(1.0 / sqrt((double)nA * (double)nB));
        for (long long o = tid; o < total; o += kFinishThreads) S[o] = c0v;
    } else {
        const T sig = T(1.0 / s->nu_k[f & 3]);
        for (long long o = tid; o < total; o += kFinishThreads) S[o] = S[o] * sig;
    }
    __syncthreads();
    __threadfence_block();

    // Greedy matching by locally dominant rounds: a free row and a free column
    // that are each other's best free partner are matched (the largest free
    // entry always is).  Rows are scanned by one wave each; columns in strips
    // of 64 (one lane per column, rows in order) so that every load of S is
    // a contiguous row segment.  Bests are recomputed only when stale (-2).
    const int nR = nB, nC = nA;
    int* rstate = reinterpret_cast<int*>(smem);
    int* rbest = rstate + nR;
    int* cstate = rbest + nR;
    int* cbest = cstate + nC;
    for (int r = tid; r < nR; r += kFinishThreads) {
        rstate[r] = -1;
        rbest[r] = -2;
    }
    for (int c = tid; c < nC; c += kFinishThreads) {
        cstate[c] = -1;
        cbest[c] = -2;
    }
    if (tid == 0) s_count = 0;
    __syncthreads();
    const int need = min(nR, nC);
    const int nstrip = (nC + 63) / 64;
    int done = 0;
    while (done < need) {
        for (int it = wave; it < nR + nstrip; it += NW) {
            if (it < nR) {
                const int r = it;
                if (uni(rstate[r]) != -1 || uni(rbest[r]) != -2) continue;
                T bv = T(-1);
                int bk = INT_MAX, bc = -1;
                const T* row = S + (long long)r * nC;
                for (int c = lane; c < nC; c += kWave) {
                    if (cstate[c] == -1) {
                        const T v = row[c];
                        const int key = r * nC + c;
                        if (better(v, key, bv, bk)) {
                            bv = v;
                            bk = key;
                            bc = c;
                        }
                    }
                }
                wave_argmax(bv, bk, bc);
                if (lane == 0) rbest[r] = bc;
            } else {
                const int c = (it - nR) * 64 + lane;
                const bool mine = c < nC && cstate[c] == -1 && cbest[c] == -2;
                if (__builtin_amdgcn_ballot_w64(mine) == 0) continue;
                T bv = T(-1);
                int bk = INT_MAX, br = -1;
                for (int r = 0; r < nR; ++r) {
                    if (uni(rstate[r]) != -1) continue;
                    if (mine) {
                        const T v = S[(long long)r * nC + c];
                        const int key = r * nC + c;
                        if (better(v, key, bv, bk)) {
                            bv = v;
                            bk = key;
                            br = r;
                        }
                    }
                }
                if (mine) cbest[c] = br;
            }
        }
        __syncthreads();
        for (int r = tid; r < nR; r += kFinishThreads) {
            if (rstate[r] == -1) {
                const int c = rbest[r];
                if (c >= 0 && cbest[c] == r) {
                    rstate[r] = c;
                    cstate[c] = r;
                    atomicAdd(&s_count, 1);
                }
            }
        }
        __syncthreads();
        for (int r = tid; r < nR; r += kFinishThreads)
            if (rstate[r] == -1 && rbest[r] >= 0 && cstate[rbest[r]] != -1) rbest[r] = -2;
        for (int c = tid; c < nC; c += kFinishThreads)
            if (cstate[c] == -1 && cbest[c] >= 0 && rstate[cbest[c]] != -1) cbest[c] = -2;
        const int now = s_count;
        __syncthreads();
        if (now == done) break;  // no progress: only possible with non-finite S
        done = now;
    }

    const int64_t mo = J.match_off ? J.match_off[p] : 0;
    double sc = 0.0;
    for (int i = tid; i < nB; i += kFinishThreads) {
        const int jj = rstate[i];
        if (jj >= 0) sc += (double)S[(long long)i * nC + jj];
        if (J.match) J.match[mo + i] = jj;
    }
    if (J.S_out) {
        T* So = reinterpret_cast<T*>(J.S_out) + J.S_off[p];
        for (long long o = tid; o < total; o += kFinishThreads) So[o] = S[o];
    }
    const double score = dev::block_sum<NW>(sc, red);
    if (tid == 0) {
        res->score = score;
        res->nu = s->nu;
        res->delta = s->delta;
        res->iters = f;
        res->status = s->status;
    }
}

}  // namespace

int large_step_grid(int num_cus) { return num_cus * 8; }

size_t large_finish_lds(int max_nodes) { return (size_t)16 * (size_t)max_nodes; }

int set_large_attributes() {
    int e = 0;
    e |= (int)hipFuncSetAttribute(reinterpret_cast<const void*>(&large_finish<float>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    e |= (int)hipFuncSetAttribute(reinterpret_cast<const void*>(&large_finish<double>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    return e;
}

int launch_large(int dtype, const LargeJob& J, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(large_init, dim3(J.n_pairs), dim3(256), 0, stream, J);
    int e = (int)hipGetLastError();
    if (e != 0) return e;
    hipLaunchKernelGGL(large_scan, dim3(1), dim3(1024), 0, stream, J);
    if ((e = (int)hipGetLastError()) != 0) return e;
    for (int k = 1; k <= J.max_iter + 1; ++k) {
        if (dtype == CFSIM_F64)
            hipLaunchKernelGGL(large_step<double>, dim3(grid), dim3(kStepThreads), 0, stream, J, k);
        else
            hipLaunchKernelGGL(large_step<float>, dim3(grid), dim3(kStepThreads), 0, stream, J, k);
        if ((e = (int)hipGetLastError()) != 0) return e;
    }
    const size_t lds = large_finish_lds(J.max_nodes);
    if (dtype == CFSIM_F64)
        hipLaunchKernelGGL(large_finish<double>, dim3(J.n_pairs), dim3(kFinishThreads), lds, stream, J);
    else
        hipLaunchKernelGGL(large_finish<float>, dim3(J.n_pairs), dim3(kFinishThreads), lds, stream, J);
    return (int)hipGetLastError();
}

}  // namespace cfsim
