// Step a9 with dense padded tiles: the products of the tiled path as
// block-sparse BF16 matrix-core products with FP32 accumulation
// (v_mfma_f32_32x32x16_bf16), for plain (not resized) FP32 calls of
// cfsim_score_large with CFSIM_FLAG_MFMA_BF16.
//
// Both transition matrices are cut into 32 x 32 blocks.  Only the blocks that
// hold an edge are stored, in BF16 and zero-padded past the graph's last
// node.  Each is stored twice, row-major and transposed, and indexed by block
// row (BSR order, whose position is the block's id) and by block column.
// With S (n_B x n_A) cut the same way, an update is two launches over the
// tiled path's 128 x 64 tile map:
//   stage 1:  T1^T = A S^T and T2^T = A^T S^T.  Per 32 x 32 output block this
//             is the sum over the nonzero blocks of one block row (block
//             column) of A; the results are stored as BF16 blocks.
//   stage 2:  Y = B T1 + B^T T2 (= B S A^T + B^T S A), times 1/nu of the
//             previous iterate.  Y is stored in FP32, row-major, which is the
//             layout the tiled path's per-pair reduction and matching read,
//             and as BF16 blocks for the next stage 1, with the norm partials
//             of every 128 x 64 tile (and the even-step change at odd k).
// Every product is D += X Z^T of two row-major blocks X and Z.  Each lane
// reads 16 bytes of each (row lane % 32, eight consecutive entries), and each
// result register is one row segment of the output block.  Rounding: S, T
// and the weights are BF16 operands and every sum is FP32; the error against
// FP64 is reported, not gated.
#include "cfsim_internal.h"
#include "large_tiles.h"
#include "pair_device.h"

namespace cfsim {

namespace {

using namespace tiled;
using dev::uni;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kPrepThreads = 1024;
constexpr int kBlockU4 = 128;  // one 32 x 32 BF16 block in 16-byte words

// Block lists of pair p's row graph (side 0) or column graph (side 1):
// brow[nb + 1] (BSR row starts; the position of an entry is its block id),
// bcol[cap] (block column of each stored block), bcp[nb + 1] (block-column
// starts), bsr[cap] (block row of each block-column entry), bst[cap] (its id).
struct BlockLists {
    const int *brow, *bcol, *bcp, *bsr, *bst;
};
__device__ inline int* idx_base(const LargeJob& J, int p, int side) {
    return J.mf_idx + ((long long)p * 2 + side) * J.mf_idx_stride;
}
__device__ inline BlockLists lists_of(const LargeJob& J, int p, int side) {
    const int* b = idx_base(J, p, side);
    BlockLists L;
    L.brow = b;
    L.bcol = L.brow + (J.mf_nb + 1);
    L.bcp = L.bcol + J.mf_cap;
    L.bsr = L.bcp + (J.mf_nb + 1);
    L.bst = L.bsr + J.mf_cap;
    return L;
}
// Stored block `id` of a side: layout 0 row-major, 1 transposed.
__device__ inline uint4* graph_block(const LargeJob& J, int p, int side, int id, int layout) {
    return J.mf_tiles + ((((long long)p * 2 + side) * J.mf_cap + id) * 2 + layout) * kBlockU4;
}
// Pair p's BF16 block arrays: 0 = Y_{k-1} ([nRb][nCb]), 1 = T1^T, 2 = T2^T ([nCb][nRb]).
__device__ inline uint4* pair_blocks(const LargeJob& J, int p, int which) {
    return J.mf_blocks + ((long long)p * 3 + which) * (long long)J.mf_nb * J.mf_nb * kBlockU4;
}

__device__ inline bf16x8 as_bf16x8(uint4 x) {
    union {
        uint4 u;
        bf16x8 b;
    } c;
    c.u = x;
    return c.b;
}

// acc += X Z^T for row-major 32 x 32 BF16 blocks X and Z.
__device__ inline void block_fma(const uint4* X, const uint4* Z, f32x16& acc, int lane) {
    const int row = lane & 31, q = lane >> 5;
    const uint4 x0 = X[row * 4 + q], x1 = X[row * 4 + 2 + q];
    const uint4 z0 = Z[row * 4 + q], z1 = Z[row * 4 + 2 + q];
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(x0), as_bf16x8(z0), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(x1), as_bf16x8(z1), acc, 0, 0, 0);
}

// Row of result register r in lane `lane` (its column is lane % 32).
__device__ inline int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

__device__ inline void store_block(uint4* dst, const f32x16& acc, int lane) {
    __bf16* d = reinterpret_cast<__bf16*>(dst);
#pragma unroll
    for (int r = 0; r < 16; ++r) d[acc_row(r, lane) * 32 + (lane & 31)] = (__bf16)acc[r];
}

// Set bits of the bitmap in [from, to).
__device__ inline int bit_count(const uint32_t* bits, int from, int to) {
    int c = 0;
    for (int b = from; b < to;) {
        const int w = b >> 5, off = b & 31, n = min(32 - off, to - b);
        const uint32_t mask = n == 32 ? 0xFFFFFFFFu : (((1u << n) - 1u) << off);
        c += __popc(bits[w] & mask);
        b += n;
    }
    return c;
}
__device__ inline bool bit_at(const uint32_t* bits, int b) { return (bits[b >> 5] >> (b & 31)) & 1u; }

// Graphs of the state: rows = B, columns = A (plain pairs, no resize).
__device__ inline void mfma_graphs(const LargeJob& J, int p, GraphRef* Rg, GraphRef* Cg) {
    if (J.single) {
        *Rg = J.gb;
        *Cg = J.ga;
        return;
    }
    *Rg = graph_of(J.set, J.pair_b[p]);
    *Cg = graph_of(J.set, J.pair_a[p]);
}

// One workgroup per pair: the block lists and stored blocks of both graphs,
// and S_0 as BF16 blocks.  A pair whose graph has more nonzero blocks than
// the workspace holds (mf_cap) is marked invalid.
__global__ __launch_bounds__(kPrepThreads) void mfma_prep(LargeJob J) {
    __shared__ uint32_t bits[kMfmaMaxBlocks * kMfmaMaxBlocks / 32];
    __shared__ int rptr[kMfmaMaxBlocks + 1], cptr[kMfmaMaxBlocks + 1];
    __shared__ int too_many;
    const int p = blockIdx.x, tid = threadIdx.x;
    LargeState* s = J.st + p;
    if (!s->active) return;  // invalid or degenerate: nothing to iterate (uniform)
    GraphRef Rg, Cg;
    mfma_graphs(J, p, &Rg, &Cg);
    for (int side = 0; side < 2; ++side) {
        const GraphRef G = side == 0 ? Rg : Cg;
        const int n = G.n, nb = (n + 31) >> 5, nbits = nb * nb;
        for (int w = tid; w < (nbits + 31) / 32; w += kPrepThreads) bits[w] = 0u;
        if (tid == 0) too_many = 0;
        __syncthreads();
        for (int u = tid; u < n; u += kPrepThreads)
            for (int e = G.rp[u]; e < G.rp[u + 1]; ++e) {
                const int b = (u >> 5) * nb + (G.ci[e] >> 5);
                atomicOr(&bits[b >> 5], 1u << (b & 31));
            }
        __syncthreads();
        for (int r = tid; r < nb; r += kPrepThreads) rptr[r + 1] = bit_count(bits, r * nb, r * nb + nb);
        for (int c = tid; c < nb; c += kPrepThreads) {
            int cnt = 0;
            for (int r = 0; r < nb; ++r) cnt += bit_at(bits, r * nb + c);
            cptr[c + 1] = cnt;
        }
        __syncthreads();
        if (tid == 0) {
            rptr[0] = cptr[0] = 0;
            for (int i = 1; i <= nb; ++i) {
                rptr[i] += rptr[i - 1];
                cptr[i] += cptr[i - 1];
            }
            too_many = rptr[nb] > J.mf_cap;
        }
        __syncthreads();
        if (too_many) {
            if (tid == 0) {
                s->active = 0;
                s->status = CFSIM_INVALID_INPUT;
            }
            return;  // uniform: too_many is one LDS word
        }
        int* base = idx_base(J, p, side);
        int* brow = base;
        int* bcol = brow + (J.mf_nb + 1);
        int* bcp = bcol + J.mf_cap;
        int* bsr = bcp + (J.mf_nb + 1);
        int* bst = bsr + J.mf_cap;
        for (int i = tid; i <= nb; i += kPrepThreads) {
            brow[i] = rptr[i];
            bcp[i] = cptr[i];
        }
        for (int r = tid; r < nb; r += kPrepThreads) {
            int q = rptr[r];
            for (int c = 0; c < nb; ++c)
                if (bit_at(bits, r * nb + c)) bcol[q++] = c;
        }
        for (int c = tid; c < nb; c += kPrepThreads) {
            int q = cptr[c];
            for (int r = 0; r < nb; ++r)
                if (bit_at(bits, r * nb + c)) {
                    bsr[q] = r;
                    bst[q] = rptr[r] + bit_count(bits, r * nb, r * nb + c);
                    ++q;
                }
        }
        const int nblk = rptr[nb];
        uint4* blocks = graph_block(J, p, side, 0, 0);
        for (long long x = tid; x < (long long)nblk * 2 * kBlockU4; x += kPrepThreads) blocks[x] = make_uint4(0, 0, 0, 0);
        __syncthreads();
        // entries: row u's jumps (sorted by target, repeated jumps adjacent and summed)
        for (int u = tid; u < n; u += kPrepThreads) {
            const int e1 = G.rp[u + 1];
            for (int e = G.rp[u]; e < e1;) {
                const int v = G.ci[e];
                double w = 0.0;
                for (; e < e1 && G.ci[e] == v; ++e) w += G.w[e];
                const int br = u >> 5, bc = v >> 5;
                const int id = rptr[br] + bit_count(bits, br * nb, br * nb + bc);
                const __bf16 x = (__bf16)(float)w;
                reinterpret_cast<__bf16*>(graph_block(J, p, side, id, 0))[(u & 31) * 32 + (v & 31)] = x;
                reinterpret_cast<__bf16*>(graph_block(J, p, side, id, 1))[(v & 31) * 32 + (u & 31)] = x;
            }
        }
        __syncthreads();
    }
    // S_0 = 1/sqrt(n_A n_B) as BF16 blocks, zero past the last row and column
    const int nR = s->nR, nC = s->nC, nRb = (nR + 31) >> 5, nCb = (nC + 31) >> 5;
    const __bf16 c0 = (__bf16)(float)(1.0 / sqrt((double)nR * (double)nC));
    __bf16* y = reinterpret_cast<__bf16*>(pair_blocks(J, p, 0));
    for (long long x = tid; x < (long long)nRb * nCb * 1024; x += kPrepThreads) {
        const int blk = (int)(x >> 10), w = (int)(x & 1023);
        const int i = (blk / nCb) * 32 + (w >> 5), j = (blk % nCb) * 32 + (w & 31);
        y[x] = (i < nR && j < nC) ? c0 : (__bf16)0.0f;
    }
}

// Stage 1 of launch k (k <= max_iter): T1^T = A S^T and T2^T = A^T S^T, S the
// BF16 blocks of Y_{k-1}.  Wave w of a 128 x 64 tile takes S's block row
// r0 / 32 + w and the tile's two block columns.  No barrier: waves whose
// block row lies past the pair's last row skip it.
__global__ __launch_bounds__(kStepThreads) void mfma_stage1(LargeJob J, int k) {
    (void)k;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const TileRange tr = tile_range(J);
    for (long long t = tr.first; t < tr.end; t += tr.stride) {
        const int p = uni(pair_of_tile(J, t));
        const LargeState* s = J.st + p;
        if (!uni(s->active)) continue;
        const Tile tl = tile_at(J, t, s, p);
        const int nRb = (uni(s->nR) + 31) >> 5, nCb = (uni(s->nC) + 31) >> 5;
        const int rb = (tl.r0 >> 5) + wave;
        if (rb >= nRb) continue;
        const BlockLists A = lists_of(J, p, 1);
        const uint4* Y = pair_blocks(J, p, 0);
        uint4* T1 = pair_blocks(J, p, 1);
        uint4* T2 = pair_blocks(J, p, 2);
        for (int jj = 0; jj < 2; ++jj) {
            const int jb = (tl.c0 >> 5) + jj;
            if (jb >= nCb) break;
            f32x16 a1 = {}, a2 = {};
            const int q1 = uni(A.brow[jb + 1]);
            for (int q = uni(A.brow[jb]); q < q1; ++q) {
                const int I = uni(A.bcol[q]);
                block_fma(graph_block(J, p, 1, q, 0), Y + ((long long)rb * nCb + I) * kBlockU4, a1, lane);
            }
            const int q2 = uni(A.bcp[jb + 1]);
            for (int q = uni(A.bcp[jb]); q < q2; ++q) {
                const int I = uni(A.bsr[q]), id = uni(A.bst[q]);
                block_fma(graph_block(J, p, 1, id, 1), Y + ((long long)rb * nCb + I) * kBlockU4, a2, lane);
            }
            store_block(T1 + ((long long)jb * nRb + rb) * kBlockU4, a1, lane);
            store_block(T2 + ((long long)jb * nRb + rb) * kBlockU4, a2, lane);
        }
    }
}

// Stage 2 of launch k: Y_k = (B T1 + B^T T2) sigma_{k-1} into buffer k % 4
// (FP32) and into the BF16 blocks, the norm partials, and at odd k >= 3 the
// partials of S_{k-1} - S_{k-3}.  Launch max_iter + 1 only takes that change.
__global__ __launch_bounds__(kStepThreads) void mfma_stage2(LargeJob J, int k) {
    __shared__ double red[2 * kNWStep];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const bool compute = k <= J.max_iter;
    const bool want_delta = (k & 1) && k >= 3;
    const TileRange tr = tile_range(J);
    for (long long t = tr.first; t < tr.end; t += tr.stride) {
        const int p = uni(pair_of_tile(J, t));
        const LargeState* s = J.st + p;
        if (!uni(s->active)) continue;  // the same for every wave of the tile
        const Tile tl = tile_at(J, t, s, p);
        const int nR = uni(s->nR), nC = uni(s->nC), nRb = (nR + 31) >> 5, nCb = (nC + 31) >> 5;
        const float sig = (float)(1.0 / s->nu_k[(k - 1) & 3]);   // sigma_{k-1} (1 for S_0)
        const float sig3 = (float)(1.0 / s->nu_k[(k - 3) & 3]);  // sigma_{k-3}
        double nu2 = 0.0, d2 = 0.0;
        const int rb = (tl.r0 >> 5) + wave;
        if (compute && rb < nRb) {
            const BlockLists B = lists_of(J, p, 0);
            const uint4* T1 = pair_blocks(J, p, 1);
            const uint4* T2 = pair_blocks(J, p, 2);
            uint4* Yb = pair_blocks(J, p, 0);
            float* dst = buf_of<float>(J, p, k & 3);
            for (int jj = 0; jj < 2; ++jj) {
                const int jb = (tl.c0 >> 5) + jj;
                if (jb >= nCb) break;
                f32x16 acc = {};
                const int q1 = uni(B.brow[rb + 1]);
                for (int q = uni(B.brow[rb]); q < q1; ++q) {
                    const int R = uni(B.bcol[q]);
                    block_fma(graph_block(J, p, 0, q, 0), T1 + ((long long)jb * nRb + R) * kBlockU4, acc, lane);
                }
                const int q2 = uni(B.bcp[rb + 1]);
                for (int q = uni(B.bcp[rb]); q < q2; ++q) {
                    const int R = uni(B.bsr[q]), id = uni(B.bst[q]);
                    block_fma(graph_block(J, p, 0, id, 1), T2 + ((long long)jb * nRb + R) * kBlockU4, acc, lane);
                }
                __bf16* yb = reinterpret_cast<__bf16*>(Yb + ((long long)rb * nCb + jb) * kBlockU4);
                const int j = jb * 32 + (lane & 31);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int m = acc_row(r, lane);
                    const int i = rb * 32 + m;
                    const float v = acc[r] * sig;
                    if (i < nR && j < nC) {
                        dst[(long long)i * nC + j] = v;
                        nu2 += (double)v * (double)v;
                    }
                    yb[m * 32 + (lane & 31)] = (__bf16)v;
                }
            }
        }
        if (want_delta) {
            const float* src = buf_of<float>(J, p, (k - 1) & 3);
            const float* old = buf_of<float>(J, p, (k - 3) & 3);
            const float c0v = (float)(1.0 / sqrt((double)s->nA * (double)s->nB));
            const int j = tl.c0 + lane;
            if (j < nC) {
                for (int rr = 0; rr < kRowsPerWave; ++rr) {
                    const int i = tl.r0 + wave * kRowsPerWave + rr;
                    if (i >= nR) break;
                    const long long o = (long long)i * nC + j;
                    const float a = src[o] * sig;                          // S_{k-1}
                    const float b = k == 3 ? c0v : old[o] * sig3;           // S_{k-3}
                    const double d = (double)a - (double)b;
                    d2 += d * d;
                }
            }
        }
        tile_partials(J, t, nu2, d2, red);
    }
}

}  // namespace

int launch_mfma_prep(const LargeJob& J, hipStream_t stream) {
    hipLaunchKernelGGL(mfma_prep, dim3(J.n_pairs), dim3(kPrepThreads), 0, stream, J);
    return (int)hipGetLastError();
}

int launch_mfma_update(const LargeJob& J, int k, int grid, hipStream_t stream) {
    if (k <= J.max_iter) {
        hipLaunchKernelGGL(mfma_stage1, dim3(grid), dim3(kStepThreads), 0, stream, J, k);
        const int e = (int)hipGetLastError();
        if (e != 0) return e;
    }
    hipLaunchKernelGGL(mfma_stage2, dim3(grid), dim3(kStepThreads), 0, stream, J, k);
    return (int)hipGetLastError();
}

}  // namespace cfsim
