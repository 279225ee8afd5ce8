// Step a9 (large pairs) and step a2 (scale to a common size) on the tiled,
// global-memory path.
//
// S no longer fits a workgroup's LDS, so every update is one grid-wide launch
// over tiles of all pairs of the call, with the iterates in HBM (the MI355X
// last-level cache holds a pair's working set).  The host captures the whole
// sequence into one HIP graph.  Every tile writes FP64 partials of the norms;
// a small per-pair kernel after each update sums them in tile order (so every
// reduction is deterministic) and takes the stopping decision.  A kernel
// boundary is the cheap synchronisation here: on MI355X a device-scope fence
// writes back and invalidates the XCD's whole L2, which a per-tile fence
// would do thousands of times per update.
//
// Plain operator (no resize): four buffers rotate per pair; launch k reads
// Y_{k-1} with sigma_{k-1} = 1/nu_{k-1} folded into the update and writes the
// un-normalised Y_k = M S_{k-1}.  The even-step change
// delta_{k-1} = ||S_{k-1} - S_{k-3}|| is accumulated by the odd launch k, the
// first one that knows both scales; launch max_iter + 1 only does that.
//
// Scale to a common size (Section 4 and Section 4.1): the smaller graph X (m
// nodes) is replaced by X' = R X R^T with the M x m linear-interpolation
// matrix R.  X' is never formed.  With the small graph on the column side,
//   Y = Rg S Cg'^T + Rg^T S Cg' = [Rg (S R) Cg^T + Rg^T (S R) Cg] R^T,
// so the iteration carries U = M_{Rg,Cg}(S R) (M x m, the plain operator at
// the small size) and V = U G with the tridiagonal G = R^T R:
//   U_k = M(V_{k-1}) / nu_{k-1},  V_k = U_k G,  nu_k^2 = <U_k, V_k> = ||Y_k||^2,
//   delta_k^2 = <D, D G> with D = U_k / nu_k - U_{k-2} / nu_{k-2},
// and S_k = U_k R^T / nu_k is expanded once at the end.  S_0 = 1/M is
// U_0 = 1/M (every row of R sums to 1).  Each update is then three launches:
// large_step (U), large_gram (V and the norm partials), large_reduce.
#include "cfsim_internal.h"
#include "large_tiles.h"
#include "pair_device.h"

namespace cfsim {

namespace {

using namespace tiled;
using dev::better;
using dev::uni;
using dev::wave_sum;

// rows whose gathers are in flight together (FP64: two, which keeps the
// gather kernel at four waves per SIMD)
template <typename T>
constexpr int unroll_of() {
    return sizeof(T) == 8 ? 2 : 4;
}
constexpr int kReduceGrid = 2048;               // workgroups of the per-pair reduction
constexpr int kFinishThreads = 1024;
constexpr int kLS = 2;                          // successors per lane column in registers
constexpr int kLP = 3;                          // predecessors per lane column in registers
constexpr int kSlotU = 0;                       // resize: U_k in slot k % 4
constexpr int kSlotV = 4;                       // resize: V
constexpr int kSlotS = 5;                       // resize: expanded final S

// First successors / predecessors of one node with their weights, the list
// lengths (which may exceed the slots), zero-weight padding.
template <typename T>
struct alignas(16) NodeRec {
    int ns, np;
    int su[kLS];
    int pu[kLP];
    T sw[kLS];
    T pw[kLP];
};
static_assert(sizeof(NodeRec<float>) == 48 && sizeof(NodeRec<double>) == 80, "large_rec_bytes()");

// Pair p's records: rows of the row graph (which = 0), columns of the column graph (1).
template <typename T>
__device__ inline NodeRec<T>* recs_of(const LargeJob& J, int p, int which) {
    return reinterpret_cast<NodeRec<T>*>(J.recs) + ((long long)p * 2 + which) * J.max_nodes;
}

template <typename T>
__device__ inline NodeRec<T> make_rec(const GraphRef& G, int v) {
    NodeRec<T> r;
    const int sb = G.rp[v], pb = G.cp[v];
    r.ns = G.rp[v + 1] - sb;
    r.np = G.cp[v + 1] - pb;
#pragma unroll
    for (int q = 0; q < kLS; ++q) {
        r.su[q] = q < r.ns ? G.ci[sb + q] : 0;
        r.sw[q] = q < r.ns ? T(G.w[sb + q]) : T(0);
    }
#pragma unroll
    for (int q = 0; q < kLP; ++q) {
        r.pu[q] = q < r.np ? G.ri[pb + q] : 0;
        r.pw[q] = q < r.np ? T(G.w[G.eid[pb + q]]) : T(0);
    }
    return r;
}


__device__ inline bool pair_graphs(const LargeJob& J, int p, GraphRef* A, GraphRef* B) {
    if (J.single) {
        *A = J.ga;
        *B = J.gb;
        return true;
    }
    const int ga = J.pair_a[p], gb = J.pair_b[p];
    if (ga < 0 || ga >= J.set.n_graphs || gb < 0 || gb >= J.set.n_graphs) return false;
    *A = graph_of(J.set, ga);
    *B = graph_of(J.set, gb);
    return true;
}

// Row graph (wave-uniform rows) and column graph (lanes) of the state.
__device__ inline void state_graphs(const LargeJob& J, int p, const LargeState* s, GraphRef* Rg, GraphRef* Cg) {
    GraphRef A, B;
    pair_graphs(J, p, &A, &B);
    *Rg = s->swap ? A : B;
    *Cg = s->swap ? B : A;
}

// ---------------------------------------------------------------- set-up
// One workgroup per pair: validity, degeneracy, state shape, initial state,
// and the node records of the row graph's rows and the column graph's columns.
// Internal state bit of a pair this call leaves alone (scored by the LDS
// kernels before; see LargeJob::filter): no tiles, no outputs.
constexpr unsigned kSkipped = 0x80000000u;

template <typename T>
__global__ __launch_bounds__(256) void large_init(LargeJob J) {
    const int p = blockIdx.x;
    __shared__ int pos[2];
    LargeState* s = J.st + p;
    if (J.filter && !(J.filter[p].status & CFSIM_INVALID_INPUT)) {
        if (threadIdx.x == 0) {
            s->ntiles = 0;
            s->active = 0;
            s->rz = 0;
            s->status = CFSIM_INVALID_INPUT | kSkipped;
        }
        return;
    }
    GraphRef A{}, B{};
    const bool ok_ids = pair_graphs(J, p, &A, &B);
    const int nA = ok_ids ? A.n : 0, nB = ok_ids ? B.n : 0;
    const int M = nA > nB ? nA : nB;
    const bool rz = J.resize && nA != nB;
    const bool ok = ok_ids && nA >= 1 && nB >= 1 && nA <= J.max_nodes && nB <= J.max_nodes &&
                    (long long)(rz ? M : nA) * (rz ? M : nB) <= J.slot_elems;
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
        s->rz = rz ? 1 : 0;
        s->swap = rz && nB < nA ? 1 : 0;  // the smaller graph takes the column side
        s->nR = rz ? M : nB;
        s->nC = rz ? (nA < nB ? nA : nB) : nA;
        s->M = rz ? M : 0;
        s->ntiles = ok ? tiles_of(s->nC, s->nR) : 0;
        s->active = (ok && pos[0] && pos[1]) ? 1 : 0;
        s->status = !ok ? CFSIM_INVALID_INPUT : (s->active ? 0u : (unsigned)CFSIM_DEGENERATE);
        s->final_step = 0;
        s->nu = 0.0;
        s->delta = __builtin_inf();
        for (int b = 0; b < 4; ++b) s->nu_k[b] = 1.0;
    }
    if (!ok) return;
    const bool swap = rz && nB < nA;
    const GraphRef& Rg = swap ? A : B;
    const GraphRef& Cg = swap ? B : A;
    NodeRec<T>* rr = recs_of<T>(J, p, 0);
    NodeRec<T>* cr = recs_of<T>(J, p, 1);
    for (int v = threadIdx.x; v < Rg.n; v += 256) rr[v] = make_rec<T>(Rg, v);
    for (int v = threadIdx.x; v < Cg.n; v += 256) cr[v] = make_rec<T>(Cg, v);
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

// Pair of every tile (so a tile finds its pair with one load).
__global__ __launch_bounds__(256) void large_tile_map(LargeJob J) {
    for (int p = blockIdx.x; p < J.n_pairs; p += gridDim.x) {
        const long long t0 = J.tile_off[p], t1 = J.tile_off[p + 1];
        for (long long t = t0 + threadIdx.x; t < t1; t += 256) J.tile_pair[t] = p;
    }
}


// After update launch k: one workgroup per active pair sums its tiles'
// partials in tile order and decides whether the pair stops.  compute: a new
// iterate was formed (k <= max_iter); want_delta: the partials of
// delta_{k-1} were accumulated (odd k >= 3).
__global__ __launch_bounds__(kStepThreads) void large_reduce(LargeJob J, int k) {
    __shared__ double red[2 * kNWStep];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const bool compute = k <= J.max_iter;
    const bool want_delta = (k & 1) && k >= 3;
    // pairs in a grid-stride loop: a call whose pairs mostly ran elsewhere
    // (resized batches) launches a few workgroups instead of one per pair
    for (int p = blockIdx.x; p < J.n_pairs; p += gridDim.x) {
        LargeState* s = J.st + p;
        if (!s->active) continue;  // the same word in every thread
        const long long t0 = J.tile_off[p], nt = s->ntiles;
        double a = 0.0, b = 0.0;
        for (long long q = tid; q < nt; q += kStepThreads) {
            a += J.part_nu[t0 + q];
            b += J.part_delta[t0 + q];
        }
        a = wave_sum(a);
        b = wave_sum(b);
        if (lane == 0) {
            red[wave] = a;
            red[kNWStep + wave] = b;
        }
        __syncthreads();
        if (tid == 0) {
            double nu2s = 0.0, d2s = 0.0;
            for (int w = 0; w < kNWStep; ++w) {
                nu2s += red[w];
                d2s += red[kNWStep + w];
            }
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
        __syncthreads();  // red is reused by the next pair
    }
}

// Sum over a row's NS successor and NP predecessor terms (wave-uniform rows u
// of the source iterate) of the lane column's gathered terms; every gather of
// the row is independent, so they are all in flight together.
template <typename T, int NS, int NP>
__device__ inline T row_terms(const T* src, int nC, const int (&ru)[kLS], const T (&rw)[kLS], const int (&qu)[kLP],
                              const T (&qw)[kLP], const NodeRec<T>& c) {
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < NS; ++a) {
        const T* row = src + (long long)ru[a] * nC;
        T in = c.sw[0] * row[c.su[0]];
#pragma unroll
        for (int q = 1; q < kLS; ++q) in = dev::fma_t(c.sw[q], row[c.su[q]], in);
        acc = dev::fma_t(rw[a], in, acc);
    }
#pragma unroll
    for (int b = 0; b < NP; ++b) {
        const T* row = src + (long long)qu[b] * nC;
        T in = c.pw[0] * row[c.pu[0]];
#pragma unroll
        for (int q = 1; q < kLP; ++q) in = dev::fma_t(c.pw[q], row[c.pu[q]], in);
        acc = dev::fma_t(qw[b], in, acc);
    }
    return acc;
}

// All first-slot terms of one row, padded (zero weights read row 0): the code
// is the same for every row, so the gathers of several rows can be issued
// before any of them is used.
template <typename T>
__device__ inline T row_padded(const T* src, int nC, const NodeRec<T>& r, const NodeRec<T>& c) {
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < kLS; ++a) {
        const T* row = src + (long long)uni(r.su[a]) * nC;
        T in = c.sw[0] * row[c.su[0]];
#pragma unroll
        for (int q = 1; q < kLS; ++q) in = dev::fma_t(c.sw[q], row[c.su[q]], in);
        acc = dev::fma_t(uni(r.sw[a]), in, acc);
    }
#pragma unroll
    for (int b = 0; b < kLP; ++b) {
        const T* row = src + (long long)uni(r.pu[b]) * nC;
        T in = c.pw[0] * row[c.pu[0]];
#pragma unroll
        for (int q = 1; q < kLP; ++q) in = dev::fma_t(c.pw[q], row[c.pu[q]], in);
        acc = dev::fma_t(uni(r.pw[b]), in, acc);
    }
    return acc;
}

// Terms of row i past its first kLS successors / kLP predecessors (CSR lists).
template <typename T>
__device__ inline T row_rest(const T* src, int nC, const GraphRef& Rg, int i, const NodeRec<T>& c) {
    T acc = T(0);
    const int e1 = uni(Rg.rp[i + 1]);
    for (int e = uni(Rg.rp[i]) + kLS; e < e1; ++e) {
        const T* row = src + (long long)uni(Rg.ci[e]) * nC;
        T in = T(0);
#pragma unroll
        for (int q = 0; q < kLS; ++q) in = dev::fma_t(c.sw[q], row[c.su[q]], in);
        acc = dev::fma_t(T(Rg.w[e]), in, acc);
    }
    const int f1 = uni(Rg.cp[i + 1]);
    for (int e = uni(Rg.cp[i]) + kLP; e < f1; ++e) {
        const T* row = src + (long long)uni(Rg.ri[e]) * nC;
        T in = T(0);
#pragma unroll
        for (int q = 0; q < kLP; ++q) in = dev::fma_t(c.pw[q], row[c.pu[q]], in);
        acc = dev::fma_t(T(Rg.w[uni(Rg.eid[e])]), in, acc);
    }
    return acc;
}

// Terms of row i that take the lane column's list entries past its first kLS
// successors / kLP predecessors (only lanes with long lists loop).
template <typename T>
__device__ inline T col_rest(const T* src, int nC, const GraphRef& Rg, int i, const GraphRef& Cg, int sb, int ns,
                             int pb, int np) {
    T acc = T(0);
    if (ns > kLS) {
        const int e1 = uni(Rg.rp[i + 1]);
        for (int e = uni(Rg.rp[i]); e < e1; ++e) {
            const T* row = src + (long long)uni(Rg.ci[e]) * nC;
            T in = T(0);
            for (int q = kLS; q < ns; ++q) in = dev::fma_t(T(Cg.w[sb + q]), row[Cg.ci[sb + q]], in);
            acc = dev::fma_t(T(Rg.w[e]), in, acc);
        }
    }
    if (np > kLP) {
        const int f1 = uni(Rg.cp[i + 1]);
        for (int e = uni(Rg.cp[i]); e < f1; ++e) {
            const T* row = src + (long long)uni(Rg.ri[e]) * nC;
            T in = T(0);
            for (int q = kLP; q < np; ++q) in = dev::fma_t(T(Cg.w[Cg.eid[pb + q]]), row[Cg.ri[pb + q]], in);
            acc = dev::fma_t(T(Rg.w[uni(Rg.eid[e])]), in, acc);
        }
    }
    return acc;
}

// ---------------------------------------------------------------- the operator
// Launch k (1 .. max_iter): X_k = M_{Rg,Cg}(src) * sigma_{k-1} over the state
// (nR x nC).  Plain pairs: src = Y_{k-1} (S_0 is the constant
// 1/sqrt(n_A n_B)), X_k = Y_k into buffer k % 4, plus the norm partials and,
// at odd k >= 3, those of S_{k-1} - S_{k-3}.  Resized pairs: src = V_{k-1},
// X_k = U_k into slot k % 4; large_gram does the rest.  Launch max_iter + 1
// computes only the last change of plain pairs.
//
// Two kernels share the tiles: large_step<T, false> every tile whose pair
// gathers at k (plain pairs from k = 2, resized pairs from k = 1), and
// large_step<T, true> the first update of plain pairs (from the constant S_0)
// and the change-only launch.  Kept apart, the gather loop's register budget
// is its own (four waves per SIMD instead of two).
template <typename T, bool EDGE>
__global__ __launch_bounds__(kStepThreads) void large_step(LargeJob J, int k) {
    __shared__ double red[2 * kNWStep];
    __shared__ NodeRec<T> trec[kTileRows];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const bool compute = k <= J.max_iter;
    const bool want_delta = (k & 1) && k >= 3;
    const TileRange tr = tile_range(J);
    for (long long t = tr.first; t < tr.end; t += tr.stride) {
        const int p = uni(pair_of_tile(J, t));
        LargeState* s = J.st + p;
        if (!uni(s->active)) continue;
        const bool rz = uni(s->rz) != 0;
        if (rz && !compute) continue;
        const bool first = k == 1 && !rz;                 // S_0 is the constant
        if ((compute && !first) == EDGE) continue;         // a tile of the other kernel
        const Tile tl = tile_at(J, t, s, p);
        const int nR = s->nR, nC = s->nC;
        const int j = tl.c0 + lane;
        const bool colv = j < nC;
        const T* src = rz ? buf_of<T>(J, p, kSlotV) : buf_of<T>(J, p, (k - 1) & 3);
        T* dst = buf_of<T>(J, p, k & 3);
        const T* old = buf_of<T>(J, p, (k - 3) & 3);
        const T c0v = T(1.0 / sqrt((double)s->nA * (double)s->nB));
        const T sig = T(1.0 / s->nu_k[(k - 1) & 3]);     // sigma_{k-1} (1 for S_0)
        const T sig3 = T(1.0 / s->nu_k[(k - 3) & 3]);    // sigma_{k-3}
        const bool old_is_s0 = k == 3;
        // the lane column's neighbour lists in Cg (padding has zero weight)
        NodeRec<T> cr{};
        if (colv) cr = recs_of<T>(J, p, 1)[j];
        const int ns = cr.ns, np = cr.np;
        double nu2 = 0.0, d2 = 0.0;
        const int i0 = tl.r0 + wave * kRowsPerWave;
        constexpr int kUnroll = unroll_of<T>();
        if constexpr (!EDGE) {
            // lanes whose column lists are longer than the slots
            const bool ovf = uni(dev::wave_max(max(ns - kLS, np - kLP))) > 0;
            // the wave's row records, staged in LDS (rows past the end get
            // an empty record); then rows in groups of kUnroll, all of a
            // group's gathers issued before any is used
            const NodeRec<T>* rrec = recs_of<T>(J, p, 0);
            if (lane < kRowsPerWave) {
                NodeRec<T> r{};
                if (i0 + lane < nR) r = rrec[i0 + lane];
                trec[wave * kRowsPerWave + lane] = r;
            }
            bool long_rows = false;
#pragma unroll 1
            for (int g = 0; g < kRowsPerWave; g += kUnroll) {
                T acc[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u)
                    acc[u] = row_padded<T>(src, nC, trec[wave * kRowsPerWave + g + u], cr);
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const NodeRec<T>& r = trec[wave * kRowsPerWave + g + u];
                    long_rows |= uni(r.ns) > kLS || uni(r.np) > kLP;
                }
                if (long_rows) {
                    GraphRef Rg2, Cg2;
                    state_graphs(J, p, s, &Rg2, &Cg2);
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u) {
                        const NodeRec<T>& r = trec[wave * kRowsPerWave + g + u];
                        if (uni(r.ns) > kLS || uni(r.np) > kLP) acc[u] += row_rest<T>(src, nC, Rg2, i0 + g + u, cr);
                    }
                    long_rows = false;
                }
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int i = i0 + g + u;
                    const T v = acc[u] * sig;
                    if (i < nR && colv) {
                        dst[(long long)i * nC + j] = v;
                        if (!ovf) nu2 += (double)v * (double)v;
                    }
                }
            }
            if (ovf) {
                // the terms of the long lists' later entries, added to the
                // entries this lane has just written (no other lane writes them)
                GraphRef Rg, Cg;
                state_graphs(J, p, s, &Rg, &Cg);
                const int sb = colv ? Cg.rp[j] : 0, pb = colv ? Cg.cp[j] : 0;
                for (int rr = 0; rr < kRowsPerWave; ++rr) {
                    const int i = i0 + rr;
                    if (i >= nR) break;
                    const T add = col_rest<T>(src, nC, Rg, i, Cg, sb, ns, pb, np);
                    if (colv) {
                        const long long o = (long long)i * nC + j;
                        const T v = dst[o] + add * sig;
                        dst[o] = v;
                        nu2 += (double)v * (double)v;
                    }
                }
            }
        } else if (compute) {
            // the first update: Y_1[i][j] = c0 (outw_Rg(i) outw_Cg(j) + inw_Rg(i) inw_Cg(j))
            GraphRef Rg, Cg;
            state_graphs(J, p, s, &Rg, &Cg);
            T ra = T(0), qa = T(0);
            if (colv) {
                const int sb = Cg.rp[j], pb = Cg.cp[j];
                for (int e = 0; e < ns; ++e) ra += T(Cg.w[sb + e]);
                for (int e = 0; e < np; ++e) qa += T(Cg.w[Cg.eid[pb + e]]);
            }
            for (int rr = 0; rr < kRowsPerWave; ++rr) {
                const int i = i0 + rr;
                if (i >= nR) break;
                T rb = T(0), qb = T(0);
                for (int e = Rg.rp[i]; e < Rg.rp[i + 1]; ++e) rb += T(Rg.w[e]);
                for (int e = Rg.cp[i]; e < Rg.cp[i + 1]; ++e) qb += T(Rg.w[Rg.eid[e]]);
                const T acc = c0v * (rb * ra + qb * qa);
                if (colv) {
                    dst[(long long)i * nC + j] = acc;
                    nu2 += (double)acc * (double)acc;
                }
            }
        }
        if (!rz && want_delta) {
            for (int rr = 0; rr < kRowsPerWave; ++rr) {
                const int i = i0 + rr;
                if (i >= nR) break;
                if (colv) {
                    const long long o = (long long)i * nC + j;
                    const T a = T(src[o] * sig);                        // S_{k-1}
                    const T b = old_is_s0 ? c0v : T(old[o] * sig3);     // S_{k-3}
                    const double d = (double)a - (double)b;
                    d2 += d * d;
                }
            }
        }
        if (rz) continue;   // norms of resized pairs come from large_gram
        tile_partials(J, t, nu2, d2, red);
    }
}

// ---------------------------------------------------------------- resize: G, norms
// Launch k (0 .. max_iter + 1) for resized pairs: V_k = U_k G (k <= max_iter;
// U_0 is the constant 1/M), nu_k^2 = <U_k, V_k> (k >= 1), and at odd k >= 3
// delta_{k-1}^2 = <D, D G>, D = U_{k-1} sigma_{k-1} - U_{k-3} sigma_{k-3}.
template <typename T>
__global__ __launch_bounds__(kStepThreads) void large_gram(LargeJob J, int k) {
    __shared__ double red[2 * kNWStep];
    __shared__ double gd[66], ge[66];  // G diagonal and coupling for columns c0 - 1 .. c0 + 64
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const bool compute = k <= J.max_iter;
    const bool want_delta = (k & 1) && k >= 3;
    const TileRange tr = tile_range(J);
    for (long long t = tr.first; t < tr.end; t += tr.stride) {
        const int p = uni(pair_of_tile(J, t));
        LargeState* s = J.st + p;
        if (!uni(s->active) || !uni(s->rz)) continue;
        const Tile tl = tile_at(J, t, s, p);
        const int nR = s->nR, m = s->nC, M = s->M;
        __syncthreads();
        for (int q = tid; q < 66; q += kStepThreads) {
            const int u = tl.c0 - 1 + q;
            double d = 0.0, e = 0.0;
            if (u >= 0 && u < m) gram_entries(u, m, M, &d, &e);
            gd[q] = d;
            ge[q] = u >= 0 && u + 1 < m ? e : 0.0;
        }
        __syncthreads();
        const int j = tl.c0 + lane;
        const bool colv = j < m;
        const int q = lane + 1;  // index of column j in gd/ge
        const double g_l = ge[q - 1], g_d = gd[q], g_r = ge[q];  // G[j][j-1], G[j][j], G[j][j+1]
        const double c0 = 1.0 / (double)M;
        const T* U = buf_of<T>(J, p, kSlotU + (k & 3));
        const T* U1 = buf_of<T>(J, p, kSlotU + ((k - 1) & 3));
        const T* U3 = buf_of<T>(J, p, kSlotU + ((k - 3) & 3));
        T* V = buf_of<T>(J, p, kSlotV);
        const double sig1 = 1.0 / s->nu_k[(k - 1) & 3], sig3 = 1.0 / s->nu_k[(k - 3) & 3];
        double nu2 = 0.0, d2 = 0.0;
        for (int rr = 0; rr < kRowsPerWave; ++rr) {
            const int i = tl.r0 + wave * kRowsPerWave + rr;
            if (i >= nR || !colv) break;
            const long long o = (long long)i * m + j;
            if (compute) {
                double ul, uc, ur;
                if (k == 0) {
                    ul = uc = ur = c0;
                } else {
                    uc = (double)U[o];
                    ul = j > 0 ? (double)U[o - 1] : 0.0;
                    ur = j + 1 < m ? (double)U[o + 1] : 0.0;
                }
                const double v = g_l * ul + g_d * uc + g_r * ur;
                V[o] = T(v);
                if (k >= 1) nu2 += uc * v;
            }
            if (want_delta) {
                auto dval = [&](long long oo) {
                    const double a = (double)U1[oo] * sig1;
                    const double b = k == 3 ? c0 : (double)U3[oo] * sig3;
                    return a - b;
                };
                const double dc = dval(o);
                const double dl = j > 0 ? dval(o - 1) : 0.0;
                const double dr = j + 1 < m ? dval(o + 1) : 0.0;
                d2 += dc * (g_l * dl + g_d * dc + g_r * dr);
            }
        }
        if (k == 0) continue;
        tile_partials(J, t, nu2, d2, red);
    }
}

// ---------------------------------------------------------------- finish
// Three kernels after the last update.  large_final forms the final S (Y_f /
// nu_f; for a resized pair the expansion U_f R^T / nu_f to M x M; S_0 for a
// degenerate pair) and S^T in 32 x 32 tiles through LDS, many workgroups per
// pair.  large_sort_lines sorts every line (each row of S and each row of
// S^T) in the greedy order, many workgroups per pair.  large_finish runs the
// matching rounds on the sorted lines and writes the outputs, one workgroup
// per pair.

// Pair p's final S and S^T, and the slot that receives the sorted lines.
template <typename T>
struct FinalBufs {
    T* S;
    T* St;
    uint16_t* lists;  // row lines [nR][nC], then column lines [nC][nR]
    int nR, nC;
};

template <typename T>
__device__ inline FinalBufs<T> final_bufs(const LargeJob& J, int p, const LargeState* s) {
    FinalBufs<T> b;
    const int f = s->final_step;
    const bool rz = s->rz != 0;
    b.nR = rz ? s->M : s->nB;   // rows of S (B side)
    b.nC = rz ? s->M : s->nA;   // columns of S (A side)
    b.S = rz ? buf_of<T>(J, p, kSlotS) : buf_of<T>(J, p, f & 3);
    b.St = rz ? buf_of<T>(J, p, kSlotU + ((f + 1) & 3)) : buf_of<T>(J, p, (f + 1) & 3);
    b.lists = reinterpret_cast<uint16_t*>(rz ? buf_of<T>(J, p, kSlotU + ((f + 2) & 3)) : buf_of<T>(J, p, (f + 2) & 3));
    return b;
}

constexpr int kFinalThreads = 256;

template <typename T>
__global__ __launch_bounds__(kFinalThreads) void large_final(LargeJob J) {
    __shared__ T tile[32][33];
    const int p = blockIdx.y;
    const LargeState* s = J.st + p;
    if (s->status & CFSIM_INVALID_INPUT) return;
    const FinalBufs<T> fb = final_bufs<T>(J, p, s);
    const int nR = fb.nR, nC = fb.nC, f = s->final_step;
    const bool rz = s->rz != 0;
    const T c0v = T(1.0 / sqrt((double)nR * (double)nC));
    const double sig = f > 0 ? 1.0 / s->nu_k[f & 3] : 1.0;
    const T sigT = T(sig);
    const T* U = rz ? buf_of<T>(J, p, kSlotU + (f & 3)) : nullptr;
    const int m = s->nC, M = s->M;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int ntc = (nC + 31) / 32, ntiles = ((nR + 31) / 32) * ntc;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int i0 = (t / ntc) * 32, j0 = (t % ntc) * 32;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = i0 + ty + 8 * k, j = j0 + tx;
            if (i < nR && j < nC) {
                T v;
                if (f == 0) {
                    v = c0v;
                } else if (!rz) {
                    v = fb.S[(long long)i * nC + j] * sigT;
                } else {
                    // state row r (node of the larger graph), expanded column qq;
                    // the state holds S (swap = 0) or S^T (swap = 1)
                    const int r = s->swap ? j : i, qq = s->swap ? i : j;
                    const Interp ip = interp_at(qq, m, M);
                    const T* urow = U + (long long)r * m;
                    double y;
                    if (ip.r1 == ip.r0)
                        y = (double)urow[ip.r0] * sig;
                    else
                        y = (1.0 - ip.f) * ((double)urow[ip.r0] * sig) + ip.f * ((double)urow[ip.r1] * sig);
                    v = T(y);
                }
                fb.S[(long long)i * nC + j] = v;
                tile[ty + 8 * k][tx] = v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int c = j0 + ty + 8 * k, r = i0 + tx;
            if (c < nC && r < nR) fb.St[(long long)c * nR + r] = tile[tx][ty + 8 * k];
        }
        __syncthreads();
    }
}

// Sort keys of the greedy order along a line: value descending (NaN after
// every number), then partner index ascending (FP32: one 64-bit word).
__device__ inline uint64_t line_key(float v, int y) { return ((uint64_t)dev::desc_bits(v) << 32) | (uint32_t)y; }
__device__ inline uint64_t line_key(double v, int) { return dev::desc_bits(v); }

constexpr int kSortThreads = 256;
constexpr int kSortElems = 2048;  // elements per workgroup pass when lines are short

__host__ __device__ inline int pow2_at_least(int n) {
    int q = 1;
    while (q < n) q <<= 1;
    return q;
}

// Every line of pair blockIdx.y in the greedy order: its partner indices in
// that order, as 16-bit words (nodes < 8192).  Lines take P slots, P the
// next power of two >= max(nR, nC), and are sorted G at a time by one
// bitonic network on G * P elements (P < kSortElems: G = kSortElems / P).
// Merge levels with a partner distance of 8 or more exchange through LDS;
// the three innermost levels run in registers on aligned groups of 8.  FP32
// keys hold the partner index in their low word; FP64 keys keep it apart.
__device__ inline bool key_gt(uint64_t ka, int ia, uint64_t kb, int ib) { return ka > kb || (ka == kb && ia > ib); }

template <typename T>
struct SortBuf {
    uint64_t* k;
    int* i;  // FP64 only
    __device__ void get(int e, uint64_t& kk, int& ii) const {
        kk = k[e];
        ii = sizeof(T) == 8 ? i[e] : 0;
    }
    __device__ void put(int e, uint64_t kk, int ii) const {
        k[e] = kk;
        if constexpr (sizeof(T) == 8) i[e] = ii;
    }
    __device__ int index_of(uint64_t kk, int ii) const { return sizeof(T) == 8 ? ii : (int)(uint32_t)kk; }
};

// Compare-exchange levels j = J0, J0 / 2, ..., 1 of merge size k on the 8
// elements at e0 (aligned to 8; J0 <= 4).
template <typename T>
__device__ inline void sort8(const SortBuf<T>& B, int e0, int k, int J0, int P) {
    uint64_t kk[8];
    int ii[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) B.get(e0 + a, kk[a], ii[a]);
    for (int j = J0; j > 0; j >>= 1) {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            if (a & j) continue;
            const int i = e0 + a;
            const bool up = k == P || (i & k) == 0;
            if (a + j < 8 && key_gt(kk[a], ii[a], kk[a + j], ii[a + j]) == up) {
                const uint64_t tk = kk[a];
                kk[a] = kk[a + j];
                kk[a + j] = tk;
                const int ti = ii[a];
                ii[a] = ii[a + j];
                ii[a + j] = ti;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) B.put(e0 + a, kk[a], ii[a]);
}

template <typename T>
__global__ __launch_bounds__(kSortThreads) void large_sort_lines(LargeJob J) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int p = blockIdx.y;
    const LargeState* s = J.st + p;
    if (s->status & CFSIM_INVALID_INPUT) return;
    const FinalBufs<T> fb = final_bufs<T>(J, p, s);
    const int nR = fb.nR, nC = fb.nC;
    const int P = pow2_at_least(nR > nC ? nR : nC);
    const int G = P >= kSortElems ? 1 : kSortElems / P;
    const int E = G * P, lgP = __builtin_ctz((unsigned)P);
    SortBuf<T> B;
    B.k = reinterpret_cast<uint64_t*>(smem);
    B.i = reinterpret_cast<int*>(smem + (size_t)E * 8);
    const int lines = nR + nC;
    for (int g = blockIdx.x; g * G < lines; g += gridDim.x) {
        for (int e = threadIdx.x; e < E; e += kSortThreads) {
            const int x = g * G + (e >> lgP), y = e & (P - 1);
            uint64_t k = ~0ull;
            int id = INT_MAX;
            if (x < lines) {
                const bool row = x < nR;
                if (y < (row ? nC : nR)) {
                    const T v = row ? fb.S[(long long)x * nC + y] : fb.St[(long long)(x - nR) * nR + y];
                    k = line_key(v, y);
                    id = y;
                }
            }
            B.put(e, k, id);
        }
        __syncthreads();
        // merge sizes 2, 4, 8 stay inside groups of 8
        for (int c = threadIdx.x; c < E / 8; c += kSortThreads)
            for (int k = 2; k <= (P < 8 ? P : 8); k <<= 1) sort8<T>(B, 8 * c, k, k >> 1, P);
        __syncthreads();
        for (int k = 16; k <= P; k <<= 1) {
            for (int j = k >> 1; j >= 8; j >>= 1) {
                for (int q = threadIdx.x; q < E / 2; q += kSortThreads) {
                    const int i = ((q & ~(j - 1)) << 1) | (q & (j - 1));
                    const int l = i + j;
                    const bool up = k == P || (i & k) == 0;  // the last merge of a line is ascending
                    uint64_t ka, kb;
                    int ia, ib;
                    B.get(i, ka, ia);
                    B.get(l, kb, ib);
                    if (key_gt(ka, ia, kb, ib) == up) {
                        B.put(i, kb, ib);
                        B.put(l, ka, ia);
                    }
                }
                __syncthreads();
            }
            for (int c = threadIdx.x; c < E / 8; c += kSortThreads) sort8<T>(B, 8 * c, k, 4, P);
            __syncthreads();
        }
        for (int e = threadIdx.x; e < E; e += kSortThreads) {
            const int x = g * G + (e >> lgP), y = e & (P - 1);
            if (x < lines) {
                const bool row = x < nR;
                if (y < (row ? nC : nR)) {
                    uint64_t kk;
                    int ii;
                    B.get(e, kk, ii);
                    uint16_t* out = row ? fb.lists + (long long)x * nC
                                        : fb.lists + (long long)nR * nC + (long long)(x - nR) * nR;
                    out[y] = (uint16_t)B.index_of(kk, ii);
                }
            }
        }
        __syncthreads();
    }
}

// First position >= q of a sorted line (n entries) whose partner is free
// (state -1), and that partner in y; n and -1 if none.  The entries are read
// W at a time: 8 for the first step (the partner is usually among them), 32
// (about one cache line) after that, so a long run of taken partners costs
// few load latencies.
template <int W>
__device__ inline int free_in_step(const uint16_t* line, int q, int n, const int* state, int& y) {
    int v[W];
#pragma unroll
    for (int a = 0; a < W; ++a) v[a] = q + a < n ? line[q + a] : 0;
    int hit = -1;
#pragma unroll
    for (int a = W - 1; a >= 0; --a)
        if (q + a < n && state[v[a]] == -1) hit = a;
    if (hit >= 0) y = v[hit];
    return hit;
}

__device__ inline int first_free(const uint16_t* line, int q, int n, const int* state, int& y) {
    if (q < n) {
        const int h = free_in_step<8>(line, q, n, state, y);
        if (h >= 0) return q + h;
        q += 8;
    }
    while (q < n) {
        const int h = free_in_step<32>(line, q, n, state, y);
        if (h >= 0) return q + h;
        q += 32;
    }
    y = -1;
    return n;
}

// One workgroup per pair: greedy matching on the sorted lines, margin, outputs
// (LDS: the state of every line, 8 bytes, within large_finish_lds).
template <typename T>
__global__ __launch_bounds__(kFinishThreads) void large_finish(LargeJob J) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NW = kFinishThreads / kWave;
    __shared__ double red[NW];
    __shared__ int s_count;
    const int p = blockIdx.x;
    const int tid = threadIdx.x;
    const LargeState* s = J.st + p;
    cfsim_pair_result* res = J.res + p;
    if (s->status & CFSIM_INVALID_INPUT) {
        if (tid == 0 && !(s->status & kSkipped)) dev::write_invalid(res);
        return;
    }
    const int f = s->final_step;
    const bool rz = s->rz != 0;
    const FinalBufs<T> fb = final_bufs<T>(J, p, s);
    const int nR = fb.nR, nC = fb.nC;
    const long long total = (long long)nR * nC;
    T* S = fb.S;
    const uint16_t* rl = fb.lists;                       // row r's columns in greedy order
    const uint16_t* cl = fb.lists + (long long)nR * nC;  // column c's rows in greedy order

    // Greedy matching by locally dominant rounds: a free row and a free column
    // that are each other's best free partner are matched (the largest free
    // entry always is).  A line's best free partner is the first free one in
    // its sorted order; partners are only ever taken, so each line keeps a
    // pointer into its order that only moves forward, and its current best in
    // LDS: only a line whose best was taken reads its order again.
    int* rstate = reinterpret_cast<int*>(smem);
    int* cstate = rstate + nR;
    uint16_t* rptr = reinterpret_cast<uint16_t*>(cstate + nC);
    uint16_t* cptr = rptr + nR;
    int16_t* rbest = reinterpret_cast<int16_t*>(cptr + nC);   // -1: no free partner left
    int16_t* cbest = rbest + nR;
    for (int r = tid; r < nR; r += kFinishThreads) {
        rstate[r] = -1;
        rptr[r] = 0;
        rbest[r] = -1;
    }
    for (int c = tid; c < nC; c += kFinishThreads) {
        cstate[c] = -1;
        cptr[c] = 0;
        cbest[c] = -1;
    }
    if (tid == 0) s_count = 0;
    __syncthreads();
    const int need = min(nR, nC);
    int done = 0;
    bool first = true;
    while (done < need) {
        for (int r = tid; r < nR; r += kFinishThreads) {
            if (rstate[r] != -1) continue;
            const int b = rbest[r];
            if (!first && (b < 0 || cstate[b] == -1)) continue;   // still the best free partner (or none left)
            int y;
            const int q = first_free(rl + (long long)r * nC, rptr[r], nC, cstate, y);
            rptr[r] = (uint16_t)q;
            rbest[r] = (int16_t)y;
        }
        for (int c = tid; c < nC; c += kFinishThreads) {
            if (cstate[c] != -1) continue;
            const int b = cbest[c];
            if (!first && (b < 0 || rstate[b] == -1)) continue;
            int y;
            const int q = first_free(cl + (long long)c * nR, cptr[c], nR, rstate, y);
            cptr[c] = (uint16_t)q;
            cbest[c] = (int16_t)y;
        }
        first = false;
        __syncthreads();
        for (int r = tid; r < nR; r += kFinishThreads) {
            const int c = rbest[r];
            if (rstate[r] == -1 && c >= 0 && cbest[c] == r) {
                rstate[r] = c;
                cstate[c] = r;
                atomicAdd(&s_count, 1);
            }
        }
        __syncthreads();
        const int now = s_count;  // s_count changes next behind the next round's first barrier
        if (now == done) break;   // guard: the earliest free entry is always a mutual best
        done = now;
    }

    // relative margin of the matching; the picks go to a free slot (a 1 x 1
    // pair, whose slot holds one element, has no rival anyway)
    double margin = __builtin_inf();
    if ((long long)nR + nC <= J.slot_elems) {
        T* pv = rz ? buf_of<T>(J, p, kSlotV) : buf_of<T>(J, p, (f + 3) & 3);
        margin = dev::greedy_margin<T, kFinishThreads>(S, nR, nC, false, rstate, cstate, pv, pv + nR, red);
        __syncthreads();  // red is reused by the score's sum
    }

    const int64_t mo = J.match_off ? J.match_off[p] : 0;
    double sc = 0.0;
    for (int i = tid; i < nR; i += kFinishThreads) {
        const int jj = rstate[i];
        if (jj >= 0) sc += (double)S[(long long)i * nC + jj];
        if (J.match) J.match[mo + i] = jj;
    }
    if (J.S_out) {
        T* So = reinterpret_cast<T*>(J.S_out) + (J.S_off ? J.S_off[p] : 0);
        for (long long o = tid; o < total; o += kFinishThreads) So[o] = S[o];
    }
    const double score = dev::block_sum<NW>(sc, red);
    if (tid == 0) {
        res->score = score;
        res->nu = s->nu;
        res->delta = s->delta;
        res->margin = margin;
        res->iters = f;
        res->status = s->status | (margin <= J.tie_tol ? CFSIM_NEAR_TIE : 0u);
    }
}

}  // namespace

int large_step_grid(int num_cus) { return num_cus * 8; }

size_t large_finish_lds(int max_nodes) { return (size_t)16 * (size_t)max_nodes; }

// Sort workspace in LDS: G * P keys (8 bytes) and, for FP64, indices (4 bytes).
size_t large_sort_lds(int max_nodes, int esize) {
    const int P = pow2_at_least(max_nodes);
    return (size_t)(P > kSortElems ? P : kSortElems) * (esize == 8 ? 12 : 8);
}

int set_large_attributes() {
    int e = 0;
    e |= (int)hipFuncSetAttribute(reinterpret_cast<const void*>(&large_finish<float>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    e |= (int)hipFuncSetAttribute(reinterpret_cast<const void*>(&large_finish<double>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    e |= (int)hipFuncSetAttribute(reinterpret_cast<const void*>(&large_sort_lines<float>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)large_sort_lds(kLargeMaxNodes, 4));
    e |= (int)hipFuncSetAttribute(reinterpret_cast<const void*>(&large_sort_lines<double>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)large_sort_lds(kLargeMaxNodes, 8));
    return e;
}

// The three kernels after the last update.  Workgroups per pair: the 32 x 32
// tiles or line groups of the largest pair, at most 64.
template <typename T>
static int launch_finish(const LargeJob& J, hipStream_t stream) {
    const int tiles = ((J.max_nodes + 31) / 32) * ((J.max_nodes + 31) / 32);
    const int P = pow2_at_least(J.max_nodes);
    const int G = P >= kSortElems ? 1 : kSortElems / P;
    const int groups = (2 * J.max_nodes + G - 1) / G;
    hipLaunchKernelGGL(large_final<T>, dim3(tiles < 64 ? tiles : 64, J.n_pairs), dim3(kFinalThreads), 0, stream, J);
    int e = (int)hipGetLastError();
    if (e != 0) return e;
    hipLaunchKernelGGL(large_sort_lines<T>, dim3(groups < 512 ? groups : 512, J.n_pairs), dim3(kSortThreads),
                       large_sort_lds(J.max_nodes, (int)sizeof(T)), stream, J);
    if ((e = (int)hipGetLastError()) != 0) return e;
    hipLaunchKernelGGL(large_finish<T>, dim3(J.n_pairs), dim3(kFinishThreads), large_finish_lds(J.max_nodes), stream,
                       J);
    return (int)hipGetLastError();
}

template <typename T>
static int launch_large_t(const LargeJob& J, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(large_init<T>, dim3(J.n_pairs), dim3(256), 0, stream, J);
    int e = (int)hipGetLastError();
    if (e != 0) return e;
    hipLaunchKernelGGL(large_scan, dim3(1), dim3(1024), 0, stream, J);
    if ((e = (int)hipGetLastError()) != 0) return e;
    hipLaunchKernelGGL(large_tile_map, dim3(J.n_pairs < 4096 ? J.n_pairs : 4096), dim3(256), 0, stream, J);
    if ((e = (int)hipGetLastError()) != 0) return e;
    // the tile kernels (gathers, matrix-core stages): up to one workgroup
    // per tile, dispatched in tile order (the hardware's dispatch balances
    // tiles of unequal cost better than a grid-stride loop: 1.19 against
    // 1.48 ms per gather launch on 64 pairs of 512-2048 nodes), at most 8x
    // the base grid; a call whose pairs mostly ran elsewhere (a pair filter
    // is set) keeps the base grid, so that its empty launches stay cheap.
    // A multiple of 8 keeps the XCD split of tile_range.
    long long gg = J.filter ? (long long)grid : (long long)J.n_pairs * large_tiles(J.max_nodes);
    gg = gg < 8ll * grid ? gg : 8ll * grid;
    gg = (gg + 7) / 8 * 8;
    const int ggrid = (int)(gg > grid ? gg : grid);
    if (J.mfma) {  // BF16 matrix-core products (plain FP32 pairs)
        if ((e = launch_mfma_prep(J, stream)) != 0) return e;
        for (int k = 1; k <= J.max_iter + 1; ++k) {
            if ((e = launch_mfma_update(J, k, ggrid, stream)) != 0) return e;
            hipLaunchKernelGGL(large_reduce, dim3(J.n_pairs < kReduceGrid ? J.n_pairs : kReduceGrid), dim3(kStepThreads), 0,
                               stream, J, k);
            if ((e = (int)hipGetLastError()) != 0) return e;
        }
        return launch_finish<T>(J, stream);
    }
    if (J.resize) {
        hipLaunchKernelGGL(large_gram<T>, dim3(grid), dim3(kStepThreads), 0, stream, J, 0);
        if ((e = (int)hipGetLastError()) != 0) return e;
    }
    for (int k = 1; k <= J.max_iter + 1; ++k) {
        // each kernel skips the tiles of the other (see large_step)
        if (k == 1 || k == J.max_iter + 1) {
            hipLaunchKernelGGL((large_step<T, true>), dim3(grid), dim3(kStepThreads), 0, stream, J, k);
            if ((e = (int)hipGetLastError()) != 0) return e;
        }
        if (k <= J.max_iter && (k >= 2 || J.resize)) {
            hipLaunchKernelGGL((large_step<T, false>), dim3(ggrid), dim3(kStepThreads), 0, stream, J, k);
            if ((e = (int)hipGetLastError()) != 0) return e;
        }
        if (J.resize) {
            hipLaunchKernelGGL(large_gram<T>, dim3(grid), dim3(kStepThreads), 0, stream, J, k);
            if ((e = (int)hipGetLastError()) != 0) return e;
        }
        hipLaunchKernelGGL(large_reduce, dim3(J.n_pairs < kReduceGrid ? J.n_pairs : kReduceGrid), dim3(kStepThreads), 0,
                               stream, J, k);
        if ((e = (int)hipGetLastError()) != 0) return e;
    }
    return launch_finish<T>(J, stream);
}

int launch_large(int dtype, const LargeJob& J, int grid, hipStream_t stream) {
    return dtype == CFSIM_F64 ? launch_large_t<double>(J, grid, stream) : launch_large_t<float>(J, grid, stream);
}

}  // namespace cfsim
