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
using dev::wave_argmax;
using dev::wave_sum;

constexpr int kUnroll = 4;                      // rows whose gathers are in flight together
constexpr int kFinishThreads = 1024;
constexpr int kCache = 8;  // cached partners per line in the matching
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

// Interpolation from m to M points at p (m - 1) / (M - 1): row p of R holds
// 1 - f at column r0 and f at column r1 (one entry 1 when r0 = r1).
struct Interp {
    int r0, r1;
    double f;
};
__device__ inline Interp interp_at(int p, int m, int M) {
    Interp q;
    if (M <= 1) {
        q.r0 = q.r1 = 0;
        q.f = 0.0;
        return q;
    }
    const long long num = (long long)p * (m - 1);
    q.r0 = (int)(num / (M - 1));
    q.f = (double)(num - (long long)q.r0 * (M - 1)) / (double)(M - 1);
    q.r1 = q.r0 + 1 < m ? q.r0 + 1 : m - 1;
    return q;
}

// First and last p with r0(p) = u.
__device__ inline void interp_rows(int u, int m, int M, int* plo, int* phi) {
    if (m <= 1) {
        *plo = 0;
        *phi = M - 1;
        return;
    }
    const long long a = (long long)u * (M - 1), b = (long long)(u + 1) * (M - 1);
    *plo = (int)((a + (m - 2)) / (m - 1));
    *phi = u == m - 1 ? M - 1 : (int)((b + (m - 2)) / (m - 1)) - 1;
}

// G = R^T R at column u: diagonal d and the coupling e = G[u][u+1].
__device__ inline void gram_entries(int u, int m, int M, double* d, double* e) {
    double dd = 0.0, ee = 0.0;
    int lo, hi;
    interp_rows(u, m, M, &lo, &hi);
    for (int p = lo; p <= hi; ++p) {
        const Interp q = interp_at(p, m, M);
        if (q.r1 == q.r0) {
            dd += 1.0;  // (1 - f + f)^2 with a single entry
        } else {
            dd += (1.0 - q.f) * (1.0 - q.f);
            ee += (1.0 - q.f) * q.f;
        }
    }
    if (u > 0) {
        interp_rows(u - 1, m, M, &lo, &hi);
        for (int p = lo; p <= hi; ++p) {
            const Interp q = interp_at(p, m, M);
            if (q.r1 == u && q.r0 != q.r1) dd += q.f * q.f;
        }
    }
    *d = dd;
    *e = ee;
}

// ---------------------------------------------------------------- set-up
// One workgroup per pair: validity, degeneracy, state shape, initial state,
// and the node records of the row graph's rows and the column graph's columns.
template <typename T>
__global__ __launch_bounds__(256) void large_init(LargeJob J) {
    const int p = blockIdx.x;
    __shared__ int pos[2];
    LargeState* s = J.st + p;
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
    const int p = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    LargeState* s = J.st + p;
    if (!s->active) return;
    const bool compute = k <= J.max_iter;
    const bool want_delta = (k & 1) && k >= 3;
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
    if (tid != 0) return;
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

// ---------------------------------------------------------------- the operator
// Launch k (1 .. max_iter): X_k = M_{Rg,Cg}(src) * sigma_{k-1} over the state
// (nR x nC).  Plain pairs: src = Y_{k-1} (S_0 is the constant
// 1/sqrt(n_A n_B)), X_k = Y_k into buffer k % 4, plus the norm partials and,
// at odd k >= 3, those of S_{k-1} - S_{k-3}.  Resized pairs: src = V_{k-1},
// X_k = U_k into slot k % 4; large_gram does the rest.  Launch max_iter + 1
// computes only the last change of plain pairs.
template <typename T>
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
        const bool first = k == 1 && !rz;                 // S_0 is the constant
        const bool old_is_s0 = k == 3;
        // the lane column's neighbour lists in Cg (padding has zero weight)
        const NodeRec<T>* rrec = recs_of<T>(J, p, 0);
        NodeRec<T> cr{};
        if (colv) cr = recs_of<T>(J, p, 1)[j];
        const int ns = cr.ns, np = cr.np;
        const bool ovf = uni(dev::wave_max(max(ns - kLS, np - kLP))) > 0;
        // CSR lists are read only by the first update and by long lists
        GraphRef Rg{}, Cg{};
        int sb = 0, pb = 0;
        if (first || ovf) {
            state_graphs(J, p, s, &Rg, &Cg);
            sb = colv ? Cg.rp[j] : 0;
            pb = colv ? Cg.cp[j] : 0;
        }
        double nu2 = 0.0, d2 = 0.0;
        const int i0 = tl.r0 + wave * kRowsPerWave;
        if (compute && !first && !ovf) {
            // the wave's row records, staged in LDS (rows past the end get
            // an empty record); then rows in groups of kUnroll, all of a
            // group's gathers issued before any is used
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
                        nu2 += (double)v * (double)v;
                    }
                }
            }
            if (!rz && want_delta) {
                for (int rr = 0; rr < kRowsPerWave; ++rr) {
                    const int i = i0 + rr;
                    if (i >= nR) break;
                    if (colv) {
                        const long long o = (long long)i * nC + j;
                        const T a = T(src[o] * sig);
                        const T b = old_is_s0 ? c0v : T(old[o] * sig3);
                        const double d = (double)a - (double)b;
                        d2 += d * d;
                    }
                }
            }
            if (rz) continue;
            tile_partials(J, t, nu2, d2, red);
            continue;
        }
        NodeRec<T> nxt = rrec[min(i0, nR - 1)];
        for (int rr = 0; rr < kRowsPerWave; ++rr) {
            const int i = i0 + rr;
            if (i >= nR) break;
            const NodeRec<T> rw = nxt;
            nxt = rrec[min(i + 1, nR - 1)];  // prefetch the wave's next row
            if (compute) {
                T acc = T(0);
                const int nsR = uni(rw.ns), npR = uni(rw.np);
                if (!first && !ovf && nsR <= kLS && npR <= kLP) {
                    int ru[kLS], qu[kLP];
                    T rwt[kLS], qwt[kLP];
#pragma unroll
                    for (int a = 0; a < kLS; ++a) {
                        ru[a] = uni(rw.su[a]);
                        rwt[a] = uni(rw.sw[a]);
                    }
#pragma unroll
                    for (int b = 0; b < kLP; ++b) {
                        qu[b] = uni(rw.pu[b]);
                        qwt[b] = uni(rw.pw[b]);
                    }
                    switch (nsR * 4 + npR) {
                        case 0: break;
                        case 1: acc = row_terms<T, 0, 1>(src, nC, ru, rwt, qu, qwt, cr); break;
                        case 2: acc = row_terms<T, 0, 2>(src, nC, ru, rwt, qu, qwt, cr); break;
                        case 3: acc = row_terms<T, 0, 3>(src, nC, ru, rwt, qu, qwt, cr); break;
                        case 4: acc = row_terms<T, 1, 0>(src, nC, ru, rwt, qu, qwt, cr); break;
                        case 5: acc = row_terms<T, 1, 1>(src, nC, ru, rwt, qu, qwt, cr); break;
                        case 6: acc = row_terms<T, 1, 2>(src, nC, ru, rwt, qu, qwt, cr); break;
                        case 7: acc = row_terms<T, 1, 3>(src, nC, ru, rwt, qu, qwt, cr); break;
                        case 8: acc = row_terms<T, 2, 0>(src, nC, ru, rwt, qu, qwt, cr); break;
                        case 9: acc = row_terms<T, 2, 1>(src, nC, ru, rwt, qu, qwt, cr); break;
                        case 10: acc = row_terms<T, 2, 2>(src, nC, ru, rwt, qu, qwt, cr); break;
                        default: acc = row_terms<T, 2, 3>(src, nC, ru, rwt, qu, qwt, cr); break;
                    }
                    acc *= sig;
                } else if (first) {
                    // S_0 constant: Y_1[i][j] = c0 (outw_Rg(i) outw_Cg(j) + inw_Rg(i) inw_Cg(j))
                    T ra = T(0), rb = T(0), qa = T(0), qb = T(0);
                    if (colv) {
                        for (int e = 0; e < ns; ++e) ra += T(Cg.w[sb + e]);
                        for (int e = 0; e < np; ++e) qa += T(Cg.w[Cg.eid[pb + e]]);
                    }
                    for (int e = Rg.rp[i]; e < Rg.rp[i + 1]; ++e) rb += T(Rg.w[e]);
                    for (int e = Rg.cp[i]; e < Rg.cp[i + 1]; ++e) qb += T(Rg.w[Rg.eid[e]]);
                    acc = c0v * (rb * ra + qb * qa);
                } else {
                    if (!ovf) state_graphs(J, p, s, &Rg, &Cg);  // a row with long lists
                    const int e1 = uni(Rg.rp[i + 1]);
                    for (int e = uni(Rg.rp[i]); e < e1; ++e) {
                        const int u = uni(Rg.ci[e]);
                        const T wu = T(Rg.w[e]);
                        const T* row = src + (long long)u * nC;
                        T in = T(0);
#pragma unroll
                        for (int q = 0; q < kLS; ++q) in = dev::fma_t(cr.sw[q], row[cr.su[q]], in);
                        if (ovf)
                            for (int q = kLS; q < ns; ++q) in = dev::fma_t(T(Cg.w[sb + q]), row[Cg.ci[sb + q]], in);
                        acc = dev::fma_t(wu, in, acc);
                    }
                    const int f1 = uni(Rg.cp[i + 1]);
                    for (int e = uni(Rg.cp[i]); e < f1; ++e) {
                        const int u = uni(Rg.ri[e]);
                        const T wu = T(Rg.w[uni(Rg.eid[e])]);
                        const T* row = src + (long long)u * nC;
                        T in = T(0);
#pragma unroll
                        for (int q = 0; q < kLP; ++q) in = dev::fma_t(cr.pw[q], row[cr.pu[q]], in);
                        if (ovf)
                            for (int q = kLP; q < np; ++q)
                                in = dev::fma_t(T(Cg.w[Cg.eid[pb + q]]), row[Cg.ri[pb + q]], in);
                        acc = dev::fma_t(wu, in, acc);
                    }
                    acc *= sig;
                }
                if (colv) {
                    dst[(long long)i * nC + j] = acc;
                    nu2 += (double)acc * (double)acc;
                }
            }
            if (!rz && want_delta && colv) {
                const long long o = (long long)i * nC + j;
                const T a = T(src[o] * sig);                        // S_{k-1}
                const T b = old_is_s0 ? c0v : T(old[o] * sig3);     // S_{k-3}
                const double d = (double)a - (double)b;
                d2 += d * d;
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
// One workgroup per pair: form the final S (Y_f / nu_f; for a resized pair
// the expansion U_f R^T / nu_f to M x M; S_0 for a degenerate pair), greedy
// matching, outputs.
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
    const int f = s->final_step;
    const bool rz = s->rz != 0;
    const int nR = rz ? s->M : s->nB;   // rows of S (B side)
    const int nC = rz ? s->M : s->nA;   // columns of S (A side)
    const long long total = (long long)nR * nC;
    T* S = rz ? buf_of<T>(J, p, kSlotS) : buf_of<T>(J, p, f & 3);
    if (f == 0) {
        const T c0v = T(1.0 / sqrt((double)nR * (double)nC));
        for (long long o = tid; o < total; o += kFinishThreads) S[o] = c0v;
    } else if (!rz) {
        const T sig = T(1.0 / s->nu_k[f & 3]);
        for (long long o = tid; o < total; o += kFinishThreads) S[o] = S[o] * sig;
    } else {
        // state row r (node of the larger graph), expanded column qq; the
        // state holds S (swap = 0) or S^T (swap = 1)
        const double sig = 1.0 / s->nu_k[f & 3];
        const T* U = buf_of<T>(J, p, kSlotU + (f & 3));
        const int m = s->nC, M = s->M;
        for (long long o = tid; o < total; o += kFinishThreads) {
            const int r = (int)(o / M), qq = (int)(o - (long long)r * M);
            const Interp ip = interp_at(qq, m, M);
            const T* urow = U + (long long)r * m;
            double y;
            if (ip.r1 == ip.r0)
                y = (double)urow[ip.r0] * sig;
            else
                y = (1.0 - ip.f) * ((double)urow[ip.r0] * sig) + ip.f * ((double)urow[ip.r1] * sig);
            if (s->swap)
                S[(long long)qq * M + r] = T(y);
            else
                S[o] = T(y);
        }
    }
    __syncthreads();
    // S^T in a free slot, so that a column's candidates are a contiguous line too
    T* St = rz ? buf_of<T>(J, p, kSlotU + ((f + 1) & 3)) : buf_of<T>(J, p, (f + 1) & 3);
    for (long long o = tid; o < total; o += kFinishThreads) {
        const int r = (int)(o / nC), c = (int)(o - (long long)r * nC);
        St[(long long)c * nR + r] = S[o];
    }
    __syncthreads();
    __threadfence_block();

    // Greedy matching by locally dominant rounds: a free row and a free column
    // that are each other's best free partner are matched (the largest free
    // entry always is).  A stale best (-2) is recomputed by one wave scanning
    // the row of S or the row of S^T (contiguous loads, eight per lane in
    // flight).  The scan keeps each lane's two best free candidates and merges
    // them into a prefix of the line's order (it stops where a lane's third
    // candidate, unseen, could come next), cached in a free slot: when the
    // line's best is taken, its next best free partner is the first cached one
    // still free (partners are only ever taken, so nothing outside the prefix
    // can rank before it), and the line is scanned again only when the cached
    // ones are gone.  Near rank-one S makes every free line stale in every
    // round; the cache saves most of those scans.  (Tiny pairs whose slot
    // cannot hold the cache rescan every stale line.)
    int* cache = (long long)(nR + nC) * kCache * (long long)sizeof(int) <= J.slot_elems * (long long)sizeof(T)
                     ? reinterpret_cast<int*>(rz ? buf_of<T>(J, p, kSlotU + ((f + 2) & 3)) : buf_of<T>(J, p, (f + 2) & 3))
                     : nullptr;
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
    int done = 0;
    while (done < need) {
        for (int it = wave; it < nR + nC; it += NW) {
            const bool is_row = it < nR;
            const int x = is_row ? it : it - nR;
            if (is_row ? (uni(rstate[x]) != -1 || uni(rbest[x]) != -2)
                       : (uni(cstate[x]) != -1 || uni(cbest[x]) != -2))
                continue;
            // candidates: row x of S (free columns) or row x of S^T (free rows)
            const T* line = is_row ? S + (long long)x * nC : St + (long long)x * nR;
            const int n = is_row ? nC : nR;
            const int* other = is_row ? cstate : rstate;
            const int kb = is_row ? x * nC : x, ks = is_row ? 1 : nC;
            // numbers first: NaN entries only if no number is left
            T v1 = T(-__builtin_inf()), v2 = T(-__builtin_inf());
            int k1 = INT_MAX, k2 = INT_MAX, i1 = -1, i2 = -1;
            bool nan_seen = false;
            for (int y0 = lane; y0 < n; y0 += 8 * kWave) {
                T v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int y = y0 + u * kWave;
                    v[u] = y < n ? line[y] : T(-1);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int y = y0 + u * kWave;
                    if (y < n && other[y] == -1) {
                        const int key = kb + y * ks;
                        if (v[u] != v[u]) {
                            nan_seen = true;
                        } else if (v[u] > v2 || (v[u] == v2 && key < k2)) {
                            if (v[u] > v1 || (v[u] == v1 && key < k1)) {
                                v2 = v1;
                                k2 = k1;
                                i2 = i1;
                                v1 = v[u];
                                k1 = key;
                                i1 = y;
                            } else {
                                v2 = v[u];
                                k2 = key;
                                i2 = y;
                            }
                        }
                    }
                }
            }
            int* cl = cache ? cache + (long long)it * kCache : nullptr;
            int head = 0, first = -1, got = 0;
            for (int j = 0; j < kCache; ++j) {
                if (__ballot(head == 2 && i2 >= 0) != 0) break;  // a lane's unseen third could be next
                const T ov = head == 0 ? v1 : (head == 1 ? v2 : T(-__builtin_inf()));
                const int ok = head == 0 ? k1 : (head == 1 ? k2 : INT_MAX);
                const int oi = head == 0 ? i1 : (head == 1 ? i2 : -1);
                T bv = ov;
                int bk = ok, bi = oi;
                wave_argmax(bv, bk, bi);
                if (bi < 0) break;                   // no candidate left
                if (oi == bi && ok == bk) ++head;   // keys are distinct: the one winning lane
                if (cl && lane == 0) cl[j] = bi;
                if (j == 0) first = bi;
                got = j + 1;
            }
            if (first < 0 && __ballot(nan_seen) != 0) {
                // no number left on the line: its free NaN entry with the smallest key
                T z0v = T(-__builtin_inf());
                int nk = INT_MAX, ni = -1;
                for (int y = lane; y < n; y += kWave) {
                    const int key = kb + y * ks;
                    if (other[y] == -1 && line[y] != line[y] && key < nk) {
                        nk = key;
                        ni = y;
                    }
                }
                if (ni >= 0) z0v = T(0);
                wave_argmax(z0v, nk, ni);
                first = ni;
                if (cl && lane == 0) cl[0] = ni;
                got = 1;
            }
            if (cl && lane == 0)
                for (int j = got; j < kCache; ++j) cl[j] = -1;
            if (lane == 0) {
                if (is_row)
                    rbest[x] = first;
                else
                    cbest[x] = first;
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
        // stale bests: the next cached free partner, else a new scan (-2)
        for (int r = tid; r < nR; r += kFinishThreads)
            if (rstate[r] == -1 && rbest[r] >= 0 && cstate[rbest[r]] != -1) {
                int nb = -2;
                if (cache) {
                    const int* cl = cache + (long long)r * kCache;
                    for (int q = 0; q < kCache; ++q) {
                        const int y = cl[q];
                        if (y >= 0 && cstate[y] == -1) {
                            nb = y;
                            break;
                        }
                    }
                }
                rbest[r] = nb;
            }
        for (int c = tid; c < nC; c += kFinishThreads)
            if (cstate[c] == -1 && cbest[c] >= 0 && rstate[cbest[c]] != -1) {
                int nb = -2;
                if (cache) {
                    const int* cl = cache + (long long)(nR + c) * kCache;
                    for (int q = 0; q < kCache; ++q) {
                        const int y = cl[q];
                        if (y >= 0 && rstate[y] == -1) {
                            nb = y;
                            break;
                        }
                    }
                }
                cbest[c] = nb;
            }
        const int now = s_count;
        __syncthreads();
        if (now == done) break;  // guard: the earliest free entry is always a mutual best
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

int set_large_attributes() {
    int e = 0;
    e |= (int)hipFuncSetAttribute(reinterpret_cast<const void*>(&large_finish<float>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    e |= (int)hipFuncSetAttribute(reinterpret_cast<const void*>(&large_finish<double>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    return e;
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
    if (J.mfma) {  // BF16 matrix-core products (plain FP32 pairs)
        if ((e = launch_mfma_prep(J, stream)) != 0) return e;
        for (int k = 1; k <= J.max_iter + 1; ++k) {
            if ((e = launch_mfma_update(J, k, grid, stream)) != 0) return e;
            hipLaunchKernelGGL(large_reduce, dim3(J.n_pairs), dim3(kStepThreads), 0, stream, J, k);
            if ((e = (int)hipGetLastError()) != 0) return e;
        }
        const size_t lds = large_finish_lds(J.max_nodes);
        hipLaunchKernelGGL(large_finish<T>, dim3(J.n_pairs), dim3(kFinishThreads), lds, stream, J);
        return (int)hipGetLastError();
    }
    if (J.resize) {
        hipLaunchKernelGGL(large_gram<T>, dim3(grid), dim3(kStepThreads), 0, stream, J, 0);
        if ((e = (int)hipGetLastError()) != 0) return e;
    }
    for (int k = 1; k <= J.max_iter + 1; ++k) {
        hipLaunchKernelGGL(large_step<T>, dim3(grid), dim3(kStepThreads), 0, stream, J, k);
        if ((e = (int)hipGetLastError()) != 0) return e;
        if (J.resize) {
            hipLaunchKernelGGL(large_gram<T>, dim3(grid), dim3(kStepThreads), 0, stream, J, k);
            if ((e = (int)hipGetLastError()) != 0) return e;
        }
        hipLaunchKernelGGL(large_reduce, dim3(J.n_pairs), dim3(kStepThreads), 0, stream, J, k);
        if ((e = (int)hipGetLastError()) != 0) return e;
    }
    const size_t lds = large_finish_lds(J.max_nodes);
    hipLaunchKernelGGL(large_finish<T>, dim3(J.n_pairs), dim3(kFinishThreads), lds, stream, J);
    return (int)hipGetLastError();
}

int launch_large(int dtype, const LargeJob& J, int grid, hipStream_t stream) {
    return dtype == CFSIM_F64 ? launch_large_t<double>(J, grid, stream) : launch_large_t<float>(J, grid, stream);
}

}  // namespace cfsim
