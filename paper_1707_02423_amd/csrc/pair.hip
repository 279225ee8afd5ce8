// Steps a3-a8 with S resident in LDS: one workgroup scores one CFG pair.
//
//   S_0 = 1/sqrt(n_A n_B); Y = B S A^T + B^T S A; S = Y / ||Y||_F   (Table 1
//   "Iso" read as the normalised power iteration of B (x) A + B^T (x) A^T),
//   even-step test ||S_k - S_{k-2}||_F < tol, greedy matching and score.
//
// Work mapping (CDNA4, wave64).  S is stored n_R x n_C (see PairShape) and
// double-buffered in LDS; wave w owns rows w, w+NW, ... and lane l owns
// columns l, l+64, ...  An entry of the update is the direct double sum
//   Y[i][j] = sum_{u in succ_R(i)} w_iu sum_{v in succ_C(j)} w_jv S[u][v]
//           + sum_{u in pred_R(i)} w_ui sum_{v in pred_C(j)} w_vj S[u][v].
// The R side is wave-uniform: a row's edge lists are broadcast from LDS into
// SGPRs and the code is specialised on the row's (successor, predecessor)
// counts, so every S read of a row is issued back to back.  The C side is per
// lane: the lane's first 2 successors and 3 predecessors (padded with zero
// weights) sit in VGPRs for the whole pair; longer lists add an overflow pass
// reading the staged C lists.  Y goes to the second buffer un-normalised;
// ||Y||^2 is reduced in FP64 in a fixed order and 1/||Y|| is folded into the
// next update (odd k) or applied in place with the even-step test (even k),
// which keeps S_{k-2} in VGPRs.
//
// Matching: greedy in the order (value desc, original flat index asc) equals
// the locally-dominant matching for a strict total order, so it runs in
// parallel rounds: every free row picks its best free column, every free
// column its best free row, mutual picks are matched.
#include <float.h>
#include <limits.h>

#include "cfsim_internal.h"

namespace cfsim {

namespace {

constexpr int kDS = 2;  // successors per lane column held in VGPRs
constexpr int kDP = 3;  // predecessors per lane column held in VGPRs

template <typename T>
struct alignas(sizeof(T) == 8 ? 16 : 8) Edge {
    int32_t u;
    T w;
};

__device__ inline int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline float uni(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ inline double uni(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ inline double wave_sum(double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}
__device__ inline int wave_max(int x) {
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, kWave));
    return x;
}
template <typename T>
__device__ inline bool better(T v, int k, T bv, int bk) {
    return v > bv || (v == bv && k < bk);
}
template <typename T>
__device__ inline void wave_argmax(T& v, int& k, int& c) {
    for (int o = 32; o > 0; o >>= 1) {
        const T ov = __shfl_xor(v, o, kWave);
        const int ok = __shfl_xor(k, o, kWave);
        const int oc = __shfl_xor(c, o, kWave);
        if (better(ov, ok, v, k)) {
            v = ov;
            k = ok;
            c = oc;
        }
    }
}

// Neighbour lists of the lane's column in one 64-column chunk, padded with
// zero weights: the first kDS successors and kDP predecessors as byte offsets
// into a row of S.  Longer lists are finished by the overflow pass.
template <typename T>
struct LaneList {
    int sv[kDS];
    T sw[kDS];
    int pv[kDP];
    T pw[kDP];
};

// Inline record of one R row, read with one broadcast: the first kDS
// successors and kDP predecessors as byte offsets of S rows, their weights,
// and the list lengths (padding has zero weight).
template <typename T>
struct alignas(16) RowRec {
    int ns, np;
    int su[kDS];
    int pu[kDP];
    T sw[kDS];
    T pw[kDP];
};

template <typename T>
__device__ inline T lds_at(const unsigned char* base, int byte_off) {
    return *reinterpret_cast<const T*>(base + byte_off);
}

template <typename T>
__device__ inline void load_lane(const int4* cinfo, const Edge<T>* cse, const Edge<T>* cpe, int c, bool valid,
                                 LaneList<T>& L) {
    const int esz = (int)sizeof(T);
    const int4 ci = cinfo[valid ? c : 0];
    const int sdeg = valid ? ci.y - ci.x : 0;
    const int pdeg = valid ? ci.w - ci.z : 0;
#pragma unroll
    for (int q = 0; q < kDS; ++q) {
        const bool has = q < sdeg;
        const Edge<T> e = cse[has ? ci.x + q : 0];
        L.sv[q] = has ? e.u * esz : 0;
        L.sw[q] = has ? e.w : T(0);
    }
#pragma unroll
    for (int q = 0; q < kDP; ++q) {
        const bool has = q < pdeg;
        const Edge<T> e = cpe[has ? ci.z + q : 0];
        L.pv[q] = has ? e.u * esz : 0;
        L.pw[q] = has ? e.w : T(0);
    }
}

// One R-side term: y + w * sum_q wl[q] S[u][v_q]  (row u at byte offset uo).
template <typename T, int D>
__device__ inline T lane_term(const unsigned char* Sb, int uo, T w, const int (&v)[D], const T (&wl)[D], T y) {
    T a = wl[0] * lds_at<T>(Sb, uo + v[0]);
#pragma unroll
    for (int q = 1; q < D; ++q) a = fma_t(wl[q], lds_at<T>(Sb, uo + v[q]), a);
    return fma_t(w, a, y);
}

// Row update specialised on the row's successor / predecessor counts: every
// S read of the row (all chunks) is independent of the others.
template <typename T, int NCH, int NS, int NP>
__device__ inline void row_fixed(const unsigned char* Sb, const int (&su)[kDS], const T (&sw)[kDS],
                                 const int (&pu)[kDP], const T (&pw)[kDP], const LaneList<T> (&L)[NCH],
                                 T (&y)[NCH]) {
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) y[ch] = T(0);
#pragma unroll
    for (int a = 0; a < NS; ++a)
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) y[ch] = lane_term<T, kDS>(Sb, su[a], sw[a], L[ch].sv, L[ch].sw, y[ch]);
#pragma unroll
    for (int b = 0; b < NP; ++b)
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) y[ch] = lane_term<T, kDP>(Sb, pu[b], pw[b], L[ch].pv, L[ch].pw, y[ch]);
}

// Rows with longer lists: loops over the staged R edges.
template <typename T, int NCH>
__device__ inline void row_loop(const unsigned char* Sb, int rowb, const Edge<T>* se, int ns, const Edge<T>* pe,
                                int np, const LaneList<T> (&L)[NCH], T (&y)[NCH]) {
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) y[ch] = T(0);
    for (int a = 0; a < ns; ++a) {
        const Edge<T> e = se[a];
        const int uo = uni(e.u) * rowb;
        const T w = uni(e.w);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) y[ch] = lane_term<T, kDS>(Sb, uo, w, L[ch].sv, L[ch].sw, y[ch]);
    }
    for (int b = 0; b < np; ++b) {
        const Edge<T> e = pe[b];
        const int uo = uni(e.u) * rowb;
        const T w = uni(e.w);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) y[ch] = lane_term<T, kDP>(Sb, uo, w, L[ch].pv, L[ch].pw, y[ch]);
    }
}

// Lane-list entries past the padded kDS / kDP of column c (long C lists).
template <typename T>
__device__ inline T row_overflow(const unsigned char* Sb, int rowb, const Edge<T>* se, int ns, const Edge<T>* pe,
                                 int np, const int4* cinfo, const Edge<T>* cse, const Edge<T>* cpe, int c,
                                 bool valid) {
    const int esz = (int)sizeof(T);
    const int4 ci = cinfo[valid ? c : 0];
    const int sdeg = valid ? ci.y - ci.x : 0;
    const int pdeg = valid ? ci.w - ci.z : 0;
    T y = T(0);
    for (int a = 0; a < ns; ++a) {
        const Edge<T> e = se[a];
        const int uo = uni(e.u) * rowb;
        T acc = T(0);
        for (int q = kDS; q < sdeg; ++q) {
            const Edge<T> x = cse[ci.x + q];
            acc = fma_t(x.w, lds_at<T>(Sb, uo + x.u * esz), acc);
        }
        y = fma_t(uni(e.w), acc, y);
    }
    for (int b = 0; b < np; ++b) {
        const Edge<T> e = pe[b];
        const int uo = uni(e.u) * rowb;
        T acc = T(0);
        for (int q = kDP; q < pdeg; ++q) {
            const Edge<T> x = cpe[ci.z + q];
            acc = fma_t(x.w, lds_at<T>(Sb, uo + x.u * esz), acc);
        }
        y = fma_t(uni(e.w), acc, y);
    }
    return y;
}

__device__ inline void write_invalid(cfsim_pair_result* r) {
    r->score = __builtin_nan("");
    r->nu = 0.0;
    r->delta = __builtin_inf();
    r->iters = 0;
    r->status = CFSIM_INVALID_INPUT;
}

struct IterOut {
    double nu, delta;
    int iters;
    unsigned status;
    int final_buf;  // 0: S in the first buffer, 1: in the second
};

// ---------------------------------------------------------------- per-pair pieces
// Graphs, orientation and result slot of pair p.
struct PairHdr {
    GraphRef A, B, R, C;
    PairShape sh;
    cfsim_pair_result* res;
};

// Resolves the graphs of pair p; false (and an INVALID result) if unusable.
__device__ inline bool resolve_graphs(const PairJob& J, int p, GraphRef& A, GraphRef& B, cfsim_pair_result*& res) {
    res = J.res + (J.single ? 0 : p);
    if (J.single) {
        A = J.ga;
        B = J.gb;
    } else {
        const int ga = J.pair_a[p], gb = J.pair_b[p];
        if (ga < 0 || ga >= J.set.n_graphs || gb < 0 || gb >= J.set.n_graphs) return false;
        A = graph_of(J.set, ga);
        B = graph_of(J.set, gb);
    }
    return A.n >= 1 && B.n >= 1;
}

// Staged graph lists of one pair in LDS (layout of lds_lists_bytes).
template <typename T>
struct Lists {
    RowRec<T>* rec;
    int2* rstart;
    Edge<T>* sedge;
    Edge<T>* pedge;
    int4* cinfo;
    Edge<T>* csedge;
    Edge<T>* cpedge;
    int *rstate, *rbest, *cstate, *cbest;
};

template <typename T>
__device__ inline Lists<T> carve_lists(unsigned char* base, int nR, int nC, int nnzR, int nnzC) {
    Lists<T> L;
    size_t off = 0;
    L.rec = reinterpret_cast<RowRec<T>*>(base + off);
    off += align16((size_t)nR * sizeof(RowRec<T>));
    L.rstart = reinterpret_cast<int2*>(base + off);
    off += align16((size_t)nR * 8);
    L.sedge = reinterpret_cast<Edge<T>*>(base + off);
    off += align16((size_t)nnzR * sizeof(Edge<T>));
    L.pedge = reinterpret_cast<Edge<T>*>(base + off);
    off += align16((size_t)nnzR * sizeof(Edge<T>));
    L.cinfo = reinterpret_cast<int4*>(base + off);
    off += align16((size_t)nC * 16);
    L.csedge = reinterpret_cast<Edge<T>*>(base + off);
    off += align16((size_t)nnzC * sizeof(Edge<T>));
    L.cpedge = reinterpret_cast<Edge<T>*>(base + off);
    off += align16((size_t)nnzC * sizeof(Edge<T>));
    L.rstate = reinterpret_cast<int*>(base + off);
    off += align16((size_t)nR * 4);
    L.rbest = reinterpret_cast<int*>(base + off);
    off += align16((size_t)nR * 4);
    L.cstate = reinterpret_cast<int*>(base + off);
    off += align16((size_t)nC * 4);
    L.cbest = reinterpret_cast<int*>(base + off);
    return L;
}

// Stages the R rows (inline records) and both edge lists, writes S_0 into S,
// and returns whether the pair is degenerate (a graph without positive weight).
template <typename T, int NT>
__device__ bool stage_pair(const GraphRef& R, const GraphRef& C, int nR, int nC, const Lists<T>& L, T* S, T s0) {
    const int tid = threadIdx.x;
    const int rowb = nC * (int)sizeof(T);
    static_assert(sizeof(RowRec<T>) == (sizeof(T) == 8 ? 80 : 48), "row record size");
    for (int r = tid; r < nR; r += NT) {
        const int sb = R.rp[r], se = R.rp[r + 1], pb = R.cp[r], pe = R.cp[r + 1];
        RowRec<T> x;
        x.ns = se - sb;
        x.np = pe - pb;
#pragma unroll
        for (int q = 0; q < kDS; ++q) {
            const bool has = q < x.ns;
            x.su[q] = has ? R.ci[sb + q] * rowb : 0;
            x.sw[q] = has ? T(R.w[sb + q]) : T(0);
        }
#pragma unroll
        for (int q = 0; q < kDP; ++q) {
            const bool has = q < x.np;
            x.pu[q] = has ? R.ri[pb + q] * rowb : 0;
            x.pw[q] = has ? T(R.w[R.eid[pb + q]]) : T(0);
        }
        L.rec[r] = x;
        L.rstart[r] = make_int2(sb, pb);
    }
    for (int c = tid; c < nC; c += NT) L.cinfo[c] = make_int4(C.rp[c], C.rp[c + 1], C.cp[c], C.cp[c + 1]);
    int posR = 0, posC = 0;
    for (int t = tid; t < R.nnz; t += NT) {
        const double w = R.w[t];
        L.sedge[t].u = R.ci[t];
        L.sedge[t].w = T(w);
        L.pedge[t].u = R.ri[t];
        L.pedge[t].w = T(R.w[R.eid[t]]);
        posR |= (w > 0.0);
    }
    for (int t = tid; t < C.nnz; t += NT) {
        const double w = C.w[t];
        L.csedge[t].u = C.ci[t];
        L.csedge[t].w = T(w);
        L.cpedge[t].u = C.ri[t];
        L.cpedge[t].w = T(C.w[C.eid[t]]);
        posC |= (w > 0.0);
    }
    const long long total = (long long)nR * nC;
    for (long long t = tid; t < total; t += NT) S[t] = s0;
    const int anyR = __syncthreads_or(posR);
    const int anyC = __syncthreads_or(posC);
    return !(anyR && anyC);
}

// One wave's update of row i: y[ch] for its NCH chunks (all S reads of the row
// issued together), plus the overflow of long lane lists.
template <typename T, int NCH>
__device__ inline void update_row(const unsigned char* Sb, int rowb, int i, const RowRec<T>& rr, const Lists<T>& G,
                                  const LaneList<T> (&L)[NCH], const bool (&ovf)[NCH], bool any_ovf,
                                  const int (&col)[NCH], const bool (&cv)[NCH], T (&y)[NCH]) {
    const int ns = uni(rr.ns), np = uni(rr.np);
    int su[kDS], pu[kDP];
    T sw[kDS], pw[kDP];
#pragma unroll
    for (int q = 0; q < kDS; ++q) {
        su[q] = uni(rr.su[q]);
        sw[q] = uni(rr.sw[q]);
    }
#pragma unroll
    for (int q = 0; q < kDP; ++q) {
        pu[q] = uni(rr.pu[q]);
        pw[q] = uni(rr.pw[q]);
    }
    switch (ns <= 2 && np <= 2 ? ns * 3 + np : -1) {
        case 0:
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) y[ch] = T(0);
            break;
        case 1: row_fixed<T, NCH, 0, 1>(Sb, su, sw, pu, pw, L, y); break;
        case 2: row_fixed<T, NCH, 0, 2>(Sb, su, sw, pu, pw, L, y); break;
        case 3: row_fixed<T, NCH, 1, 0>(Sb, su, sw, pu, pw, L, y); break;
        case 4: row_fixed<T, NCH, 1, 1>(Sb, su, sw, pu, pw, L, y); break;
        case 5: row_fixed<T, NCH, 1, 2>(Sb, su, sw, pu, pw, L, y); break;
        case 6: row_fixed<T, NCH, 2, 0>(Sb, su, sw, pu, pw, L, y); break;
        case 7: row_fixed<T, NCH, 2, 1>(Sb, su, sw, pu, pw, L, y); break;
        case 8: row_fixed<T, NCH, 2, 2>(Sb, su, sw, pu, pw, L, y); break;
        default: {
            const int2 st = G.rstart[i];
            row_loop<T, NCH>(Sb, rowb, G.sedge + uni(st.x), ns, G.pedge + uni(st.y), np, L, y);
            break;
        }
    }
    if (any_ovf) {
        const int2 st = G.rstart[i];
        const Edge<T>* se = G.sedge + uni(st.x);
        const Edge<T>* pe = G.pedge + uni(st.y);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
            if (ovf[ch]) y[ch] += row_overflow<T>(Sb, rowb, se, ns, pe, np, G.cinfo, G.csedge, G.cpedge, col[ch], cv[ch]);
    }
}

template <typename T>
__device__ inline void lane_setup(const Lists<T>& G, int ch, int nC, LaneList<T>& L, int& col, bool& cv, bool& ovf) {
    const int c = ch * kWave + (int)(threadIdx.x & (kWave - 1));
    cv = c < nC;
    col = cv ? c : 0;
    load_lane(G.cinfo, G.csedge, G.cpedge, c, cv, L);
    const int4 ci = G.cinfo[col];
    const int extra = cv ? max(ci.y - ci.x - kDS, ci.w - ci.z - kDP) : 0;
    ovf = uni(wave_max(extra)) > 0;
}

// Reduces a per-wave double over the workgroup in a fixed order (every
// thread gets the same value); `red` has NW slots; one barrier.
template <int NW>
__device__ inline double block_sum(double x, double* red) {
    x = wave_sum(x);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = x;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < NW; ++w) t += red[w];
    return t;
}

// Steps a4-a6 with S in LDS (NCH = exact chunk count); S_{k-2} lives in the
// workgroup's global slot Sp.  Returns the buffer holding the final S.
template <typename T, int NT, int NCH>
__device__ IterOut iterate_lds(const PairJob& J, unsigned char* smem, const PairShape& sh, size_t sbytes,
                               const Lists<T>& G, bool degenerate, T* Sp, double* red) {
    constexpr int NW = NT / kWave;
    const int wave = uni((int)threadIdx.x / kWave);
    const int nR = sh.nR, nC = sh.nC;
    const int esz = (int)sizeof(T);
    const int rowb = nC * esz;

    LaneList<T> L[NCH];
    int col[NCH];
    bool cv[NCH], ovf[NCH];
    bool any_ovf = false;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        lane_setup(G, ch, nC, L[ch], col[ch], cv[ch], ovf[ch]);
        any_ovf |= ovf[ch];
    }

    IterOut out{0.0, __builtin_inf(), 0, 0u, 0};
    if (degenerate) {
        out.status = CFSIM_DEGENERATE;
        return out;
    }
    const unsigned char* Sb = smem;     // S_{k-1} (times sigma)
    unsigned char* Nb = smem + sbytes;  // update target
    int cur = 0;
    T sigma = T(1);
    const int last = nR - 1;
    for (int k = 1; k <= J.max_iter; ++k) {
        double nu2 = 0.0;
        RowRec<T> nxt = G.rec[min(wave, last)];
        for (int i = wave; i < nR; i += NW) {
            const RowRec<T> rr = nxt;
            nxt = G.rec[min(i + NW, last)];  // prefetch the wave's next row
            T y[NCH];
            update_row<T, NCH>(Sb, rowb, i, rr, G, L, ovf, any_ovf, col, cv, y);
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const T v = y[ch] * sigma;
                if (cv[ch]) {
                    *reinterpret_cast<T*>(Nb + i * rowb + col[ch] * esz) = v;
                    nu2 += (double)v * (double)v;
                }
            }
        }
        const double tot = block_sum<NW>(nu2, red + (k & 1) * NW);
        if (!(tot > 0.0) || !isfinite(tot)) {  // cannot normalise: keep S_{k-1}
            out.status = CFSIM_DEGENERATE;
            break;
        }
        out.nu = sqrt(tot);
        out.iters = k;
        const T inv = T(1.0 / out.nu);
        {
            const unsigned char* t = Sb;
            Sb = Nb;
            Nb = const_cast<unsigned char*>(t);
            cur ^= 1;
        }
        if (k & 1) {
            sigma = inv;
            continue;
        }
        // even k: normalise in place and take the step against S_{k-2}
        double d2 = 0.0;
        unsigned char* Sw = const_cast<unsigned char*>(Sb);
        for (int i = wave; i < nR; i += NW) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                if (cv[ch]) {
                    T* q = reinterpret_cast<T*>(Sw + i * rowb + col[ch] * esz);
                    T* pq = Sp + i * nC + col[ch];
                    const T sv = *q * inv;
                    const T old = *pq;
                    *q = sv;
                    *pq = sv;
                    const double d = (double)sv - (double)old;
                    d2 += d * d;
                }
            }
        }
        sigma = T(1);
        out.delta = sqrt(block_sum<NW>(d2, red + 2 * NW));
        if (out.delta < J.tol) {
            out.status = CFSIM_CONVERGED;
            break;
        }
    }
    if (out.status == 0) out.status = CFSIM_HIT_MAX_ITER;
    if (sigma != T(1)) {  // stopped after an odd update: normalise
        T* Sw = reinterpret_cast<T*>(const_cast<unsigned char*>(Sb));
        for (int t = threadIdx.x; t < nR * nC; t += NT) Sw[t] *= sigma;
    }
    out.final_buf = cur;
    return out;
}

// Steps a4-a6 with S_cur, S_next and S_{k-2} in global memory (one slot per
// workgroup, L2/MALL resident while the pair runs).  Chunks are processed one
// after the other, each with its lane lists reloaded from LDS.
template <typename T, int NT>
__device__ IterOut iterate_global(const PairJob& J, const PairShape& sh, const Lists<T>& G, T* S0, T* S1, T* Sp,
                                  bool degenerate, double* red) {
    constexpr int NW = NT / kWave;
    const int wave = uni((int)threadIdx.x / kWave);
    const int nR = sh.nR, nC = sh.nC, nchunk = sh.nchunk;
    const int esz = (int)sizeof(T);
    const int rowb = nC * esz;
    const long long total = (long long)nR * nC;

    IterOut out{0.0, __builtin_inf(), 0, 0u, 0};
    if (degenerate) {
        out.status = CFSIM_DEGENERATE;
        return out;
    }
    for (long long t = threadIdx.x; t < total; t += NT) Sp[t] = S0[t];
    const unsigned char* Sb = reinterpret_cast<const unsigned char*>(S0);
    unsigned char* Nb = reinterpret_cast<unsigned char*>(S1);
    int cur = 0;
    T sigma = T(1);
    const int last = nR - 1;
    for (int k = 1; k <= J.max_iter; ++k) {
        double nu2 = 0.0;
        for (int ch = 0; ch < nchunk; ++ch) {
            LaneList<T> L[1];
            int col[1];
            bool cv[1], ovf[1];
            lane_setup(G, ch, nC, L[0], col[0], cv[0], ovf[0]);
            RowRec<T> nxt = G.rec[min(wave, last)];
            for (int i = wave; i < nR; i += NW) {
                const RowRec<T> rr = nxt;
                nxt = G.rec[min(i + NW, last)];
                T y[1];
                update_row<T, 1>(Sb, rowb, i, rr, G, L, ovf, ovf[0], col, cv, y);
                const T v = y[0] * sigma;
                if (cv[0]) {
                    *reinterpret_cast<T*>(Nb + (long long)i * rowb + col[0] * esz) = v;
                    nu2 += (double)v * (double)v;
                }
            }
        }
        const double tot = block_sum<NW>(nu2, red + (k & 1) * NW);
        if (!(tot > 0.0) || !isfinite(tot)) {
            out.status = CFSIM_DEGENERATE;
            break;
        }
        out.nu = sqrt(tot);
        out.iters = k;
        const T inv = T(1.0 / out.nu);
        {
            const unsigned char* t = Sb;
            Sb = Nb;
            Nb = const_cast<unsigned char*>(t);
            cur ^= 1;
        }
        if (k & 1) {
            sigma = inv;
            continue;
        }
        double d2 = 0.0;
        T* Sw = reinterpret_cast<T*>(const_cast<unsigned char*>(Sb));
        for (long long t = threadIdx.x; t < total; t += NT) {
            const T sv = Sw[t] * inv;
            Sw[t] = sv;
            const double d = (double)sv - (double)Sp[t];
            d2 += d * d;
            Sp[t] = sv;
        }
        sigma = T(1);
        out.delta = sqrt(block_sum<NW>(d2, red + 2 * NW));
        if (out.delta < J.tol) {
            out.status = CFSIM_CONVERGED;
            break;
        }
    }
    if (out.status == 0) out.status = CFSIM_HIT_MAX_ITER;
    if (sigma != T(1)) {
        T* Sw = reinterpret_cast<T*>(const_cast<unsigned char*>(Sb));
        for (long long t = threadIdx.x; t < total; t += NT) Sw[t] *= sigma;
        __syncthreads();
    }
    out.final_buf = cur;
    return out;
}

// Step a7 and the outputs: greedy matching by locally-dominant rounds on the
// stored S (compute orientation), score in original row order, S_out, result.
template <typename T, int NT>
__device__ void match_and_write(const PairJob& J, int p, const GraphRef& A, const GraphRef& B, const PairShape& sh,
                                const T* S, const Lists<T>& G, const IterOut& it, cfsim_pair_result* res,
                                double* red, int* s_count) {
    constexpr int NW = NT / kWave;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = uni(tid / kWave);
    const int nR = sh.nR, nC = sh.nC;
    int* rstate = G.rstate;
    int* rbest = G.rbest;
    int* cstate = G.cstate;
    int* cbest = G.cbest;
    for (int r = tid; r < nR; r += NT) rstate[r] = -1;
    for (int c = tid; c < nC; c += NT) cstate[c] = -1;
    if (tid == 0) *s_count = 0;
    __syncthreads();
    const int need = min(nR, nC);
    const bool swp = sh.swap != 0;
    int done = 0;
    while (done < need) {
        for (int r = wave; r < nR; r += NW) {
            if (uni(rstate[r]) != -1) continue;
            T bv = T(-1);
            int bk = INT_MAX, bc = -1;
            for (int c = lane; c < nC; c += kWave) {
                if (cstate[c] == -1) {
                    const T v = S[(long long)r * nC + c];
                    const int key = swp ? c * nR + r : r * nC + c;
                    if (better(v, key, bv, bk)) {
                        bv = v;
                        bk = key;
                        bc = c;
                    }
                }
            }
            wave_argmax(bv, bk, bc);
            if (lane == 0) rbest[r] = bc;
        }
        for (int c = tid; c < nC; c += NT) {
            if (cstate[c] != -1) continue;
            T bv = T(-1);
            int bk = INT_MAX, br = -1;
            for (int r = 0; r < nR; ++r) {
                if (rstate[r] == -1) {
                    const T v = S[(long long)r * nC + c];
                    const int key = swp ? c * nR + r : r * nC + c;
                    if (better(v, key, bv, bk)) {
                        bv = v;
                        bk = key;
                        br = r;
                    }
                }
            }
            cbest[c] = br;
        }
        __syncthreads();
        for (int r = tid; r < nR; r += NT) {
            if (rstate[r] == -1) {
                const int c = rbest[r];
                if (c >= 0 && cbest[c] == r) {
                    rstate[r] = c;
                    cstate[c] = r;
                    atomicAdd(s_count, 1);
                }
            }
        }
        __syncthreads();
        const int now = *s_count;
        __syncthreads();
        if (now == done) break;  // no progress: only possible with non-finite S
        done = now;
    }

    const int nA = A.n, nB = B.n;
    const int64_t mo = (J.single || !J.match_off) ? 0 : J.match_off[p];
    double sc = 0.0;
    for (int i = tid; i < nB; i += NT) {
        int jj;
        T v = T(0);
        if (!swp) {
            jj = rstate[i];
            if (jj >= 0) v = S[(long long)i * nC + jj];
        } else {
            jj = cstate[i];
            if (jj >= 0) v = S[(long long)jj * nC + i];
        }
        if (jj >= 0) sc += (double)v;
        if (J.match) J.match[mo + i] = jj;
    }
    if (J.S_out) {
        const int64_t so = (J.single || !J.S_off) ? 0 : J.S_off[p];
        T* So = reinterpret_cast<T*>(J.S_out) + so;
        const long long total = (long long)nA * nB;
        for (long long o = tid; o < total; o += NT) {
            if (!swp) {
                So[o] = S[o];
            } else {
                const long long i = o / nA, jj = o - i * nA;
                So[o] = S[jj * nC + i];
            }
        }
    }
    const double score = block_sum<NW>(sc, red + 3 * NW);
    if (tid == 0) {
        res->score = score;
        res->nu = it.nu;
        res->delta = it.delta;
        res->iters = it.iters;
        res->status = it.status;
    }
    __syncthreads();
}

template <typename T, int NT, int NCHMAX>
__device__ void lds_pair(const PairJob& J, int p, unsigned char* smem, double* red, int* s_count) {
    GraphRef A{}, B{};
    cfsim_pair_result* res;
    PairShape sh{};
    const bool ok = resolve_graphs(J, p, A, B, res) &&
                    choose_shape(A.n, B.n, A.nnz, B.nnz, J.variant, (int)sizeof(T), &sh) && sh.nchunk <= NCHMAX &&
                    (long long)A.n * B.n <= J.slot_elems;
    if (!ok) {
        if (threadIdx.x == 0) write_invalid(res);
        return;
    }
    const GraphRef R = sh.swap ? A : B;
    const GraphRef C = sh.swap ? B : A;
    const int nR = sh.nR, nC = sh.nC;
    const size_t sbytes = align16((size_t)nR * nC * sizeof(T));
    const Lists<T> G = carve_lists<T>(smem + 2 * sbytes, nR, nC, R.nnz, C.nnz);
    const T s0 = T(1.0 / sqrt((double)nR * (double)nC));
    T* Sp = reinterpret_cast<T*>(J.gws) + (size_t)blockIdx.x * (size_t)J.slot_elems;
    for (int t = threadIdx.x; t < nR * nC; t += NT) Sp[t] = s0;
    const bool degenerate = stage_pair<T, NT>(R, C, nR, nC, G, reinterpret_cast<T*>(smem), s0);
    IterOut it;
    if (sh.nchunk == 1)
        it = iterate_lds<T, NT, 1>(J, smem, sh, sbytes, G, degenerate, Sp, red);
    else if (NCHMAX >= 2 && sh.nchunk == 2)
        it = iterate_lds<T, NT, (NCHMAX >= 2 ? 2 : 1)>(J, smem, sh, sbytes, G, degenerate, Sp, red);
    else
        it = iterate_lds<T, NT, NCHMAX>(J, smem, sh, sbytes, G, degenerate, Sp, red);
    const T* S = reinterpret_cast<const T*>(smem + (it.final_buf ? sbytes : 0));
    match_and_write<T, NT>(J, p, A, B, sh, S, G, it, res, red, s_count);
}

template <typename T, int NT>
__device__ void global_pair(const PairJob& J, int p, unsigned char* smem, double* red, int* s_count) {
    GraphRef A{}, B{};
    cfsim_pair_result* res;
    PairShape sh{};
    const bool ok = resolve_graphs(J, p, A, B, res) &&
                    global_fits(A.n, B.n, A.nnz, B.nnz, (int)sizeof(T), J.slot_elems, &sh);
    if (!ok) {
        if (threadIdx.x == 0) write_invalid(res);
        return;
    }
    const GraphRef R = sh.swap ? A : B;
    const GraphRef C = sh.swap ? B : A;
    const int nR = sh.nR, nC = sh.nC;
    const Lists<T> G = carve_lists<T>(smem, nR, nC, R.nnz, C.nnz);
    T* slot = reinterpret_cast<T*>(J.gws) + (size_t)blockIdx.x * 3 * (size_t)J.slot_elems;
    T* S0 = slot;
    T* S1 = slot + J.slot_elems;
    T* Sp = slot + 2 * J.slot_elems;
    const T s0 = T(1.0 / sqrt((double)nR * (double)nC));
    const bool degenerate = stage_pair<T, NT>(R, C, nR, nC, G, S0, s0);
    const IterOut it = iterate_global<T, NT>(J, sh, G, S0, S1, Sp, degenerate, red);
    match_and_write<T, NT>(J, p, A, B, sh, it.final_buf ? S1 : S0, G, it, res, red, s_count);
}

// Persistent driver: one pair at a time per workgroup, pulled from the
// bucket's queue (or the single pair of the plain path).
template <bool GLOBAL, typename T, int NT, int NCH>
__device__ inline void drive(const PairJob& J, unsigned char* smem, double* red, int* s_item, int* s_count) {
    if (J.single) {
        if (blockIdx.x == 0) {
            if constexpr (GLOBAL)
                global_pair<T, NT>(J, 0, smem, red, s_count);
            else
                lds_pair<T, NT, NCH>(J, 0, smem, red, s_count);
        }
        return;
    }
    const int begin = J.bounds[0], end = J.bounds[1];
    for (;;) {
        if (threadIdx.x == 0) *s_item = begin + atomicAdd(J.queue, 1);
        __syncthreads();
        const int item = *s_item;
        __syncthreads();
        if (item >= end) break;
        if constexpr (GLOBAL)
            global_pair<T, NT>(J, J.order[item], smem, red, s_count);
        else
            lds_pair<T, NT, NCH>(J, J.order[item], smem, red, s_count);
    }
}

// Occupancy the LDS budget of each variant allows (waves per SIMD); the
// register allocation is held to it so that the LDS budget is the limit.
template <int NT>
constexpr int waves_per_simd() {
    return NT == 64 ? 3 : 4;
}

template <typename T, int NT, int NCH>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(waves_per_simd<NT>())))
void pair_lds_kernel(PairJob J) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[4 * (NT / kWave)];
    __shared__ int s_item, s_count;
    drive<false, T, NT, NCH>(J, smem, red, &s_item, &s_count);
}

template <typename T>
__global__ __launch_bounds__(kGlobalThreads) __attribute__((amdgpu_waves_per_eu(4)))
void pair_global_kernel(PairJob J) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[4 * (kGlobalThreads / kWave)];
    __shared__ int s_item, s_count;
    drive<true, T, kGlobalThreads, 1>(J, smem, red, &s_item, &s_count);
}

// Pairs no kernel can take get an INVALID_INPUT result.
__global__ void invalid_kernel(PairJob J) {
    const int begin = J.bounds[0], end = J.bounds[1];
    for (int it = begin + blockIdx.x * blockDim.x + threadIdx.x; it < end; it += gridDim.x * blockDim.x)
        write_invalid(J.res + J.order[it]);
}

// ---------------------------------------------------------------- plan (step a8)
constexpr int kPlanThreads = 1024;
constexpr int kClasses = 128;

__device__ void classify(const PlanJob& P, int64_t p, int* bucket, int* cls) {
    const int ga = P.pair_a[p], gb = P.pair_b[p];
    *cls = 0;
    *bucket = kBucketInvalid;
    if (ga < 0 || ga >= P.set.n_graphs || gb < 0 || gb >= P.set.n_graphs) return;
    const int nA = (int)(P.set.node_off[ga + 1] - P.set.node_off[ga]);
    const int nB = (int)(P.set.node_off[gb + 1] - P.set.node_off[gb]);
    const int mA = (int)(P.set.edge_off[ga + 1] - P.set.edge_off[ga]);
    const int mB = (int)(P.set.edge_off[gb + 1] - P.set.edge_off[gb]);
    if (nA < 1 || nB < 1) return;
    PairShape sh;
    int b = kBucketInvalid;
    for (int v = 0; v < kNumVariants && b == kBucketInvalid; ++v)
        if (choose_shape(nA, nB, mA, mB, v, P.esize, &sh)) b = v;
    if (b == kBucketInvalid && global_fits(nA, nB, mA, mB, P.esize, P.slot_elems, &sh)) b = kBucketGlobal;
    // longest first: cost class from log2 of the work estimate
    const double work = (double)nA * (double)nB * (1.0 + (double)(mA + mB) / (double)(nA + nB + 1));
    int c = (int)(4.0 * log2(work > 1.0 ? work : 1.0));
    c = c < 0 ? 0 : (c >= kClasses ? kClasses - 1 : c);
    *bucket = b;
    *cls = kClasses - 1 - c;
}

__global__ __launch_bounds__(kPlanThreads) void plan_kernel(PlanJob P) {
    __shared__ int hist[kBuckets * kClasses];
    const int tid = threadIdx.x;
    for (int i = tid; i < kBuckets * kClasses; i += kPlanThreads) hist[i] = 0;
    __syncthreads();
    for (int64_t p = tid; p < P.n_pairs; p += kPlanThreads) {
        int b, c;
        classify(P, p, &b, &c);
        atomicAdd(&hist[b * kClasses + c], 1);
    }
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int b = 0; b < kBuckets; ++b) {
            P.bounds[2 * b] = run;
            for (int c = 0; c < kClasses; ++c) {
                const int t = hist[b * kClasses + c];
                hist[b * kClasses + c] = run;
                run += t;
            }
            P.bounds[2 * b + 1] = run;
            P.queues[b] = 0;
        }
    }
    __syncthreads();
    for (int64_t p = tid; p < P.n_pairs; p += kPlanThreads) {
        int b, c;
        classify(P, p, &b, &c);
        const int slot = atomicAdd(&hist[b * kClasses + c], 1);
        P.order[slot] = (int32_t)p;
    }
}

template <typename T, int NT, int NCH>
const void* kernel_ptr() {
    return reinterpret_cast<const void*>(&pair_lds_kernel<T, NT, NCH>);
}

// Instantiations must match variant_info().
const void* variant_kernel(int v, int dtype) {
    if (v == kBucketGlobal)
        return dtype == CFSIM_F64 ? reinterpret_cast<const void*>(&pair_global_kernel<double>)
                                  : reinterpret_cast<const void*>(&pair_global_kernel<float>);
    if (dtype == CFSIM_F64) {
        switch (v) {
            case 0: return kernel_ptr<double, 64, 1>();
            case 1: return kernel_ptr<double, 256, 2>();
            case 2: return kernel_ptr<double, 512, 2>();
            case 3: return kernel_ptr<double, 1024, 2>();
            default: return kernel_ptr<double, 1024, 4>();
        }
    }
    switch (v) {
        case 0: return kernel_ptr<float, 64, 2>();
        case 1: return kernel_ptr<float, 256, 4>();
        case 2: return kernel_ptr<float, 512, 2>();
        case 3: return kernel_ptr<float, 1024, 2>();
        default: return kernel_ptr<float, 1024, 4>();
    }
}

int threads_of(int v, int esize) { return v == kBucketGlobal ? kGlobalThreads : variant_info(v, esize).nt; }
int lds_of(int v, int esize) { return v == kBucketGlobal ? kGlobalLds : variant_info(v, esize).lds_bytes; }

}  // namespace

int launch_pair_lds(int variant, int dtype, const PairJob& job, int grid, hipStream_t stream) {
    if (variant == kBucketInvalid) {
        hipLaunchKernelGGL(invalid_kernel, dim3(64), dim3(256), 0, stream, job);
        return (int)hipGetLastError();
    }
    const int esize = dtype == CFSIM_F64 ? 8 : 4;
    void* args[] = {const_cast<PairJob*>(&job)};
    return (int)hipLaunchKernel(variant_kernel(variant, dtype), dim3(grid), dim3(threads_of(variant, esize)), args,
                                (size_t)lds_of(variant, esize), stream);
}

int launch_plan(const PlanJob& job, hipStream_t stream) {
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(kPlanThreads), 0, stream, job);
    return (int)hipGetLastError();
}

int set_kernel_attributes() {
    int e = 0;
    for (int v = 0; v <= kBucketGlobal; ++v) {
        e |= (int)hipFuncSetAttribute(variant_kernel(v, CFSIM_F32), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      lds_of(v, 4));
        e |= (int)hipFuncSetAttribute(variant_kernel(v, CFSIM_F64), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      lds_of(v, 8));
    }
    return e;
}

int occupancy_of(int variant, int dtype, int* blocks) {
    const int esize = dtype == CFSIM_F64 ? 8 : 4;
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, variant_kernel(variant, dtype),
                                                            threads_of(variant, esize), (size_t)lds_of(variant, esize));
}

}  // namespace cfsim
