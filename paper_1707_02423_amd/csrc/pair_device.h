// Device building blocks shared by the forward (pair.hip) and adjoint
// (adjoint.hip) kernels: edge and row records, per-lane neighbour lists, the
// update of one row of Y = B S A^T + B^T S A, staging of a pair's lists into
// LDS, and fixed-order reductions.
#pragma once

#include <float.h>
#include <limits.h>

#include "cfsim_internal.h"

namespace cfsim {
namespace dev {

constexpr int kDS = 2;  // successors per lane column held in VGPRs
constexpr int kDP = 4;  // predecessors per lane column held in VGPRs

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

// Wave reductions without LDS round trips: DPP moves inside each 16-lane row
// (partner = lane ^ 1, lane ^ 2, then the mirrored lane of the half row and of
// the row, which after the first two steps combine disjoint groups), then the
// four row results are read with readlane and combined in a fixed order.
// Every lane returns the same value; the whole wave must be active.
constexpr int kDppXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141; // row_half_mirror
constexpr int kDppMirror = 0x140;     // row_mirror

template <int CTRL>
__device__ inline int dpp(int x) {
    return __builtin_amdgcn_update_dpp(x, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ inline float dpp(float x) {
    return __int_as_float(dpp<CTRL>(__float_as_int(x)));
}
template <int CTRL>
__device__ inline double dpp(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = dpp<CTRL>((int)(b & 0xffffffffll)), hi = dpp<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline int lane_value(int x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ inline float lane_value(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ inline double lane_value(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double wave_fmin(double x) {
    x = fmin(x, dpp<kDppXor1>(x));
    x = fmin(x, dpp<kDppXor2>(x));
    x = fmin(x, dpp<kDppHalfMirror>(x));
    x = fmin(x, dpp<kDppMirror>(x));
    return fmin(fmin(lane_value(x, 0), lane_value(x, 16)), fmin(lane_value(x, 32), lane_value(x, 48)));
}
__device__ inline double wave_sum(double x) {
    x += dpp<kDppXor1>(x);
    x += dpp<kDppXor2>(x);
    x += dpp<kDppHalfMirror>(x);
    x += dpp<kDppMirror>(x);
    return (lane_value(x, 0) + lane_value(x, 16)) + (lane_value(x, 32) + lane_value(x, 48));
}
__device__ inline int wave_max(int x) {
    x = max(x, dpp<kDppXor1>(x));
    x = max(x, dpp<kDppXor2>(x));
    x = max(x, dpp<kDppHalfMirror>(x));
    x = max(x, dpp<kDppMirror>(x));
    return max(max(lane_value(x, 0), lane_value(x, 16)), max(lane_value(x, 32), lane_value(x, 48)));
}
// Greedy order of S entries for the score's matching: value descending, ties by
// the flat row-major index ascending; NaN entries (only from non-finite S)
// come after every number, by index.  better(v, k, bv, bk): (v, k) is
// strictly earlier than (bv, bk).
template <typename T>
__device__ inline bool better(T v, int k, T bv, int bk) {
    const bool vn = v != v, bn = bv != bv;
    if (vn || bn) return vn == bn ? k < bk : bn;
    return v > bv || (v == bv && k < bk);
}

// The same order as one unsigned key per entry (smaller = earlier): the value
// mapped to bits that grow as it falls (NaN largest, -0 as +0), then `lo`.
__device__ inline uint32_t desc_bits(float v) {
    if (v != v) return 0xFFFFFFFFu;
    const uint32_t u = __float_as_uint(v == 0.0f ? 0.0f : v);
    return (u & 0x80000000u) ? u : ~(u | 0x80000000u);
}
__device__ inline uint64_t desc_bits(double v) {
    if (v != v) return ~0ull;
    const uint64_t u = (uint64_t)__double_as_longlong(v == 0.0 ? 0.0 : v);
    return (u & 0x8000000000000000ull) ? u : ~(u | 0x8000000000000000ull);
}
template <typename T>
struct Rank;
template <>
struct Rank<float> {  // value bits and lo packed in one word
    uint64_t k;
    __device__ static Rank make(float v, uint32_t lo) { return Rank{((uint64_t)desc_bits(v) << 32) | lo}; }
    __device__ static Rank none() { return Rank{~0ull}; }
    __device__ bool operator<(const Rank& o) const { return k < o.k; }
    __device__ bool is_none() const { return k == ~0ull; }
    __device__ uint32_t lo() const { return (uint32_t)k; }
    __device__ bool operator==(const Rank& o) const { return k == o.k; }
    __device__ Rank xor_lane(int m) const { return Rank{(uint64_t)__shfl_xor((unsigned long long)k, m)}; }
    template <int CTRL>
    __device__ Rank dpp_move() const {
        const uint32_t lo = (uint32_t)dpp<CTRL>((int)(uint32_t)k);
        const uint32_t hi = (uint32_t)dpp<CTRL>((int)(uint32_t)(k >> 32));
        return Rank{((uint64_t)hi << 32) | lo};
    }
    __device__ Rank read_lane(int ln) const {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)k, ln);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(k >> 32), ln);
        return Rank{((uint64_t)hi << 32) | lo};
    }
};
template <>
struct Rank<double> {
    uint64_t hi;
    uint32_t l;
    __device__ static Rank make(double v, uint32_t lo) { return Rank{desc_bits(v), lo}; }
    __device__ static Rank none() { return Rank{~0ull, ~0u}; }
    __device__ bool operator<(const Rank& o) const { return hi < o.hi || (hi == o.hi && l < o.l); }
    __device__ bool is_none() const { return hi == ~0ull && l == ~0u; }
    __device__ uint32_t lo() const { return l; }
    __device__ bool operator==(const Rank& o) const { return hi == o.hi && l == o.l; }
    __device__ Rank xor_lane(int m) const {
        return Rank{(uint64_t)__shfl_xor((unsigned long long)hi, m), (uint32_t)__shfl_xor((int)l, m)};
    }
    template <int CTRL>
    __device__ Rank dpp_move() const {
        const uint32_t h0 = (uint32_t)dpp<CTRL>((int)(uint32_t)hi);
        const uint32_t h1 = (uint32_t)dpp<CTRL>((int)(uint32_t)(hi >> 32));
        return Rank{((uint64_t)h1 << 32) | h0, (uint32_t)dpp<CTRL>((int)l)};
    }
    __device__ Rank read_lane(int ln) const {
        const uint32_t h0 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)hi, ln);
        const uint32_t h1 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(hi >> 32), ln);
        return Rank{((uint64_t)h1 << 32) | h0, (uint32_t)__builtin_amdgcn_readlane((int)l, ln)};
    }
};
// Smallest rank over the wave (DPP steps inside the 16-lane rows, then the
// four row results), in every lane; the whole wave must be active.
template <int CTRL, typename T>
__device__ inline void rank_min_step(Rank<T>& x) {
    const Rank<T> y = x.template dpp_move<CTRL>();
    if (y < x) x = y;
}
__device__ inline uint32_t wave_min_u32(uint32_t x) {
    x = min(x, (uint32_t)dpp<kDppXor1>((int)x));
    x = min(x, (uint32_t)dpp<kDppXor2>((int)x));
    x = min(x, (uint32_t)dpp<kDppHalfMirror>((int)x));
    x = min(x, (uint32_t)dpp<kDppMirror>((int)x));
    const uint32_t a = min((uint32_t)__builtin_amdgcn_readlane((int)x, 0), (uint32_t)__builtin_amdgcn_readlane((int)x, 16));
    const uint32_t b = min((uint32_t)__builtin_amdgcn_readlane((int)x, 32), (uint32_t)__builtin_amdgcn_readlane((int)x, 48));
    return min(a, b);
}
// FP32 ranks: the value word first, then the key among the lanes that hold
// the smallest value word (two 32-bit reductions instead of one 64-bit one).
__device__ inline Rank<float> wave_min(Rank<float> x) {
    const uint32_t h = (uint32_t)(x.k >> 32);
    const uint32_t hm = wave_min_u32(h);
    const uint32_t lm = wave_min_u32(h == hm ? (uint32_t)x.k : 0xFFFFFFFFu);
    return Rank<float>{((uint64_t)hm << 32) | lm};
}
template <typename T>
__device__ inline Rank<T> wave_min(Rank<T> x) {
    rank_min_step<kDppXor1>(x);
    rank_min_step<kDppXor2>(x);
    rank_min_step<kDppHalfMirror>(x);
    rank_min_step<kDppMirror>(x);
    Rank<T> b = x.read_lane(0);
#pragma unroll
    for (int r = 16; r < kWave; r += 16) {
        const Rank<T> y = x.read_lane(r);
        if (y < b) b = y;
    }
    return b;
}
template <int CTRL, typename T>
__device__ inline void argmax_step(T& v, int& k, int& c) {
    const T ov = dpp<CTRL>(v);
    const int ok = dpp<CTRL>(k);
    const int oc = dpp<CTRL>(c);
    if (better(ov, ok, v, k)) {
        v = ov;
        k = ok;
        c = oc;
    }
}
// Best (value desc, key asc) over the wave; (v, k, c) of the winner in every lane.
template <typename T>
__device__ inline void wave_argmax(T& v, int& k, int& c) {
    argmax_step<kDppXor1>(v, k, c);
    argmax_step<kDppXor2>(v, k, c);
    argmax_step<kDppHalfMirror>(v, k, c);
    argmax_step<kDppMirror>(v, k, c);
    T bv = lane_value(v, 0);
    int bk = lane_value(k, 0), bc = lane_value(c, 0);
#pragma unroll
    for (int r = 16; r < 64; r += 16) {
        const T rv = lane_value(v, r);
        const int rk = lane_value(k, r), rc = lane_value(c, r);
        if (better(rv, rk, bv, bk)) {
            bv = rv;
            bk = rk;
            bc = rc;
        }
    }
    v = bv;
    k = bk;
    c = bc;
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

// Chunks whose S reads are issued together (more would spill registers).
template <typename T>
constexpr int chunks_per_phase() {
    return sizeof(T) == 8 ? 1 : 2;
}

// Row update specialised on the row's successor / predecessor counts: every
// S read of a phase is independent of the others, so all of them are issued
// before the first is used; the scheduling barrier keeps the compiler from
// interleaving them with the arithmetic to save registers, which would leave
// each pair of reads waiting out the LDS latency on its own.
template <typename T, int NCH, int NS, int NP>
__device__ inline void row_fixed(const unsigned char* Sb, const int (&su)[kDS], const T (&sw)[kDS],
                                 const int (&pu)[kDP], const T (&pw)[kDP], const LaneList<T> (&L)[NCH],
                                 T (&y)[NCH]) {
    constexpr int CG = NCH < chunks_per_phase<T>() ? NCH : chunks_per_phase<T>();
#pragma unroll
    for (int c0 = 0; c0 < NCH; c0 += CG) {
        // the phase's S reads are all issued before the arithmetic that uses them
        T xs[NS > 0 ? NS : 1][CG][kDS], xp[NP > 0 ? NP : 1][CG][kDP];
#pragma unroll
        for (int a = 0; a < NS; ++a)
#pragma unroll
            for (int c = 0; c < CG; ++c)
#pragma unroll
                for (int q = 0; q < kDS; ++q) xs[a][c][q] = lds_at<T>(Sb, su[a] + L[c0 + c].sv[q]);
#pragma unroll
        for (int b = 0; b < NP; ++b)
#pragma unroll
            for (int c = 0; c < CG; ++c)
#pragma unroll
                for (int q = 0; q < kDP; ++q) xp[b][c][q] = lds_at<T>(Sb, pu[b] + L[c0 + c].pv[q]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < CG; ++c) {
            const LaneList<T>& l = L[c0 + c];
            T acc = T(0);
#pragma unroll
            for (int a = 0; a < NS; ++a) {
                T t = l.sw[0] * xs[a][c][0];
#pragma unroll
                for (int q = 1; q < kDS; ++q) t = fma_t(l.sw[q], xs[a][c][q], t);
                acc = fma_t(sw[a], t, acc);
            }
#pragma unroll
            for (int b = 0; b < NP; ++b) {
                T t = l.pw[0] * xp[b][c][0];
#pragma unroll
                for (int q = 1; q < kDP; ++q) t = fma_t(l.pw[q], xp[b][c][q], t);
                acc = fma_t(pw[b], t, acc);
            }
            y[c0 + c] = acc;
        }
    }
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
    r->margin = __builtin_nan("");
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

// a if first, else b, field by field (a select of whole structs can leave
// them in scratch memory).
__device__ inline GraphRef pick_graph(bool first, const GraphRef& a, const GraphRef& b) {
    GraphRef g;
    g.n = first ? a.n : b.n;
    g.nnz = first ? a.nnz : b.nnz;
    g.rp = first ? a.rp : b.rp;
    g.ci = first ? a.ci : b.ci;
    g.w = first ? a.w : b.w;
    g.cp = first ? a.cp : b.cp;
    g.ri = first ? a.ri : b.ri;
    g.eid = first ? a.eid : b.eid;
    return g;
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
__device__ __forceinline__ bool stage_pair(const GraphRef& R, const GraphRef& C, int nR, int nC, const Lists<T>& L, T* S, T s0) {
    const int tid = threadIdx.x;
    const int rowb = nC * (int)sizeof(T);
    static_assert(sizeof(RowRec<T>) == (sizeof(T) == 8 ? 80 : 64), "row record size");
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

// Lane-list entries past kDS / kDP for the lanes in `mask` (one chunk), for a
// row whose R terms sit in SGPRs.  Every access is wave-uniform (broadcast
// LDS reads), so a column with a long list costs a few scalar-controlled
// reads per row instead of a divergent loop in every lane.
template <typename T>
__device__ inline T row_extras(const unsigned char* Sb, uint64_t mask, int ch, const Lists<T>& G, int ns, int np,
                               const int (&su)[kDS], const T (&sw)[kDS], const int (&pu)[kDP], const T (&pw)[kDP]) {
    const int esz = (int)sizeof(T);
    const int lane = (int)(threadIdx.x & (kWave - 1));
    T add = T(0);
    while (mask) {
        const int l = (int)__builtin_ctzll(mask);
        mask &= mask - 1;
        const int4 ci = G.cinfo[ch * kWave + l];
        const int se = uni(ci.y), pe = uni(ci.w);
        T acc = T(0);
        for (int q = uni(ci.x) + kDS; q < se; ++q) {
            const Edge<T> e = G.csedge[q];
            const int vo = uni(e.u) * esz;
            T s = T(0);
#pragma unroll
            for (int a = 0; a < kDS; ++a)
                if (a < ns) s = fma_t(sw[a], lds_at<T>(Sb, su[a] + vo), s);
            acc = fma_t(uni(e.w), s, acc);
        }
        for (int q = uni(ci.z) + kDP; q < pe; ++q) {
            const Edge<T> e = G.cpedge[q];
            const int vo = uni(e.u) * esz;
            T s = T(0);
#pragma unroll
            for (int b = 0; b < kDP; ++b)
                if (b < np) s = fma_t(pw[b], lds_at<T>(Sb, pu[b] + vo), s);
            acc = fma_t(uni(e.w), s, acc);
        }
        add += lane == l ? acc : T(0);
    }
    return add;
}

// One wave's update of row i: y[ch] for its NCH chunks (all S reads of the row
// issued together), plus the entries of long lane lists.  L[ch] holds chunk
// ch0 + ch; ovf[ch] is the (uniform) mask of its lanes whose lists exceed
// kDS / kDP.
template <typename T, int NCH>
__device__ inline void update_row(const unsigned char* Sb, int rowb, int i, const RowRec<T>& rr, const Lists<T>& G,
                                  const LaneList<T> (&L)[NCH], const uint64_t (&ovf)[NCH], bool any_ovf,
                                  const int (&col)[NCH], const bool (&cv)[NCH], T (&y)[NCH], int ch0 = 0) {
    // Only the row's class drives control flow and is taken into SGPRs; its
    // offsets and weights stay in VGPRs (a broadcast: every lane holds the same
    // values), which saves a readfirstlane per field and row.
    const int ns = uni(rr.ns), np = uni(rr.np);
    int su[kDS], pu[kDP];
    T sw[kDS], pw[kDP];
#pragma unroll
    for (int q = 0; q < kDS; ++q) {
        su[q] = rr.su[q];
        sw[q] = rr.sw[q];
    }
#pragma unroll
    for (int q = 0; q < kDP; ++q) {
        pu[q] = rr.pu[q];
        pw[q] = rr.pw[q];
    }
    const bool fixed = ns <= kDS && np <= 3;  // the specialised classes
    // the four common CFG rows first (tested on both counts so that the tests
    // stay a chain, most frequent first), the rest through the switch
    if (ns == 1 && np == 1) {
        row_fixed<T, NCH, 1, 1>(Sb, su, sw, pu, pw, L, y);
    } else if (ns == 2 && np == 1) {
        row_fixed<T, NCH, 2, 1>(Sb, su, sw, pu, pw, L, y);
    } else if (ns == 1 && np == 2) {
        row_fixed<T, NCH, 1, 2>(Sb, su, sw, pu, pw, L, y);
    } else if (ns == 2 && np == 2) {
        row_fixed<T, NCH, 2, 2>(Sb, su, sw, pu, pw, L, y);
    } else switch (fixed ? ns * 4 + np : -1) {
        case 0:
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) y[ch] = T(0);
            break;
        case 1: row_fixed<T, NCH, 0, 1>(Sb, su, sw, pu, pw, L, y); break;
        case 2: row_fixed<T, NCH, 0, 2>(Sb, su, sw, pu, pw, L, y); break;
        case 3: row_fixed<T, NCH, 0, 3>(Sb, su, sw, pu, pw, L, y); break;
        case 4: row_fixed<T, NCH, 1, 0>(Sb, su, sw, pu, pw, L, y); break;
        case 7: row_fixed<T, NCH, 1, 3>(Sb, su, sw, pu, pw, L, y); break;
        case 8: row_fixed<T, NCH, 2, 0>(Sb, su, sw, pu, pw, L, y); break;
        case 11: row_fixed<T, NCH, 2, 3>(Sb, su, sw, pu, pw, L, y); break;
        default: {
            const int2 st = G.rstart[i];
            row_loop<T, NCH>(Sb, rowb, G.sedge + uni(st.x), ns, G.pedge + uni(st.y), np, L, y);
            break;
        }
    }
    if (any_ovf) {
        if (fixed) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                if (ovf[ch]) y[ch] += row_extras<T>(Sb, ovf[ch], ch0 + ch, G, ns, np, su, sw, pu, pw);
        } else {
            const int2 st = G.rstart[i];
            const Edge<T>* se = G.sedge + uni(st.x);
            const Edge<T>* pe = G.pedge + uni(st.y);
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                if (ovf[ch])
                    y[ch] += row_overflow<T>(Sb, rowb, se, ns, pe, np, G.cinfo, G.csedge, G.cpedge, col[ch], cv[ch]);
        }
    }
}

// Row classes: 12 specialised (successor, predecessor) counts (ns <= 2,
// np <= 3) and one for every other row.
constexpr int kRowClasses = 13;
__device__ inline int row_class(int ns, int np) { return (ns <= kDS && np <= 3) ? ns * 4 + np : kRowClasses - 1; }

// update_row for a row known to be in class CLS (no dispatch).
template <typename T, int NCH, int CLS>
__device__ __forceinline__ void update_row_class(const unsigned char* Sb, int rowb, int i, const RowRec<T>& rr,
                                                 const Lists<T>& G, const LaneList<T> (&L)[NCH],
                                                 const uint64_t (&ovf)[NCH], bool any_ovf, const int (&col)[NCH],
                                                 const bool (&cv)[NCH], T (&y)[NCH]) {
    int su[kDS], pu[kDP];
    T sw[kDS], pw[kDP];
#pragma unroll
    for (int q = 0; q < kDS; ++q) {
        su[q] = rr.su[q];
        sw[q] = rr.sw[q];
    }
#pragma unroll
    for (int q = 0; q < kDP; ++q) {
        pu[q] = rr.pu[q];
        pw[q] = rr.pw[q];
    }
    if constexpr (CLS == 0) {
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) y[ch] = T(0);
    } else if constexpr (CLS < kRowClasses - 1) {
        row_fixed<T, NCH, CLS / 4, CLS % 4>(Sb, su, sw, pu, pw, L, y);
    }
    if constexpr (CLS < kRowClasses - 1) {
        if (any_ovf) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                if (ovf[ch]) y[ch] += row_extras<T>(Sb, ovf[ch], ch, G, CLS / 4, CLS % 4, su, sw, pu, pw);
        }
    } else {
        const int ns = uni(rr.ns), np = uni(rr.np);
        const int2 st = G.rstart[i];
        const Edge<T>* se = G.sedge + uni(st.x);
        const Edge<T>* pe = G.pedge + uni(st.y);
        row_loop<T, NCH>(Sb, rowb, se, ns, pe, np, L, y);
        if (any_ovf) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                if (ovf[ch])
                    y[ch] += row_overflow<T>(Sb, rowb, se, ns, pe, np, G.cinfo, G.csedge, G.cpedge, col[ch], cv[ch]);
        }
    }
}

// Lane lists of chunk ch; ovf = mask of the lanes whose lists are longer.
template <typename T>
__device__ inline void lane_setup(const Lists<T>& G, int ch, int nC, LaneList<T>& L, int& col, bool& cv,
                                  uint64_t& ovf) {
    const int c = ch * kWave + (int)(threadIdx.x & (kWave - 1));
    cv = c < nC;
    col = cv ? c : 0;
    load_lane(G.cinfo, G.csedge, G.cpedge, c, cv, L);
    const int4 ci = G.cinfo[col];
    const int extra = cv ? max(ci.y - ci.x - kDS, ci.w - ci.z - kDP) : 0;
    ovf = __builtin_amdgcn_ballot_w64(extra > 0);
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

// Smallest per-thread value over the workgroup (every thread gets it); `red`
// has NW slots; one barrier.
template <int NW>
__device__ inline double block_min(double x, double* red) {
    x = wave_fmin(x);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = x;
    __syncthreads();
    double t = red[0];
    for (int w = 1; w < NW; ++w) t = fmin(t, red[w]);
    return t;
}

// Relative margin of a finished greedy matching on S (nR x nC, row stride
// nC; `swp`: S is stored transposed, so the order key of (r, c) is
// c * nR + r).  A rival of the pick (r, c) is an entry of row r or column c
// whose other line was still free when (r, c) was taken, that is, its other
// line is unmatched or matched by a pick later in the greedy order.  The
// margin is the smallest 1 - q / v over picks v and their rivals q (+inf if
// there is none); a pick below the smallest normal number of T counts 0 (its
// relative precision is gone).  Every thread of the workgroup must call it
// after the matching's last barrier; pv_r[nR] and pv_c[nC] are scratch
// (free memory the caller owns); one barrier before the reduction.
template <typename T, int NT>
__device__ inline double greedy_margin(const T* S, int nR, int nC, bool swp, const int* rstate, const int* cstate,
                                       T* pv_r, T* pv_c, double* red) {
    constexpr int NW = NT / kWave;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = uni(tid / kWave);
    for (int r = tid; r < nR; r += NT) {
        const int c = rstate[r];
        pv_r[r] = c >= 0 ? S[(long long)r * nC + c] : T(0);
    }
    for (int c = tid; c < nC; c += NT) {
        const int r = cstate[c];
        pv_c[c] = r >= 0 ? S[(long long)r * nC + c] : T(0);
    }
    __syncthreads();
    const T tiny = sizeof(T) == 8 ? T(DBL_MIN) : T(FLT_MIN);
    double m = __builtin_inf();
    for (int r = wave; r < nR; r += NW) {
        const int pr = uni(rstate[r]);
        const T va = pv_r[r];
        const Rank<T> ra = pr >= 0 ? Rank<T>::make(va, (uint32_t)(swp ? pr * nR + r : r * nC + pr)) : Rank<T>::none();
        const T* line = S + (long long)r * nC;
        for (int c = lane; c < nC; c += kWave) {
            if (c == pr) continue;
            const int pc = cstate[c];
            const T vb = pv_c[c];
            bool row_rival = pr >= 0, col_rival = false;
            if (pc >= 0) {
                const Rank<T> rb = Rank<T>::make(vb, (uint32_t)(swp ? c * nR + pc : pc * nC + c));
                row_rival = pr >= 0 && ra < rb;
                col_rival = !row_rival;
            }
            if (row_rival || col_rival) {
                const T v = row_rival ? va : vb;
                const double rel = v >= tiny ? 1.0 - (double)line[c] / (double)v : 0.0;
                m = fmin(m, rel);
            }
        }
    }
    return block_min<NW>(m, red);
}

}  // namespace dev
}  // namespace cfsim
