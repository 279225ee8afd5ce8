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
// The R side is wave-uniform: a row's record is broadcast from LDS to every
// lane and the code is specialised on the row's (successor, predecessor)
// counts, so every S read of a row is issued back to back.  The C side is per
// lane: the lane's first 2 successors and 4 predecessors (padded with zero
// weights) sit in VGPRs for the whole pair; longer lists add an overflow pass
// reading the staged C lists.  Y goes to the second buffer un-normalised;
// ||Y||^2 is reduced in FP64 in a fixed order and 1/||Y|| is folded into the
// next update; the even-step test needs no third buffer (see EvenSums).
//
// Matching: greedy in the order (value desc, original flat index asc) equals
// the locally-dominant matching for a strict total order, so it runs in
// parallel rounds: every free row picks its best free column, every free
// column its best free row, mutual picks are matched.
#include <float.h>
#include <limits.h>

#include "cfsim_internal.h"
#include "pair_device.h"

namespace cfsim {

namespace {

using namespace dev;

// The kernel's argument block, read anew through a pointer the compiler cannot
// see through: values it loaded from the block before are not reused, so none
// of them is held in registers across a pair's iteration (which needs every
// register it can get to keep its LDS reads in flight).  The block holds the
// one PairJob argument of the pair kernels at offset 0.
__device__ inline const PairJob& job_args() {
    auto p = __builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return *(const PairJob*)p;
}

// The even-step test without a stored S_{k-2}.  The buffers only ever hold
// un-normalised iterates Y_j (S_j = Y_j / nu_j), and an even update k writes
// Y_k over the buffer that holds Y_{k-2}.  Each thread reads the old value of
// every entry it is about to write, so with dy = Y_k - Y_{k-2}, a = 1/nu_{k-2}
// (1 for k = 2, whose S_0 is stored as is) and b = 1/nu_k - a,
//   S_k - S_{k-2} = a dy + b Y_k,
//   ||S_k - S_{k-2}||^2 = a^2 sum dy^2 + 2ab sum dy Y_k + b^2 nu_k^2,
// three FP64 sums taken in the same pass as nu_k^2.  Near convergence dy and b
// are both of the order of the step, so the three terms are small and do not
// cancel from O(1) magnitudes; every entry's difference is formed before any
// squaring, as the direct definition does.
struct EvenSums {
    double nu2, dy2, dyy;
};

// Block reduction of the three even-step sums (red holds 3 * NW doubles).
template <int NW>
__device__ inline EvenSums block_sum_even(EvenSums s, double* red) {
    s.nu2 = wave_sum(s.nu2);
    s.dy2 = wave_sum(s.dy2);
    s.dyy = wave_sum(s.dyy);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        const int w = threadIdx.x / kWave;
        red[w] = s.nu2;
        red[NW + w] = s.dy2;
        red[2 * NW + w] = s.dyy;
    }
    __syncthreads();
    EvenSums t{0.0, 0.0, 0.0};
    for (int w = 0; w < NW; ++w) {
        t.nu2 += red[w];
        t.dy2 += red[NW + w];
        t.dyy += red[2 * NW + w];
    }
    return t;
}

// ||S_k - S_{k-2}|| from the even-step sums (a = 1/nu_{k-2}, inv = 1/nu_k).
__device__ inline double even_step_delta(const EvenSums& t, double a, double inv) {
    const double b = inv - a;
    const double d2 = a * a * t.dy2 + 2.0 * a * b * t.dyy + b * b * t.nu2;
    return sqrt(fmax(d2, 0.0));
}

// Per-entry part of the even-step sums: y_new is the entry written, y_old the
// value it replaces.
template <typename T>
__device__ __forceinline__ void even_terms(EvenSums& s, T y_new, T y_old) {
    const double v = (double)y_new;
    const double dy = v - (double)y_old;
    s.dy2 += dy * dy;
    s.dyy += dy * v;
}

// Rows of class CLS (order[b..e)) of one update, for the one-wave variant:
// a class's rows share one straight-line body, no per-row dispatch.
template <bool EVEN, typename T, int NT, int NCH, int CLS>
__device__ __forceinline__ void class_rows(const int* order, int b, int e, const unsigned char* Sb, unsigned char* Nb,
                                           int rowb, const Lists<T>& G, const LaneList<T> (&L)[NCH],
                                           const uint64_t (&ovf)[NCH], bool any_ovf, const int (&col)[NCH],
                                           const bool (&cv)[NCH], T sigma, EvenSums& es) {
    // b, e come from one LDS word each (the same in every lane) and the loop
    // has no barrier: both hold only while the workgroup is one wave
    static_assert(NT == kWave, "class-ordered rows are for one-wave workgroups");
    for (int k = b; k < e; ++k) {
        const int i = uni(order[k]);
        const RowRec<T> rr = G.rec[i];
        T* dst = reinterpret_cast<T*>(Nb + i * rowb);
        T old[NCH];
        if constexpr (EVEN) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) old[ch] = cv[ch] ? dst[col[ch]] : T(0);
        }
        T y[NCH];
        update_row_class<T, NCH, CLS>(Sb, rowb, i, rr, G, L, ovf, any_ovf, col, cv, y);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const T v = y[ch] * sigma;
            if (cv[ch]) {
                dst[col[ch]] = v;
                es.nu2 += (double)v * (double)v;
                if constexpr (EVEN) even_terms(es, v, old[ch]);
            }
        }
    }
}

// Rows in class order, stable (ascending row index within a class): order[0..nR)
// and the class boundaries seg[0..kRowClasses], by the one wave of the
// workgroup with two ballot passes.
template <typename T, int NT>
__device__ __forceinline__ void order_rows(const Lists<T>& G, int nR, int* order, int* seg) {
    // written by this wave only and read back by it without a barrier
    static_assert(NT == kWave, "class-ordered rows are for one-wave workgroups");
    const int lane = (int)(threadIdx.x & (kWave - 1));
    int cnt[kRowClasses];
#pragma unroll
    for (int c = 0; c < kRowClasses; ++c) cnt[c] = 0;
    for (int base = 0; base < nR; base += kWave) {
        const int r = base + lane;
        const int cls = r < nR ? row_class(G.rec[r].ns, G.rec[r].np) : -1;
#pragma unroll
        for (int c = 0; c < kRowClasses; ++c) cnt[c] += __popcll(__ballot(cls == c));
    }
    int pos[kRowClasses];
    int acc = 0;
#pragma unroll
    for (int c = 0; c < kRowClasses; ++c) {
        pos[c] = acc;
        if (lane == 0) seg[c] = acc;
        acc += cnt[c];
    }
    if (lane == 0) seg[kRowClasses] = acc;
    for (int base = 0; base < nR; base += kWave) {
        const int r = base + lane;
        const int cls = r < nR ? row_class(G.rec[r].ns, G.rec[r].np) : -1;
#pragma unroll
        for (int c = 0; c < kRowClasses; ++c) {
            const uint64_t m = __ballot(cls == c);
            if (cls == c) {
                const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
                order[pos[c] + below] = r;
            }
            pos[c] += __popcll(m);
        }
    }
}

// One update's rows of a wave: Y = (B S A^T + B^T S A) * sigma into Nb, with
// nu^2 and, on even updates (EVEN), the even-step sums.
template <bool EVEN, typename T, int NT, int NCH>
__device__ __forceinline__ void lds_rows(const unsigned char* Sb, unsigned char* Nb, int rowb, int nR, const Lists<T>& G,
                                         const LaneList<T> (&L)[NCH], const uint64_t (&ovf)[NCH], bool any_ovf,
                                         const int (&col)[NCH], const bool (&cv)[NCH], T sigma, EvenSums& es,
                                         const int* order, const int* seg) {
    if constexpr (NT == kWave) {
        // one wave: the rows class by class (for the larger variants the
        // thirteen loop bodies cost more in registers and instruction cache
        // than the dispatch they save)
#define CFSIM_CLASS_ROWS(C)                                                                                       \
    class_rows<EVEN, T, NT, NCH, C>(order, uni(seg[C]), uni(seg[(C) + 1]), Sb, Nb, rowb, G, L, ovf, any_ovf, col, cv, \
                                sigma, es)
        CFSIM_CLASS_ROWS(0);
        CFSIM_CLASS_ROWS(1);
        CFSIM_CLASS_ROWS(2);
        CFSIM_CLASS_ROWS(3);
        CFSIM_CLASS_ROWS(4);
        CFSIM_CLASS_ROWS(5);
        CFSIM_CLASS_ROWS(6);
        CFSIM_CLASS_ROWS(7);
        CFSIM_CLASS_ROWS(8);
        CFSIM_CLASS_ROWS(9);
        CFSIM_CLASS_ROWS(10);
        CFSIM_CLASS_ROWS(11);
        CFSIM_CLASS_ROWS(12);
#undef CFSIM_CLASS_ROWS
        static_assert(kRowClasses == 13, "one call per row class");
        return;
    }
    constexpr int NW = NT / kWave;
    const int wave = uni((int)threadIdx.x / kWave);
    for (int i = wave; i < nR; i += NW) {
        const RowRec<T> rr = G.rec[i];
        T* dst = reinterpret_cast<T*>(Nb + i * rowb);
        T old[NCH];
        if constexpr (EVEN) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) old[ch] = cv[ch] ? dst[col[ch]] : T(0);
        }
        T y[NCH];
        update_row<T, NCH>(Sb, rowb, i, rr, G, L, ovf, any_ovf, col, cv, y);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const T v = y[ch] * sigma;
            if (cv[ch]) {
                dst[col[ch]] = v;
                es.nu2 += (double)v * (double)v;
                if constexpr (EVEN) even_terms(es, v, old[ch]);
            }
        }
    }
}

// Forward checkpoint of update k: S_k = sigma Y_k (Y_k stored in the compute
// orientation) into dst in the n_B x n_A orientation.  Reads only; the next
// update reads the same buffer and writes the other.
template <typename T, int NT>
__device__ __forceinline__ void write_checkpoint(T* dst, const unsigned char* Yb, T sigma, long long total, int nA,
                                                 int nC, bool swp) {
    const T* Y = reinterpret_cast<const T*>(Yb);
    for (long long o = threadIdx.x; o < total; o += NT) {
        if (!swp) {
            dst[o] = Y[o] * sigma;
        } else {
            const long long i = o / nA, jj = o - i * nA;
            dst[o] = Y[jj * nC + i] * sigma;
        }
    }
}

// Checkpoint buffer of pair p (NULL if the call takes none).
template <typename T>
__device__ inline T* checkpoint_base(const PairJob& J, int p) {
    if (!J.ckpt || J.refine) return nullptr;
    return reinterpret_cast<T*>(J.ckpt) + J.ckpt_off[J.single ? 0 : p];
}

// Steps a4-a6 with S in LDS (NCH = exact chunk count).  The two buffers hold
// un-normalised iterates; 1/nu of the stored one (sigma) is folded into the
// next update and applied in place once, at the end.  Returns the buffer
// holding the final S.
template <typename T, int NT, int NCH>
__device__ __forceinline__ IterOut iterate_lds(const PairJob& J, unsigned char* smem, const PairShape& sh, size_t sbytes,
                               const Lists<T>& G, bool degenerate, double* red, const int* seg, T* ck) {
    constexpr int NW = NT / kWave;
    const int nR = sh.nR, nC = sh.nC;
    const int esz = (int)sizeof(T);
    const int rowb = nC * esz;

    LaneList<T> L[NCH];
    int col[NCH];
    bool cv[NCH];
    uint64_t ovf[NCH];
    bool any_ovf = false;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        lane_setup(G, ch, nC, L[ch], col[ch], cv[ch], ovf[ch]);
        any_ovf |= ovf[ch] != 0;
    }

    IterOut out{0.0, __builtin_inf(), 0, 0u, 0};
    if (degenerate) {
        out.status = CFSIM_DEGENERATE;
        return out;
    }
    const unsigned char* Sb = smem;     // Y_{k-1} (S_{k-1} = sigma * Y_{k-1})
    unsigned char* Nb = smem + sbytes;  // update target, holds Y_{k-2}
    int cur = 0;
    T sigma = T(1);
    double a_even = 1.0;  // 1/nu of the last even iterate (S_0 is stored normalised)
    for (int k = 1; k <= J.max_iter; ++k) {
        const bool even = (k & 1) == 0;
        EvenSums es{0.0, 0.0, 0.0};
        if (even)
            lds_rows<true, T, NT, NCH>(Sb, Nb, rowb, nR, G, L, ovf, any_ovf, col, cv, sigma, es, G.rstate, seg);
        else
            lds_rows<false, T, NT, NCH>(Sb, Nb, rowb, nR, G, L, ovf, any_ovf, col, cv, sigma, es, G.rstate, seg);
        double tot;
        if (even)
            es = block_sum_even<NW>(es, red);
        tot = even ? es.nu2 : block_sum<NW>(es.nu2, red + 3 * NW);
        if (!(tot > 0.0) || !isfinite(tot)) {  // cannot normalise: keep S_{k-1}
            out.status = CFSIM_DEGENERATE;
            break;
        }
        out.nu = sqrt(tot);
        out.iters = k;
        const double inv = 1.0 / out.nu;
        sigma = T(inv);
        {
            const unsigned char* t = Sb;
            Sb = Nb;
            Nb = const_cast<unsigned char*>(t);
            cur ^= 1;
        }
        if (ck && k % J.ckpt_every == 0)
            write_checkpoint<T, NT>(ck + (long long)(k / J.ckpt_every - 1) * nR * nC, Sb, sigma, (long long)nR * nC,
                                    sh.swap ? nR : nC, nC, sh.swap != 0);
        if (even) {
            out.delta = even_step_delta(es, a_even, inv);
            a_even = inv;
            if (out.delta < J.tol) {
                out.status = CFSIM_CONVERGED;
                break;
            }
        }
    }
    if (out.status == 0) out.status = CFSIM_HIT_MAX_ITER;
    if (sigma != T(1)) {  // S = sigma * Y (sigma is the same in every thread)
        T* Sw = reinterpret_cast<T*>(const_cast<unsigned char*>(Sb));
        for (int t = threadIdx.x; t < nR * nC; t += NT) Sw[t] *= sigma;
        // the matching reads whole rows across waves
        __syncthreads();
    }
    out.final_buf = cur;
    return out;
}

// Steps a4-a6 with both iterates in global memory (one slot per workgroup,
// L2/MALL resident while the pair runs).  Chunks are processed one after the
// other, each with its lane lists reloaded from LDS.  Same even-step sums and
// folding as the LDS kernel.
template <typename T, int NT>
__device__ __forceinline__ IterOut iterate_global(const PairJob& J, const PairShape& sh, const Lists<T>& G, T* S0, T* S1,
                                  bool degenerate, double* red, T* ck) {
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
    const unsigned char* Sb = reinterpret_cast<const unsigned char*>(S0);
    unsigned char* Nb = reinterpret_cast<unsigned char*>(S1);
    int cur = 0;
    T sigma = T(1);
    double a_even = 1.0;
    const int last = nR - 1;
    for (int k = 1; k <= J.max_iter; ++k) {
        const bool even = (k & 1) == 0;
        EvenSums es{0.0, 0.0, 0.0};
        for (int ch = 0; ch < nchunk; ++ch) {
            LaneList<T> L[1];
            int col[1];
            bool cv[1];
            uint64_t ovf[1];
            lane_setup(G, ch, nC, L[0], col[0], cv[0], ovf[0]);
            RowRec<T> nxt = G.rec[min(wave, last)];
            for (int i = wave; i < nR; i += NW) {
                const RowRec<T> rr = nxt;
                nxt = G.rec[min(i + NW, last)];
                T* dst = reinterpret_cast<T*>(Nb + (long long)i * rowb);
                const T old = (even && cv[0]) ? dst[col[0]] : T(0);
                T y[1];
                update_row<T, 1>(Sb, rowb, i, rr, G, L, ovf, ovf[0] != 0, col, cv, y, ch);
                const T v = y[0] * sigma;
                if (cv[0]) {
                    dst[col[0]] = v;
                    es.nu2 += (double)v * (double)v;
                    if (even) even_terms(es, v, old);
                }
            }
        }
        if (even)
            es = block_sum_even<NW>(es, red);
        const double tot = even ? es.nu2 : block_sum<NW>(es.nu2, red + 3 * NW);
        if (!(tot > 0.0) || !isfinite(tot)) {
            out.status = CFSIM_DEGENERATE;
            break;
        }
        out.nu = sqrt(tot);
        out.iters = k;
        const double inv = 1.0 / out.nu;
        sigma = T(inv);
        {
            const unsigned char* t = Sb;
            Sb = Nb;
            Nb = const_cast<unsigned char*>(t);
            cur ^= 1;
        }
        if (ck && k % J.ckpt_every == 0)
            write_checkpoint<T, NT>(ck + (long long)(k / J.ckpt_every - 1) * nR * nC, Sb, sigma, (long long)nR * nC,
                                    sh.swap ? nR : nC, nC, sh.swap != 0);
        if (even) {
            out.delta = even_step_delta(es, a_even, inv);
            a_even = inv;
            if (out.delta < J.tol) {
                out.status = CFSIM_CONVERGED;
                break;
            }
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

// What a pair kernel computes: the measure of Table 1's "Iso" row as read
// throughout (the normalised power iteration), its damped form, or the
// former with the scale to a common size.
constexpr int kModePlain = 0;
constexpr int kModeDamped = 1;
constexpr int kModeResized = 2;

// ---------------------------------------------------------------- damped measure
// Table 1's "Iso" row in its full form, (I - alpha Q x P) x = (1 - alpha) E,
// read with IsoRank's normalisation: M_hat = M D^-1, D the column sums of the
// coupled operator M = B (x) A + B^T (x) A^T, and a prior E of unit sum.
// Column (u, v) of M sums to
//   d_uv = c^B_u c^A_v + r^B_u r^A_v   (c: column sums, r: row sums),
// so M_hat x = M (x / d) entry by entry: the update is the undamped gather,
// run over Z = x / d.  The two buffers hold Z_k (x_k itself where d = 0: such
// an entry heads a zero column of M and no update reads it with a non-zero
// weight), and an update of entry (i, j) is
//   x_{k+1} = alpha (M Z_k)_ij + (1 - alpha) E_ij,   Z_{k+1} = x_{k+1} / d_ij,
// with x_k = Z_k d_ij (one rounding away) for the stopping test.  Per update,
// in FP64 and a fixed order: delta = ||x_{k+1} - x_k||_1 and ||x_{k+1}||_F^2.
// The iteration contracts by alpha in the 1-norm; it stops at the first
// delta < tol or at max_iter, and S = x / ||x||_F is what the matching reads.

struct DampedSums {
    double d1, n2;
};

// Block reduction of both sums (red holds 2 * NW doubles); one barrier.
template <int NW>
__device__ inline DampedSums block_sum_damped(DampedSums s, double* red) {
    s.d1 = wave_sum(s.d1);
    s.n2 = wave_sum(s.n2);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        red[threadIdx.x / kWave] = s.d1;
        red[NW + threadIdx.x / kWave] = s.n2;
    }
    __syncthreads();
    DampedSums t{0.0, 0.0};
    for (int w = 0; w < NW; ++w) {
        t.d1 += red[w];
        t.n2 += red[NW + w];
    }
    return t;
}

// The prior of a pair: E[i * si + c * sc] * scale for stored entry (i, c),
// or the uniform 1 / (n_A n_B) (= scale) when E is NULL.
struct DampedPrior {
    const double* E;
    long long si, sc;
    double scale;
};

// Row and column sums of the R node of stored row i, from the staged lists.
template <typename T>
__device__ inline void row_node_sums(const Lists<T>& G, int i, int ns, int np, T& r, T& c) {
    const int2 st = G.rstart[i];
    T a = T(0), b = T(0);
    for (int q = 0; q < ns; ++q) a += G.sedge[st.x + q].w;
    for (int q = 0; q < np; ++q) b += G.pedge[st.y + q].w;
    r = a;
    c = b;
}

// Lanes of NCH consecutive 64-column chunks starting at chunk ch0: neighbour
// lists, columns and the row and column sums of each lane's C node.
template <typename T, int NCH>
struct DampedLanes {
    LaneList<T> L[NCH];
    int col[NCH];
    bool cv[NCH];
    uint64_t ovf[NCH];
    bool any_ovf;
    T cr[NCH], cc[NCH];
};

template <typename T, int NCH>
__device__ inline void damped_lanes(const Lists<T>& G, int ch0, int nC, DampedLanes<T, NCH>& c) {
    c.any_ovf = false;
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
        lane_setup(G, ch0 + q, nC, c.L[q], c.col[q], c.cv[q], c.ovf[q]);
        c.any_ovf |= c.ovf[q] != 0;
        T a = T(0), b = T(0);
        if (c.cv[q]) {
            const int4 ci = G.cinfo[c.col[q]];
            for (int t = ci.x; t < ci.y; ++t) a += G.csedge[t].w;
            for (int t = ci.z; t < ci.w; ++t) b += G.cpedge[t].w;
        }
        c.cr[q] = a;
        c.cc[q] = b;
    }
}

template <typename T>
__device__ inline T prior_at(const DampedPrior& P, int i, int c) {
    return P.E ? T(P.E[(long long)i * P.si + (long long)c * P.sc] * P.scale) : T(P.scale);
}

// Passes over the entries of the wave's rows in the chunks of `c`:
// PASS 0: Z_0 = E / d into Zn;  PASS 1: one update Zc -> Zn with the sums;
// PASS 2: S = Z d * inv in place in Zn (the final buffer).
template <int PASS, typename T, int NCH>
__device__ __forceinline__ void damped_pass(const unsigned char* Zc, unsigned char* Zn, int rowb, int nR, int NW,
                                            const Lists<T>& G, const DampedLanes<T, NCH>& c, int ch0, T alpha,
                                            T omega, const DampedPrior& P, T inv, DampedSums& s) {
    const int wave = uni((int)threadIdx.x / kWave);
    for (int i = wave; i < nR; i += NW) {
        const RowRec<T> rr = G.rec[i];
        T rs, cs;
        row_node_sums(G, i, uni(rr.ns), uni(rr.np), rs, cs);
        T y[NCH];
        if constexpr (PASS == 1) update_row<T, NCH>(Zc, rowb, i, rr, G, c.L, c.ovf, c.any_ovf, c.col, c.cv, y, ch0);
        const T* zc = reinterpret_cast<const T*>(Zc + (long long)i * rowb);
        T* zn = reinterpret_cast<T*>(Zn + (long long)i * rowb);
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
            if (!c.cv[q]) continue;
            const int j = c.col[q];
            const T d = fma_t(cs, c.cc[q], rs * c.cr[q]);
            if constexpr (PASS == 0) {
                const T e = prior_at<T>(P, i, j);
                zn[j] = d > T(0) ? e / d : e;
            } else if constexpr (PASS == 1) {
                const T zo = zc[j];
                const T xo = d > T(0) ? zo * d : zo;
                const T xn = fma_t(alpha, y[q], omega * prior_at<T>(P, i, j));
                s.d1 += fabs((double)xn - (double)xo);
                s.n2 += (double)xn * (double)xn;
                zn[j] = d > T(0) ? xn / d : xn;
            } else {
                const T z = zn[j];
                zn[j] = (d > T(0) ? z * d : z) * inv;
            }
        }
    }
}

// The damped iteration of one pair; B0, B1 are the two iterate buffers (LDS,
// or a global-memory slot when GLOBAL, chunk by chunk as in iterate_global).
// Returns the buffer holding S = x / ||x||_F.
template <typename T, int NT, int NCH, bool GLOBAL>
__device__ __forceinline__ IterOut iterate_damped(const PairJob& J, const PairShape& sh, const Lists<T>& G,
                                                  unsigned char* B0, unsigned char* B1, const DampedPrior& P,
                                                  double* red) {
    constexpr int NW = NT / kWave;
    const int nR = sh.nR, nC = sh.nC;
    const int rowb = nC * (int)sizeof(T);
    const T alpha = T(J.alpha), omega = T(1.0 - J.alpha);
    IterOut out{0.0, __builtin_inf(), 0, 0u, 0};
    unsigned char* Zc = B0;
    unsigned char* Zn = B1;
    int cur = 0;
    DampedSums s{0.0, 0.0};
    DampedLanes<T, NCH> lanes;
    if constexpr (!GLOBAL) damped_lanes<T, NCH>(G, 0, nC, lanes);
    auto each_chunk = [&](auto&& f) {
        if constexpr (GLOBAL) {
            for (int ch = 0; ch < sh.nchunk; ++ch) {
                damped_lanes<T, NCH>(G, ch, nC, lanes);
                f(ch);
            }
        } else {
            f(0);
        }
    };
    each_chunk([&](int ch0) {  // Z_0 = E / d into the first buffer
        damped_pass<0, T, NCH>(nullptr, Zc, rowb, nR, NW, G, lanes, ch0, alpha, omega, P, T(1), s);
    });
    __syncthreads();
    double n2 = 0.0;
    for (int k = 1; k <= J.max_iter; ++k) {
        s = DampedSums{0.0, 0.0};
        each_chunk([&](int ch0) {
            damped_pass<1, T, NCH>(Zc, Zn, rowb, nR, NW, G, lanes, ch0, alpha, omega, P, T(1), s);
        });
        // the two reductions of consecutive updates use disjoint slots
        s = block_sum_damped<NW>(s, red + ((k & 1) ? 0 : 2 * NW));
        unsigned char* t = Zc;
        Zc = Zn;
        Zn = t;
        cur ^= 1;
        out.iters = k;
        out.delta = s.d1;
        n2 = s.n2;
        if (s.d1 < J.tol) {
            out.status = CFSIM_CONVERGED;
            break;
        }
    }
    if (out.status == 0) out.status = CFSIM_HIT_MAX_ITER;
    if (!(n2 > 0.0) || !isfinite(n2)) {  // only with max_iter updates of a non-finite prior
        out.status = CFSIM_DEGENERATE;
        n2 = 1.0;
    }
    out.nu = sqrt(n2);
    const T inv = T(1.0 / out.nu);
    each_chunk([&](int ch0) {
        damped_pass<2, T, NCH>(Zc, Zc, rowb, nR, NW, G, lanes, ch0, alpha, omega, P, inv, s);
    });
    __syncthreads();
    out.final_buf = cur;
    return out;
}

// Prior of pair p (uniform when the call has none).  A caller's prior must
// be finite and non-negative with a positive sum, else the pair is invalid
// (false, the same in every thread).
template <typename T, int NT>
__device__ inline bool damped_prior(const PairJob& J, int p, int nA, int nB, const PairShape& sh, DampedPrior& P,
                                    double* red) {
    constexpr int NW = NT / kWave;
    P.E = nullptr;
    P.scale = 1.0 / ((double)nA * (double)nB);
    // stored entry (i, c) is S[i][c], or S[c][i] when the pair is stored transposed
    P.si = sh.swap ? 1 : nA;
    P.sc = sh.swap ? nA : 1;
    if (!J.prior) return true;
    const double* E = J.prior + (J.single ? 0 : J.prior_off[p]);
    const long long total = (long long)nA * nB;
    double part = 0.0;
    int bad = 0;
    for (long long t = threadIdx.x; t < total; t += NT) {
        const double v = E[t];
        bad |= !(v >= 0.0) || !isfinite(v);
        part += v;
    }
    if (__syncthreads_or(bad)) return false;
    const double sum = block_sum<NW>(part, red);
    if (!(sum > 0.0) || !isfinite(sum)) return false;
    P.E = E;
    P.scale = 1.0 / sum;
    return true;
}

// ---------------------------------------------------------------- resized mode
// Scale to a common size (Section 4 and Section 4.1) for a pair of unequal
// sizes: the smaller graph X (m nodes) becomes X' = R X R^T with the M x m
// interpolation R, M the larger node count.  With the larger graph L on the
// rows,
//   Y = L S X'^T + L^T S X' = [L (S R) X^T + L^T (S R) X] R^T,
// so the iteration carries M x m matrices only:
//   U_k = M_{L,X}(V_{k-1}) / nu_{k-1},   V_k = U_k G   (G = R^T R, tridiagonal),
//   nu_k^2 = <U_k, U_k G> = ||Y_k||_F^2,  S_k = U_k R^T / nu_k,
// from U_0 = 1/M (S_0 = 1/M: every row of R sums to 1).  One pass per update
// forms each row of U_k with the plain gathers over V_{k-1}, then that row of
// V_k from U_k's neighbouring columns (lane shuffles; a row's chunks are all
// in one wave) into the other V buffer.  With D = U_k/nu_k - U_{k-2}/nu_{k-2}
// = a dU + b U_k (dU = U_k - U_{k-2}, a = 1/nu_{k-2}, b = 1/nu_k - a),
//   delta^2 = <D, D G> = a^2 <dU, dU G> + 2ab <dU, U_k G> + b^2 nu_k^2,
// three FP64 sums of the same pass (the even-step sums of the plain kernel
// with G applied).  U is kept only at even updates and at the last one, over
// U_{k-2}.  The final S (M x M) is expanded in place for the matching.

// Value of column j - 1 (UP) or j + 1 of the same row: lane shuffles inside a
// chunk, the neighbouring chunk's edge lane across chunks, 0 past the ends.
template <bool LEFT, typename T, int NCH>
__device__ __forceinline__ T neighbour(const T (&x)[NCH], int ch) {
    const int lane = (int)(threadIdx.x & (kWave - 1));
    if constexpr (LEFT) {
        T v = __shfl_up(x[ch], 1, kWave);
        if (lane == 0) v = ch > 0 ? lane_value(x[ch > 0 ? ch - 1 : 0], kWave - 1) : T(0);
        return v;
    } else {
        T v = __shfl_down(x[ch], 1, kWave);
        if (lane == kWave - 1) v = ch + 1 < NCH ? lane_value(x[ch + 1 < NCH ? ch + 1 : 0], 0) : T(0);
        return v;
    }
}

// One update of the resized iteration over the wave's rows: U = sigma M(Vc)
// (written to Ue when STORE), V = U G into Vn, and the sums.
template <bool EVEN, bool STORE, typename T, int NT, int NCH>
__device__ __forceinline__ void resized_rows(const unsigned char* Vc, unsigned char* Vn, unsigned char* Ue, int rowb,
                                             int nR, const Lists<T>& G, const LaneList<T> (&L)[NCH],
                                             const uint64_t (&ovf)[NCH], bool any_ovf, const int (&col)[NCH],
                                             const bool (&cv)[NCH], const T (&gd)[NCH], const T (&ge)[NCH],
                                             const T (&gm)[NCH], T sigma, EvenSums& es) {
    constexpr int NW = NT / kWave;
    const int wave = uni((int)threadIdx.x / kWave);
    for (int i = wave; i < nR; i += NW) {
        const RowRec<T> rr = G.rec[i];
        T y[NCH], u[NCH], du[NCH];
        update_row<T, NCH>(Vc, rowb, i, rr, G, L, ovf, any_ovf, col, cv, y);
        T* ue = reinterpret_cast<T*>(Ue + (long long)i * rowb);
        T* vn = reinterpret_cast<T*>(Vn + (long long)i * rowb);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            u[ch] = cv[ch] ? y[ch] * sigma : T(0);
            du[ch] = T(0);
            if constexpr (STORE) {
                if (cv[ch]) {
                    if constexpr (EVEN) du[ch] = u[ch] - ue[col[ch]];
                    ue[col[ch]] = u[ch];
                }
            }
        }
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const T vg = gm[ch] * neighbour<true, T, NCH>(u, ch) + gd[ch] * u[ch] + ge[ch] * neighbour<false, T, NCH>(u, ch);
            if (cv[ch]) vn[col[ch]] = vg;
            es.nu2 += (double)u[ch] * (double)vg;
            if constexpr (EVEN) {
                const T dg =
                    gm[ch] * neighbour<true, T, NCH>(du, ch) + gd[ch] * du[ch] + ge[ch] * neighbour<false, T, NCH>(du, ch);
                es.dy2 += (double)du[ch] * (double)dg;
                es.dyy += (double)du[ch] * (double)vg;
            }
        }
    }
}

// The resized iteration of one pair (M = nR rows of the larger graph, m = nC
// columns of the smaller); buffers Ue | Va | Vb of B1 bytes each from smem.
// Returns the outcome; S_final = Ue R^T * out.nu^-1 (Ue = 1/M, nu = 1 if degenerate).
template <typename T, int NT, int NCH>
__device__ __forceinline__ IterOut iterate_resized(const PairJob& J, unsigned char* smem, size_t B1,
                                                   const PairShape& sh, const Lists<T>& G, bool degenerate,
                                                   double* red) {
    constexpr int NW = NT / kWave;
    const int wave = uni((int)threadIdx.x / kWave);
    const int M = sh.nR, m = sh.nC;
    const int rowb = m * (int)sizeof(T);
    unsigned char* Ue = smem;
    unsigned char* Vc = smem + B1;
    unsigned char* Vn = smem + 2 * B1;
    LaneList<T> L[NCH];
    int col[NCH];
    bool cv[NCH];
    uint64_t ovf[NCH];
    bool any_ovf = false;
    T gd[NCH], ge[NCH], gm[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        lane_setup(G, ch, m, L[ch], col[ch], cv[ch], ovf[ch]);
        any_ovf |= ovf[ch] != 0;
        double d = 0.0, e = 0.0, el = 0.0, dl = 0.0;
        if (cv[ch]) {
            gram_entries(col[ch], m, M, &d, &e);
            if (col[ch] > 0) gram_entries(col[ch] - 1, m, M, &dl, &el);
        }
        gd[ch] = T(d);
        ge[ch] = T(e);
        gm[ch] = T(el);
    }
    const T u0 = T(1.0 / (double)M);
    for (int i = wave; i < M; i += NW) {
        T* ue = reinterpret_cast<T*>(Ue + (long long)i * rowb);
        T* vc = reinterpret_cast<T*>(Vc + (long long)i * rowb);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
            if (cv[ch]) {
                ue[col[ch]] = u0;
                vc[col[ch]] = u0 * (gm[ch] + gd[ch] + ge[ch]);
            }
    }
    __syncthreads();
    IterOut out{0.0, __builtin_inf(), 0, 0u, 0};
    if (degenerate) {
        out.status = CFSIM_DEGENERATE;
        return out;
    }
    T sigma = T(1);
    double a_even = 1.0;  // 1/nu of the last even iterate (U_0 belongs to nu_0 = 1)
    for (int k = 1; k <= J.max_iter; ++k) {
        const bool even = (k & 1) == 0, last = k == J.max_iter;
        EvenSums es{0.0, 0.0, 0.0};
        if (even)
            resized_rows<true, true, T, NT, NCH>(Vc, Vn, Ue, rowb, M, G, L, ovf, any_ovf, col, cv, gd, ge, gm, sigma,
                                                 es);
        else if (last)
            resized_rows<false, true, T, NT, NCH>(Vc, Vn, Ue, rowb, M, G, L, ovf, any_ovf, col, cv, gd, ge, gm,
                                                  sigma, es);
        else
            resized_rows<false, false, T, NT, NCH>(Vc, Vn, Ue, rowb, M, G, L, ovf, any_ovf, col, cv, gd, ge, gm,
                                                   sigma, es);
        double tot;
        if (even)
            es = block_sum_even<NW>(es, red);
        tot = even ? es.nu2 : block_sum<NW>(es.nu2, red + 3 * NW);
        if (!(tot > 0.0) || !isfinite(tot)) {
            out.status = CFSIM_DEGENERATE;
            break;
        }
        out.nu = sqrt(tot);
        out.iters = k;
        const double inv = 1.0 / out.nu;
        sigma = T(inv);
        unsigned char* t = Vc;
        Vc = Vn;
        Vn = t;
        if (even) {
            out.delta = even_step_delta(es, a_even, inv);
            a_even = inv;
            if (out.delta < J.tol) {
                out.status = CFSIM_CONVERGED;
                break;
            }
        } else if (last) {
            // the last update is odd: U_k stands in Ue and the loop ends
        }
    }
    if (out.status == 0) out.status = CFSIM_HIT_MAX_ITER;
    return out;
}

// S = U R^T * inv (M x M) over U (M x m) in place, both from smem: rows are
// expanded from the last group of NW rows to the first; a group reads its U
// rows into registers, waits, and writes its S rows, whose bytes only cover
// U rows at or after their own (M >= m).
template <typename T, int NT>
__device__ __forceinline__ void expand_resized(unsigned char* smem, int M, int m, T inv) {
    constexpr int NW = NT / kWave;
    constexpr int MCH = 4;  // output chunks of 64 columns: M <= 256 (the LDS and global fits ensure it)
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int wave = (int)threadIdx.x / kWave;
    T* U = reinterpret_cast<T*>(smem);
    const int groups = (M + NW - 1) / NW;
    for (int g = groups - 1; g >= 0; --g) {
        const int i = g * NW + wave;
        T o[MCH];
#pragma unroll
        for (int c = 0; c < MCH; ++c) {
            const int q = c * kWave + lane;
            o[c] = T(0);
            if (i < M && q < M) {
                const Interp ip = interp_at(q, m, M);
                const T* ur = U + (long long)i * m;
                o[c] = (T(1.0 - ip.f) * ur[ip.r0] + T(ip.f) * ur[ip.r1]) * inv;
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < MCH; ++c) {
            const int q = c * kWave + lane;
            if (i < M && q < M) U[(long long)i * M + q] = o[c];
        }
    }
    __syncthreads();
}

// Step a7, rows of at most kSortCols entries: the greedy order itself.  Each
// stored row's columns are sorted once in that order (bitonic network, one
// wave per row, 64 * E slots); then one wave repeats: the earliest entry among
// every free row's first free column is matched, and rows whose column was
// just taken move their pointer on past taken columns.  Each step is a wave
// reduction instead of a workgroup round, which matters for nearly rank-one S,
// where rounds of mutual bests match one pair each.  The sorted lists (16-bit
// column indices) live in St; rptr in the lists' space, free by now.
constexpr int kSortCols = 256;

// One stage of the bitonic network over 64 * E slots (slot m * 64 + lane) of
// RG independent rows, then the rest of the network; compile-time sizes keep
// x[][] in registers.
template <typename T, int E, int RG, int SIZE, int STRIDE>
__device__ __forceinline__ void bitonic_from(Rank<T> (&x)[RG][E], int lane) {
    if constexpr (SIZE <= kWave * E) {
        if constexpr (STRIDE == 0) {
            bitonic_from<T, E, RG, SIZE * 2, SIZE>(x, lane);
        } else {
            if constexpr (STRIDE >= kWave) {  // partner in the same lane
                constexpr int MS = STRIDE / kWave;
#pragma unroll
                for (int g = 0; g < RG; ++g)
#pragma unroll
                    for (int m = 0; m < E; ++m) {
                        if ((m & MS) == 0) {
                            const bool up = ((m * kWave) & SIZE) == 0;
                            const Rank<T> a = x[g][m], b = x[g][m | MS];
                            if (up ? (b < a) : (a < b)) {
                                x[g][m] = b;
                                x[g][m | MS] = a;
                            }
                        }
                    }
            } else {
                Rank<T> y[RG][E];
#pragma unroll
                for (int g = 0; g < RG; ++g)
#pragma unroll
                    for (int m = 0; m < E; ++m) y[g][m] = x[g][m].xor_lane(STRIDE);
#pragma unroll
                for (int g = 0; g < RG; ++g)
#pragma unroll
                    for (int m = 0; m < E; ++m) {
                        const int i = m * kWave + lane;
                        const bool keep_min = ((i & STRIDE) == 0) == ((i & SIZE) == 0);
                        if (keep_min ? (y[g][m] < x[g][m]) : (x[g][m] < y[g][m])) x[g][m] = y[g][m];
                    }
            }
            bitonic_from<T, E, RG, SIZE, STRIDE / 2>(x, lane);
        }
    }
}

// Sorts rows r0, r0 + step, ... (RG of them; those at or past nR are padding)
// together: their networks are independent, so each stage's lane exchanges
// for the RG rows are in flight at once.
template <typename T, int E, int RG>
__device__ __forceinline__ void sort_rows(const T* S, int nR, int nC, int r0, int step, uint16_t* ord) {
    const int lane = (int)(threadIdx.x & (kWave - 1));
    Rank<T> x[RG][E];
#pragma unroll
    for (int g = 0; g < RG; ++g) {
        const int r = r0 + g * step;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int c = m * kWave + lane;
            x[g][m] = (r < nR && c < nC) ? Rank<T>::make(S[r * nC + c], (uint32_t)c) : Rank<T>::none();
        }
    }
    bitonic_from<T, E, RG, 2, 1>(x, lane);
#pragma unroll
    for (int g = 0; g < RG; ++g) {
        const int r = r0 + g * step;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int p = m * kWave + lane;
            if (r < nR && p < nC) ord[r * nC + p] = (uint16_t)x[g][m].lo();
        }
    }
}

// Greedy walk over the sorted rows by one wave, rows r = lane + 64 m held in
// registers (m < RM, instantiated for the row count): each lane keeps its
// rows' current candidates, so a step is a register minimum, one wave
// reduction and the pointer moves of the rows that wanted the column just
// taken.
constexpr int kWalkRows = 4;  // the most rows per lane held in registers

template <typename T, int RM>
__device__ __forceinline__ void greedy_walk(const PairShape& sh, const T* S, const uint16_t* ord, const Lists<T>& G) {
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int nR = sh.nR, nC = sh.nC;
    const bool swp = sh.swap != 0;
    int* rstate = G.rstate;
    int* cstate = G.cstate;
    auto key_of = [&](int r, int c) { return (uint32_t)(swp ? c * nR + r : r * nC + c); };
    Rank<T> cr[RM];
    int cc[RM], cp[RM];
#pragma unroll
    for (int m = 0; m < RM; ++m) {
        const int r = m * kWave + lane;
        cp[m] = 0;
        cc[m] = -1;
        cr[m] = Rank<T>::none();
        if (r < nR) {
            rstate[r] = -1;
            cc[m] = ord[r * nC];
            cr[m] = Rank<T>::make(S[r * nC + cc[m]], key_of(r, cc[m]));
        }
    }
    for (int c = lane; c < nC; c += kWave) cstate[c] = -1;
    const int need = min(nR, nC);
    for (int done = 0; done < need; ++done) {
        Rank<T> lb = cr[0];
        int lm = 0;
#pragma unroll
        for (int m = 1; m < RM; ++m)
            if (cr[m] < lb) {
                lb = cr[m];
                lm = m;
            }
        const Rank<T> gb = wave_min(lb);
        if (gb.is_none()) break;
        // ranks of real entries are distinct: exactly one lane holds the winner
        const int wl = (int)__builtin_ctzll(__ballot(lb == gb));
        int my_c = cc[0];
#pragma unroll
        for (int m = 1; m < RM; ++m)
            if (lm == m) my_c = cc[m];
        const int r0 = __builtin_amdgcn_readlane(lm * kWave + lane, wl);
        const int c0 = __builtin_amdgcn_readlane(my_c, wl);
        if (lane == wl) {
#pragma unroll
            for (int m = 0; m < RM; ++m)
                if (lm == m) cr[m] = Rank<T>::none();
        }
        if (lane == 0) {
            rstate[r0] = c0;
            cstate[c0] = r0;
        }
        // Rows whose column was just taken move on to their next free column.
        // The wave's LDS accesses complete in order: the marks above are seen
        // by the reads below.
#pragma unroll
        for (int m = 0; m < RM; ++m) {
            if (!cr[m].is_none() && cc[m] == c0) {
                const int r = m * kWave + lane;
                const uint16_t* o = ord + r * nC;
                int q = cp[m] + 1;
                while (q < nC && cstate[o[q]] != -1) ++q;
                cp[m] = q;
                if (q < nC) {
                    cc[m] = o[q];
                    cr[m] = Rank<T>::make(S[r * nC + cc[m]], key_of(r, cc[m]));
                } else {
                    cc[m] = -1;
                    cr[m] = Rank<T>::none();
                }
            }
        }
    }
}

// The same walk with the rows' state in LDS (more than 64 * kWalkRows rows).
template <typename T>
__device__ __forceinline__ void greedy_walk_lds(const PairShape& sh, const T* S, const uint16_t* ord, const Lists<T>& G) {
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int nR = sh.nR, nC = sh.nC;
    const bool swp = sh.swap != 0;
    int* rstate = G.rstate;
    int* rbest = G.rbest;
    int* cstate = G.cstate;
    int* rptr = reinterpret_cast<int*>(G.rec);
    for (int r = lane; r < nR; r += kWave) {
        rstate[r] = -1;
        rptr[r] = 0;
        rbest[r] = ord[r * nC];
    }
    for (int c = lane; c < nC; c += kWave) cstate[c] = -1;
    const int need = min(nR, nC);
    for (int done = 0; done < need; ++done) {
        Rank<T> best = Rank<T>::none();
        for (int r = lane; r < nR; r += kWave) {
            const int c = rbest[r];
            if (rstate[r] == -1 && c >= 0) {
                const Rank<T> q = Rank<T>::make(S[r * nC + c], (uint32_t)(swp ? c * nR + r : r * nC + c));
                if (q < best) best = q;
            }
        }
        best = wave_min(best);
        if (best.is_none()) break;
        const int key = (int)best.lo();
        const int r0 = swp ? key % nR : key / nC;
        const int c0 = swp ? key / nR : key % nC;
        if (lane == 0) {
            rstate[r0] = c0;
            cstate[c0] = r0;
        }
        for (int r = lane; r < nR; r += kWave) {
            if (rstate[r] == -1 && rbest[r] == c0) {
                const uint16_t* o = ord + r * nC;
                int q = rptr[r] + 1;
                while (q < nC && cstate[o[q]] != -1) ++q;
                rptr[r] = q;
                rbest[r] = q < nC ? (int)o[q] : -1;
            }
        }
    }
}

// Kept out of line: runs once per pair, and inlined it constrains the
// register allocation of the update loop in the same kernel.  Its arguments
// are scalars: a shape or list record passed by reference would have to live
// in the caller's stack, written once per pair by every thread.
template <typename T, int NT>
__device__ __noinline__ void greedy_sorted(int nR, int nC, int swp, const T* S, T* St, int* rstate, int* rbest,
                                           int* cstate, void* rec) {
    constexpr int NW = NT / kWave;
    const int wave = uni((int)threadIdx.x / kWave);
    PairShape sh{};
    sh.swap = swp;
    sh.nR = nR;
    sh.nC = nC;
    Lists<T> G{};
    G.rstate = rstate;
    G.rbest = rbest;
    G.cstate = cstate;
    G.rec = reinterpret_cast<RowRec<T>*>(rec);
    uint16_t* ord = reinterpret_cast<uint16_t*>(St);
    // rows sorted together by a wave: 4 short ones, 2 of 65-128 entries, 1 longer
    if (nC <= kWave) {
        for (int r = wave; r < nR; r += 4 * NW) sort_rows<T, 1, 4>(S, nR, nC, r, NW, ord);
    } else if (nC <= 2 * kWave) {
        for (int r = wave; r < nR; r += 2 * NW) sort_rows<T, 2, 2>(S, nR, nC, r, NW, ord);
    } else {
        for (int r = wave; r < nR; r += NW) sort_rows<T, 4, 1>(S, nR, nC, r, NW, ord);
    }
    __syncthreads();
    if (wave == 0) {
        if (nR <= kWave)
            greedy_walk<T, 1>(sh, S, ord, G);
        else if (nR <= 2 * kWave)
            greedy_walk<T, 2>(sh, S, ord, G);
        else if (nR <= kWalkRows * kWave)
            greedy_walk<T, kWalkRows>(sh, S, ord, G);
        else
            greedy_walk_lds<T>(sh, S, ord, G);
    }
    __syncthreads();
}

// Step a7, longer rows: locally-dominant rounds, which for a strict total
// order reach the same matching as the greedy order.
template <typename T, int NT>
__device__ __forceinline__ void greedy_rounds(const PairShape& sh, const T* S, T* St, const Lists<T>& G, int* s_count) {
    constexpr int NW = NT / kWave;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = uni(tid / kWave);
    const int nR = sh.nR, nC = sh.nC;
    const bool swp = sh.swap != 0;
    int* rstate = G.rstate;
    int* rbest = G.rbest;
    int* cstate = G.cstate;
    int* cbest = G.cbest;
    // Incremental rounds: a free row's best free column (and a free column's
    // best free row) only changes when that partner gets matched, so each round
    // recomputes just the stale rows/columns, listed in `todo` (items < nR are
    // rows, the rest columns); mutual bests are matched.  Columns are scanned
    // on S^T (St, the buffer the iteration no longer needs) so that every scan
    // reads consecutive words.  The lists' LDS space (row records onwards) is
    // free by now and holds `todo`.
    int* todo = reinterpret_cast<int*>(G.rec);
    for (long long o = tid; o < (long long)nR * nC; o += NT) {
        const int r = (int)(o / nC), c = (int)(o - (long long)r * nC);
        St[(long long)c * nR + r] = S[o];
    }
    for (int r = tid; r < nR; r += NT) {
        rstate[r] = -1;
        rbest[r] = -2;
    }
    for (int c = tid; c < nC; c += NT) {
        cstate[c] = -1;
        cbest[c] = -2;
    }
    for (int x = tid; x < nR + nC; x += NT) todo[x] = x;
    if (tid == 0) {
        s_count[0] = 0;
        s_count[1] = nR + nC;
    }
    __syncthreads();
    const int need = min(nR, nC);
    int done = 0;
    while (done < need) {
        const int ntodo = s_count[1];
        for (int k = wave; k < ntodo; k += NW) {
            const int x = uni(todo[k]);
            const bool is_row = x < nR;
            const int y0 = is_row ? x : x - nR;
            const T* line = is_row ? S + (long long)y0 * nC : St + (long long)y0 * nR;
            const int n = is_row ? nC : nR;
            const int* other = is_row ? cstate : rstate;
            T bv = T(-__builtin_inf());  // numbers first: NaN entries only if no number is left
            bool nan_seen = false;
            int bk = INT_MAX, bi = -1;
            for (int z0 = lane; z0 < n; z0 += 4 * kWave) {
                T v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int z = z0 + u * kWave;
                    v[u] = z < n ? line[z] : T(-1);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int z = z0 + u * kWave;
                    if (z < n && other[z] == -1) {
                        const int r = is_row ? y0 : z, c = is_row ? z : y0;
                        const int key = swp ? c * nR + r : r * nC + c;
                        if (v[u] != v[u]) {
                            nan_seen = true;
                        } else if (v[u] > bv || (v[u] == bv && key < bk)) {
                            bv = v[u];
                            bk = key;
                            bi = z;
                        }
                    }
                }
            }
            wave_argmax(bv, bk, bi);
            if (bi < 0 && __ballot(nan_seen) != 0) {
                // no number left on the line: its free NaN entry with the smallest key
                T z0v = T(-__builtin_inf());
                int nk = INT_MAX, ni = -1;
                for (int z = lane; z < n; z += kWave) {
                    const int r = is_row ? y0 : z, c = is_row ? z : y0;
                    const int key = swp ? c * nR + r : r * nC + c;
                    if (other[z] == -1 && line[z] != line[z] && key < nk) {
                        nk = key;
                        ni = z;
                    }
                }
                if (ni >= 0) z0v = T(0);
                wave_argmax(z0v, nk, ni);
                bi = ni;
            }
            if (lane == 0) {
                if (is_row)
                    rbest[y0] = bi;
                else
                    cbest[y0] = bi;
            }
        }
        __syncthreads();
        if (tid == 0) s_count[1] = 0;
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
        // stale: free rows/columns whose best was just taken by someone else
        for (int r = tid; r < nR; r += NT)
            if (rstate[r] == -1 && rbest[r] >= 0 && cstate[rbest[r]] != -1) {
                rbest[r] = -2;
                todo[atomicAdd(s_count + 1, 1)] = r;
            }
        for (int c = tid; c < nC; c += NT)
            if (cstate[c] == -1 && cbest[c] >= 0 && rstate[cbest[c]] != -1) {
                cbest[c] = -2;
                todo[atomicAdd(s_count + 1, 1)] = nR + c;
            }
        const int now = s_count[0];
        __syncthreads();
        if (now == done) break;  // guard: the earliest free entry is always a mutual best
        done = now;
    }

}

// S (compute orientation, maybe transposed) to the n_B x n_A output.
template <typename T, typename O, int NT>
__device__ __forceinline__ void write_S(O* So, const T* S, long long total, int nA, int nC, bool swp) {
    for (long long o = threadIdx.x; o < total; o += NT) {
        if (!swp) {
            So[o] = O(S[o]);
        } else {
            const long long i = o / nA, jj = o - i * nA;
            So[o] = O(S[jj * nC + i]);
        }
    }
}

// Step a7 and the outputs: greedy matching on the stored S (compute
// orientation), its relative margin, score in original row order, S_out,
// result.
template <typename T, int NT>
__device__ __forceinline__ void match_and_write(const PairJob& J, int p, const GraphRef& A, const GraphRef& B, const PairShape& sh,
                                 const T* S, T* St, const Lists<T>& G, const IterOut& it, cfsim_pair_result* res,
                                 double* red, int* s_count) {
    constexpr int NW = NT / kWave;
    const int tid = threadIdx.x;
    const int nC = sh.nC;
    const bool swp = sh.swap != 0;
    int* rstate = G.rstate;
    int* cstate = G.cstate;
    if (nC <= kSortCols)
        greedy_sorted<T, NT>(sh.nR, nC, sh.swap, S, St, G.rstate, G.rbest, G.cstate, G.rec);
    else
        greedy_rounds<T, NT>(sh, S, St, G, s_count);
    // the row records and column infos are free now: they hold the picks
    const double margin = greedy_margin<T, NT>(S, sh.nR, nC, swp, rstate, cstate, reinterpret_cast<T*>(G.rec),
                                               reinterpret_cast<T*>(G.cinfo), red);

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
        const long long total = (long long)nA * nB;
        // the FP64 pass of an FP32 call writes FP32
        if (sizeof(T) == 8 && J.refine)
            write_S<T, float, NT>(reinterpret_cast<float*>(J.S_out) + so, S, total, nA, nC, swp);
        else
            write_S<T, T, NT>(reinterpret_cast<T*>(J.S_out) + so, S, total, nA, nC, swp);
    }
    const double score = block_sum<NW>(sc, red + 3 * NW);
    if (tid == 0) {
        res->score = score;
        res->nu = it.nu;
        res->delta = it.delta;
        res->margin = margin;
        res->iters = it.iters;
        res->status = it.status | (margin <= J.tie_tol ? CFSIM_NEAR_TIE : 0u) | (J.refine ? CFSIM_FP64_FINAL : 0u);
    }
    __syncthreads();
}

// FP64 pass of an FP32 call: pairs whose FP32 result is not a near tie keep
// it (the same global word in every thread, so the exit is uniform).
__device__ inline bool refine_skips(const PairJob& J, int p) {
    if (!J.refine) return false;
    const unsigned st = J.res[J.single ? 0 : p].status;
    return !(st & CFSIM_NEAR_TIE) || (st & CFSIM_INVALID_INPUT);
}

// A pair of unequal sizes in the resized mode: the larger graph takes the
// rows (stored S^T when that is A); iteration at M x m, expansion to M x M,
// matching and outputs at M x M (S_out and match as for the tiled path).
template <typename T, int NT, int NCHMAX, bool GLOBAL>
__device__ __forceinline__ void resized_pair(const PairJob& J, int p, const GraphRef& A, const GraphRef& B,
                                             cfsim_pair_result* res, unsigned char* smem, double* red,
                                             int* s_count) {
    constexpr int NW = NT / kWave;
    const bool swp = B.n < A.n;  // rows = A's nodes: S is stored transposed
    const GraphRef Lg = pick_graph(swp, A, B);
    const GraphRef Xg = pick_graph(swp, B, A);
    const int M = Lg.n, m = Xg.n;
    const int esz = (int)sizeof(T);
    const bool fits = GLOBAL ? resized_global_fits(M, m, Lg.nnz, Xg.nnz, esz, J.slot_elems)
                             : resized_fits(M, m, Lg.nnz, Xg.nnz, J.variant, esz);
    if ((m + 63) / 64 > NCHMAX || !fits) {
        if (threadIdx.x == 0) write_invalid(res);
        return;
    }
    // the iterates and then S, S^T: LDS, or this workgroup's global slot
    unsigned char* buf =
        GLOBAL ? reinterpret_cast<unsigned char*>(J.gws) + (size_t)blockIdx.x * resized_slot_bytes(J.slot_elems, esz)
               : smem;
    PairShape sh{};
    sh.swap = swp ? 1 : 0;
    sh.nR = M;
    sh.nC = m;
    sh.nchunk = (m + 63) / 64;
    sh.rows = (M + NW - 1) / NW;
    const size_t B1 = align16((size_t)M * m * esz);
    IterOut it;
    {
        const Lists<T> G = carve_lists<T>(GLOBAL ? smem : smem + 3 * B1, M, m, Lg.nnz, Xg.nnz);
        const bool degenerate = stage_pair<T, NT>(Lg, Xg, M, m, G, reinterpret_cast<T*>(buf), T(0));
        if (NCHMAX == 1 || sh.nchunk == 1)
            it = iterate_resized<T, NT, 1>(J, buf, B1, sh, G, degenerate, red);
        else if (NCHMAX == 2 || sh.nchunk == 2)
            it = iterate_resized<T, NT, (NCHMAX >= 2 ? 2 : 1)>(J, buf, B1, sh, G, degenerate, red);
        else
            it = iterate_resized<T, NT, NCHMAX>(J, buf, B1, sh, G, degenerate, red);
    }
    const T inv = it.status == CFSIM_DEGENERATE && it.iters == 0 ? T(1) : T(1.0 / it.nu);
    expand_resized<T, NT>(buf, M, m, inv);
    const size_t SB = align16((size_t)M * M * esz);
    PairShape shm = sh;
    shm.nC = M;
    shm.nchunk = (M + 63) / 64;
    const Lists<T> Gm = carve_lists<T>(GLOBAL ? smem : smem + 2 * SB, M, M, 0, 0);
    GraphRef Am = A, Bm = B;  // outputs are n_M x n_M
    Am.n = M;
    Bm.n = M;
    match_and_write<T, NT>(J, p, Am, Bm, shm, reinterpret_cast<const T*>(buf), reinterpret_cast<T*>(buf + SB), Gm,
                           it, res, red, s_count);
}

template <typename T, int NT, int NCHMAX, int MODE>
__device__ __forceinline__ void lds_pair(const PairJob& J, int p, unsigned char* smem, double* red, int* s_count,
                                         int* s_seg) {
    if (refine_skips(J, p)) return;
    if constexpr (MODE == kModeResized) {
        GraphRef A{}, B{};
        cfsim_pair_result* res;
        if (resolve_graphs(J, p, A, B, res) && A.n != B.n) {
            resized_pair<T, NT, NCHMAX, false>(J, p, A, B, res, smem, red, s_count);
            return;
        }
    }
    constexpr bool DAMPED = MODE == kModeDamped;
    IterOut it;
    {
        GraphRef A{}, B{};
        cfsim_pair_result* res;
        PairShape sh{};
        const bool ok = resolve_graphs(J, p, A, B, res) &&
                        choose_shape(A.n, B.n, A.nnz, B.nnz, J.variant, (int)sizeof(T), &sh) && sh.nchunk <= NCHMAX;
        if (!ok) {
            if (threadIdx.x == 0) write_invalid(res);
            return;
        }
        const GraphRef R = pick_graph(sh.swap != 0, A, B);
        const GraphRef C = pick_graph(sh.swap != 0, B, A);
        const int nR = sh.nR, nC = sh.nC;
        const size_t sbytes = align16((size_t)nR * nC * sizeof(T));
        const Lists<T> G = carve_lists<T>(smem + 2 * sbytes, nR, nC, R.nnz, C.nnz);
        const T s0 = T(1.0 / sqrt((double)nR * (double)nC));
        const bool degenerate = stage_pair<T, NT>(R, C, nR, nC, G, reinterpret_cast<T*>(smem), s0);
        if constexpr (DAMPED) {
            DampedPrior P;
            if (!damped_prior<T, NT>(J, p, A.n, B.n, sh, P, red)) {
                if (threadIdx.x == 0) write_invalid(res);
                return;
            }
            unsigned char* B1 = smem + sbytes;
            if (NCHMAX == 1 || sh.nchunk == 1)
                it = iterate_damped<T, NT, 1, false>(J, sh, G, smem, B1, P, red);
            else if (NCHMAX == 2 || sh.nchunk == 2)
                it = iterate_damped<T, NT, (NCHMAX >= 2 ? 2 : 1), false>(J, sh, G, smem, B1, P, red);
            else
                it = iterate_damped<T, NT, NCHMAX, false>(J, sh, G, smem, B1, P, red);
        } else {
        if constexpr (NT == kWave) order_rows<T, NT>(G, nR, G.rstate, s_seg);  // one wave: no barrier needed
        if (NCHMAX == 1 || sh.nchunk == 1)
            it = iterate_lds<T, NT, 1>(J, smem, sh, sbytes, G, degenerate, red, s_seg, checkpoint_base<T>(J, p));
        else if (NCHMAX == 2 || sh.nchunk == 2)
            it = iterate_lds<T, NT, (NCHMAX >= 2 ? 2 : 1)>(J, smem, sh, sbytes, G, degenerate, red, s_seg,
                                                           checkpoint_base<T>(J, p));
        else
            it = iterate_lds<T, NT, NCHMAX>(J, smem, sh, sbytes, G, degenerate, red, s_seg, checkpoint_base<T>(J, p));
        }
    }
    // The pair's graphs, shape and lists again, from fresh reads of the
    // arguments (the same values: the iteration does not change them).
    const PairJob& Jr = job_args();
    GraphRef A{}, B{};
    cfsim_pair_result* res;
    PairShape sh{};
    resolve_graphs(Jr, p, A, B, res);
    choose_shape(A.n, B.n, A.nnz, B.nnz, Jr.variant, (int)sizeof(T), &sh);
    const int nnzR = sh.swap ? A.nnz : B.nnz, nnzC = sh.swap ? B.nnz : A.nnz;
    const size_t sbytes = align16((size_t)sh.nR * sh.nC * sizeof(T));
    const Lists<T> G = carve_lists<T>(smem + 2 * sbytes, sh.nR, sh.nC, nnzR, nnzC);
    const T* S = reinterpret_cast<const T*>(smem + (it.final_buf ? sbytes : 0));
    T* St = reinterpret_cast<T*>(smem + (it.final_buf ? 0 : sbytes));
    match_and_write<T, NT>(Jr, p, A, B, sh, S, St, G, it, res, red, s_count);
}

template <typename T, int NT, int NCH, int MODE>
__device__ __forceinline__ void global_pair(const PairJob& J, int p, unsigned char* smem, double* red, int* s_count) {
    constexpr bool DAMPED = MODE == kModeDamped;
    if constexpr (MODE == kModeResized) {
        GraphRef A{}, B{};
        cfsim_pair_result* res;
        if (refine_skips(J, p)) return;
        if (resolve_graphs(J, p, A, B, res) && A.n != B.n) {
            resized_pair<T, NT, NCH, true>(J, p, A, B, res, smem, red, s_count);
            return;
        }
    }
    if (refine_skips(J, p)) return;
    GraphRef A{}, B{};
    cfsim_pair_result* res;
    PairShape sh{};
    const bool ok = resolve_graphs(J, p, A, B, res) &&
                    global_fits(A.n, B.n, A.nnz, B.nnz, (int)sizeof(T), J.slot_elems, &sh);
    if (!ok) {
        if (threadIdx.x == 0) write_invalid(res);
        return;
    }
    const GraphRef R = pick_graph(sh.swap != 0, A, B);
    const GraphRef C = pick_graph(sh.swap != 0, B, A);
    const int nR = sh.nR, nC = sh.nC;
    const Lists<T> G = carve_lists<T>(smem, nR, nC, R.nnz, C.nnz);
    T* slot = reinterpret_cast<T*>(J.gws) + (size_t)blockIdx.x * 2 * (size_t)J.slot_elems;
    T* S0 = slot;
    T* S1 = slot + J.slot_elems;
    const T s0 = T(1.0 / sqrt((double)nR * (double)nC));
    const bool degenerate = stage_pair<T, NT>(R, C, nR, nC, G, S0, s0);
    IterOut it;
    if constexpr (DAMPED) {
        DampedPrior P;
        if (!damped_prior<T, NT>(J, p, A.n, B.n, sh, P, red)) {
            if (threadIdx.x == 0) write_invalid(res);
            return;
        }
        it = iterate_damped<T, NT, 1, true>(J, sh, G, reinterpret_cast<unsigned char*>(S0),
                                            reinterpret_cast<unsigned char*>(S1), P, red);
    } else {
        it = iterate_global<T, NT>(J, sh, G, S0, S1, degenerate, red, checkpoint_base<T>(J, p));
    }
    match_and_write<T, NT>(J, p, A, B, sh, it.final_buf ? S1 : S0, it.final_buf ? S0 : S1, G, it, res, red, s_count);
}

// Persistent driver: one pair at a time per workgroup, pulled from the
// bucket's queue (or the single pair of the plain path).
template <bool GLOBAL, typename T, int NT, int NCH, int MODE>
__device__ __forceinline__ void drive(const PairJob& J, unsigned char* smem, double* red, int* s_item, int* s_count,
                                      int* s_seg) {
    if (J.single) {
        if (blockIdx.x == 0) {
            if constexpr (GLOBAL)
                global_pair<T, NT, NCH, MODE>(J, 0, smem, red, s_count);
            else
                lds_pair<T, NT, NCH, MODE>(J, 0, smem, red, s_count, s_seg);
        }
        return;
    }
    for (;;) {
        const PairJob& Jl = job_args();
        if (threadIdx.x == 0) *s_item = Jl.bounds[0] + atomicAdd(Jl.queue, 1);
        __syncthreads();
        const int item = *s_item;
        __syncthreads();
        if (item >= Jl.bounds[1]) break;
        if constexpr (GLOBAL)
            global_pair<T, NT, NCH, MODE>(Jl, Jl.order[item], smem, red, s_count);
        else
            lds_pair<T, NT, NCH, MODE>(Jl, Jl.order[item], smem, red, s_count, s_seg);
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
    __shared__ int s_item, s_count[2], s_seg[kRowClasses + 1];
    drive<false, T, NT, NCH, kModePlain>(J, smem, red, &s_item, s_count, s_seg);
}

// The damped measure on the same variants and schedule.
template <typename T, int NT, int NCH>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(waves_per_simd<NT>())))
void damped_lds_kernel(PairJob J) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[4 * (NT / kWave)];
    __shared__ int s_item, s_count[2], s_seg[kRowClasses + 1];
    drive<false, T, NT, NCH, kModeDamped>(J, smem, red, &s_item, s_count, s_seg);
}

// The scale-to-common-size mode on the same variants and schedule.
template <typename T, int NT, int NCH>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(waves_per_simd<NT>())))
void resized_lds_kernel(PairJob J) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[4 * (NT / kWave)];
    __shared__ int s_item, s_count[2], s_seg[kRowClasses + 1];
    drive<false, T, NT, NCH, kModeResized>(J, smem, red, &s_item, s_count, s_seg);
}

template <typename T>
__global__ __launch_bounds__(kGlobalThreads) __attribute__((amdgpu_waves_per_eu(4)))
void pair_global_kernel(PairJob J) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[4 * (kGlobalThreads / kWave)];
    __shared__ int s_item, s_count[2];
    drive<true, T, kGlobalThreads, 1, kModePlain>(J, smem, red, &s_item, s_count, nullptr);
}

template <typename T>
__global__ __launch_bounds__(kGlobalThreads) __attribute__((amdgpu_waves_per_eu(4)))
void resized_global_kernel(PairJob J) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[4 * (kGlobalThreads / kWave)];
    __shared__ int s_item, s_count[2];
    drive<true, T, kGlobalThreads, 2, kModeResized>(J, smem, red, &s_item, s_count, nullptr);
}

template <typename T>
__global__ __launch_bounds__(kGlobalThreads) __attribute__((amdgpu_waves_per_eu(4)))
void damped_global_kernel(PairJob J) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[4 * (kGlobalThreads / kWave)];
    __shared__ int s_item, s_count[2];
    drive<true, T, kGlobalThreads, 1, kModeDamped>(J, smem, red, &s_item, s_count, nullptr);
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
    if (P.filter) {  // FP64 pass of an FP32 call: near-tie pairs only
        const unsigned st = P.filter[p].status;
        if (!(st & CFSIM_NEAR_TIE) || (st & CFSIM_INVALID_INPUT)) {
            *bucket = -1;
            return;
        }
    }
    if (ga < 0 || ga >= P.set.n_graphs || gb < 0 || gb >= P.set.n_graphs) return;
    const int nA = (int)(P.set.node_off[ga + 1] - P.set.node_off[ga]);
    const int nB = (int)(P.set.node_off[gb + 1] - P.set.node_off[gb]);
    const int mA = (int)(P.set.edge_off[ga + 1] - P.set.edge_off[ga]);
    const int mB = (int)(P.set.edge_off[gb + 1] - P.set.edge_off[gb]);
    if (nA < 1 || nB < 1) return;
    PairShape sh;
    int b = kBucketInvalid;
    if (P.resize && nA != nB) {
        // resized mode: the first LDS variant that holds the resized pair, else
        // the global-memory kernel; the rest stay in the invalid bucket and
        // take the tiled path
        const int M = nA > nB ? nA : nB, m = nA > nB ? nB : nA;
        const int nnzL = nA > nB ? mA : mB, nnzX = nA > nB ? mB : mA;
        for (int v = 0; v < kNumVariants && b == kBucketInvalid; ++v)
            if (resized_fits(M, m, nnzL, nnzX, v, P.esize)) b = v;
        if (b == kBucketInvalid && resized_global_fits(M, m, nnzL, nnzX, P.esize, P.slot_elems)) b = kBucketGlobal;
    } else {
        for (int v = 0; v < kNumVariants && b == kBucketInvalid; ++v)
            if (choose_shape(nA, nB, mA, mB, v, P.esize, &sh)) b = v;
        if (b < kNumVariants) {  // a tuned larger variant for the pair's class, if it holds the pair
            const int t = P.tune[tune_class(nA, nB)];
            if (t > b && t < kNumVariants && choose_shape(nA, nB, mA, mB, t, P.esize, &sh)) b = t;
        }
        if (b == kBucketInvalid && !P.resize && global_fits(nA, nB, mA, mB, P.esize, P.slot_elems, &sh))
            b = kBucketGlobal;
    }
    if (P.filter && b == kBucketInvalid) {  // no FP64 kernel holds it: the FP32 result stays
        *bucket = -1;
        return;
    }
    // longest first: cost class from log2 of the work estimate (the resized
    // state is M x m, the iteration's shape either way)
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
        if (b >= 0) atomicAdd(&hist[b * kClasses + c], 1);
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
        if (b < 0) continue;
        const int slot = atomicAdd(&hist[b * kClasses + c], 1);
        P.order[slot] = (int32_t)p;
    }
}

__global__ __launch_bounds__(256) void buckets_kernel(PlanJob P, int32_t* bucket) {
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < P.n_pairs; p += (int64_t)gridDim.x * 256) {
        int b, c;
        classify(P, p, &b, &c);
        bucket[p] = b;
    }
}

template <typename T, int NT, int NCH>
const void* kernel_ptr(int mode) {
    return mode == kModeDamped    ? reinterpret_cast<const void*>(&damped_lds_kernel<T, NT, NCH>)
           : mode == kModeResized ? reinterpret_cast<const void*>(&resized_lds_kernel<T, NT, NCH>)
                                  : reinterpret_cast<const void*>(&pair_lds_kernel<T, NT, NCH>);
}

template <typename T>
const void* global_kernel_ptr(int mode) {
    return mode == kModeDamped    ? reinterpret_cast<const void*>(&damped_global_kernel<T>)
           : mode == kModeResized ? reinterpret_cast<const void*>(&resized_global_kernel<T>)
                                  : reinterpret_cast<const void*>(&pair_global_kernel<T>);
}

// Instantiations must match variant_info().
const void* variant_kernel(int v, int dtype, int mode = kModePlain) {
    if (v == kBucketGlobal)
        return dtype == CFSIM_F64 ? global_kernel_ptr<double>(mode) : global_kernel_ptr<float>(mode);
    if (dtype == CFSIM_F64) {
        switch (v) {
            case 0: return kernel_ptr<double, 64, 1>(mode);
            case 1: return kernel_ptr<double, 256, 2>(mode);
            case 2: return kernel_ptr<double, 512, 2>(mode);
            case 3: return kernel_ptr<double, 1024, 2>(mode);
            default: return kernel_ptr<double, 1024, 4>(mode);
        }
    }
    switch (v) {
        case 0: return kernel_ptr<float, 64, 2>(mode);
        case 1: return kernel_ptr<float, 256, 4>(mode);
        case 2: return kernel_ptr<float, 512, 2>(mode);
        case 3: return kernel_ptr<float, 1024, 2>(mode);
        default: return kernel_ptr<float, 1024, 4>(mode);
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
    const int mode = job.damped ? kModeDamped : (job.resize ? kModeResized : kModePlain);
    return (int)hipLaunchKernel(variant_kernel(variant, dtype, mode), dim3(grid),
                                dim3(threads_of(variant, esize)), args,
                                (size_t)lds_of(variant, esize), stream);
}

int launch_plan(const PlanJob& job, hipStream_t stream) {
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(kPlanThreads), 0, stream, job);
    return (int)hipGetLastError();
}

int launch_buckets(const PlanJob& job, int32_t* bucket, hipStream_t stream) {
    const int64_t blocks = (job.n_pairs + 255) / 256;
    hipLaunchKernelGGL(buckets_kernel, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256), 0, stream, job,
                       bucket);
    return (int)hipGetLastError();
}

// Kernel names as profilers list them (template arguments as in variant_kernel).
const char* bucket_kernel_name(int bucket, int dtype) {
    static const char* const f64[kBucketGlobal + 1] = {
        "pair_lds_kernel<double, 64, 1>", "pair_lds_kernel<double, 256, 2>", "pair_lds_kernel<double, 512, 2>",
        "pair_lds_kernel<double, 1024, 2>", "pair_lds_kernel<double, 1024, 4>", "pair_global_kernel<double>"};
    static const char* const f32[kBucketGlobal + 1] = {
        "pair_lds_kernel<float, 64, 2>", "pair_lds_kernel<float, 256, 4>", "pair_lds_kernel<float, 512, 2>",
        "pair_lds_kernel<float, 1024, 2>", "pair_lds_kernel<float, 1024, 4>", "pair_global_kernel<float>"};
    if (bucket < 0 || bucket > kBucketGlobal || (dtype != CFSIM_F64 && dtype != CFSIM_F32)) return "";
    return dtype == CFSIM_F64 ? f64[bucket] : f32[bucket];
}

int set_kernel_attributes() {
    int e = 0;
    for (int v = 0; v <= kBucketGlobal; ++v)
        for (int mode = kModePlain; mode <= kModeResized; ++mode) {
            e |= (int)hipFuncSetAttribute(variant_kernel(v, CFSIM_F32, mode),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, lds_of(v, 4));
            e |= (int)hipFuncSetAttribute(variant_kernel(v, CFSIM_F64, mode),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, lds_of(v, 8));
        }
    return e;
}

int occupancy_of(int variant, int dtype, int* blocks) {
    const int esize = dtype == CFSIM_F64 ? 8 : 4;
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, variant_kernel(variant, dtype),
                                                            threads_of(variant, esize), (size_t)lds_of(variant, esize));
}

}  // namespace cfsim
