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
// zero weights: the first kDS successors and kDP predecessors as LDS byte
// offsets into a row of S, plus where the full lists start in the staged C
// lists (entries past the padding go through the overflow pass).
template <typename T>
struct LanePad {
    int sv[kDS];
    T sw[kDS];
    int pv[kDP];
    T pw[kDP];
    int sbeg, sdeg, pbeg, pdeg;
};

template <typename T>
__device__ inline T lds_at(const unsigned char* base, int byte_off) {
    return *reinterpret_cast<const T*>(base + byte_off);
}

template <typename T>
__device__ inline void load_lane(const int4* cinfo, const Edge<T>* cse, const Edge<T>* cpe, int c, bool valid,
                                 LanePad<T>& L) {
    const int esz = (int)sizeof(T);
    const int4 ci = cinfo[valid ? c : 0];
    L.sbeg = ci.x;
    L.sdeg = valid ? ci.y - ci.x : 0;
    L.pbeg = ci.z;
    L.pdeg = valid ? ci.w - ci.z : 0;
#pragma unroll
    for (int q = 0; q < kDS; ++q) {
        const bool has = q < L.sdeg;
        const Edge<T> e = cse[has ? ci.x + q : 0];
        L.sv[q] = has ? e.u * esz : 0;
        L.sw[q] = has ? e.w : T(0);
    }
#pragma unroll
    for (int q = 0; q < kDP; ++q) {
        const bool has = q < L.pdeg;
        const Edge<T> e = cpe[has ? ci.z + q : 0];
        L.pv[q] = has ? e.u * esz : 0;
        L.pw[q] = has ? e.w : T(0);
    }
}

// One R-side term: y += w * sum_q wl[q] S[u][v_q]  (row u at byte offset uo).
template <typename T, int D>
__device__ inline T lane_term(const unsigned char* Sb, int uo, T w, const int (&v)[D], const T (&wl)[D], T y) {
    T a = wl[0] * lds_at<T>(Sb, uo + v[0]);
#pragma unroll
    for (int q = 1; q < D; ++q) a = fma_t(wl[q], lds_at<T>(Sb, uo + v[q]), a);
    return fma_t(w, a, y);
}

// Row update specialised on the row's successor / predecessor counts.
template <typename T, int NS, int NP>
__device__ inline T row_fixed(const unsigned char* Sb, int rowb, const Edge<T>* se, const Edge<T>* pe,
                              const LanePad<T>& L) {
    int us[NS > 0 ? NS : 1], up[NP > 0 ? NP : 1];
    T ws[NS > 0 ? NS : 1], wp[NP > 0 ? NP : 1];
#pragma unroll
    for (int a = 0; a < NS; ++a) {
        const Edge<T> e = se[a];
        us[a] = uni(e.u) * rowb;
        ws[a] = uni(e.w);
    }
#pragma unroll
    for (int b = 0; b < NP; ++b) {
        const Edge<T> e = pe[b];
        up[b] = uni(e.u) * rowb;
        wp[b] = uni(e.w);
    }
    T y = T(0);
#pragma unroll
    for (int a = 0; a < NS; ++a) y = lane_term<T, kDS>(Sb, us[a], ws[a], L.sv, L.sw, y);
#pragma unroll
    for (int b = 0; b < NP; ++b) y = lane_term<T, kDP>(Sb, up[b], wp[b], L.pv, L.pw, y);
    return y;
}

// Any row: loops over the R edges (rows with long lists).
template <typename T>
__device__ inline T row_loop(const unsigned char* Sb, int rowb, const Edge<T>* se, int ns, const Edge<T>* pe,
                             int np, const LanePad<T>& L) {
    T y = T(0);
    for (int a = 0; a < ns; ++a) {
        const Edge<T> e = se[a];
        y = lane_term<T, kDS>(Sb, uni(e.u) * rowb, uni(e.w), L.sv, L.sw, y);
    }
    for (int b = 0; b < np; ++b) {
        const Edge<T> e = pe[b];
        y = lane_term<T, kDP>(Sb, uni(e.u) * rowb, uni(e.w), L.pv, L.pw, y);
    }
    return y;
}

// Lane-list entries past the padded kDS / kDP (long C lists).
template <typename T>
__device__ inline T row_overflow(const unsigned char* Sb, int rowb, const Edge<T>* se, int ns, const Edge<T>* pe,
                                 int np, const Edge<T>* cse, const Edge<T>* cpe, const LanePad<T>& L) {
    const int esz = (int)sizeof(T);
    T y = T(0);
    for (int a = 0; a < ns; ++a) {
        const Edge<T> e = se[a];
        const int uo = uni(e.u) * rowb;
        T acc = T(0);
        for (int q = kDS; q < L.sdeg; ++q) {
            const Edge<T> c = cse[L.sbeg + q];
            acc = fma_t(c.w, lds_at<T>(Sb, uo + c.u * esz), acc);
        }
        y = fma_t(uni(e.w), acc, y);
    }
    for (int b = 0; b < np; ++b) {
        const Edge<T> e = pe[b];
        const int uo = uni(e.u) * rowb;
        T acc = T(0);
        for (int q = kDP; q < L.pdeg; ++q) {
            const Edge<T> c = cpe[L.pbeg + q];
            acc = fma_t(c.w, lds_at<T>(Sb, uo + c.u * esz), acc);
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

// Steps a4-a6: NCH is the variant's maximum number of 64-column chunks.
template <typename T, int NT, int NCH, int MAXR>
__device__ IterOut iterate(const PairJob& J, unsigned char* smem, const PairShape& sh, size_t sbytes,
                           const int4* rinfo, const Edge<T>* sedge, const Edge<T>* pedge, const int4* cinfo,
                           const Edge<T>* csedge, const Edge<T>* cpedge, bool degenerate, T s0, double* red) {
    constexpr int NW = NT / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uni((int)threadIdx.x / kWave);
    const int nR = sh.nR, nC = sh.nC, nchunk = sh.nchunk;
    const int esz = (int)sizeof(T);
    const int rowb = nC * esz;

    // per chunk: does any lane of this wave have lists past the padding?
    bool ovf[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        const int c = ch * kWave + lane;
        const bool valid = ch < nchunk && c < nC;
        const int4 ci = cinfo[valid ? c : 0];
        const int extra = valid ? max(ci.y - ci.x - kDS, ci.w - ci.z - kDP) : 0;
        ovf[ch] = uni(wave_max(extra)) > 0;
    }

    T Sp[MAXR][NCH];
#pragma unroll
    for (int r = 0; r < MAXR; ++r)
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) Sp[r][ch] = s0;

    IterOut out{0.0, __builtin_inf(), 0, 0u, 0};
    if (degenerate) {
        out.status = CFSIM_DEGENERATE;
        return out;
    }
    const unsigned char* Sb = smem;     // S_{k-1} (times sigma)
    unsigned char* Nb = smem + sbytes;  // update target
    int cur = 0;
    T sigma = T(1);
    for (int k = 1; k <= J.max_iter; ++k) {
        double nu2 = 0.0;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            if (ch >= nchunk) break;
            const int c = ch * kWave + lane;
            const bool cv = c < nC;
            LanePad<T> L;
            load_lane(cinfo, csedge, cpedge, c, cv, L);
            for (int i = wave; i < nR; i += NW) {
                const int4 ri = rinfo[i];
                const int sb = uni(ri.x), ns = uni(ri.y) - sb, pb = uni(ri.z), np = uni(ri.w) - pb;
                const Edge<T>* se = sedge + sb;
                const Edge<T>* pe = pedge + pb;
                T y;
                switch (ns <= 2 && np <= 3 ? ns * 4 + np : -1) {
                    case 0: y = T(0); break;
                    case 1: y = row_fixed<T, 0, 1>(Sb, rowb, se, pe, L); break;
                    case 2: y = row_fixed<T, 0, 2>(Sb, rowb, se, pe, L); break;
                    case 3: y = row_fixed<T, 0, 3>(Sb, rowb, se, pe, L); break;
                    case 4: y = row_fixed<T, 1, 0>(Sb, rowb, se, pe, L); break;
                    case 5: y = row_fixed<T, 1, 1>(Sb, rowb, se, pe, L); break;
                    case 6: y = row_fixed<T, 1, 2>(Sb, rowb, se, pe, L); break;
                    case 7: y = row_fixed<T, 1, 3>(Sb, rowb, se, pe, L); break;
                    case 8: y = row_fixed<T, 2, 0>(Sb, rowb, se, pe, L); break;
                    case 9: y = row_fixed<T, 2, 1>(Sb, rowb, se, pe, L); break;
                    case 10: y = row_fixed<T, 2, 2>(Sb, rowb, se, pe, L); break;
                    case 11: y = row_fixed<T, 2, 3>(Sb, rowb, se, pe, L); break;
                    default: y = row_loop<T>(Sb, rowb, se, ns, pe, np, L); break;
                }
                if (ovf[ch]) y += row_overflow<T>(Sb, rowb, se, ns, pe, np, csedge, cpedge, L);
                y *= sigma;
                if (cv) {
                    *reinterpret_cast<T*>(Nb + i * rowb + c * esz) = y;
                    nu2 += (double)y * (double)y;
                }
            }
        }
        nu2 = wave_sum(nu2);
        double* rnu = red + (k & 1) * NW;
        if (lane == 0) rnu[wave] = nu2;
        __syncthreads();
        double tot = 0.0;
        for (int w = 0; w < NW; ++w) tot += rnu[w];
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
#pragma unroll
        for (int r = 0; r < MAXR; ++r) {
            const int i = wave + r * NW;
            if (i >= nR) break;
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                if (ch >= nchunk) break;
                const int c = ch * kWave + lane;
                if (c < nC) {
                    T* q = reinterpret_cast<T*>(Sw + i * rowb + c * esz);
                    const T sv = *q * inv;
                    *q = sv;
                    const double d = (double)sv - (double)Sp[r][ch];
                    d2 += d * d;
                    Sp[r][ch] = sv;
                }
            }
        }
        sigma = T(1);
        d2 = wave_sum(d2);
        if (lane == 0) red[2 * NW + wave] = d2;
        __syncthreads();
        double dt = 0.0;
        for (int w = 0; w < NW; ++w) dt += red[2 * NW + w];
        out.delta = sqrt(dt);
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

template <typename T, int NT, int NCHMAX, int MAXR>
__device__ void lds_pair(const PairJob& J, int p, unsigned char* smem, double* red, int* s_count) {
    constexpr int NW = NT / kWave;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = uni(tid / kWave);

    GraphRef A{}, B{};
    bool bad = false;
    if (J.single) {
        A = J.ga;
        B = J.gb;
    } else {
        const int ga = J.pair_a[p], gb = J.pair_b[p];
        if (ga < 0 || ga >= J.set.n_graphs || gb < 0 || gb >= J.set.n_graphs) {
            bad = true;
        } else {
            A = graph_of(J.set, ga);
            B = graph_of(J.set, gb);
        }
    }
    cfsim_pair_result* res = J.res + (J.single ? 0 : p);
    PairShape sh{};
    if (!bad) {
        bad = A.n < 1 || B.n < 1 || !choose_shape(A.n, B.n, A.nnz, B.nnz, J.variant, (int)sizeof(T), &sh);
        if (!bad && (sh.nchunk > NCHMAX || sh.rows > MAXR)) bad = true;
    }
    if (bad) {
        if (tid == 0) write_invalid(res);
        return;
    }
    const GraphRef R = sh.swap ? A : B;
    const GraphRef C = sh.swap ? B : A;
    const int nR = sh.nR, nC = sh.nC;

    // ---- carve LDS (layout of lds_pair_bytes)
    const size_t sbytes = align16((size_t)nR * nC * sizeof(T));
    size_t off = 2 * sbytes;
    int4* rinfo = reinterpret_cast<int4*>(smem + off);
    off += align16((size_t)nR * 16);
    Edge<T>* sedge = reinterpret_cast<Edge<T>*>(smem + off);
    off += align16((size_t)R.nnz * sizeof(Edge<T>));
    Edge<T>* pedge = reinterpret_cast<Edge<T>*>(smem + off);
    off += align16((size_t)R.nnz * sizeof(Edge<T>));
    int4* cinfo = reinterpret_cast<int4*>(smem + off);
    off += align16((size_t)nC * 16);
    Edge<T>* csedge = reinterpret_cast<Edge<T>*>(smem + off);
    off += align16((size_t)C.nnz * sizeof(Edge<T>));
    Edge<T>* cpedge = reinterpret_cast<Edge<T>*>(smem + off);
    off += align16((size_t)C.nnz * sizeof(Edge<T>));
    int* rstate = reinterpret_cast<int*>(smem + off);
    off += align16((size_t)nR * 4);
    int* rbest = reinterpret_cast<int*>(smem + off);
    off += align16((size_t)nR * 4);
    int* cstate = reinterpret_cast<int*>(smem + off);
    off += align16((size_t)nC * 4);
    int* cbest = reinterpret_cast<int*>(smem + off);

    // ---- stage both graphs and S_0; check both for a positive weight
    for (int r = tid; r < nR; r += NT) rinfo[r] = make_int4(R.rp[r], R.rp[r + 1], R.cp[r], R.cp[r + 1]);
    for (int c = tid; c < nC; c += NT) cinfo[c] = make_int4(C.rp[c], C.rp[c + 1], C.cp[c], C.cp[c + 1]);
    int posR = 0, posC = 0;
    for (int t = tid; t < R.nnz; t += NT) {
        const double w = R.w[t];
        sedge[t].u = R.ci[t];
        sedge[t].w = T(w);
        pedge[t].u = R.ri[t];
        pedge[t].w = T(R.w[R.eid[t]]);
        posR |= (w > 0.0);
    }
    for (int t = tid; t < C.nnz; t += NT) {
        const double w = C.w[t];
        csedge[t].u = C.ci[t];
        csedge[t].w = T(w);
        cpedge[t].u = C.ri[t];
        cpedge[t].w = T(C.w[C.eid[t]]);
        posC |= (w > 0.0);
    }
    const T s0 = T(1.0 / sqrt((double)nR * (double)nC));
    T* S0buf = reinterpret_cast<T*>(smem);
    for (int t = tid; t < nR * nC; t += NT) S0buf[t] = s0;
    const int anyR = __syncthreads_or(posR);
    const int anyC = __syncthreads_or(posC);
    const bool degenerate = !(anyR && anyC);

    const IterOut it = iterate<T, NT, NCHMAX, MAXR>(J, smem, sh, sbytes, rinfo, sedge, pedge, cinfo, csedge,
                                                    cpedge, degenerate, s0, red);
    const double nu = it.nu, delta = it.delta;
    const int iters = it.iters;
    const unsigned status = it.status;
    const T* S = reinterpret_cast<const T*>(smem + (it.final_buf ? sbytes : 0));

    // ---- greedy matching by locally-dominant rounds
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
                    const T v = S[r * nC + c];
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
                    const T v = S[r * nC + c];
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

    // ---- score (original rows i = nodes of B, ascending), outputs
    const int nA = A.n, nB = B.n;
    const int64_t mo = (J.single || !J.match_off) ? 0 : J.match_off[p];
    double sc = 0.0;
    for (int i = tid; i < nB; i += NT) {
        int jj;
        T v = T(0);
        if (!swp) {
            jj = rstate[i];
            if (jj >= 0) v = S[i * nC + jj];
        } else {
            jj = cstate[i];
            if (jj >= 0) v = S[jj * nC + i];
        }
        if (jj >= 0) sc += (double)v;
        if (J.match) J.match[mo + i] = jj;
    }
    sc = wave_sum(sc);
    if (lane == 0) red[3 * NW + wave] = sc;
    if (J.S_out) {
        const int64_t so = (J.single || !J.S_off) ? 0 : J.S_off[p];
        T* So = reinterpret_cast<T*>(J.S_out) + so;
        const int total = nA * nB;
        for (int o = tid; o < total; o += NT) {
            if (!swp) {
                So[o] = S[o];
            } else {
                const int i = o / nA, jj = o - i * nA;
                So[o] = S[jj * nC + i];
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        double score = 0.0;
        for (int w = 0; w < NW; ++w) score += red[3 * NW + w];
        res->score = score;
        res->nu = nu;
        res->delta = delta;
        res->iters = iters;
        res->status = status;
    }
    __syncthreads();
}

template <typename T, int NT, int NCH, int MAXR>
__global__ __launch_bounds__(NT) void pair_lds_kernel(PairJob J) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[4 * (NT / kWave)];
    __shared__ int s_item, s_count;
    if (J.single) {
        if (blockIdx.x == 0) lds_pair<T, NT, NCH, MAXR>(J, 0, smem, red, &s_count);
        return;
    }
    const int begin = J.bounds[0], end = J.bounds[1];
    for (;;) {
        if (threadIdx.x == 0) s_item = begin + atomicAdd(J.queue, 1);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= end) break;
        lds_pair<T, NT, NCH, MAXR>(J, J.order[item], smem, red, &s_count);
    }
}

// Pairs that no LDS variant can hold (and pairs with bad graph ids) get an
// INVALID_INPUT result until a larger path takes them.
__global__ void unfit_kernel(PairJob J) {
    const int begin = J.bounds[0], end = J.bounds[1];
    for (int it = begin + blockIdx.x * blockDim.x + threadIdx.x; it < end; it += gridDim.x * blockDim.x)
        write_invalid(J.res + J.order[it]);
}

// ---------------------------------------------------------------- plan (step a8)
constexpr int kPlanThreads = 1024;
constexpr int kClasses = 128;
constexpr int kBuckets = kNumVariants + 1;

__device__ void classify(const PlanJob& P, int64_t p, int* bucket, int* cls) {
    const int ga = P.pair_a[p], gb = P.pair_b[p];
    if (ga < 0 || ga >= P.set.n_graphs || gb < 0 || gb >= P.set.n_graphs) {
        *bucket = kNumVariants;
        *cls = 0;
        return;
    }
    const int nA = (int)(P.set.node_off[ga + 1] - P.set.node_off[ga]);
    const int nB = (int)(P.set.node_off[gb + 1] - P.set.node_off[gb]);
    const int mA = (int)(P.set.edge_off[ga + 1] - P.set.edge_off[ga]);
    const int mB = (int)(P.set.edge_off[gb + 1] - P.set.edge_off[gb]);
    int b = kNumVariants;
    if (nA >= 1 && nB >= 1) {
        for (int v = 0; v < kNumVariants; ++v) {
            PairShape sh;
            if (choose_shape(nA, nB, mA, mB, v, P.esize, &sh)) {
                b = v;
                break;
            }
        }
    }
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

template <typename T, int NT, int NCH, int MAXR>
const void* kernel_ptr() {
    return reinterpret_cast<const void*>(&pair_lds_kernel<T, NT, NCH, MAXR>);
}

// Instantiations must match variant_info().
const void* variant_kernel(int v, int dtype) {
    if (dtype == CFSIM_F64) {
        switch (v) {
            case 0: return kernel_ptr<double, 64, 1, 16>();
            case 1: return kernel_ptr<double, 256, 2, 8>();
            case 2: return kernel_ptr<double, 512, 2, 8>();
            default: return kernel_ptr<double, 1024, 2, 8>();
        }
    }
    switch (v) {
        case 0: return kernel_ptr<float, 64, 2, 16>();
        case 1: return kernel_ptr<float, 256, 4, 8>();
        case 2: return kernel_ptr<float, 512, 2, 16>();
        default: return kernel_ptr<float, 1024, 4, 8>();
    }
}

}  // namespace

int launch_pair_lds(int variant, int dtype, const PairJob& job, int grid, hipStream_t stream) {
    if (variant == kNumVariants) {
        hipLaunchKernelGGL(unfit_kernel, dim3(64), dim3(256), 0, stream, job);
        return (int)hipGetLastError();
    }
    const int esize = dtype == CFSIM_F64 ? 8 : 4;
    const Variant v = variant_info(variant, esize);
    void* args[] = {const_cast<PairJob*>(&job)};
    return (int)hipLaunchKernel(variant_kernel(variant, dtype), dim3(grid), dim3(v.nt), args,
                                (size_t)job.lds_bytes, stream);
}

int launch_plan(const PlanJob& job, hipStream_t stream) {
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(kPlanThreads), 0, stream, job);
    return (int)hipGetLastError();
}

int set_kernel_attributes() {
    int e = 0;
    for (int v = 0; v < kNumVariants; ++v) {
        e |= (int)hipFuncSetAttribute(variant_kernel(v, CFSIM_F32), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      variant_info(v, 4).lds_bytes);
        e |= (int)hipFuncSetAttribute(variant_kernel(v, CFSIM_F64), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      variant_info(v, 8).lds_bytes);
    }
    return e;
}

int occupancy_of(int variant, int dtype, int* blocks) {
    const Variant v = variant_info(variant, dtype == CFSIM_F64 ? 8 : 4);
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, variant_kernel(variant, dtype), v.nt,
                                                            (size_t)v.lds_bytes);
}

}  // namespace cfsim
