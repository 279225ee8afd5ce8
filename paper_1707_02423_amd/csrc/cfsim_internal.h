// Internal declarations shared by the HIP translation units of libcfsim.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cfsim.h"

namespace cfsim {

constexpr int kWave = 64;

// ---------------------------------------------------------------- graphs
// Device pointers of one graph in the packed layout described in cfsim.h.
struct GraphRef {
    int n, nnz;
    const int32_t* rp;   // [n+1] successor offsets
    const int32_t* ci;   // [nnz] successor ids
    const double* w;     // [nnz] weights (CSR order)
    const int32_t* cp;   // [n+1] predecessor offsets
    const int32_t* ri;   // [nnz] predecessor ids
    const int32_t* eid;  // [nnz] CSR position of each CSC entry
};

struct SetRef {
    const int64_t* node_off;
    const int64_t* edge_off;
    const int32_t* rp;
    const int32_t* ci;
    const double* w;
    const int32_t* cp;
    const int32_t* ri;
    const int32_t* eid;
    int n_graphs;
};

__host__ __device__ inline GraphRef graph_of(const SetRef& s, int g) {
    GraphRef r;
    int64_t n0 = s.node_off[g], n1 = s.node_off[g + 1];
    int64_t e0 = s.edge_off[g], e1 = s.edge_off[g + 1];
    r.n = (int)(n1 - n0);
    r.nnz = (int)(e1 - e0);
    r.rp = s.rp + n0 + g;
    r.cp = s.cp + n0 + g;
    r.ci = s.ci + e0;
    r.w = s.w + e0;
    r.ri = s.ri + e0;
    r.eid = s.eid + e0;
    return r;
}

// ---------------------------------------------------------------- pair shape
// The kernels store S in a "compute orientation": rows are the nodes of the
// R graph (handled wave-uniformly), columns the nodes of the C graph (one lane
// per column, in 64-column chunks).  R = B, C = A keeps S as n_B x n_A; the
// swapped choice (R = A, C = B) stores S^T.  Wave w owns rows w, w + NW, ...
struct PairShape {
    int swap;    // 1: stored matrix is S^T (rows = A, columns = B)
    int nR, nC;  // stored rows / columns
    int nchunk;  // ceil(nC / 64)
    int rows;    // rows per wave, ceil(nR / NW)
};

// Kernel-variant table of the LDS-resident pair kernel.
struct Variant {
    int nt;         // threads per workgroup
    int nch;        // max 64-column chunks per lane
    int maxr;       // max rows per wave (S_{k-2} registers = nch * maxr)
    int lds_bytes;  // dynamic LDS per workgroup
};

constexpr int kNumVariants = 4;
// Larger variants serve larger pairs; a pair runs on the first that fits.
// FP64 keeps half as many S_{k-2} values per lane in registers.
__host__ __device__ inline Variant variant_info(int v, int esize) {
    if (esize == 8) {
        switch (v) {
            case 0: return Variant{64, 1, 16, 16 * 1024};
            case 1: return Variant{256, 2, 8, 40 * 1024};
            case 2: return Variant{512, 2, 8, 78 * 1024};
            default: return Variant{1024, 2, 8, 159 * 1024};
        }
    }
    switch (v) {
        case 0: return Variant{64, 2, 16, 16 * 1024};
        case 1: return Variant{256, 4, 8, 40 * 1024};
        case 2: return Variant{512, 2, 16, 78 * 1024};
        default: return Variant{1024, 4, 8, 159 * 1024};
    }
}

__host__ __device__ inline size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

__host__ __device__ inline PairShape make_shape(int nA, int nB, int swap, int NW) {
    PairShape s;
    s.swap = swap;
    s.nR = swap ? nA : nB;
    s.nC = swap ? nB : nA;
    s.nchunk = (s.nC + 63) / 64;
    s.rows = (s.nR + NW - 1) / NW;
    return s;
}

// Bytes of dynamic LDS one pair needs in the LDS-resident kernel.
// Layout: S_cur, S_next [nR*nC] | R rows int4 [nR] | R succ, pred edges [nnzR]
//         | C columns int4 [nC] | C succ, pred edges [nnzC]
//         | rstate, rbest [nR] | cstate, cbest [nC]
__host__ __device__ inline size_t lds_pair_bytes(const PairShape& s, int nnzR, int nnzC, int esize) {
    const size_t edge = (esize == 8) ? 16 : 8;
    size_t b = 2 * align16((size_t)s.nR * s.nC * esize);
    b += align16((size_t)s.nR * 16) + 2 * align16((size_t)nnzR * edge);
    b += align16((size_t)s.nC * 16) + 2 * align16((size_t)nnzC * edge);
    b += 2 * align16((size_t)s.nR * 4);
    b += 2 * align16((size_t)s.nC * 4);
    return b;
}

// Orientation choice: prefer the one that fills 64-lane chunks better; take
// the other if only it fits the variant.  Returns false if neither fits.
__host__ __device__ inline bool choose_shape(int nA, int nB, int nnzA, int nnzB, int variant, int esize,
                                             PairShape* out) {
    const Variant v = variant_info(variant, esize);
    const int NW = v.nt / 64;
    const int cA = (nA + 63) / 64, cB = (nB + 63) / 64;
    const int pref = ((long long)nB * cA > (long long)nA * cB) ? 1 : 0;
    for (int k = 0; k < 2; ++k) {
        const int swap = k == 0 ? pref : 1 - pref;
        const PairShape s = make_shape(nA, nB, swap, NW);
        const int nnzR = swap ? nnzA : nnzB;
        const int nnzC = swap ? nnzB : nnzA;
        if (s.nchunk <= v.nch && s.rows <= v.maxr &&
            lds_pair_bytes(s, nnzR, nnzC, esize) <= (size_t)v.lds_bytes) {
            *out = s;
            return true;
        }
    }
    return false;
}

// ---------------------------------------------------------------- launch descriptors
struct PairJob {
    // pairs: either one explicit pair (single = 1) or pairs of a graph set
    int single;
    GraphRef ga, gb;
    SetRef set;
    const int32_t* pair_a;
    const int32_t* pair_b;
    // schedule: items [bounds[0], bounds[1]) of `order`, pulled through `queue`
    const int32_t* order;
    const int32_t* bounds;
    int32_t* queue;
    // options
    int max_iter;
    double tol;
    // outputs
    cfsim_pair_result* res;
    int32_t* match;
    const int64_t* match_off;
    void* S_out;
    const int64_t* S_off;
    int variant;
    int lds_bytes;
};

// Plan: assign every pair a variant (bucket) and order each bucket longest
// first.  Writes order[n_pairs], bounds[2*(kNumVariants+1)] and zeroes the
// queues[kNumVariants+1].  Bucket kNumVariants holds pairs no variant fits.
struct PlanJob {
    SetRef set;
    const int32_t* pair_a;
    const int32_t* pair_b;
    int64_t n_pairs;
    int esize;
    int32_t* order;
    int32_t* bounds;
    int32_t* queues;
};

// Host-side launchers (return hipError_t as int).
int launch_pair_lds(int variant, int dtype, const PairJob& job, int grid, hipStream_t stream);
int launch_plan(const PlanJob& job, hipStream_t stream);
int set_kernel_attributes();
int occupancy_of(int variant, int dtype, int* blocks);

struct PackJob {
    int n_graphs;
    const int64_t* node_off;
    const int64_t* edge_off;
    const int32_t* src;
    const int32_t* dst;
    const double* count;
    int32_t* rp;
    int32_t* ci;
    double* w;
    int32_t* cp;
    int32_t* ri;
    int32_t* eid;
    int32_t* err;
    int32_t* cursor;   // [total_nodes] workspace
    int32_t* eorig;    // [total_edges] workspace
    int32_t* csrpos;   // [total_edges] workspace
};
int launch_pack(const PackJob& job, hipStream_t stream);

}  // namespace cfsim
