// Graph-quality evaluation: working arrays and launchers shared by the
// library's entry points and the graph kernels.
#pragma once

#include "bkm_internal.h"

namespace bkm {

// Per-block working arrays of the graph metrics.
struct GraphDev {
    int64_t* comm;            // [k] communication volume
    int32_t* size;            // [k] vertices
    int32_t* seed;            // [k] lowest vertex (INT_MAX if empty)
    int32_t* conn;            // [k] 1 if the first search reached the whole block
    long long* cut2;          // [1] cut entries (each undirected edge twice)
    long long* sums;          // [3] max comm, total comm, disconnected blocks
    int* bad;                 // [1] invalid input seen
    // vertex lists: block b's vertices are mem[moff[b] .. moff[b+1])
    int32_t* moff;            // [k+1]
    int32_t* mem;             // [n]
    int32_t* fill;            // [k] list cursor while the lists are built
    // diameter bound (4-sweep, then iFUB rounds)
    int32_t* ecc1;            // [k] eccentricity of a1
    int32_t* lval;            // [k] l = max(ecc(a1), ecc(a2))
    int32_t* fi;              // [k] iFUB level i after the rounds
    int32_t* lb;              // [k] lower bound
    int32_t* ub;              // [k] upper bound
    int32_t* far1;            // [k] a1, the farthest vertex of the first search
    int32_t* nlev;            // [k] levels of the first search
    int32_t* clist;           // [k] connected blocks, in the order found
    int* ccount;              // [1] their count
    // the blocks' induced subgraphs relabelled: local id = position in mem
    int32_t* ldeg;            // [n] own-block neighbours of each vertex (input index)
    int2* al;                 // [n] block and local id of each vertex
    int64_t* lrp;             // [n+1] rows by local id
    int32_t* lcol;            // [<= nnz] own-block neighbours as local ids
};

// Points of the k-nearest-neighbour search: FP64 coordinates of the padded
// layout, one array per axis.
struct KnnPts {
    const double* x[3];
    const double* pbox;       // [8 ngroups][2d] boxes of the groups' 8-point parts
};
constexpr int kKnnParts = 8;  // parts per 64-point group
hipError_t launch_knn_widen(const RunDev& r, double* x, hipStream_t s);
hipError_t launch_knn_partbox(const RunDev& r, const KnnPts& P, double* hb, hipStream_t s);
hipError_t launch_knn(const RunDev& r, const KnnPts& P, int K, int32_t* nbr,
                      unsigned long long* visits, hipStream_t s);
// an optional vertex order (a permutation of 0..n-1, checked first) for the
// entry passes of the symmetrisation; NULL = input order
hipError_t launch_order_check(int64_t n, const int32_t* order, int32_t* mark, int* bad,
                              hipStream_t s);
// entries whose partner is missing: one bit each in miss (n*K bits, in the
// counting pass's order), read back by the fill
hipError_t launch_sym_count(int64_t n, int K, const int32_t* nbr, const int32_t* order,
                            int32_t* extra, unsigned long long* miss, int* bad, hipStream_t s);
int64_t scan_parts(int64_t n);
hipError_t launch_sym_rows(int64_t n, int K, const int32_t* extra, int64_t* part,
                           int64_t* row_ptr, hipStream_t s);
hipError_t launch_sym_fill(int64_t n, int K, const int32_t* nbr, const int32_t* order,
                           const unsigned long long* miss, const int64_t* row_ptr,
                           int32_t* cursor, int32_t* col, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_gm_vertex(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col,
                            const int32_t* A, int k, const GraphDev& g, hipStream_t s);
// diameter bounds: every block's vertex list (offsets, then members), then
// the first search of every block and the rest for the connected ones
hipError_t launch_block_lists(int64_t n, const int32_t* A, int k, const GraphDev& g, hipStream_t s);
hipError_t launch_local_rows(int64_t n, const int64_t* row_ptr, const int32_t* col,
                             const int32_t* A, const GraphDev& g, int32_t* dl, int64_t* part,
                             hipStream_t s);
hipError_t launch_diam_first(const int64_t* row_ptr, const int32_t* col, const int32_t* A, int k,
                             const GraphDev& g, int32_t* dist, int32_t* qa, int32_t* qb,
                             int32_t* levels, hipStream_t s);
hipError_t launch_diam_rest(int nconn, const GraphDev& g, int32_t* dist, int32_t* du, int32_t* qa,
                            int32_t* qb, int32_t* fr, unsigned long long* seen,
                            unsigned long long* arr0, unsigned long long* arr1, int32_t* levels,
                            hipStream_t s);
hipError_t launch_gm_final(int k, const GraphDev& g, int32_t* diam_out, int32_t* diam_ub_out,
                           int64_t* comm_out, double* summary, hipStream_t s);

}  // namespace bkm
