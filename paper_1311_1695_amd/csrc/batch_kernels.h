// Batched Jacobi-Davidson: many independent graphs, one persistent launch
// (batch.hip kernels, batch.cpp host side).
#pragma once

#include "lapeig_internal.h"

namespace lapeig {

constexpr int kBatchMaxK = 8;    // pairs per graph, the zero pair included
constexpr int kBatchMaxM = 16;   // largest m_max

struct BGraph {
    int n, nlong, k, pad;
    long long rp, ci;        // offsets into the packed row pointers and columns
    long long w64, w32;      // offsets (elements) into the workspaces
    long long out_vec;       // offset of the n x k eigenvector block
    long long out_val;       // offset of the k eigenvalues
};

struct BResult {
    int nconv, outer, inner, status;
    long long mvp;
};

struct BatchArgs {
    int ngraphs;
    const BGraph *graphs;
    const int *order;        // graph indices by decreasing nnz
    unsigned *queue;         // next position in `order`
    const int *rowptr, *col;
    const float *w32;        // edge weights (weighted batches), else null
    const double *w64;
    double *ws64;            // FP64 workspace
    void *ws32;              // PCG workspace (8 bytes per element reserved)
    double *out_vec, *out_val, *out_res;
    BResult *results;
    int m_min, m_max, itmax, kmax;
    double tol, rtol_pcg;
    unsigned long long seed;
    int lds_elems;           // PCG elements the launch's dynamic LDS holds (set by batch_launch)
};

void batch_launch(const BatchArgs &a, bool mixed, bool weighted, int grid, hipStream_t s);
// eigenvector blocks (src, plan order) into the caller's order with the sign
// convention; perm_all + perm_off[g]: graph g's caller -> plan map
void batch_unpack_launch(const BGraph *graphs, const BResult *results, const int *perm_all, const long long *perm_off,
                         int ngraphs, const double *src, double *dst, hipStream_t s);
// y = G x on every graph with the solver's row engine (x, y: FP32 when mixed,
// else FP64; graph g's entries at voff[g]); w32 non-null for weighted batches
void batch_spmv_launch(const BGraph *graphs, int ngraphs, const long long *voff, const int *rowptr, const int *col,
                       const float *w32, const double *w64, bool mixed, const void *x, void *y, int grid,
                       hipStream_t s);

}  // namespace lapeig
