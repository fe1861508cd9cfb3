// Internal declarations of the gfx950 Jacobi-Davidson library.
//
// Vertex order.  A plan renumbers the vertices by decreasing degree; inside
// one degree, vertices that share their first neighbour sit side by side
// (ties by the caller's index).  Every device array of a plan, and every
// kernel, works in that "plan order"; the C ABI converts at its edges.
//
// Matrix layout (plan order).  Only the adjacency part of G = D - A is
// stored: the Laplacian product is evaluated in edge-difference form
//   (G x)_i = sum_{j in N(i)} w_ij (x_i - x_j),
// which is G x for G = D - A (Section 2) with D_ii = sum_j w_ij, needs no
// diagonal, and has no cancellation between d_i x_i and sum_j w_ij x_j.
//   rows [0, n_huge)        degree > huge threshold: one workgroup per row (CSR)
//   rows [n_huge, n_long)   degree > long threshold (and the next rows up to a
//                           multiple of 32): one wavefront per row (CSR)
//   rows [n_long, n)        64-row slices, column-major inside a slice
//                           ("sliced ELLPACK"): lane l of a wavefront owns row
//                           n_long + 64 s + l and reads its s-th neighbour at
//                           sell_col[sell_off[slice] + 64 s + l]; padding
//                           entries point at the row itself, weight 0.
// On graphs small enough that the grid holds only a few units per SIMD, the
// row engine visits the first nslices_mid slices (those wider than kMidWidth
// slots) through the CSR arrays instead, eight lanes per row and eight rows
// per wavefront, so that no wavefront gathers much more than 64 kMidWidth
// entries and the widest slices no longer finish last; the block product
// reads them as slices.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <memory>
#include <vector>

#include "../../include/lapeig.h"

namespace lapeig {

constexpr int kBlock = 256;          // threads per workgroup (4 wavefronts)
constexpr int kWave = 64;
constexpr int kWavesPerBlock = kBlock / kWave;

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
const char *get_error();

struct Failure {
    lap_status code;
    std::string msg;
};

#define LAP_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::lapeig::Failure{LAP_EDEVICE, std::string(#call) + ": " +            \
                                                     hipGetErrorString(e_)};            \
    } while (0)

#define LAP_REQUIRE(cond, code, msg)                                                    \
    do {                                                                                \
        if (!(cond)) throw ::lapeig::Failure{code, msg};                                \
    } while (0)

// ------------------------------------------------------- device buffers
template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) count = 1;
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            throw Failure{LAP_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) +
                                          " bytes failed: " + hipGetErrorString(e)};
        }
        n = count;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    T *get() const { return p; }
};

// ------------------------------------------------------------ the graph
constexpr int kChunk = 64;   // edges per chunk of a long row in the block product
constexpr int kMidWidth = 8; // slices wider than this are visited eight lanes per row

struct Graph {
    int n = 0;
    int n_huge = 0, n_long = 0;   // row-class boundaries (plan order)
    int nslices = 0;              // 64-row slices covering [n_long, n)
    int nslices_mid = 0;          // leading slices visited eight lanes per row (row engine)
    int nchunks = 0;              // kChunk-edge chunks of the rows [0, n_long)
    int n_multi = 0;              // rows [0, n_multi) have two chunks or more (degree > kChunk)
    const int *chunk_row = nullptr;  // row of each chunk
    const int *chunk_off = nullptr;  // first chunk of each long row (n_long + 1)
    const int *rowptr = nullptr;  // CSR of A, plan order, n + 1
    const int *col = nullptr;
    const int *sell_off = nullptr;  // nslices + 1 offsets into sell_col
    const int *sell_col = nullptr;
};

template <typename T>
struct Weights {
    const T *csr = nullptr;   // weight of each CSR entry, or nullptr (unweighted)
    const T *sell = nullptr;  // weight of each slice entry, or nullptr
};

}  // namespace lapeig

namespace lapeig {
// FSAI factor Z of S = G + tau D in plan order (P = Z'Z ~ S^{-1}), stored
// along the CSR of A: for entry e of row i, zv[e] = Z(i, col[e]) when
// col[e] < i (row i of Z, the lower part [rowptr[i], mid[i])) and
// Z(col[e], i) when col[e] > i (column i of Z, the upper part
// [mid[i], rowptr[i+1])); zd[i] = Z(i, i).
template <typename T>
struct FsaiView {
    const int *rowptr = nullptr, *col = nullptr, *mid = nullptr;
    const T *zv = nullptr, *zd = nullptr;
    int n = 0, n_wave = 0;  // rows [0, n_wave) are summed by a wavefront each
};
}  // namespace lapeig

// The opaque plan of the C ABI.
namespace lapeig {
// Work areas a solver keeps in its plan between calls (device buffers and
// captured launch graphs), so repeated solves on one plan allocate nothing.
struct SolverCache {
    virtual ~SolverCache() = default;
};
}  // namespace lapeig

struct lap_plan {
    int n = 0;
    long long nnz_a = 0;     // off-diagonal entries (2 per edge)
    bool weighted = false;
    int device = 0;
    hipStream_t stream = nullptr;
    int huge_threshold = 0, long_threshold = 0;

    std::vector<int> perm;    // caller index -> plan index
    std::vector<int> iperm;   // plan index -> caller index
    std::vector<int> comp;    // component label per plan index, 0..ncomp-1
    std::vector<int> comp_size;
    int ncomp = 0;
    int max_degree = 0;

    lapeig::DevBuf<int> d_perm, d_iperm, d_comp;
    lapeig::DevBuf<int> d_rowptr, d_col, d_sell_off, d_sell_col, d_chunk_row, d_chunk_off;
    lapeig::DevBuf<float> d_w32, d_sellw32, d_dinv32;
    lapeig::DevBuf<double> d_w64, d_sellw64, d_dinv64;
    lapeig::Graph g;
    // scratch of the building-block entry points
    lapeig::DevBuf<double> d_shift;
    lapeig::DevBuf<char> tmp_x, tmp_y;
    lapeig::DevBuf<char> chunk_part;  // per-chunk partial sums of the block product
    // FSAI preconditioner (built on first use, plan order; see fsai.cpp)
    bool fsai_ready = false;
    double fsai_tau = 0.0;
    int fsai_max_row = 0;  // largest |P_v| of the factor
    lapeig::DevBuf<int> d_fsai_mid;
    lapeig::DevBuf<double> d_fsai_zv64, d_fsai_zd64;
    lapeig::DevBuf<float> d_fsai_zv32, d_fsai_zd32;
    template <typename T>
    lapeig::FsaiView<T> fsai() const;
    std::unique_ptr<lapeig::SolverCache> jd_cache;   // single-vector solver work areas
    std::unique_ptr<lapeig::SolverCache> jdb_cache;  // block solver work areas
    // plan-order CSR of A on the host (rebuilding the row classes needs it)
    std::vector<int> h_rowptr, h_col;
    std::vector<double> h_w;

    template <typename T>
    lapeig::Weights<T> weights() const;
    template <typename T>
    const T *dinv() const;
};

template <>
inline lapeig::FsaiView<float> lap_plan::fsai<float>() const {
    return {d_rowptr.get(), d_col.get(), d_fsai_mid.get(), d_fsai_zv32.get(), d_fsai_zd32.get(), n, g.n_long};
}
template <>
inline lapeig::FsaiView<double> lap_plan::fsai<double>() const {
    return {d_rowptr.get(), d_col.get(), d_fsai_mid.get(), d_fsai_zv64.get(), d_fsai_zd64.get(), n, g.n_long};
}

template <>
inline lapeig::Weights<float> lap_plan::weights<float>() const {
    return weighted ? lapeig::Weights<float>{d_w32.get(), d_sellw32.get()} : lapeig::Weights<float>{};
}
template <>
inline lapeig::Weights<double> lap_plan::weights<double>() const {
    return weighted ? lapeig::Weights<double>{d_w64.get(), d_sellw64.get()} : lapeig::Weights<double>{};
}
template <>
inline const float *lap_plan::dinv<float>() const { return d_dinv32.get(); }
template <>
inline const double *lap_plan::dinv<double>() const { return d_dinv64.get(); }

namespace lapeig {

// ------------------------------------------------------------- plan.cpp
void validate_laplacian(const lap_csr *L);  // throws Failure (no HIP calls)
// Validate (host), renumber, classify rows, build slices, upload.
// hub_order: inside a degree, group vertices by their first neighbour in plan
// order (else keep the caller's order)
void build_plan(const lap_csr *L, hipStream_t stream, lap_plan *plan, bool hub_order = true,
                int long_threshold = 32, int huge_threshold = 512);
// Rebuild the row classes of an existing plan for other thresholds.
void build_layout(lap_plan *plan, int long_threshold, int huge_threshold);

// ------------------------------------------------------------- tune.cpp
void autotune(lap_plan *plan, lap_dtype dt, int b, int target, const char *cache_path, lap_tune_info *info);

// -------------------------------------------------------------- dacg.hip
// Algorithm 3 (DACG): k smallest pairs, FP64, Jacobi preconditioner;
// o.kmax limits the iterations of each pair (0: 20000).
lap_status dacg_solve(lap_plan *P, int k, double tol, const lap_eigs_opts &o, double *evals, double *evecs,
                      int evecs_on_device, double *res_out, lap_eigs_info *info);

// -------------------------------------------------------------- irlm.hip
// Lanczos on G^+ with PCG inner solves and thick restarts (Algorithm 1 right).
lap_status irlm_solve(lap_plan *P, int k, double tol, int m, double rtol_inner, int itmax_inner,
                      const lap_eigs_opts &o, double *evals, double *evecs, int evecs_on_device, double *res_out,
                      lap_eigs_info *info);

// -------------------------------------------------------- consumers.hip
// Spectral bisection by the Fiedler vector f (device, caller order): part
// (device, caller order) = 0 for the n1 smallest entries (ties by index),
// 1 otherwise; cut (host or null) = weight of the edges between the sides.
lap_status fiedler_bisect(lap_plan *P, const double *f, int n1, int *part, double *cut, hipStream_t s);
// Y = T^(k) X (sigma = 0) or S^(k) X (sigma > 0); V, X, Y device column-major.
lap_status pinv_apply(int n, int k, const double *evals, const double *V, double sigma, int b, const double *X,
                      double *Y, hipStream_t s);

// ------------------------------------------------------------- fsai.cpp
constexpr double kFsaiTau = 1e-8;
// Builds the FSAI factor of the plan once (host, then uploaded); no-op when built.
void fsai_ensure(lap_plan *P);

// ------------------------------------------------------------- spmv.hip
// y = (G - sigma I) x, b = 1, plan order.
template <typename T>
void spmv(const lap_plan &P, const T *x, T *y, double sigma, hipStream_t s);
// Y = G X - X diag(shift) for n x b row-major blocks, plan order.
template <typename T>
void spmm(const lap_plan &P, int b, const T *X, T *Y, const double *shift_dev, hipStream_t s);
template <typename T>
void spmm(const lap_plan &P, int b, const T *X, int ldx, T *Y, int ldy, const double *shift_dev, hipStream_t s);
// the same with the per-chunk partial sums of the hub rows in `part`
// (P.g.nchunks x b values) instead of the plan's own area (null: the plan's)
template <typename T>
void spmm_part(const lap_plan &P, int b, const T *X, int ldx, T *Y, int ldy, const double *shift_dev, T *part,
               hipStream_t s);
// Y = G X - X diag(shift) for n x b blocks (ld b, b <= 32), and the column
// sums of X o Y as rows of 64 partials (columns past b zero) in dpart; returns
// the number of rows written, at most spmm_dot_rows(P, b), which dpart_rows
// must cover.  The rows add up in a fixed order (k_bfold).
template <typename T>
int spmm_dot(const lap_plan &P, int b, const T *X, T *Y, const double *shift_dev, T *dpart, size_t dpart_rows,
             hipStream_t s);
int spmm_dot_rows(const lap_plan &P, int b);

// Failure-path test hooks, read from the environment variable LAPEIG_FAULT
// (comma-separated names) at each solve:
//   nan_init       the first entry of the caller's start block becomes NaN
//                  once it is on the device, so the solver's own check drops
//                  the column and the seeded start takes its place;
//   pcg_breakdown  every correction equation is solved with the shift moved
//                  above the spectrum (4 max_i d_i + 1), so the projected
//                  operator is negative definite and the PCG stops at its
//                  first iteration on p'(G - theta I)p <= 0 and returns M(-r).
// Both force the condition from the host; every kernel runs as usual.
bool fault_enabled(const char *name);
// the shift of the pcg_breakdown hook for the plan's graph
double fault_breakdown_shift(const lap_plan &P);

// Reduction scratch: per-block partial sums and a completion counter.
struct ReduceScratch {
    DevBuf<double> partial;      // >= max_blocks * max_values doubles
    DevBuf<unsigned> counter;    // one counter per reduction site
    int max_blocks = 0;
    int max_values = 0;
    void ensure(int blocks, int values);
    // Deferred sums: two areas of darea x 64 doubles for per-workgroup
    // partial rows that the consuming launch folds (no fence, no counter);
    // darea = max(kDeferRows, 2 workgroups per compute unit).
    // After jd_orth: the 1-value rows of ||v||^2 (first area); after
    // jd_hborder (m + 1 <= kDeferBorderMax): the rows of the H border
    // (second area, stride border_ld, at most kDeferRows rows).
    DevBuf<double> dpart;
    int darea = 0;
    const double *norm_rows = nullptr;
    int norm_nrows = 0;
    const double *border_rows = nullptr;
    int border_nrows = 0, border_ld = 0;
    void ensure_deferred();
};
constexpr int kDeferRows = 256;       // grid of the kernels whose sums are deferred
constexpr int kDeferBorderMax = 32;   // H border values folded by the Rayleigh-Ritz kernel

// Gathers and scatters between caller order and plan order.
template <typename T>
void permute_rows(const int *map, int n, int b, const T *in, T *out, hipStream_t s);

// ------------------------------------------------------------ jd.cpp
lap_status jd_solve(lap_plan *P, int k, double tol, const lap_eigs_opts &o, double *evals,
                    double *evecs, int evecs_on_device, double *res, lap_eigs_info *info);

// ------------------------------------------------------------ blas.hip / pcg.hip
lap_status orth_block(int n, int q, const double *Q, int b, double *W, int *rank_out,
                      hipStream_t s);
lap_status pcg_entry(lap_plan *P, lap_dtype dt, int b, const double *theta_host, const double *Q,
                     int q, const double *R, double *T, int itmax, double rtol, int *iters_out,
                     int flags, hipStream_t s);

int device_cu_count();

lap_status batch_create(const lap_csr *Ls, int nb, lap_batch **out);
// time the row-class threshold candidates for the precision; keeps and
// returns the fastest (seconds per product pass over the batch in *secs)
int batch_autotune(lap_batch *B, bool mixed, int reps, double *secs);
// the threshold in use for the precision and whether it was tuned
void batch_layout(const lap_batch *B, bool mixed, int *long_threshold, int *tuned);
void batch_destroy(lap_batch *B);
int batch_total_n(const lap_batch *B);
lap_status batch_solve(lap_batch *B, int k, double tol, const lap_eigs_opts &o, double *evals, double *evecs,
                       int evecs_on_device, double *res, lap_eigs_info *infos, hipStream_t user);

}  // namespace lapeig
