// Launchers and state of the block Jacobi-Davidson path (block.hip,
// jd_block.cpp).  Block vectors are row-major with an explicit leading
// dimension; the basis [X | V] is one row-major n x (k + m_max) array.
#pragma once

#include "jd_kernels.h"

namespace lapeig {

constexpr int kMaxBlock = 32;
// largest per-workgroup partial matrix of the fused block-PCG pass (and of
// its totals): (2 x 32 + 2) rows of 32 columns
constexpr int kFusedMax = (2 * 32 + 2) * 32;

// Partial tiles of the tall-skinny products: up to 2 x CUs workgroups,
// 128 x 32 entries each.
struct BlockScratch {
    DevBuf<double> part;
    void ensure() {
        if (part.get()) return;
        part.alloc((size_t)2 * device_cu_count() * 128 * 32);
    }
};

struct BlockStatus {
    double theta[kMaxBlock], rnorm[kMaxBlock], unorm[kMaxBlock];
    int kept;
};

// Block PCG state.  A launch never reads what workgroups of the same
// launch write: the per-column flags and rho alternate between two slots,
// and the folded sums of consecutive reductions between tot_a and tot_b.
template <typename T>
struct BPcgState {
    T tot_a[64], tot_b[64];  // column sums of the last reductions (value c, or 32 + c)
    T r0[kMaxBlock];
    T rho[2][kMaxBlock];
    int act[2][kMaxBlock];   // column still iterating
    int its[kMaxBlock], brk[kMaxBlock];
};

template <typename T>
struct BPcgWork {
    DevBuf<T> res, p, s, y, z, C, part;
    // fused iteration (b, q <= 32): per-workgroup partial tiles, their
    // totals, and the totals of the W = Q'D^{-1}Q pass (kFusedMax each)
    DevBuf<T> kt_part, kt_tot, kt_w;
    // the block product's rows of p'Ap partials (spmm_dot), 64 values a row
    DevBuf<T> dpart;
    DevBuf<BPcgState<T>> st;
    void ensure_dot(size_t rows) {
        if (dpart.n < rows * 64) dpart.alloc(rows * 64);
    }
    void ensure(int n, int b, int qmax) {
        if (res.get()) return;
        res.alloc((size_t)n * b); p.alloc((size_t)n * b); s.alloc((size_t)n * b); y.alloc((size_t)n * b);
        z.alloc((size_t)n * b);
        C.alloc((size_t)(qmax + 1) * b);
        // per-workgroup partial rows, also the 1024 first-stage rows of the
        // product's p'Ap sums
        part.alloc((size_t)std::max(4 * device_cu_count() + kMaxBlock, 1024) * 64);
        kt_part.alloc((size_t)2 * device_cu_count() * kFusedMax);
        kt_tot.alloc(kFusedMax);
        kt_w.alloc(kFusedMax);
        st.alloc(1);
    }
};

// C (ka x kb, column-major ldc) = alpha A'B  (A n x ka, B n x kb, row-major); when
// mirror is given, also mirror[j + i ldm] = C(i, j) for i < ka - kb (the
// border of a symmetric matrix whose new kb x kb corner C already holds).
// kb <= 32, ka <= 128.
template <typename T>
void ts_tn(int n, const T *A, int lda, int ka, const T *B, int ldb, int kb, T *out, int ldc, T *mirror, int ldm,
           T alpha, BlockScratch &bs, hipStream_t s);
// Out = alpha A C + (addend if given, else beta Out); C ka x kb column-major.
// Out may be the same rows as A (in-place rotation).  ka, kb <= 128.
template <typename T>
void ts_prepare();
template <typename T>
void ts_nn(int n, const T *A, int lda, int ka, const T *C, int ldc, int kb, T *Out, int ldo, const T *addend,
           int ldadd, T alpha, T beta, hipStream_t s);

// SVQB scaling: keep eigenvalues above max(rel lam_max, abs_thr)
void blk_svqb(int b, const double *lam, const double *Z, int ldz, double rel, double abs_thr, double *M, int ldm,
              BlockStatus *st, hipStream_t s);
// CholQR coefficients of a block from its Gram matrix S (b x b, ld lds, b <=
// 32): M (b x b, ld ldm) such that V M has st->kept orthonormal columns
// (pivoted Cholesky, the same drop thresholds as blk_svqb), then zero columns
void blk_cholqr(int b, const double *S, int lds, double rel, double abs_thr, double *M, int ldm, BlockStatus *st,
                hipStream_t s);
template <typename T>
void blk_zero_space(int n, int nz, const int *comp, const double *isz, double *XV, int ldb, T *Q, int ldq,
                    hipStream_t s);
void blk_extract(int n, int nc, const double *in, int ldi, double *out, hipStream_t s);
// flags_dev[c] |= 1 for each column c of the n x b column-major block with a non-finite entry
void blk_nonfinite_cols(int n, int b, const double *in, int *flags_dev, hipStream_t s);
// out[map[i] * ldo + c] = in[i + c n] (map NULL: identity)
void blk_cm_to_rm(int n, int b, const double *in, const int *map, double *out, int ldo, hipStream_t s);
template <typename T>
void blk_resid(int n, int bu, const double *U, int ldu, const double *GU, int ldg, int ldr, const double *theta,
               double *R, T *Q, int ldq, int qoff, double *u0, ReduceScratch &rs, BlockStatus *st, hipStream_t s);
template <typename S>
void blk_to_f64(int n, int b, const S *in, int ldi, double *out, int ldo, hipStream_t s);
void blk_random(int n, int b, uint64_t seed, long long colbase, const int *iperm, double *out, int ldo,
                hipStream_t s);
// Enqueues iterations it_first .. it_last (of at most itmax) of the block
// PCG; it_first == 1 also enqueues its set-up.  After a segment that ends
// before itmax, w.st->act[0][0..b) flags the columns still iterating.
template <typename T>
void bpcg_enqueue(const lap_plan &P, int b, const double *theta_dev, const T *Q, int ldq, int q, const double *R,
                  int ldr, T *X, BPcgWork<T> &w, BlockScratch &bs, int itmax, int it_first, int it_last, double rtol,
                  hipStream_t s);

lap_status jd_block_solve(lap_plan *P, int k, double tol, const lap_eigs_opts &o, double *evals, double *evecs,
                          int evecs_on_device, double *res, lap_eigs_info *info);

}  // namespace lapeig
