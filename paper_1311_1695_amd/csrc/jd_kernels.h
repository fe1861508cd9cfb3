// Launchers of the Jacobi-Davidson kernels (blas.hip, pcg.hip) used by the
// host driver (jd.cpp) and the C ABI.
#pragma once

#include <algorithm>

#include "lapeig_internal.h"

namespace lapeig {

constexpr int kMaxBasis = 64;   // columns of [X | V] handled by the single-vector kernels
constexpr int kMaxQ = 62;       // projector columns in the PCG kernels

// Small status block written by the kernels and read by the host once per
// outer iteration.
struct JDStatus {
    double coef[kMaxBasis];
    double orth_n0, orth_n1, inv_norm;
    double theta, unorm, rnorm;
    double cert_theta, cert_unorm2, cert_rnorm;
    int degenerate, rr_sweeps;
};

// PCG scalars that outlive one launch.  Launch number sq of a solve is a
// no-op once stop_seq is nonzero and <= sq; a launch that decides to stop
// writes stop_seq = sq + 1, which no other workgroup of the same launch
// treats as a stop, so the flag never races with its readers.
// The few status values the host decides on, published by the kernel that
// finishes them into host-coherent pinned memory: payload first, then a
// system-scope fence, then the sequence number the host waits for.
struct HostMirror {
    double theta, unorm, rnorm, cert_theta, cert_rnorm;
    int degenerate, pad;
    unsigned seq, pad2;
};

constexpr int kPipeQ = 14;  // widest projector of the one-launch-per-iteration PCG

// Column stride of the PCG's column-major operands: n rounded up to 32
// values, so every column starts on a 128-byte line as the vectors do.
__host__ __device__ inline size_t col_ld(size_t n) { return (n + 31) & ~(size_t)31; }

template <typename T>
struct PcgState {
    T rho[2];   // rho = res' M res of the last two iterations, by parity
    T r0;       // norm of the right-hand side
    // pipelined form: gamma, alpha and Q's of the last two iterations
    T gam[2], alp[2], cs[2][16];
    int stop_seq, iters, breakdown;
    int total;  // products of all solves since the host last cleared it
};

// Workgroups of one PCG launch, bounded so that folding the partial sums of
// the previous launch stays cheap in every workgroup: at most four per
// compute unit (the scratch areas are sized for that), two for the vector
// kernels; the one-launch iteration takes as many as fit at once.
inline int pcg_max_groups() { return 4 * device_cu_count(); }
inline int pcg_vec_groups() { return 2 * device_cu_count(); }

template <typename S>
void jd_orth(int n, const double *B, int nb, const S *src, double *v, ReduceScratch &rs, JDStatus *st,
             hipStream_t s);
// V[:, m] = v / ||v|| and W[:, m] = G V[:, m], the norm folded from the
// partial rows that jd_orth left in rs (which also records it in st)
void jd_expand(const lap_plan &P, const double *v, double *vcol, double *wcol, JDStatus *st,
               const ReduceScratch &rs, hipStream_t s);
void jd_hborder(int n, const double *V, int m, const double *wcol, double *H, int ldh, ReduceScratch &rs,
                hipStream_t s);
// Eigenpairs of the m x m H (column-major, ld ldh): theta ascending, Y
// column-major (ld ldy).  mprev in [1, m): theta and Y still hold the
// eigenpairs of the leading mprev x mprev block, which has not changed
// since (warm start); 0: none.  border: the partial rows that jd_hborder
// left for the last column of H, folded (and written to H) first, or null
// (then H is only read).  st->rr_sweeps: -1 after the secular-equation
// path, else the Jacobi sweeps.  wide: H is not an arrowhead (block JD), so
// even m <= 32 takes the many-wavefront Jacobi launch.
void jd_rr(int m, double *H, int ldh, double *theta, double *Y, int ldy, JDStatus *st, hipStream_t s,
           int mprev = 0, const ReduceScratch *border = nullptr, bool wide = false);
template <typename T>
void jd_ritz(int n, const double *V, const double *W, int m, const double *Y, const double *theta, double *u,
             double *r, T *Q, int ldq, int qcol, ReduceScratch &rs, JDStatus *st, hipStream_t s,
             HostMirror *hm = nullptr, unsigned seq = 0);
void jd_certify(const lap_plan &P, const double *u, double *gu, ReduceScratch &rs, JDStatus *st, hipStream_t s,
                HostMirror *hm = nullptr, unsigned seq = 0);
void jd_rotate(int n, int m, const double *Y, int ldy, const double *vin, double *vout, int vc0, int vnc,
               const double *vscale0, const double *win, double *wout, int wc0, int wnc, hipStream_t s);
void jd_hdiag(double *H, int ldh, int cnt, const double *theta, int off, hipStream_t s);
template <typename T>
void jd_zero_space(int n, int nz, const int *comp, const double *inv_sqrt_size, double *B, T *Q, int ldq,
                   hipStream_t s);
void jd_random(int n, uint64_t seed, long long colidx, const int *iperm, double *v, hipStream_t s);
// out = v * inv_norm (the normalization left by jd_orth)
// out = v / ||v|| with the norm folded from the partial rows jd_orth left in rs
void jd_scale_copy(int n, const double *v, double *out, JDStatus *st, const ReduceScratch &rs, hipStream_t s);

// Eigenvector output: out (n x nconv column-major, caller order, device) =
// columns order[j] of X (plan order, element (i, c) at X[i sr + c sc]),
// each with its largest-magnitude entry made positive (ties: lowest index).
// part: device scratch of 2 nconv final_chunks(n) doubles.
int final_chunks(int n);
void jd_finalize(int n, int nconv, const double *X, long long sr, long long sc, const int *order_dev,
                 const int *perm_dev, double *out_dev, double *part, hipStream_t s);

// Writes the nconv locked pairs (values lam, residuals resid, vectors the
// columns of X as for jd_finalize) in ascending order to the caller's
// buffers (evecs on the device or in host memory), then synchronizes s.
void emit_pairs(const lap_plan &P, int nconv, const double *X, long long sr, long long sc,
                const std::vector<double> &lam, const std::vector<double> &resid, double *evals, double *evecs,
                int evecs_on_device, double *res_out, DevBuf<double> &scratch, hipStream_t s);

// PCG work vectors (plan order, type T).
template <typename T>
struct PcgWork {
    DevBuf<T> res, p, s, y;
    DevBuf<T> gq;    // G Q, row-major like Q
    DevBuf<T> part;  // two areas of per-workgroup partial sums (ping-pong)
    // pipelined form: u = M res, w ~ A u, wh = D^{-1} w (two buffers), q, z;
    // qq = [Q | D^{-1}Q] and gqq = G qq (row-major, 2q columns); K = Q'D^{-1}Q
    DevBuf<T> u, w, wh, qv, z, qq, gqq, kmat, kpart;
    // the same operands column-major for the iterations: Q (q columns) and
    // [G Q | G D^{-1}Q] (2q columns), ld n
    DevBuf<T> qcm, gqcm;
    DevBuf<PcgState<T>> st;
    void ensure(int n, int ldq) {
        if (res.n < (size_t)n || !st.get()) {
            res.alloc(n); p.alloc(n); s.alloc(n); y.alloc(n);
            u.alloc(n); w.alloc(n); wh.alloc(2 * (size_t)n); qv.alloc(n); z.alloc(n);
            part.alloc(2 * (size_t)pcg_max_groups() * 64);
            kmat.alloc(256);
            kpart.alloc((size_t)pcg_max_groups() * 256);
            st.alloc(1);
        }
        if (gq.n < (size_t)n * ldq) gq.alloc((size_t)n * ldq);
        const size_t wq = 2 * (size_t)std::min(ldq, kPipeQ);
        if (qq.n < (size_t)n * wq) {
            qq.alloc((size_t)n * wq); gqq.alloc((size_t)n * wq);
            qcm.alloc(col_ld(n) * (wq / 2)); gqcm.alloc(col_ld(n) * wq);
        }
    }
};

// One correction equation: t solves the projected system for theta (device
// scalar), projector Q (row-major n x ldq, first q columns), right-hand side
// -r (r double, plan order).  Enqueues everything; nothing is read back.
// inc: the previous call on w had the same q and Q, except possibly its last
// column (the products of the first q - 1 columns are then reused).
// fsai: P = Z'Z (the plan's FSAI factor, fsai_ensure first) instead of D^{-1},
// in the two-launch form with the two FSAI products between its launches.
// classic: the two-launch form even where the pipelined one applies (its
// recurrences keep the true residual closer to the computed one, which
// accurate solves need).
template <typename T>
void pcg_enqueue(const lap_plan &P, const double *theta_dev, const T *Q, int ldq, int q, const double *r, T *t,
                 PcgWork<T> &w, int itmax, double rtol, hipStream_t s, bool inc = false, bool fsai = false,
                 bool classic = false);

}  // namespace lapeig
