// PCG on the projected correction equation (Algorithm 2 step 8):
//   (I - QQ')(G - theta I)(I - QQ') t = -r,   t orthogonal to Q,
// with the projected preconditioner M = (I-QQ')P(I-QQ') of the comments on
// Algorithm 2 and P = D^{-1} (Jacobi).  Q = [x_1 .. x_{j-1} u] as in
// eq. (JDsismorethanone).  The residual stays orthogonal to Q, so
//   M res = (I - QQ') D^{-1} res,   A_p p = (I - QQ')(G - theta I) p,
//   rho = res' M res = res' D^{-1} res.
// One iteration is two launches; each one folds the partial sums that the
// launch before it left (see fold_partials), so no launch needs a
// cross-workgroup synchronization of its own.  With GQ = G Q formed once
// per solve, s = (G - theta I) p follows p through the recurrence
//   p' = (y - Q c1) + beta p
//   s' = (G - theta I) y - GQ c1 + theta Q c1 + beta s
// so the product only gathers y, which the previous launch completed:
//   KA  fold ||res||, rho', c1 = Q'y;  stop test;  beta = rho'/rho;
//       p and s as above;                           partials p's, Q's
//   KB  fold pAp, c2 = Q's;  alpha = rho / pAp;  t += alpha p;
//       res -= alpha (s - Q c2);  y = D^{-1} res;    partials res'res, res'y, Q'y
// A device flag turns the remaining launches into no-ops once the iteration
// stops, so the whole solve is enqueued without host round trips.
#include <cstdlib>

#include "lapeig_dev.h"
#include "jd_kernels.h"

namespace lapeig {

namespace {

// launch numbers within one solve: init1 0, init2 1, then per iteration
// it = 1, 2, ...: KA 2it, KB 2it+1
template <typename T>
__device__ __forceinline__ bool stopped(const PcgState<T> *st, int sq) {
    const int v = st->stop_seq;
    return v != 0 && v <= sq;
}

__device__ __forceinline__ bool leader() { return blockIdx.x == 0 && threadIdx.x == 0; }

// init1: res = -r, t = 0;  partials r'r, -Q'r
template <typename T, int NV>
__global__ __launch_bounds__(kBlock) void k_pcg_init1(int n, const double *__restrict__ r, T *__restrict__ res,
                                                      T *__restrict__ t, const T *__restrict__ Q, int ldq, int q,
                                                      T *__restrict__ part_out, PcgState<T> *st) {
    if (leader()) {
        st->stop_seq = 0;
        st->iters = 0;
        st->breakdown = 0;
    }
    T acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = T(0);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const T ri = (T)r[i];
        res[i] = -ri;
        t[i] = T(0);
        acc[0] += ri * ri;
#pragma unroll
        for (int j = 0; j < NV - 1; ++j)
            if (j < q) acc[1 + j] -= Q[(size_t)i * ldq + j] * ri;
    }
    write_partials<T, NV>(acc, q + 1, part_out);
}

// init2: r0 = ||r||, c0 = -Q'r;  res -= Q c0 (project the right-hand side);
// y = D^{-1} res;  partials res'y, Q'y
// With FSAI the preconditioned vector comes from the two launches that
// follow (k_fsai_lo, k_fsai_up), which also leave the partial sums: here
// only the projection of res.
template <typename T, int NV, bool FSAI>
__global__ __launch_bounds__(kBlock) void k_pcg_init2(int n, T *__restrict__ res, T *__restrict__ y,
                                                      const T *__restrict__ dinv, const T *__restrict__ Q, int ldq,
                                                      int q, const T *__restrict__ part_in, int nb_in,
                                                      T *__restrict__ part_out, PcgState<T> *st) {
    __shared__ T tot[NV];
    fold_partials<T, NV>(part_in, nb_in, q + 1, tot);
    const T r0 = sqrt(tot[0]);
    if (leader()) {
        st->r0 = r0;
        if (!(r0 > T(0))) st->stop_seq = 2;
    }
    if (!(r0 > T(0))) return;
    T acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = T(0);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const T *qi = Q + (size_t)i * ldq;
        T proj = T(0);
#pragma unroll
        for (int j = 0; j < NV - 1; ++j)
            if (j < q) proj += qi[j] * tot[1 + j];
        const T ri = res[i] - proj;
        res[i] = ri;
        if (FSAI) continue;
        const T yi = dinv[i] * ri;
        y[i] = yi;
        acc[0] += ri * yi;
#pragma unroll
        for (int j = 0; j < NV - 1; ++j)
            if (j < q) acc[1 + j] += qi[j] * yi;
    }
    if (!FSAI) write_partials<T, NV>(acc, q + 1, part_out);
}

// KA.  INIT (first iteration): fold rho = res'y and c1 = Q'y of init2, beta
// = 0.  Otherwise fold ||res||, rho' and c1 of KB, stop when ||res|| <=
// rtol ||r||, beta = rho'/rho.  Then p = (y - Q c1) + beta p and
// s = (G - theta I) p by the recurrence;  partials p's, Q's.
template <typename T, int NV>
struct PsRow {
    T p, s, qv[NV], gq[NV];
};

template <typename T, int NV, bool Wt, bool INIT>
__global__ __launch_bounds__(kBlock) void k_pcg_ps(Graph g, Weights<T> w, const double *__restrict__ theta,
                                                   const T *__restrict__ y, T *__restrict__ p, T *__restrict__ s,
                                                   const T *__restrict__ Q, const T *__restrict__ GQ, int ldq, int q,
                                                   const T *__restrict__ part_in, int nb_in, T *__restrict__ part_out,
                                                   PcgState<T> *st, int sq, int it, T rtol) {
    constexpr int OFF = INIT ? 1 : 2;
    constexpr int NQ = NV - OFF;
    // scalars first, so that their latency overlaps the fold
    const int stop_v = st->stop_seq;
    const T th = (T)theta[0];
    const T r0 = st->r0;
    const T rho_prev = st->rho[it & 1];  // rho of the iteration before (parity it - 2)
    __shared__ T tot[NV];
    fold_partials<T, NV>(part_in, nb_in, q + OFF, tot);
    if (stop_v != 0 && stop_v <= sq) return;
    T beta = T(0);
    if (INIT) {
        if (leader()) st->rho[0] = tot[0];
    } else {
        const T rn = sqrt(tot[0]);
        if (rn <= rtol * r0) {
            if (leader()) st->stop_seq = sq + 1;
            return;
        }
        beta = tot[1] / rho_prev;
        if (leader()) st->rho[(it - 1) & 1] = tot[1];
    }
    T acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = T(0);
    // narrow projectors: the rows of Q and GQ are requested before the
    // gathers; wide ones (too many registers) load them after
    constexpr bool PREF = NV <= 16;
    constexpr int NQP = PREF ? NQ : 1;
    auto pre = [&](int i) {
        PsRow<T, NQP> d;
        d.p = INIT ? T(0) : p[i];
        d.s = INIT ? T(0) : s[i];
        if (PREF) {
            const T *qi = Q + (size_t)i * ldq;
            const T *gi = GQ + (size_t)i * ldq;
#pragma unroll
            for (int j = 0; j < NQP; ++j) {
                d.qv[j] = j < q ? qi[j] : T(0);
                d.gq[j] = j < q ? gi[j] : T(0);
            }
        }
        return d;
    };
    for_each_row_pre<T, Wt, false>(g, w, y, pre, [&](int i, T yi, T gyi, T, const PsRow<T, NQP> &d) {
        const T *qi = Q + (size_t)i * ldq;
        const T *gi = GQ + (size_t)i * ldq;
        auto qval = [&](int j) { return PREF ? d.qv[j < NQP ? j : 0] : (j < q ? qi[j] : T(0)); };
        auto gval = [&](int j) { return PREF ? d.gq[j < NQP ? j : 0] : (j < q ? gi[j] : T(0)); };
        T qc = T(0), gc = T(0);
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            qc += qval(j) * tot[OFF + j];
            gc += gval(j) * tot[OFF + j];
        }
        T pi = yi - qc;
        T si = ((gyi - th * yi) - gc) + th * qc;
        if (!INIT) {
            pi += beta * d.p;
            si += beta * d.s;
        }
        p[i] = pi;
        s[i] = si;
        acc[0] += pi * si;
#pragma unroll
        for (int j = 0; j < NV - 1; ++j)
            if (j < NQ) acc[1 + j] += qval(j) * si;
    });
    write_partials<T, NV>(acc, q + 1, part_out);
}

// KB: fold pAp and c2 = Q's; breakdown test; alpha = rho / pAp;
// t += alpha p;  res -= alpha (s - Q c2);  y = D^{-1} res;
// partials res'res, res'y, Q'y
template <typename T, int NV>
struct UpRow {
    T t, p, res, s, dinv, qv[NV];
};

template <typename T, int NV, bool FSAI>
__global__ __launch_bounds__(kBlock) void k_pcg_update(int n, T *__restrict__ t, T *__restrict__ res,
                                                       const T *__restrict__ p, const T *__restrict__ s,
                                                       T *__restrict__ y, const T *__restrict__ dinv,
                                                       const T *__restrict__ Q, int ldq, int q,
                                                       const T *__restrict__ part_in, int nb_in,
                                                       T *__restrict__ part_out, PcgState<T> *st, int sq, int it) {
    constexpr int NQ = NV - 2;
    constexpr bool PREF = NV <= 16;  // wide projectors: Q rows are loaded where used
    constexpr int NQP = PREF ? NQ : 1;
    auto load = [&](int i) {
        UpRow<T, NQP> d;
        d.t = t[i];
        d.p = p[i];
        d.res = res[i];
        d.s = s[i];
        d.dinv = dinv[i];
        if (PREF) {
            const T *qi = Q + (size_t)i * ldq;
#pragma unroll
            for (int j = 0; j < NQP; ++j) d.qv[j] = j < q ? qi[j] : T(0);
        }
        return d;
    };
    // the first row's operands and the scalars are requested before the fold
    const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    const int stop_v = st->stop_seq;
    const T rho = st->rho[(it - 1) & 1];
    UpRow<T, NQP> d0;
    if (i0 < n) d0 = load(i0);
    __shared__ T tot[NV];
    fold_partials<T, NV>(part_in, nb_in, q + 1, tot);
    if (stop_v != 0 && stop_v <= sq) return;
    const T pap = tot[0];
    if (!(pap > T(0))) {  // the projected operator is indefinite along p
        if (leader()) {
            st->stop_seq = sq + 1;
            st->breakdown = it;
            st->total += 1;  // the product of the failed step counts
        }
        // no step was taken before the breakdown: return M(-r), which p holds
        if (it == 1)
            for (int i = i0; i < n; i += stride) t[i] = p[i];
        return;
    }
    const T alpha = rho / pap;
    if (leader()) {
        st->iters = it;
        st->total += 1;
    }
    T acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = T(0);
    for (int i = i0; i < n; i += stride) {
        const UpRow<T, NQP> d = i == i0 ? d0 : load(i);
        const T *qi = Q + (size_t)i * ldq;
        auto qval = [&](int j) { return PREF ? d.qv[j < NQP ? j : 0] : (j < q ? qi[j] : T(0)); };
        T proj = T(0);
#pragma unroll
        for (int j = 0; j < NQ; ++j) proj += qval(j) * tot[1 + j];
        t[i] = d.t + alpha * d.p;
        const T ri = d.res - alpha * (d.s - proj);
        res[i] = ri;
        if (FSAI) continue;
        const T yi = d.dinv * ri;
        y[i] = yi;
        acc[0] += ri * ri;
        acc[1] += ri * yi;
#pragma unroll
        for (int j = 0; j < NQ; ++j) acc[2 + j] += qval(j) * yi;
    }
    if (!FSAI) write_partials<T, NV>(acc, q + 2, part_out);
}

// ---------------------------------------------------------------------------
// FSAI application y = (Z'Z) res in two launches (the preconditioner
// P = Z'Z, fsai.cpp), each a sparse product along the CSR of A:
//   k_fsai_lo   h = Z res:  h_i = Z_ii res_i + sum over the lower part of row i
//   k_fsai_up   y = Z'h:    y_i = Z_ii h_i + sum over the upper part of row i,
//               then the partial sums the next KA folds: res'res (not at
//               INIT), res'y and Q'y (the projection of M = (I-QQ')P(I-QQ')
//               happens there, through c1 = Q'y)
// Rows [0, n_wave), the high-degree ones, are summed by a wavefront each,
// the others by one lane each, in a fixed order.  Both are no-ops once the
// iteration has stopped (launch number sq, see stopped()).
// ---------------------------------------------------------------------------
template <typename T, bool UPPER>
__device__ __forceinline__ T fsai_row_lane(const FsaiView<T> &f, int i, const T *__restrict__ x) {
    const int e0 = UPPER ? f.mid[i] : f.rowptr[i];
    const int e1 = UPPER ? f.rowptr[i + 1] : f.mid[i];
    T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
    int e = e0;
    for (; e + 4 <= e1; e += 4) {
        const int c0 = f.col[e], c1 = f.col[e + 1], c2 = f.col[e + 2], c3 = f.col[e + 3];
        const T z0 = f.zv[e], z1 = f.zv[e + 1], z2 = f.zv[e + 2], z3 = f.zv[e + 3];
        a0 += z0 * x[c0];
        a1 += z1 * x[c1];
        a2 += z2 * x[c2];
        a3 += z3 * x[c3];
    }
    for (; e < e1; ++e) a0 += f.zv[e] * x[f.col[e]];
    return (a0 + a1) + (a2 + a3);
}

template <typename T, bool UPPER>
__device__ __forceinline__ T fsai_row_wave(const FsaiView<T> &f, int i, const T *__restrict__ x) {
    const int e0 = UPPER ? f.mid[i] : f.rowptr[i];
    const int e1 = UPPER ? f.rowptr[i + 1] : f.mid[i];
    T a = T(0);
    for (int e = e0 + lane_id(); e < e1; e += kWave) a += f.zv[e] * x[f.col[e]];
    return wave_sum(a);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fsai_lo(FsaiView<T> f, const T *__restrict__ x, T *__restrict__ h,
                                                    const PcgState<T> *st, int sq) {
    if (stopped(st, sq)) return;
    const int waves = gridDim.x * kWavesPerBlock;
    for (int i = blockIdx.x * kWavesPerBlock + wave_id(); i < f.n_wave; i += waves) {
        const T s = fsai_row_wave<T, false>(f, i, x);
        if (lane_id() == 0) h[i] = f.zd[i] * x[i] + s;
    }
    for (int i = f.n_wave + blockIdx.x * blockDim.x + threadIdx.x; i < f.n; i += gridDim.x * blockDim.x)
        h[i] = f.zd[i] * x[i] + fsai_row_lane<T, false>(f, i, x);
}

template <typename T, int NV, bool INIT>
__global__ __launch_bounds__(kBlock) void k_fsai_up(FsaiView<T> f, const T *__restrict__ h, T *__restrict__ y,
                                                    const T *__restrict__ res, const T *__restrict__ Q, int ldq, int q,
                                                    T *__restrict__ part_out, const PcgState<T> *st, int sq) {
    if (stopped(st, sq)) return;
    constexpr int OFF = INIT ? 1 : 2;  // [res'res,] res'y, Q'y
    T acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = T(0);
    auto row_done = [&](int i, T yi) {
        y[i] = yi;
        const T ri = res[i];
        if (!INIT) acc[0] += ri * ri;
        acc[OFF - 1] += ri * yi;
        const T *qi = Q + (size_t)i * ldq;
#pragma unroll
        for (int j = 0; j < NV - OFF; ++j)
            if (j < q) acc[OFF + j] += qi[j] * yi;
    };
    const int waves = gridDim.x * kWavesPerBlock;
    for (int i = blockIdx.x * kWavesPerBlock + wave_id(); i < f.n_wave; i += waves) {
        const T s = fsai_row_wave<T, true>(f, i, h);
        if (lane_id() == 0) row_done(i, f.zd[i] * h[i] + s);
    }
    for (int i = f.n_wave + blockIdx.x * blockDim.x + threadIdx.x; i < f.n; i += gridDim.x * blockDim.x)
        row_done(i, f.zd[i] * h[i] + fsai_row_lane<T, true>(f, i, h));
    write_partials<T, NV>(acc, q + OFF, part_out);
}

// ===========================================================================
// Pipelined form: one launch per iteration (projectors of up to kPipeQ
// columns).  The recurrences of Ghysels and Vanroose's pipelined CG carry
// A u and the preconditioned products along, so each launch needs only the
// inner products of the launch before it:
//   u = M res,  w = A u,  m = M w,  n = A m,  s = A p,  q = M s,  z = A q
//   beta = gamma / gamma_prev,  alpha = gamma / (delta - beta gamma / alpha_prev)
//   z = n + beta z,  q = m + beta q,  s = w + beta s,  p = u + beta p
//   t += alpha p,  res -= alpha s,  u -= alpha q,  w -= alpha z
// with gamma = res'u and delta = w'u.  The projections stay exact: w, s and
// z are kept without their Q components (w~ = (G - theta I) u etc.), whose
// coefficients follow from folded inner products: Q'w~ directly, Q's~ by
// its own recurrence, and m = M w = D^{-1}(w~ - Q c_w) - Q c_m with
// c_w = Q'w~, c_m = Q'D^{-1}w~ - K c_w, K = Q'D^{-1}Q.  The product
// n~ = (G - theta I) m gathers only wh = D^{-1} w~ and corrects with the
// rows of G Q and G D^{-1} Q, formed once per solve.
constexpr int kPP = 16;  // init1 / init2 partials: q + 1 values
// init3 / iteration partials for projectors of up to QM columns (QM = 6 or
// kPipeQ; narrow projectors fold and reduce half as many values), layout
// [0] res'u  [1] w~'u  [2] res'res  [3 + j] Q'w~  [3 + QM + j] Q'wh
template <int QM>
struct PLay {
    static constexpr int CW = 3, CD = 3 + QM, NV = 3 + 2 * QM;
    static constexpr int N = NV <= 16 ? 16 : 32;  // row stride (a power of two)
};
constexpr int kNarrowQ = 6;
constexpr int kMidQ = 10;

// init1: res = -r, t = 0, qq rows [Q_i | dinv_i Q_i]; partials r'r, -Q'r;
// and this workgroup's share of K = Q'D^{-1}Q on the matrix cores (each
// wavefront accumulates 4-row chunks into one 16x16 tile).
// Inc: only the last column u of Q is new since the previous setup on this
// work area (G Q, G D^{-1} Q and K of the others are still in place): qq
// receives the two vectors u and D^{-1}u instead, and the partials also
// carry Q'D^{-1}u, the new row of K.
constexpr int kIncK = 1 + kPipeQ;   // where Q'D^{-1}u starts in the Inc partials
constexpr int kIncNV = 32;          // Inc partial row: [r'r, -Q'r (kPipeQ), Q'D^{-1}u (kPipeQ)]
template <typename T, bool Inc>
__global__ __launch_bounds__(kBlock) void k_pp_init1(int n, const double *__restrict__ r, T *__restrict__ res,
                                                     T *__restrict__ t, const T *__restrict__ Q, int ldq, int q,
                                                     const T *__restrict__ dinv, T *__restrict__ qq,
                                                     T *__restrict__ qcm, T *__restrict__ part_out,
                                                     T *__restrict__ kpart, PcgState<T> *st) {
    if (leader()) {
        st->stop_seq = 0;
        st->iters = 0;
        st->breakdown = 0;
    }
    const int q2 = 2 * q;
    constexpr int NP = Inc ? kIncNV : kPP;
    T acc[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) acc[j] = T(0);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const T ri = (T)r[i];
        const T di = dinv[i];
        res[i] = -ri;
        t[i] = T(0);
        acc[0] += ri * ri;
        if constexpr (Inc) {
            const T ui = Q[(size_t)i * ldq + (q - 1)];
            const T dui = di * ui;
            qq[i] = ui;
            qq[(size_t)n + i] = dui;
            qcm[(size_t)(q - 1) * col_ld(n) + i] = ui;
#pragma unroll
            for (int j = 0; j < kPipeQ; ++j)
                if (j < q) {
                    const T qij = Q[(size_t)i * ldq + j];
                    acc[1 + j] -= qij * ri;
                    acc[kIncK + j] += qij * dui;
                }
        } else {
#pragma unroll
            for (int j = 0; j < kPipeQ; ++j)
                if (j < q) {
                    const T qij = Q[(size_t)i * ldq + j];
                    acc[1 + j] -= qij * ri;
                    qq[(size_t)i * q2 + j] = qij;
                    qq[(size_t)i * q2 + q + j] = di * qij;
                    qcm[(size_t)j * col_ld(n) + i] = qij;
                }
        }
    }
    write_partials<T, NP>(acc, Inc ? kIncK + q : q + 1, part_out);
    if constexpr (Inc) return;

    using V4 = typename Mfma<T>::v4;
    V4 kc = V4{T(0), T(0), T(0), T(0)};
    const int lane = lane_id(), mi = lane & 15, kk = lane >> 4;
    const int step = gridDim.x * kWavesPerBlock * 4;
    for (int k0 = (blockIdx.x * kWavesPerBlock + wave_id()) * 4; k0 < n; k0 += step) {
        const int row = k0 + kk;
        T a = T(0), b = T(0);
        if (row < n && mi < q) {
            a = Q[(size_t)row * ldq + mi];
            b = dinv[row] * a;
        }
        kc = Mfma<T>::mac(a, b, kc);
    }
    __shared__ T ks[256];
    for (int w = 0; w < kWavesPerBlock; ++w) {
        if (wave_id() == w)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int at = Mfma<T>::row(lane, e) * 16 + mi;
                ks[at] = (w == 0 ? T(0) : ks[at]) + kc[e];
            }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < 256; e += blockDim.x) kpart[(size_t)blockIdx.x * 256 + e] = ks[e];
}

// init2: K = sum of the Gram tiles (one wavefront per entry); r0 = ||r||,
// c0 = -Q'r, stop if r = 0; res -= Q c0; yh = D^{-1} res;  partials res'yh, Q'yh
template <typename T, bool Inc>
__global__ __launch_bounds__(kBlock) void k_pp_init2(int n, T *__restrict__ res, T *__restrict__ yh,
                                                     const T *__restrict__ dinv, const T *__restrict__ Qc, int q, const T *__restrict__ part_in, int nb_in,
                                                     T *__restrict__ part_out, const T *__restrict__ kpart, int nk,
                                                     T *__restrict__ kmat, PcgState<T> *st) {
    constexpr int NP = Inc ? kIncNV : kPP;
    __shared__ T tot[NP];
    fold_partials<T, NP>(part_in, nb_in, Inc ? kIncK + q : q + 1, tot);
    if constexpr (Inc) {
        // the new row and column of K; the rest is unchanged
        if (blockIdx.x == 0 && threadIdx.x < q) {
            const T v = tot[kIncK + threadIdx.x];
            kmat[threadIdx.x * 16 + (q - 1)] = v;
            kmat[(q - 1) * 16 + threadIdx.x] = v;
        }
    } else {
        const int lane = lane_id();
        for (int e = blockIdx.x * kWavesPerBlock + wave_id(); e < 256; e += gridDim.x * kWavesPerBlock) {
            T sum = T(0);
            for (int b = lane; b < nk; b += kWave) sum += kpart[(size_t)b * 256 + e];
            sum = wave_sum(sum);
            if (lane == 0) kmat[e] = sum;
        }
    }
    const T r0 = sqrt(tot[0]);
    if (leader()) {
        st->r0 = r0;
        if (!(r0 > T(0))) st->stop_seq = 2;
    }
    if (!(r0 > T(0))) return;
    T acc[kPP];
#pragma unroll
    for (int j = 0; j < kPP; ++j) acc[j] = T(0);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        T qv[kPipeQ];
        T proj = T(0);
#pragma unroll
        for (int j = 0; j < kPipeQ; ++j) {
            qv[j] = j < q ? Qc[(size_t)j * col_ld(n) + i] : T(0);
            proj += qv[j] * tot[1 + j];
        }
        const T ri = res[i] - proj;
        res[i] = ri;
        const T yi = dinv[i] * ri;
        yh[i] = yi;
        acc[0] += ri * yi;
#pragma unroll
        for (int j = 0; j < kPipeQ; ++j) acc[1 + j] += qv[j] * yi;
    }
    write_partials<T, kPP>(acc, q + 1, part_out);
}

// Inc setup: the two new columns of G [Q | D^{-1}Q] (row-major, 2q wide),
// G u and G D^{-1}u, from the vectors u and D^{-1}u that init1 left in ud.
template <typename T, bool Wt>
__global__ __launch_bounds__(kBlock) void k_pp_gq2(Graph g, Weights<T> w, const T *__restrict__ ud, int q,
                                                   T *__restrict__ gqc) {
    const size_t ldc = col_ld(g.n);
    for_each_row<T, Wt, false>(g, w, ud, [&](int i, T, T yi, T) { gqc[(size_t)(q - 1) * ldc + i] = yi; });
    for_each_row<T, Wt, false>(g, w, ud + g.n, [&](int i, T, T yi, T) { gqc[(size_t)(2 * q - 1) * ldc + i] = yi; });
}

// out (column-major, ld n) = in (n x wd, row-major): 64-row tiles through LDS,
// both sides coalesced
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rm_to_cm(int n, int wd, const T *__restrict__ in, T *__restrict__ out) {
    __shared__ T tile[kWave * 2 * kPipeQ];
    for (int r0 = blockIdx.x * kWave; r0 < n; r0 += gridDim.x * kWave) {
        const int rows = min(kWave, n - r0);
        const int cnt = rows * wd;
        const T *src = in + (size_t)r0 * wd;
        for (int e = threadIdx.x; e < cnt; e += blockDim.x) tile[e] = src[e];
        __syncthreads();
        for (int e = threadIdx.x; e < kWave * wd; e += blockDim.x) {
            const int j = e / kWave, r = e % kWave;
            if (r < rows) out[(size_t)j * col_ld(n) + r0 + r] = tile[r * wd + j];
        }
        __syncthreads();
    }
}

// init3: c_y = Q'yh;  u = yh - Q c_y;  w~ = (G - theta I) u, gathered as
// (G - theta I) yh - GQ c_y + theta Q c_y;  wh = D^{-1} w~;  iteration partials
template <typename T, int QM>
struct P3Row {
    T q[QM], gq[QM];
    T dinv, res;
};

template <typename T, bool Wt, int QM>
__global__ __launch_bounds__(kBlock) void k_pp_init3(Graph g, Weights<T> w, const double *__restrict__ theta,
                                                     const T *__restrict__ Qc, const T *__restrict__ gqc,
                                                     int q, const T *__restrict__ dinv, const T *__restrict__ res,
                                                     const T *__restrict__ yh, T *__restrict__ u, T *__restrict__ wv,
                                                     T *__restrict__ wh, const T *__restrict__ part_in, int nb_in,
                                                     T *__restrict__ part_out, const PcgState<T> *st, int sq) {
    const int stop_v = st->stop_seq;
    const T th = (T)theta[0];
    __shared__ T tot[kPP];
    fold_partials<T, kPP>(part_in, nb_in, q + 1, tot);
    if (stop_v != 0 && stop_v <= sq) return;
    const size_t ldc = col_ld(g.n);
    using L = PLay<QM>;
    T acc[L::N];
#pragma unroll
    for (int j = 0; j < L::N; ++j) acc[j] = T(0);
    auto pre = [&](int i) {
        P3Row<T, QM> d;
#pragma unroll
        for (int j = 0; j < QM; ++j) {
            d.q[j] = j < q ? Qc[(size_t)j * ldc + i] : T(0);
            d.gq[j] = j < q ? gqc[(size_t)j * ldc + i] : T(0);
        }
        d.dinv = dinv[i];
        d.res = res[i];
        return d;
    };
    for_each_row_pre<T, Wt, false>(g, w, yh, pre, [&](int i, T yi, T gyi, T, const P3Row<T, QM> &d) {
        T qc = T(0), gc = T(0);
#pragma unroll
        for (int j = 0; j < QM; ++j) {
            qc += d.q[j] * tot[1 + j];
            gc += d.gq[j] * tot[1 + j];
        }
        const T ui = yi - qc;
        const T wi = ((gyi - th * yi) - gc) + th * qc;
        const T hi = d.dinv * wi;
        u[i] = ui;
        wv[i] = wi;
        wh[i] = hi;
        acc[0] += d.res * ui;
        acc[1] += wi * ui;
        acc[2] += d.res * d.res;
#pragma unroll
        for (int j = 0; j < QM; ++j) {
            acc[L::CW + j] += d.q[j] * wi;
            acc[L::CD + j] += d.q[j] * hi;
        }
    });
    write_partials<T, L::N>(acc, L::NV, part_out);
}

// Iteration i (launch 3 + i): fold gamma, delta, ||res||^2, c_w, c_dw;
// stop test (i > 0); beta, alpha or breakdown; then the row updates above.
template <typename T, int QM>
struct PIRow {
    T q[QM], gq[QM], gdq[QM];
    T dinv, t, res, u, w, p, s, qv, z;
};

template <typename T, bool Wt, int QM>
__global__ __launch_bounds__(kBlock) void k_pp_iter(
    // what the fold and the scalar step read first leads the list, so that it
    // arrives in preloaded SGPRs rather than after a kernel-argument load
    const T *__restrict__ part_in, PcgState<T> *st, int nb_in, int sq, int it, int q,
    const T *__restrict__ kmat, const double *__restrict__ theta, T rtol,
    Graph g, Weights<T> w, const T *__restrict__ Qc,
    const T *__restrict__ gqc, const T *__restrict__ dinv, T *__restrict__ t,
    T *__restrict__ res, T *__restrict__ u, T *__restrict__ wv, const T *__restrict__ wh_in,
    T *__restrict__ wh_out, T *__restrict__ p, T *__restrict__ s, T *__restrict__ qv, T *__restrict__ z,
    T *__restrict__ part_out) {
    // scalars and the small operands first, so that their latency overlaps the fold
    const int stop_v = st->stop_seq;
    const T th = (T)theta[0];
    const T r0 = st->r0;
    const T gam_prev = st->gam[(it + 1) & 1], alp_prev = st->alp[(it + 1) & 1];
    const int tj = threadIdx.x;
    T krow[QM];
    T cs_prev = T(0);
    if (tj < q) {
#pragma unroll
        for (int a = 0; a < QM; ++a) krow[a] = a < q ? kmat[tj * 16 + a] : T(0);
        if (it > 0) cs_prev = st->cs[(it + 1) & 1][tj];
    }
    using L = PLay<QM>;
    __shared__ T tot[L::N];
    __shared__ T coef[3][QM];  // c_w, c_s, c_m
    fold_partials<T, L::N>(part_in, nb_in, L::NV, tot);
    if (stop_v != 0 && stop_v <= sq) return;
    const T gam = tot[0], dlt = tot[1], rr = tot[2];
    if (it > 0 && sqrt(rr) <= rtol * r0) {
        if (leader()) st->stop_seq = sq + 1;
        return;
    }
    const T beta = it > 0 ? gam / gam_prev : T(0);
    const T den = it > 0 ? dlt - beta * gam / alp_prev : dlt;  // p'A p
    if (!(den > T(0))) {  // the projected operator is indefinite along p
        if (leader()) {
            st->stop_seq = sq + 1;
            st->breakdown = it + 1;
            st->total += 1;  // the product of the failed step counts
        }
        // no step was taken before the breakdown: return M(-r), which u holds
        if (it == 0)
            for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += gridDim.x * blockDim.x) t[i] = u[i];
        return;
    }
    const T alpha = gam / den;
    if (tj < QM) {
        T cw = T(0), cs = T(0), cm = T(0);
        if (tj < q) {
            cw = tot[L::CW + tj];
            cs = cw + beta * cs_prev;
            T kc = T(0);
#pragma unroll
            for (int a = 0; a < QM; ++a) kc += krow[a] * tot[L::CW + a];
            cm = tot[L::CD + tj] - kc;
            if (blockIdx.x == 0) st->cs[it & 1][tj] = cs;
        }
        coef[0][tj] = cw;
        coef[1][tj] = cs;
        coef[2][tj] = cm;
    }
    if (leader()) {
        st->gam[it & 1] = gam;
        st->alp[it & 1] = alpha;
        st->iters = it + 1;
        st->total += 1;
    }
    __syncthreads();
    const size_t ldc = col_ld(g.n);
    const bool first = it == 0;
    T acc[L::N];
#pragma unroll
    for (int j = 0; j < L::N; ++j) acc[j] = T(0);
    auto pre = [&](int i) {
        PIRow<T, QM> d;
#pragma unroll
        for (int j = 0; j < QM; ++j) {
            d.q[j] = j < q ? Qc[(size_t)j * ldc + i] : T(0);
            d.gq[j] = j < q ? gqc[(size_t)j * ldc + i] : T(0);
            d.gdq[j] = j < q ? gqc[(size_t)(q + j) * ldc + i] : T(0);
        }
        d.dinv = dinv[i];
        d.t = t[i];
        d.res = res[i];
        d.u = u[i];
        d.w = wv[i];
        d.p = first ? T(0) : p[i];
        d.s = first ? T(0) : s[i];
        d.qv = first ? T(0) : qv[i];
        d.z = first ? T(0) : z[i];
        return d;
    };
    for_each_row_pre<T, Wt, false>(g, w, wh_in, pre, [&](int i, T hi, T ghi, T, const PIRow<T, QM> &d) {
        T qcw = T(0), qcs = T(0), qcm = T(0), gcw = T(0), gcm = T(0);
#pragma unroll
        for (int j = 0; j < QM; ++j) {
            qcw += d.q[j] * coef[0][j];
            qcs += d.q[j] * coef[1][j];
            qcm += d.q[j] * coef[2][j];
            gcw += d.gdq[j] * coef[0][j];
            gcm += d.gq[j] * coef[2][j];
        }
        const T dqcw = d.dinv * qcw;
        const T mi = (hi - dqcw) - qcm;                                         // m = M w
        const T ni = ((ghi - th * hi) - (gcw - th * dqcw)) - (gcm - th * qcm);  // (G - theta I) m
        const T zi = first ? ni : ni + beta * d.z;
        const T qi = first ? mi : mi + beta * d.qv;
        const T si = first ? d.w : d.w + beta * d.s;
        const T pi = first ? d.u : d.u + beta * d.p;
        const T tn = d.t + alpha * pi;
        const T rn = d.res - alpha * (si - qcs);
        const T un = d.u - alpha * qi;
        const T wn = d.w - alpha * zi;
        const T hn = d.dinv * wn;
        t[i] = tn;
        res[i] = rn;
        u[i] = un;
        wv[i] = wn;
        wh_out[i] = hn;
        p[i] = pi;
        s[i] = si;
        qv[i] = qi;
        z[i] = zi;
        acc[0] += rn * un;
        acc[1] += wn * un;
        acc[2] += rn * rn;
#pragma unroll
        for (int j = 0; j < QM; ++j) {
            acc[L::CW + j] += d.q[j] * wn;
            acc[L::CD + j] += d.q[j] * hn;
        }
    });
    write_partials<T, L::N>(acc, L::NV, part_out);
}

inline int vgrid(int n) {
    int g = (n + kBlock - 1) / kBlock;
    const int cap = pcg_vec_groups();
    return g < 1 ? 1 : (g > cap ? cap : g);
}

// Row grid cap of the one-launch iteration: as many workgroups as its
// register use lets every compute unit hold at once (at most four per unit),
// so that large graphs keep enough waves in flight in a single round.
template <typename T, bool Wt, int QM>
int pp_iter_groups() {
    static const int groups = [] {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pp_iter<T, Wt, QM>, kBlock, 0) != hipSuccess || nb < 1)
            nb = 2;
        return std::min(nb, 4) * device_cu_count();
    }();
    return groups;
}

template <typename T, int NV>
void enqueue_nv(const lap_plan &P, const double *theta, const T *Q, int ldq, int q, const double *r, T *t,
                PcgWork<T> &w, int itmax, double rtol, hipStream_t s, bool fsai = false) {
    const int n = P.n;
    const int gv = vgrid(n);
    const int gr = row_grid(P.g, pcg_vec_groups());
    const FsaiView<T> fz = fsai ? P.fsai<T>() : FsaiView<T>{};
    LAP_REQUIRE(!fsai || P.fsai_ready, LAP_EDEVICE, "FSAI factor not built");
    const int gz = pcg_vec_groups();  // grid of the FSAI launches
    T *hbuf = w.u.get();              // Z res (the pipelined form's u is free here)
    LAP_REQUIRE(w.gq.n >= (size_t)n * ldq, LAP_EDEVICE, "PCG work area too small for the projector");
    T *pa = w.part.get();
    T *pb = pa + (size_t)pcg_max_groups() * 64;
    PcgState<T> *st = w.st.get();
    const T *dinv = P.dinv<T>();
    const T tol = (T)rtol;
    T *gq = w.gq.get();
    if (q > 0) spmm<T>(P, q, Q, ldq, gq, ldq, nullptr, s);
    hipLaunchKernelGGL((k_pcg_init1<T, NV>), dim3(gv), dim3(kBlock), 0, s, n, r, w.res.get(), t, Q, ldq, q, pa, st);
    int nb_y = gv;  // partial rows the next KA folds
    if (fsai) {
        hipLaunchKernelGGL((k_pcg_init2<T, NV, true>), dim3(gv), dim3(kBlock), 0, s, n, w.res.get(), w.y.get(), dinv,
                           Q, ldq, q, pa, gv, pb, st);
        hipLaunchKernelGGL((k_fsai_lo<T>), dim3(gz), dim3(kBlock), 0, s, fz, w.res.get(), hbuf, st, 2);
        hipLaunchKernelGGL((k_fsai_up<T, NV, true>), dim3(gz), dim3(kBlock), 0, s, fz, hbuf, w.y.get(), w.res.get(),
                           Q, ldq, q, pb, st, 2);
        nb_y = gz;
    } else {
        hipLaunchKernelGGL((k_pcg_init2<T, NV, false>), dim3(gv), dim3(kBlock), 0, s, n, w.res.get(), w.y.get(), dinv,
                           Q, ldq, q, pa, gv, pb, st);
    }
    for (int it = 1; it <= itmax; ++it) {
        const int sq = 2 * it;
        const int gv_in = nb_y;
        if (it == 1) {
            if (P.weighted)
                hipLaunchKernelGGL((k_pcg_ps<T, NV, true, true>), dim3(gr), dim3(kBlock), 0, s, P.g, P.weights<T>(),
                                   theta, w.y.get(), w.p.get(), w.s.get(), Q, gq, ldq, q, pb, gv_in, pa, st, sq, it, tol);
            else
                hipLaunchKernelGGL((k_pcg_ps<T, NV, false, true>), dim3(gr), dim3(kBlock), 0, s, P.g, P.weights<T>(),
                                   theta, w.y.get(), w.p.get(), w.s.get(), Q, gq, ldq, q, pb, gv_in, pa, st, sq, it, tol);
        } else {
            if (P.weighted)
                hipLaunchKernelGGL((k_pcg_ps<T, NV, true, false>), dim3(gr), dim3(kBlock), 0, s, P.g, P.weights<T>(),
                                   theta, w.y.get(), w.p.get(), w.s.get(), Q, gq, ldq, q, pb, gv_in, pa, st, sq, it, tol);
            else
                hipLaunchKernelGGL((k_pcg_ps<T, NV, false, false>), dim3(gr), dim3(kBlock), 0, s, P.g,
                                   P.weights<T>(), theta, w.y.get(), w.p.get(), w.s.get(), Q, gq, ldq, q, pb, gv_in,
                                   pa, st, sq, it, tol);
        }
        if (fsai) {
            hipLaunchKernelGGL((k_pcg_update<T, NV, true>), dim3(gv), dim3(kBlock), 0, s, n, t, w.res.get(),
                               w.p.get(), w.s.get(), w.y.get(), dinv, Q, ldq, q, pa, gr, pb, st, sq + 1, it);
            // launches sq + 2: no-ops after a stop decided by KA or KB of this iteration
            hipLaunchKernelGGL((k_fsai_lo<T>), dim3(gz), dim3(kBlock), 0, s, fz, w.res.get(), hbuf, st, sq + 2);
            hipLaunchKernelGGL((k_fsai_up<T, NV, false>), dim3(gz), dim3(kBlock), 0, s, fz, hbuf, w.y.get(),
                               w.res.get(), Q, ldq, q, pb, st, sq + 2);
        } else {
            hipLaunchKernelGGL((k_pcg_update<T, NV, false>), dim3(gv), dim3(kBlock), 0, s, n, t, w.res.get(),
                               w.p.get(), w.s.get(), w.y.get(), dinv, Q, ldq, q, pa, gr, pb, st, sq + 1, it);
        }
    }
    LAP_HIP(hipGetLastError());
}

template <typename T, int QM>
void enqueue_pipelined_qm(const lap_plan &P, const double *theta, const T *Q, int ldq, int q, const double *r, T *t,
                          PcgWork<T> &w, int itmax, double rtol, bool inc, hipStream_t s) {
    const int n = P.n;
    const int gv = vgrid(n);
    const int gr = row_grid(P.g, P.weighted ? pp_iter_groups<T, true, QM>() : pp_iter_groups<T, false, QM>());
    const int q2 = 2 * q;
    LAP_REQUIRE(w.qq.n >= (size_t)n * q2 && w.qcm.n >= col_ld(n) * q && w.gqcm.n >= col_ld(n) * q2 &&
                    w.kpart.n >= (size_t)gv * 256,
                LAP_EDEVICE, "PCG work area too small for the projector");
    T *pa = w.part.get();
    T *pb = pa + (size_t)pcg_max_groups() * 64;
    PcgState<T> *st = w.st.get();
    const T *dinv = P.dinv<T>();
    const T tol = (T)rtol;
    T *wh0 = w.wh.get(), *wh1 = wh0 + n;
    // the per-row operands of init3 and the iterations, column-major (one
    // coalesced load per column): Q, then G Q and G D^{-1}Q
    T *qc = w.qcm.get(), *gqc = w.gqcm.get();
    if (inc) {
        hipLaunchKernelGGL((k_pp_init1<T, true>), dim3(gv), dim3(kBlock), 0, s, n, r, w.res.get(), t, Q, ldq, q,
                           dinv, w.qq.get(), qc, pa, w.kpart.get(), st);
        const int grow = row_grid(P.g, 1 << 20);
        if (P.weighted)
            hipLaunchKernelGGL((k_pp_gq2<T, true>), dim3(grow), dim3(kBlock), 0, s, P.g, P.weights<T>(), w.qq.get(),
                               q, gqc);
        else
            hipLaunchKernelGGL((k_pp_gq2<T, false>), dim3(grow), dim3(kBlock), 0, s, P.g, P.weights<T>(), w.qq.get(),
                               q, gqc);
        hipLaunchKernelGGL((k_pp_init2<T, true>), dim3(gv), dim3(kBlock), 0, s, n, w.res.get(), wh1, dinv, qc, q, pa,
                           gv, pb, w.kpart.get(), gv, w.kmat.get(), st);
    } else {
        hipLaunchKernelGGL((k_pp_init1<T, false>), dim3(gv), dim3(kBlock), 0, s, n, r, w.res.get(), t, Q, ldq, q,
                           dinv, w.qq.get(), qc, pa, w.kpart.get(), st);
        if (q > 0) {
            spmm<T>(P, q2, w.qq.get(), q2, w.gqq.get(), q2, nullptr, s);
            const int tg = std::min((n + kWave - 1) / kWave, 8 * device_cu_count());
            hipLaunchKernelGGL((k_rm_to_cm<T>), dim3(tg), dim3(kBlock), 0, s, n, q2, w.gqq.get(), gqc);
        }
        hipLaunchKernelGGL((k_pp_init2<T, false>), dim3(gv), dim3(kBlock), 0, s, n, w.res.get(), wh1, dinv, qc, q,
                           pa, gv, pb, w.kpart.get(), gv, w.kmat.get(), st);
    }
    if (P.weighted)
        hipLaunchKernelGGL((k_pp_init3<T, true, QM>), dim3(gr), dim3(kBlock), 0, s, P.g, P.weights<T>(), theta, qc,
                           gqc, q, dinv, w.res.get(), wh1, w.u.get(), w.w.get(), wh0, pb, gv, pa, st, 2);
    else
        hipLaunchKernelGGL((k_pp_init3<T, false, QM>), dim3(gr), dim3(kBlock), 0, s, P.g, P.weights<T>(), theta, qc,
                           gqc, q, dinv, w.res.get(), wh1, w.u.get(), w.w.get(), wh0, pb, gv, pa, st, 2);
    for (int it = 0; it < itmax; ++it) {
        T *pin = (it & 1) ? pb : pa;
        T *pout = (it & 1) ? pa : pb;
        const T *hin = (it & 1) ? wh1 : wh0;
        T *hout = (it & 1) ? wh0 : wh1;
        if (P.weighted)
            hipLaunchKernelGGL((k_pp_iter<T, true, QM>), dim3(gr), dim3(kBlock), 0, s, pin, st, gr, 3 + it, it, q,
                               w.kmat.get(), theta, tol, P.g, P.weights<T>(), qc, gqc, dinv, t, w.res.get(),
                               w.u.get(), w.w.get(), hin, hout, w.p.get(), w.s.get(), w.qv.get(), w.z.get(), pout);
        else
            hipLaunchKernelGGL((k_pp_iter<T, false, QM>), dim3(gr), dim3(kBlock), 0, s, pin, st, gr, 3 + it, it, q,
                               w.kmat.get(), theta, tol, P.g, P.weights<T>(), qc, gqc, dinv, t, w.res.get(),
                               w.u.get(), w.w.get(), hin, hout, w.p.get(), w.s.get(), w.qv.get(), w.z.get(), pout);
    }
    LAP_HIP(hipGetLastError());
}

// Projectors of up to kNarrowQ columns take the narrow instantiation.
template <typename T>
void enqueue_pipelined(const lap_plan &P, const double *theta, const T *Q, int ldq, int q, const double *r, T *t,
                       PcgWork<T> &w, int itmax, double rtol, bool inc, hipStream_t s) {
    if (q <= kNarrowQ) enqueue_pipelined_qm<T, kNarrowQ>(P, theta, Q, ldq, q, r, t, w, itmax, rtol, inc, s);
    else if (q <= kMidQ) enqueue_pipelined_qm<T, kMidQ>(P, theta, Q, ldq, q, r, t, w, itmax, rtol, inc, s);
    else enqueue_pipelined_qm<T, kPipeQ>(P, theta, Q, ldq, q, r, t, w, itmax, rtol, inc, s);
}

// The one-launch form unless the projector is too wide for it (or the
// two-launch form is asked for, which the tests use to cover both).
inline bool use_pipelined(int q) {
    return q <= kPipeQ && std::getenv("LAPEIG_PCG_TWO_LAUNCH") == nullptr;
}

// ---- conversions used by the C ABI entry point
template <typename T>
__global__ void k_pack_q(int n, int q, const double *__restrict__ Qc, const int *__restrict__ map, T *__restrict__ Qr,
                         int ldq) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int dst = map ? map[i] : i;
        for (int j = 0; j < q; ++j) Qr[(size_t)dst * ldq + j] = (T)Qc[(size_t)j * n + i];
    }
}

__global__ void k_gather_col(int n, const double *__restrict__ in, const int *__restrict__ map,
                             double *__restrict__ out) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        out[map ? map[i] : i] = in[i];
}

template <typename T>
__global__ void k_scatter_t(int n, const T *__restrict__ t, const int *__restrict__ iperm, double *__restrict__ out) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x)
        out[iperm ? iperm[p] : p] = (double)t[p];
}

template <typename T>
lap_status pcg_entry_t(lap_plan *P, int b, const double *theta_host, const double *Q, int q, const double *R,
                       double *Tout, int itmax, double rtol, int *iters_out, int flags, hipStream_t s) {
    const int n = P->n;
    const bool plan_order = flags & LAP_ORDER_PLAN;
    const bool fsai = flags & LAP_PCG_FSAI;
    if (fsai) fsai_ensure(P);
    const int *map = plan_order ? nullptr : P->d_perm.get();
    const int *imap = plan_order ? nullptr : P->d_iperm.get();
    const int ldq = q > 0 ? q : 1;
    DevBuf<T> Qr((size_t)n * ldq), t(n);
    DevBuf<double> r(n), th(1);
    PcgWork<T> w;
    w.ensure(n, ldq);
    const int gv = vgrid(n);
    if (q > 0)
        hipLaunchKernelGGL((k_pack_q<T>), dim3(gv), dim3(kBlock), 0, s, n, q, Q, map, Qr.get(), ldq);
    for (int c = 0; c < b; ++c) {
        LAP_HIP(hipMemcpyAsync(th.get(), theta_host + c, sizeof(double), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_gather_col, dim3(gv), dim3(kBlock), 0, s, n, R + (size_t)c * n, map, r.get());
        if (!fsai && use_pipelined(q))
            enqueue_pipelined<T>(*P, th.get(), Qr.get(), ldq, q, r.get(), t.get(), w, itmax, rtol, false, s);
        else if (q <= 14)
            enqueue_nv<T, 16>(*P, th.get(), Qr.get(), ldq, q, r.get(), t.get(), w, itmax, rtol, s, fsai);
        else
            enqueue_nv<T, 64>(*P, th.get(), Qr.get(), ldq, q, r.get(), t.get(), w, itmax, rtol, s, fsai);
        hipLaunchKernelGGL((k_scatter_t<T>), dim3(gv), dim3(kBlock), 0, s, n, t.get(), imap, Tout + (size_t)c * n);
        PcgState<T> hs;
        LAP_HIP(hipMemcpyAsync(&hs, w.st.get(), sizeof(hs), hipMemcpyDeviceToHost, s));
        LAP_HIP(hipStreamSynchronize(s));
        if (iters_out) iters_out[c] = hs.breakdown ? hs.breakdown : hs.iters;
    }
    LAP_HIP(hipGetLastError());
    return LAP_OK;
}

}  // namespace

template <typename T>
void pcg_enqueue(const lap_plan &P, const double *theta_dev, const T *Q, int ldq, int q, const double *r, T *t,
                 PcgWork<T> &w, int itmax, double rtol, hipStream_t s, bool inc, bool fsai, bool classic) {
    LAP_REQUIRE(q >= 0 && q <= kMaxQ, LAP_EUNSUPPORTED, "projector wider than 62 columns");
    if (!fsai && !classic && use_pipelined(q))
        enqueue_pipelined<T>(P, theta_dev, Q, ldq, q, r, t, w, itmax, rtol, inc && q >= 1, s);
    else if (q <= 14)
        enqueue_nv<T, 16>(P, theta_dev, Q, ldq, q, r, t, w, itmax, rtol, s, fsai);
    else
        enqueue_nv<T, 64>(P, theta_dev, Q, ldq, q, r, t, w, itmax, rtol, s, fsai);
}
template void pcg_enqueue<float>(const lap_plan &, const double *, const float *, int, int, const double *, float *,
                                 PcgWork<float> &, int, double, hipStream_t, bool, bool, bool);
template void pcg_enqueue<double>(const lap_plan &, const double *, const double *, int, int, const double *,
                                  double *, PcgWork<double> &, int, double, hipStream_t, bool, bool, bool);

lap_status pcg_entry(lap_plan *P, lap_dtype dt, int b, const double *theta_host, const double *Q, int q,
                     const double *R, double *T, int itmax, double rtol, int *iters_out, int flags, hipStream_t s) {
    LAP_REQUIRE(q >= 0 && q <= kMaxQ, LAP_EUNSUPPORTED, "projector wider than 62 columns");
    if (dt == LAP_F32)
        return pcg_entry_t<float>(P, b, theta_host, Q, q, R, T, itmax, rtol, iters_out, flags, s);
    return pcg_entry_t<double>(P, b, theta_host, Q, q, R, T, itmax, rtol, iters_out, flags, s);
}

}  // namespace lapeig
