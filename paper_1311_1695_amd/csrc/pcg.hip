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
template <typename T, int NV>
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
        const T yi = dinv[i] * ri;
        y[i] = yi;
        acc[0] += ri * yi;
#pragma unroll
        for (int j = 0; j < NV - 1; ++j)
            if (j < q) acc[1 + j] += qi[j] * yi;
    }
    write_partials<T, NV>(acc, q + 1, part_out);
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
    auto pre = [&](int i) {
        PsRow<T, NQ> d;
        d.p = INIT ? T(0) : p[i];
        d.s = INIT ? T(0) : s[i];
        const T *qi = Q + (size_t)i * ldq;
        const T *gi = GQ + (size_t)i * ldq;
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            d.qv[j] = j < q ? qi[j] : T(0);
            d.gq[j] = j < q ? gi[j] : T(0);
        }
        return d;
    };
    for_each_row_pre<T, Wt, false>(g, w, y, pre, [&](int i, T yi, T gyi, T, const PsRow<T, NQ> &d) {
        T qc = T(0), gc = T(0);
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            qc += d.qv[j] * tot[OFF + j];
            gc += d.gq[j] * tot[OFF + j];
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
            if (j < NQ) acc[1 + j] += d.qv[j] * si;
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

template <typename T, int NV>
__global__ __launch_bounds__(kBlock) void k_pcg_update(int n, T *__restrict__ t, T *__restrict__ res,
                                                       const T *__restrict__ p, const T *__restrict__ s,
                                                       T *__restrict__ y, const T *__restrict__ dinv,
                                                       const T *__restrict__ Q, int ldq, int q,
                                                       const T *__restrict__ part_in, int nb_in,
                                                       T *__restrict__ part_out, PcgState<T> *st, int sq, int it) {
    constexpr int NQ = NV - 2;
    auto load = [&](int i) {
        UpRow<T, NQ> d;
        d.t = t[i];
        d.p = p[i];
        d.res = res[i];
        d.s = s[i];
        d.dinv = dinv[i];
        const T *qi = Q + (size_t)i * ldq;
#pragma unroll
        for (int j = 0; j < NQ; ++j) d.qv[j] = j < q ? qi[j] : T(0);
        return d;
    };
    // the first row's operands and the scalars are requested before the fold
    const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    const int stop_v = st->stop_seq;
    const T rho = st->rho[(it - 1) & 1];
    UpRow<T, NQ> d0;
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
        const UpRow<T, NQ> d = i == i0 ? d0 : load(i);
        T proj = T(0);
#pragma unroll
        for (int j = 0; j < NQ; ++j) proj += d.qv[j] * tot[1 + j];
        t[i] = d.t + alpha * d.p;
        const T ri = d.res - alpha * (d.s - proj);
        res[i] = ri;
        const T yi = d.dinv * ri;
        y[i] = yi;
        acc[0] += ri * ri;
        acc[1] += ri * yi;
#pragma unroll
        for (int j = 0; j < NQ; ++j) acc[2 + j] += d.qv[j] * yi;
    }
    write_partials<T, NV>(acc, q + 2, part_out);
}

inline int vgrid(int n) {
    int g = (n + kBlock - 1) / kBlock;
    const int cap = pcg_max_groups();
    return g < 1 ? 1 : (g > cap ? cap : g);
}

template <typename T, int NV>
void enqueue_nv(const lap_plan &P, const double *theta, const T *Q, int ldq, int q, const double *r, T *t,
                PcgWork<T> &w, int itmax, double rtol, hipStream_t s) {
    const int n = P.n;
    const int gv = vgrid(n);
    const int gr = row_grid(P.g, pcg_max_groups());
    LAP_REQUIRE(w.gq.n >= (size_t)n * ldq, LAP_EDEVICE, "PCG work area too small for the projector");
    T *pa = w.part.get();
    T *pb = pa + (size_t)pcg_max_groups() * 64;
    PcgState<T> *st = w.st.get();
    const T *dinv = P.dinv<T>();
    const T tol = (T)rtol;
    T *gq = w.gq.get();
    if (q > 0) spmm<T>(P, q, Q, ldq, gq, ldq, nullptr, s);
    hipLaunchKernelGGL((k_pcg_init1<T, NV>), dim3(gv), dim3(kBlock), 0, s, n, r, w.res.get(), t, Q, ldq, q, pa, st);
    hipLaunchKernelGGL((k_pcg_init2<T, NV>), dim3(gv), dim3(kBlock), 0, s, n, w.res.get(), w.y.get(), dinv, Q, ldq,
                       q, pa, gv, pb, st);
    for (int it = 1; it <= itmax; ++it) {
        const int sq = 2 * it;
        if (it == 1) {
            if (P.weighted)
                hipLaunchKernelGGL((k_pcg_ps<T, NV, true, true>), dim3(gr), dim3(kBlock), 0, s, P.g, P.weights<T>(),
                                   theta, w.y.get(), w.p.get(), w.s.get(), Q, gq, ldq, q, pb, gv, pa, st, sq, it, tol);
            else
                hipLaunchKernelGGL((k_pcg_ps<T, NV, false, true>), dim3(gr), dim3(kBlock), 0, s, P.g, P.weights<T>(),
                                   theta, w.y.get(), w.p.get(), w.s.get(), Q, gq, ldq, q, pb, gv, pa, st, sq, it, tol);
        } else {
            if (P.weighted)
                hipLaunchKernelGGL((k_pcg_ps<T, NV, true, false>), dim3(gr), dim3(kBlock), 0, s, P.g, P.weights<T>(),
                                   theta, w.y.get(), w.p.get(), w.s.get(), Q, gq, ldq, q, pb, gv, pa, st, sq, it, tol);
            else
                hipLaunchKernelGGL((k_pcg_ps<T, NV, false, false>), dim3(gr), dim3(kBlock), 0, s, P.g,
                                   P.weights<T>(), theta, w.y.get(), w.p.get(), w.s.get(), Q, gq, ldq, q, pb, gv, pa,
                                   st, sq, it, tol);
        }
        hipLaunchKernelGGL((k_pcg_update<T, NV>), dim3(gv), dim3(kBlock), 0, s, n, t, w.res.get(), w.p.get(),
                           w.s.get(), w.y.get(), dinv, Q, ldq, q, pa, gr, pb, st, sq + 1, it);
    }
    LAP_HIP(hipGetLastError());
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
        if (q <= 14)
            enqueue_nv<T, 16>(*P, th.get(), Qr.get(), ldq, q, r.get(), t.get(), w, itmax, rtol, s);
        else
            enqueue_nv<T, 64>(*P, th.get(), Qr.get(), ldq, q, r.get(), t.get(), w, itmax, rtol, s);
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
                 PcgWork<T> &w, int itmax, double rtol, hipStream_t s) {
    LAP_REQUIRE(q >= 0 && q <= kMaxQ, LAP_EUNSUPPORTED, "projector wider than 62 columns");
    if (q <= 14)
        enqueue_nv<T, 16>(P, theta_dev, Q, ldq, q, r, t, w, itmax, rtol, s);
    else
        enqueue_nv<T, 64>(P, theta_dev, Q, ldq, q, r, t, w, itmax, rtol, s);
}
template void pcg_enqueue<float>(const lap_plan &, const double *, const float *, int, int, const double *, float *,
                                 PcgWork<float> &, int, double, hipStream_t);
template void pcg_enqueue<double>(const lap_plan &, const double *, const double *, int, int, const double *,
                                  double *, PcgWork<double> &, int, double, hipStream_t);

lap_status pcg_entry(lap_plan *P, lap_dtype dt, int b, const double *theta_host, const double *Q, int q,
                     const double *R, double *T, int itmax, double rtol, int *iters_out, int flags, hipStream_t s) {
    LAP_REQUIRE(q >= 0 && q <= kMaxQ, LAP_EUNSUPPORTED, "projector wider than 62 columns");
    if (dt == LAP_F32)
        return pcg_entry_t<float>(P, b, theta_host, Q, q, R, T, itmax, rtol, iters_out, flags, s);
    return pcg_entry_t<double>(P, b, theta_host, Q, q, R, T, itmax, rtol, iters_out, flags, s);
}

}  // namespace lapeig
