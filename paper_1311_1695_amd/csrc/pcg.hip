// PCG on the projected correction equation (Algorithm 2 step 8):
//   (I - QQ')(G - theta I)(I - QQ') t = -r,   t orthogonal to Q,
// with the projected preconditioner M = (I-QQ')P(I-QQ') of the comments on
// Algorithm 2 and P = D^{-1} (Jacobi).  Q = [x_1 .. x_{j-1} u] as in
// eq. (JDsismorethanone).  The residual stays orthogonal to Q, so
//   M res = (I - QQ') D^{-1} res,   A_p p = (I - QQ')(G - theta I) p,
//   rho = res' M res = res' D^{-1} res,
// and one iteration needs two cross-workgroup reductions:
//   K1  s = (G - theta I) p;             pAp = p's,  c2 = Q's
//   K2  alpha = rho / pAp;  t += alpha p;  res -= alpha (s - Q c2);
//       y = D^{-1} res;  ||res||, rho' = res'y, c1 = Q'y;  beta = rho'/rho;
//       stop test
//   K3  p = (y - Q c1) + beta p
// A device flag turns the remaining launches into no-ops once the iteration
// stops, so the whole solve is enqueued without host round trips.
#include "lapeig_dev.h"
#include "jd_kernels.h"

namespace lapeig {

namespace {

template <typename T, int NV>
__global__ __launch_bounds__(kBlock) void k_pcg_init1(int n, const double *__restrict__ r, T *__restrict__ res,
                                                      T *__restrict__ t, const T *__restrict__ Q, int ldq, int q,
                                                      T *partial, unsigned *counter, PcgState<T> *st) {
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
    __shared__ T out[NV];
    if (grid_reduce<T, NV>(acc, q + 1, partial, counter, out)) {
        for (int j = threadIdx.x; j < q; j += blockDim.x) st->c0[j] = out[1 + j];
        if (threadIdx.x == 0) {
            st->r0 = sqrt(out[0]);
            st->stop = !(st->r0 > T(0));
            st->iters = 0;
            st->breakdown = 0;
        }
    }
}

// init: res -= Q c0 (project the right-hand side); y = D^{-1} res;
// rho = res'y; c1 = Q'y
template <typename T, int NV>
__global__ __launch_bounds__(kBlock) void k_pcg_init2(int n, T *__restrict__ res, T *__restrict__ y,
                                                      const T *__restrict__ dinv, const T *__restrict__ Q, int ldq,
                                                      int q, T *partial, unsigned *counter, PcgState<T> *st) {
    if (st->stop) return;
    __shared__ T c[NV];
    for (int j = threadIdx.x; j < q; j += blockDim.x) c[j] = st->c0[j];
    __syncthreads();
    T acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = T(0);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const T *qi = Q + (size_t)i * ldq;
        T proj = T(0);
#pragma unroll
        for (int j = 0; j < NV - 1; ++j)
            if (j < q) proj += qi[j] * c[j];
        const T ri = res[i] - proj;
        res[i] = ri;
        const T yi = dinv[i] * ri;
        y[i] = yi;
        acc[0] += ri * yi;
#pragma unroll
        for (int j = 0; j < NV - 1; ++j)
            if (j < q) acc[1 + j] += qi[j] * yi;
    }
    __shared__ T out[NV];
    if (grid_reduce<T, NV>(acc, q + 1, partial, counter, out)) {
        for (int j = threadIdx.x; j < q; j += blockDim.x) st->c1[j] = out[1 + j];
        if (threadIdx.x == 0) {
            st->rho = out[0];
            st->beta = T(0);
        }
    }
}

// K3 (and init): p = (y - Q c1) + beta p   [= z + beta p with z = M res]
template <typename T, int NV, bool INIT>
__global__ __launch_bounds__(kBlock) void k_pcg_p(int n, const T *__restrict__ y, T *__restrict__ p,
                                                  const T *__restrict__ Q, int ldq, int q, const PcgState<T> *st) {
    if (st->stop) return;
    __shared__ T c[NV];
    for (int j = threadIdx.x; j < q; j += blockDim.x) c[j] = st->c1[j];
    __syncthreads();
    const T beta = st->beta;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const T *qi = Q + (size_t)i * ldq;
        T proj = T(0);
#pragma unroll
        for (int j = 0; j < NV - 1; ++j)
            if (j < q) proj += qi[j] * c[j];
        const T zi = y[i] - proj;
        p[i] = INIT ? zi : zi + beta * p[i];
    }
}

// K1: s = (G - theta I) p; pAp = p's; c2 = Q's
template <typename T, int NV, bool Wt>
__global__ __launch_bounds__(kBlock) void k_pcg_ap(Graph g, Weights<T> w, const double *__restrict__ theta,
                                                   const T *__restrict__ p, T *__restrict__ s,
                                                   const T *__restrict__ Q, int ldq, int q, T *partial,
                                                   unsigned *counter, PcgState<T> *st, int it) {
    if (st->stop) return;
    const T th = (T)theta[0];
    T acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = T(0);
    for_each_row<T, Wt, false>(g, w, p, [&](int i, T pi, T yi, T) {
        const T si = yi - th * pi;
        s[i] = si;
        acc[0] += pi * si;
        const T *qi = Q + (size_t)i * ldq;
#pragma unroll
        for (int j = 0; j < NV - 1; ++j)
            if (j < q) acc[1 + j] += qi[j] * si;
    });
    __shared__ T out[NV];
    if (grid_reduce<T, NV>(acc, q + 1, partial, counter, out)) {
        for (int j = threadIdx.x; j < q; j += blockDim.x) st->c2[j] = out[1 + j];
        if (threadIdx.x == 0) {
            const T pap = out[0];
            st->pAp = pap;
            if (!(pap > T(0))) {  // the projected operator is indefinite along p
                st->stop = 1;
                st->breakdown = it;
            } else {
                st->alpha = st->rho / pap;
            }
        }
    }
}

// K2: update t and res, precondition, rho', beta, stop test
template <typename T, int NV>
__global__ __launch_bounds__(kBlock) void k_pcg_update(int n, T *__restrict__ t, T *__restrict__ res,
                                                       const T *__restrict__ p, const T *__restrict__ s,
                                                       T *__restrict__ y, const T *__restrict__ dinv,
                                                       const T *__restrict__ Q, int ldq, int q, T *partial,
                                                       unsigned *counter, PcgState<T> *st, int it, T rtol) {
    if (st->stop) {
        // no step was taken before the breakdown: return M(-r), which p still holds
        if (st->breakdown == it && it == 1)
            for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) t[i] = p[i];
        return;
    }
    const T alpha = st->alpha;
    __shared__ T c[NV];
    for (int j = threadIdx.x; j < q; j += blockDim.x) c[j] = st->c2[j];
    __syncthreads();
    T acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = T(0);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const T *qi = Q + (size_t)i * ldq;
        T proj = T(0);
#pragma unroll
        for (int j = 0; j < NV - 2; ++j)
            if (j < q) proj += qi[j] * c[j];
        t[i] += alpha * p[i];
        const T ri = res[i] - alpha * (s[i] - proj);
        res[i] = ri;
        const T yi = dinv[i] * ri;
        y[i] = yi;
        acc[0] += ri * ri;
        acc[1] += ri * yi;
#pragma unroll
        for (int j = 0; j < NV - 2; ++j)
            if (j < q) acc[2 + j] += qi[j] * yi;
    }
    __shared__ T out[NV];
    if (grid_reduce<T, NV>(acc, q + 2, partial, counter, out)) {
        for (int j = threadIdx.x; j < q; j += blockDim.x) st->c1[j] = out[2 + j];
        if (threadIdx.x == 0) {
            st->rn = sqrt(out[0]);
            st->iters = it;
            st->beta = out[1] / st->rho;
            st->rho = out[1];
            if (st->rn <= rtol * st->r0) st->stop = 1;
        }
    }
}

inline int vgrid(int n) {
    int g = (n + kBlock - 1) / kBlock;
    const int cap = 4 * device_cu_count();
    return g < 1 ? 1 : (g > cap ? cap : g);
}

template <typename T, int NV>
void enqueue_nv(const lap_plan &P, const double *theta, const T *Q, int ldq, int q, const double *r, T *t,
                PcgWork<T> &w, ReduceScratch &rs, int itmax, double rtol, hipStream_t s) {
    const int n = P.n;
    const int gv = vgrid(n);
    const int gr = row_grid(P.g, 4 * device_cu_count());
    rs.ensure(std::max(gv, gr), 64);
    T *part = reinterpret_cast<T *>(rs.partial.get());
    unsigned *cnt = rs.counter.get();
    PcgState<T> *st = w.st.get();
    const T *dinv = P.dinv<T>();
    hipLaunchKernelGGL((k_pcg_init1<T, NV>), dim3(gv), dim3(kBlock), 0, s, n, r, w.res.get(), t, Q, ldq, q, part,
                       cnt, st);
    hipLaunchKernelGGL((k_pcg_init2<T, NV>), dim3(gv), dim3(kBlock), 0, s, n, w.res.get(), w.y.get(), dinv, Q, ldq,
                       q, part, cnt, st);
    hipLaunchKernelGGL((k_pcg_p<T, NV, true>), dim3(gv), dim3(kBlock), 0, s, n, w.y.get(), w.p.get(), Q, ldq, q, st);
    for (int it = 1; it <= itmax; ++it) {
        if (P.weighted)
            hipLaunchKernelGGL((k_pcg_ap<T, NV, true>), dim3(gr), dim3(kBlock), 0, s, P.g, P.weights<T>(), theta,
                               w.p.get(), w.s.get(), Q, ldq, q, part, cnt, st, it);
        else
            hipLaunchKernelGGL((k_pcg_ap<T, NV, false>), dim3(gr), dim3(kBlock), 0, s, P.g, P.weights<T>(), theta,
                               w.p.get(), w.s.get(), Q, ldq, q, part, cnt, st, it);
        hipLaunchKernelGGL((k_pcg_update<T, NV>), dim3(gv), dim3(kBlock), 0, s, n, t, w.res.get(), w.p.get(),
                           w.s.get(), w.y.get(), dinv, Q, ldq, q, part, cnt, st, it, (T)rtol);
        if (it == itmax) break;
        hipLaunchKernelGGL((k_pcg_p<T, NV, false>), dim3(gv), dim3(kBlock), 0, s, n, w.y.get(), w.p.get(), Q, ldq, q,
                           st);
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
    w.ensure(n);
    ReduceScratch rs;
    const int gv = vgrid(n);
    if (q > 0)
        hipLaunchKernelGGL((k_pack_q<T>), dim3(gv), dim3(kBlock), 0, s, n, q, Q, map, Qr.get(), ldq);
    for (int c = 0; c < b; ++c) {
        LAP_HIP(hipMemcpyAsync(th.get(), theta_host + c, sizeof(double), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_gather_col, dim3(gv), dim3(kBlock), 0, s, n, R + (size_t)c * n, map, r.get());
        if (q <= 14)
            enqueue_nv<T, 16>(*P, th.get(), Qr.get(), ldq, q, r.get(), t.get(), w, rs, itmax, rtol, s);
        else
            enqueue_nv<T, 64>(*P, th.get(), Qr.get(), ldq, q, r.get(), t.get(), w, rs, itmax, rtol, s);
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
                 PcgWork<T> &w, ReduceScratch &rs, int itmax, double rtol, hipStream_t s) {
    LAP_REQUIRE(q >= 0 && q <= kMaxQ, LAP_EUNSUPPORTED, "projector wider than 62 columns");
    if (q <= 14)
        enqueue_nv<T, 16>(P, theta_dev, Q, ldq, q, r, t, w, rs, itmax, rtol, s);
    else
        enqueue_nv<T, 64>(P, theta_dev, Q, ldq, q, r, t, w, rs, itmax, rtol, s);
}
template void pcg_enqueue<float>(const lap_plan &, const double *, const float *, int, int, const double *, float *,
                                 PcgWork<float> &, ReduceScratch &, int, double, hipStream_t);
template void pcg_enqueue<double>(const lap_plan &, const double *, const double *, int, int, const double *,
                                  double *, PcgWork<double> &, ReduceScratch &, int, double, hipStream_t);

lap_status pcg_entry(lap_plan *P, lap_dtype dt, int b, const double *theta_host, const double *Q, int q,
                     const double *R, double *T, int itmax, double rtol, int *iters_out, int flags, hipStream_t s) {
    LAP_REQUIRE(q >= 0 && q <= kMaxQ, LAP_EUNSUPPORTED, "projector wider than 62 columns");
    if (dt == LAP_F32)
        return pcg_entry_t<float>(P, b, theta_host, Q, q, R, T, itmax, rtol, iters_out, flags, s);
    return pcg_entry_t<double>(P, b, theta_host, Q, q, R, T, itmax, rtol, iters_out, flags, s);
}

}  // namespace lapeig
