// Algorithm 3 (DACG) on the device: the k smallest eigenpairs one after the
// other, each by minimizing the Rayleigh quotient q(x) = x'Gx / x'x over the
// vectors orthogonal to the pairs already found (the columns of U), with a
// preconditioned nonlinear conjugate gradient (the DACG of Bergamaschi,
// Gambolati and Pini that the paper cites):
//   q = x'Gx / x'x,  g = 2 (G x - q x) / x'x,  h = D^{-1} g
//   beta = g'h / (g'h of the previous iteration)   (0 at the first)
//   p = (I - UU') h + beta p                        (deflated direction)
//   x <- x - alpha p, alpha minimizing q on span{x, p}: the smaller
//   eigenpair of the 2 x 2 pencil ([x p]'G[x p], [x p]'[x p])
// G x follows x through the same update with G p, so an iteration costs one
// Laplacian product, one preconditioner application and one deflation, the
// three costs the comments on Algorithm 3 name.  Four launches per
// iteration, each folding the partial sums the launch before it left:
//   KA  fold x'Gx, x'x; r = Gx - q x, g, h;        partials |r|^2, g'h, U'h
//   KB  fold; stop when |r| / |x| <= tol min(q, 1); beta; p
//   KC  Gp (row engine gathering p);               partials p'Gp, x'Gp, p'p, x'p
//   KD  fold; alpha; x -= alpha p, Gx -= alpha Gp; partials x'Gx, x'x
// Launch numbers turn the rest of a chunk into no-ops once KB has stopped
// (as in the PCG); the host enqueues chunks of iterations and reads the
// state between them.  A stopped pair is certified like a JD pair (fresh
// product, quotient of eq. (1)) and locked into U.  Double precision
// throughout; the zero pairs are the normalized component indicators,
// locked first (as in JD).
#include <chrono>
#include <cmath>
#include <vector>

#include "lapeig_dev.h"
#include "jd_kernels.h"

namespace lapeig {

namespace {

constexpr int kDacgNV = 64;  // values of the widest partial row (3 + U columns)

struct DacgState {
    double c, f;      // x'Gx and x'x of the current iterate (written by KA)
    double gh[2];     // g'h of the last two iterations, by parity
    double q, rn;     // quotient and residual norm when KB stopped
    int stop_seq, stop_it;
};

__device__ __forceinline__ bool dacg_stopped(const DacgState *st, int sq) {
    const int v = st->stop_seq;
    return v != 0 && v <= sq;
}

// partials x'Gx, x'x of the start vector
__global__ __launch_bounds__(kBlock) void k_dacg_cf(int n, const double *__restrict__ x,
                                                    const double *__restrict__ gx, double *__restrict__ part_out,
                                                    DacgState *st) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->stop_seq = 0;
        st->stop_it = -1;
    }
    double acc[2] = {0.0, 0.0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        acc[0] += x[i] * gx[i];
        acc[1] += x[i] * x[i];
    }
    write_partials<double, 2>(acc, 2, part_out);
}

// KA
__global__ __launch_bounds__(kBlock) void k_dacg_grad(int n, const double *__restrict__ x,
                                                      const double *__restrict__ gx, const double *__restrict__ dinv,
                                                      const double *__restrict__ U, int nu, double *__restrict__ h,
                                                      const double *__restrict__ part_in, int nb_in,
                                                      double *__restrict__ part_out, DacgState *st, int sq) {
    __shared__ double cf[2];
    fold_partials<double, 2>(part_in, nb_in, 2, cf);
    if (dacg_stopped(st, sq)) return;
    const double c = cf[0], f = cf[1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->c = c;
        st->f = f;
    }
    const double q = c / f, s2 = 2.0 / f;
    double acc[kDacgNV];
#pragma unroll
    for (int j = 0; j < kDacgNV; ++j) acc[j] = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double r = gx[i] - q * x[i];
        const double g = s2 * r;
        const double hi = dinv[i] * g;
        h[i] = hi;
        acc[0] += r * r;
        acc[1] += g * hi;
#pragma unroll
        for (int j = 0; j < kDacgNV - 2; ++j)
            if (j < nu) acc[2 + j] += U[(size_t)j * n + i] * hi;
    }
    write_partials<double, kDacgNV>(acc, nu + 2, part_out);
}

// KB
__global__ __launch_bounds__(kBlock) void k_dacg_dir(int n, const double *__restrict__ h,
                                                     const double *__restrict__ U, int nu, double *__restrict__ p,
                                                     const double *__restrict__ part_in, int nb_in, DacgState *st,
                                                     int sq, int it, double tol) {
    const double c = st->c, f = st->f;
    const double ghp = st->gh[(it + 1) & 1];  // the previous iteration's g'h
    __shared__ double tot[kDacgNV];
    fold_partials<double, kDacgNV>(part_in, nb_in, nu + 2, tot);
    if (dacg_stopped(st, sq)) return;
    const double q = c / f;
    const double rn = sqrt(tot[0] / f);
    if (rn <= tol * (q < 1.0 ? q : 1.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->stop_seq = sq + 1;
            st->stop_it = it;
            st->q = q;
            st->rn = rn;
        }
        return;
    }
    const double gh = tot[1];
    const double beta = it == 0 ? 0.0 : gh / ghp;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->gh[it & 1] = gh;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double proj = 0.0;
        for (int j = 0; j < nu; ++j) proj += U[(size_t)j * n + i] * tot[2 + j];
        const double pi = h[i] - proj;
        p[i] = it == 0 ? pi : pi + beta * p[i];
    }
}

// KC
template <bool Wt>
__global__ __launch_bounds__(kBlock) void k_dacg_gp(Graph g, Weights<double> w, const double *__restrict__ p,
                                                    const double *__restrict__ x, double *__restrict__ gp,
                                                    double *__restrict__ part_out, const DacgState *st, int sq) {
    if (dacg_stopped(st, sq)) return;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for_each_row<double, Wt, false>(g, w, p, [&](int i, double pi, double gpi, double) {
        gp[i] = gpi;
        const double xi = x[i];
        acc[0] += pi * gpi;
        acc[1] += xi * gpi;
        acc[2] += pi * pi;
        acc[3] += xi * pi;
    });
    write_partials<double, 4>(acc, 4, part_out);
}

// KD
__global__ __launch_bounds__(kBlock) void k_dacg_update(int n, double *__restrict__ x, double *__restrict__ gx,
                                                        const double *__restrict__ p, const double *__restrict__ gp,
                                                        const double *__restrict__ part_in, int nb_in,
                                                        double *__restrict__ part_out, const DacgState *st, int sq) {
    const double c = st->c, f = st->f;
    __shared__ double t[4];
    fold_partials<double, 4>(part_in, nb_in, 4, t);
    if (dacg_stopped(st, sq)) return;
    const double a = t[0], b = t[1], d = t[2], e = t[3];
    // the smaller root mu of det([c b; b a] - mu [f e; e d]) = 0, in the
    // cancellation-free form 2C / (B + sqrt(B^2 - 4AC)); then alpha from the
    // better conditioned row of the singular 2 x 2 system
    const double A2 = f * d - e * e, B2 = a * f + c * d - 2.0 * b * e, C2 = c * a - b * b;
    double disc = B2 * B2 - 4.0 * A2 * C2;
    if (disc < 0.0) disc = 0.0;
    const double mu = 2.0 * C2 / (B2 + sqrt(disc));
    const double den1 = a - mu * d, den2 = b - mu * e;
    const double alpha = fabs(den1) >= fabs(den2) ? den2 / den1 : (c - mu * f) / den2;
    double acc[2] = {0.0, 0.0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double xi = x[i] - alpha * p[i];
        const double gi = gx[i] - alpha * gp[i];
        x[i] = xi;
        gx[i] = gi;
        acc[0] += xi * gi;
        acc[1] += xi * xi;
    }
    write_partials<double, 2>(acc, 2, part_out);
}

// u = x / sqrt(x'x)
__global__ void k_dacg_lock(int n, const double *__restrict__ x, const DacgState *st, double *__restrict__ u) {
    const double s = 1.0 / sqrt(st->f);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) u[i] = x[i] * s;
}

inline int dgrid(int n) {
    int g = (n + kBlock - 1) / kBlock;
    const int cap = 2 * device_cu_count();
    return g < 1 ? 1 : (g > cap ? cap : g);
}

}  // namespace

lap_status dacg_solve(lap_plan *P, int k, double tol, const lap_eigs_opts &o, double *evals, double *evecs,
                      int evecs_on_device, double *res_out, lap_eigs_info *info) {
    const auto t_start = std::chrono::steady_clock::now();
    const int n = P->n;
    LAP_REQUIRE(k <= kDacgNV - 2, LAP_EUNSUPPORTED, "DACG computes at most 62 pairs");
    LAP_REQUIRE(o.precond == LAP_PRECOND_JACOBI, LAP_EUNSUPPORTED, "DACG preconditions with D^{-1}");
    const int itmax = o.kmax > 0 ? o.kmax : 20000;
    LAP_HIP(hipStreamSynchronize(P->stream));
    hipStream_t s = P->stream;
    const int nz = std::min(P->ncomp, k);
    DevBuf<double> U((size_t)n * k), x(n), gx(n), h(n), p(n), gp(n), v(n), vrand(n), gu(n), isz(std::max(nz, 1)),
        qdummy((size_t)n * std::max(nz, 1));
    const int gv = dgrid(n);
    const int gr = row_grid(P->g, pcg_vec_groups());
    DevBuf<double> part_cf((size_t)std::max(gv, gr) * 2), part_g((size_t)gv * kDacgNV),
        part_s((size_t)std::max(gv, gr) * 4);
    DevBuf<DacgState> dst(1);
    DevBuf<JDStatus> jst(1);
    ReduceScratch rs;
    rs.ensure(std::max(4 * device_cu_count(), gr), 64);
    std::vector<double> lam, resid;
    {
        std::vector<double> inv(std::max(nz, 1));
        for (int c = 0; c < nz; ++c) inv[c] = 1.0 / std::sqrt((double)P->comp_size[c]);
        LAP_HIP(hipMemcpyAsync(isz.get(), inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice, s));
        if (nz > 0) jd_zero_space<double>(n, nz, P->d_comp.get(), isz.get(), U.get(), qdummy.get(), nz, s);
        for (int c = 0; c < nz; ++c) { lam.push_back(0.0); resid.push_back(0.0); }
    }
    int nu = nz;
    long long mvp = 0, iters = 0, start_col = 0;
    int pairs = 0;
    lap_status status = LAP_OK;
    const double *dinv = P->d_dinv64.get();
    constexpr int kChunk = 32;
    while (nu < k) {
        // x_0: the seeded start vector, orthogonal to U, normalized; Gx_0
        jd_random(n, o.seed, start_col++, P->d_iperm.get(), vrand.get(), s);
        jd_orth<double>(n, U.get(), nu, vrand.get(), v.get(), rs, jst.get(), s);
        jd_expand(*P, v.get(), x.get(), gx.get(), jst.get(), rs, s);
        ++mvp;
        hipLaunchKernelGGL(k_dacg_cf, dim3(gv), dim3(kBlock), 0, s, n, x.get(), gx.get(), part_cf.get(), dst.get());
        LAP_HIP(hipGetLastError());
        int it0 = 0;  // iterations of this pair so far
        bool locked = false;
        while (!locked) {
            if (it0 >= itmax) break;
            const int chunk = std::min(kChunk, itmax - it0);
            for (int j = 0; j < chunk; ++j) {
                const int it = it0 + j;
                const int sq = 4 * it + 1;
                hipLaunchKernelGGL(k_dacg_grad, dim3(gv), dim3(kBlock), 0, s, n, x.get(), gx.get(), dinv, U.get(), nu,
                                   h.get(), part_cf.get(), gv, part_g.get(), dst.get(), sq);
                hipLaunchKernelGGL(k_dacg_dir, dim3(gv), dim3(kBlock), 0, s, n, h.get(), U.get(), nu, p.get(),
                                   part_g.get(), gv, dst.get(), sq + 1, it, tol);
                if (P->weighted)
                    hipLaunchKernelGGL((k_dacg_gp<true>), dim3(gr), dim3(kBlock), 0, s, P->g, P->weights<double>(),
                                       p.get(), x.get(), gp.get(), part_s.get(), dst.get(), sq + 2);
                else
                    hipLaunchKernelGGL((k_dacg_gp<false>), dim3(gr), dim3(kBlock), 0, s, P->g, P->weights<double>(),
                                       p.get(), x.get(), gp.get(), part_s.get(), dst.get(), sq + 2);
                hipLaunchKernelGGL(k_dacg_update, dim3(gv), dim3(kBlock), 0, s, n, x.get(), gx.get(), p.get(),
                                   gp.get(), part_s.get(), gr, part_cf.get(), dst.get(), sq + 3);
            }
            LAP_HIP(hipGetLastError());
            DacgState hs;
            LAP_HIP(hipMemcpyAsync(&hs, dst.get(), sizeof(hs), hipMemcpyDeviceToHost, s));
            LAP_HIP(hipStreamSynchronize(s));
            if (hs.stop_seq == 0) {
                it0 += chunk;
                mvp += chunk;
                continue;
            }
            // stopped inside this chunk at iteration stop_it (its product not taken)
            mvp += hs.stop_it - it0;
            it0 = hs.stop_it;
            // lock u = x / ||x|| after a certificate with a fresh product (eq. (1))
            double *u = U.get() + (size_t)nu * n;
            hipLaunchKernelGGL(k_dacg_lock, dim3(gv), dim3(kBlock), 0, s, n, x.get(), dst.get(), u);
            jd_certify(*P, u, gu.get(), rs, jst.get(), s);
            ++mvp;
            JDStatus js;
            LAP_HIP(hipMemcpyAsync(&js, jst.get(), sizeof(js), hipMemcpyDeviceToHost, s));
            LAP_HIP(hipStreamSynchronize(s));
            const double ct = js.cert_theta, cr = js.cert_rnorm;
            LAP_REQUIRE(std::isfinite(ct) && std::isfinite(cr), LAP_EDEVICE, "non-finite DACG iterate");
            if (cr <= tol * (ct < 1.0 ? ct : 1.0)) {
                lam.push_back(ct);
                resid.push_back(cr);
                ++nu;
                locked = true;
            } else {
                // not certified in FP64: continue from x with a fresh conjugate direction
                hipLaunchKernelGGL(k_dacg_cf, dim3(gv), dim3(kBlock), 0, s, n, x.get(), gx.get(), part_cf.get(),
                                   dst.get());
                LAP_HIP(hipGetLastError());
            }
        }
        iters += it0;
        ++pairs;
        if (!locked) {
            status = LAP_ENOCONV;
            set_error("DACG iteration limit " + std::to_string(itmax) + " reached with " + std::to_string(nu) +
                      " of " + std::to_string(k) + " pairs certified");
            break;
        }
    }
    const int nconv = std::min(nu, k);
    DevBuf<double> outbuf;
    emit_pairs(*P, nconv, U.get(), 1, n, lam, resid, evals, evecs, evecs_on_device, res_out, outbuf, s);
    if (info) {
        info->nconv = nconv;
        info->ncomp = P->ncomp;
        info->outer = pairs;
        info->inner = (int)std::min<long long>(iters, 2147483647LL);
        info->mvp = mvp;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        info->warm_start_used = 0;
    }
    return status;
}

}  // namespace lapeig
