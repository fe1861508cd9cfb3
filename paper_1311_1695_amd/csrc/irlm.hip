// The Implicitly Restarted Lanczos Method on the inverse (Section 3.1,
// Algorithm 1 right), on the device: Lanczos on G^+ (the inverse of G on the
// complement of its zero space), each step solving G w = v_j with the
// projected PCG of the correction equation (theta = 0, Q = the zero space),
// restarted until the wanted Ritz values of G^+ (the largest), whose
// reciprocals are the smallest nonzero eigenvalues of G, hold JD's
// certificate.
//   step j:  w = G^+ v_j (PCG to rtol_inner);  T(0..j, j) = V(:, 0..j)' w;
//            w orthogonalized against [Z V(:, 0..j)] (classical Gram-Schmidt
//            twice);  v_{j+1} = w / ||w||
//   cycle:   eig(T) (Jacobi in one workgroup); the wanted Ritz vectors
//            certified with a fresh product (the quotient of eq. (1));
//            otherwise a thick restart: V(:, 0..p) = V Y(:, largest p),
//            v_p = v_m, T = diag(theta) bordered by ||w_m|| Y(m-1, .)
// Thick restart with the wanted Ritz vectors and the last Lanczos vector
// (Wu & Simon) spans the space of Sorensen's implicit restart with exact
// shifts; the full column of T is kept (not only the tridiagonal), so the
// Rayleigh-Ritz step sees the projected matrix itself.  Double precision
// throughout.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "lapeig_dev.h"
#include "jd_kernels.h"

namespace lapeig {

namespace {

__global__ void k_irlm_neg(int n, const double *__restrict__ v, double *__restrict__ out) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = -v[i];
}

// partial rows of V(:, 0..nv)' w, nv <= 64
__global__ __launch_bounds__(kBlock) void k_irlm_coef(int n, const double *__restrict__ V, int nv,
                                                      const double *__restrict__ w, double *__restrict__ part_out) {
    double acc[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) acc[j] = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double wi = w[i];
#pragma unroll
        for (int j = 0; j < 64; ++j)
            if (j < nv) acc[j] += V[(size_t)j * n + i] * wi;
    }
    write_partials<double, 64>(acc, nv, part_out);
}

// T(i, j) = T(j, i) = h_i for i < nv (one workgroup)
__global__ __launch_bounds__(kBlock) void k_irlm_tcol(const double *__restrict__ part_in, int nb, int nv, double *T,
                                                      int ldt, int j) {
    __shared__ double h[64];
    fold_partials<double, 64>(part_in, nb, nv, h);
    for (int i = threadIdx.x; i < nv; i += blockDim.x) {
        T[(size_t)j * ldt + i] = h[i];
        T[(size_t)i * ldt + j] = h[i];
    }
}

inline int igrid(int n) {
    int g = (n + kBlock - 1) / kBlock;
    const int cap = 2 * device_cu_count();
    return g < 1 ? 1 : (g > cap ? cap : g);
}

}  // namespace

lap_status irlm_solve(lap_plan *P, int k, double tol, int m_in, double rtol_inner, int itmax_inner,
                      const lap_eigs_opts &o, double *evals, double *evecs, int evecs_on_device, double *res_out,
                      lap_eigs_info *info) {
    const auto t_start = std::chrono::steady_clock::now();
    const int n = P->n;
    const int nz = std::min(P->ncomp, k);
    const int nzall = P->ncomp;
    const int want = k - nz;
    LAP_REQUIRE(o.precond == LAP_PRECOND_JACOBI || o.precond == LAP_PRECOND_FSAI, LAP_EINVAL, "bad precond");
    const bool fsai = o.precond == LAP_PRECOND_FSAI;
    if (fsai) fsai_ensure(P);
    int m = m_in > 0 ? m_in : std::max(3 * want, want + 6);
    m = std::min(m, n - nzall);
    LAP_REQUIRE(nzall + m + 1 <= kMaxBasis - 1, LAP_EUNSUPPORTED,
                "zero space + Krylov size + 1 must not exceed 63 columns");
    LAP_REQUIRE(nzall <= 14, LAP_EUNSUPPORTED, "at most 14 connected components");
    LAP_REQUIRE(want == 0 || m > want, LAP_EINVAL, "the Krylov size must exceed the wanted pairs");
    const int p = want + (m - want) / 2;
    const int max_restarts = o.kmax > 0 ? o.kmax : 1000;
    const double rtol_pcg = rtol_inner > 0.0 ? rtol_inner : 1e-12;
    const int itmax_pcg = itmax_inner > 0 ? itmax_inner : 1000;
    LAP_HIP(hipStreamSynchronize(P->stream));
    hipStream_t s = P->stream;

    // B = [Z | V]: the zero space, then the Lanczos basis (column-major)
    const int nb = nzall + m + 1;
    DevBuf<double> B((size_t)n * nb), Qz((size_t)n * std::max(nzall, 1)), isz(std::max(nzall, 1));
    DevBuf<double> r(n), t(n), w(n), vrand(n), gu(n), T((size_t)m * m), theta(m), Y((size_t)m * m),
        Ubuf((size_t)n * std::max(want, 1)), th0(1);
    DevBuf<JDStatus> jst(1);
    ReduceScratch rs;
    rs.ensure(4 * device_cu_count(), 64);
    PcgWork<double> pw;
    pw.ensure(n, std::max(nzall, 1));
    const int gv = igrid(n);
    DevBuf<double> part((size_t)gv * 64);
    {
        std::vector<double> inv(std::max(nzall, 1));
        for (int c = 0; c < nzall; ++c) inv[c] = 1.0 / std::sqrt((double)P->comp_size[c]);
        LAP_HIP(hipMemcpyAsync(isz.get(), inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice, s));
        if (nzall > 0) jd_zero_space<double>(n, nzall, P->d_comp.get(), isz.get(), B.get(), Qz.get(), nzall, s);
        LAP_HIP(hipMemsetAsync(th0.get(), 0, sizeof(double), s));
        LAP_HIP(hipMemsetAsync(pw.st.get(), 0, sizeof(PcgState<double>), s));
    }
    std::vector<double> lam(nz, 0.0), resid(nz, 0.0);
    double *V = B.get() + (size_t)nzall * n;
    long long mvp = 0, steps = 0;
    int restarts = 0;  // thick restarts so far
    lap_status status = LAP_OK;
    bool done = want == 0;
    std::vector<double> hT((size_t)m * m), hth(m), hY((size_t)m * m);
    if (!done) {
        // v_0: the seeded start vector of JD, orthogonal to the zero space, unit length
        jd_random(n, o.seed, 0, P->d_iperm.get(), vrand.get(), s);
        jd_orth<double>(n, B.get(), nzall, vrand.get(), w.get(), rs, jst.get(), s);
        jd_scale_copy(n, w.get(), V, jst.get(), rs, s);
        LAP_HIP(hipMemsetAsync(T.get(), 0, sizeof(double) * m * m, s));
    }
    int j0 = 0;
    while (!done) {
        for (int j = j0; j < m; ++j) {
            double *vj = V + (size_t)j * n;
            // w = G^+ v_j:  the projected PCG solves G t = -r for r = -v_j
            hipLaunchKernelGGL(k_irlm_neg, dim3(gv), dim3(kBlock), 0, s, n, vj, r.get());
            pcg_enqueue<double>(*P, th0.get(), Qz.get(), std::max(nzall, 1), nzall, r.get(), t.get(), pw, itmax_pcg,
                                rtol_pcg, s, false, fsai, true);
            // the column of the projected matrix, then the next Lanczos vector
            hipLaunchKernelGGL(k_irlm_coef, dim3(gv), dim3(kBlock), 0, s, n, V, j + 1, t.get(), part.get());
            hipLaunchKernelGGL(k_irlm_tcol, dim3(1), dim3(kBlock), 0, s, part.get(), gv, j + 1, T.get(), m, j);
            LAP_HIP(hipGetLastError());
            jd_orth<double>(n, B.get(), nzall + j + 1, t.get(), w.get(), rs, jst.get(), s);
            jd_scale_copy(n, w.get(), V + (size_t)(j + 1) * n, jst.get(), rs, s);
            ++steps;
        }
        // Rayleigh-Ritz on T (ascending Ritz values of G^+)
        jd_rr(m, T.get(), m, theta.get(), Y.get(), m, jst.get(), s, 0, nullptr, true);
        JDStatus js;
        LAP_HIP(hipMemcpyAsync(hth.data(), theta.get(), sizeof(double) * m, hipMemcpyDeviceToHost, s));
        LAP_HIP(hipMemcpyAsync(hY.data(), Y.get(), sizeof(double) * m * m, hipMemcpyDeviceToHost, s));
        LAP_HIP(hipMemcpyAsync(&js, jst.get(), sizeof(js), hipMemcpyDeviceToHost, s));
        LAP_HIP(hipStreamSynchronize(s));
        const double beta_m = js.orth_n1;  // ||w|| of the last step
        // the wanted Ritz vectors (the `want` largest theta), certified on G
        jd_rotate(n, m, Y.get(), m, V, Ubuf.get(), m - want, want, nullptr, nullptr, nullptr, 0, 0, s);
        std::vector<double> cl(want), cr(want);
        bool all = true;
        for (int i = 0; i < want; ++i) {
            jd_certify(*P, Ubuf.get() + (size_t)i * n, gu.get(), rs, jst.get(), s);
            ++mvp;
            LAP_HIP(hipMemcpyAsync(&js, jst.get(), sizeof(js), hipMemcpyDeviceToHost, s));
            LAP_HIP(hipStreamSynchronize(s));
            cl[i] = js.cert_theta;
            cr[i] = js.cert_rnorm;
            LAP_REQUIRE(std::isfinite(cl[i]) && std::isfinite(cr[i]), LAP_EDEVICE, "non-finite Ritz pair");
            if (!(cr[i] <= tol * std::min(cl[i], 1.0))) all = false;
        }
        if (all) {
            for (int i = 0; i < want; ++i) {
                lam.push_back(cl[i]);
                resid.push_back(cr[i]);
            }
            done = true;
            break;
        }
        if (restarts >= max_restarts) {
            status = LAP_ENOCONV;
            set_error("IRLM restart limit " + std::to_string(max_restarts) + " reached");
            break;
        }
        ++restarts;
        // thick restart: V(:, 0..p) = V Y(:, m-p..m), v_p = v_m, T = arrow
        jd_rotate(n, m, Y.get(), m, V, V, m - p, p, nullptr, nullptr, nullptr, 0, 0, s);
        LAP_HIP(hipMemcpyAsync(V + (size_t)p * n, V + (size_t)m * n, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        std::fill(hT.begin(), hT.end(), 0.0);
        for (int i = 0; i < p; ++i) {
            const int c = m - p + i;
            hT[(size_t)i * m + i] = hth[c];
            const double sv = beta_m * hY[(size_t)c * m + (m - 1)];
            hT[(size_t)p * m + i] = sv;
            hT[(size_t)i * m + p] = sv;
        }
        LAP_HIP(hipMemcpyAsync(T.get(), hT.data(), sizeof(double) * m * m, hipMemcpyHostToDevice, s));
        j0 = p;
    }
    {
        PcgState<double> ps;
        LAP_HIP(hipMemcpyAsync(&ps, pw.st.get(), sizeof(ps), hipMemcpyDeviceToHost, s));
        LAP_HIP(hipStreamSynchronize(s));
        mvp += ps.total;
        if (info) info->inner = ps.total;
    }
    // output: the zero pairs (columns of Z) and the certified Ritz pairs;
    // the Ritz vectors are moved next to Z so one call emits them all
    const int nconv = done ? k : nz;
    if (done && want > 0)
        LAP_HIP(hipMemcpyAsync(B.get() + (size_t)nz * n, Ubuf.get(), sizeof(double) * n * want,
                                hipMemcpyDeviceToDevice, s));
    DevBuf<double> outbuf;
    emit_pairs(*P, nconv, B.get(), 1, n, lam, resid, evals, evecs, evecs_on_device, res_out, outbuf, s);
    if (info) {
        info->nconv = nconv;
        info->ncomp = P->ncomp;
        info->outer = (int)steps;
        info->mvp = mvp;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        info->warm_start_used = 0;
    }
    return status;
}

}  // namespace lapeig
