// Host driver of Jacobi-Davidson (Algorithm 2 with the deflation of eq.
// JDsismorethanone and the m_min/m_max restart of Section 3.2).  All vectors
// stay on the device; the host reads back one small status block per outer
// iteration (plus one per certification) to take the lock/restart decisions.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <numeric>

#include "block_kernels.h"

namespace lapeig {

namespace {

bool converged(double rnorm, double theta, double tol) {
    // certificate ||G u - theta u|| <= tol * min(theta, 1) for ||u|| = 1:
    // implies the paper's ||r||/theta <= tol (Section 4) and ||r|| <= tol
    const double scale = theta < 1.0 ? theta : 1.0;
    return rnorm <= tol * scale;
}

// The PCG launch sequence of one correction equation (Algorithm 2 step 8)
// captured once per projector width q and replayed every outer iteration:
// its arguments are device pointers fixed for the solve, so one graph serves
// until a lock widens Q.  The graph holds kernel nodes only.
template <typename T>
struct PcgGraphs {
    std::vector<hipGraphExec_t> exec;  // indexed by key
    ~PcgGraphs() {
        for (auto e : exec)
            if (e) (void)hipGraphExecDestroy(e);
    }
    hipGraphExec_t get(int q, hipStream_t s, const std::function<void()> &enqueue) {
        if ((int)exec.size() <= q) exec.resize(q + 1, nullptr);
        if (!exec[q]) {
            hipGraph_t g = nullptr;
            LAP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            try {
                enqueue();
            } catch (...) {
                (void)hipStreamEndCapture(s, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            LAP_HIP(hipStreamEndCapture(s, &g));
            hipGraphExec_t e = nullptr;
            hipError_t err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            LAP_HIP(err);
            exec[q] = e;
        }
        return exec[q];
    }
};

// A non-blocking stream of default priority owned by one solve.
struct OwnStream {
    hipStream_t s = nullptr;
    OwnStream() { LAP_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking)); }
    ~OwnStream() { if (s) (void)hipStreamDestroy(s); }
};

}  // namespace

void emit_pairs(const lap_plan &P, int nconv, const double *X, long long sr, long long sc,
                const std::vector<double> &lam, const std::vector<double> &resid, double *evals, double *evecs,
                int evecs_on_device, double *res_out, DevBuf<double> &scratch, hipStream_t s) {
    const int n = P.n;
    std::vector<int> order(nconv);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return lam[a] < lam[b]; });
    for (int j = 0; j < nconv; ++j) {
        evals[j] = lam[order[j]];
        if (res_out) res_out[j] = resid[order[j]];
    }
    if (evecs && nconv > 0) {
        DevBuf<int> dorder(nconv);
        DevBuf<double> dpart(2 * (size_t)nconv * final_chunks(n));
        LAP_HIP(hipMemcpyAsync(dorder.get(), order.data(), sizeof(int) * nconv, hipMemcpyHostToDevice, s));
        double *dst = evecs;
        if (!evecs_on_device) {
            if (scratch.n < (size_t)n * nconv) scratch.alloc((size_t)n * nconv);
            dst = scratch.get();
        }
        jd_finalize(n, nconv, X, sr, sc, dorder.get(), P.d_perm.get(), dst, dpart.get(), s);
        if (!evecs_on_device)
            LAP_HIP(hipMemcpyAsync(evecs, dst, sizeof(double) * n * nconv, hipMemcpyDeviceToHost, s));
        LAP_HIP(hipStreamSynchronize(s));
    }
    LAP_HIP(hipStreamSynchronize(s));
}

namespace {

// Host-coherent pinned status the kernels publish into (see HostMirror).
struct PinnedMirror {
    HostMirror *h = nullptr;
    PinnedMirror() {
        LAP_HIP(hipHostMalloc((void **)&h, sizeof(HostMirror), hipHostMallocMapped | hipHostMallocCoherent));
        std::memset(h, 0, sizeof(HostMirror));
    }
    ~PinnedMirror() { if (h) (void)hipHostFree(h); }
    PinnedMirror(const PinnedMirror &) = delete;
    PinnedMirror &operator=(const PinnedMirror &) = delete;
};

// Waits until the kernels have published sequence number `seq`.  Spins on
// the pinned word; if the stream drains without it, that is an error.
void wait_published(const HostMirror *hm, unsigned seq, hipStream_t s) {
    for (unsigned spin = 1;; ++spin) {
        if (__atomic_load_n(&hm->seq, __ATOMIC_ACQUIRE) == seq) return;
        if ((spin & 255) == 0) {
            const hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) {
                if (__atomic_load_n(&hm->seq, __ATOMIC_ACQUIRE) == seq) return;
                throw Failure{LAP_EDEVICE, "solver status was not published"};
            }
            if (e != hipErrorNotReady) LAP_HIP(e);
        }
    }
}

// Work areas of the single-vector solver, kept in the plan between solves
// of the same shape (n, k, m_max) and inner-solve settings.
template <typename T>
struct JdWork : SolverCache {
    int n, k, mmax, itmax, precond;
    double rtol;
    DevBuf<double> B, W, H, theta, Y, v, u, r, gu, vrand, isz;
    DevBuf<T> Q, t;
    DevBuf<JDStatus> st;
    PinnedMirror hm;
    ReduceScratch rs;
    PcgWork<T> pw;
    PcgGraphs<T> graphs;
    DevBuf<double> outbuf;  // eigenvectors on their way to host memory
    OwnStream own;          // the solver's stream
    JdWork(int n_, int k_, int mmax_, int itmax_, double rtol_, int precond_)
        : n(n_), k(k_), mmax(mmax_), itmax(itmax_), precond(precond_), rtol(rtol_) {
        B.alloc((size_t)n * (k + mmax));
        W.alloc((size_t)n * mmax);
        H.alloc((size_t)mmax * mmax);
        theta.alloc(mmax);
        Y.alloc((size_t)mmax * mmax);
        v.alloc(n); u.alloc(n); r.alloc(n); gu.alloc(n); vrand.alloc(n);
        isz.alloc(std::max(k, 1));
        Q.alloc((size_t)n * k);
        t.alloc(n);
        st.alloc(1);
        rs.ensure(std::max(4 * device_cu_count(), 1), 64);
        pw.ensure(n, k);
    }
    bool fits(int n_, int k_, int mmax_, int itmax_, double rtol_, int precond_) const {
        return n == n_ && k == k_ && mmax == mmax_ && itmax == itmax_ && rtol == rtol_ && precond == precond_;
    }
};

template <typename T>
lap_status jd_run(lap_plan *P, int k, double tol, const lap_eigs_opts &o, double *evals, double *evecs,
                  int evecs_on_device, double *res_out, lap_eigs_info *info) {
    const auto t_start = std::chrono::steady_clock::now();
    const int n = P->n;
    // work on a stream of our own (capturable even when the caller uses the
    // default stream), ordered after the caller's pending work
    LAP_HIP(hipStreamSynchronize(P->stream));
    // the pcg_breakdown hook solves every correction equation with a shift
    // above the spectrum (launched directly: the captured graphs hold theta)
    const bool brk_fault = fault_enabled("pcg_breakdown");
    DevBuf<double> theta_fault;
    if (brk_fault) {
        const double v = fault_breakdown_shift(*P);
        theta_fault.alloc(1);
        LAP_HIP(hipMemcpy(theta_fault.get(), &v, sizeof(double), hipMemcpyHostToDevice));
    }
    const bool use_graph = std::getenv("LAPEIG_NO_GRAPH") == nullptr && !brk_fault;
    const int mmax = o.m_max, mmin = o.m_min;
    const int kmax = o.kmax > 0 ? o.kmax : 1000 * k;
    LAP_REQUIRE(k + mmax <= kMaxBasis, LAP_EUNSUPPORTED,
                "k + m_max must not exceed 64 in the single-vector solver");
    const int nz = std::min(P->ncomp, k);
    const int ldq = k;

    const bool fsai = o.precond == LAP_PRECOND_FSAI;
    if (fsai) fsai_ensure(P);
    auto *cache = dynamic_cast<JdWork<T> *>(P->jd_cache.get());
    if (!cache || !cache->fits(n, k, mmax, o.itmax, o.rtol_pcg, o.precond)) {
        P->jd_cache.reset();
        P->jd_cache.reset(cache = new JdWork<T>(n, k, mmax, o.itmax, o.rtol_pcg, o.precond));
    }
    JdWork<T> &wk = *cache;
    hipStream_t s = wk.own.s;
    DevBuf<double> &B = wk.B, &W = wk.W, &H = wk.H, &theta = wk.theta, &Y = wk.Y, &v = wk.v, &u = wk.u, &r = wk.r,
                   &gu = wk.gu, &vrand = wk.vrand, &isz = wk.isz;
    DevBuf<T> &Q = wk.Q, &t = wk.t;
    DevBuf<JDStatus> &st = wk.st;
    HostMirror *hm = wk.hm.h;
    unsigned seq = hm->seq;
    ReduceScratch &rs = wk.rs;
    PcgWork<T> &pw = wk.pw;
    PcgGraphs<T> &graphs = wk.graphs;
    LAP_HIP(hipMemsetAsync(H.get(), 0, sizeof(double) * mmax * mmax, s));
    LAP_HIP(hipMemsetAsync(pw.st.get(), 0, sizeof(PcgState<T>), s));

    std::vector<double> lam, resid;
    lam.reserve(k);
    resid.reserve(k);
    // zero eigenpairs: one normalized indicator per connected component
    {
        std::vector<double> inv(std::max(nz, 1));
        for (int c = 0; c < nz; ++c) inv[c] = 1.0 / std::sqrt((double)P->comp_size[c]);
        LAP_HIP(hipMemcpyAsync(isz.get(), inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice, s));
        if (nz > 0) jd_zero_space<T>(n, nz, P->d_comp.get(), isz.get(), B.get(), Q.get(), ldq, s);
        for (int c = 0; c < nz; ++c) { lam.push_back(0.0); resid.push_back(0.0); }
    }
    // it: correction equations solved (the documented outer-iteration count);
    // steps: expansions of the search space, the loading of a start block included
    int nx = nz, m = 0, it = 0;
    long long steps = 0;
    const long long max_steps = 2LL * kmax + mmax + 64;
    int pcg_q = -1;  // projector width of the last correction equation of this solve
    int y_rows = 0;  // order of the block of H that theta and Y diagonalize
    long long mvp = 0, inner = 0;
    long long start_col = 0;
    lap_status status = LAP_OK;

    // start vectors: the caller's block (renumbered) or seeded random columns
    DevBuf<double> init_dev;
    int init_left = 0, init_next = 0, init_used = 0;
    bool src_from_init = false;  // the direction being added is a column of the caller's block
    if (o.init && o.init_cols > 0) {
        init_dev.alloc((size_t)n * o.init_cols);
        DevBuf<double> tmp((size_t)n * o.init_cols);
        LAP_HIP(hipMemcpyAsync(tmp.get(), o.init, sizeof(double) * n * o.init_cols,
                                o.init_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        if (fault_enabled("nan_init")) {
            static const double qnan = NAN;
            LAP_HIP(hipMemcpyAsync(tmp.get(), &qnan, sizeof(double), hipMemcpyHostToDevice, s));
        }
        for (int c = 0; c < o.init_cols; ++c)
            permute_rows<double>(P->d_perm.get(), n, 1, tmp.get() + (size_t)c * n, init_dev.get() + (size_t)c * n, s);
        LAP_HIP(hipStreamSynchronize(s));
        init_left = std::min(o.init_cols, mmax - 1);
    }
    // a column of the caller's block while any is left (one that is
    // non-finite or lies in span[X V] comes out of the orthogonalization as
    // a degenerate direction and is dropped), then seeded random columns
    auto next_start = [&]() -> const double * {
        if (init_left > 0) {
            --init_left;
            src_from_init = true;
            return init_dev.get() + (size_t)(init_next++) * n;
        }
        src_from_init = false;
        jd_random(n, o.seed, start_col++, P->d_iperm.get(), vrand.get(), s);
        return vrand.get();
    };

    bool src_is_t = false;
    const double *src = nullptr;
    if (nx < k) src = next_start();

    while (nx < k) {
        if (it >= kmax || steps >= max_steps) {
            status = LAP_ENOCONV;
            set_error("outer-iteration limit " + std::to_string(kmax) + " reached with " + std::to_string(nx) +
                      " of " + std::to_string(k) + " pairs certified");
            break;
        }
        ++steps;
        // step 2: orthogonalize against [X | V]; step 3: normalize, w = G v
        if (src_is_t) jd_orth<T>(n, B.get(), nx + m, t.get(), v.get(), rs, st.get(), s);
        else jd_orth<double>(n, B.get(), nx + m, src, v.get(), rs, st.get(), s);
        double *Vb = B.get() + (size_t)nx * n;
        jd_expand(*P, v.get(), Vb + (size_t)m * n, W.get() + (size_t)m * n, st.get(), rs, s);
        ++mvp;
        // step 4: border H
        jd_hborder(n, Vb, m, W.get() + (size_t)m * n, H.get(), mmax, rs, s);
        ++m;
        bool need_pcg = true;
        bool first = true;
        for (;;) {
            // step 5: eigenpairs of H; step 6: Ritz vector and residual
            // warm start when theta and Y still diagonalize the leading block
            // (the first pass folds the new border column that jd_hborder left)
            jd_rr(m, H.get(), mmax, theta.get(), Y.get(), mmax, st.get(), s, y_rows == m - 1 ? y_rows : 0,
                  first ? &rs : nullptr);
            y_rows = m;
            Vb = B.get() + (size_t)nx * n;
            jd_ritz<T>(n, Vb, W.get(), m, Y.get(), theta.get(), u.get(), r.get(), Q.get(), ldq, nx, rs, st.get(), s,
                       hm, ++seq);
            wait_published(hm, seq, s);
            if (first && hm->degenerate) {
                // the new direction lay in span[X V] (or was not finite): drop
                // it, take a fresh start vector
                --m;
                need_pcg = false;
                src_is_t = false;
                src = next_start();
                break;
            }
            if (first && src_from_init && !src_is_t) ++init_used;
            first = false;
            const double th = hm->theta, rn = hm->rnorm;
            if (!std::isfinite(th) || !std::isfinite(rn))
                throw Failure{LAP_EDEVICE, "non-finite Ritz value or residual"};
            // step 7: exit test, certified with a fresh product and eq. (1)
            if (!converged(rn, th, tol)) break;
            jd_certify(*P, u.get(), gu.get(), rs, st.get(), s, hm, ++seq);
            ++mvp;
            wait_published(hm, seq, s);
            const double ct = hm->cert_theta, cr = hm->cert_rnorm;
            if (!converged(cr, ct, tol)) break;
            // lock u = V y_1 as x_{nx}; keep V y_2.. as the new basis, H = diag
            jd_rotate(n, m, Y.get(), mmax, Vb, Vb, 0, m, nullptr, W.get(), W.get(), 1, m - 1, s);
            lam.push_back(ct);
            resid.push_back(cr);
            ++nx;
            --m;
            jd_hdiag(H.get(), mmax, m, theta.get(), 1, s);
            y_rows = 0;
            if (nx >= k) { need_pcg = false; break; }
            if (m == 0) {
                need_pcg = false;
                src_is_t = false;
                src = next_start();
                break;
            }
        }
        if (nx >= k) break;
        if (!need_pcg) continue;
        if (init_left > 0) {  // still loading the caller's start block
            src_is_t = false;
            src = next_start();
            continue;
        }
        // restart: keep the m_min Ritz vectors of smallest Ritz value
        if (m >= mmax) {
            Vb = B.get() + (size_t)nx * n;
            jd_rotate(n, m, Y.get(), mmax, Vb, Vb, 0, mmin, nullptr, W.get(), W.get(), 0, mmin, s);
            jd_hdiag(H.get(), mmax, mmin, theta.get(), 0, s);
            m = mmin;
            y_rows = 0;
        }
        // step 8: correction equation with Q = [X u]
        {
            // Q = [X u]: with no lock since the last equation, only u is new
            const int q = nx + 1;
            const bool inc = q == pcg_q;
            pcg_q = q;
            auto enqueue = [&]() {
                pcg_enqueue<T>(*P, brk_fault ? theta_fault.get() : theta.get(), Q.get(), ldq, q, r.get(), t.get(), pw,
                               o.itmax, o.rtol_pcg, s, inc, fsai);
            };
            if (use_graph) LAP_HIP(hipGraphLaunch(graphs.get(2 * q + (inc ? 1 : 0), s, enqueue), s));
            else enqueue();
            ++it;
        }
        src_is_t = true;
        src_from_init = false;
    }
    {
        // inner products of all correction equations of this solve
        PcgState<T> pstate;
        LAP_HIP(hipMemcpyAsync(&pstate, pw.st.get(), sizeof(pstate), hipMemcpyDeviceToHost, s));
        LAP_HIP(hipStreamSynchronize(s));
        inner = pstate.total;
        mvp += pstate.total;
    }

    // ---- output: ascending order, caller's vertex order, canonical signs
    const int nconv = std::min(nx, k);
    emit_pairs(*P, nconv, B.get(), 1, n, lam, resid, evals, evecs, evecs_on_device, res_out, wk.outbuf, s);
    if (info) {
        info->nconv = nconv;
        info->ncomp = P->ncomp;
        info->outer = it;
        info->inner = (int)inner;
        info->mvp = mvp;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        info->warm_start_used = init_used;
    }
    return status;
}

}  // namespace

lap_status jd_solve(lap_plan *P, int k, double tol, const lap_eigs_opts &o, double *evals, double *evecs,
                    int evecs_on_device, double *res, lap_eigs_info *info) {
    if (o.block > 1) return jd_block_solve(P, k, tol, o, evals, evecs, evecs_on_device, res, info);
    if (o.precision == LAP_PREC_MIXED)
        return jd_run<float>(P, k, tol, o, evals, evecs, evecs_on_device, res, info);
    return jd_run<double>(P, k, tol, o, evals, evecs, evecs_on_device, res, info);
}

}  // namespace lapeig
