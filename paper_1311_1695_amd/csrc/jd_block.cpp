// Block Jacobi-Davidson: Algorithm 2 with b corrections per outer iteration.
//
// Each outer iteration solves the correction equations of the b smallest
// unconverged Ritz pairs together (one block PCG over an n x b SpMM, shared
// projector Q = [X, U]), orthonormalizes the b corrections against [X V] and
// among themselves, and expands V, W = GV and H = V'W by b columns at once.
// Deflation, restart and certification are those of Algorithm 2 (eq.
// JDsismorethanone; m_min/m_max of Section 3.2), applied to the leading Ritz
// pair.  Basis storage is row-major: [X | V] is n x (k + m_max), W n x m_max.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <functional>
#include <map>
#include <numeric>

#include "block_kernels.h"

namespace lapeig {

namespace {

bool converged_b(double rnorm, double theta, double tol) {
    const double scale = theta < 1.0 ? theta : 1.0;
    return rnorm <= tol * scale;
}

struct OwnStreamB {
    hipStream_t s = nullptr;
    OwnStreamB() { LAP_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking)); }
    ~OwnStreamB() { if (s) (void)hipStreamDestroy(s); }
};

template <typename Tp>
struct PinnedB {
    Tp *h = nullptr;
    PinnedB() { LAP_HIP(hipHostMalloc((void **)&h, sizeof(Tp), hipHostMallocDefault)); }
    ~PinnedB() { if (h) (void)hipHostFree(h); }
};

// graphs of the block PCG keyed by (q, b, first iteration, last iteration)
struct GraphCache {
    std::map<std::array<int, 4>, hipGraphExec_t> exec;
    ~GraphCache() {
        for (auto &e : exec)
            if (e.second) (void)hipGraphExecDestroy(e.second);
    }
    hipGraphExec_t get(int q, int b, int it_first, int it_last, hipStream_t s, const std::function<void()> &enqueue) {
        const std::array<int, 4> key{q, b, it_first, it_last};
        auto it = exec.find(key);
        if (it != exec.end()) return it->second;
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
        exec[key] = e;
        return e;
    }
};

// Work areas of the block solver, kept in the plan between solves of the
// same shape (n, k, b, m_max) and inner-solve settings.
template <typename T>
struct JdbWork : SolverCache {
    int n, k, b, mmax, itmax;
    double rtol;
    DevBuf<double> XV, W, H, theta, Y, Vn, Cc, S, Sth, Sz, M, U, GU, R, u0, gu, isz, outbuf;
    DevBuf<T> Q, Tt;
    DevBuf<BlockStatus> bst;
    DevBuf<JDStatus> jst;
    DevBuf<double> init_tmp;  // a caller's start block (taken on its first use)
    DevBuf<int> init_bad;
    PinnedB<BlockStatus> hb;
    PinnedB<JDStatus> hj;
    PinnedB<BPcgState<T>> hp;
    ReduceScratch rs;
    BlockScratch bs;
    BPcgWork<T> pw;
    GraphCache graphs;
    OwnStreamB own;
    JdbWork(int n_, int k_, int b_, int mmax_, int itmax_, double rtol_)
        : n(n_), k(k_), b(b_), mmax(mmax_), itmax(itmax_), rtol(rtol_) {
        const int ldb = k + mmax, ldq = k + b;
        XV.alloc((size_t)n * ldb); W.alloc((size_t)n * mmax); H.alloc((size_t)mmax * mmax); theta.alloc(mmax);
        Y.alloc((size_t)mmax * mmax); Vn.alloc((size_t)n * b); Cc.alloc((size_t)ldb * b); S.alloc((size_t)b * b);
        Sth.alloc(b); Sz.alloc((size_t)b * b); M.alloc((size_t)b * b); U.alloc((size_t)n * b);
        GU.alloc((size_t)n * b); R.alloc((size_t)n * b); u0.alloc(n); gu.alloc(n); isz.alloc(std::max(k, 1));
        Q.alloc((size_t)n * ldq); Tt.alloc((size_t)n * b);
        bst.alloc(1); jst.alloc(1);
        rs.ensure(4 * device_cu_count(), 64);
        bs.ensure();
        pw.ensure(n, b, ldq);
    }
    bool fits(int n_, int k_, int b_, int mmax_, int itmax_, double rtol_) const {
        return n == n_ && k == k_ && b == b_ && mmax == mmax_ && itmax == itmax_ && rtol == rtol_;
    }
};

template <typename T>
lap_status jdb_run(lap_plan *P, int k, double tol, const lap_eigs_opts &o, double *evals, double *evecs,
                   int evecs_on_device, double *res_out, lap_eigs_info *info) {
    const auto t_start = std::chrono::steady_clock::now();
    const int n = P->n;
    const int b = o.block, mmax = o.m_max, mmin = o.m_min;
    LAP_REQUIRE(b >= 2 && b <= kMaxBlock, LAP_EUNSUPPORTED, "block size must be 2..32");
    LAP_REQUIRE(mmin >= b && mmin + b <= mmax, LAP_EINVAL, "block solver needs m_min >= b and m_min + b <= m_max");
    LAP_REQUIRE(mmax <= 96, LAP_EUNSUPPORTED, "m_max above 96");
    LAP_REQUIRE(k + mmax <= 128, LAP_EUNSUPPORTED, "k + m_max above 128");
    const int kmax = o.kmax > 0 ? o.kmax : 1000 * k;
    LAP_HIP(hipStreamSynchronize(P->stream));
    // the pcg_breakdown hook (see fault_enabled): shifts above the spectrum
    const bool brk_fault = fault_enabled("pcg_breakdown");
    DevBuf<double> theta_fault;
    if (brk_fault) {
        const std::vector<double> v(kMaxBlock, fault_breakdown_shift(*P));
        theta_fault.alloc(kMaxBlock);
        LAP_HIP(hipMemcpy(theta_fault.get(), v.data(), sizeof(double) * kMaxBlock, hipMemcpyHostToDevice));
    }
    const bool use_graph = std::getenv("LAPEIG_NO_GRAPH") == nullptr && !brk_fault;
    ts_prepare<double>();
    ts_prepare<T>();
    auto *cache = dynamic_cast<JdbWork<T> *>(P->jdb_cache.get());
    if (!cache || !cache->fits(n, k, b, mmax, o.itmax, o.rtol_pcg)) {
        P->jdb_cache.reset();
        P->jdb_cache.reset(cache = new JdbWork<T>(n, k, b, mmax, o.itmax, o.rtol_pcg));
        // sized for this plan's layout (a new layout drops the cache)
        cache->pw.ensure_dot((size_t)spmm_dot_rows(*P, b));
    }
    JdbWork<T> &wk = *cache;
    hipStream_t s = wk.own.s;
    GraphCache &graphs = wk.graphs;

    const int ldb = k + mmax, ldh = mmax, ldq = k + b;
    const int nz = std::min(P->ncomp, k);
    DevBuf<double> &XV = wk.XV, &W = wk.W, &H = wk.H, &theta = wk.theta, &Y = wk.Y, &Vn = wk.Vn, &Cc = wk.Cc,
                   &S = wk.S, &Sth = wk.Sth, &Sz = wk.Sz, &M = wk.M, &U = wk.U, &GU = wk.GU, &R = wk.R, &u0 = wk.u0,
                   &gu = wk.gu, &isz = wk.isz;
    DevBuf<T> &Q = wk.Q, &Tt = wk.Tt;
    DevBuf<BlockStatus> &bst = wk.bst;
    DevBuf<JDStatus> &jst = wk.jst;
    PinnedB<BlockStatus> &hb = wk.hb;
    PinnedB<JDStatus> &hj = wk.hj;
    PinnedB<BPcgState<T>> &hp = wk.hp;
    ReduceScratch &rs = wk.rs;
    BlockScratch &bs = wk.bs;
    BPcgWork<T> &pw = wk.pw;

    std::vector<double> lam, resid;
    {
        std::vector<double> inv(std::max(nz, 1));
        for (int c = 0; c < nz; ++c) inv[c] = 1.0 / std::sqrt((double)P->comp_size[c]);
        LAP_HIP(hipMemcpyAsync(isz.get(), inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice, s));
        if (nz > 0) blk_zero_space<T>(n, nz, P->d_comp.get(), isz.get(), XV.get(), ldb, Q.get(), ldq, s);
        for (int c = 0; c < nz; ++c) { lam.push_back(0.0); resid.push_back(0.0); }
    }
    int nx = nz, m = 0, it = 0;
    int y_rows = 0;  // order of the block of H that theta and Y diagonalize
    long long mvp = 0, inner = 0, colbase = 0;
    lap_status status = LAP_OK;

    // the first block: the caller's start vectors (up to b), then random columns
    int src_cols = 0;     // columns waiting in Vn (double) or Tt (T)
    bool src_is_t = false;
    auto random_block = [&]() {
        blk_random(n, b, o.seed, colbase, P->d_iperm.get(), Vn.get(), b, s);
        colbase += b;
        src_cols = b;
        src_is_t = false;
    };
    int init_used = 0;
    if (o.init && o.init_cols > 0) {
        // the caller's start vectors (column-major, caller order) first, then
        // random columns; a column with a non-finite entry is left out (its
        // place keeps a random column)
        const int c0 = std::min(o.init_cols, b);
        if (!wk.init_tmp.get()) {
            wk.init_tmp.alloc((size_t)n * b);
            wk.init_bad.alloc(b);
        }
        DevBuf<double> &tmp = wk.init_tmp;
        DevBuf<int> &bad = wk.init_bad;
        LAP_HIP(hipMemcpyAsync(tmp.get(), o.init, sizeof(double) * n * c0,
                                o.init_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        if (fault_enabled("nan_init")) {
            static const double qnan = NAN;
            LAP_HIP(hipMemcpyAsync(tmp.get(), &qnan, sizeof(double), hipMemcpyHostToDevice, s));
        }
        LAP_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int) * c0, s));
        blk_nonfinite_cols(n, c0, tmp.get(), bad.get(), s);
        std::vector<int> hbad(c0);
        LAP_HIP(hipMemcpyAsync(hbad.data(), bad.get(), sizeof(int) * c0, hipMemcpyDeviceToHost, s));
        blk_random(n, b, o.seed, colbase, P->d_iperm.get(), Vn.get(), b, s);
        colbase += b;
        LAP_HIP(hipStreamSynchronize(s));
        for (int c = 0; c < c0; ++c)
            if (!hbad[c]) blk_cm_to_rm(n, 1, tmp.get() + (size_t)c * n, P->d_perm.get(), Vn.get() + init_used++, b, s);
        src_cols = b;
        src_is_t = false;
    } else if (nx < k) {
        random_block();
    }
    bool pcg_pending = false;
    int pcg_cols = 0;

    int pcg_last = 3;  // iterations of the last block PCG (its longest column)
    auto account_pcg = [&]() {
        if (!pcg_pending) return;
        int longest = 0;
        for (int c = 0; c < pcg_cols; ++c) {
            const int its = hp.h->brk[c] ? hp.h->brk[c] : hp.h->its[c];
            inner += its;
            mvp += its;
            longest = std::max(longest, its);
        }
        pcg_last = longest;
        pcg_pending = false;
    };

    // SVQB of Vn's `cur` columns; result into dest (ld); returns the kept
    // count.  Without `wait` the host does not read that count: all `cur`
    // columns are formed by CholQR (the dropped ones as zero columns) and
    // `cur` is returned; the last pass of a block is an SVQB that waits and
    // compacts.
    auto svqb = [&](int cur, double rel, double abs_thr, double *dest, int lddest, bool wait) -> int {
        ts_tn<double>(n, Vn.get(), b, cur, Vn.get(), b, cur, S.get(), b, nullptr, 0, 1.0, bs, s);
        if (!wait) {
            // the passes before the last: CholQR (pivoted Cholesky of the
            // Gram matrix, one wavefront) instead of its eigen-decomposition
            blk_cholqr(cur, S.get(), b, rel, abs_thr, M.get(), b, bst.get(), s);
            ts_nn<double>(n, Vn.get(), b, cur, M.get(), b, cur, dest, lddest, nullptr, 0, 1.0, 0.0, s);
            return cur;
        }
        jd_rr(cur, S.get(), b, Sth.get(), Sz.get(), b, nullptr, s, 0, nullptr, true);
        blk_svqb(cur, Sth.get(), Sz.get(), b, rel, abs_thr, M.get(), b, bst.get(), s);
        LAP_HIP(hipMemcpyAsync(hb.h, bst.get(), sizeof(BlockStatus), hipMemcpyDeviceToHost, s));
        if (pcg_pending) LAP_HIP(hipMemcpyAsync(hp.h, pw.st.get(), sizeof(BPcgState<T>), hipMemcpyDeviceToHost, s));
        LAP_HIP(hipStreamSynchronize(s));
        account_pcg();
        const int kept = hb.h->kept;
        if (kept > 0) ts_nn<double>(n, Vn.get(), b, cur, M.get(), b, kept, dest, lddest, nullptr, 0, 1.0, 0.0, s);
        return kept;
    };

    while (nx < k) {
        if (it >= kmax) {
            status = LAP_ENOCONV;
            set_error("outer-iteration limit " + std::to_string(kmax) + " reached with " + std::to_string(nx) +
                      " of " + std::to_string(k) + " pairs certified");
            break;
        }
        ++it;
        if (src_is_t) blk_to_f64<T>(n, src_cols, Tt.get(), src_cols, Vn.get(), b, s);
        // orthonormalize the new block: SVQB (scale), then twice
        // [classical Gram-Schmidt against [X V]; SVQB]; only the last SVQB
        // waits for its kept count (columns dropped before it stay as zero
        // columns until then)
        int cur = svqb(src_cols, 1e-20, 0.0, Vn.get(), b, false);
        for (int pass = 0; pass < 2 && cur > 0; ++pass) {
            const int nb = nx + m;
            if (nb > 0) {
                ts_tn<double>(n, XV.get(), ldb, nb, Vn.get(), b, cur, Cc.get(), ldb, nullptr, 0, 1.0, bs, s);
                ts_nn<double>(n, XV.get(), ldb, nb, Cc.get(), ldb, cur, Vn.get(), b, nullptr, 0, -1.0, 1.0, s);
            }
            double *dest = pass == 1 ? XV.get() + nx + m : Vn.get();
            const int ld = pass == 1 ? ldb : b;
            cur = svqb(cur, 1e-20, 1e-20, dest, ld, pass == 1);
        }
        if (cur == 0) {  // the corrections lay in span[X V]
            random_block();
            continue;
        }
        const int add = std::min(cur, mmax - m);
        double *Vb = XV.get() + nx;
        // W(:, m:m+add) = G V(:, m:m+add);  H border
        spmm<double>(*P, add, Vb + m, ldb, W.get() + m, mmax, nullptr, s);
        mvp += add;
        ts_tn<double>(n, Vb, ldb, m + add, W.get() + m, mmax, add, H.get() + (size_t)m * ldh, ldh, H.get() + m, ldh,
                      1.0, bs, s);
        m += add;

        bool need_pcg = true;
        int bu = 0;
        // H diagonal with ascending entries (as a lock leaves it): Rayleigh-Ritz
        // then returns Y = I exactly (no rotation, ranks in index order), so
        // U = V Y, GU = W Y and the rotations V Y, W Y(:, keep) are the
        // leading columns as they stand and are not formed
        bool y_ident = false;
        for (;;) {
            // warm start when theta and Y still diagonalize the leading block
            jd_rr(m, H.get(), ldh, theta.get(), Y.get(), mmax, nullptr, s, y_rows < m ? y_rows : 0, nullptr, true);
            y_rows = m;
            Vb = XV.get() + nx;
            bu = std::min(std::min(b, m), k - nx);
            if (y_ident) {
                blk_resid<T>(n, bu, Vb, ldb, W.get(), mmax, b, theta.get(), R.get(), Q.get(), ldq, nx, u0.get(), rs,
                             bst.get(), s);
            } else {
                ts_nn<double>(n, Vb, ldb, m, Y.get(), mmax, bu, U.get(), b, nullptr, 0, 1.0, 0.0, s);
                ts_nn<double>(n, W.get(), mmax, m, Y.get(), mmax, bu, GU.get(), b, nullptr, 0, 1.0, 0.0, s);
                blk_resid<T>(n, bu, U.get(), b, GU.get(), b, b, theta.get(), R.get(), Q.get(), ldq, nx, u0.get(), rs,
                             bst.get(), s);
            }
            LAP_HIP(hipMemcpyAsync(hb.h, bst.get(), sizeof(BlockStatus), hipMemcpyDeviceToHost, s));
            if (pcg_pending)
                LAP_HIP(hipMemcpyAsync(hp.h, pw.st.get(), sizeof(BPcgState<T>), hipMemcpyDeviceToHost, s));
            LAP_HIP(hipStreamSynchronize(s));
            account_pcg();
            const double th = hb.h->theta[0], rn = hb.h->rnorm[0];
            if (!std::isfinite(th) || !std::isfinite(rn))
                throw Failure{LAP_EDEVICE, "non-finite Ritz value or residual"};
            if (!converged_b(rn, th, tol)) break;
            jd_certify(*P, u0.get(), gu.get(), rs, jst.get(), s);
            ++mvp;
            LAP_HIP(hipMemcpyAsync(hj.h, jst.get(), sizeof(JDStatus), hipMemcpyDeviceToHost, s));
            LAP_HIP(hipStreamSynchronize(s));
            const double ct = hj.h->cert_theta, cr = hj.h->cert_rnorm;
            if (!converged_b(cr, ct, tol)) break;
            // lock: V <- V Y (the first column, u, joins X); W <- W Y(:, 2:m)
            if (!y_ident) ts_nn<double>(n, Vb, ldb, m, Y.get(), mmax, m, Vb, ldb, nullptr, 0, 1.0, 0.0, s);
            if (m > 1)
                ts_nn<double>(n, W.get(), mmax, m, Y.get() + mmax, mmax, m - 1, W.get(), mmax, nullptr, 0, 1.0, 0.0, s);
            jd_hdiag(H.get(), ldh, m - 1, theta.get(), 1, s);
            y_rows = 0;
            y_ident = true;
            lam.push_back(ct);
            resid.push_back(cr);
            ++nx;
            --m;
            if (nx >= k) { need_pcg = false; break; }
            if (m == 0) {
                need_pcg = false;
                random_block();
                break;
            }
        }
        if (nx >= k) break;
        if (!need_pcg) continue;
        // restart before the basis would outgrow m_max
        if (m + b > mmax) {
            const int keep = std::max(mmin, bu);
            Vb = XV.get() + nx;
            if (!y_ident) {
                ts_nn<double>(n, Vb, ldb, m, Y.get(), mmax, keep, Vb, ldb, nullptr, 0, 1.0, 0.0, s);
                ts_nn<double>(n, W.get(), mmax, m, Y.get(), mmax, keep, W.get(), mmax, nullptr, 0, 1.0, 0.0, s);
            }
            jd_hdiag(H.get(), ldh, keep, theta.get(), 0, s);
            m = keep;
            y_rows = 0;
        }
        // block PCG on the bu correction equations, Q = [X U], in up to two
        // segments: the first ends two iterations past the length of the
        // previous block PCG (all itmax when that one used them all); the
        // second runs only if some column is still iterating after it, so
        // equations that stop early do not pay for the whole itmax
        {
            const int q = nx + bu;
            const int split = std::min(o.itmax, pcg_last + 2);
            auto segment = [&](int i0, int i1) {
                auto enqueue = [&]() {
                    bpcg_enqueue<T>(*P, bu, brk_fault ? theta_fault.get() : theta.get(), Q.get(), ldq, q, R.get(), b,
                                    Tt.get(), pw, bs, o.itmax, i0, i1, o.rtol_pcg, s);
                };
                if (use_graph) LAP_HIP(hipGraphLaunch(graphs.get(q, bu, i0, i1, s, enqueue), s));
                else enqueue();
            };
            if (split == o.itmax && o.itmax > 2) {
                // one segment: launched as two graphs back to back, so the
                // device starts on the first two iterations while the host
                // still submits the rest
                segment(1, 2);
                segment(3, o.itmax);
            } else {
                segment(1, split);
            }
            if (split < o.itmax) {
                LAP_HIP(hipMemcpyAsync(hp.h->act[0], pw.st.get()->act[0], sizeof(int) * bu, hipMemcpyDeviceToHost, s));
                LAP_HIP(hipStreamSynchronize(s));
                bool any = false;
                for (int c = 0; c < bu; ++c) any |= hp.h->act[0][c] != 0;
                if (any) segment(split + 1, o.itmax);
            }
        }
        pcg_pending = true;
        pcg_cols = bu;
        src_is_t = true;
        src_cols = bu;
    }
    if (pcg_pending) {
        LAP_HIP(hipMemcpyAsync(hp.h, pw.st.get(), sizeof(BPcgState<T>), hipMemcpyDeviceToHost, s));
        LAP_HIP(hipStreamSynchronize(s));
        account_pcg();
    }

    // ---- output (as the single-vector solver)
    const int nconv = std::min(nx, k);
    emit_pairs(*P, nconv, XV.get(), ldb, 1, lam, resid, evals, evecs, evecs_on_device, res_out, wk.outbuf, s);
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

lap_status jd_block_solve(lap_plan *P, int k, double tol, const lap_eigs_opts &o, double *evals, double *evecs,
                          int evecs_on_device, double *res, lap_eigs_info *info) {
    if (o.precision == LAP_PREC_MIXED)
        return jdb_run<float>(P, k, tol, o, evals, evecs, evecs_on_device, res, info);
    return jdb_run<double>(P, k, tol, o, evals, evecs, evecs_on_device, res, info);
}

}  // namespace lapeig
