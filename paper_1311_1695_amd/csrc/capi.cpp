// extern "C" entry points of lapeig.h: argument validation (on the host,
// before any HIP call), error codes and messages, order conversions.
#include <cmath>
#include <memory>
#include <new>
#include <vector>

#include "block_kernels.h"
#include "mpnn_internal.h"

namespace lapeig {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }
const char *get_error() { return g_last_error.c_str(); }

// Orthonormalize the b columns of W against Q and among themselves
// (Algorithm 2 step 2, block form).  Against Q: classical Gram-Schmidt twice,
// as one block product per pass (W -= Q (Q'W), on the matrix cores when
// b >= 2); within W: the single-vector CGS2 kernels column by column.
lap_status orth_block(int n, int q, const double *Q, int b, double *W, int *rank_out, hipStream_t s) {
    LAP_REQUIRE(b <= kMaxBasis - 1, LAP_EUNSUPPORTED, "b must not exceed 63");
    LAP_REQUIRE(q + b <= 160, LAP_EUNSUPPORTED, "q + b must not exceed 160");
    DevBuf<double> v(n);
    DevBuf<JDStatus> st(1);
    ReduceScratch rs;
    bool projected = false;
    std::vector<double> norm0(b, 0.0);
    if (q > 0 && b >= 2 && q <= 128 && b <= 32) {
        // column norms before the projection: the reference of the drop test
        {
            std::vector<double> hw((size_t)n * b);
            LAP_HIP(hipMemcpyAsync(hw.data(), W, sizeof(double) * n * b, hipMemcpyDeviceToHost, s));
            LAP_HIP(hipStreamSynchronize(s));
            for (int c = 0; c < b; ++c) {
                double acc = 0.0;
                for (int i = 0; i < n; ++i) acc += hw[(size_t)c * n + i] * hw[(size_t)c * n + i];
                norm0[c] = std::sqrt(acc);
            }
        }
        DevBuf<double> Qr((size_t)n * q), Wr((size_t)n * b), C((size_t)q * b);
        BlockScratch bs;
        bs.ensure();
        blk_cm_to_rm(n, q, Q, nullptr, Qr.get(), q, s);
        blk_cm_to_rm(n, b, W, nullptr, Wr.get(), b, s);
        for (int pass = 0; pass < 2; ++pass) {
            ts_tn<double>(n, Qr.get(), q, q, Wr.get(), b, b, C.get(), q, nullptr, 0, 1.0, bs, s);
            ts_nn<double>(n, Qr.get(), q, q, C.get(), q, b, Wr.get(), b, nullptr, 0, -1.0, 1.0, s);
        }
        blk_extract(n, b, Wr.get(), b, W, s);
        LAP_HIP(hipStreamSynchronize(s));
        projected = true;
    }
    // [Q | kept columns] for the column-by-column pass
    const int qb = projected ? 0 : q;
    LAP_REQUIRE(qb + b <= kMaxBasis - 1, LAP_EUNSUPPORTED, "q + b must not exceed 63 for one column");
    DevBuf<double> Bq((size_t)n * (qb + b));
    if (qb > 0) LAP_HIP(hipMemcpyAsync(Bq.get(), Q, sizeof(double) * n * qb, hipMemcpyDeviceToDevice, s));
    int rank = 0;
    JDStatus h;
    for (int c = 0; c < b; ++c) {
        jd_orth<double>(n, Bq.get(), qb + rank, W + (size_t)c * n, v.get(), rs, st.get(), s);
        jd_scale_copy(n, v.get(), Bq.get() + (size_t)(qb + rank) * n, st.get(), rs, s);
        LAP_HIP(hipMemcpyAsync(&h, st.get(), sizeof(JDStatus), hipMemcpyDeviceToHost, s));
        LAP_HIP(hipStreamSynchronize(s));
        const bool dropped = h.degenerate || (projected && !(h.orth_n1 > 1e-12 * norm0[c]));
        if (!dropped) ++rank;
    }
    if (rank > 0)
        LAP_HIP(hipMemcpyAsync(W, Bq.get() + (size_t)qb * n, sizeof(double) * n * rank, hipMemcpyDeviceToDevice, s));
    if (rank < b)
        LAP_HIP(hipMemsetAsync(W + (size_t)rank * n, 0, sizeof(double) * n * (b - rank), s));
    LAP_HIP(hipStreamSynchronize(s));
    if (rank_out) *rank_out = rank;
    return LAP_OK;
}

}  // namespace lapeig

using lapeig::Failure;

#define LAP_GUARD_BEGIN \
    lapeig::set_error("");  \
    try {
#define LAP_GUARD_END                                                       \
    }                                                                       \
    catch (const Failure &f) {                                              \
        lapeig::set_error(f.msg);                                           \
        return f.code;                                                      \
    }                                                                       \
    catch (const std::bad_alloc &) {                                        \
        lapeig::set_error("host allocation failed");                        \
        return LAP_ENOMEM;                                                  \
    }                                                                       \
    catch (...) {                                                           \
        lapeig::set_error("unexpected exception");                          \
        return LAP_EDEVICE;                                                 \
    }

extern "C" {

void lap_eigs_default_opts(lap_eigs_opts *o) {
    if (!o) return;
    o->m_min = 5;
    o->m_max = 10;
    o->itmax = 20;
    o->rtol_pcg = 1e-2;
    o->kmax = 0;
    o->precision = LAP_PREC_MIXED;
    o->block = 1;
    o->seed = 1;
    o->init = nullptr;
    o->init_cols = 0;
    o->init_on_device = 0;
    o->precond = LAP_PRECOND_JACOBI;
}

lap_status lap_mpnn_create(const lap_mpnn_config *cfg, lap_mpnn **out) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(cfg && out, LAP_EINVAL, "config or output pointer is NULL");
    *out = nullptr;
    std::unique_ptr<lap_mpnn> m(new lap_mpnn);
    lapeig::mpnn_init(m.get(), *cfg);
    *out = m.release();
    return LAP_OK;
    LAP_GUARD_END
}

void lap_mpnn_destroy(lap_mpnn *m) {
    if (!m) return;
    (void)hipSetDevice(m->device);
    delete m;
}

int64_t lap_mpnn_num_params(const lap_mpnn *m) { return m ? (int64_t)m->nparams : 0; }

lap_status lap_mpnn_get_config(const lap_mpnn *m, lap_mpnn_config *cfg) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(m && cfg, LAP_EINVAL, "network or config is NULL");
    *cfg = m->cfg;
    return LAP_OK;
    LAP_GUARD_END
}

lap_status lap_mpnn_get_params(const lap_mpnn *m, float *params) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(m && params, LAP_EINVAL, "network or params is NULL");
    LAP_HIP(hipSetDevice(m->device));
    LAP_HIP(hipMemcpy(params, m->params.get(), sizeof(float) * m->nparams, hipMemcpyDeviceToHost));
    return LAP_OK;
    LAP_GUARD_END
}

lap_status lap_mpnn_set_params(lap_mpnn *m, const float *params) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(m && params, LAP_EINVAL, "network or params is NULL");
    for (long long t = 0; t < m->nparams; ++t)
        LAP_REQUIRE(std::isfinite(params[t]), LAP_EINVAL, "params hold non-finite values");
    LAP_HIP(hipSetDevice(m->device));
    LAP_HIP(hipMemcpy(m->params.get(), params, sizeof(float) * m->nparams, hipMemcpyHostToDevice));
    LAP_HIP(hipMemset(m->adam_m.get(), 0, sizeof(float) * m->nparams));
    LAP_HIP(hipMemset(m->adam_v.get(), 0, sizeof(float) * m->nparams));
    m->step = 0;
    return LAP_OK;
    LAP_GUARD_END
}

static void check_net(const lap_mpnn *m, const lap_plan *p) {
    LAP_REQUIRE(m && p, LAP_EINVAL, "network or plan is NULL");
    LAP_REQUIRE(m->device == p->device, LAP_EINVAL, "network and plan live on different devices");
}

lap_status lap_mpnn_infer(lap_mpnn *m, lap_plan *p, uint64_t feature_seed, double *V0, void *stream) {
    LAP_GUARD_BEGIN
    check_net(m, p);
    LAP_REQUIRE(V0, LAP_EINVAL, "V0 is NULL");
    LAP_HIP(hipSetDevice(p->device));
    hipStream_t s = (hipStream_t)stream;
    lapeig::mpnn_forward(m, *p, feature_seed, s);
    lapeig::mpnn_output(m, *p, V0, s);
    LAP_HIP(hipStreamSynchronize(s));
    return LAP_OK;
    LAP_GUARD_END
}

lap_status lap_mpnn_loss_grad(lap_mpnn *m, lap_plan *p, uint64_t feature_seed, const double *X, int kx, double *loss,
                              float *grad, void *stream) {
    LAP_GUARD_BEGIN
    check_net(m, p);
    LAP_REQUIRE(X && loss, LAP_EINVAL, "X or loss is NULL");
    LAP_REQUIRE(kx >= 1 && m->cfg.out_cols + kx <= lapeig::kMpnnMaxCols, LAP_EINVAL,
                "need 1 <= kx and out_cols + kx <= 32");
    LAP_HIP(hipSetDevice(p->device));
    hipStream_t s = (hipStream_t)stream;
    *loss = lapeig::mpnn_loss_grad(m, *p, feature_seed, X, kx, s);
    if (grad)
        LAP_HIP(hipMemcpy(grad, m->grad.get(), sizeof(float) * m->nparams, hipMemcpyDeviceToHost));
    return LAP_OK;
    LAP_GUARD_END
}

lap_status lap_mpnn_train_step(lap_mpnn *m, lap_plan *p, uint64_t feature_seed, const double *X, int kx, float lr,
                               double *loss, void *stream) {
    LAP_GUARD_BEGIN
    check_net(m, p);
    LAP_REQUIRE(X, LAP_EINVAL, "X is NULL");
    LAP_REQUIRE(kx >= 1 && m->cfg.out_cols + kx <= lapeig::kMpnnMaxCols, LAP_EINVAL,
                "need 1 <= kx and out_cols + kx <= 32");
    LAP_REQUIRE(std::isfinite(lr) && lr > 0.f, LAP_EINVAL, "lr must be > 0");
    LAP_HIP(hipSetDevice(p->device));
    hipStream_t s = (hipStream_t)stream;
    const double l = lapeig::mpnn_loss_grad(m, *p, feature_seed, X, kx, s);
    lapeig::mpnn_adam(m, lr, s);
    LAP_HIP(hipStreamSynchronize(s));
    if (loss) *loss = l;
    return LAP_OK;
    LAP_GUARD_END
}

const char *lap_status_string(lap_status s) {
    switch (s) {
        case LAP_OK: return "LAP_OK";
        case LAP_EINVAL: return "LAP_EINVAL: invalid argument";
        case LAP_ENOTLAPLACIAN: return "LAP_ENOTLAPLACIAN: not the Laplacian of a simple weighted graph";
        case LAP_ENOMEM: return "LAP_ENOMEM: allocation failed";
        case LAP_EDEVICE: return "LAP_EDEVICE: HIP runtime error";
        case LAP_ENOCONV: return "LAP_ENOCONV: outer-iteration limit reached";
        case LAP_EUNSUPPORTED: return "LAP_EUNSUPPORTED: not supported by this build";
    }
    return "unknown lap_status";
}

const char *lap_last_error(void) { return lapeig::get_error(); }

lap_status lap_plan_create(const lap_csr *L, void *stream, lap_plan **out) {
    return lap_plan_create_ex(L, stream, LAP_PLAN_ORDER_HUB, out);
}

lap_status lap_plan_create_ex(const lap_csr *L, void *stream, int order, lap_plan **out) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(out != nullptr, LAP_EINVAL, "out is NULL");
    *out = nullptr;
    LAP_REQUIRE(order == LAP_PLAN_ORDER_HUB || order == LAP_PLAN_ORDER_CALLER, LAP_EINVAL,
                "order must be LAP_PLAN_ORDER_HUB or LAP_PLAN_ORDER_CALLER");
    lap_plan *p = new lap_plan();
    try {
        lapeig::build_plan(L, (hipStream_t)stream, p, order == LAP_PLAN_ORDER_HUB);
    } catch (...) {
        delete p;
        throw;
    }
    *out = p;
    return LAP_OK;
    LAP_GUARD_END
}

void lap_plan_destroy(lap_plan *p) { delete p; }

int32_t lap_plan_n(const lap_plan *p) { return p ? p->n : 0; }

lap_status lap_plan_perm(const lap_plan *p, int32_t *perm) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(p && perm, LAP_EINVAL, "plan or perm is NULL");
    for (int i = 0; i < p->n; ++i) perm[i] = p->perm[i];
    return LAP_OK;
    LAP_GUARD_END
}

lap_status lap_plan_set_layout(lap_plan *p, int32_t long_threshold, int32_t huge_threshold) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(p, LAP_EINVAL, "plan is NULL");
    LAP_REQUIRE(long_threshold >= 1 && huge_threshold >= long_threshold, LAP_EINVAL,
                "row-class thresholds must satisfy 1 <= long <= huge");
    lapeig::build_layout(p, long_threshold, huge_threshold);
    return LAP_OK;
    LAP_GUARD_END
}

lap_status lap_plan_layout(const lap_plan *p, int32_t *long_threshold, int32_t *huge_threshold) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(p && long_threshold && huge_threshold, LAP_EINVAL, "plan or output pointer is NULL");
    *long_threshold = p->long_threshold;
    *huge_threshold = p->huge_threshold;
    return LAP_OK;
    LAP_GUARD_END
}

lap_status lap_plan_autotune(lap_plan *p, lap_tune_target target, lap_dtype dtype, int32_t b, const char *cache_path,
                             lap_tune_info *info) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(p, LAP_EINVAL, "plan is NULL");
    LAP_REQUIRE(target == LAP_TUNE_PRODUCT || target == LAP_TUNE_PCG, LAP_EINVAL, "unknown tuning target");
    LAP_REQUIRE(dtype == LAP_F32 || dtype == LAP_F64, LAP_EINVAL, "dtype must be LAP_F32 or LAP_F64");
    LAP_REQUIRE(b >= 1 && b <= 64, LAP_EINVAL, "block width must be in [1, 64]");
    LAP_REQUIRE(target == LAP_TUNE_PRODUCT || b == 1, LAP_EINVAL, "the PCG target takes b = 1");
    lapeig::autotune(p, dtype, b, (int)target, cache_path, info);
    return LAP_OK;
    LAP_GUARD_END
}

static void check_opts(const lap_eigs_opts &o, int n) {
    LAP_REQUIRE(o.m_min >= 1 && o.m_max > o.m_min, LAP_EINVAL, "need 1 <= m_min < m_max");
    LAP_REQUIRE(o.itmax >= 1, LAP_EINVAL, "itmax must be >= 1");
    LAP_REQUIRE(o.rtol_pcg > 0.0 && std::isfinite(o.rtol_pcg), LAP_EINVAL, "rtol_pcg must be > 0");
    LAP_REQUIRE(o.precision == LAP_PREC_FP64 || o.precision == LAP_PREC_MIXED, LAP_EINVAL, "bad precision");
    LAP_REQUIRE(o.block >= 1, LAP_EINVAL, "block must be >= 1");
    LAP_REQUIRE(o.init_cols >= 0 && (o.init_cols == 0 || o.init != nullptr), LAP_EINVAL,
                "init_cols > 0 needs an init block");
    LAP_REQUIRE(o.init_on_device == 0 || o.init_on_device == 1, LAP_EINVAL, "init_on_device must be 0 or 1");
    LAP_REQUIRE(o.precond == LAP_PRECOND_JACOBI || o.precond == LAP_PRECOND_FSAI, LAP_EINVAL,
                "precond must be LAP_PRECOND_JACOBI or LAP_PRECOND_FSAI");
    LAP_REQUIRE(o.precond == LAP_PRECOND_JACOBI || o.block <= 1, LAP_EUNSUPPORTED,
                "the FSAI preconditioner is available to the single-vector solver (block = 1)");
    // columns of a start block with non-finite entries are not an error: the
    // solvers skip them (host and device blocks alike) and report the columns
    // used in lap_eigs_info.warm_start_used
    (void)n;
}

lap_status lap_eigs(lap_plan *p, int k, double tol, const lap_eigs_opts *opts, double *evals, double *evecs,
                    int evecs_on_device, double *res, lap_eigs_info *info) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(p != nullptr, LAP_EINVAL, "plan is NULL");
    LAP_REQUIRE(k >= 1 && k < p->n, LAP_EINVAL, "need 1 <= k < n");
    LAP_REQUIRE(tol > 0.0 && std::isfinite(tol), LAP_EINVAL, "tol must be > 0");
    LAP_REQUIRE(evals != nullptr, LAP_EINVAL, "evals is NULL");
    lap_eigs_opts o;
    if (opts) o = *opts;
    else lap_eigs_default_opts(&o);
    check_opts(o, p->n);
    LAP_HIP(hipSetDevice(p->device));
    return lapeig::jd_solve(p, k, tol, o, evals, evecs, evecs_on_device, res, info);
    LAP_GUARD_END
}

lap_status lap_eigs_dacg(lap_plan *p, int k, double tol, const lap_eigs_opts *opts, double *evals, double *evecs,
                         int evecs_on_device, double *res, lap_eigs_info *info) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(p != nullptr, LAP_EINVAL, "plan is NULL");
    LAP_REQUIRE(k >= 1 && k < p->n, LAP_EINVAL, "need 1 <= k < n");
    LAP_REQUIRE(tol > 0.0 && std::isfinite(tol), LAP_EINVAL, "tol must be > 0");
    LAP_REQUIRE(evals != nullptr, LAP_EINVAL, "evals is NULL");
    lap_eigs_opts o;
    if (opts) o = *opts;
    else lap_eigs_default_opts(&o);
    LAP_REQUIRE(o.precond == LAP_PRECOND_JACOBI || o.precond == LAP_PRECOND_FSAI, LAP_EINVAL, "bad precond");
    LAP_HIP(hipSetDevice(p->device));
    return lapeig::dacg_solve(p, k, tol, o, evals, evecs, evecs_on_device, res, info);
    LAP_GUARD_END
}

lap_status lap_eigs_irlm(lap_plan *p, int k, double tol, int m, double rtol_inner, int itmax_inner,
                         const lap_eigs_opts *opts, double *evals, double *evecs, int evecs_on_device, double *res,
                         lap_eigs_info *info) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(p != nullptr, LAP_EINVAL, "plan is NULL");
    LAP_REQUIRE(k >= 1 && k < p->n, LAP_EINVAL, "need 1 <= k < n");
    LAP_REQUIRE(tol > 0.0 && std::isfinite(tol), LAP_EINVAL, "tol must be > 0");
    LAP_REQUIRE(evals != nullptr, LAP_EINVAL, "evals is NULL");
    LAP_REQUIRE(m >= 0 && std::isfinite(rtol_inner) && itmax_inner >= 0, LAP_EINVAL,
                "need m >= 0, finite rtol_inner, itmax_inner >= 0");
    lap_eigs_opts o;
    if (opts) o = *opts;
    else lap_eigs_default_opts(&o);
    LAP_HIP(hipSetDevice(p->device));
    return lapeig::irlm_solve(p, k, tol, m, rtol_inner, itmax_inner, o, evals, evecs, evecs_on_device, res, info);
    LAP_GUARD_END
}

lap_status lap_eigs_csr(const lap_csr *L, int k, double tol, const lap_eigs_opts *opts, double *evals,
                        double *evecs, double *res, lap_eigs_info *info) {
    lap_plan *p = nullptr;
    lap_status s = lap_plan_create(L, nullptr, &p);
    if (s != LAP_OK) return s;
    s = lap_eigs(p, k, tol, opts, evals, evecs, 0, res, info);
    lap_plan_destroy(p);
    return s;
}

lap_status lap_spmv(lap_plan *p, lap_dtype dt, int b, const void *X, void *Y, const double *shift, int flags,
                    void *stream) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(p != nullptr, LAP_EINVAL, "plan is NULL");
    LAP_REQUIRE(dt == LAP_F32 || dt == LAP_F64, LAP_EINVAL, "dtype must be LAP_F32 or LAP_F64");
    LAP_REQUIRE(b >= 1 && b <= 64, LAP_EINVAL, "need 1 <= b <= 64");
    LAP_REQUIRE(X && Y, LAP_EINVAL, "X or Y is NULL");
    LAP_REQUIRE((flags & ~LAP_ORDER_PLAN) == 0, LAP_EINVAL, "unknown flags");
    if (shift)
        for (int c = 0; c < b; ++c) LAP_REQUIRE(std::isfinite(shift[c]), LAP_EINVAL, "non-finite shift");
    hipStream_t s = (hipStream_t)stream;
    const int n = p->n;
    const size_t es = dt == LAP_F32 ? sizeof(float) : sizeof(double);
    const double *sh = nullptr;
    if (shift) {
        if (!p->d_shift.get()) p->d_shift.alloc(64);
        LAP_HIP(hipMemcpyAsync(p->d_shift.get(), shift, sizeof(double) * b, hipMemcpyHostToDevice, s));
        sh = p->d_shift.get();
    }
    const bool plan_order = flags & LAP_ORDER_PLAN;
    const void *xin = X;
    void *yout = Y;
    if (!plan_order) {
        const size_t bytes = (size_t)n * b * es;
        if (p->tmp_x.n < bytes) { p->tmp_x.alloc(bytes); p->tmp_y.alloc(bytes); }
        xin = p->tmp_x.get();
        yout = p->tmp_y.get();
        if (dt == LAP_F32)
            lapeig::permute_rows<float>(p->d_perm.get(), n, b, (const float *)X, (float *)p->tmp_x.get(), s);
        else
            lapeig::permute_rows<double>(p->d_perm.get(), n, b, (const double *)X, (double *)p->tmp_x.get(), s);
    }
    if (b == 1 && !sh) {
        if (dt == LAP_F32) lapeig::spmv<float>(*p, (const float *)xin, (float *)yout, 0.0, s);
        else lapeig::spmv<double>(*p, (const double *)xin, (double *)yout, 0.0, s);
    } else {
        if (dt == LAP_F32) lapeig::spmm<float>(*p, b, (const float *)xin, (float *)yout, sh, s);
        else lapeig::spmm<double>(*p, b, (const double *)xin, (double *)yout, sh, s);
    }
    if (!plan_order) {
        if (dt == LAP_F32)
            lapeig::permute_rows<float>(p->d_iperm.get(), n, b, (const float *)yout, (float *)Y, s);
        else
            lapeig::permute_rows<double>(p->d_iperm.get(), n, b, (const double *)yout, (double *)Y, s);
    }
    return LAP_OK;
    LAP_GUARD_END
}

lap_status lap_orth(lap_dtype dt, int n, int q, const double *Q, int b, double *W, int *rank_out, void *stream) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(dt == LAP_F64, LAP_EINVAL, "lap_orth works in double precision (LAP_F64)");
    LAP_REQUIRE(n >= 1 && q >= 0 && b >= 1, LAP_EINVAL, "need n >= 1, q >= 0, b >= 1");
    LAP_REQUIRE(q == 0 || Q, LAP_EINVAL, "Q is NULL");
    LAP_REQUIRE(W != nullptr, LAP_EINVAL, "W is NULL");
    return lapeig::orth_block(n, q, Q, b, W, rank_out, (hipStream_t)stream);
    LAP_GUARD_END
}

lap_status lap_sym_eig(int m, const double *H, double *theta, double *Y, int *sweeps_out, void *stream) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(m >= 1 && m <= 96, LAP_EINVAL, "need 1 <= m <= 96");
    LAP_REQUIRE(H && theta && Y, LAP_EINVAL, "H, theta or Y is NULL");
    const hipStream_t s = (hipStream_t)stream;
    lapeig::DevBuf<lapeig::JDStatus> st;
    if (sweeps_out) st.alloc(1);
    // H is only read: no border rows are passed, so nothing is written back
    lapeig::jd_rr(m, const_cast<double *>(H), m, theta, Y, m, sweeps_out ? st.get() : nullptr, s);
    if (sweeps_out) {
        lapeig::JDStatus hs;
        LAP_HIP(hipMemcpyAsync(&hs, st.get(), sizeof(hs), hipMemcpyDeviceToHost, s));
        LAP_HIP(hipStreamSynchronize(s));
        *sweeps_out = hs.rr_sweeps;
    }
    return LAP_OK;
    LAP_GUARD_END
}

lap_status lap_pcg(lap_plan *p, lap_dtype dt, int b, const double *theta, const double *Q, int q, const double *R,
                   double *T, int itmax, double rtol, int *iters_out, int flags, void *stream) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(p != nullptr, LAP_EINVAL, "plan is NULL");
    LAP_REQUIRE(dt == LAP_F32 || dt == LAP_F64, LAP_EINVAL, "dtype must be LAP_F32 or LAP_F64");
    LAP_REQUIRE(b >= 1 && b <= 32, LAP_EINVAL, "need 1 <= b <= 32");
    LAP_REQUIRE(q >= 0 && (q == 0 || Q), LAP_EINVAL, "bad Q");
    LAP_REQUIRE(theta && R && T, LAP_EINVAL, "theta, R or T is NULL");
    LAP_REQUIRE(itmax >= 1, LAP_EINVAL, "itmax must be >= 1");
    LAP_REQUIRE(rtol > 0.0 && std::isfinite(rtol), LAP_EINVAL, "rtol must be > 0");
    LAP_REQUIRE((flags & ~(LAP_ORDER_PLAN | LAP_PCG_FSAI)) == 0, LAP_EINVAL, "unknown flags");
    for (int c = 0; c < b; ++c) LAP_REQUIRE(std::isfinite(theta[c]), LAP_EINVAL, "non-finite theta");
    return lapeig::pcg_entry(p, dt, b, theta, Q, q, R, T, itmax, rtol, iters_out, flags, (hipStream_t)stream);
    LAP_GUARD_END
}

lap_status lap_fiedler_bisect(lap_plan *p, const double *fiedler, int n1, int32_t *part, double *cut,
                              void *stream) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(p != nullptr, LAP_EINVAL, "plan is NULL");
    LAP_REQUIRE(fiedler && part, LAP_EINVAL, "fiedler or part is NULL");
    LAP_REQUIRE(n1 >= 0 && n1 <= p->n, LAP_EINVAL, "need 0 <= n1 <= n");
    return lapeig::fiedler_bisect(p, fiedler, n1, part, cut, (hipStream_t)stream);
    LAP_GUARD_END
}

lap_status lap_pinv_apply(int n, int k, const double *evals, const double *evecs, double sigma, int b,
                          const double *X, double *Y, void *stream) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(n >= 1 && k >= 1 && b >= 1, LAP_EINVAL, "need n, k, b >= 1");
    LAP_REQUIRE(k <= 64, LAP_EUNSUPPORTED, "k must not exceed 64");
    LAP_REQUIRE(evals && evecs && X && Y, LAP_EINVAL, "evals, evecs, X or Y is NULL");
    LAP_REQUIRE(std::isfinite(sigma) && sigma >= 0.0, LAP_EINVAL, "sigma must be 0 (T) or > 0 (S)");
    for (int j = 0; j < k; ++j)
        LAP_REQUIRE(std::isfinite(evals[j]) && evals[j] >= 0.0, LAP_EINVAL, "eigenvalues must be finite and >= 0");
    return lapeig::pinv_apply(n, k, evals, evecs, sigma, b, X, Y, (hipStream_t)stream);
    LAP_GUARD_END
}

lap_status lap_batch_create(const lap_csr *Ls, int nb, lap_batch **out) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(out != nullptr, LAP_EINVAL, "out is NULL");
    *out = nullptr;
    return lapeig::batch_create(Ls, nb, out);
    LAP_GUARD_END
}

void lap_batch_destroy(lap_batch *b) { lapeig::batch_destroy(b); }

int32_t lap_batch_total_n(const lap_batch *b) { return lapeig::batch_total_n(b); }

lap_status lap_batch_autotune(lap_batch *b, int precision, int32_t *long_threshold, double *seconds) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(b != nullptr, LAP_EINVAL, "batch is NULL");
    LAP_REQUIRE(precision == LAP_PREC_FP64 || precision == LAP_PREC_MIXED, LAP_EINVAL, "unknown precision");
    double secs = 0.0;
    const int thr = lapeig::batch_autotune(b, precision == LAP_PREC_MIXED, 5, &secs);
    if (long_threshold) *long_threshold = thr;
    if (seconds) *seconds = secs;
    return LAP_OK;
    LAP_GUARD_END
}

lap_status lap_batch_layout(const lap_batch *b, int precision, int32_t *long_threshold, int32_t *tuned) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(b && long_threshold && tuned, LAP_EINVAL, "batch or output pointer is NULL");
    LAP_REQUIRE(precision == LAP_PREC_FP64 || precision == LAP_PREC_MIXED, LAP_EINVAL, "unknown precision");
    int thr = 0, tu = 0;
    lapeig::batch_layout(b, precision == LAP_PREC_MIXED, &thr, &tu);
    *long_threshold = thr;
    *tuned = tu;
    return LAP_OK;
    LAP_GUARD_END
}

lap_status lap_batch_eigs(lap_batch *b, int k, double tol, const lap_eigs_opts *opts, double *evals, double *evecs,
                          double *res, lap_eigs_info *infos, void *stream) {
    return lap_batch_eigs_ex(b, k, tol, opts, evals, evecs, 0, res, infos, stream);
}

lap_status lap_batch_eigs_ex(lap_batch *b, int k, double tol, const lap_eigs_opts *opts, double *evals,
                             double *evecs, int evecs_on_device, double *res, lap_eigs_info *infos, void *stream) {
    LAP_GUARD_BEGIN
    LAP_REQUIRE(b != nullptr, LAP_EINVAL, "batch is NULL");
    LAP_REQUIRE(tol > 0.0 && std::isfinite(tol), LAP_EINVAL, "tol must be > 0");
    LAP_REQUIRE(evals != nullptr, LAP_EINVAL, "evals is NULL");
    lap_eigs_opts o;
    if (opts) o = *opts;
    else lap_eigs_default_opts(&o);
    check_opts(o, 0);
    return lapeig::batch_solve(b, k, tol, o, evals, evecs, evecs_on_device, res, infos, (hipStream_t)stream);
    LAP_GUARD_END
}

lap_status lap_eigs_batch(const lap_csr *Ls, int nb, int k, double tol, const lap_eigs_opts *opts, double *evals,
                          double *evecs, double *res, lap_eigs_info *infos, void *stream) {
    lap_batch *b = nullptr;
    lap_status s = lap_batch_create(Ls, nb, &b);
    if (s != LAP_OK) return s;
    s = lap_batch_eigs(b, k, tol, opts, evals, evecs, res, infos, stream);
    lap_batch_destroy(b);
    return s;
}

}  // extern "C"
