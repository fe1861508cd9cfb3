// Host side of the batched solver: validation, per-graph degree
// renumbering, packing (largest job first), one graph-captured persistent
// launch, and unpacking into the caller's vertex order.
#include <algorithm>
#include <memory>
#include <chrono>
#include <cmath>
#include <numeric>

#include "batch_kernels.h"

namespace lapeig {
// Device buffers and the captured launch of the last solve, reused while the
// key (k, options, precision, threshold) stays the same: a repeated solve is
// one graph launch and the copies of its results.
struct BatchWork {
    int k = 0, m_min = 0, m_max = 0, itmax = 0, kmax = 0, precision = -1, thr = -1;
    double tol = 0.0, rtol = 0.0;
    uint64_t seed = 0;
    std::vector<BGraph> gd;
    long long ov = 0;
    DevBuf<BGraph> dg;
    DevBuf<int> dord;
    DevBuf<unsigned> dq;
    DevBuf<double> ws64, outv, outl, outr, unp;
    DevBuf<double> ws32;  // PCG workspace, 8 bytes per element
    DevBuf<BResult> dres;
    hipStream_t s = nullptr;
    hipGraphExec_t exec = nullptr;
    ~BatchWork() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (s) (void)hipStreamDestroy(s);
    }
};
}  // namespace lapeig

struct lap_batch {
    int nb = 0;
    bool weighted = false;
    std::vector<int> n;                        // vertices per graph
    std::vector<std::vector<int>> perm;        // caller -> plan index, per graph
    std::vector<long long> rp_off, ci_off;
    std::vector<std::vector<int>> degs;        // row degrees in plan order (decreasing), per graph
    int long_threshold[2] = {32, 32};          // row-class threshold per precision (FP64, mixed)
    bool tuned[2] = {false, false};
    double tune_seconds[2] = {0.0, 0.0};
    lapeig::DevBuf<int> rowptr, col;
    lapeig::DevBuf<float> w32;
    lapeig::DevBuf<double> w64;
    lapeig::DevBuf<int> dperm;             // every graph's caller -> plan map, concatenated
    lapeig::DevBuf<long long> dperm_off;   // where graph g's map starts
    long long total_n = 0, total_nnz = 0;
    std::unique_ptr<lapeig::BatchWork> work;
};

namespace lapeig {

namespace {

// Row-class thresholds the autotuner times: rows above the threshold get a
// wavefront each, the others a thread each (the last candidate: none long).
constexpr int kBatchLongCandidates[] = {4, 8, 16, 32, 64, 128, 256, 1 << 30};

// rows of graph g with degree above thr (a prefix: degrees decrease)
int nlong_of(const lap_batch *B, int g, int thr) {
    const std::vector<int> &d = B->degs[g];
    return (int)(std::upper_bound(d.begin(), d.end(), thr, [](int t, int v) { return t > v; }) - d.begin());
}

void pack(lap_batch *B, const lap_csr *Ls, int nb) {
    for (int g = 0; g < nb; ++g) {
        try {
            validate_laplacian(&Ls[g]);
        } catch (const Failure &f) {
            throw Failure{f.code, "graph " + std::to_string(g) + ": " + f.msg};
        }
    }
    std::vector<int> rp_all, ci_all;
    std::vector<double> w_all;
    B->nb = nb;
    for (int g = 0; g < nb; ++g) {
        const lap_csr &L = Ls[g];
        for (int i = 0; i < L.n; ++i)
            for (int e = L.rowptr[i]; e < L.rowptr[i + 1]; ++e)
                if (L.col[e] != i && L.val[e] != -1.0) B->weighted = true;
    }
    for (int g = 0; g < nb; ++g) {
        const lap_csr &L = Ls[g];
        const int n = L.n;
        std::vector<int> deg(n, 0);
        for (int i = 0; i < n; ++i)
            for (int e = L.rowptr[i]; e < L.rowptr[i + 1]; ++e)
                if (L.col[e] != i) ++deg[i];
        std::vector<int> iperm(n);
        std::iota(iperm.begin(), iperm.end(), 0);
        std::stable_sort(iperm.begin(), iperm.end(), [&](int a, int b) { return deg[a] > deg[b]; });
        std::vector<int> perm(n);
        for (int p = 0; p < n; ++p) perm[iperm[p]] = p;
        // connectivity: the batched solver deflates the single zero pair e/sqrt(n)
        {
            std::vector<char> seen(n, 0);
            std::vector<int> q(n);
            int head = 0, tail = 0;
            q[tail++] = 0;
            seen[0] = 1;
            while (head < tail) {
                const int i = q[head++];
                for (int e = L.rowptr[i]; e < L.rowptr[i + 1]; ++e)
                    if (!seen[L.col[e]]) { seen[L.col[e]] = 1; q[tail++] = L.col[e]; }
            }
            LAP_REQUIRE(tail == n, LAP_EUNSUPPORTED,
                        "graph " + std::to_string(g) + " is not connected (the batched solver needs connected graphs)");
        }
        B->rp_off.push_back((long long)rp_all.size());
        B->ci_off.push_back((long long)ci_all.size());
        int acc = 0;
        std::vector<std::pair<int, double>> tmp;
        rp_all.push_back(0);
        for (int p = 0; p < n; ++p) {
            const int i = iperm[p];
            tmp.clear();
            for (int e = L.rowptr[i]; e < L.rowptr[i + 1]; ++e)
                if (L.col[e] != i) tmp.emplace_back(perm[L.col[e]], -L.val[e]);
            std::sort(tmp.begin(), tmp.end());
            for (auto &t : tmp) {
                ci_all.push_back(t.first);
                w_all.push_back(t.second);
            }
            acc += (int)tmp.size();
            rp_all.push_back(acc);
        }
        std::vector<int> dsorted(n);
        for (int p = 0; p < n; ++p) dsorted[p] = deg[iperm[p]];
        B->n.push_back(n);
        B->degs.push_back(std::move(dsorted));
        B->perm.push_back(std::move(perm));
        B->total_n += n;
        B->total_nnz += acc;
    }
    {
        std::vector<int> pall;
        std::vector<long long> poff;
        for (int g = 0; g < nb; ++g) {
            poff.push_back((long long)pall.size());
            pall.insert(pall.end(), B->perm[g].begin(), B->perm[g].end());
        }
        B->dperm.alloc(pall.size());
        B->dperm_off.alloc(poff.size());
        LAP_HIP(hipMemcpy(B->dperm.get(), pall.data(), sizeof(int) * pall.size(), hipMemcpyHostToDevice));
        LAP_HIP(hipMemcpy(B->dperm_off.get(), poff.data(), sizeof(long long) * poff.size(), hipMemcpyHostToDevice));
    }
    B->rowptr.alloc(rp_all.size());
    B->col.alloc(std::max<size_t>(ci_all.size(), 1));
    LAP_HIP(hipMemcpy(B->rowptr.get(), rp_all.data(), sizeof(int) * rp_all.size(), hipMemcpyHostToDevice));
    if (!ci_all.empty())
        LAP_HIP(hipMemcpy(B->col.get(), ci_all.data(), sizeof(int) * ci_all.size(), hipMemcpyHostToDevice));
    if (B->weighted) {
        std::vector<float> wf(w_all.begin(), w_all.end());
        B->w64.alloc(std::max<size_t>(w_all.size(), 1));
        B->w32.alloc(std::max<size_t>(w_all.size(), 1));
        LAP_HIP(hipMemcpy(B->w64.get(), w_all.data(), sizeof(double) * w_all.size(), hipMemcpyHostToDevice));
        LAP_HIP(hipMemcpy(B->w32.get(), wf.data(), sizeof(float) * wf.size(), hipMemcpyHostToDevice));
    }
}

}  // namespace

// Seconds per product pass over the whole batch (one workgroup per graph,
// the solver's row engine) for each threshold candidate: `reps` passes
// captured in a graph on a stream of our own, replayed three times, best
// replay.  Keeps the fastest candidate (ties: the smaller threshold).
int batch_autotune(lap_batch *B, bool mixed, int reps, double *best_seconds) {
    const int nb = B->nb;
    const size_t elem = mixed ? 4 : 8;
    std::vector<long long> voff(nb);
    long long tot = 0;
    for (int g = 0; g < nb; ++g) { voff[g] = tot; tot += B->n[g]; }
    DevBuf<char> x((size_t)tot * elem), y((size_t)tot * elem);
    DevBuf<long long> dvoff(nb);
    DevBuf<BGraph> dg(nb);
    LAP_HIP(hipMemset(x.get(), 0, (size_t)tot * elem));
    LAP_HIP(hipMemcpy(dvoff.get(), voff.data(), sizeof(long long) * nb, hipMemcpyHostToDevice));
    hipStream_t s = nullptr;
    LAP_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipGraphExec_t ge = nullptr;
    int best_thr = B->long_threshold[mixed ? 1 : 0];
    double best = 1e300;
    try {
        LAP_HIP(hipEventCreate(&e0));
        LAP_HIP(hipEventCreate(&e1));
        const float *w32 = B->weighted ? B->w32.get() : nullptr;
        const double *w64 = B->weighted ? B->w64.get() : nullptr;
        for (int thr : kBatchLongCandidates) {
            std::vector<BGraph> gd(nb);
            for (int g = 0; g < nb; ++g) {
                gd[g] = BGraph{};
                gd[g].n = B->n[g];
                gd[g].nlong = nlong_of(B, g, thr);
                gd[g].rp = B->rp_off[g];
                gd[g].ci = B->ci_off[g];
            }
            LAP_HIP(hipMemcpyAsync(dg.get(), gd.data(), sizeof(BGraph) * nb, hipMemcpyHostToDevice, s));
            auto pass = [&]() {
                batch_spmv_launch(dg.get(), nb, dvoff.get(), B->rowptr.get(), B->col.get(), w32, w64, mixed, x.get(),
                                  y.get(), nb, s);
            };
            pass();  // code objects loaded, caches warm
            LAP_HIP(hipStreamSynchronize(s));
            hipGraph_t gr = nullptr;
            LAP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            try {
                for (int r = 0; r < reps; ++r) pass();
            } catch (...) {
                (void)hipStreamEndCapture(s, &gr);
                if (gr) (void)hipGraphDestroy(gr);
                throw;
            }
            LAP_HIP(hipStreamEndCapture(s, &gr));
            const hipError_t ierr = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            LAP_HIP(ierr);
            double t = 1e300;
            for (int rep = 0; rep < 3; ++rep) {
                LAP_HIP(hipEventRecord(e0, s));
                LAP_HIP(hipGraphLaunch(ge, s));
                LAP_HIP(hipEventRecord(e1, s));
                LAP_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                LAP_HIP(hipEventElapsedTime(&ms, e0, e1));
                t = std::min(t, 1e-3 * ms / reps);
            }
            LAP_HIP(hipGraphExecDestroy(ge));
            ge = nullptr;
            if (t < best) { best = t; best_thr = thr; }
        }
    } catch (...) {
        if (ge) (void)hipGraphExecDestroy(ge);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamDestroy(s);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    LAP_HIP(hipStreamDestroy(s));
    B->long_threshold[mixed ? 1 : 0] = best_thr;
    B->tuned[mixed ? 1 : 0] = true;
    B->tune_seconds[mixed ? 1 : 0] = best;
    if (best_seconds) *best_seconds = best;
    return best_thr;
}

lap_status batch_create(const lap_csr *Ls, int nb, lap_batch **out) {
    LAP_REQUIRE(Ls && nb >= 1 && out, LAP_EINVAL, "need graphs, nb >= 1 and an output handle");
    lap_batch *B = new lap_batch();
    try {
        pack(B, Ls, nb);
    } catch (...) {
        delete B;
        throw;
    }
    *out = B;
    return LAP_OK;
}

void batch_destroy(lap_batch *B) { delete B; }

void batch_layout(const lap_batch *B, bool mixed, int *long_threshold, int *tuned) {
    *long_threshold = B->long_threshold[mixed ? 1 : 0];
    *tuned = B->tuned[mixed ? 1 : 0] ? 1 : 0;
}
int batch_total_n(const lap_batch *B) { return B ? (int)B->total_n : 0; }

lap_status batch_solve(lap_batch *B, int k, double tol, const lap_eigs_opts &o, double *evals, double *evecs,
                       int evecs_on_device,
                       double *res, lap_eigs_info *infos, hipStream_t user) {
    const auto t0 = std::chrono::steady_clock::now();
    LAP_REQUIRE(k >= 1 && k <= kBatchMaxK, LAP_EUNSUPPORTED, "the batched solver supports 1 <= k <= 8");
    LAP_REQUIRE(o.m_max <= kBatchMaxM && o.m_min >= 1 && o.m_min < o.m_max, LAP_EUNSUPPORTED,
                "the batched solver supports m_max <= 16");
    LAP_REQUIRE(o.block == 1, LAP_EUNSUPPORTED, "the batched solver corrects one pair per outer iteration");
    LAP_REQUIRE(o.precond == LAP_PRECOND_JACOBI, LAP_EUNSUPPORTED, "the batched solver preconditions with D^{-1}");
    const int nb = B->nb;
    for (int g = 0; g < nb; ++g)
        LAP_REQUIRE(k < B->n[g], LAP_EINVAL, "graph " + std::to_string(g) + " has n <= k");
    const bool mixed = o.precision == LAP_PREC_MIXED;
    // row classes: the autotuned threshold of this precision (tuned on first use)
    if (!B->tuned[mixed ? 1 : 0]) batch_autotune(B, mixed, 5, nullptr);
    const int thr = B->long_threshold[mixed ? 1 : 0];
    const int kmax = o.kmax > 0 ? o.kmax : 1000 * k;
    if (!B->work) B->work.reset(new BatchWork());
    BatchWork &W = *B->work;
    const bool same = W.exec && W.k == k && W.m_min == o.m_min && W.m_max == o.m_max && W.itmax == o.itmax &&
                      W.kmax == kmax && W.precision == o.precision && W.thr == thr && W.tol == tol &&
                      W.rtol == o.rtol_pcg && W.seed == o.seed;
    LAP_HIP(hipStreamSynchronize(user));
    if (!W.s) LAP_HIP(hipStreamCreateWithFlags(&W.s, hipStreamNonBlocking));
    hipStream_t s = W.s;
    if (!same) {
        if (W.exec) {
            LAP_HIP(hipGraphExecDestroy(W.exec));
            W.exec = nullptr;
        }
        // descriptors and workspace offsets
        W.gd.assign(nb, BGraph{});
        long long w64 = 0, w32 = 0, ov = 0;
        for (int g = 0; g < nb; ++g) {
            const long long n = B->n[g];
            BGraph &d = W.gd[g];
            d.n = (int)n;
            d.nlong = nlong_of(B, g, thr);
            d.k = k;
            d.pad = 0;
            d.rp = B->rp_off[g];
            d.ci = B->ci_off[g];
            d.w64 = w64;
            d.w32 = w32;
            d.out_vec = ov;
            d.out_val = (long long)g * k;
            w64 += n * (k + 2LL * o.m_max + 4);
            w32 += n * (k + 5LL);
            ov += n * k;
        }
        W.ov = ov;
        // largest job first
        std::vector<int> order(nb);
        std::iota(order.begin(), order.end(), 0);
        {
            std::vector<long long> nnz(nb);
            for (int g = 0; g < nb; ++g) nnz[g] = (g + 1 < nb ? B->ci_off[g + 1] : B->total_nnz) - B->ci_off[g];
            std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return nnz[a] > nnz[c]; });
        }
        if (W.dg.n < (size_t)nb) { W.dg.alloc(nb); W.dord.alloc(nb); W.dres.alloc(nb); }
        if (!W.dq.get()) W.dq.alloc(1);
        if (W.ws64.n < (size_t)w64) W.ws64.alloc(w64);
        if (W.ws32.n < (size_t)w32) W.ws32.alloc(w32);
        if (W.outv.n < (size_t)ov) { W.outv.alloc(ov); W.unp.alloc(ov); }
        if (W.outl.n < (size_t)nb * k) { W.outl.alloc((size_t)nb * k); W.outr.alloc((size_t)nb * k); }
        LAP_HIP(hipMemcpyAsync(W.dg.get(), W.gd.data(), sizeof(BGraph) * nb, hipMemcpyHostToDevice, s));
        LAP_HIP(hipMemcpyAsync(W.dord.get(), order.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s));
        BatchArgs a{};
        a.ngraphs = nb;
        a.graphs = W.dg.get();
        a.order = W.dord.get();
        a.queue = W.dq.get();
        a.rowptr = B->rowptr.get();
        a.col = B->col.get();
        a.w32 = B->weighted ? B->w32.get() : nullptr;
        a.w64 = B->weighted ? B->w64.get() : nullptr;
        a.ws64 = W.ws64.get();
        a.ws32 = W.ws32.get();
        a.out_vec = W.outv.get();
        a.out_val = W.outl.get();
        a.out_res = W.outr.get();
        a.results = W.dres.get();
        a.m_min = o.m_min;
        a.m_max = o.m_max;
        a.itmax = o.itmax;
        a.kmax = kmax;
        a.tol = tol;
        a.rtol_pcg = o.rtol_pcg;
        a.seed = o.seed;
        const int grid = std::min(nb, device_cu_count());
        // one graph: queue reset, the persistent solver, the eigenvectors
        // into the caller's order
        hipGraph_t graph = nullptr;
        LAP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
            batch_launch(a, mixed, B->weighted, grid, s);
            batch_unpack_launch(W.dg.get(), W.dres.get(), B->dperm.get(), B->dperm_off.get(), nb, W.outv.get(),
                                W.unp.get(), s);
        } catch (...) {
            (void)hipStreamEndCapture(s, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        LAP_HIP(hipStreamEndCapture(s, &graph));
        hipError_t err = hipGraphInstantiate(&W.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (err != hipSuccess) W.exec = nullptr;
        LAP_HIP(err);
        W.k = k; W.m_min = o.m_min; W.m_max = o.m_max; W.itmax = o.itmax; W.kmax = kmax;
        W.precision = o.precision; W.thr = thr; W.tol = tol; W.rtol = o.rtol_pcg; W.seed = o.seed;
    }
    LAP_HIP(hipGraphLaunch(W.exec, s));
    // results
    std::vector<BResult> hres(nb);
    std::vector<double> hl((size_t)nb * k), hr((size_t)nb * k);
    LAP_HIP(hipMemcpyAsync(hres.data(), W.dres.get(), sizeof(BResult) * nb, hipMemcpyDeviceToHost, s));
    LAP_HIP(hipMemcpyAsync(hl.data(), W.outl.get(), sizeof(double) * nb * k, hipMemcpyDeviceToHost, s));
    LAP_HIP(hipMemcpyAsync(hr.data(), W.outr.get(), sizeof(double) * nb * k, hipMemcpyDeviceToHost, s));
    if (evecs)
        LAP_HIP(hipMemcpyAsync(evecs, W.unp.get(), sizeof(double) * W.ov,
                               evecs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    LAP_HIP(hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    lap_status status = LAP_OK;
    for (int g = 0; g < nb; ++g) {
        const int nc = std::min(hres[g].nconv, k);
        if (nc < k) status = LAP_ENOCONV;
        for (int j = 0; j < k; ++j) {
            evals[(size_t)g * k + j] = j < nc ? hl[(size_t)g * k + j] : NAN;
            if (res) res[(size_t)g * k + j] = j < nc ? hr[(size_t)g * k + j] : NAN;
        }
        if (infos) {
            infos[g].nconv = nc;
            infos[g].ncomp = 1;
            infos[g].outer = hres[g].outer;
            infos[g].inner = hres[g].inner;
            infos[g].mvp = hres[g].mvp;
            infos[g].seconds = secs;
            infos[g].warm_start_used = 0;
        }
    }
    if (status == LAP_ENOCONV) set_error("some graphs reached the outer-iteration limit (see infos[g].nconv)");
    return status;
}

}  // namespace lapeig
