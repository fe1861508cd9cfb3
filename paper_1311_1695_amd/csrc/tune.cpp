// Row-class autotuning of the Laplacian product.
//
// The product kernels split the rows (plan order, decreasing degree) into
// three classes at two degree thresholds: workgroup per row above `huge`,
// wavefront per row above `long`, 64-row column-major slices below.  Which
// thresholds are fastest depends on the degree distribution and on the
// block width, so they are chosen by timing: each candidate layout is built,
// a graph of back-to-back products is replayed between two HIP events, and
// the fastest layout is kept.  The choice can be cached in a small JSON file
// keyed by the device, the block width, the precision and a log2 histogram
// of the row degrees.
#include <algorithm>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <utility>

#include "jd_kernels.h"

namespace lapeig {

namespace {

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    EventPair() {
        LAP_HIP(hipEventCreate(&a));
        LAP_HIP(hipEventCreate(&b));
    }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Seconds per product of the current layout: `reps` launches captured into
// a graph on a stream of our own, replayed three times, best replay.
double time_product(lap_plan *P, lap_dtype dt, int b, int reps) {
    const int n = P->n;
    const size_t elem = dt == LAP_F32 ? 4 : 8;
    DevBuf<char> x((size_t)n * b * elem), y((size_t)n * b * elem);
    LAP_HIP(hipMemset(x.get(), 0, (size_t)n * b * elem));
    hipStream_t s = nullptr;
    LAP_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    double best = 1e300;
    try {
        auto launch = [&]() {
            if (dt == LAP_F32) {
                if (b == 1) spmv<float>(*P, (const float *)x.get(), (float *)y.get(), 0.0, s);
                else spmm<float>(*P, b, (const float *)x.get(), (float *)y.get(), nullptr, s);
            } else {
                if (b == 1) spmv<double>(*P, (const double *)x.get(), (double *)y.get(), 0.0, s);
                else spmm<double>(*P, b, (const double *)x.get(), (double *)y.get(), nullptr, s);
            }
        };
        launch();  // first launch outside the capture (code objects loaded)
        LAP_HIP(hipStreamSynchronize(s));
        LAP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
            for (int r = 0; r < reps; ++r) launch();
        } catch (...) {
            (void)hipStreamEndCapture(s, &g);
            throw;
        }
        LAP_HIP(hipStreamEndCapture(s, &g));
        LAP_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        EventPair ev;
        LAP_HIP(hipGraphLaunch(ge, s));  // warm
        for (int t = 0; t < 3; ++t) {
            LAP_HIP(hipEventRecord(ev.a, s));
            LAP_HIP(hipGraphLaunch(ge, s));
            LAP_HIP(hipEventRecord(ev.b, s));
            LAP_HIP(hipEventSynchronize(ev.b));
            float ms = 0.f;
            LAP_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
            best = std::min(best, 1e-3 * ms / reps);
        }
    } catch (...) {
        if (ge) (void)hipGraphExecDestroy(ge);
        if (g) (void)hipGraphDestroy(g);
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
        throw;
    }
    (void)hipGraphExecDestroy(ge);
    (void)hipGraphDestroy(g);
    LAP_HIP(hipStreamSynchronize(s));
    LAP_HIP(hipStreamDestroy(s));
    return best;
}

// Seconds per iteration launch of the projected PCG (the single-vector
// solver's inner loop) on the current layout: Q = the first q unit vectors,
// theta = 0 (the projected operator is then positive definite), rtol so
// small that no iteration stops; graphs of 6 and 16 iterations are replayed
// and their difference divided by 10.
template <typename T>
double time_pcg(lap_plan *P, int q) {
    const int n = P->n;
    PcgWork<T> w;
    w.ensure(n, q);
    DevBuf<T> Q((size_t)n * q), t(n);
    DevBuf<double> r(n), theta(1);
    LAP_HIP(hipMemset(Q.get(), 0, sizeof(T) * n * q));
    LAP_HIP(hipMemset(theta.get(), 0, sizeof(double)));
    const T one = T(1);
    for (int j = 0; j < q; ++j)
        LAP_HIP(hipMemcpy(Q.get() + (size_t)j * q + j, &one, sizeof(T), hipMemcpyHostToDevice));
    {
        std::vector<double> h(n);
        unsigned long long x = 0x9e3779b97f4a7c15ull;
        for (int i = 0; i < n; ++i) {
            x ^= x << 13; x ^= x >> 7; x ^= x << 17;
            h[i] = i < q ? 0.0 : (double)(x >> 11) * (1.0 / 9007199254740992.0) - 0.5;
        }
        LAP_HIP(hipMemcpy(r.get(), h.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    }
    hipStream_t s = nullptr;
    LAP_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    double per[2] = {0.0, 0.0};
    const int its[2] = {6, 16};
    try {
        EventPair ev;
        for (int v = 0; v < 2; ++v) {
            hipGraph_t g = nullptr;
            hipGraphExec_t ge = nullptr;
            pcg_enqueue<T>(*P, theta.get(), Q.get(), q, q, r.get(), t.get(), w, its[v], 1e-30, s);  // warm
            LAP_HIP(hipStreamSynchronize(s));
            LAP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            try {
                pcg_enqueue<T>(*P, theta.get(), Q.get(), q, q, r.get(), t.get(), w, its[v], 1e-30, s);
            } catch (...) {
                (void)hipStreamEndCapture(s, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            LAP_HIP(hipStreamEndCapture(s, &g));
            hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            LAP_HIP(e);
            double best = 1e300;
            for (int rep = 0; rep < 4; ++rep) {
                LAP_HIP(hipEventRecord(ev.a, s));
                LAP_HIP(hipGraphLaunch(ge, s));
                LAP_HIP(hipEventRecord(ev.b, s));
                LAP_HIP(hipEventSynchronize(ev.b));
                float ms = 0.f;
                LAP_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
                best = std::min(best, 1e-3 * ms);
            }
            (void)hipGraphExecDestroy(ge);
            per[v] = best;
        }
    } catch (...) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
        throw;
    }
    LAP_HIP(hipStreamSynchronize(s));
    LAP_HIP(hipStreamDestroy(s));
    return std::max(per[1] - per[0], 0.0) / (its[1] - its[0]);
}

// Rows of the long and huge classes for a pair of thresholds.
std::pair<int, int> classes(const lap_plan *P, int lt, int ht) {
    int nl = 0, nh = 0;
    const int n = P->n;
    while (nl < n && P->h_rowptr[nl + 1] - P->h_rowptr[nl] > lt) ++nl;
    while (nh < n && P->h_rowptr[nh + 1] - P->h_rowptr[nh] > ht) ++nh;
    return {nl, nh};
}

std::string cache_key(const lap_plan *P, lap_dtype dt, int b, int target) {
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&prop, P->device) == hipSuccess) arch = prop.gcnArchName;
    for (char &c : arch)
        if (c == '"' || c == '\\') c = '_';
    int hist[32] = {0};
    for (int r = 0; r < P->n; ++r) {
        int d = P->h_rowptr[r + 1] - P->h_rowptr[r], bin = 0;
        while (d > 0) { ++bin; d >>= 1; }
        ++hist[bin];
    }
    std::ostringstream k;
    k << arch << (target == LAP_TUNE_PCG ? "|pcg" : "|product") << "|b" << b << "|" << (dt == LAP_F32 ? "f32" : "f64") << "|w" << (P->weighted ? 1 : 0) << "|n"
      << P->n << "|nnz" << P->nnz_a << "|h";
    for (int i = 0; i < 32; ++i)
        if (hist[i]) k << i << ":" << hist[i] << ",";
    return k.str();
}

struct Entry {
    std::string key;
    int lt = 0, ht = 0;
    double us = 0.0;
};

// One entry per line: {"key": "...", "long": L, "huge": H, "us": U}
std::vector<Entry> read_cache(const char *path) {
    std::vector<Entry> out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t k0 = line.find("{\"key\": \"");
        if (k0 == std::string::npos) continue;
        const size_t ks = k0 + 9, ke = line.find('"', ks);
        const size_t l0 = line.find("\"long\": "), h0 = line.find("\"huge\": "), u0 = line.find("\"us\": ");
        if (ke == std::string::npos || l0 == std::string::npos || h0 == std::string::npos) continue;
        Entry e;
        e.key = line.substr(ks, ke - ks);
        e.lt = std::atoi(line.c_str() + l0 + 8);
        e.ht = std::atoi(line.c_str() + h0 + 8);
        e.us = u0 == std::string::npos ? 0.0 : std::atof(line.c_str() + u0 + 6);
        if (e.lt >= 1 && e.ht >= e.lt) out.push_back(e);
    }
    return out;
}

void write_cache(const char *path, const std::vector<Entry> &entries) {
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        LAP_REQUIRE(f.good(), LAP_EINVAL, std::string("cannot write the tuning cache ") + path);
        f << "{\"lapeig_row_classes\": 1, \"entries\": [\n";
        for (size_t i = 0; i < entries.size(); ++i) {
            char us[64];
            std::snprintf(us, sizeof(us), "%.4f", entries[i].us);
            f << "{\"key\": \"" << entries[i].key << "\", \"long\": " << entries[i].lt << ", \"huge\": "
              << entries[i].ht << ", \"us\": " << us << "}" << (i + 1 < entries.size() ? "," : "") << "\n";
        }
        f << "]}\n";
    }
    LAP_REQUIRE(std::rename(tmp.c_str(), path) == 0, LAP_EINVAL,
                std::string("cannot replace the tuning cache ") + path);
}

}  // namespace

void autotune(lap_plan *P, lap_dtype dt, int b, int target, const char *cache_path, lap_tune_info *info) {
    LAP_REQUIRE(dt == LAP_F32 || dt == LAP_F64, LAP_EINVAL, "dtype must be LAP_F32 or LAP_F64");
    LAP_REQUIRE(target == LAP_TUNE_PRODUCT || target == LAP_TUNE_PCG, LAP_EINVAL, "unknown tuning target");
    LAP_REQUIRE(b >= 1 && b <= 64, LAP_EINVAL, "block width must be in [1, 64]");
    LAP_REQUIRE(target != LAP_TUNE_PCG || b == 1, LAP_EINVAL, "the PCG target takes b = 1");
    LAP_REQUIRE(target != LAP_TUNE_PCG || P->n > 16, LAP_EINVAL, "the PCG target needs n > 16");
    const int def_lt = 32, def_ht = 512;
    const std::string key = cache_key(P, dt, b, target);
    lap_tune_info out{};
    if (cache_path) {
        for (const Entry &e : read_cache(cache_path)) {
            if (e.key != key) continue;
            if (P->long_threshold != e.lt || P->huge_threshold != e.ht) build_layout(P, e.lt, e.ht);
            out.long_threshold = e.lt;
            out.huge_threshold = e.ht;
            out.best_us = e.us;
            out.from_cache = 1;
            if (info) *info = out;
            return;
        }
    }
    const int reps = P->n >= 200000 ? 20 : 100;
    // candidate thresholds; pairs that classify the rows alike are timed once
    const int longs[] = {2, 4, 8, 16, 32, 64, 128};
    const int huges[] = {128, 256, 512, 1024, 2048, 8192};
    std::vector<std::pair<int, int>> cand, seen;
    cand.push_back({def_lt, def_ht});
    seen.push_back(classes(P, def_lt, def_ht));
    for (int lt : longs)
        for (int ht : huges) {
            if (ht < lt) continue;
            const auto c = classes(P, lt, ht);
            if (std::find(seen.begin(), seen.end(), c) != seen.end()) continue;
            seen.push_back(c);
            cand.push_back({lt, ht});
        }
    double best = 1e300, def_t = 0.0;
    std::pair<int, int> best_c = cand[0];
    for (size_t i = 0; i < cand.size(); ++i) {
        build_layout(P, cand[i].first, cand[i].second);
        const double t = target == LAP_TUNE_PCG
                             ? (dt == LAP_F32 ? time_pcg<float>(P, 8) : time_pcg<double>(P, 8))
                             : time_product(P, dt, b, reps);
        if (i == 0) def_t = t;
        if (t < best) {
            best = t;
            best_c = cand[i];
        }
    }
    if (P->long_threshold != best_c.first || P->huge_threshold != best_c.second)
        build_layout(P, best_c.first, best_c.second);
    out.long_threshold = best_c.first;
    out.huge_threshold = best_c.second;
    out.best_us = best * 1e6;
    out.default_us = def_t * 1e6;
    out.candidates = (int)cand.size();
    out.from_cache = 0;
    if (cache_path) {
        std::vector<Entry> entries = read_cache(cache_path);
        entries.erase(std::remove_if(entries.begin(), entries.end(), [&](const Entry &e) { return e.key == key; }),
                      entries.end());
        entries.push_back(Entry{key, best_c.first, best_c.second, best * 1e6});
        write_cache(cache_path, entries);
    }
    if (info) *info = out;
}

}  // namespace lapeig
