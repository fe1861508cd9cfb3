// Saving and loading the warm-start network (lap_mpnn_save, lap_mpnn_load):
// a versioned file with a one-line JSON header and a binary payload.
//
//   line 1   "LAPEIG-MPNN"
//   line 2   {"format": 1, "layers": L, "hidden": H, "random_channels": R,
//             "out_cols": P, "seed": S, "num_params": N, "adam_step": T,
//             "payload_bytes": 12 N, "fnv1a64": "<16 hex digits>"}
//   payload  N parameters, then Adam's first and second moments (N each),
//            float32 little-endian, in the flat order of lap_mpnn_get_params
//
// The checksum is FNV-1a (64-bit) of the payload bytes.  Loading checks the
// whole file on the host (magic, header fields, sizes, checksum, finite
// values) before any HIP call.
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "mpnn_internal.h"

namespace lapeig {
void set_error(const std::string &msg);
}

namespace {

using lapeig::Failure;

constexpr const char *kMagic = "LAPEIG-MPNN";
constexpr int kFormat = 1;
constexpr size_t kMaxHeader = 4096;

uint64_t fnv1a64(const unsigned char *p, size_t n) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

// Parameters the configuration implies: per layer a 2 F_in x F_out matrix
// and F_out biases, F_0 = 3 + random_channels, hidden width after, output last.
long long params_for(const lap_mpnn_config &c) {
    long long at = 0;
    int fin = 3 + c.random_channels;
    for (int l = 0; l <= c.layers; ++l) {
        const int fout = l < c.layers ? c.hidden : c.out_cols;
        at += 2LL * fin * fout + fout;
        fin = fout;
    }
    return at;
}

// The integer after "key": in a one-line JSON object (our own writer's form).
bool json_int(const std::string &hdr, const char *key, long long *out) {
    const std::string k = std::string("\"") + key + "\":";
    const size_t at = hdr.find(k);
    if (at == std::string::npos) return false;
    const char *p = hdr.c_str() + at + k.size();
    while (*p == ' ') ++p;
    char *end = nullptr;
    errno = 0;
    const long long v = std::strtoll(p, &end, 10);
    if (end == p || errno != 0) return false;
    *out = v;
    return true;
}

bool json_u64(const std::string &hdr, const char *key, uint64_t *out) {
    const std::string k = std::string("\"") + key + "\":";
    const size_t at = hdr.find(k);
    if (at == std::string::npos) return false;
    const char *p = hdr.c_str() + at + k.size();
    while (*p == ' ') ++p;
    if (*p < '0' || *p > '9') return false;
    char *end = nullptr;
    errno = 0;
    const unsigned long long v = std::strtoull(p, &end, 10);
    if (end == p || errno != 0) return false;
    *out = v;
    return true;
}

bool json_hex(const std::string &hdr, const char *key, uint64_t *out) {
    const std::string k = std::string("\"") + key + "\":";
    const size_t at = hdr.find(k);
    if (at == std::string::npos) return false;
    const char *p = hdr.c_str() + at + k.size();
    while (*p == ' ') ++p;
    if (*p != '"') return false;
    ++p;
    char *end = nullptr;
    errno = 0;
    const unsigned long long v = std::strtoull(p, &end, 16);
    if (end != p + 16 || *end != '"' || errno != 0) return false;
    *out = v;
    return true;
}

struct FileCloser {
    void operator()(FILE *f) const {
        if (f) std::fclose(f);
    }
};

}  // namespace

extern "C" {

lap_status lap_mpnn_save(const lap_mpnn *m, const char *path) {
    lapeig::set_error("");
    try {
        LAP_REQUIRE(m && path, LAP_EINVAL, "network or path is NULL");
        const long long N = m->nparams;
        std::vector<float> buf((size_t)3 * N);
        LAP_HIP(hipSetDevice(m->device));
        LAP_HIP(hipMemcpy(buf.data(), m->params.get(), sizeof(float) * N, hipMemcpyDeviceToHost));
        LAP_HIP(hipMemcpy(buf.data() + N, m->adam_m.get(), sizeof(float) * N, hipMemcpyDeviceToHost));
        LAP_HIP(hipMemcpy(buf.data() + 2 * N, m->adam_v.get(), sizeof(float) * N, hipMemcpyDeviceToHost));
        const size_t bytes = sizeof(float) * buf.size();
        const uint64_t sum = fnv1a64(reinterpret_cast<const unsigned char *>(buf.data()), bytes);
        char hdr[kMaxHeader];
        const int len = std::snprintf(
            hdr, sizeof hdr,
            "{\"format\": %d, \"layers\": %d, \"hidden\": %d, \"random_channels\": %d, \"out_cols\": %d, "
            "\"seed\": %llu, \"num_params\": %lld, \"adam_step\": %lld, \"payload_bytes\": %zu, "
            "\"dtype\": \"float32-le\", \"fnv1a64\": \"%016llx\"}\n",
            kFormat, m->cfg.layers, m->cfg.hidden, m->cfg.random_channels, m->cfg.out_cols,
            (unsigned long long)m->cfg.seed, N, m->step, bytes, (unsigned long long)sum);
        LAP_REQUIRE(len > 0 && (size_t)len < sizeof hdr, LAP_EDEVICE, "header too long");
        const std::string tmp = std::string(path) + ".tmp";
        {
            std::unique_ptr<FILE, FileCloser> f(std::fopen(tmp.c_str(), "wb"));
            LAP_REQUIRE(f != nullptr, LAP_EINVAL, "cannot open " + tmp + " for writing");
            bool ok = std::fprintf(f.get(), "%s\n", kMagic) > 0;
            ok = ok && std::fwrite(hdr, 1, (size_t)len, f.get()) == (size_t)len;
            ok = ok && std::fwrite(buf.data(), 1, bytes, f.get()) == bytes;
            ok = ok && std::fflush(f.get()) == 0;
            if (!ok) {
                f.reset();
                std::remove(tmp.c_str());
                throw Failure{LAP_EINVAL, "write to " + tmp + " failed"};
            }
        }
        if (std::rename(tmp.c_str(), path) != 0) {
            std::remove(tmp.c_str());
            throw Failure{LAP_EINVAL, std::string("cannot rename the saved network to ") + path};
        }
        return LAP_OK;
    } catch (const Failure &f) {
        lapeig::set_error(f.msg);
        return f.code;
    } catch (const std::bad_alloc &) {
        lapeig::set_error("host allocation failed");
        return LAP_ENOMEM;
    }
}

lap_status lap_mpnn_load(const char *path, lap_mpnn **out) {
    lapeig::set_error("");
    try {
        LAP_REQUIRE(path && out, LAP_EINVAL, "path or output pointer is NULL");
        *out = nullptr;
        std::unique_ptr<FILE, FileCloser> f(std::fopen(path, "rb"));
        LAP_REQUIRE(f != nullptr, LAP_EINVAL, std::string("cannot open ") + path);
        // magic line, then the header line
        char line[kMaxHeader];
        LAP_REQUIRE(std::fgets(line, sizeof line, f.get()) != nullptr, LAP_EINVAL, "empty network file");
        LAP_REQUIRE(std::strcmp(line, "LAPEIG-MPNN\n") == 0, LAP_EINVAL, "not a lapeig network file");
        LAP_REQUIRE(std::fgets(line, sizeof line, f.get()) != nullptr, LAP_EINVAL, "network file has no header");
        const std::string hdr(line);
        LAP_REQUIRE(!hdr.empty() && hdr.back() == '\n', LAP_EINVAL, "network file header too long");
        long long fmt = 0, layers = -1, hidden = -1, rc = -1, oc = -1, np = -1, step = -1, bytes = -1;
        uint64_t seed = 0, sum = 0;
        LAP_REQUIRE(json_int(hdr, "format", &fmt) && json_int(hdr, "layers", &layers) &&
                        json_int(hdr, "hidden", &hidden) && json_int(hdr, "random_channels", &rc) &&
                        json_int(hdr, "out_cols", &oc) && json_u64(hdr, "seed", &seed) &&
                        json_int(hdr, "num_params", &np) && json_int(hdr, "adam_step", &step) &&
                        json_int(hdr, "payload_bytes", &bytes) && json_hex(hdr, "fnv1a64", &sum),
                    LAP_EINVAL, "network file header lacks a field");
        LAP_REQUIRE(fmt == kFormat, LAP_EUNSUPPORTED, "network file format " + std::to_string(fmt) +
                                                          " (this build reads format 1)");
        LAP_REQUIRE(layers >= 0 && layers <= 8 && hidden >= 1 && hidden <= lapeig::kMpnnMaxCols && rc >= 0 &&
                        rc <= 16 && oc >= 1 && oc < lapeig::kMpnnMaxCols && step >= 0,
                    LAP_EINVAL, "network file header holds an invalid configuration");
        lap_mpnn_config cfg{(int32_t)layers, (int32_t)hidden, (int32_t)rc, (int32_t)oc, seed};
        LAP_REQUIRE(np == params_for(cfg), LAP_EINVAL, "num_params does not match the configuration");
        LAP_REQUIRE(bytes == 12 * np, LAP_EINVAL, "payload_bytes does not match num_params");
        std::vector<float> buf((size_t)3 * np);
        LAP_REQUIRE(std::fread(buf.data(), 1, (size_t)bytes, f.get()) == (size_t)bytes, LAP_EINVAL,
                    "network file is truncated");
        LAP_REQUIRE(std::fgetc(f.get()) == EOF, LAP_EINVAL, "network file has trailing bytes");
        LAP_REQUIRE(fnv1a64(reinterpret_cast<const unsigned char *>(buf.data()), (size_t)bytes) == sum, LAP_EINVAL,
                    "network file checksum mismatch");
        for (const float x : buf) LAP_REQUIRE(std::isfinite(x), LAP_EINVAL, "network file holds non-finite values");
        for (long long t = 0; t < np; ++t)
            LAP_REQUIRE(buf[(size_t)(2 * np + t)] >= 0.f, LAP_EINVAL, "negative second moment in network file");
        // the file is valid: build the network on the current device
        std::unique_ptr<lap_mpnn> m(new lap_mpnn);
        lapeig::mpnn_init(m.get(), cfg);
        LAP_REQUIRE(m->nparams == np, LAP_EDEVICE, "parameter layout mismatch");
        LAP_HIP(hipMemcpy(m->params.get(), buf.data(), sizeof(float) * np, hipMemcpyHostToDevice));
        LAP_HIP(hipMemcpy(m->adam_m.get(), buf.data() + np, sizeof(float) * np, hipMemcpyHostToDevice));
        LAP_HIP(hipMemcpy(m->adam_v.get(), buf.data() + 2 * np, sizeof(float) * np, hipMemcpyHostToDevice));
        m->step = step;
        *out = m.release();
        return LAP_OK;
    } catch (const Failure &f) {
        lapeig::set_error(f.msg);
        return f.code;
    } catch (const std::bad_alloc &) {
        lapeig::set_error("host allocation failed");
        return LAP_ENOMEM;
    }
}

}  // extern "C"
