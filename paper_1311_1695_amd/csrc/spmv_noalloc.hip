// lap_spmv_noalloc: the Laplacian product of lap_spmv without any device
// allocation, for callers that cannot allocate (code under stream capture,
// tight serving loops).  Its scratch -- the renumbered copies of X and Y
// when the caller's vertex order is used, the shifts, and the per-chunk
// partial sums of the hub rows of a block product -- lives in one
// file-scope device array of kNoAllocScratchBytes, resolved once per device
// with hipGetSymbolAddress.
#include <cmath>
#include <mutex>
#include <new>
#include <string>

#include "lapeig_dev.h"

namespace {

constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's copy of `scratch` (each device holds
// its own copy at its own address); looked up on the first call per device.
unsigned char *scratch_on(int device) {
    LAP_REQUIRE(device >= 0 && device < kMaxDevices, LAP_EUNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        LAP_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        LAP_REQUIRE(ptr != nullptr, LAP_EDEVICE, "scratch symbol has no device address");
        g_scratch_ptr[device] = ptr;
    }
    return static_cast<unsigned char *>(g_scratch_ptr[device]);
}

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

template <typename T>
void product(const lap_plan &P, int b, const T *X, T *Y, const double *shift, bool plan_order, unsigned char *base,
             hipStream_t s) {
    const int n = P.n;
    const size_t vec = round256((size_t)n * b * sizeof(T));
    size_t at = 0;
    const T *xin = X;
    T *yout = Y;
    if (!plan_order) {
        xin = reinterpret_cast<const T *>(base + at);
        T *xp = reinterpret_cast<T *>(base + at);
        at += vec;
        yout = reinterpret_cast<T *>(base + at);
        at += vec;
        lapeig::permute_rows<T>(P.d_perm.get(), n, b, X, xp, s);
    }
    if (b == 1 && !shift) {
        lapeig::spmv<T>(P, xin, yout, 0.0, s);
    } else {
        T *part = P.g.nchunks > 0 ? reinterpret_cast<T *>(base + at) : nullptr;
        lapeig::spmm_part<T>(P, b, xin, b, yout, b, shift, part, s);
    }
    if (!plan_order) lapeig::permute_rows<T>(P.d_iperm.get(), n, b, yout, Y, s);
}

}  // namespace

extern "C" lap_status lap_spmv_noalloc(lap_plan *p, lap_dtype dt, int b, const void *X, void *Y, const double *shift,
                                       int flags, void *stream) {
    lapeig::set_error("");
    try {
        LAP_REQUIRE(p != nullptr, LAP_EINVAL, "plan is NULL");
        LAP_REQUIRE(dt == LAP_F32 || dt == LAP_F64, LAP_EINVAL, "dtype must be LAP_F32 or LAP_F64");
        LAP_REQUIRE(b >= 1 && b <= 64, LAP_EINVAL, "need 1 <= b <= 64");
        LAP_REQUIRE(X && Y, LAP_EINVAL, "X or Y is NULL");
        LAP_REQUIRE((flags & ~LAP_ORDER_PLAN) == 0, LAP_EINVAL, "unknown flags");
        if (shift)
            for (int c = 0; c < b; ++c) LAP_REQUIRE(std::isfinite(shift[c]), LAP_EINVAL, "non-finite shift");
        const bool plan_order = flags & LAP_ORDER_PLAN;
        const size_t es = dt == LAP_F32 ? sizeof(float) : sizeof(double);
        // layout of the scratch: [X copy | Y copy] (caller order only), the
        // hub-row chunk partials (block product only), the shifts
        const bool block = b > 1 || shift;
        const size_t need = (plan_order ? 0 : 2 * round256((size_t)p->n * b * es)) +
                            (block ? round256((size_t)p->g.nchunks * b * es) : 0) + (shift ? 512 : 0);
        LAP_REQUIRE(need <= kNoAllocScratchBytes, LAP_EINVAL,
                    "lap_spmv_noalloc needs " + std::to_string(need) + " bytes of scratch for n = " +
                        std::to_string(p->n) + ", b = " + std::to_string(b) + "; its fixed scratch holds " +
                        std::to_string(kNoAllocScratchBytes));
        int dev = -1;
        LAP_HIP(hipGetDevice(&dev));
        LAP_REQUIRE(dev == p->device, LAP_EINVAL, "the plan lives on another device than the current one");
        hipStream_t s = (hipStream_t)stream;
        unsigned char *base = scratch_on(dev);
        const double *sh = nullptr;
        if (shift) {
            double *d = reinterpret_cast<double *>(base + need - 512);
            LAP_HIP(hipMemcpyAsync(d, shift, sizeof(double) * b, hipMemcpyHostToDevice, s));
            sh = d;
        }
        if (dt == LAP_F32)
            product<float>(*p, b, (const float *)X, (float *)Y, sh, plan_order, base, s);
        else
            product<double>(*p, b, (const double *)X, (double *)Y, sh, plan_order, base, s);
        return LAP_OK;
    } catch (const lapeig::Failure &f) {
        lapeig::set_error(f.msg);
        return f.code;
    } catch (const std::bad_alloc &) {
        lapeig::set_error("host allocation failed");
        return LAP_ENOMEM;
    }
}
