// Measurement helper of bench.py (not part of the solver library): the rate
// at which the device serves random 4-byte reads from a vector of a given
// size.  Each thread forms its indices in registers (an integer hash mapped
// onto [0, size) by a multiply-shift), so no index stream competes with the reads and
// the indices have no locality; the sum of the values read is stored once
// per thread.  The result bounds what the neighbour gathers of a sparse
// product can reach on a graph without locality at that footprint.
#include <hip/hip_runtime.h>

namespace {

__device__ __forceinline__ unsigned mix32(unsigned x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

constexpr int kReads = 32;  // random reads per thread

__global__ __launch_bounds__(256) void k_random_reads(const float *__restrict__ x, unsigned size,
                                                      float *__restrict__ out, unsigned salt) {
    const unsigned t = blockIdx.x * 256u + threadIdx.x;
    unsigned h = mix32(t ^ salt);
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < kReads; ++j) {
        h = mix32(h + (unsigned)j);
        acc += x[(unsigned)(((unsigned long long)h * size) >> 32)];
    }
    out[t] = acc;
}

}  // namespace

// Random 4-byte reads per second over a vector of n_elems values
// (1 <= n_elems <= 2^28), at least `count`
// reads per launch (rounded up to whole workgroups), best of `reps` timed
// launches after one warm-up.  Allocates and frees its own device memory on
// the current device.  Returns 0, or -1 for bad arguments, -2 for a HIP error.
extern "C" int bench_random_reads(long long n_elems, long long count, int reps, double *reads_per_s) {
    if (n_elems < 1 || n_elems > (1LL << 28) || count < 1 || count > (1LL << 31) || reps < 1 || !reads_per_s)
        return -1;
    const long long size = n_elems;
    const long long threads = ((count + kReads - 1) / kReads + 255) / 256 * 256;
    float *x = nullptr, *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    float best = -1.f;
    if (hipMalloc(&x, size * sizeof(float)) != hipSuccess || hipMalloc(&out, threads * sizeof(float)) != hipSuccess ||
        hipMemset(x, 0, size * sizeof(float)) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        rc = -2;
    } else {
        const dim3 grid((unsigned)(threads / 256)), block(256);
        hipLaunchKernelGGL(k_random_reads, grid, block, 0, 0, x, (unsigned)size, out, 1u);
        for (int r = 0; r < reps && rc == 0; ++r) {
            float ms = 0.f;
            if (hipEventRecord(e0, 0) != hipSuccess) { rc = -2; break; }
            hipLaunchKernelGGL(k_random_reads, grid, block, 0, 0, x, (unsigned)size, out, 100u + (unsigned)r);
            if (hipEventRecord(e1, 0) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                rc = -2;
            else if (best < 0.f || ms < best)
                best = ms;
        }
        if (rc == 0 && hipGetLastError() != hipSuccess) rc = -2;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (x) (void)hipFree(x);
    if (out) (void)hipFree(out);
    if (rc == 0) *reads_per_s = (double)(threads * kReads) / (best * 1e-3);
    return rc;
}
