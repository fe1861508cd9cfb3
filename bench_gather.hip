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

// Random whole-row reads of an n x b FP32 row-major array: each row is read
// by b / 2 lanes with one 8-byte load each (the lane layout of the block
// product for even b), every lane has 8 reads in flight, and the row index
// comes from the same register hash, so again there is no index stream and no
// locality.  The rate bounds the neighbour gathers of the block product on a
// graph without locality at that footprint.
template <int GL>
__global__ __launch_bounds__(256) void k_random_rows(const float2 *__restrict__ x, unsigned nrows,
                                                     float *__restrict__ out, unsigned salt) {
    constexpr unsigned RPW = 64 / GL;
    const unsigned lane = threadIdx.x & 63u;
    const unsigned sub = lane / GL, c = lane % GL;
    const unsigned wave = (blockIdx.x * 256u + threadIdx.x) >> 6;
    float acc = 0.f;
    if (sub < RPW) {
        unsigned h = mix32((wave * RPW + sub) ^ salt);
        for (int j0 = 0; j0 < kReads; j0 += 8) {
            float2 v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                h = mix32(h + (unsigned)(j0 + k));
                const unsigned row = (unsigned)(((unsigned long long)h * nrows) >> 32);
                v[k] = x[(size_t)row * GL + c];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) acc += v[k].x + v[k].y;
        }
    }
    out[blockIdx.x * 256u + threadIdx.x] = acc;
}

}  // namespace

// Random row reads per second from an n_rows x b FP32 array (b in
// {8, 10, 16, 20}; 1 <= n_rows, n_rows * b <= 2^28), at least `count` row
// reads per launch, best of `reps` timed launches after one warm-up.
// Allocates and frees its own device memory on the current device.
// Returns 0, or -1 for bad arguments, -2 for a HIP error.
extern "C" int bench_random_rows(long long n_rows, int b, long long count, int reps, double *rows_per_s) {
    if (n_rows < 1 || (b != 8 && b != 10 && b != 16 && b != 20) || n_rows * b > (1LL << 28) || count < 1 ||
        count > (1LL << 31) || reps < 1 || !rows_per_s)
        return -1;
    const int gl = b / 2;
    const long long rpw = 64 / gl;                     // rows per wavefront and step
    const long long waves = (count + rpw * kReads - 1) / (rpw * kReads);
    const long long threads = (waves * 64 + 255) / 256 * 256;
    float *x = nullptr, *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    float best = -1.f;
    const size_t bytes = (size_t)n_rows * b * sizeof(float);
    if (hipMalloc(&x, bytes) != hipSuccess || hipMalloc(&out, threads * sizeof(float)) != hipSuccess ||
        hipMemset(x, 0, bytes) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        rc = -2;
    } else {
        const dim3 grid((unsigned)(threads / 256)), block(256);
        auto launch = [&](unsigned salt) {
            const float2 *xv = reinterpret_cast<const float2 *>(x);
            switch (gl) {
                case 4: hipLaunchKernelGGL(k_random_rows<4>, grid, block, 0, 0, xv, (unsigned)n_rows, out, salt); break;
                case 5: hipLaunchKernelGGL(k_random_rows<5>, grid, block, 0, 0, xv, (unsigned)n_rows, out, salt); break;
                case 8: hipLaunchKernelGGL(k_random_rows<8>, grid, block, 0, 0, xv, (unsigned)n_rows, out, salt); break;
                default: hipLaunchKernelGGL(k_random_rows<10>, grid, block, 0, 0, xv, (unsigned)n_rows, out, salt); break;
            }
        };
        launch(1u);
        for (int r = 0; r < reps && rc == 0; ++r) {
            float ms = 0.f;
            if (hipEventRecord(e0, 0) != hipSuccess) { rc = -2; break; }
            launch(100u + (unsigned)r);
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
    if (rc == 0) *rows_per_s = (double)(threads / 64 * rpw * kReads) / (best * 1e-3);
    return rc;
}

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
