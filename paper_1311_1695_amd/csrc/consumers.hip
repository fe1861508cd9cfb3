// Consumers of the smallest eigenpairs (Section 2 of the paper):
//
// * spectral bisection: the relaxed minimum-cut problem with prescribed
//   sizes n1 + n2 = n is solved by x = (n1 - n2)/(2n) e + sqrt(n1 n2/n) v_2,
//   so the partition takes the n1 vertices where the Fiedler vector v_2 is
//   smallest (equal entries by vertex index); its cut size is the sum of
//   the weights of the edges between the two sides (x'Gx for x = +-1/2,
//   eq. (1)), bounded below by n1 n2 lambda_2 / n.
//   The n1-th smallest entry is found by a radix select: eight passes over
//   the bytes of an order-preserving 64-bit key of the entries (a histogram
//   of the entries that share the prefix found so far, per pass), then four
//   passes over the bytes of the vertex index among the entries equal to
//   it; each pass reads back 256 counts.
// * the pseudo-inverse approximations of current-flow betweenness:
//   T^(k) = sum_j (1/lambda_j) v_j v_j' over the positive pairs, and
//   S^(k) = (1/sigma)(I - sum over the zero pairs v v') + sum_j
//   (1/lambda_j - 1/sigma) v_j v_j', applied to a block of vectors:
//   C = V'X by deterministic partial sums, then Y = a X + V diag(c) C.
#include <cmath>
#include <vector>

#include "lapeig_dev.h"

namespace lapeig {

namespace {

constexpr int kBins = 256;

// order-preserving map of a finite double to an unsigned 64-bit key (-0 and
// +0 compare equal, so both map to the key of +0)
__device__ __forceinline__ unsigned long long order_key(double x) {
    if (x == 0.0) x = 0.0;
    unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// Histogram of byte `shift/8` of the keys (phase 0) or of the vertex index
// (phase 1, among keys equal to `prefix`) of the entries whose higher bytes
// equal `prefix` (phase 0: key >> (shift + 8) == prefix).  bad: counts
// non-finite entries (first pass only).
__global__ __launch_bounds__(kBlock) void k_select_hist(int n, const double *__restrict__ f, int phase, int shift,
                                                        unsigned long long prefix, unsigned long long key_eq,
                                                        unsigned *__restrict__ hist, unsigned *__restrict__ bad) {
    __shared__ unsigned h[kBins];
    for (int b = threadIdx.x; b < kBins; b += blockDim.x) h[b] = 0;
    __syncthreads();
    unsigned nbad = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double x = f[i];
        if (!isfinite(x)) {
            ++nbad;
            continue;
        }
        const unsigned long long k = order_key(x);
        if (phase == 0) {
            const unsigned long long hi = shift == 56 ? 0ull : (k >> (shift + 8));
            if (hi == prefix) atomicAdd(&h[(k >> shift) & 0xff], 1u);
        } else if (k == key_eq) {
            const unsigned long long idx = (unsigned long long)(unsigned)i;
            const unsigned long long hi = shift == 24 ? 0ull : (idx >> (shift + 8));
            if (hi == prefix) atomicAdd(&h[(idx >> shift) & 0xff], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBins; b += blockDim.x)
        if (h[b]) atomicAdd(&hist[b], h[b]);
    if (bad && nbad) atomicAdd(bad, nbad);
}

// part[i] = 0 for entries below the threshold pair (key_t, idx_t) in the
// order (key, index), 1 otherwise; also the plan-order copy of the labels.
__global__ __launch_bounds__(kBlock) void k_select_label(int n, const double *__restrict__ f,
                                                         unsigned long long key_t, long long idx_t,
                                                         const int *__restrict__ perm, int *__restrict__ part,
                                                         int *__restrict__ part_plan) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const unsigned long long k = order_key(f[i]);
        const int lab = (k < key_t || (k == key_t && (long long)i <= idx_t)) ? 0 : 1;
        part[i] = lab;
        part_plan[perm[i]] = lab;
    }
}

// partial sums of the weights of the cut edges (each edge once, from its
// lower endpoint), one row per workgroup
template <bool Wt>
__global__ __launch_bounds__(kBlock) void k_cut(int n, const int *__restrict__ rowptr, const int *__restrict__ col,
                                                const double *__restrict__ w, const int *__restrict__ lab,
                                                double *__restrict__ part_out) {
    double acc[1] = {0.0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int li = lab[i];
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const int j = col[e];
            if (j > i && lab[j] != li) acc[0] += Wt ? w[e] : 1.0;
        }
    }
    write_partials<double, 1>(acc, 1, part_out);
}

__global__ __launch_bounds__(kBlock) void k_fold1(const double *__restrict__ part, int nb, double *__restrict__ out) {
    __shared__ double t[1];
    fold_partials<double, 1>(part, nb, 1, t);
    if (threadIdx.x == 0) out[0] = t[0];
}

// C = V'x (k <= 64 values) as partial rows
__global__ __launch_bounds__(kBlock) void k_pinv_coef(int n, int k, const double *__restrict__ V,
                                                      const double *__restrict__ x, double *__restrict__ part_out) {
    double acc[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) acc[j] = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double xi = x[i];
#pragma unroll
        for (int j = 0; j < 64; ++j)
            if (j < k) acc[j] += V[(size_t)j * n + i] * xi;
    }
    write_partials<double, 64>(acc, k, part_out);
}

// y = a x + sum_j coef_j C_j v_j, C folded from the partial rows
__global__ __launch_bounds__(kBlock) void k_pinv_apply(int n, int k, const double *__restrict__ V,
                                                       const double *__restrict__ coef, double a,
                                                       const double *__restrict__ part_in, int nb,
                                                       const double *__restrict__ x, double *__restrict__ y) {
    __shared__ double c[64];
    fold_partials<double, 64>(part_in, nb, k, c);
    __shared__ double cc[64];
    if (threadIdx.x < 64) cc[threadIdx.x] = threadIdx.x < k ? coef[threadIdx.x] * c[threadIdx.x] : 0.0;
    __syncthreads();
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s = a * x[i];
        for (int j = 0; j < k; ++j) s += cc[j] * V[(size_t)j * n + i];
        y[i] = s;
    }
}

inline int cgrid(int n) {
    int g = (n + kBlock - 1) / kBlock;
    const int cap = 2 * device_cu_count();
    return g < 1 ? 1 : (g > cap ? cap : g);
}

}  // namespace

lap_status fiedler_bisect(lap_plan *P, const double *f, int n1, int *part, double *cut, hipStream_t s) {
    const int n = P->n;
    LAP_REQUIRE(n1 >= 0 && n1 <= n, LAP_EINVAL, "need 0 <= n1 <= n");
    DevBuf<unsigned> hist(kBins + 1);
    DevBuf<int> part_plan(n);
    const int g = cgrid(n);
    std::vector<unsigned> h(kBins + 1);
    unsigned long long key_t = 0;  // n1 = 0: nothing is below (key 0, index -1)
    long long idx_t = -1;
    // the first histogram pass also counts non-finite entries
    LAP_HIP(hipMemsetAsync(hist.get(), 0, sizeof(unsigned) * (kBins + 1), s));
    hipLaunchKernelGGL(k_select_hist, dim3(g), dim3(kBlock), 0, s, n, f, 0, 56, 0ull, 0ull, hist.get(),
                       hist.get() + kBins);
    LAP_HIP(hipGetLastError());
    LAP_HIP(hipMemcpyAsync(h.data(), hist.get(), sizeof(unsigned) * (kBins + 1), hipMemcpyDeviceToHost, s));
    LAP_HIP(hipStreamSynchronize(s));
    LAP_REQUIRE(h[kBins] == 0, LAP_EINVAL, "the vector holds non-finite entries");
    if (n1 == n) {
        key_t = ~0ull;  // every finite key is below
        idx_t = n;
    } else if (n1 > 0) {
        // rank of the last vertex of the first side, 0-based
        unsigned long long t = (unsigned long long)(n1 - 1);
        unsigned long long prefix = 0;
        for (int pass = 0; pass < 8; ++pass) {
            const int shift = 56 - 8 * pass;
            if (pass > 0) {  // pass 0's counts are those read above
                LAP_HIP(hipMemsetAsync(hist.get(), 0, sizeof(unsigned) * kBins, s));
                hipLaunchKernelGGL(k_select_hist, dim3(g), dim3(kBlock), 0, s, n, f, 0, shift, prefix, 0ull,
                                   hist.get(), nullptr);
                LAP_HIP(hipGetLastError());
                LAP_HIP(hipMemcpyAsync(h.data(), hist.get(), sizeof(unsigned) * kBins, hipMemcpyDeviceToHost, s));
                LAP_HIP(hipStreamSynchronize(s));
            }
            int b = 0;
            while (b < kBins - 1 && t >= h[b]) t -= h[b++];
            prefix = (prefix << 8) | (unsigned long long)b;
        }
        key_t = prefix;
        // among the entries equal to key_t, the t-th smallest index
        unsigned long long iprefix = 0;
        for (int pass = 0; pass < 4; ++pass) {
            const int shift = 24 - 8 * pass;
            LAP_HIP(hipMemsetAsync(hist.get(), 0, sizeof(unsigned) * kBins, s));
            hipLaunchKernelGGL(k_select_hist, dim3(g), dim3(kBlock), 0, s, n, f, 1, shift, iprefix, key_t,
                               hist.get(), nullptr);
            LAP_HIP(hipGetLastError());
            LAP_HIP(hipMemcpyAsync(h.data(), hist.get(), sizeof(unsigned) * kBins, hipMemcpyDeviceToHost, s));
            LAP_HIP(hipStreamSynchronize(s));
            int b = 0;
            while (b < kBins - 1 && t >= h[b]) t -= h[b++];
            iprefix = (iprefix << 8) | (unsigned long long)b;
        }
        idx_t = (long long)iprefix;
    }
    hipLaunchKernelGGL(k_select_label, dim3(g), dim3(kBlock), 0, s, n, f, key_t, idx_t, P->d_perm.get(), part,
                       part_plan.get());
    LAP_HIP(hipGetLastError());
    if (cut) {
        DevBuf<double> pc(g), tot(1);
        if (P->weighted)
            hipLaunchKernelGGL(k_cut<true>, dim3(g), dim3(kBlock), 0, s, n, P->d_rowptr.get(), P->d_col.get(),
                               P->d_w64.get(), part_plan.get(), pc.get());
        else
            hipLaunchKernelGGL(k_cut<false>, dim3(g), dim3(kBlock), 0, s, n, P->d_rowptr.get(), P->d_col.get(),
                               nullptr, part_plan.get(), pc.get());
        hipLaunchKernelGGL(k_fold1, dim3(1), dim3(kBlock), 0, s, pc.get(), g, tot.get());
        LAP_HIP(hipGetLastError());
        LAP_HIP(hipMemcpyAsync(cut, tot.get(), sizeof(double), hipMemcpyDeviceToHost, s));
    }
    LAP_HIP(hipStreamSynchronize(s));
    return LAP_OK;
}

lap_status pinv_apply(int n, int k, const double *evals, const double *V, double sigma, int b, const double *X,
                      double *Y, hipStream_t s) {
    LAP_REQUIRE(k >= 1 && k <= 64, LAP_EUNSUPPORTED, "need 1 <= k <= 64");
    std::vector<double> coef(k);
    for (int j = 0; j < k; ++j) {
        LAP_REQUIRE(std::isfinite(evals[j]) && evals[j] >= 0.0, LAP_EINVAL, "eigenvalues must be finite and >= 0");
        if (sigma > 0.0) coef[j] = evals[j] > 0.0 ? 1.0 / evals[j] - 1.0 / sigma : -1.0 / sigma;
        else coef[j] = evals[j] > 0.0 ? 1.0 / evals[j] : 0.0;
    }
    const double a = sigma > 0.0 ? 1.0 / sigma : 0.0;
    const int g = cgrid(n);
    DevBuf<double> dcoef(64), part((size_t)g * 64);
    LAP_HIP(hipMemcpyAsync(dcoef.get(), coef.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
    for (int c = 0; c < b; ++c) {
        const double *x = X + (size_t)c * n;
        hipLaunchKernelGGL(k_pinv_coef, dim3(g), dim3(kBlock), 0, s, n, k, V, x, part.get());
        hipLaunchKernelGGL(k_pinv_apply, dim3(g), dim3(kBlock), 0, s, n, k, V, dcoef.get(), a, part.get(), g, x,
                           Y + (size_t)c * n);
        LAP_HIP(hipGetLastError());
    }
    LAP_HIP(hipStreamSynchronize(s));
    return LAP_OK;
}

}  // namespace lapeig
