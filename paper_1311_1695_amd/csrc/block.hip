// Block Jacobi-Davidson kernels: b corrections per outer iteration.
//
// Tall-skinny products on the matrix cores.  With n rows and at most a few
// dozen columns these are HBM-bound (a few flops per byte), but the 16x16x4
// MFMA tiles keep every loaded element's multiply-adds in one instruction:
//   k_ts_tn  C = A'B   (A n x ka, B n x kb, row-major): each wavefront
//            accumulates 16x16 tiles over its 4-row chunks, the four
//            wavefronts are summed in LDS, each workgroup writes one partial
//            tile set, and k_ts_reduce adds the partials (one wavefront per
//            output element, in a fixed order).
//   k_ts_nn  Out = alpha A C + (addend | beta Out)  (C ka x kb column-major,
//            staged in LDS): each wavefront owns 16-row blocks, so Out may
//            overlap A (in-place rotation of a basis).
// (MFMA operand and accumulator layouts: see Mfma in lapeig_dev.h.)
#include "lapeig_dev.h"
#include "block_kernels.h"

namespace lapeig {

namespace {

template <typename T, int TI, int TJ>
__global__ __launch_bounds__(kBlock) void k_ts_tn(int n, const T *__restrict__ A, int lda, int ka,
                                                  const T *__restrict__ B, int ldb, int kb, T *__restrict__ part) {
    using V4 = typename Mfma<T>::v4;
    constexpr int PI = TI * 16, PJ = TJ * 16;
    __shared__ T red[PI * PJ];
    const int lane = lane_id(), wave = wave_id();
    const int mi = lane & 15, kk = lane >> 4;
    V4 acc[TI][TJ];
#pragma unroll
    for (int ti = 0; ti < TI; ++ti)
#pragma unroll
        for (int tj = 0; tj < TJ; ++tj) acc[ti][tj] = V4{T(0), T(0), T(0), T(0)};
    const int step = gridDim.x * kWavesPerBlock * 4;
    for (int k0 = (blockIdx.x * kWavesPerBlock + wave) * 4; k0 < n; k0 += step) {
        const int row = k0 + kk;
        const bool ok = row < n;
        T a[TI], b[TJ];
#pragma unroll
        for (int ti = 0; ti < TI; ++ti) {
            const int col = ti * 16 + mi;
            a[ti] = (ok && col < ka) ? A[(size_t)row * lda + col] : T(0);
        }
#pragma unroll
        for (int tj = 0; tj < TJ; ++tj) {
            const int col = tj * 16 + mi;
            b[tj] = (ok && col < kb) ? B[(size_t)row * ldb + col] : T(0);
        }
#pragma unroll
        for (int ti = 0; ti < TI; ++ti)
#pragma unroll
            for (int tj = 0; tj < TJ; ++tj) acc[ti][tj] = Mfma<T>::mac(a[ti], b[tj], acc[ti][tj]);
    }
    // sum the four wavefronts in a fixed order
    for (int w = 0; w < kWavesPerBlock; ++w) {
        if (wave == w) {
#pragma unroll
            for (int ti = 0; ti < TI; ++ti)
#pragma unroll
                for (int tj = 0; tj < TJ; ++tj)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = ti * 16 + Mfma<T>::row(lane, r), j = tj * 16 + (lane & 15);
                        red[i * PJ + j] = (w == 0 ? T(0) : red[i * PJ + j]) + acc[ti][tj][r];
                    }
        }
        __syncthreads();
    }
    T *out = part + (size_t)blockIdx.x * PI * PJ;
    for (int t = threadIdx.x; t < PI * PJ; t += blockDim.x) out[t] = red[t];
}

// out[i + j ldc] = alpha * sum_g part_g[i][j]  (and mirror[j + i ldm] when given).
// One wavefront per output element: lane l adds partials l, l + 64, ... in
// order, then a fixed butterfly sums the lanes (deterministic for a given G).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ts_reduce(int G, const T *__restrict__ part, int pj, int ps, int ka,
                                                      int kb, T *out, int ldc, T *mirror, int ldm, int mirror_rows,
                                                      T alpha) {
    const int lane = lane_id();
    for (int idx = blockIdx.x * kWavesPerBlock + wave_id(); idx < ka * kb; idx += gridDim.x * kWavesPerBlock) {
        const int i = idx / kb, j = idx % kb;
        const T *src = part + i * pj + j;
        T s = T(0);
        int g = lane;
        for (; g + 3 * kWave < G; g += 4 * kWave) {
            const T a0 = src[(size_t)g * ps], a1 = src[(size_t)(g + kWave) * ps];
            const T a2 = src[(size_t)(g + 2 * kWave) * ps], a3 = src[(size_t)(g + 3 * kWave) * ps];
            s += a0; s += a1; s += a2; s += a3;
        }
        for (; g < G; g += kWave) s += src[(size_t)g * ps];
        s = wave_sum(s) * alpha;
        if (lane == 0) {
            out[i + (size_t)j * ldc] = s;
            if (mirror && i < mirror_rows) mirror[j + (size_t)i * ldm] = s;
        }
    }
}

template <typename T, int TJ>
__global__ __launch_bounds__(kBlock) void k_ts_nn(int n, const T *A, int lda, int ka, const T *__restrict__ C,
                                                  int ldc, int kb, T *Out, int ldo, const T *addend, int ldadd,
                                                  T alpha, T beta) {
    using V4 = typename Mfma<T>::v4;
    extern __shared__ char lds_raw[];
    T *Cs = reinterpret_cast<T *>(lds_raw);  // kap x (TJ*16), row-major
    constexpr int PJ = TJ * 16;
    const int kap = (ka + 3) & ~3;
    for (int t = threadIdx.x; t < kap * PJ; t += blockDim.x) {
        const int k = t / PJ, j = t % PJ;
        Cs[t] = (k < ka && j < kb) ? C[k + (size_t)j * ldc] : T(0);
    }
    __syncthreads();
    const int lane = lane_id();
    const int mi = lane & 15, kk = lane >> 4;
    const int nrb = (n + 15) / 16;
    for (int rb = blockIdx.x * kWavesPerBlock + wave_id(); rb < nrb; rb += gridDim.x * kWavesPerBlock) {
        const int r0 = rb * 16;
        V4 acc[TJ];
#pragma unroll
        for (int tj = 0; tj < TJ; ++tj) acc[tj] = V4{T(0), T(0), T(0), T(0)};
        const int row = r0 + mi;
        const bool rok = row < n;
        for (int k0 = 0; k0 < kap; k0 += 4) {
            const int kc = k0 + kk;
            const T a = (rok && kc < ka) ? A[(size_t)row * lda + kc] : T(0);
#pragma unroll
            for (int tj = 0; tj < TJ; ++tj) acc[tj] = Mfma<T>::mac(a, Cs[(k0 + kk) * PJ + tj * 16 + mi], acc[tj]);
        }
#pragma unroll
        for (int tj = 0; tj < TJ; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = r0 + Mfma<T>::row(lane, r), j = tj * 16 + (lane & 15);
                if (i < n && j < kb) {
                    T base = T(0);
                    if (addend) base = addend[(size_t)i * ldadd + j];
                    else if (beta != T(0)) base = beta * Out[(size_t)i * ldo + j];
                    Out[(size_t)i * ldo + j] = alpha * acc[tj][r] + base;
                }
            }
    }
}

inline int ts_grid(int n) {
    int g = (n + 63) / 64;
    const int cap = 2 * device_cu_count();
    return g < 1 ? 1 : (g > cap ? cap : g);
}

template <typename T, int TI, int TJ>
void ts_tn_launch(int n, const T *A, int lda, int ka, const T *B, int ldb, int kb, T *out, int ldc, T *mirror,
                  int ldm, T alpha, BlockScratch &bs, hipStream_t s) {
    const int G = ts_grid(n);
    constexpr int PS = TI * 16 * TJ * 16;
    T *part = reinterpret_cast<T *>(bs.part.get());
    LAP_REQUIRE((size_t)G * PS * sizeof(T) <= bs.part.n * sizeof(double), LAP_EUNSUPPORTED, "GEMM scratch too small");
    hipLaunchKernelGGL((k_ts_tn<T, TI, TJ>), dim3(G), dim3(kBlock), 0, s, n, A, lda, ka, B, ldb, kb, part);
    const int tot = ka * kb;
    // rows of C at or past ka - kb pair with the new square block, which the
    // direct write already holds in full: mirror only the rows above it
    const int rgrid = std::min((tot + kWavesPerBlock - 1) / kWavesPerBlock, 4 * device_cu_count());
    hipLaunchKernelGGL((k_ts_reduce<T>), dim3(rgrid), dim3(kBlock), 0, s, G, part, TJ * 16, PS, ka, kb, out, ldc,
                       mirror, ldm, ka - kb, alpha);
    LAP_HIP(hipGetLastError());
}

template <typename T, int TJ>
void ts_tn_ti(int n, const T *A, int lda, int ka, const T *B, int ldb, int kb, T *out, int ldc, T *mirror, int ldm,
              T alpha, BlockScratch &bs, hipStream_t s) {
    const int ti = (ka + 15) / 16;
    switch (ti) {
        case 1: ts_tn_launch<T, 1, TJ>(n, A, lda, ka, B, ldb, kb, out, ldc, mirror, ldm, alpha, bs, s); break;
        case 2: ts_tn_launch<T, 2, TJ>(n, A, lda, ka, B, ldb, kb, out, ldc, mirror, ldm, alpha, bs, s); break;
        case 3: ts_tn_launch<T, 3, TJ>(n, A, lda, ka, B, ldb, kb, out, ldc, mirror, ldm, alpha, bs, s); break;
        case 4: ts_tn_launch<T, 4, TJ>(n, A, lda, ka, B, ldb, kb, out, ldc, mirror, ldm, alpha, bs, s); break;
        case 5: ts_tn_launch<T, 5, TJ>(n, A, lda, ka, B, ldb, kb, out, ldc, mirror, ldm, alpha, bs, s); break;
        case 6: ts_tn_launch<T, 6, TJ>(n, A, lda, ka, B, ldb, kb, out, ldc, mirror, ldm, alpha, bs, s); break;
        case 7:
        case 8: ts_tn_launch<T, 8, TJ>(n, A, lda, ka, B, ldb, kb, out, ldc, mirror, ldm, alpha, bs, s); break;
        default: throw Failure{LAP_EUNSUPPORTED, "tall-skinny product wider than 128 columns"};
    }
}

}  // namespace

template <typename T>
void ts_tn(int n, const T *A, int lda, int ka, const T *B, int ldb, int kb, T *out, int ldc, T *mirror, int ldm,
           T alpha, BlockScratch &bs, hipStream_t s) {
    if (ka <= 0 || kb <= 0) return;
    if (kb <= 16) ts_tn_ti<T, 1>(n, A, lda, ka, B, ldb, kb, out, ldc, mirror, ldm, alpha, bs, s);
    else if (kb <= 32) ts_tn_ti<T, 2>(n, A, lda, ka, B, ldb, kb, out, ldc, mirror, ldm, alpha, bs, s);
    else throw Failure{LAP_EUNSUPPORTED, "tall-skinny product with more than 32 right-hand columns"};
}

template <typename T>
void ts_prepare() {
    // LDS above 64 KB needs an opt-in per kernel; done once, outside any capture
    static bool done = false;
    if (done) return;
    LAP_HIP(hipFuncSetAttribute((const void *)k_ts_nn<T, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                128 * 16 * (int)sizeof(T)));
    LAP_HIP(hipFuncSetAttribute((const void *)k_ts_nn<T, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                128 * 32 * (int)sizeof(T)));
    LAP_HIP(hipFuncSetAttribute((const void *)k_ts_nn<T, 4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                128 * 64 * (int)sizeof(T)));
    LAP_HIP(hipFuncSetAttribute((const void *)k_ts_nn<T, 8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                128 * 128 * (int)sizeof(T)));
    done = true;
}
template void ts_prepare<float>();
template void ts_prepare<double>();

template <typename T>
void ts_nn(int n, const T *A, int lda, int ka, const T *C, int ldc, int kb, T *Out, int ldo, const T *addend,
           int ldadd, T alpha, T beta, hipStream_t s) {
    if (kb <= 0) return;
    LAP_REQUIRE(ka <= 128 && kb <= 128, LAP_EUNSUPPORTED, "tall-skinny product wider than 128 columns");
    const int kap = (ka + 3) & ~3;
    int nrb = (n + 15) / 16;
    int grid = (nrb + kWavesPerBlock - 1) / kWavesPerBlock;
    const int cap = 4 * device_cu_count();
    grid = grid < 1 ? 1 : (grid > cap ? cap : grid);
    ts_prepare<T>();
    auto launch = [&](auto tjc) {
        constexpr int TJ = decltype(tjc)::value;
        const size_t lds = (size_t)kap * TJ * 16 * sizeof(T);
        hipLaunchKernelGGL((k_ts_nn<T, TJ>), dim3(grid), dim3(kBlock), lds, s, n, A, lda, ka, C, ldc, kb, Out, ldo,
                           addend, ldadd, alpha, beta);
    };
    if (kb <= 16) launch(std::integral_constant<int, 1>{});
    else if (kb <= 32) launch(std::integral_constant<int, 2>{});
    else if (kb <= 64) launch(std::integral_constant<int, 4>{});
    else launch(std::integral_constant<int, 8>{});
    LAP_HIP(hipGetLastError());
}

template void ts_tn<double>(int, const double *, int, int, const double *, int, int, double *, int, double *, int,
                            double, BlockScratch &, hipStream_t);
template void ts_tn<float>(int, const float *, int, int, const float *, int, int, float *, int, float *, int, float,
                           BlockScratch &, hipStream_t);
template void ts_nn<double>(int, const double *, int, int, const double *, int, int, double *, int, const double *,
                            int, double, double, hipStream_t);
template void ts_nn<float>(int, const float *, int, int, const float *, int, int, float *, int, const float *, int,
                           float, float, hipStream_t);

// ===========================================================================
// Block Jacobi-Davidson helpers (double precision unless noted)
// ===========================================================================
namespace {

// SVQB scaling (Stathopoulos & Wu): with S = V'V = Z diag(lam) Z', the block
// V Z diag(lam)^{-1/2} over the eigenvalues above drop * lam_max has
// orthonormal columns.  Writes M (b x kept, column-major ld ldm) and kept.
__global__ void k_svqb(int b, const double *__restrict__ lam, const double *__restrict__ Z, int ldz, double rel,
                       double abs_thr, double *__restrict__ M, int ldm, BlockStatus *st) {
    __shared__ int first;
    if (threadIdx.x == 0) {
        const double lmax = lam[b - 1];
        int f = b;
        for (int j = 0; j < b; ++j)
            if (lam[j] > rel * lmax && lam[j] > abs_thr && lam[j] > 0.0) { f = j; break; }
        first = f;
        st->kept = b - f;
    }
    __syncthreads();
    const int f = first;
    // kept columns in descending eigenvalue order (the best-conditioned first)
    for (int t = threadIdx.x; t < b * (b - f); t += blockDim.x) {
        const int i = t % b, jj = t / b;
        const int j = b - 1 - jj;
        M[i + (size_t)jj * ldm] = Z[i + (size_t)j * ldz] / sqrt(lam[j]);
    }
}

// R = GU - U diag(theta);  ||R_c||^2, ||U_c||^2;  U also into Q (type T,
// columns qoff..) and column 0 of U into u0 (for the certificate).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_block_resid(int n, int bu, const double *__restrict__ U,
                                                        const double *__restrict__ GU, int ldu,
                                                        const double *__restrict__ theta, double *__restrict__ R,
                                                        T *__restrict__ Q, int ldq, int qoff, double *__restrict__ u0,
                                                        double *partial, unsigned *counter, BlockStatus *st) {
    __shared__ double th[32];
    for (int c = threadIdx.x; c < bu; c += blockDim.x) th[c] = theta[c];
    __syncthreads();
    double acc[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) acc[j] = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
#pragma unroll
        for (int c = 0; c < 32; ++c) {
            if (c < bu) {
                const double uv = U[(size_t)i * ldu + c];
                const double rv = GU[(size_t)i * ldu + c] - th[c] * uv;
                R[(size_t)i * ldu + c] = rv;
                Q[(size_t)i * ldq + qoff + c] = (T)uv;
                acc[c] += rv * rv;
                acc[32 + c] += uv * uv;
            }
        }
        u0[i] = U[(size_t)i * ldu];
    }
    __shared__ double out[64];
    if (grid_reduce<double, 64>(acc, 64, partial, counter, out)) {
        for (int c = threadIdx.x; c < bu; c += blockDim.x) {
            st->unorm[c] = sqrt(out[32 + c]);
            st->rnorm[c] = sqrt(out[c]) / st->unorm[c];
            st->theta[c] = th[c];
        }
    }
}

template <typename S>
__global__ void k_to_f64_block(int n, int b, const S *__restrict__ in, int ldi, double *__restrict__ out, int ldo) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < (size_t)n * b; t += (size_t)gridDim.x * blockDim.x) {
        const size_t i = t / b, c = t % b;
        out[i * ldo + c] = (double)in[i * ldi + c];
    }
}

__device__ __forceinline__ double splitmix_unit_b(unsigned long long seed, unsigned long long idx) {
    unsigned long long z = seed + (idx + 1ULL) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

// columns colbase .. colbase+b-1 of the SplitMix64 start-vector stream
__global__ void k_random_block(int n, int b, unsigned long long seed, long long colbase, const int *__restrict__ iperm,
                               double *__restrict__ out, int ldo) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < (size_t)n * b; t += (size_t)gridDim.x * blockDim.x) {
        const size_t i = t / b, c = t % b;
        out[i * ldo + c] = splitmix_unit_b(seed, (unsigned long long)(colbase + (long long)c) * (unsigned long long)n + iperm[i]);
    }
}

// ---------------------------------------------------------------- block PCG
// Columns c < b solve (I-QQ')(G - theta_c I)(I-QQ') t_c = -r_c with a shared
// projector Q (row-major, q columns, type T).  Per-column state; a column
// stops on its own (tolerance or breakdown) and is masked afterwards.

// init 1: Res = -R (convert), T = 0; ||r_c||
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bpcg_init1(int n, int b, const double *__restrict__ R, int ldr,
                                                       T *__restrict__ Res, T *__restrict__ X, T *partial,
                                                       unsigned *counter, BPcgState<T> *st) {
    T acc[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) acc[c] = T(0);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
#pragma unroll
        for (int c = 0; c < 32; ++c)
            if (c < b) {
                const T r = (T)R[(size_t)i * ldr + c];
                Res[(size_t)i * b + c] = -r;
                X[(size_t)i * b + c] = T(0);
                acc[c] += r * r;
            }
    }
    __shared__ T out[32];
    if (grid_reduce<T, 32>(acc, b, partial, counter, out)) {
        for (int c = threadIdx.x; c < b; c += blockDim.x) {
            st->r0[c] = sqrt(out[c]);
            st->active[c] = st->r0[c] > T(0);
            st->its[c] = 0;
            st->brk[c] = 0;
            st->copy_p[c] = 0;
        }
        if (threadIdx.x == 0) {
            int a = 0;
            for (int c = 0; c < b; ++c) a += st->r0[c] > T(0);
            st->nactive = a;
        }
    }
}

// Y = D^{-1} Res;  rho_c = Res_c' Y_c   (init)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bpcg_init2(int n, int b, const T *__restrict__ Res, T *__restrict__ Y,
                                                       const T *__restrict__ dinv, T *partial, unsigned *counter,
                                                       BPcgState<T> *st) {
    if (st->nactive == 0) return;
    T acc[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) acc[c] = T(0);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const T d = dinv[i];
#pragma unroll
        for (int c = 0; c < 32; ++c)
            if (c < b) {
                const T r = Res[(size_t)i * b + c];
                const T y = d * r;
                Y[(size_t)i * b + c] = y;
                acc[c] += r * y;
            }
    }
    __shared__ T out[32];
    if (grid_reduce<T, 32>(acc, b, partial, counter, out)) {
        for (int c = threadIdx.x; c < b; c += blockDim.x) {
            st->rho[c] = out[c];
            st->beta[c] = T(0);
        }
    }
}

// pAp_c = P_c' S_c;  alpha_c or breakdown
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bpcg_pap(int n, int b, const T *__restrict__ P, const T *__restrict__ S,
                                                     T *partial, unsigned *counter, BPcgState<T> *st, int it) {
    if (st->nactive == 0) return;
    T acc[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) acc[c] = T(0);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
#pragma unroll
        for (int c = 0; c < 32; ++c)
            if (c < b) acc[c] += P[(size_t)i * b + c] * S[(size_t)i * b + c];
    }
    __shared__ T out[32];
    if (grid_reduce<T, 32>(acc, b, partial, counter, out)) {
        if (threadIdx.x == 0) {
            int a = 0;
            for (int c = 0; c < b; ++c) {
                st->copy_p[c] = 0;
                if (!st->active[c]) continue;
                const T pap = out[c];
                if (!(pap > T(0))) {  // indefinite along p: stop this column
                    st->active[c] = 0;
                    st->brk[c] = it;
                    st->copy_p[c] = (it == 1);
                } else {
                    st->alpha[c] = st->rho[c] / pap;
                    ++a;
                }
            }
            st->nactive_step = a;
        }
    }
}

// update: X += alpha P;  Res -= alpha Z  (Z = (I - QQ')S);  Y = D^{-1} Res;
// ||Res_c||, rho'_c;  beta, stop test
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bpcg_update(int n, int b, T *__restrict__ X, T *__restrict__ Res,
                                                        const T *__restrict__ P, const T *__restrict__ Z,
                                                        T *__restrict__ Y, const T *__restrict__ dinv, T *partial,
                                                        unsigned *counter, BPcgState<T> *st, int it, T rtol) {
    if (st->nactive == 0) return;
    __shared__ T al[32];
    __shared__ int act[32], cp[32];
    for (int c = threadIdx.x; c < b; c += blockDim.x) {
        act[c] = st->active[c];
        al[c] = st->alpha[c];
        cp[c] = st->copy_p[c];
    }
    __syncthreads();
    T acc[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) acc[j] = T(0);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const T d = dinv[i];
#pragma unroll
        for (int c = 0; c < 32; ++c) {
            if (c < b) {
                const size_t at = (size_t)i * b + c;
                if (cp[c]) X[at] = P[at];  // no step taken before the breakdown: M(-r)
                if (act[c]) {
                    X[at] += al[c] * P[at];
                    const T r = Res[at] - al[c] * Z[at];
                    Res[at] = r;
                    const T y = d * r;
                    Y[at] = y;
                    acc[c] += r * r;
                    acc[32 + c] += r * y;
                }
            }
        }
    }
    __shared__ T out[64];
    if (grid_reduce<T, 64>(acc, 64, partial, counter, out)) {
        if (threadIdx.x == 0) {
            int a = 0;
            for (int c = 0; c < b; ++c) {
                if (!act[c]) continue;
                st->its[c] = it;
                st->rn[c] = sqrt(out[c]);
                st->beta[c] = out[32 + c] / st->rho[c];
                st->rho[c] = out[32 + c];
                if (st->rn[c] <= rtol * st->r0[c]) st->active[c] = 0;
                else ++a;
            }
            st->nactive = a;
        }
    }
}

// P = Z + beta P  (Z = (I - QQ')Y; active columns; init: P = Z)
template <typename T, bool INIT>
__global__ __launch_bounds__(kBlock) void k_bpcg_p(int n, int b, const T *__restrict__ Z, T *__restrict__ P,
                                                   const BPcgState<T> *st) {
    if (st->nactive == 0) return;
    __shared__ T be[32];
    __shared__ int act[32];
    for (int c = threadIdx.x; c < b; c += blockDim.x) {
        be[c] = st->beta[c];
        act[c] = st->active[c];
    }
    __syncthreads();
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < (size_t)n * b; t += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(t % b);
        if (!act[c]) continue;
        P[t] = INIT ? Z[t] : Z[t] + be[c] * P[t];
    }
}

// nactive from the per-column flags, for the stopping of the whole block
template <typename T>
__global__ void k_bpcg_count(int b, BPcgState<T> *st) {
    if (threadIdx.x == 0) {
        int a = 0;
        for (int c = 0; c < b; ++c) a += st->active[c];
        st->nactive = a;
    }
}

// zero eigenvectors (normalized component indicators) into [X | V] and Q
template <typename T>
__global__ void k_zero_space_rm(int n, int nz, const int *__restrict__ comp, const double *__restrict__ isz,
                                double *__restrict__ XV, int ldb, T *__restrict__ Q, int ldq) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int c = comp[i];
        for (int j = 0; j < nz; ++j) {
            const double v = (c == j) ? isz[j] : 0.0;
            XV[(size_t)i * ldb + j] = v;
            Q[(size_t)i * ldq + j] = (T)v;
        }
    }
}

// out (n x nc column-major) = columns [0, nc) of a row-major block
__global__ void k_extract_cols(int n, int nc, const double *__restrict__ in, int ldi, double *__restrict__ out) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < (size_t)n * nc; t += (size_t)gridDim.x * blockDim.x) {
        const size_t c = t / n, i = t % n;
        out[t] = in[i * ldi + c];
    }
}

// row-major (ld ldo, plan order via map when given) <- column-major n x b
__global__ void k_cm_to_rm(int n, int b, const double *__restrict__ in, const int *__restrict__ map,
                           double *__restrict__ out, int ldo) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < (size_t)n * b; t += (size_t)gridDim.x * blockDim.x) {
        const size_t c = t / n, i = t % n;
        const size_t dst = map ? (size_t)map[i] : i;
        out[dst * ldo + c] = in[t];
    }
}

inline int bgrid(size_t work) {
    size_t g = (work + kBlock - 1) / kBlock;
    const size_t cap = 4 * (size_t)device_cu_count();
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

void blk_svqb(int b, const double *lam, const double *Z, int ldz, double rel, double abs_thr, double *M, int ldm,
              BlockStatus *st, hipStream_t s) {
    hipLaunchKernelGGL(k_svqb, dim3(1), dim3(kBlock), 0, s, b, lam, Z, ldz, rel, abs_thr, M, ldm, st);
    LAP_HIP(hipGetLastError());
}

template <typename T>
void blk_resid(int n, int bu, const double *U, const double *GU, int ldu, const double *theta, double *R, T *Q,
               int ldq, int qoff, double *u0, ReduceScratch &rs, BlockStatus *st, hipStream_t s) {
    LAP_REQUIRE(bu <= 32, LAP_EUNSUPPORTED, "block wider than 32");
    const int grid = bgrid(n);
    rs.ensure(grid, 64);
    hipLaunchKernelGGL((k_block_resid<T>), dim3(grid), dim3(kBlock), 0, s, n, bu, U, GU, ldu, theta, R, Q, ldq, qoff,
                       u0, rs.partial.get(), rs.counter.get(), st);
    LAP_HIP(hipGetLastError());
}
template void blk_resid<float>(int, int, const double *, const double *, int, const double *, double *, float *, int,
                               int, double *, ReduceScratch &, BlockStatus *, hipStream_t);
template void blk_resid<double>(int, int, const double *, const double *, int, const double *, double *, double *,
                                int, int, double *, ReduceScratch &, BlockStatus *, hipStream_t);

template <typename S>
void blk_to_f64(int n, int b, const S *in, int ldi, double *out, int ldo, hipStream_t s) {
    hipLaunchKernelGGL((k_to_f64_block<S>), dim3(bgrid((size_t)n * b)), dim3(kBlock), 0, s, n, b, in, ldi, out, ldo);
    LAP_HIP(hipGetLastError());
}
template void blk_to_f64<float>(int, int, const float *, int, double *, int, hipStream_t);
template void blk_to_f64<double>(int, int, const double *, int, double *, int, hipStream_t);

template <typename T>
void blk_zero_space(int n, int nz, const int *comp, const double *isz, double *XV, int ldb, T *Q, int ldq,
                    hipStream_t s) {
    hipLaunchKernelGGL((k_zero_space_rm<T>), dim3(bgrid(n)), dim3(kBlock), 0, s, n, nz, comp, isz, XV, ldb, Q, ldq);
    LAP_HIP(hipGetLastError());
}
template void blk_zero_space<float>(int, int, const int *, const double *, double *, int, float *, int, hipStream_t);
template void blk_zero_space<double>(int, int, const int *, const double *, double *, int, double *, int, hipStream_t);

void blk_cm_to_rm(int n, int b, const double *in, const int *map, double *out, int ldo, hipStream_t s) {
    hipLaunchKernelGGL(k_cm_to_rm, dim3(bgrid((size_t)n * b)), dim3(kBlock), 0, s, n, b, in, map, out, ldo);
    LAP_HIP(hipGetLastError());
}

void blk_extract(int n, int nc, const double *in, int ldi, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_extract_cols, dim3(bgrid((size_t)n * nc)), dim3(kBlock), 0, s, n, nc, in, ldi, out);
    LAP_HIP(hipGetLastError());
}

void blk_random(int n, int b, uint64_t seed, long long colbase, const int *iperm, double *out, int ldo, hipStream_t s) {
    hipLaunchKernelGGL(k_random_block, dim3(bgrid((size_t)n * b)), dim3(kBlock), 0, s, n, b, (unsigned long long)seed,
                       colbase, iperm, out, ldo);
    LAP_HIP(hipGetLastError());
}

template <typename T>
void bpcg_enqueue(const lap_plan &P, int b, const double *theta_dev, const T *Q, int ldq, int q, const double *R,
                  int ldr, T *X, BPcgWork<T> &w, ReduceScratch &rs, BlockScratch &bs, int itmax, double rtol,
                  hipStream_t s) {
    LAP_REQUIRE(b >= 1 && b <= 32, LAP_EUNSUPPORTED, "block wider than 32");
    const int n = P.n;
    const int gv = bgrid(n);
    rs.ensure(gv, 64);
    T *part = reinterpret_cast<T *>(rs.partial.get());
    unsigned *cnt = rs.counter.get();
    BPcgState<T> *st = w.st.get();
    const T *dinv = P.dinv<T>();
    T *C = w.C.get();  // q x b column-major coefficients
    hipLaunchKernelGGL((k_bpcg_init1<T>), dim3(gv), dim3(kBlock), 0, s, n, b, R, ldr, w.res.get(), X, part, cnt, st);
    T *Z = w.z.get();
    const int gp = bgrid((size_t)n * b);
    // Res <- (I - QQ')Res
    if (q > 0) {
        ts_tn<T>(n, Q, ldq, q, w.res.get(), b, b, C, q, nullptr, 0, T(1), bs, s);
        ts_nn<T>(n, Q, ldq, q, C, q, b, w.res.get(), b, nullptr, 0, T(-1), T(1), s);
    }
    hipLaunchKernelGGL((k_bpcg_init2<T>), dim3(gv), dim3(kBlock), 0, s, n, b, w.res.get(), w.y.get(), dinv, part, cnt,
                       st);
    // P = (I - QQ') Y
    const T *Zy = w.y.get();
    if (q > 0) {
        ts_tn<T>(n, Q, ldq, q, w.y.get(), b, b, C, q, nullptr, 0, T(1), bs, s);
        ts_nn<T>(n, Q, ldq, q, C, q, b, Z, b, w.y.get(), b, T(-1), T(0), s);
        Zy = Z;
    }
    hipLaunchKernelGGL((k_bpcg_p<T, true>), dim3(gp), dim3(kBlock), 0, s, n, b, Zy, w.p.get(), st);
    for (int it = 1; it <= itmax; ++it) {
        // S = G P - P diag(theta);  Z = (I - QQ') S
        spmm<T>(P, b, w.p.get(), b, w.s.get(), b, theta_dev, s);
        const T *Zs = w.s.get();
        if (q > 0) {
            ts_tn<T>(n, Q, ldq, q, w.s.get(), b, b, C, q, nullptr, 0, T(1), bs, s);
            ts_nn<T>(n, Q, ldq, q, C, q, b, Z, b, w.s.get(), b, T(-1), T(0), s);
            Zs = Z;
        }
        hipLaunchKernelGGL((k_bpcg_pap<T>), dim3(gv), dim3(kBlock), 0, s, n, b, w.p.get(), w.s.get(), part, cnt, st, it);
        hipLaunchKernelGGL((k_bpcg_update<T>), dim3(gv), dim3(kBlock), 0, s, n, b, X, w.res.get(), w.p.get(), Zs,
                           w.y.get(), dinv, part, cnt, st, it, (T)rtol);
        if (it == itmax) break;
        // P = (I - QQ') Y + beta P
        Zy = w.y.get();
        if (q > 0) {
            ts_tn<T>(n, Q, ldq, q, w.y.get(), b, b, C, q, nullptr, 0, T(1), bs, s);
            ts_nn<T>(n, Q, ldq, q, C, q, b, Z, b, w.y.get(), b, T(-1), T(0), s);
            Zy = Z;
        }
        hipLaunchKernelGGL((k_bpcg_p<T, false>), dim3(gp), dim3(kBlock), 0, s, n, b, Zy, w.p.get(), st);
    }
    hipLaunchKernelGGL((k_bpcg_count<T>), dim3(1), dim3(64), 0, s, b, st);
    LAP_HIP(hipGetLastError());
}
template void bpcg_enqueue<float>(const lap_plan &, int, const double *, const float *, int, int, const double *, int,
                                  float *, BPcgWork<float> &, ReduceScratch &, BlockScratch &, int, double, hipStream_t);
template void bpcg_enqueue<double>(const lap_plan &, int, const double *, const double *, int, int, const double *,
                                   int, double *, BPcgWork<double> &, ReduceScratch &, BlockScratch &, int, double,
                                   hipStream_t);

}  // namespace lapeig
