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
    // U of the wavefront's 4-row chunks per pass: all their loads are issued
    // before the first multiply, and the chunks are accumulated in the same
    // order as one at a time
    constexpr int U = TI * TJ <= 2 ? 4 : 2;
    const int step = gridDim.x * kWavesPerBlock * 4;
    for (int k0 = (blockIdx.x * kWavesPerBlock + wave) * 4; k0 < n; k0 += U * step) {
        T a[U][TI], b[U][TJ];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int row = k0 + u * step + kk;
            const bool ok = row < n;
#pragma unroll
            for (int ti = 0; ti < TI; ++ti) {
                const int col = ti * 16 + mi;
                a[u][ti] = (ok && col < ka) ? A[(size_t)row * lda + col] : T(0);
            }
#pragma unroll
            for (int tj = 0; tj < TJ; ++tj) {
                const int col = tj * 16 + mi;
                b[u][tj] = (ok && col < kb) ? B[(size_t)row * ldb + col] : T(0);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int ti = 0; ti < TI; ++ti)
#pragma unroll
                for (int tj = 0; tj < TJ; ++tj) acc[ti][tj] = Mfma<T>::mac(a[u][ti], b[u][tj], acc[ti][tj]);
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

template <typename T, int TJ, int KS>
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
        const int row = r0 + mi;
        const bool rok = row < n;
        // every load of the 16-row block (KS 4-column steps cover ka) is
        // issued before the first multiply
        T a[KS];
#pragma unroll
        for (int t = 0; t < KS; ++t) {
            const int kc = 4 * t + kk;
            a[t] = (rok && kc < ka) ? A[(size_t)row * lda + kc] : T(0);
        }
        V4 acc[TJ];
#pragma unroll
        for (int tj = 0; tj < TJ; ++tj) acc[tj] = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int t = 0; t < KS; ++t)
            if (4 * t < kap) {
#pragma unroll
                for (int tj = 0; tj < TJ; ++tj)
                    acc[tj] = Mfma<T>::mac(a[t], Cs[(4 * t + kk) * PJ + tj * 16 + mi], acc[tj]);
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

template <typename T, int TJ>
void ts_nn_attr() {
    const int bytes = 128 * TJ * 16 * (int)sizeof(T);
    LAP_HIP(hipFuncSetAttribute((const void *)k_ts_nn<T, TJ, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    LAP_HIP(hipFuncSetAttribute((const void *)k_ts_nn<T, TJ, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    LAP_HIP(hipFuncSetAttribute((const void *)k_ts_nn<T, TJ, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    LAP_HIP(hipFuncSetAttribute((const void *)k_ts_nn<T, TJ, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
}

template <typename T>
void ts_prepare() {
    // LDS above 64 KB needs an opt-in per kernel; done once, outside any capture
    static bool done = false;
    if (done) return;
    ts_nn_attr<T, 1>();
    ts_nn_attr<T, 2>();
    ts_nn_attr<T, 4>();
    ts_nn_attr<T, 8>();
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
        auto go = [&](auto ksc) {
            constexpr int KS = decltype(ksc)::value;
            hipLaunchKernelGGL((k_ts_nn<T, TJ, KS>), dim3(grid), dim3(kBlock), lds, s, n, A, lda, ka, C, ldc, kb, Out,
                               ldo, addend, ldadd, alpha, beta);
        };
        if (kap <= 16) go(std::integral_constant<int, 4>{});
        else if (kap <= 32) go(std::integral_constant<int, 8>{});
        else if (kap <= 64) go(std::integral_constant<int, 16>{});
        else go(std::integral_constant<int, 32>{});
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
    // kept columns in descending eigenvalue order (the best-conditioned first),
    // then zero columns up to b, so a caller that does not wait for the kept
    // count can apply all b columns (the dropped directions come out as zero
    // columns, which the next SVQB drops in turn)
    for (int t = threadIdx.x; t < b * b; t += blockDim.x) {
        const int i = t % b, jj = t / b;
        const int j = b - 1 - jj;
        M[i + (size_t)jj * ldm] = jj < b - f ? Z[i + (size_t)j * ldz] / sqrt(lam[j]) : 0.0;
    }
}

// CholQR of a block V with b <= 32 columns from its Gram matrix S = V'V
// (column-major, ld lds), in one wavefront: pivoted Cholesky P'SP = R'R, the
// pivot each step the largest remaining diagonal, stopping at the first pivot
// not above max(rel * (largest diagonal of S), abs_thr, 0); then M = P R^-1
// on the kept columns and zero elsewhere (b x b, ld ldm), so that V M has
// `kept` orthonormal columns spanning what V spans above the threshold, then
// zero columns.  st->kept = the number kept.
__global__ __launch_bounds__(kWave) void k_cholqr(int b, const double *__restrict__ S, int lds, double rel,
                                                  double abs_thr, double *__restrict__ M, int ldm,
                                                  BlockStatus *st) {
    __shared__ double A[32][33];  // the trailing Schur complement (row-major); later R^-1
    __shared__ double R[32][33];
    __shared__ int piv[32];
    const int lane = threadIdx.x;
    for (int t = lane; t < 32 * 32; t += kWave) {
        const int i = t >> 5, j = t & 31;
        A[i][j] = (i < b && j < b) ? S[i + (size_t)j * lds] : 0.0;
        R[i][j] = 0.0;
    }
    if (lane < 32) piv[lane] = lane;
    __syncthreads();
    double dmax = lane < b ? A[lane][lane] : 0.0;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, kWave));
    const double thr = fmax(rel * dmax, abs_thr);
    int rank = 0;
    for (int j = 0; j < b; ++j) {
        // pivot: the largest remaining diagonal (ties to the smaller index)
        double v = (lane >= j && lane < b) ? A[lane][lane] : -1.0;
        int idx = lane;
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            const double ov = __shfl_xor(v, o, kWave);
            const int oi = __shfl_xor(idx, o, kWave);
            if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
        }
        if (!(v > thr) || !(v > 0.0)) break;
        const int p = idx;
        if (p != j) {
            if (lane < b) {
                const double t0 = A[j][lane];
                A[j][lane] = A[p][lane];
                A[p][lane] = t0;
            }
            __syncthreads();
            if (lane < b) {
                const double t0 = A[lane][j];
                A[lane][j] = A[lane][p];
                A[lane][p] = t0;
            }
            if (lane < j) {
                const double t0 = R[lane][j];
                R[lane][j] = R[lane][p];
                R[lane][p] = t0;
            }
            if (lane == 0) {
                const int t0 = piv[j];
                piv[j] = piv[p];
                piv[p] = t0;
            }
            __syncthreads();
        }
        const double rjj = sqrt(A[j][j]);
        if (lane == j) R[j][j] = rjj;
        else if (lane > j && lane < b) R[j][lane] = A[j][lane] / rjj;
        __syncthreads();
        const int w = b - j - 1;
        for (int t = lane; t < w * w; t += kWave) {
            const int i = j + 1 + t / w, k = j + 1 + t % w;
            A[i][k] -= R[j][i] * R[j][k];
        }
        __syncthreads();
        rank = j + 1;
    }
    // R^-1 (upper triangular, rank x rank) into A: lane c takes column c
    if (lane < rank) {
        const int c = lane;
        A[c][c] = 1.0 / R[c][c];
        for (int i = c - 1; i >= 0; --i) {
            double acc = 0.0;
            for (int k = i + 1; k <= c; ++k) acc += R[i][k] * A[k][c];
            A[i][c] = -acc / R[i][i];
        }
    }
    __syncthreads();
    // M = P R^-1: row piv[i] of column c holds R^-1[i][c]
    for (int t = lane; t < b * b; t += kWave) {
        const int r = t % b, c = t / b;
        M[r + (size_t)c * ldm] = 0.0;
    }
    __syncthreads();
    for (int t = lane; t < b * b; t += kWave) {
        const int i = t % b, c = t / b;
        if (c < rank && i <= c) M[piv[i] + (size_t)c * ldm] = A[i][c];
    }
    if (lane == 0) st->kept = rank;
}

template <typename T, int NQ>
__device__ __forceinline__ void col_partials(const T (&acc)[NQ], int b, T *__restrict__ part) {
    __shared__ T red[NQ][kBlock];
#pragma unroll
    for (int j = 0; j < NQ; ++j) red[j][threadIdx.x] = acc[j];
    __syncthreads();
    if ((int)threadIdx.x < b) {
        const int base = (int)(((size_t)blockIdx.x * blockDim.x) % (size_t)b);
        const int t0 = ((int)threadIdx.x - base + b) % b;  // first thread of this column
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            T s = T(0);
            for (int t = t0; t < kBlock; t += b) s += red[j][t];
            part[(size_t)blockIdx.x * 64 + 32 * j + threadIdx.x] = s;
        }
    }
}

// totals[v] = sum over the nb partial rows of value v (v < nv; row stride 64)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bfold(const T *__restrict__ part, int nb, int nv, T *__restrict__ totals) {
    const int lane = lane_id();
    for (int v = blockIdx.x * kWavesPerBlock + wave_id(); v < nv; v += gridDim.x * kWavesPerBlock) {
        T s = T(0);
        int g = lane;
        for (; g + 3 * kWave < nb; g += 4 * kWave) {
            const T a0 = part[(size_t)g * 64 + v], a1 = part[(size_t)(g + kWave) * 64 + v];
            const T a2 = part[(size_t)(g + 2 * kWave) * 64 + v], a3 = part[(size_t)(g + 3 * kWave) * 64 + v];
            s += a0; s += a1; s += a2; s += a3;
        }
        for (; g < nb; g += kWave) s += part[(size_t)g * 64 + v];
        s = wave_sum(s);
        if (lane == 0) totals[v] = s;
    }
}

// First stage of a fold of many partial rows (64 values each): workgroup g
// adds rows [g per, (g + 1) per), wavefront w rows w, w + 4, ... of them
// (lane l value l), then the four wavefront sums in order, into row g of out.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bfold_rows(const T *__restrict__ part, int nb, int per,
                                                       T *__restrict__ out) {
    __shared__ T ws[kWavesPerBlock][kWave];
    const int lane = lane_id(), w = wave_id();
    const int r1 = min((blockIdx.x + 1) * per, nb);
    T s = T(0);
    int r = blockIdx.x * per + w;
    for (; r + 3 * kWavesPerBlock < r1; r += 4 * kWavesPerBlock) {
        const T a0 = part[(size_t)r * 64 + lane], a1 = part[(size_t)(r + kWavesPerBlock) * 64 + lane];
        const T a2 = part[(size_t)(r + 2 * kWavesPerBlock) * 64 + lane];
        const T a3 = part[(size_t)(r + 3 * kWavesPerBlock) * 64 + lane];
        s += a0; s += a1; s += a2; s += a3;
    }
    for (; r < r1; r += kWavesPerBlock) s += part[(size_t)r * 64 + lane];
    ws[w][lane] = s;
    __syncthreads();
    if (w == 0) {
        T t = T(0);
        for (int i = 0; i < kWavesPerBlock; ++i) t += ws[i][lane];
        out[(size_t)blockIdx.x * 64 + lane] = t;
    }
}

// k_bfold for many rows: one workgroup per value, its four wavefronts add
// interleaved rows (lane l of wavefront w: rows w 64 + l, then + 256, ...),
// then the wavefront sums in wavefront order
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bfold_wide(const T *__restrict__ part, int nb, T *__restrict__ totals) {
    __shared__ T ws[kWavesPerBlock];
    const int v = blockIdx.x;
    T s = T(0);
    int g = threadIdx.x;
    for (; g + 3 * kBlock < nb; g += 4 * kBlock) {
        const T a0 = part[(size_t)g * 64 + v], a1 = part[(size_t)(g + kBlock) * 64 + v];
        const T a2 = part[(size_t)(g + 2 * kBlock) * 64 + v], a3 = part[(size_t)(g + 3 * kBlock) * 64 + v];
        s += a0; s += a1; s += a2; s += a3;
    }
    for (; g < nb; g += kBlock) s += part[(size_t)g * 64 + v];
    s = wave_sum(s);
    if (lane_id() == 0) ws[wave_id()] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = T(0);
        for (int w = 0; w < kWavesPerBlock; ++w) t += ws[w];
        totals[v] = t;
    }
}

// R = GU - U diag(theta);  U also into Q (type T, columns qoff..) and
// column 0 of U into u0 (for the certificate).  U, GU and R are row-major
// with leading dimensions ldu, ldg and ldr.  Column grid over the n x ldr
// blocks (columns c >= bu are skipped); partials ||R_c||^2, ||U_c||^2.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_block_resid(int n, int bu, const double *__restrict__ U, int ldu,
                                                        const double *__restrict__ GU, int ldg, int ldr,
                                                        const double *__restrict__ theta, double *__restrict__ R,
                                                        T *__restrict__ Q, int ldq, int qoff, double *__restrict__ u0,
                                                        double *__restrict__ part) {
    const size_t tot = (size_t)n * ldr, stride = (size_t)gridDim.x * blockDim.x;
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = (int)(t % ldr);
    double acc[2] = {0.0, 0.0};
    if (c < bu) {
        const double th = theta[c];
        for (; t < tot; t += stride) {
            const size_t i = t / ldr;
            const double uv = U[i * ldu + c];
            const double rv = GU[i * ldg + c] - th * uv;
            R[t] = rv;
            Q[i * ldq + qoff + c] = (T)uv;
            if (c == 0) u0[i] = uv;
            acc[0] += rv * rv;
            acc[1] += uv * uv;
        }
    }
    col_partials<double, 2>(acc, ldr, part);
}

// Ritz residual norms of the block from the folded sums
__global__ void k_block_resid_status(int bu, const double *__restrict__ theta, const double *__restrict__ tot,
                                     BlockStatus *st) {
    for (int c = threadIdx.x; c < bu; c += blockDim.x) {
        const double un = sqrt(tot[32 + c]);
        st->unorm[c] = un;
        st->rnorm[c] = sqrt(tot[c]) / un;
        st->theta[c] = theta[c];
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
//
// The elementwise launches run on a "column grid": its stride (workgroups x
// 256) is a multiple of b, so every thread keeps one column of the row-major
// n x b blocks for its whole loop, loads are coalesced, and each thread
// accumulates one value per quantity.  Workgroups leave per-column partial
// sums (row stride 64: quantity j of column c at 32 j + c), which k_bfold
// adds (one wavefront per value, fixed order) into a totals slot of the
// state read by the next launch.

__device__ __forceinline__ bool leader0() { return blockIdx.x == 0 && threadIdx.x == 0; }

// any column still iterating (flags of slot a)
template <typename T>
__device__ __forceinline__ bool any_active(const BPcgState<T> *st, int a, int b) {
    int any = 0;
    for (int c = 0; c < b; ++c) any |= st->act[a][c];
    return any != 0;
}

// init 1: Res = -R (converted), X = 0;  partials ||r_c||^2
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bpcg_init1(int n, int b, const double *__restrict__ R, int ldr,
                                                       T *__restrict__ Res, T *__restrict__ X, T *__restrict__ part) {
    const size_t tot = (size_t)n * b, stride = (size_t)gridDim.x * blockDim.x;
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = (int)(t % b);
    T acc[1] = {T(0)};
    for (; t < tot; t += stride) {
        const size_t i = t / b;
        const T r = (T)R[i * ldr + c];
        Res[t] = -r;
        X[t] = T(0);
        acc[0] += r * r;
    }
    col_partials<T, 1>(acc, b, part);
}

// init 2 (after Res <- (I - QQ')Res): r0_c and the flags; Y = D^{-1} Res;
// partials rho_c = Res_c'Y_c
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bpcg_init2(int n, int b, const T *__restrict__ Res, T *__restrict__ Y,
                                                       const T *__restrict__ dinv, T *__restrict__ part,
                                                       BPcgState<T> *st) {
    if (blockIdx.x == 0 && (int)threadIdx.x < b) {
        const int c = threadIdx.x;
        const T r0 = sqrt(st->tot_a[c]);
        st->r0[c] = r0;
        st->act[0][c] = r0 > T(0);
        st->its[c] = 0;
        st->brk[c] = 0;
    }
    const size_t tot = (size_t)n * b, stride = (size_t)gridDim.x * blockDim.x;
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    T acc[1] = {T(0)};
    for (; t < tot; t += stride) {
        const T r = Res[t];
        const T y = dinv[t / b] * r;
        Y[t] = y;
        acc[0] += r * y;
    }
    col_partials<T, 1>(acc, b, part);
}

// p0: rho_c from the folded sums; P = Z  (Z = (I - QQ')Y)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bpcg_p0(int n, int b, const T *__restrict__ Z, T *__restrict__ P,
                                                    BPcgState<T> *st) {
    if (blockIdx.x == 0 && (int)threadIdx.x < b) st->rho[0][threadIdx.x] = st->tot_b[threadIdx.x];
    const size_t tot = (size_t)n * b;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x)
        P[t] = Z[t];
}

// pap: partials P_c'S_c  (= P_c'(I-QQ')S_c, P orthogonal to Q)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bpcg_pap(int n, int b, const T *__restrict__ P, const T *__restrict__ S,
                                                     T *__restrict__ part, const BPcgState<T> *st) {
    if (!any_active(st, 0, b)) return;
    const size_t tot = (size_t)n * b, stride = (size_t)gridDim.x * blockDim.x;
    T acc[1] = {T(0)};
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) acc[0] += P[t] * S[t];
    col_partials<T, 1>(acc, b, part);
}

// update (iteration it): alpha_c = rho_c / pAp_c or breakdown; X += alpha P;
// Res -= alpha Z (Z = (I-QQ')S); Y = D^{-1} Res; partials Res'Res, Res'Y.
// Reads flags of slot 0, writes slot 1.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bpcg_update(int n, int b, T *__restrict__ X, T *__restrict__ Res,
                                                        const T *__restrict__ P, const T *__restrict__ Z,
                                                        T *__restrict__ Y, const T *__restrict__ dinv,
                                                        T *__restrict__ part, BPcgState<T> *st, int it) {
    if (!any_active(st, 0, b)) {
        if (blockIdx.x == 0 && (int)threadIdx.x < b) st->act[1][threadIdx.x] = 0;
        return;
    }
    const size_t tot = (size_t)n * b, stride = (size_t)gridDim.x * blockDim.x;
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = (int)(t % b);
    const int act = st->act[0][c];
    const T pap = st->tot_a[c];
    const bool brk = act && !(pap > T(0));  // the projected operator is indefinite along p
    const bool step = act && !brk;
    const T alpha = step ? st->rho[(it + 1) & 1][c] / pap : T(0);
    if (blockIdx.x == 0 && (int)threadIdx.x < b) {
        // threads 0..b-1 of workgroup 0 own columns 0..b-1
        st->act[1][c] = step;
        if (brk) st->brk[c] = it;
        if (step) st->its[c] = it;
    }
    T acc[2] = {T(0), T(0)};
    if (step) {
        for (; t < tot; t += stride) {
            X[t] += alpha * P[t];
            const T r = Res[t] - alpha * Z[t];
            Res[t] = r;
            const T y = dinv[t / b] * r;
            Y[t] = y;
            acc[0] += r * r;
            acc[1] += r * y;
        }
    } else if (brk && it == 1) {
        for (; t < tot; t += stride) X[t] = P[t];  // no step was taken before the breakdown: M(-r)
    }
    col_partials<T, 2>(acc, b, part);
}

// p (iteration it): ||Res_c|| <= rtol r0_c stops column c; else
// beta = rho'/rho, P = Z + beta P (Z = (I-QQ')Y).  Reads flags of slot 1,
// writes slot 0.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bpcg_p(int n, int b, const T *__restrict__ Z, T *__restrict__ P,
                                                   BPcgState<T> *st, int it, T rtol) {
    if (!any_active(st, 1, b)) {
        if (blockIdx.x == 0 && (int)threadIdx.x < b) st->act[0][threadIdx.x] = 0;
        return;
    }
    const size_t tot = (size_t)n * b, stride = (size_t)gridDim.x * blockDim.x;
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = (int)(t % b);
    const int act = st->act[1][c];
    const T rn = sqrt(st->tot_b[c]);
    const T rho_new = st->tot_b[32 + c];
    const bool go = act && !(rn <= rtol * st->r0[c]);
    const T beta = go ? rho_new / st->rho[(it + 1) & 1][c] : T(0);
    if (blockIdx.x == 0 && (int)threadIdx.x < b) {
        st->act[0][c] = go;
        if (go) st->rho[it & 1][c] = rho_new;
    }
    if (!go) return;
    for (; t < tot; t += stride) P[t] = Z[t] + beta * P[t];
}

// ------------------------------------------- fused block PCG (b, q <= 32)
// Same iteration, same per-column state and stop rules, with the residual
// carried as R~: the step subtracts alpha S (not alpha (I-QQ')S) and the
// projection is taken once per iteration afterwards.  With W = Q'D^{-1}Q
// (formed once per solve), one tall-skinny pass over [Q | R~] gives every
// coefficient the two projections of an iteration need:
//   KT  alpha; X += alpha P; R~ -= alpha S;  partial tiles G1 = Q'R~,
//       G2 = Q'D^{-1}R~ and column sums R~'R~, R~'D^{-1}R~  (matrix cores)
//   KN  C1 = G1, C2 = G2 - W C1;  Res = R~ - Q C1 (so Q'Res = 0);
//       ||Res||^2 = R~'R~ - |C1|^2;  rho' = Res'D^{-1}Res
//       = R~'D^{-1}R~ - C1'G2 - C1'C2;  stop test, beta = rho'/rho;
//       P = (D^{-1}Res - Q C2) + beta P = (I-QQ')D^{-1}Res + beta P;  R~ = Res
// R~ starts each iteration orthogonal to Q, so C1 holds one step's drift
// (alpha Q'S, small beside Res while Q holds Ritz vectors) and the two
// expansions lose nothing to cancellation.  Q has up to TI x 16 columns, the
// block up to TJ x 16.  The per-workgroup partials of KT form a
// (2 PI + 2) x PJ matrix (rows: G1, G2, R~'R~, R~'D^{-1}R~; PI = 16 TI,
// PJ = 16 TJ), added by k_ts_reduce in a fixed order into totals with
// 2 PI + 2 rows.
template <int TI>
constexpr int fused_ld() { return 2 * 16 * TI + 2; }

// KT (WM = false) and, with WM, the same pass over [Q | D^{-1}Q] that gives
// W in rows PI .. 2 PI - 1 of the totals (TJ = TI then).
template <typename T, bool WM, int TI, int TJ>
__global__ __launch_bounds__(kBlock) void k_bpcg_kt(int n, int b, int q, T *__restrict__ X, T *__restrict__ R,
                                                    const T *__restrict__ P, const T *__restrict__ S,
                                                    const T *__restrict__ dinv, const T *__restrict__ Q, int ldq,
                                                    T *__restrict__ part, BPcgState<T> *st, int it) {
    using V4 = typename Mfma<T>::v4;
    constexpr int PI = 16 * TI, PJ = 16 * TJ;
    constexpr int PS = (2 * PI + 2) * PJ;
    __shared__ T red[PS];
    const int lane = lane_id(), wave = wave_id();
    const int mi = lane & 15, kk = lane >> 4;
    T alpha[TJ];
    bool step[TJ], brk1[TJ];
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj) { alpha[tj] = T(0); step[tj] = false; brk1[tj] = false; }
    if (!WM) {
        if (!any_active(st, 0, b)) {
            if (blockIdx.x == 0 && (int)threadIdx.x < b) st->act[1][threadIdx.x] = 0;
            return;
        }
#pragma unroll
        for (int tj = 0; tj < TJ; ++tj) {
            const int c = tj * 16 + mi;
            if (c < b) {
                const int act = st->act[0][c];
                const T pap = st->tot_a[c];
                const bool brk = act && !(pap > T(0));  // the projected operator is indefinite along p
                step[tj] = act && !brk;
                brk1[tj] = brk && it == 1;
                alpha[tj] = step[tj] ? st->rho[(it + 1) & 1][c] / pap : T(0);
                // wavefront 0, kk = 0: lane mi (with tj) owns column c
                if (blockIdx.x == 0 && wave == 0 && kk == 0) {
                    st->act[1][c] = step[tj];
                    if (brk) st->brk[c] = it;
                    if (step[tj]) st->its[c] = it;
                }
            }
        }
    }
    V4 acc1[TI][TJ], acc2[TI][TJ];
#pragma unroll
    for (int ti = 0; ti < TI; ++ti)
#pragma unroll
        for (int tj = 0; tj < TJ; ++tj) acc1[ti][tj] = acc2[ti][tj] = V4{T(0), T(0), T(0), T(0)};
    T s1[TJ], s2[TJ];
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj) s1[tj] = s2[tj] = T(0);
    constexpr int U = TI * TJ == 1 ? 4 : 2;  // 4-row chunks per pass, all loads issued first
    const int stride = gridDim.x * kWavesPerBlock * 4;
    for (int k0 = (blockIdx.x * kWavesPerBlock + wave) * 4; k0 < n; k0 += U * stride) {
        T a[U][TI], v[U][TJ], d[U], x[U][TJ], p[U][TJ], sv[U][TJ];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int row = k0 + u * stride + kk;
            const bool ok = row < n;
#pragma unroll
            for (int ti = 0; ti < TI; ++ti) {
                const int col = ti * 16 + mi;
                a[u][ti] = (ok && col < q) ? Q[(size_t)row * ldq + col] : T(0);
            }
            d[u] = ok ? dinv[row] : T(0);
#pragma unroll
            for (int tj = 0; tj < TJ; ++tj) {
                const int c = tj * 16 + mi;
                if (WM) {
                    v[u][tj] = (ok && c < q) ? Q[(size_t)row * ldq + c] : T(0);
                } else {
                    const bool in = ok && c < b;
                    const size_t e = (size_t)row * b + c;
                    v[u][tj] = in ? R[e] : T(0);
                    x[u][tj] = (in && step[tj]) ? X[e] : T(0);
                    p[u][tj] = (in && (step[tj] || brk1[tj])) ? P[e] : T(0);
                    sv[u][tj] = (in && step[tj]) ? S[e] : T(0);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int row = k0 + u * stride + kk;
#pragma unroll
            for (int tj = 0; tj < TJ; ++tj) {
                if (!WM) {
                    const int c = tj * 16 + mi;
                    if (row < n && c < b) {
                        const size_t e = (size_t)row * b + c;
                        if (step[tj]) {
                            X[e] = x[u][tj] + alpha[tj] * p[u][tj];
                            v[u][tj] = v[u][tj] - alpha[tj] * sv[u][tj];
                            R[e] = v[u][tj];
                        } else if (brk1[tj]) {
                            X[e] = p[u][tj];  // no step was taken before the breakdown: M(-r)
                        }
                    }
                }
                const T dv = d[u] * v[u][tj];
#pragma unroll
                for (int ti = 0; ti < TI; ++ti) {
                    acc1[ti][tj] = Mfma<T>::mac(a[u][ti], v[u][tj], acc1[ti][tj]);
                    acc2[ti][tj] = Mfma<T>::mac(a[u][ti], dv, acc2[ti][tj]);
                }
                s1[tj] += v[u][tj] * v[u][tj];
                s2[tj] += v[u][tj] * dv;
            }
        }
    }
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj) {
        s1[tj] += __shfl_xor(s1[tj], 16, kWave);
        s1[tj] += __shfl_xor(s1[tj], 32, kWave);
        s2[tj] += __shfl_xor(s2[tj], 16, kWave);
        s2[tj] += __shfl_xor(s2[tj], 32, kWave);
    }
    // the four wavefronts in a fixed order
    for (int w = 0; w < kWavesPerBlock; ++w) {
        if (wave == w) {
#pragma unroll
            for (int ti = 0; ti < TI; ++ti)
#pragma unroll
                for (int tj = 0; tj < TJ; ++tj)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = ti * 16 + Mfma<T>::row(lane, r), j = tj * 16 + (lane & 15);
                        red[i * PJ + j] = (w == 0 ? T(0) : red[i * PJ + j]) + acc1[ti][tj][r];
                        red[(PI + i) * PJ + j] = (w == 0 ? T(0) : red[(PI + i) * PJ + j]) + acc2[ti][tj][r];
                    }
            if (kk == 0) {
#pragma unroll
                for (int tj = 0; tj < TJ; ++tj) {
                    const int j = tj * 16 + mi;
                    red[2 * PI * PJ + j] = (w == 0 ? T(0) : red[2 * PI * PJ + j]) + s1[tj];
                    red[(2 * PI + 1) * PJ + j] = (w == 0 ? T(0) : red[(2 * PI + 1) * PJ + j]) + s2[tj];
                }
            }
        }
        __syncthreads();
    }
    T *out = part + (size_t)blockIdx.x * PS;
    for (int t = threadIdx.x; t < PS; t += blockDim.x) out[t] = red[t];
}

// KN.  tot: totals of KT (element (i, j) at i + j (2 PI + 2)); totw: those of
// the W pass.  Reads flags of slot 1, writes slot 0.
template <typename T, int TI, int TJ>
__global__ __launch_bounds__(kBlock) void k_bpcg_kn(int n, int b, int q, T *__restrict__ R, T *__restrict__ P,
                                                    const T *__restrict__ dinv, const T *__restrict__ Q, int ldq,
                                                    const T *__restrict__ tot, const T *__restrict__ totw,
                                                    BPcgState<T> *st, int it, T rtol) {
    using V4 = typename Mfma<T>::v4;
    constexpr int PI = 16 * TI, PJ = 16 * TJ;
    constexpr int LD = 2 * PI + 2;
    __shared__ T c1s[PI * PJ], c2s[PI * PJ];  // [k][j]: Q column k, block column j
    __shared__ T betas[PJ];
    __shared__ int gos[PJ];
    if (!any_active(st, 1, b)) {
        if (blockIdx.x == 0 && (int)threadIdx.x < b) st->act[0][threadIdx.x] = 0;
        return;
    }
    for (int t = threadIdx.x; t < PI * PJ; t += blockDim.x) {
        const int kq = t / PJ, jc = t % PJ;
        c1s[t] = (kq < q && jc < b) ? tot[kq + jc * LD] : T(0);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < PI * PJ; t += blockDim.x) {
        const int kq = t / PJ, jc = t % PJ;
        T c2 = T(0);
        if (kq < q && jc < b) {
            c2 = tot[PI + kq + jc * LD];
            for (int m = 0; m < q; ++m) c2 -= totw[PI + kq + m * LD] * c1s[m * PJ + jc];
        }
        c2s[t] = c2;
    }
    __syncthreads();
    if ((int)threadIdx.x < PJ) {
        const int c = threadIdx.x;
        bool go = false;
        T beta = T(0);
        if (c < b) {
            T rr = tot[2 * PI + c * LD], rho_new = tot[2 * PI + 1 + c * LD];
            for (int k = 0; k < q; ++k) {
                const T g1 = c1s[k * PJ + c];
                rr -= g1 * g1;
                rho_new -= g1 * (tot[PI + k + c * LD] + c2s[k * PJ + c]);
            }
            const T rn = sqrt(rr > T(0) ? rr : T(0));
            go = st->act[1][c] && !(rn <= rtol * st->r0[c]);
            beta = go ? rho_new / st->rho[(it + 1) & 1][c] : T(0);
            if (blockIdx.x == 0) {
                st->act[0][c] = go;
                if (go) st->rho[it & 1][c] = rho_new;
            }
        }
        gos[c] = go;
        betas[c] = beta;
    }
    __syncthreads();
    const int lane = lane_id();
    const int mi = lane & 15, kk = lane >> 4;
    const int nrb = (n + 15) / 16;
    for (int rb = blockIdx.x * kWavesPerBlock + wave_id(); rb < nrb; rb += gridDim.x * kWavesPerBlock) {
        const int r0 = rb * 16;
        const int row = r0 + mi;
        const bool rok = row < n;
        V4 acc1[TJ], acc2[TJ];
#pragma unroll
        for (int tj = 0; tj < TJ; ++tj) acc1[tj] = acc2[tj] = V4{T(0), T(0), T(0), T(0)};
        for (int k0 = 0; k0 < q; k0 += 4) {
            const int kc = k0 + kk;
            const T a = (rok && kc < q) ? Q[(size_t)row * ldq + kc] : T(0);
#pragma unroll
            for (int tj = 0; tj < TJ; ++tj) {
                acc1[tj] = Mfma<T>::mac(a, c1s[kc * PJ + tj * 16 + mi], acc1[tj]);
                acc2[tj] = Mfma<T>::mac(a, c2s[kc * PJ + tj * 16 + mi], acc2[tj]);
            }
        }
#pragma unroll
        for (int tj = 0; tj < TJ; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = r0 + Mfma<T>::row(lane, r), j = tj * 16 + (lane & 15);
                if (i < n && j < b && gos[j]) {
                    const size_t e = (size_t)i * b + j;
                    const T res = R[e] - acc1[tj][r];
                    R[e] = res;
                    const T z = dinv[i] * res - acc2[tj][r];
                    P[e] = z + betas[j] * P[e];
                }
            }
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

// flags[c] != 0 when column c of the n x b column-major block holds a
// non-finite entry (flags cleared by the caller)
__global__ void k_nonfinite_cols(int n, int b, const double *__restrict__ in, int *__restrict__ flags) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < (size_t)n * b; t += (size_t)gridDim.x * blockDim.x)
        if (!isfinite(in[t])) atomicOr(flags + t / n, 1);
}

inline int bgrid(size_t work) {
    size_t g = (work + kBlock - 1) / kBlock;
    const size_t cap = 4 * (size_t)device_cu_count();
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

// Grid of a column kernel: stride (workgroups x 256) a multiple of b.
inline int cgrid(size_t n, int b) {
    int g = bgrid(n * (size_t)b);
    int a = b, c = kBlock;
    while (c) { const int r = a % c; a = c; c = r; }  // gcd(b, 256)
    const int m = b / a;
    return ((g + m - 1) / m) * m;
}

}  // namespace

void blk_svqb(int b, const double *lam, const double *Z, int ldz, double rel, double abs_thr, double *M, int ldm,
              BlockStatus *st, hipStream_t s) {
    hipLaunchKernelGGL(k_svqb, dim3(1), dim3(kBlock), 0, s, b, lam, Z, ldz, rel, abs_thr, M, ldm, st);
    LAP_HIP(hipGetLastError());
}
void blk_cholqr(int b, const double *S, int lds, double rel, double abs_thr, double *M, int ldm, BlockStatus *st,
                hipStream_t s) {
    LAP_REQUIRE(b >= 1 && b <= 32, LAP_EUNSUPPORTED, "CholQR of more than 32 columns");
    hipLaunchKernelGGL(k_cholqr, dim3(1), dim3(kWave), 0, s, b, S, lds, rel, abs_thr, M, ldm, st);
    LAP_HIP(hipGetLastError());
}


template <typename T>
void blk_resid(int n, int bu, const double *U, int ldu, const double *GU, int ldg, int ldr, const double *theta,
               double *R, T *Q, int ldq, int qoff, double *u0, ReduceScratch &rs, BlockStatus *st, hipStream_t s) {
    LAP_REQUIRE(bu <= 32 && ldr <= 32 && bu <= ldr && bu <= ldu && bu <= ldg, LAP_EUNSUPPORTED,
                "block wider than 32");
    const int grid = cgrid(n, ldr);
    rs.ensure(grid + 1, 64);
    double *part = rs.partial.get();
    double *tot = part + (size_t)grid * 64;  // one more row for the totals
    hipLaunchKernelGGL((k_block_resid<T>), dim3(grid), dim3(kBlock), 0, s, n, bu, U, ldu, GU, ldg, ldr, theta, R, Q,
                       ldq, qoff, u0, part);
    hipLaunchKernelGGL((k_bfold<double>), dim3(16), dim3(kBlock), 0, s, part, grid, 64, tot);
    hipLaunchKernelGGL(k_block_resid_status, dim3(1), dim3(64), 0, s, bu, theta, tot, st);
    LAP_HIP(hipGetLastError());
}
template void blk_resid<float>(int, int, const double *, int, const double *, int, int, const double *, double *,
                               float *, int, int, double *, ReduceScratch &, BlockStatus *, hipStream_t);
template void blk_resid<double>(int, int, const double *, int, const double *, int, int, const double *, double *,
                                double *, int, int, double *, ReduceScratch &, BlockStatus *, hipStream_t);

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

void blk_nonfinite_cols(int n, int b, const double *in, int *flags_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_nonfinite_cols, dim3(bgrid((size_t)n * b)), dim3(kBlock), 0, s, n, b, in, flags_dev);
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
                  int ldr, T *X, BPcgWork<T> &w, BlockScratch &bs, int itmax, int it_first, int it_last, double rtol,
                  hipStream_t s) {
    LAP_REQUIRE(b >= 1 && b <= kMaxBlock, LAP_EUNSUPPORTED, "block wider than 32");
    LAP_REQUIRE(it_first >= 1 && it_first <= it_last && it_last <= itmax, LAP_EINVAL, "bad PCG iteration range");
    const int n = P.n;
    const int gc = cgrid(n, b);
    LAP_REQUIRE(w.part.n >= (size_t)gc * 64, LAP_EDEVICE, "block PCG work area too small");
    T *part = w.part.get();
    BPcgState<T> *st = w.st.get();
    const T *dinv = P.dinv<T>();
    T *C = w.C.get();  // q x b column-major coefficients
    T *Z = w.z.get();
    auto fold = [&](int nv, T *totals) {
        const int fg = std::min((nv + kWavesPerBlock - 1) / kWavesPerBlock, 16);
        hipLaunchKernelGGL((k_bfold<T>), dim3(fg), dim3(kBlock), 0, s, part, gc, nv, totals);
    };
    if (it_first == 1) {
        hipLaunchKernelGGL((k_bpcg_init1<T>), dim3(gc), dim3(kBlock), 0, s, n, b, R, ldr, w.res.get(), X, part);
        fold(b, st->tot_a);
        // Res <- (I - QQ')Res
        if (q > 0) {
            ts_tn<T>(n, Q, ldq, q, w.res.get(), b, b, C, q, nullptr, 0, T(1), bs, s);
            ts_nn<T>(n, Q, ldq, q, C, q, b, w.res.get(), b, nullptr, 0, T(-1), T(1), s);
        }
        hipLaunchKernelGGL((k_bpcg_init2<T>), dim3(gc), dim3(kBlock), 0, s, n, b, w.res.get(), w.y.get(), dinv, part,
                           st);
        fold(b, st->tot_b);
        // P = (I - QQ') Y
        const T *Zy = w.y.get();
        if (q > 0) {
            ts_tn<T>(n, Q, ldq, q, w.y.get(), b, b, C, q, nullptr, 0, T(1), bs, s);
            ts_nn<T>(n, Q, ldq, q, C, q, b, Z, b, w.y.get(), b, T(-1), T(0), s);
            Zy = Z;
        }
        hipLaunchKernelGGL((k_bpcg_p0<T>), dim3(gc), dim3(kBlock), 0, s, n, b, Zy, w.p.get(), st);
    }
    constexpr int kFoldRows = 1024;
    LAP_REQUIRE(w.part.n >= (size_t)kFoldRows * 64, LAP_EDEVICE, "block PCG work area too small");
    // the fused iteration for projectors and blocks of up to 32 columns
    const bool fused = q <= 32;
    const int ti = q <= 16 ? 1 : 2, tj = b <= 16 ? 1 : 2;
    const int gt = ts_grid(n);
    const int gn = std::min((n + 63) / 64, 8 * device_cu_count());
    auto reduce = [&](int rows, int cols, T *out) {
        const int rg = std::min((rows * cols + kWavesPerBlock - 1) / kWavesPerBlock, 4 * device_cu_count());
        hipLaunchKernelGGL((k_ts_reduce<T>), dim3(rg), dim3(kBlock), 0, s, gt, w.kt_part.get(), cols, rows * cols, rows,
                           cols, out, rows, nullptr, 0, 0, T(1));
    };
    if (fused) LAP_REQUIRE(w.kt_part.n >= (size_t)gt * kFusedMax, LAP_EDEVICE, "block PCG work area too small");
    if (fused && it_first == 1) {
        // W = Q'D^{-1}Q: rows PI .. 2 PI - 1 of the totals
        if (ti == 1)
            hipLaunchKernelGGL((k_bpcg_kt<T, true, 1, 1>), dim3(gt), dim3(kBlock), 0, s, n, b, q, nullptr, nullptr,
                               nullptr, nullptr, dinv, Q, ldq, w.kt_part.get(), st, 0);
        else
            hipLaunchKernelGGL((k_bpcg_kt<T, true, 2, 2>), dim3(gt), dim3(kBlock), 0, s, n, b, q, nullptr, nullptr,
                               nullptr, nullptr, dinv, Q, ldq, w.kt_part.get(), st, 0);
        reduce(ti == 1 ? fused_ld<1>() : fused_ld<2>(), 16 * ti, w.kt_w.get());
    }
    for (int it = it_first; it <= it_last; ++it) {
        if (fused) {
            // S = G P - P diag(theta) with the column sums p'S (p'Ap) in the same pass
            const int rows = spmm_dot<T>(P, b, w.p.get(), w.s.get(), theta_dev, w.dpart.get(), w.dpart.n / 64, s);
            // the product leaves a row per workgroup (tens of thousands on
            // large graphs): added in two stages, through at most 1024 rows
            const int per = (rows + kFoldRows - 1) / kFoldRows;
            const int f1 = (rows + per - 1) / per;
            hipLaunchKernelGGL((k_bfold_rows<T>), dim3(f1), dim3(kBlock), 0, s, w.dpart.get(), rows, per, part);
            hipLaunchKernelGGL((k_bfold_wide<T>), dim3(b), dim3(kBlock), 0, s, part, f1, st->tot_a);
#define LAP_KT(TI_, TJ_)                                                                                       \
    hipLaunchKernelGGL((k_bpcg_kt<T, false, TI_, TJ_>), dim3(gt), dim3(kBlock), 0, s, n, b, q, X, w.res.get(), \
                       w.p.get(), w.s.get(), dinv, Q, ldq, w.kt_part.get(), st, it)
#define LAP_KN(TI_, TJ_)                                                                                      \
    hipLaunchKernelGGL((k_bpcg_kn<T, TI_, TJ_>), dim3(gn), dim3(kBlock), 0, s, n, b, q, w.res.get(), w.p.get(), \
                       dinv, Q, ldq, w.kt_tot.get(), w.kt_w.get(), st, it, (T)rtol)
            if (ti == 1 && tj == 1) LAP_KT(1, 1);
            else if (ti == 1) LAP_KT(1, 2);
            else if (tj == 1) LAP_KT(2, 1);
            else LAP_KT(2, 2);
            if (it == itmax) break;
            reduce(ti == 1 ? fused_ld<1>() : fused_ld<2>(), 16 * tj, w.kt_tot.get());
            if (ti == 1 && tj == 1) LAP_KN(1, 1);
            else if (ti == 1) LAP_KN(1, 2);
            else if (tj == 1) LAP_KN(2, 1);
            else LAP_KN(2, 2);
#undef LAP_KT
#undef LAP_KN
            continue;
        }
        // S = G P - P diag(theta);  Z = (I - QQ') S
        spmm<T>(P, b, w.p.get(), b, w.s.get(), b, theta_dev, s);
        const T *Zs = w.s.get();
        if (q > 0) {
            ts_tn<T>(n, Q, ldq, q, w.s.get(), b, b, C, q, nullptr, 0, T(1), bs, s);
            ts_nn<T>(n, Q, ldq, q, C, q, b, Z, b, w.s.get(), b, T(-1), T(0), s);
            Zs = Z;
        }
        hipLaunchKernelGGL((k_bpcg_pap<T>), dim3(gc), dim3(kBlock), 0, s, n, b, w.p.get(), w.s.get(), part, st);
        fold(b, st->tot_a);
        hipLaunchKernelGGL((k_bpcg_update<T>), dim3(gc), dim3(kBlock), 0, s, n, b, X, w.res.get(), w.p.get(), Zs,
                           w.y.get(), dinv, part, st, it);
        if (it == itmax) break;
        fold(32 + b, st->tot_b);
        // P = (I - QQ') Y + beta P
        const T *Zy2 = w.y.get();
        if (q > 0) {
            ts_tn<T>(n, Q, ldq, q, w.y.get(), b, b, C, q, nullptr, 0, T(1), bs, s);
            ts_nn<T>(n, Q, ldq, q, C, q, b, Z, b, w.y.get(), b, T(-1), T(0), s);
            Zy2 = Z;
        }
        hipLaunchKernelGGL((k_bpcg_p<T>), dim3(gc), dim3(kBlock), 0, s, n, b, Zy2, w.p.get(), st, it, (T)rtol);
    }
    LAP_HIP(hipGetLastError());
}
template void bpcg_enqueue<float>(const lap_plan &, int, const double *, const float *, int, int, const double *, int,
                                  float *, BPcgWork<float> &, BlockScratch &, int, int, int, double, hipStream_t);
template void bpcg_enqueue<double>(const lap_plan &, int, const double *, const double *, int, int, const double *,
                                   int, double *, BPcgWork<double> &, BlockScratch &, int, int, int, double, hipStream_t);

}  // namespace lapeig
