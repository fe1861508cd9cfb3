// Laplacian products: the matrix-vector product (MVP) of Section 3,
// y = (G - sigma I) x, and its n x b block form, in plan order.
#include "lapeig_dev.h"

namespace lapeig {

namespace {

template <typename T, bool W>
__global__ __launch_bounds__(kBlock) void k_spmv(Graph g, Weights<T> w, const T *__restrict__ x,
                                                 T *__restrict__ y, T sigma) {
    for_each_row<T, W, false>(g, w, x, [&](int i, T xi, T yi, T) { y[i] = yi - sigma * xi; });
}

// Block product, n x b row-major.  One lane per (row, column) for slice rows:
// a wavefront handles 64 / BL rows with BL lanes each (BL >= b columns, a power
// of two), so a neighbour gather reads b contiguous values.  Long and huge
// rows: a wavefront (or workgroup) per row, each lane striding the row for
// one column group.
template <typename T, bool W, int BL>
__global__ __launch_bounds__(kBlock) void k_spmm(Graph g, Weights<T> w, int b,
                                                 const T *__restrict__ X, int ldx, T *__restrict__ Y, int ldy,
                                                 const double *__restrict__ shift) {
    constexpr int RPW = kWave / BL;  // rows per wavefront in the slice part
    const int lane = lane_id();
    const int c = lane % BL;         // column of this lane
    const int sub = lane / BL;       // row slot within the wavefront
    // long and huge rows: wavefront per row, lanes (sub) stride edges, c columns
    const int nrow_wave = g.n_long;
    for (int r = blockIdx.x * kWavesPerBlock + wave_id(); r < nrow_wave;
         r += gridDim.x * kWavesPerBlock) {
        T acc = T(0);
        T xi = c < b ? X[(size_t)r * ldx + c] : T(0);
        const int e1 = g.rowptr[r + 1];
        for (int e = g.rowptr[r] + sub; e < e1; e += RPW) {
            if (c < b) {
                const T d = xi - X[(size_t)g.col[e] * ldx + c];
                acc += (W ? w.csr[e] : T(1)) * d;
            }
        }
        // reduce over the RPW row slots holding the same column
#pragma unroll
        for (int o = BL; o < kWave; o <<= 1) acc += __shfl_xor(acc, o, kWave);
        if (sub == 0 && c < b) {
            const T s = shift ? T(shift[c]) : T(0);
            Y[(size_t)r * ldy + c] = acc - s * xi;
        }
    }
    // slice rows: each slice of 64 rows is handled by 64 / RPW passes
    const int nslices = g.nslices;
    const int units = nslices * BL;  // (slice, group of RPW rows)
    for (int u = blockIdx.x * kWavesPerBlock + wave_id(); u < units; u += gridDim.x * kWavesPerBlock) {
        const int s = u / BL;
        const int grp = u % BL;
        const int l = grp * RPW + sub;  // lane of the slice this row occupies
        const int r = g.n_long + s * kWave + l;
        if (r < g.n && c < b) {
            const int off = g.sell_off[s];
            const int width = (g.sell_off[s + 1] - off) >> 6;
            const T xi = X[(size_t)r * ldx + c];
            T acc = T(0);
#pragma unroll 4
            for (int t = 0; t < width; ++t) {
                const int at = off + t * kWave + l;
                const T d = xi - X[(size_t)g.sell_col[at] * ldx + c];
                acc += (W ? w.sell[at] : T(1)) * d;
            }
            const T sh = shift ? T(shift[c]) : T(0);
            Y[(size_t)r * ldy + c] = acc - sh * xi;
        }
    }
}

template <typename T>
__global__ void k_permute_rows(const int *__restrict__ map, int n, int b, const T *__restrict__ in,
                               T *__restrict__ out) {
    const size_t total = (size_t)n * b;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        const size_t i = t / b, c = t % b;
        out[(size_t)map[i] * b + c] = in[t];
    }
}

}  // namespace

template <typename T>
void spmv(const lap_plan &P, const T *x, T *y, double sigma, hipStream_t s) {
    const int grid = row_grid(P.g, 1 << 20);
    if (P.weighted)
        hipLaunchKernelGGL((k_spmv<T, true>), dim3(grid), dim3(kBlock), 0, s, P.g, P.weights<T>(), x, y,
                           T(sigma));
    else
        hipLaunchKernelGGL((k_spmv<T, false>), dim3(grid), dim3(kBlock), 0, s, P.g, P.weights<T>(), x,
                           y, T(sigma));
    LAP_HIP(hipGetLastError());
}

template <typename T, int BL>
static void spmm_launch(const lap_plan &P, int b, const T *X, int ldx, T *Y, int ldy, const double *shift,
                        hipStream_t s) {
    const Graph &g = P.g;
    long long units = (long long)g.nslices * BL;
    if (g.n_long > units) units = g.n_long;
    int grid = (int)((units + kWavesPerBlock - 1) / kWavesPerBlock);
    if (grid < 1) grid = 1;
    if (grid > (1 << 20)) grid = 1 << 20;
    if (P.weighted)
        hipLaunchKernelGGL((k_spmm<T, true, BL>), dim3(grid), dim3(kBlock), 0, s, g, P.weights<T>(), b, X,
                           ldx, Y, ldy, shift);
    else
        hipLaunchKernelGGL((k_spmm<T, false, BL>), dim3(grid), dim3(kBlock), 0, s, g, P.weights<T>(), b, X,
                           ldx, Y, ldy, shift);
    LAP_HIP(hipGetLastError());
}

template <typename T>
void spmm(const lap_plan &P, int b, const T *X, int ldx, T *Y, int ldy, const double *shift_dev, hipStream_t s) {
    if (b <= 1) spmm_launch<T, 1>(P, b, X, ldx, Y, ldy, shift_dev, s);
    else if (b <= 2) spmm_launch<T, 2>(P, b, X, ldx, Y, ldy, shift_dev, s);
    else if (b <= 4) spmm_launch<T, 4>(P, b, X, ldx, Y, ldy, shift_dev, s);
    else if (b <= 8) spmm_launch<T, 8>(P, b, X, ldx, Y, ldy, shift_dev, s);
    else if (b <= 16) spmm_launch<T, 16>(P, b, X, ldx, Y, ldy, shift_dev, s);
    else if (b <= 32) spmm_launch<T, 32>(P, b, X, ldx, Y, ldy, shift_dev, s);
    else spmm_launch<T, 64>(P, b, X, ldx, Y, ldy, shift_dev, s);
}

template <typename T>
void spmm(const lap_plan &P, int b, const T *X, T *Y, const double *shift_dev, hipStream_t s) {
    spmm<T>(P, b, X, b, Y, b, shift_dev, s);
}

template <typename T>
void permute_rows(const int *map, int n, int b, const T *in, T *out, hipStream_t s) {
    size_t total = (size_t)n * b;
    int grid = (int)std::min<size_t>((total + kBlock - 1) / kBlock, 65536);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((k_permute_rows<T>), dim3(grid), dim3(kBlock), 0, s, map, n, b, in, out);
    LAP_HIP(hipGetLastError());
}

template void spmv<float>(const lap_plan &, const float *, float *, double, hipStream_t);
template void spmv<double>(const lap_plan &, const double *, double *, double, hipStream_t);
template void spmm<float>(const lap_plan &, int, const float *, float *, const double *, hipStream_t);
template void spmm<double>(const lap_plan &, int, const double *, double *, const double *, hipStream_t);
template void spmm<float>(const lap_plan &, int, const float *, int, float *, int, const double *, hipStream_t);
template void spmm<double>(const lap_plan &, int, const double *, int, double *, int, const double *, hipStream_t);
template void permute_rows<float>(const int *, int, int, const float *, float *, hipStream_t);
template void permute_rows<double>(const int *, int, int, const double *, double *, hipStream_t);

void ReduceScratch::ensure(int blocks, int values) {
    if (blocks <= max_blocks && values <= max_values && partial.get()) return;
    max_blocks = std::max(blocks, max_blocks);
    max_values = std::max(values, max_values);
    partial.alloc((size_t)max_blocks * max_values);
    counter.alloc(64);
    LAP_HIP(hipMemset(counter.get(), 0, 64 * sizeof(unsigned)));
}

}  // namespace lapeig
