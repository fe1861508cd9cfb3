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

// Block product, n x b row-major (leading dimensions ldx, ldy).  A lane owns
// one column c < BL of one row slot; a gather of neighbour j reads the b
// contiguous values X[j, 0..b).
//   long rows (degree > the long threshold): split into kChunk-edge chunks,
//     one wavefront per chunk with 64 / BL edge slots; a row of one chunk is
//     written directly, longer rows leave per-chunk partial sums that
//     k_spmm_combine adds in chunk order (deterministic);
//   slice rows: 64 / BL rows per wavefront pass, one lane per (row, column).
template <typename T, bool W, int BL>
__global__ __launch_bounds__(kBlock) void k_spmm(Graph g, Weights<T> w, int b,
                                                 const T *__restrict__ X, int ldx, T *__restrict__ Y, int ldy,
                                                 const double *__restrict__ shift, T *__restrict__ part) {
    constexpr int RPW = kWave / BL;  // row (or edge) slots per wavefront
    const int lane = lane_id();
    const int c = lane % BL;
    const int sub = lane / BL;
    const int gw = blockIdx.x * kWavesPerBlock + wave_id();
    const int nw = gridDim.x * kWavesPerBlock;
    for (int u = gw; u < g.nchunks; u += nw) {
        const int r = g.chunk_row[u];
        const int first = g.chunk_off[r];
        const int nch = g.chunk_off[r + 1] - first;
        const int e0 = g.rowptr[r] + (u - first) * kChunk;
        const int e1 = min(e0 + kChunk, g.rowptr[r + 1]);
        T acc = T(0);
        const T xi = c < b ? X[(size_t)r * ldx + c] : T(0);
        if (c < b) {
            int e = e0 + sub;
            for (; e + 3 * RPW < e1; e += 4 * RPW) {
                const int j0 = g.col[e], j1 = g.col[e + RPW], j2 = g.col[e + 2 * RPW], j3 = g.col[e + 3 * RPW];
                const T d0 = xi - X[(size_t)j0 * ldx + c], d1 = xi - X[(size_t)j1 * ldx + c];
                const T d2 = xi - X[(size_t)j2 * ldx + c], d3 = xi - X[(size_t)j3 * ldx + c];
                if (W) {
                    acc += w.csr[e] * d0; acc += w.csr[e + RPW] * d1;
                    acc += w.csr[e + 2 * RPW] * d2; acc += w.csr[e + 3 * RPW] * d3;
                } else {
                    acc += d0; acc += d1; acc += d2; acc += d3;
                }
            }
            for (; e < e1; e += RPW) acc += (W ? w.csr[e] : T(1)) * (xi - X[(size_t)g.col[e] * ldx + c]);
        }
#pragma unroll
        for (int o = BL; o < kWave; o <<= 1) acc += __shfl_xor(acc, o, kWave);
        if (sub == 0 && c < b) {
            if (nch == 1) {
                const T sh = shift ? T(shift[c]) : T(0);
                Y[(size_t)r * ldy + c] = acc - sh * xi;
            } else {
                part[(size_t)u * b + c] = acc;
            }
        }
    }
    // slice rows: lane groups of b lanes (not BL), 64 / b rows per pass, so a
    // b that is not a power of two leaves at most b - 1 lanes idle; one
    // lane per (row, column), a gather of neighbour j reads its b values
    const int srpw = kWave / b;                 // rows per pass
    const int spass = (kWave + srpw - 1) / srpw;  // passes per 64-row slice
    const int sc = lane % b, ssub = lane / b;
    const int units = g.nslices * spass;
    for (int u = gw; u < units; u += nw) {
        const int s = u / spass;
        const int grp = u % spass;
        const int l = grp * srpw + ssub;
        const int r = g.n_long + s * kWave + l;
        const int c = sc;
        if (ssub < srpw && l < kWave && r < g.n) {
            const int off = g.sell_off[s];
            const int width = (g.sell_off[s + 1] - off) >> 6;
            const T xi = X[(size_t)r * ldx + c];
            T acc = T(0);
            int t = 0;
            for (; t + 3 < width; t += 4) {
                const int a0 = off + t * kWave + l;
                const int j0 = g.sell_col[a0], j1 = g.sell_col[a0 + kWave], j2 = g.sell_col[a0 + 2 * kWave],
                          j3 = g.sell_col[a0 + 3 * kWave];
                const T d0 = xi - X[(size_t)j0 * ldx + c], d1 = xi - X[(size_t)j1 * ldx + c];
                const T d2 = xi - X[(size_t)j2 * ldx + c], d3 = xi - X[(size_t)j3 * ldx + c];
                if (W) {
                    acc += w.sell[a0] * d0; acc += w.sell[a0 + kWave] * d1;
                    acc += w.sell[a0 + 2 * kWave] * d2; acc += w.sell[a0 + 3 * kWave] * d3;
                } else {
                    acc += d0; acc += d1; acc += d2; acc += d3;
                }
            }
            for (; t < width; ++t) {
                const int at = off + t * kWave + l;
                acc += (W ? w.sell[at] : T(1)) * (xi - X[(size_t)g.sell_col[at] * ldx + c]);
            }
            const T sh = shift ? T(shift[c]) : T(0);
            Y[(size_t)r * ldy + c] = acc - sh * xi;
        }
    }
}

// rows split into several chunks: Y = sum of the chunk partials (in chunk
// order) - shift * x.  One wavefront per row of two chunks or more: the
// row's partials (nch x b, contiguous) pass through LDS in tiles of 64
// chunks, each tile loaded with all its loads in flight, and lane c < b adds
// column c of the tile in chunk order.
template <typename T>
__global__ __launch_bounds__(kWave) void k_spmm_combine(Graph g, int b, const T *__restrict__ X, int ldx,
                                                        T *__restrict__ Y, int ldy,
                                                        const double *__restrict__ shift,
                                                        const T *__restrict__ part) {
    constexpr int kTile = kWave;  // chunks per tile
    constexpr int kBatch = 16;    // loads in flight per lane
    __shared__ T tile[kTile * 64];
    const int r = blockIdx.x;
    const int lane = threadIdx.x;
    const int first = g.chunk_off[r], nch = g.chunk_off[r + 1] - first;
    T acc = T(0);
    for (int u0 = 0; u0 < nch; u0 += kTile) {
        const int cnt = (nch - u0 < kTile ? nch - u0 : kTile) * b;
        const T *src = part + (size_t)(first + u0) * b;
        for (int e0 = 0; e0 < cnt; e0 += kBatch * kWave) {
            T v[kBatch];
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const int e = e0 + k * kWave + lane;
                v[k] = e < cnt ? src[e] : T(0);
            }
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const int e = e0 + k * kWave + lane;
                if (e < cnt) tile[e] = v[k];
            }
        }
        __syncthreads();
        if (lane < b)
            for (int e = lane; e < cnt; e += b) acc += tile[e];
        __syncthreads();
    }
    if (lane < b) {
        const T sh = shift ? T(shift[lane]) : T(0);
        Y[(size_t)r * ldy + lane] = acc - sh * X[(size_t)r * ldx + lane];
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
                        T *part_in, hipStream_t s) {
    const Graph &g = P.g;
    long long units = (long long)g.nslices * BL;
    if (g.nchunks > units) units = g.nchunks;
    int grid = (int)((units + kWavesPerBlock - 1) / kWavesPerBlock);
    if (grid < 1) grid = 1;
    if (grid > (1 << 20)) grid = 1 << 20;
    {  // slice passes of 64 / b rows
        const int srpw = kWave / b;
        const long long sunits = (long long)g.nslices * ((kWave + srpw - 1) / srpw);
        const long long vunits = std::max<long long>(sunits, g.nchunks);
        grid = (int)std::min<long long>((vunits + kWavesPerBlock - 1) / kWavesPerBlock, 1 << 20);
        if (grid < 1) grid = 1;
    }
    T *part = nullptr;
    if (g.nchunks > 0) {
        if (part_in) {
            part = part_in;
        } else {
            const size_t bytes = (size_t)g.nchunks * b * sizeof(T);
            lap_plan &mp = const_cast<lap_plan &>(P);
            LAP_REQUIRE(mp.chunk_part.n >= bytes, LAP_EDEVICE, "block-product scratch not reserved");
            part = reinterpret_cast<T *>(mp.chunk_part.get());
        }
    }
    if (P.weighted)
        hipLaunchKernelGGL((k_spmm<T, true, BL>), dim3(grid), dim3(kBlock), 0, s, g, P.weights<T>(), b, X, ldx, Y,
                           ldy, shift, part);
    else
        hipLaunchKernelGGL((k_spmm<T, false, BL>), dim3(grid), dim3(kBlock), 0, s, g, P.weights<T>(), b, X, ldx, Y,
                           ldy, shift, part);
    if (g.n_multi > 0)
        hipLaunchKernelGGL((k_spmm_combine<T>), dim3(g.n_multi), dim3(kWave), 0, s, g, b, X, ldx, Y, ldy, shift,
                           part);
    LAP_HIP(hipGetLastError());
}

template <typename T>
void spmm_part(const lap_plan &P, int b, const T *X, int ldx, T *Y, int ldy, const double *shift_dev, T *part,
               hipStream_t s) {
    if (b <= 1) spmm_launch<T, 1>(P, b, X, ldx, Y, ldy, shift_dev, part, s);
    else if (b <= 2) spmm_launch<T, 2>(P, b, X, ldx, Y, ldy, shift_dev, part, s);
    else if (b <= 4) spmm_launch<T, 4>(P, b, X, ldx, Y, ldy, shift_dev, part, s);
    else if (b <= 8) spmm_launch<T, 8>(P, b, X, ldx, Y, ldy, shift_dev, part, s);
    else if (b <= 16) spmm_launch<T, 16>(P, b, X, ldx, Y, ldy, shift_dev, part, s);
    else if (b <= 32) spmm_launch<T, 32>(P, b, X, ldx, Y, ldy, shift_dev, part, s);
    else spmm_launch<T, 64>(P, b, X, ldx, Y, ldy, shift_dev, part, s);
}

template <typename T>
void spmm(const lap_plan &P, int b, const T *X, int ldx, T *Y, int ldy, const double *shift_dev, hipStream_t s) {
    spmm_part<T>(P, b, X, ldx, Y, ldy, shift_dev, nullptr, s);
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
template void spmm_part<float>(const lap_plan &, int, const float *, int, float *, int, const double *, float *,
                               hipStream_t);
template void spmm_part<double>(const lap_plan &, int, const double *, int, double *, int, const double *, double *,
                                hipStream_t);
template void spmm<double>(const lap_plan &, int, const double *, int, double *, int, const double *, hipStream_t);
template void permute_rows<float>(const int *, int, int, const float *, float *, hipStream_t);
template void permute_rows<double>(const int *, int, int, const double *, double *, hipStream_t);

void ReduceScratch::ensure_deferred() {
    if (!dpart.get()) {
        darea = std::max(kDeferRows, 2 * device_cu_count());
        dpart.alloc(2 * (size_t)darea * 64);
    }
}

void ReduceScratch::ensure(int blocks, int values) {
    if (blocks <= max_blocks && values <= max_values && partial.get()) return;
    max_blocks = std::max(blocks, max_blocks);
    max_values = std::max(values, max_values);
    partial.alloc((size_t)max_blocks * max_values);
    counter.alloc(64);
    LAP_HIP(hipMemset(counter.get(), 0, 64 * sizeof(unsigned)));
}

}  // namespace lapeig
