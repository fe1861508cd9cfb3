// Laplacian products: the matrix-vector product (MVP) of Section 3,
// y = (G - sigma I) x, and its n x b block form, in plan order.
#include <type_traits>

#include "lapeig_dev.h"

namespace lapeig {

namespace {

template <typename T, bool W>
__global__ __launch_bounds__(kBlock) void k_spmv(Graph g, Weights<T> w, const T *__restrict__ x,
                                                 T *__restrict__ y, T sigma) {
    for_each_row<T, W, false>(g, w, x, [&](int i, T xi, T yi, T) { y[i] = yi - sigma * xi; });
}

// V consecutive values moved by one V-wide load or store (the address is
// aligned to V values: the host checks it before choosing V > 1)
template <typename T, int V>
struct alignas(sizeof(T) * V) Pack {
    T v[V];
};
template <typename T, int V>
__device__ __forceinline__ Pack<T, V> load_pack(const T *p) {
    return *reinterpret_cast<const Pack<T, V> *>(p);
}
template <typename T, int V>
__device__ __forceinline__ void store_pack(T *p, const Pack<T, V> &x) {
    *reinterpret_cast<Pack<T, V> *>(p) = x;
}

// Block product, n x b row-major (leading dimensions ldx, ldy).  A lane owns
// one column c < BL of one row slot; a gather of neighbour j reads the b
// contiguous values X[j, 0..b).
//   long rows (degree > the long threshold): split into kChunk-edge chunks,
//     one wavefront per chunk with 64 / BL edge slots; a row of one chunk is
//     written directly, longer rows leave per-chunk partial sums that
//     k_spmm_combine adds in chunk order (deterministic);
//   slice rows: see below.
//   DOT: also the column sums of X o Y over the rows the workgroup writes,
//     one row of 64 values per workgroup in dpart (columns past b zero),
//     each added in a fixed lane and wavefront order.
template <typename T, bool W, int BL, int V, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmm(Graph g, Weights<T> w, int b,
                                                 const T *__restrict__ X, int ldx, T *__restrict__ Y, int ldy,
                                                 const double *__restrict__ shift, T *__restrict__ part,
                                                 T *__restrict__ dpart) {
    constexpr int RPW = kWave / BL;  // row (or edge) slots per wavefront
    T dch = T(0), dsl[V];  // X o Y sums: chunk rows (column c), slice rows (columns vc..)
#pragma unroll
    for (int e = 0; e < V; ++e) dsl[e] = T(0);
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
                const T yv = acc - sh * xi;
                Y[(size_t)r * ldy + c] = yv;
                if (DOT) dch += xi * yv;
            } else {
                part[(size_t)u * b + c] = acc;
            }
        }
    }
    // slice rows: a lane owns V consecutive columns of one row (one V-wide
    // load per gather), b / V lanes per row and 64 / (b / V) rows per
    // wavefront; a unit's rows run on across slice boundaries (each lane
    // finds its own slice), so only the lanes past the last whole row group
    // idle.  Edges go in batches of 8 independent gathers, then one of 4, then
    // a last batch of 4 whose entries past the slice width read the row
    // itself with weight 0 (exact zeros, as the slice padding does); every
    // column adds its edges in slice order.
    const int gl = b / V;
    const int spr = kWave / gl;
    const int vsub = lane / gl;
    const int vc = (lane % gl) * V;
    const int nsr = g.n - g.n_long;
    const int sunits = (nsr + spr - 1) / spr;
    for (int u = gw; u < sunits; u += nw) {
        const int q = u * spr + vsub;
        if (vsub >= spr || q >= nsr) continue;
        const int r = g.n_long + q;
        const int s = q >> 6;
        const int off = g.sell_off[s] + (q & (kWave - 1));
        const int width = (g.sell_off[s + 1] - g.sell_off[s]) >> 6;
        const Pack<T, V> xi = load_pack<T, V>(X + (size_t)r * ldx + vc);
        Pack<T, V> acc;
#pragma unroll
        for (int e = 0; e < V; ++e) acc.v[e] = T(0);
        auto batch = [&](int t, auto ucount, auto masked) {
            constexpr int U = decltype(ucount)::value;
            constexpr bool M = decltype(masked)::value;
            int j[U];
            T wt[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int tk = t + k;
                const int a = off + (M && tk >= width ? width - 1 : tk) * kWave;
                const int jj = g.sell_col[a];
                j[k] = M && tk >= width ? r : jj;
                if (W) wt[k] = M && tk >= width ? T(0) : w.sell[a];
            }
            Pack<T, V> xv[U];
#pragma unroll
            for (int k = 0; k < U; ++k) xv[k] = load_pack<T, V>(X + (size_t)j[k] * ldx + vc);
#pragma unroll
            for (int k = 0; k < U; ++k)
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    if (W) acc.v[e] += wt[k] * (xi.v[e] - xv[k].v[e]);
                    else acc.v[e] += xi.v[e] - xv[k].v[e];
                }
        };
        int t = 0;
        for (; t + 8 <= width; t += 8) batch(t, std::integral_constant<int, 8>(), std::false_type());
        if (t + 4 <= width) {
            batch(t, std::integral_constant<int, 4>(), std::false_type());
            t += 4;
        }
        if (t < width) batch(t, std::integral_constant<int, 4>(), std::true_type());
        Pack<T, V> out;
#pragma unroll
        for (int e = 0; e < V; ++e) out.v[e] = acc.v[e] - (shift ? T(shift[vc + e]) : T(0)) * xi.v[e];
        store_pack<T, V>(Y + (size_t)r * ldy + vc, out);
        if (DOT) {
#pragma unroll
            for (int e = 0; e < V; ++e) dsl[e] += xi.v[e] * out.v[e];
        }
    }
    if constexpr (DOT) {
        __shared__ T red[kBlock * (V + 1)];
#pragma unroll
        for (int e = 0; e < V; ++e) red[threadIdx.x * (V + 1) + e] = dsl[e];
        red[threadIdx.x * (V + 1) + V] = dch;
        __syncthreads();
        if (threadIdx.x < kWave) {
            const int j = threadIdx.x;
            T sum = T(0);
            if (j < b) {
                // chunk rows: lane j of each wavefront (sub 0, column j);
                // slice rows: lanes (j / V) + gl t, t < spr, element j % V
                const int lg = j / V, e = j % V;
                for (int wv = 0; wv < kWavesPerBlock; ++wv) {
                    const T *rw = red + (size_t)wv * kWave * (V + 1);
                    sum += rw[j * (V + 1) + V];
                    for (int t = 0; t < spr; ++t) sum += rw[(lg + gl * t) * (V + 1) + e];
                }
            }
            dpart[(size_t)blockIdx.x * kWave + j] = sum;
        }
    }
}

// rows split into several chunks: Y = sum of the chunk partials (in chunk
// order) - shift * x.  Lane groups of b lanes, 64 / b rows per wavefront:
// lane c of a group adds column c of its row's partials (nch x b,
// contiguous), eight loads in flight, in chunk order.
// DOT: the column sums of X o Y over these rows, as k_spmm leaves them.
template <typename T, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmm_combine(Graph g, int b, const T *__restrict__ X, int ldx,
                                                         T *__restrict__ Y, int ldy,
                                                         const double *__restrict__ shift,
                                                         const T *__restrict__ part, T *__restrict__ dpart) {
    const int lane = lane_id();
    const int rpw = kWave / b;
    const int sub = lane / b, c = lane % b;
    T dsum = T(0);
    const int gw = blockIdx.x * kWavesPerBlock + wave_id();
    const int nw = gridDim.x * kWavesPerBlock;
    const int units = (g.n_multi + rpw - 1) / rpw;
    for (int u = gw; u < units; u += nw) {
        const int r = u * rpw + sub;
        if (sub >= rpw || r >= g.n_multi) continue;
        const int first = g.chunk_off[r], nch = g.chunk_off[r + 1] - first;
        const T *src = part + (size_t)first * b + c;
        T acc = T(0);
        int k = 0;
        for (; k + 8 <= nch; k += 8) {
            T v[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) v[m] = src[(size_t)(k + m) * b];
#pragma unroll
            for (int m = 0; m < 8; ++m) acc += v[m];
        }
        for (; k < nch; ++k) acc += src[(size_t)k * b];
        const T sh = shift ? T(shift[c]) : T(0);
        const T xv = X[(size_t)r * ldx + c];
        const T yv = acc - sh * xv;
        Y[(size_t)r * ldy + c] = yv;
        if (DOT) dsum += xv * yv;
    }
    if constexpr (DOT) {
        __shared__ T red[kBlock];
        red[threadIdx.x] = dsum;
        __syncthreads();
        if (threadIdx.x < kWave) {
            const int j = threadIdx.x;
            T sum = T(0);
            if (j < b)
                for (int wv = 0; wv < kWavesPerBlock; ++wv)
                    for (int t = 0; t < rpw; ++t) sum += red[wv * kWave + j + b * t];
            dpart[(size_t)blockIdx.x * kWave + j] = sum;
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

// Widest lane vector V (values per lane in the slice rows, at most 16
// bytes) that divides b, leaves at least four lanes per row (a gather
// instruction then spans at most 16 rows: wider loads spread over more rows
// measured slower), and keeps every row of X and Y aligned to V values.
template <typename T>
static int spmm_vec_width(int b, const T *X, int ldx, const T *Y, int ldy) {
    for (int v = 16 / (int)sizeof(T); v > 1; v >>= 1) {
        const uintptr_t al = (uintptr_t)v * sizeof(T);
        if (b % v == 0 && b / v >= 4 && b / v <= kWave && ldx % v == 0 && ldy % v == 0 &&
            (uintptr_t)X % al == 0 && (uintptr_t)Y % al == 0)
            return v;
    }
    return 1;
}

// workgroups of the block product: one unit (a chunk, or a group of slice
// rows of spr rows) per wavefront
static int spmm_grid(const Graph &g, int spr) {
    const long long sunits = ((long long)(g.n - g.n_long) + spr - 1) / spr;
    const long long units = std::max<long long>(sunits, g.nchunks);
    return (int)std::max<long long>(1, std::min<long long>((units + kWavesPerBlock - 1) / kWavesPerBlock, 1 << 20));
}


// workgroups of the hub-row combine (rows of more than one chunk)
static int combine_grid(const Graph &g, int b) {
    const int rpw = kWave / b;
    const int cunits = (g.n_multi + rpw - 1) / rpw;
    return (cunits + kWavesPerBlock - 1) / kWavesPerBlock;
}

template <typename T, int BL, int V, bool DOT>
static int spmm_launch_v(const lap_plan &P, int b, const T *X, int ldx, T *Y, int ldy, const double *shift,
                         T *part, T *dpart, hipStream_t s) {
    const Graph &g = P.g;
    const int grid = spmm_grid(g, kWave / (b / V));
    if (P.weighted)
        hipLaunchKernelGGL((k_spmm<T, true, BL, V, DOT>), dim3(grid), dim3(kBlock), 0, s, g, P.weights<T>(), b, X,
                           ldx, Y, ldy, shift, part, dpart);
    else
        hipLaunchKernelGGL((k_spmm<T, false, BL, V, DOT>), dim3(grid), dim3(kBlock), 0, s, g, P.weights<T>(), b, X,
                           ldx, Y, ldy, shift, part, dpart);
    return grid;
}

template <typename T, int BL, bool DOT = false>
static int spmm_launch(const lap_plan &P, int b, const T *X, int ldx, T *Y, int ldy, const double *shift,
                       T *part_in, hipStream_t s, T *dpart = nullptr) {
    const Graph &g = P.g;
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
    const int v = spmm_vec_width<T>(b, X, ldx, Y, ldy);
    int rows;
    if (v == 4) rows = spmm_launch_v<T, BL, 4, DOT>(P, b, X, ldx, Y, ldy, shift, part, dpart, s);
    else if (v == 2) rows = spmm_launch_v<T, BL, 2, DOT>(P, b, X, ldx, Y, ldy, shift, part, dpart, s);
    else rows = spmm_launch_v<T, BL, 1, DOT>(P, b, X, ldx, Y, ldy, shift, part, dpart, s);
    if (g.n_multi > 0) {
        const int cg = combine_grid(g, b);
        hipLaunchKernelGGL((k_spmm_combine<T, DOT>), dim3(cg), dim3(kBlock), 0, s, g, b, X, ldx, Y, ldy, shift, part,
                           DOT ? dpart + (size_t)rows * kWave : nullptr);
        rows += cg;
    }
    LAP_HIP(hipGetLastError());
    return rows;
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

int spmm_dot_rows(const lap_plan &P, int b) {
    // one value per lane (V = 1) gives the fewest rows per wavefront, hence
    // the most workgroups, for every width up to b
    const int bmax = std::max(1, std::min(b, kWave));
    return spmm_grid(P.g, kWave / bmax) + (P.g.n_multi > 0 ? combine_grid(P.g, bmax) : 0);
}

template <typename T>
int spmm_dot(const lap_plan &P, int b, const T *X, T *Y, const double *shift_dev, T *dpart, size_t dpart_rows,
             hipStream_t s) {
    LAP_REQUIRE(b >= 1 && b <= 32, LAP_EUNSUPPORTED, "block product with sums wider than 32");
    LAP_REQUIRE((size_t)spmm_dot_rows(P, b) <= dpart_rows, LAP_EDEVICE, "block-product sum area too small");
    if (b <= 1) return spmm_launch<T, 1, true>(P, b, X, b, Y, b, shift_dev, nullptr, s, dpart);
    if (b <= 2) return spmm_launch<T, 2, true>(P, b, X, b, Y, b, shift_dev, nullptr, s, dpart);
    if (b <= 4) return spmm_launch<T, 4, true>(P, b, X, b, Y, b, shift_dev, nullptr, s, dpart);
    if (b <= 8) return spmm_launch<T, 8, true>(P, b, X, b, Y, b, shift_dev, nullptr, s, dpart);
    if (b <= 16) return spmm_launch<T, 16, true>(P, b, X, b, Y, b, shift_dev, nullptr, s, dpart);
    return spmm_launch<T, 32, true>(P, b, X, b, Y, b, shift_dev, nullptr, s, dpart);
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
template int spmm_dot<float>(const lap_plan &, int, const float *, float *, const double *, float *, size_t,
                             hipStream_t);
template int spmm_dot<double>(const lap_plan &, int, const double *, double *, const double *, double *, size_t,
                              hipStream_t);
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
