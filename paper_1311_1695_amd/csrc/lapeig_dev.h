// Device-side building blocks shared by the kernels: wavefront and workgroup
// reductions, the deterministic cross-workgroup reduction, and the row
// engine that evaluates Laplacian rows in edge-difference form.
#pragma once

#include "lapeig_internal.h"

namespace lapeig {

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / kWave; }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum over the 256 threads of a workgroup; every thread gets the result.
// Fixed combination order, so the result is deterministic.
template <typename T>
__device__ __forceinline__ T block_sum(T v) {
    __shared__ T sm[kWavesPerBlock];
    v = wave_sum(v);
    __syncthreads();
    if (lane_id() == 0) sm[wave_id()] = v;
    __syncthreads();
    T r = sm[0];
#pragma unroll
    for (int w = 1; w < kWavesPerBlock; ++w) r += sm[w];
    return r;
}

// Device-coherent stores and loads (visible across XCDs within a launch).
template <typename T>
__device__ __forceinline__ void store_agent(T *p, T v) {
    if constexpr (sizeof(T) == 8) {
        __hip_atomic_store(reinterpret_cast<unsigned long long *>(p),
                           __builtin_bit_cast(unsigned long long, v), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    } else {
        static_assert(sizeof(T) == 4, "4- or 8-byte types only");
        __hip_atomic_store(reinterpret_cast<unsigned *>(p), __builtin_bit_cast(unsigned, v),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}
template <typename T>
__device__ __forceinline__ T load_agent(const T *p) {
    if constexpr (sizeof(T) == 8) {
        unsigned long long b = __hip_atomic_load(
            reinterpret_cast<unsigned long long *>(const_cast<T *>(p)), __ATOMIC_RELAXED,
            __HIP_MEMORY_SCOPE_AGENT);
        return __builtin_bit_cast(T, b);
    } else {
        static_assert(sizeof(T) == 4, "4- or 8-byte types only");
        unsigned b = __hip_atomic_load(reinterpret_cast<unsigned *>(const_cast<T *>(p)),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return __builtin_bit_cast(T, b);
    }
}

// Cross-workgroup sum of nv <= NV <= 64 per-thread values (acc[0..nv)).
// Every workgroup writes its nv partial sums (wavefront 0 does it, so one
// release fence by its lane 0 orders them before the completion counter);
// the last workgroup to finish adds all partials, in workgroup order, with
// every thread loading a share in parallel, and leaves the totals in
// out[0..nv) (its shared memory), resets the counter, and returns true.
// Deterministic: the summation order depends only on the grid size.
// All workgroups of the grid must call it (no early exits before it).
template <typename T, int NV>
__device__ bool grid_reduce(const T (&acc)[NV], int nv, T *partial, unsigned *counter, T *out) {
    static_assert(NV <= kWave, "at most 64 values per reduction");
    constexpr int NVP = NV <= 1 ? 1 : NV <= 2 ? 2 : NV <= 4 ? 4 : NV <= 8 ? 8 : NV <= 16 ? 16 : NV <= 32 ? 32 : 64;
    constexpr int GROUPS = kBlock / NVP;
    __shared__ T red[kWavesPerBlock][NV];
    __shared__ T fin[GROUPS][NVP];
    __shared__ int is_last;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        if (j < nv) {
            T s = wave_sum(acc[j]);
            if (lane_id() == 0) red[wave_id()][j] = s;
        }
    }
    __syncthreads();
    if (threadIdx.x < kWave) {
        const int j = threadIdx.x;
        if (j < nv) {
            T s = red[0][j];
#pragma unroll
            for (int w = 1; w < kWavesPerBlock; ++w) s += red[w][j];
            store_agent(partial + (size_t)blockIdx.x * NV + j, s);
        }
        if (j == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            is_last = (prev == gridDim.x - 1);
            if (is_last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
    }
    __syncthreads();
    if (!is_last) return false;
    {
        const int j = threadIdx.x % NVP, g = threadIdx.x / NVP;
        T s = T(0);
        if (j < nv)
            for (int b = g; b < (int)gridDim.x; b += GROUPS) s += load_agent(partial + (size_t)b * NV + j);
        fin[g][j] = s;
    }
    __syncthreads();
    if (threadIdx.x < nv) {
        T s = fin[0][threadIdx.x];
        for (int g = 1; g < GROUPS; ++g) s += fin[g][threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) store_agent(counter, 0u);
    return true;
}

// Matrix-core 16x16x4 multiply-accumulate, wave64.  Operand layout: lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator element r of
// lane l is D[row(l, r)][l % 16] with row = 4 (l / 16) + r for the FP32
// instruction and row = l / 16 + 4 r for the FP64 one (both checked on the
// device).
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Deferred cross-workgroup sums.  A producer launch leaves one row of nv
// partial sums per workgroup (plain stores); the launch after it, which the
// kernel boundary makes them visible to, folds them in every workgroup in
// the same fixed order, so all workgroups obtain bit-identical totals with
// no atomics and no cache maintenance inside either kernel.
constexpr int pow2_at_least(int v) { return v <= 1 ? 1 : v <= 2 ? 2 : v <= 4 ? 4 : v <= 8 ? 8 : v <= 16 ? 16 : v <= 32 ? 32 : 64; }

// x of lane (lane ^ M) for M = 1, 2, 4, 8 by data-parallel moves on the
// vector ALU (quad permutations for 1 and 2; for 4 the row shifted by four
// lanes one way or the other by lane bit 2; for 8 the 16-lane row rotated
// by eight), 16 and 32 through the LDS crossbar (ds_bpermute).  The partner
// is the same either way, so results do not depend on the route.  Every
// lane of the wavefront must be active.
template <int M>
__device__ __forceinline__ int lane_xor32(int x) {
    if constexpr (M == 1) {
        return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);  // quad_perm [1, 0, 3, 2]
    } else if constexpr (M == 2) {
        return __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);  // quad_perm [2, 3, 0, 1]
    } else if constexpr (M == 4) {
        const int from_up = __builtin_amdgcn_update_dpp(0, x, 0x104, 0xF, 0xF, false);  // row_shl:4
        const int from_dn = __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);  // row_shr:4
        return (threadIdx.x & 4) ? from_dn : from_up;
    } else {
        static_assert(M == 8, "M must be 1, 2, 4 or 8");
        return __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false);  // row_ror:8
    }
}
template <int M, typename T>
__device__ __forceinline__ T lane_xor(T v) {
    if constexpr (M >= 16) {
        return __shfl_xor(v, M, kWave);
    } else if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, lane_xor32<M>(__builtin_bit_cast(int, v)));
    } else {
        static_assert(sizeof(T) == 8, "4- or 8-byte types only");
        const long long b = __builtin_bit_cast(long long, v);
        const unsigned lo = (unsigned)lane_xor32<M>((int)b), hi = (unsigned)lane_xor32<M>((int)(b >> 32));
        return __builtin_bit_cast(T, (long long)(((unsigned long long)hi << 32) | lo));
    }
}

// Reduce-scatter of NV per-lane values over the wavefront (NV a power of
// two): each butterfly step trades half of the remaining values with the
// partner lane, so NV values cost NV - 1 + log2(64 / NV) shuffles instead of
// 6 NV (the four lowest steps move data on the vector ALU, lane_xor).
// Afterwards v[0] holds the wavefront total of value idx, where idx
// collects the halving bits of the lane; lanes that agree on them hold the
// same total, and every total is added in one fixed order.
template <typename T, int NV, int CNT, int M>
__device__ __forceinline__ void rs_step(T (&v)[NV], int lane, int &idx) {
    if constexpr (M >= 1) {
        if constexpr (CNT > 1) {
            constexpr int half = CNT / 2;
            const bool up = (lane & M) != 0;
#pragma unroll
            for (int i = 0; i < half; ++i) {
                const T keep = up ? v[half + i] : v[i];
                const T give = up ? v[i] : v[half + i];
                v[i] = keep + lane_xor<M>(give);
            }
            if (up) idx += half;
            rs_step<T, NV, half, M / 2>(v, lane, idx);
        } else {
            v[0] += lane_xor<M>(v[0]);
            rs_step<T, NV, 1, M / 2>(v, lane, idx);
        }
    }
}

template <typename T, int NV>
__device__ __forceinline__ int wave_reduce_scatter(T (&v)[NV]) {
    static_assert((NV & (NV - 1)) == 0 && NV >= 1 && NV <= kWave, "NV must be a power of two <= 64");
    int idx = 0;
    rs_step<T, NV, NV, kWave / 2>(v, lane_id(), idx);
    return idx;
}

// Leaves this workgroup's nv sums of acc (destroyed) in part[blockIdx.x][.].
template <typename T, int NV>
__device__ __forceinline__ void write_partials(T (&acc)[NV], int nv, T *__restrict__ part) {
    static_assert(NV <= kWave, "at most 64 values per reduction");
    __shared__ T red[kWavesPerBlock][NV];
    const int idx = wave_reduce_scatter<T, NV>(acc);
    if ((lane_id() & (kWave / NV - 1)) == 0 && idx < nv) red[wave_id()][idx] = acc[0];
    __syncthreads();
    if (threadIdx.x < nv) {
        T s = red[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < kWavesPerBlock; ++w) s += red[w][threadIdx.x];
        part[(size_t)blockIdx.x * NV + threadIdx.x] = s;
    }
}

// out[0..nv) = sum over the nb partial rows of part (row stride NV).  Thread
// (g, j) adds rows g, g + G, g + 2G, ... of value j in row order, with up to
// 32 loads in flight (8 for 64 double values); the G group sums are then added in group order;
// out[nv..NV) is set to zero.  Synchronizes the workgroup.
template <typename T, int NV>
__device__ __forceinline__ void fold_partials(const T *__restrict__ part, int nb, int nv, T *out) {
    constexpr int NVP = pow2_at_least(NV);
    constexpr int GROUPS = kBlock / NVP;
    constexpr int U = (sizeof(T) == 8 && NV >= 64) ? 8 : 32;  // registers of the widest case
    __shared__ T fin[GROUPS][NVP];
    const int j = threadIdx.x % NVP, g = threadIdx.x / NVP;
    T s = T(0);
    if (j < nv) {
        for (int b0 = g; b0 < nb; b0 += U * GROUPS) {
            T a[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int b = b0 + u * GROUPS;
                a[u] = b < nb ? part[(size_t)b * NV + j] : T(0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) s += a[u];
        }
    }
    fin[g][j] = s;
    __syncthreads();
    if (threadIdx.x < NV) {  // values nv .. NV-1 come out as zeros
        T t = fin[0][threadIdx.x];
#pragma unroll
        for (int q = 1; q < GROUPS; ++q) t += fin[q][threadIdx.x];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Row engine.  For every row i of the grid's share it computes
//   y_i = sum_{j in N(i)} w_ij (x_i - x_j)        ( = (G x)_i )
//   q_i = sum_{j in N(i)} w_ij (x_i - x_j)^2      (only when QF; sum_i q_i = 2 x'Gx, eq. (1))
// and calls f(i, x_i, y_i, q_i) on exactly one lane per row (for_each_row_pre
// also passes f what pre(i) loaded for the row before its gathers began).  Rows are
// visited workgroup-per-row (huge), wavefront-per-row (long), eight
// lanes per row (the rows of the wide slices), then lane-per-row inside
// 64-row slices; the grid strides over the units.
// Every loop keeps four independent index->gather chains in flight, and the
// summation order is fixed, so results are reproducible bit for bit.
// f must not synchronize.
// ---------------------------------------------------------------------------
template <typename T, bool WEIGHTED, bool QF>
__device__ __forceinline__ void edge_terms(const int *__restrict__ col, const T *__restrict__ wt,
                                           const T *__restrict__ x, T xi, int e, int e1, int stride,
                                           T &acc, T &aq) {
    for (; e + 3 * stride < e1; e += 4 * stride) {
        const int j0 = col[e], j1 = col[e + stride], j2 = col[e + 2 * stride], j3 = col[e + 3 * stride];
        T w0 = T(1), w1 = T(1), w2 = T(1), w3 = T(1);
        if (WEIGHTED) { w0 = wt[e]; w1 = wt[e + stride]; w2 = wt[e + 2 * stride]; w3 = wt[e + 3 * stride]; }
        const T d0 = xi - x[j0], d1 = xi - x[j1], d2 = xi - x[j2], d3 = xi - x[j3];
        acc += w0 * d0; acc += w1 * d1; acc += w2 * d2; acc += w3 * d3;
        if (QF) { aq += w0 * d0 * d0; aq += w1 * d1 * d1; aq += w2 * d2 * d2; aq += w3 * d3 * d3; }
    }
    for (; e < e1; e += stride) {
        const T d = xi - x[col[e]];
        const T w = WEIGHTED ? wt[e] : T(1);
        acc += w * d;
        if (QF) aq += w * d * d;
    }
}

template <typename T, bool WEIGHTED, bool QF, class Pre, class F>
__device__ __forceinline__ void for_each_row_pre(const Graph &g, const Weights<T> &w,
                                                 const T *__restrict__ x, Pre &&pre, F &&f) {
    const int lane = lane_id();
    // huge rows: the whole workgroup strides over the row
    for (int r = blockIdx.x; r < g.n_huge; r += gridDim.x) {
        const auto pd = pre(r);
        const T xi = x[r];
        T acc = T(0), aq = T(0);
        edge_terms<T, WEIGHTED, QF>(g.col, w.csr, x, xi, g.rowptr[r] + threadIdx.x, g.rowptr[r + 1], blockDim.x,
                                    acc, aq);
        acc = block_sum(acc);
        if (QF) aq = block_sum(aq);
        if (threadIdx.x == 0) f(r, xi, acc, aq, pd);
    }
    const int nlong = g.n_long - g.n_huge;
    const int nmid = g.nslices_mid * (kWave / 8);  // eight rows per unit
    const int units = nlong + nmid + (g.nslices - g.nslices_mid);
    for (int u = blockIdx.x * kWavesPerBlock + wave_id(); u < units; u += gridDim.x * kWavesPerBlock) {
        if (u >= nlong && u < nlong + nmid) {
            // eight lanes per row; the eight partial sums meet in the row's first lane
            const int r = g.n_long + (u - nlong) * 8 + (lane >> 3);
            const bool live = r < g.n;
            const int rr = live ? r : g.n - 1;
            const auto pd = pre(rr);
            const T xi = x[rr];
            T acc = T(0), aq = T(0);
            if (live)
                edge_terms<T, WEIGHTED, QF>(g.col, w.csr, x, xi, g.rowptr[r] + (lane & 7), g.rowptr[r + 1], 8, acc,
                                            aq);
#pragma unroll
            for (int o = 1; o < 8; o <<= 1) {
                acc += __shfl_xor(acc, o, kWave);
                if (QF) aq += __shfl_xor(aq, o, kWave);
            }
            if (live && (lane & 7) == 0) f(r, xi, acc, aq, pd);
        } else if (u < nlong) {
            const int r = g.n_huge + u;
            const auto pd = pre(r);
            const T xi = x[r];
            T acc = T(0), aq = T(0);
            edge_terms<T, WEIGHTED, QF>(g.col, w.csr, x, xi, g.rowptr[r] + lane, g.rowptr[r + 1], kWave, acc, aq);
            acc = wave_sum(acc);
            if (QF) aq = wave_sum(aq);
            if (lane == 0) f(r, xi, acc, aq, pd);
        } else {
            const int s = u - nlong - nmid + g.nslices_mid;
            const int r = g.n_long + s * kWave + lane;
            if (r < g.n) {
                // operands of f are requested before the gathers start
                const auto pd = pre(r);
                const int off = g.sell_off[s];
                const int end = g.sell_off[s + 1];
                const T xi = x[r];
                T acc = T(0), aq = T(0);
                edge_terms<T, WEIGHTED, QF>(g.sell_col, w.sell, x, xi, off + lane, end, kWave, acc, aq);
                f(r, xi, acc, aq, pd);
            }
        }
    }
}

template <typename T, bool WEIGHTED, bool QF, class F>
__device__ __forceinline__ void for_each_row(const Graph &g, const Weights<T> &w, const T *__restrict__ x, F &&f) {
    for_each_row_pre<T, WEIGHTED, QF>(
        g, w, x, [](int) { return 0; }, [&](int i, T xi, T yi, T qi, int) { f(i, xi, yi, qi); });
}

// Grid size for a row-engine launch: enough wavefronts to cover the units,
// capped so that one pass of partial sums stays small.
inline int row_grid(const Graph &g, int cap) {
    const int units = (g.n_long - g.n_huge) + g.nslices_mid * (kWave / 8) + (g.nslices - g.nslices_mid);
    int blocks = (units + kWavesPerBlock - 1) / kWavesPerBlock;
    blocks = blocks > g.n_huge ? blocks : g.n_huge;
    if (blocks < 1) blocks = 1;
    return blocks < cap ? blocks : cap;
}

}  // namespace lapeig
