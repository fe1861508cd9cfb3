// Batched Jacobi-Davidson: many independent graphs in one persistent launch.
//
// One 1024-thread workgroup runs the whole of Algorithm 2 for one graph
// (orthogonalization, the MVP, the H border, eig(H), Ritz pair,
// certificate, deflation, restart and the projected PCG), with every
// reduction inside the workgroup (wavefront shuffles + LDS), so workgroups
// never wait on each other.  Workgroups take graph indices from an atomic
// counter over a list sorted by decreasing nnz (largest job first); every
// loop is bounded (k_max outer iterations, ITMAX PCG steps), so every
// workgroup reaches the end of the queue and exits.
//
// Precision as in the single-graph solver: FP32 products and PCG in mixed
// mode, FP64 for W = GV, orthogonalization, H, Ritz pairs and certificates.
// Graphs are connected (checked on the host), so the zero pair is e/sqrt(n).
// The launch takes all the LDS a workgroup may have; the PCG direction, the
// vector every inner product gathers from, lives there as far as it fits.
#include "lapeig_dev.h"
#include "batch_kernels.h"

namespace lapeig {

namespace {

constexpr int kBT = 1024;            // threads per workgroup
constexpr int kBW = kBT / kWave;     // wavefronts per workgroup
constexpr int kBM = kBatchMaxM;      // largest basis (m_max)
constexpr int kBK = kBatchMaxK;      // largest k
constexpr int NVB = kBK + kBM + 2;   // widest workgroup reduction

struct Shared {
    double red[kBW][NVB];
    double out[NVB];
    double H[kBM * kBM];
    double A[kBM * kBM];
    double Z[kBM * kBM];
    double Y[kBM * kBM];
    double theta[kBM];
    double coef[kBM + kBK + 2];
    double cs[kBM / 2], sn[kBM / 2];
    int pp[kBM / 2], qq[kBM / 2];
    double lam[kBK], rlock[kBK];  // locked pairs: Ritz value, certified residual
    int order[kBK];               // locked pairs by ascending value
    int any_rot;
    int job;
};

// sum of nv <= NVB values over the workgroup; result in sh.out
template <typename T, int NV>
__device__ void wg_sum(const T (&acc)[NV], int nv, Shared &sh) {
#pragma unroll
    for (int j = 0; j < NV; ++j)
        if (j < nv) {
            const double s = (double)wave_sum(acc[j]);
            if (lane_id() == 0) sh.red[wave_id()][j] = s;
        }
    __syncthreads();
    if (threadIdx.x < nv) {
        double s = 0.0;
        for (int w = 0; w < kBW; ++w) s += sh.red[w][threadIdx.x];
        sh.out[threadIdx.x] = s;
    }
    __syncthreads();
}

// wg_sum of nv values and one more FP64 value, in one pair of barriers:
// sh.out[0..nv) as wg_sum gives them, sh.out[nv] the sum of `extra`
template <typename T, int NV>
__device__ void wg_sum_x(const T (&acc)[NV], int nv, double extra, Shared &sh) {
#pragma unroll
    for (int j = 0; j < NV; ++j)
        if (j < nv) {
            const double s = (double)wave_sum(acc[j]);
            if (lane_id() == 0) sh.red[wave_id()][j] = s;
        }
    {
        const double e = wave_sum(extra);
        if (lane_id() == 0) sh.red[wave_id()][nv] = e;
    }
    __syncthreads();
    if ((int)threadIdx.x <= nv) {
        double s = 0.0;
        for (int w = 0; w < kBW; ++w) s += sh.red[w][threadIdx.x];
        sh.out[threadIdx.x] = s;
    }
    __syncthreads();
}

// pk[0..q) = proj, pk[q] = scalar (static register indexing only)
template <typename T, int NV>
__device__ __forceinline__ void pack_q(const T (&proj)[kBK], int q, T scalar, T (&pk)[NV]) {
#pragma unroll
    for (int j = 0; j < NV; ++j) pk[j] = j < kBK && j < q ? proj[j < kBK ? j : 0] : (j == q ? scalar : T(0));
}

struct GView {
    int n, nlong;
    const int *rp, *ci;
    const float *w32;
    const double *w64;
};

// The PCG direction: entries [0, cap) in the workgroup's LDS, the rest in the
// graph's workspace.  Vertices come in decreasing degree, so the LDS part
// takes the entries that the products gather most often.
template <typename T>
struct SplitVec {
    T *lds, *mem;
    int cap;
    __device__ __forceinline__ T &operator[](int i) const { return i < cap ? lds[i] : mem[i]; }
};

// Visits this thread's rows i = tid, tid + kBT, ... in that order: ld(i)
// loads a row's operands, op(i, loaded) uses them.  With 4-byte T two rows
// go at a time (both loads in flight together); FP64 operands take one row
// per step, since two would not fit the 128-register budget.
template <typename T, class Ld, class Op>
__device__ __forceinline__ void row_pass(int n, Ld &&ld, Op &&op) {
    if constexpr (sizeof(T) == 4) {
        for (int i = threadIdx.x; i < n; i += 2 * kBT) {
            const int i2 = i + kBT;
            const bool two = i2 < n;
            const auto a = ld(i);
            const auto b = ld(two ? i2 : i);
            op(i, a);
            if (two) op(i2, b);
        }
    } else {
        for (int i = threadIdx.x; i < n; i += kBT) op(i, ld(i));
    }
}

// a row of the projector Q (the product's operands of a row)
template <typename T>
struct QRow {
    T q[kBK];
};

// operands of one row of a PCG pass
template <typename T>
struct RowQ {
    T q[kBK];
    T a, b, c, d;
    int e0, e1;
};

// row operands a wg_rows caller loads nothing for
struct NoRow {};
struct NoPre {
    __device__ __forceinline__ NoRow operator()(int) const { return NoRow{}; }
};

// y_i = sum_j w_ij (x_i - x_j) for the rows of one graph: rows [0, nlong)
// one wavefront each, the rest one thread each.  pre(i) loads the caller's
// operands of row i, f(i, x_i, y_i, q_i, pre(i)) uses them.
// x: a pointer, or any vector with operator[] (the split PCG direction)
template <typename T, bool WT, bool QF, class X, class Pre, class F>
__device__ void wg_rows(const GView &g, const X &x, Pre &&pre, F &&f) {
    const int lane = lane_id();
    for (int r = wave_id(); r < g.nlong; r += kBW) {
        const auto op = pre(r);  // loaded before the edges (every lane, one address)
        const T xi = x[r];
        T acc = T(0), aq = T(0);
        for (int e = g.rp[r] + lane; e < g.rp[r + 1]; e += kWave) {
            const T d = xi - x[g.ci[e]];
            T wt = T(1);
            if (WT) wt = sizeof(T) == 4 ? (T)g.w32[e] : (T)g.w64[e];
            acc += wt * d;
            if (QF) aq += wt * d * d;
        }
        acc = wave_sum(acc);
        if (QF) aq = wave_sum(aq);
        if (lane == 0) f(r, xi, acc, aq, op);
    }
    // one row per thread: the next row's offsets and this row's operands are
    // loaded before its edges, and the edges go four at a time (indices,
    // then gathers), so a row costs about one memory round trip per four
    // edges; the sum is still taken in edge order
    auto wt_of = [&](int e) -> T { return WT ? (sizeof(T) == 4 ? (T)g.w32[e] : (T)g.w64[e]) : T(1); };
    int r = g.nlong + threadIdx.x;
    int e0 = r < g.n ? g.rp[r] : 0, e1 = r < g.n ? g.rp[r + 1] : 0;
    for (; r < g.n; r += kBT) {
        const int rn = r + kBT;
        const int n0 = rn < g.n ? g.rp[rn] : 0, n1 = rn < g.n ? g.rp[rn + 1] : 0;
        const auto op = pre(r);
        const T xi = x[r];
        T acc = T(0), aq = T(0);
        int e = e0;
        for (; e + 3 < e1; e += 4) {
            const int j0 = g.ci[e], j1 = g.ci[e + 1], j2 = g.ci[e + 2], j3 = g.ci[e + 3];
            const T w0 = wt_of(e), w1 = wt_of(e + 1), w2 = wt_of(e + 2), w3 = wt_of(e + 3);
            const T d0 = xi - x[j0], d1 = xi - x[j1], d2 = xi - x[j2], d3 = xi - x[j3];
            acc += w0 * d0;
            if (QF) aq += w0 * d0 * d0;
            acc += w1 * d1;
            if (QF) aq += w1 * d1 * d1;
            acc += w2 * d2;
            if (QF) aq += w2 * d2 * d2;
            acc += w3 * d3;
            if (QF) aq += w3 * d3 * d3;
        }
        for (; e < e1; ++e) {
            const T d = xi - x[g.ci[e]];
            const T wt = wt_of(e);
            acc += wt * d;
            if (QF) aq += wt * d * d;
        }
        f(r, xi, acc, aq, op);
        e0 = n0;
        e1 = n1;
    }
}

// all eigenpairs of the m x m matrix sh.H (column-major, ld kBM): cyclic
// Jacobi in tournament order (as the single-graph eigensolver), results in
// sh.theta (ascending) and sh.Y (column-major, ld kBM)
__device__ void wg_eig(int m, Shared &sh) {
    const int me = (m + 1) & ~1;
    const int tid = threadIdx.x;
    for (int t = tid; t < me * me; t += kBT) {
        const int i = t / me, j = t % me;
        sh.A[t] = (i < m && j < m) ? sh.H[j * kBM + i] : 0.0;
        sh.Z[t] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    double fro = 0.0;
    for (int t = 0; t < me * me; ++t) fro += sh.A[t] * sh.A[t];
    const double tol = 2.220446049250313e-16 * sqrt(fro) / (double)me;
    const int half = me / 2;
    for (int sweep = 0; sweep < 60 && me > 1; ++sweep) {
        if (tid == 0) sh.any_rot = 0;
        __syncthreads();
        for (int round = 0; round < me - 1; ++round) {
            if (tid < half) {
                auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + round) % (me - 1); };
                const int a = player(tid), b = player(me - 1 - tid);
                const int p = a < b ? a : b, q = a < b ? b : a;
                double c = 1.0, s = 0.0;
                const double apq = sh.A[p * me + q];
                if (fabs(apq) > tol) {
                    const double tau = (sh.A[q * me + q] - sh.A[p * me + p]) / (2.0 * apq);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                    sh.any_rot = 1;
                }
                sh.pp[tid] = p; sh.qq[tid] = q; sh.cs[tid] = c; sh.sn[tid] = s;
            }
            __syncthreads();
            for (int t = tid; t < half * me; t += kBT) {
                const int k = t / me, j = t % me;
                const int p = sh.pp[k], q = sh.qq[k];
                const double c = sh.cs[k], s = sh.sn[k];
                if (s != 0.0) {
                    const double ap = sh.A[p * me + j], aq = sh.A[q * me + j];
                    sh.A[p * me + j] = c * ap - s * aq;
                    sh.A[q * me + j] = s * ap + c * aq;
                }
            }
            __syncthreads();
            for (int t = tid; t < half * me; t += kBT) {
                const int k = t / me, i = t % me;
                const int p = sh.pp[k], q = sh.qq[k];
                const double c = sh.cs[k], s = sh.sn[k];
                if (s != 0.0) {
                    const double ap = sh.A[i * me + p], aq = sh.A[i * me + q];
                    sh.A[i * me + p] = c * ap - s * aq;
                    sh.A[i * me + q] = s * ap + c * aq;
                    const double zp = sh.Z[i * me + p], zq = sh.Z[i * me + q];
                    sh.Z[i * me + p] = c * zp - s * zq;
                    sh.Z[i * me + q] = s * zp + c * zq;
                }
            }
            __syncthreads();
            if (tid < half && sh.sn[tid] != 0.0) {
                sh.A[sh.pp[tid] * me + sh.qq[tid]] = 0.0;
                sh.A[sh.qq[tid] * me + sh.pp[tid]] = 0.0;
            }
            __syncthreads();
        }
        const int rotated = sh.any_rot;
        __syncthreads();
        if (!rotated) break;
    }
    for (int i = tid; i < m; i += kBT) {
        const double di = sh.A[i * me + i];
        int rank = 0;
        for (int j = 0; j < m; ++j) {
            const double dj = sh.A[j * me + j];
            rank += (dj < di) || (dj == di && j < i);
        }
        sh.theta[rank] = di;
        for (int r = 0; r < m; ++r) sh.Y[rank * kBM + r] = sh.Z[r * me + i];
    }
    __syncthreads();
}

// B(:, c) = sum_j B(:, j) Yc(j, c) for c < nc (B n x m column-major, ld n;
// Yc columns kBM apart): each thread rotates its rows in place, holding one
// row of B in registers, the columns summed in index order.
__device__ __forceinline__ void rotate_rows(int n, int m, double *B, const double *Yc, int nc) {
    for (int i = threadIdx.x; i < n; i += kBT) {
        double br[kBM];
#pragma unroll
        for (int j = 0; j < kBM; ++j)
            if (j < m) br[j] = B[(size_t)j * n + i];
        for (int c = 0; c < nc; ++c) {
            double sv = 0.0;
#pragma unroll
            for (int j = 0; j < kBM; ++j)
                if (j < m) sv += br[j] * Yc[c * kBM + j];
            B[(size_t)c * n + i] = sv;
        }
    }
}

__device__ __forceinline__ double splitmix_b(unsigned long long seed, unsigned long long idx) {
    unsigned long long z = seed + (idx + 1ULL) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

template <typename T, bool WT>
__device__ void solve_graph(const BatchArgs &a, int gid, Shared &sh, T *lds) {
    const BGraph G = a.graphs[gid];
    const int n = G.n, k = G.k, tid = threadIdx.x;
    const int mmax = a.m_max, mmin = a.m_min;
    GView gv{n, G.nlong, a.rowptr + G.rp, a.col + G.ci, a.w32 ? a.w32 + G.ci : nullptr,
             a.w64 ? a.w64 + G.ci : nullptr};
    // workspace slabs (column-major n-vectors)
    double *ws = a.ws64 + G.w64;
    double *X = ws;                       // n x k
    double *V = X + (size_t)n * k;        // n x mmax
    double *W = V + (size_t)n * mmax;     // n x mmax
    double *v = W + (size_t)n * mmax;
    double *u = v + n, *r = u + n, *gu = r + n;
    T *wt = reinterpret_cast<T *>(a.ws32) + G.w32;
    T *Q = wt;                            // n x k row-major
    T *t = Q + (size_t)n * k;
    T *res = t + n, *p = res + n, *s = p + n, *y = s + n;
    // the PCG direction, which every product gathers from, in LDS as far as it fits
    const SplitVec<T> pv{lds, p, n < a.lds_elems ? n : a.lds_elems};
    double *lam = sh.lam, *rlock = sh.rlock;
    // zero pair: e / sqrt(n) (connected graph)
    const double e0 = 1.0 / sqrt((double)n);
    for (int i = tid; i < n; i += kBT) {
        X[i] = e0;
        Q[(size_t)i * k] = (T)e0;
        v[i] = splitmix_b(a.seed, ((unsigned long long)gid << 32) + (unsigned long long)i);
    }
    if (tid == 0) {
        lam[0] = 0.0;
        rlock[0] = 0.0;
    }
    int nx = 1, m = 0, it = 0;
    long long mvp = 0, inner = 0;
    bool from_t = false;
    long long restart_col = 1;
    __syncthreads();
    while (nx < k && it < a.kmax) {
        ++it;
        // step 2: classical Gram-Schmidt twice against [X V] (nb columns)
        const int nb = nx + m;
        auto basis = [&](int j, int i) -> double {
            return j < nx ? X[(size_t)j * n + i] : V[(size_t)(j - nx) * n + i];
        };
        double vn2 = 0.0;
        for (int pass = 0; pass < 3; ++pass) {
            double acc[NVB];
#pragma unroll
            for (int j = 0; j < NVB; ++j) acc[j] = 0.0;
            for (int i = tid; i < n; i += kBT) {
                double vi = (pass == 0 && from_t) ? (double)t[i] : v[i];
                if (pass > 0) {
                    // four columns per step (their loads in flight together), in column order
                    double sub = 0.0;
                    int j = 0;
                    for (; j + 3 < nb; j += 4) {
                        const double b0 = basis(j, i), b1 = basis(j + 1, i), b2 = basis(j + 2, i),
                                     b3 = basis(j + 3, i);
                        sub += b0 * sh.coef[j];
                        sub += b1 * sh.coef[j + 1];
                        sub += b2 * sh.coef[j + 2];
                        sub += b3 * sh.coef[j + 3];
                    }
                    for (; j < nb; ++j) sub += basis(j, i) * sh.coef[j];
                    vi -= sub;
                }
                v[i] = vi;
                if (pass < 2) {
                    // four columns per step, loaded at clamped (valid) indices so the
                    // loads are unconditional and in flight together
#pragma unroll
                    for (int j0 = 0; j0 < NVB - 1; j0 += 4) {
                        if (j0 < nb) {
                            double b[4];
#pragma unroll
                            for (int c = 0; c < 4; ++c) b[c] = basis(min(j0 + c, nb - 1), i);
#pragma unroll
                            for (int c = 0; c < 4; ++c)
                                if (j0 + c < NVB - 1 && j0 + c < nb) acc[j0 + c] += b[c] * vi;
                        }
                    }
                } else {
                    acc[0] += vi * vi;
                }
            }
            __syncthreads();
            wg_sum<double, NVB>(acc, pass < 2 ? nb : 1, sh);
            if (pass < 2) {
                for (int j = tid; j < nb; j += kBT) sh.coef[j] = sh.out[j];
            } else {
                vn2 = sh.out[0];
            }
            __syncthreads();
        }
        double vn = sqrt(vn2);
        // step 3: V(:, m) = v / ||v||, W(:, m) = G V(:, m)
        {
            double *vc = V + (size_t)m * n, *wc = W + (size_t)m * n;
            const double sc = 1.0 / vn;
            for (int i = tid; i < n; i += kBT) vc[i] = v[i] * sc;
            __syncthreads();
            wg_rows<double, WT, false>(gv, vc, NoPre{}, [&](int i, double, double yi, double, NoRow) { wc[i] = yi; });
            ++mvp;
            __syncthreads();
            // step 4: H border
            double acc[NVB];
#pragma unroll
            for (int j = 0; j < NVB; ++j) acc[j] = 0.0;
            for (int i = tid; i < n; i += kBT) {
                const double wi = wc[i];
#pragma unroll
                for (int j0 = 0; j0 < kBM; j0 += 4) {
                    if (j0 <= m) {
                        double b[4];
#pragma unroll
                        for (int c = 0; c < 4; ++c) b[c] = V[(size_t)min(j0 + c, m) * n + i];
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            if (j0 + c <= m) acc[j0 + c] += b[c] * wi;
                    }
                }
            }
            wg_sum<double, NVB>(acc, m + 1, sh);
            for (int j = tid; j <= m; j += kBT) {
                sh.H[m * kBM + j] = sh.out[j];
                sh.H[j * kBM + m] = sh.out[j];
            }
            __syncthreads();
            ++m;
        }
        bool need_pcg = true;
        for (;;) {
            wg_eig(m, sh);
            // step 6: u = V y, Gu = W y, r = Gu - theta u
            const double th = sh.theta[0];
            double acc[2] = {0.0, 0.0};
            for (int i = tid; i < n; i += kBT) {
                double ui = 0.0, gi = 0.0;
                int j = 0;
                for (; j + 1 < m; j += 2) {
                    const double v0 = V[(size_t)j * n + i], v1 = V[(size_t)(j + 1) * n + i];
                    const double w0 = W[(size_t)j * n + i], w1 = W[(size_t)(j + 1) * n + i];
                    ui += v0 * sh.Y[j];
                    gi += w0 * sh.Y[j];
                    ui += v1 * sh.Y[j + 1];
                    gi += w1 * sh.Y[j + 1];
                }
                for (; j < m; ++j) {
                    ui += V[(size_t)j * n + i] * sh.Y[j];
                    gi += W[(size_t)j * n + i] * sh.Y[j];
                }
                u[i] = ui;
                r[i] = gi - th * ui;
                Q[(size_t)i * k + nx] = (T)ui;
                acc[0] += r[i] * r[i];
                acc[1] += ui * ui;
            }
            wg_sum<double, 2>(acc, 2, sh);
            const double rn = sqrt(sh.out[0] / sh.out[1]);
            __syncthreads();
            if (!(rn <= a.tol * fmin(th, 1.0))) break;
            // certificate: fresh G u, theta from eq. (1)
            double c2[2] = {0.0, 0.0};
            wg_rows<double, WT, true>(gv, u, NoPre{}, [&](int i, double xi, double yi, double qi, NoRow) {
                gu[i] = yi;
                c2[0] += qi;
                c2[1] += xi * xi;
            });
            ++mvp;
            wg_sum<double, 2>(c2, 2, sh);
            const double ct = 0.5 * sh.out[0] / sh.out[1], un2 = sh.out[1];
            __syncthreads();
            double c3[1] = {0.0};
            for (int i = tid; i < n; i += kBT) {
                const double d = gu[i] - ct * u[i];
                c3[0] += d * d;
            }
            wg_sum<double, 1>(c3, 1, sh);
            const double cr = sqrt(sh.out[0] / un2);
            __syncthreads();
            if (!(cr <= a.tol * fmin(ct, 1.0))) break;
            // lock: X(:, nx) = u / ||u||; V <- V Y(:, 2..m), W <- W Y(:, 2..m)
            const double us = 1.0 / sqrt(un2);
            for (int i = tid; i < n; i += kBT) X[(size_t)nx * n + i] = u[i] * us;
            rotate_rows(n, m, V, sh.Y + kBM, m - 1);
            rotate_rows(n, m, W, sh.Y + kBM, m - 1);
            if (tid < kBM * kBM) {
                const int i = tid / kBM, j = tid % kBM;
                sh.H[tid] = (i == j && i < m - 1) ? sh.theta[i + 1] : 0.0;
            }
            if (tid == 0) {
                lam[nx] = ct;
                rlock[nx] = cr;
            }
            ++nx;
            --m;
            __syncthreads();
            if (nx >= k) { need_pcg = false; break; }
            if (m == 0) {
                for (int i = tid; i < n; i += kBT)
                    v[i] = splitmix_b(a.seed + 7ULL, (unsigned long long)restart_col * (unsigned long long)n + i);
                ++restart_col;
                from_t = false;
                need_pcg = false;
                __syncthreads();
                break;
            }
        }
        if (!need_pcg) continue;
        // restart: keep the m_min Ritz vectors of smallest Ritz value
        if (m >= mmax) {
            rotate_rows(n, m, V, sh.Y, mmin);
            rotate_rows(n, m, W, sh.Y, mmin);
            if (tid < kBM * kBM) {
                const int i = tid / kBM, j = tid % kBM;
                sh.H[tid] = (i == j && i < mmin) ? sh.theta[i] : 0.0;
            }
            m = mmin;
            __syncthreads();
        }
        // step 8: PCG on the projected correction equation, Q = [X u]
        {
            const int q = nx + 1;
            const T th = (T)sh.theta[0];
            // res = -(I - QQ')r;  t = 0
            T a0[kBK], nr = T(0);
#pragma unroll
            for (int j = 0; j < kBK; ++j) a0[j] = T(0);
            for (int i = tid; i < n; i += kBT) {
                const T ri = (T)r[i];
                t[i] = T(0);
                res[i] = -ri;
                nr += ri * ri;
#pragma unroll
                for (int j = 0; j < kBK; ++j)
                    if (j < q) a0[j] -= Q[(size_t)i * k + j] * ri;
            }
            {
                T pk[kBK + 2];
                pack_q<T, kBK + 2>(a0, q, nr, pk);
                wg_sum<T, kBK + 2>(pk, q + 1, sh);
            }
            T c0[kBK];
#pragma unroll
            for (int j = 0; j < kBK; ++j) c0[j] = j < q ? (T)sh.out[j] : T(0);
            const T r0 = (T)sqrt(sh.out[q]);
            __syncthreads();
            auto precond = [&](const T (&cq)[kBK], T &rho_out) {
                // res -= Q cq (first call only, cq = c0); y = D^-1 res; c1 = Q'y; rho = res'y
                T acc[kBK], rr = T(0);
#pragma unroll
                for (int j = 0; j < kBK; ++j) acc[j] = T(0);
                row_pass<T>(
                    n,
                    [&](int i) {
                        RowQ<T> o;
#pragma unroll
                        for (int j = 0; j < kBK; ++j) o.q[j] = j < q ? Q[(size_t)i * k + j] : T(0);
                        o.a = res[i];
                        o.e0 = gv.rp[i];
                        o.e1 = gv.rp[i + 1];
                        return o;
                    },
                    [&](int i, const RowQ<T> &o) {
                        T ri = o.a;
                        T proj = T(0);
#pragma unroll
                        for (int j = 0; j < kBK; ++j)
                            if (j < q) proj += o.q[j] * cq[j];
                        ri -= proj;
                        res[i] = ri;
                        const int e0 = o.e0, e1 = o.e1;
                        T dsum = T(0);
                        if (WT) {
                            for (int e = e0; e < e1; ++e) dsum += sizeof(T) == 4 ? (T)gv.w32[e] : (T)gv.w64[e];
                        } else {
                            dsum = (T)(e1 - e0);
                        }
                        const T yi = dsum > T(0) ? ri / dsum : ri;
                        y[i] = yi;
                        rr += ri * yi;
#pragma unroll
                        for (int j = 0; j < kBK; ++j)
                            if (j < q) acc[j] += o.q[j] * yi;
                    });
                T pk[kBK + 2];
                pack_q<T, kBK + 2>(acc, q, rr, pk);
                wg_sum<T, kBK + 2>(pk, q + 1, sh);
                rho_out = (T)sh.out[q];
            };
            T rho = T(0);
            precond(c0, rho);
            T c1[kBK];
#pragma unroll
            for (int j = 0; j < kBK; ++j) c1[j] = j < q ? (T)sh.out[j] : T(0);
            __syncthreads();
            // p = y - Q c1
            for (int i = tid; i < n; i += kBT) {
                T proj = T(0);
#pragma unroll
                for (int j = 0; j < kBK; ++j)
                    if (j < q) proj += Q[(size_t)i * k + j] * c1[j];
                pv[i] = y[i] - proj;
            }
            __syncthreads();
            int its = 0;
            bool stop = !(r0 > T(0));
            for (int pit = 1; pit <= a.itmax && !stop; ++pit) {
                // s = (G - theta I) p;  pAp, c2 = Q's
                T a1[kBK], pa = T(0);
#pragma unroll
                for (int j = 0; j < kBK; ++j) a1[j] = T(0);
                wg_rows<T, WT, false>(
                    gv, pv,
                    [&](int i) {
                        QRow<T> o;
#pragma unroll
                        for (int j = 0; j < kBK; ++j) o.q[j] = j < q ? Q[(size_t)i * k + j] : T(0);
                        return o;
                    },
                    [&](int i, T pi, T yi, T, const QRow<T> &o) {
                        const T si = yi - th * pi;
                        s[i] = si;
                        pa += pi * si;
#pragma unroll
                        for (int j = 0; j < kBK; ++j)
                            if (j < q) a1[j] += o.q[j] * si;
                    });
                {
                    T pk[kBK + 2];
                    pack_q<T, kBK + 2>(a1, q, pa, pk);
                    wg_sum<T, kBK + 2>(pk, q + 1, sh);
                }
                const T pap = (T)sh.out[q];
                T c2[kBK];
#pragma unroll
                for (int j = 0; j < kBK; ++j) c2[j] = j < q ? (T)sh.out[j] : T(0);
                __syncthreads();
                ++mvp;
                if (!(pap > T(0))) {
                    if (pit == 1)
                        for (int i = tid; i < n; i += kBT) t[i] = pv[i];
                    its = pit;
                    __syncthreads();
                    break;
                }
                const T alpha = rho / pap;
                // one pass: t += alpha p; res -= alpha (s - Q c2); y = D^-1 res;
                // partial sums of Q'y and res'y (PCG precision) and ||res||^2
                // (FP64), each thread adding its rows in the same order as the
                // separate update, preconditioner and norm passes did
                T acc[kBK], rr = T(0);
#pragma unroll
                for (int j = 0; j < kBK; ++j) acc[j] = T(0);
                double nrm = 0.0;
                row_pass<T>(
                    n,
                    [&](int i) {
                        RowQ<T> o;
#pragma unroll
                        for (int j = 0; j < kBK; ++j) o.q[j] = j < q ? Q[(size_t)i * k + j] : T(0);
                        o.a = pv[i];
                        o.b = s[i];
                        o.c = res[i];
                        o.d = t[i];
                        o.e0 = gv.rp[i];
                        o.e1 = gv.rp[i + 1];
                        return o;
                    },
                    [&](int i, const RowQ<T> &o) {
                        T proj = T(0);
#pragma unroll
                        for (int j = 0; j < kBK; ++j)
                            if (j < q) proj += o.q[j] * c2[j];
                        t[i] = o.d + alpha * o.a;
                        const T ri = o.c - alpha * (o.b - proj);
                        res[i] = ri;
                        T dsum = T(0);
                        if (WT) {
                            for (int e = o.e0; e < o.e1; ++e) dsum += sizeof(T) == 4 ? (T)gv.w32[e] : (T)gv.w64[e];
                        } else {
                            dsum = (T)(o.e1 - o.e0);
                        }
                        const T yi = dsum > T(0) ? ri / dsum : ri;
                        y[i] = yi;
                        rr += ri * yi;
#pragma unroll
                        for (int j = 0; j < kBK; ++j)
                            if (j < q) acc[j] += o.q[j] * yi;
                        nrm += (double)ri * (double)ri;
                    });
                {
                    T pk[kBK + 2];
                    pack_q<T, kBK + 2>(acc, q, rr, pk);
                    wg_sum_x<T, kBK + 2>(pk, q + 1, nrm, sh);
                }
                const T rho_new = (T)sh.out[q];
#pragma unroll
                for (int j = 0; j < kBK; ++j) c1[j] = j < q ? (T)sh.out[j] : T(0);
                const T rn2 = (T)sqrt(sh.out[q + 1]);
                __syncthreads();
                its = pit;
                if (rn2 <= (T)a.rtol_pcg * r0 || pit == a.itmax) break;
                const T beta = rho_new / rho;
                rho = rho_new;
                row_pass<T>(
                    n,
                    [&](int i) {
                        RowQ<T> o;
#pragma unroll
                        for (int j = 0; j < kBK; ++j) o.q[j] = j < q ? Q[(size_t)i * k + j] : T(0);
                        o.a = y[i];
                        o.b = pv[i];
                        return o;
                    },
                    [&](int i, const RowQ<T> &o) {
                        T proj = T(0);
#pragma unroll
                        for (int j = 0; j < kBK; ++j)
                            if (j < q) proj += o.q[j] * c1[j];
                        pv[i] = (o.a - proj) + beta * o.b;
                    });
                __syncthreads();
            }
            inner += its;
            from_t = true;
            __syncthreads();
        }
    }
    // results: sort the locked pairs (insertion sort, one thread, in LDS)
    int *order = sh.order;
    __syncthreads();
    if (tid == 0) {
        for (int j = 0; j < nx; ++j) order[j] = j;
        for (int j = 1; j < nx; ++j) {
            int x = order[j], i = j - 1;
            while (i >= 0 && lam[order[i]] > lam[x]) { order[i + 1] = order[i]; --i; }
            order[i + 1] = x;
        }
    }
    __syncthreads();
    double *ov = a.out_vec + G.out_vec;
    for (int j = 0; j < nx; ++j)
        for (int i = tid; i < n; i += kBT) ov[(size_t)j * n + i] = X[(size_t)order[j] * n + i];
    if (tid == 0) {
        for (int j = 0; j < nx; ++j) {
            a.out_val[G.out_val + j] = lam[order[j]];
            a.out_res[G.out_val + j] = rlock[order[j]];
        }
        BResult res_{};
        res_.nconv = nx;
        res_.outer = it;
        res_.inner = (int)inner;
        res_.mvp = mvp;
        res_.status = nx >= k ? 0 : 1;
        a.results[gid] = res_;
    }
    __syncthreads();
}

template <typename T, bool WT>
__global__ __launch_bounds__(kBT) void k_batch_jd(BatchArgs a) {
    __shared__ Shared sh;
    extern __shared__ __align__(16) unsigned char batch_lds[];
    for (;;) {
        if (threadIdx.x == 0)
            sh.job = (int)__hip_atomic_fetch_add(a.queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int job = sh.job;
        __syncthreads();
        if (job >= a.ngraphs) break;
        solve_graph<T, WT>(a, a.order[job], sh, reinterpret_cast<T *>(batch_lds));
    }
}

__global__ void k_batch_reset(unsigned *queue) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0u;
}

// Eigenvector blocks into the caller's vertex order (dst[i] = src[perm[i]])
// with the sign convention of the single-graph solver: the entry of largest
// magnitude is positive, the first such entry in caller order deciding;
// columns past a graph's nconv are zero.  One workgroup per graph.
__global__ __launch_bounds__(kBT) void k_batch_unpack(const BGraph *__restrict__ graphs,
                                                      const BResult *__restrict__ results,
                                                      const int *__restrict__ perm_all,
                                                      const long long *__restrict__ perm_off, int ngraphs,
                                                      const double *__restrict__ src, double *__restrict__ dst) {
    __shared__ double wbest[kBW];
    __shared__ int widx[kBW];
    __shared__ double sgn;
    const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
    for (int gi = blockIdx.x; gi < ngraphs; gi += gridDim.x) {
        const BGraph G = graphs[gi];
        const int n = G.n, k = G.k;
        const int nc = min(results[gi].nconv, k);
        const int *pm = perm_all + perm_off[gi];
        for (int j = 0; j < k; ++j) {
            const double *x = src + G.out_vec + (long long)j * n;
            double *y = dst + G.out_vec + (long long)j * n;
            if (j >= nc) {
                for (int i = tid; i < n; i += kBT) y[i] = 0.0;
                continue;
            }
            double best = -1.0;
            int bi = n;
            for (int i = tid; i < n; i += kBT) {
                const double v = fabs(x[pm[i]]);
                if (v > best) { best = v; bi = i; }  // i grows: the first maximum of this thread
            }
            for (int o = kWave / 2; o > 0; o >>= 1) {
                const double ob = __shfl_xor(best, o, kWave);
                const int oi = __shfl_xor(bi, o, kWave);
                if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
            }
            if (lane == 0) { wbest[wv] = best; widx[wv] = bi; }
            __syncthreads();
            if (tid == 0) {
                double b = wbest[0];
                int i0 = widx[0];
                for (int w = 1; w < kBW; ++w)
                    if (wbest[w] > b || (wbest[w] == b && widx[w] < i0)) { b = wbest[w]; i0 = widx[w]; }
                sgn = (i0 < n && x[pm[i0]] < 0.0) ? -1.0 : 1.0;
            }
            __syncthreads();
            const double sg = sgn;
            for (int i = tid; i < n; i += kBT) y[i] = sg * x[pm[i]];
            __syncthreads();
        }
    }
}

// The solver's product on every graph of the batch (y = G x, graph g's
// vectors at voff[g]), one workgroup per graph as in the solver, for timing
// the row-class threshold candidates.
template <typename T, bool WT>
__global__ __launch_bounds__(kBT) void k_batch_spmv(const BGraph *__restrict__ graphs, int ngraphs,
                                                    const long long *__restrict__ voff, const int *__restrict__ rowptr,
                                                    const int *__restrict__ col, const float *__restrict__ w32,
                                                    const double *__restrict__ w64, const T *__restrict__ x,
                                                    T *__restrict__ y) {
    for (int gi = blockIdx.x; gi < ngraphs; gi += gridDim.x) {
        const BGraph G = graphs[gi];
        const GView gv{G.n, G.nlong, rowptr + G.rp, col + G.ci, w32 ? w32 + G.ci : nullptr,
                       w64 ? w64 + G.ci : nullptr};
        const T *xg = x + voff[gi];
        T *yg = y + voff[gi];
        wg_rows<T, WT, false>(gv, xg, NoPre{}, [&](int i, T, T yi, T, NoRow) { yg[i] = yi; });
        __syncthreads();
    }
}

}  // namespace

namespace {

// Launches k on all of the LDS that one workgroup may have beyond the
// kernel's static arrays (the PCG direction of graphs that fit goes there).
template <typename T, bool WT>
void launch_jd(BatchArgs a, int grid, hipStream_t s) {
    auto *k = k_batch_jd<T, WT>;
    int dev = 0, max_lds = 0;
    hipFuncAttributes fa{};
    size_t dyn = 0;
    // a failed query leaves the global-memory path (and its error is cleared)
    bool ok = hipGetDevice(&dev) == hipSuccess &&
              hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
              hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(k)) == hipSuccess;
    if (ok && max_lds > (int)fa.sharedSizeBytes) dyn = ((size_t)max_lds - fa.sharedSizeBytes) & ~(size_t)15;
    if (dyn > 0 && hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)dyn) != hipSuccess) {
        ok = false;
        dyn = 0;
    }
    if (!ok) (void)hipGetLastError();
    a.lds_elems = (int)(dyn / sizeof(T));
    hipLaunchKernelGGL(k, dim3(grid), dim3(kBT), dyn, s, a);
}

}  // namespace

void batch_spmv_launch(const BGraph *graphs, int ngraphs, const long long *voff, const int *rowptr, const int *col,
                       const float *w32, const double *w64, bool mixed, const void *x, void *y, int grid,
                       hipStream_t s) {
    const bool wt = w32 != nullptr;
    if (mixed) {
        if (wt)
            hipLaunchKernelGGL((k_batch_spmv<float, true>), dim3(grid), dim3(kBT), 0, s, graphs, ngraphs, voff, rowptr,
                               col, w32, w64, (const float *)x, (float *)y);
        else
            hipLaunchKernelGGL((k_batch_spmv<float, false>), dim3(grid), dim3(kBT), 0, s, graphs, ngraphs, voff,
                               rowptr, col, w32, w64, (const float *)x, (float *)y);
    } else {
        if (wt)
            hipLaunchKernelGGL((k_batch_spmv<double, true>), dim3(grid), dim3(kBT), 0, s, graphs, ngraphs, voff,
                               rowptr, col, w32, w64, (const double *)x, (double *)y);
        else
            hipLaunchKernelGGL((k_batch_spmv<double, false>), dim3(grid), dim3(kBT), 0, s, graphs, ngraphs, voff,
                               rowptr, col, w32, w64, (const double *)x, (double *)y);
    }
    LAP_HIP(hipGetLastError());
}

void batch_unpack_launch(const BGraph *graphs, const BResult *results, const int *perm_all, const long long *perm_off,
                         int ngraphs, const double *src, double *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_unpack, dim3(std::min(ngraphs, 4 * device_cu_count())), dim3(kBT), 0, s, graphs,
                       results, perm_all, perm_off, ngraphs, src, dst);
    LAP_HIP(hipGetLastError());
}

void batch_launch(const BatchArgs &a, bool mixed, bool weighted, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, a.queue);
    if (mixed) {
        if (weighted) launch_jd<float, true>(a, grid, s);
        else launch_jd<float, false>(a, grid, s);
    } else {
        if (weighted) launch_jd<double, true>(a, grid, s);
        else launch_jd<double, false>(a, grid, s);
    }
    LAP_HIP(hipGetLastError());
}

}  // namespace lapeig
