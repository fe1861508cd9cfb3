// The warm-start network: forward, subspace loss, backward and Adam, all on
// the device.  An engineering addition (the paper starts JD from a single
// unit vector, Algorithm 2): its columns only seed the search space, and the
// FP64 certificate of lap_eigs decides the answer.
//
// Plan order, row-major FP32 blocks throughout.  The neighbour mean is
//   D^{-1} A h = h - D^{-1} (G h)      (A = D - G, rows with d = 0 give 0),
// one edge-difference block product, and its transpose A D^{-1} g =
// g - G (D^{-1} g) likewise; the dense parts run on the matrix cores through
// the tall-skinny products (k_ts_nn for [h | agg] W, k_ts_tn for the weight
// gradients and the Gram matrices).  The p x p algebra of the loss runs in
// FP64 in one workgroup.
#include <cmath>

#include "lapeig_dev.h"
#include "mpnn_internal.h"

namespace lapeig {

namespace {

__device__ __forceinline__ float splitmix_unit_f(unsigned long long seed, unsigned long long i) {
    unsigned long long z = seed + (i + 1ull) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z = z ^ (z >> 31);
    return (float)((double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0);
}

__device__ __forceinline__ bool has_edges(const Graph &g, int i) { return g.rowptr[i + 1] > g.rowptr[i]; }

// features of row i (plan order): 1, log(1 + d_i), (f2 later), random channels
__global__ void k_feat(Graph g, const float *__restrict__ wcsr, const int *__restrict__ iperm, int R,
                       unsigned long long seed, float *__restrict__ hc, int ld) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += gridDim.x * blockDim.x) {
        float d = 0.f;
        if (wcsr)
            for (int e = g.rowptr[i]; e < g.rowptr[i + 1]; ++e) d += wcsr[e];
        else
            d = (float)(g.rowptr[i + 1] - g.rowptr[i]);
        float *row = hc + (size_t)i * ld;
        row[0] = 1.f;
        row[1] = log1pf(d);
        row[2] = 0.f;
        const unsigned long long base = (unsigned long long)iperm[i] * (unsigned long long)R;
        for (int c = 0; c < R; ++c) row[3 + c] = 1.7320508075688772f * splitmix_unit_f(seed, base + c);
    }
}

// dst[i][j] = (d_i > 0) ? src[i][j] - dinv_i gs[i][j] : 0     (D^{-1} A h)
__global__ void k_agg(Graph g, const float *__restrict__ dinv, int F, const float *__restrict__ src, int lds,
                      const float *__restrict__ gs, int ldg, float *__restrict__ dst, int ldd) {
    const size_t tot = (size_t)g.n * F;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / F), j = (int)(t % F);
        dst[(size_t)i * ldd + j] =
            has_edges(g, i) ? src[(size_t)i * lds + j] - dinv[i] * gs[(size_t)i * ldg + j] : 0.f;
    }
}

// u[i][j] = (d_i > 0) ? dinv_i g[i][j] : 0
__global__ void k_aggt_pre(Graph g, const float *__restrict__ dinv, int F, const float *__restrict__ gsrc, int ldg,
                           float *__restrict__ u) {
    const size_t tot = (size_t)g.n * F;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / F), j = (int)(t % F);
        u[t] = has_edges(g, i) ? dinv[i] * gsrc[(size_t)i * ldg + j] : 0.f;
    }
}

// gh[i][j] = gself[i][j] + A D^{-1} gagg = gself + (d_i > 0 ? gagg : 0) - (G u)[i][j]
__global__ void k_aggt_post(Graph g, int F, const float *__restrict__ ghc, int ldh, const float *__restrict__ gu,
                            float *__restrict__ gh) {
    const size_t tot = (size_t)g.n * F;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / F), j = (int)(t % F);
        const float self = ghc[(size_t)i * ldh + j];
        const float agg = has_edges(g, i) ? ghc[(size_t)i * ldh + F + j] : 0.f;
        gh[t] = (self + agg) - gu[t];
    }
}

// z += b; out = relu(z) (hidden layers), or z += b (output)
__global__ void k_bias_act(int n, int F, float *__restrict__ z, int ldz, const float *__restrict__ b, int relu,
                           float *__restrict__ out, int ldo) {
    const size_t tot = (size_t)n * F;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / F), j = (int)(t % F);
        const float v = z[(size_t)i * ldz + j] + b[j];
        z[(size_t)i * ldz + j] = v;
        if (relu) out[(size_t)i * ldo + j] = v > 0.f ? v : 0.f;
    }
}

// g *= (z > 0)
__global__ void k_relu_bwd(size_t tot, const float *__restrict__ z, float *__restrict__ g) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x)
        if (!(z[t] > 0.f)) g[t] = 0.f;
}

// y[i][j] -= colsum[j] / n   (projection off the constant vector)
__global__ void k_center(int n, int F, float *__restrict__ y, int ld, const float *__restrict__ colsum) {
    const size_t tot = (size_t)n * F;
    const float inv_n = 1.f / (float)n;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / F), j = (int)(t % F);
        y[(size_t)i * ld + j] -= colsum[j] * inv_n;
    }
}

// W' (c x r column-major) of W (r x c column-major)
__global__ void k_transpose(int r, int c, const float *__restrict__ W, float *__restrict__ WT) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < r * c; t += gridDim.x * blockDim.x) {
        const int i = t % r, j = t / r;
        WT[j + (size_t)i * c] = W[t];
    }
}

// X (caller order, n x kx column-major, double) into columns off.. of yx (plan order)
__global__ void k_load_x(int n, int kx, const double *__restrict__ X, const int *__restrict__ perm,
                         float *__restrict__ yx, int ld, int off) {
    const size_t tot = (size_t)n * kx;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(t / n), i = (int)(t % n);
        yx[(size_t)perm[i] * ld + off + c] = (float)X[t];
    }
}

// V0 (caller order, n x p column-major, double) from yx (plan order)
__global__ void k_store_v(int n, int p, const float *__restrict__ yx, int ld, const int *__restrict__ perm,
                          double *__restrict__ V0) {
    const size_t tot = (size_t)n * p;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(t / n), i = (int)(t % n);
        V0[t] = (double)yx[(size_t)perm[i] * ld + c];
    }
}

__global__ void k_fill(size_t tot, float v, float *__restrict__ x) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x)
        x[t] = v;
}

// The p x p algebra of the loss, FP64, one workgroup:  SC = [S | C]
// (p x (p + kx) column-major, S = Yh'Yh, C = Yh'X).  S^{-1} by Gauss-Jordan
// with partial pivoting; M = C C'; loss = 1 - trace(S^{-1} M) / kx;
// coef ((p + kx) x p column-major) = (2 / kx) [S^{-1} M S^{-1} ; -C' S^{-1}],
// so that the gradient with respect to Yh is [Yh | X] coef.
__global__ __launch_bounds__(kBlock) void k_loss(int p, int kx, const float *__restrict__ SC,
                                                 float *__restrict__ coef, double *__restrict__ loss) {
    constexpr int M = kMpnnMaxCols;
    __shared__ double A[M][2 * M + 1];  // [S | I] -> [I | S^{-1}]
    __shared__ double C[M][M], T[M][M];
    __shared__ int piv;
    __shared__ int singular;
    const int tid = threadIdx.x;
    for (int t = tid; t < p * 2 * p; t += blockDim.x) {
        const int i = t / (2 * p), j = t % (2 * p);
        A[i][j] = j < p ? (double)SC[i + (size_t)j * p] : (j - p == i ? 1.0 : 0.0);
    }
    for (int t = tid; t < p * kx; t += blockDim.x) {
        const int i = t / kx, j = t % kx;
        C[i][j] = (double)SC[i + (size_t)(p + j) * p];
    }
    if (tid == 0) singular = 0;
    __syncthreads();
    for (int c = 0; c < p; ++c) {
        if (tid == 0) {
            int best = c;
            for (int r = c + 1; r < p; ++r)
                if (fabs(A[r][c]) > fabs(A[best][c])) best = r;
            piv = best;
            if (!(fabs(A[best][c]) > 0.0)) singular = 1;
        }
        __syncthreads();
        if (singular) break;
        if (piv != c)
            for (int j = tid; j < 2 * p; j += blockDim.x) {
                const double a = A[c][j];
                A[c][j] = A[piv][j];
                A[piv][j] = a;
            }
        __syncthreads();
        const double inv = 1.0 / A[c][c];
        __syncthreads();
        for (int j = tid; j < 2 * p; j += blockDim.x) A[c][j] *= inv;
        __syncthreads();
        for (int t = tid; t < p * 2 * p; t += blockDim.x) {
            const int r = t / (2 * p), j = t % (2 * p);
            if (r != c && j != c) A[r][j] -= A[r][c] * A[c][j];
        }
        __syncthreads();
        for (int r = tid; r < p; r += blockDim.x)
            if (r != c) A[r][c] = 0.0;
        __syncthreads();
    }
    if (singular) {
        if (tid == 0) *loss = NAN;
        return;
    }
    // T = S^{-1} M = S^{-1} C C'
    for (int t = tid; t < p * p; t += blockDim.x) {
        const int i = t / p, j = t % p;
        double s = 0.0;
        for (int a = 0; a < p; ++a) {
            double m = 0.0;
            for (int b = 0; b < kx; ++b) m += C[a][b] * C[j][b];
            s += A[i][p + a] * m;
        }
        T[i][j] = s;
    }
    __syncthreads();
    if (tid == 0) {
        double tr = 0.0;
        for (int i = 0; i < p; ++i) tr += T[i][i];
        *loss = 1.0 - tr / kx;
    }
    const double sc = 2.0 / kx;
    const int ldc = p + kx;
    for (int t = tid; t < p * p; t += blockDim.x) {  // rows < p: T S^{-1}
        const int i = t / p, j = t % p;
        double s = 0.0;
        for (int a = 0; a < p; ++a) s += T[i][a] * A[a][p + j];
        coef[i + (size_t)j * ldc] = (float)(sc * s);
    }
    for (int t = tid; t < kx * p; t += blockDim.x) {  // rows p..: -C' S^{-1}
        const int i = t / p, j = t % p;
        double s = 0.0;
        for (int a = 0; a < p; ++a) s += C[a][i] * A[a][p + j];
        coef[(p + i) + (size_t)j * ldc] = (float)(-sc * s);
    }
}

__global__ void k_adam(long long np, float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float omb1, float omb2, float eps,
                       float inv_bc1, float inv_bc2) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < np; t += (long long)gridDim.x * blockDim.x) {
        const float gt = g[t];
        const float mt = b1 * m[t] + omb1 * gt;
        const float vt = b2 * v[t] + omb2 * gt * gt;
        m[t] = mt;
        v[t] = vt;
        w[t] -= lr * (mt * inv_bc1) / (sqrtf(vt * inv_bc2) + eps);
    }
}

inline int egrid(size_t work) {
    size_t g = (work + kBlock - 1) / kBlock;
    const size_t cap = 4 * (size_t)device_cu_count();
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

int in_width(const lap_mpnn *m, int l) { return l == 0 ? 3 + m->cfg.random_channels : m->cfg.hidden; }

void ensure_work(lap_mpnn *m, int n) {
    if (m->n_alloc >= n) return;
    const int L = m->cfg.layers, H = m->cfg.hidden, p = m->cfg.out_cols;
    m->hc.clear();
    m->zp.clear();
    for (int l = 0; l <= L; ++l) m->hc.emplace_back((size_t)n * 2 * in_width(m, l));
    for (int l = 0; l < L; ++l) m->zp.emplace_back((size_t)n * H);
    const int wmax = std::max(2 * std::max(H, in_width(m, 0)), kMpnnMaxCols);
    m->yx.alloc((size_t)n * kMpnnMaxCols);
    m->gy.alloc((size_t)n * std::max(p, H));
    m->ghc.alloc((size_t)n * wmax);
    m->gh.alloc((size_t)n * std::max(H, 1));
    m->tmp.alloc((size_t)n * wmax);
    m->ones.alloc(n);
    hipLaunchKernelGGL(k_fill, dim3(egrid(n)), dim3(kBlock), 0, 0, (size_t)n, 1.f, m->ones.get());
    LAP_HIP(hipGetLastError());
    LAP_HIP(hipDeviceSynchronize());
    m->n_alloc = n;
}

// dst (ld 2F, columns F..2F) = D^{-1} A h,  h = columns 0..F of the same rows
void aggregate(lap_mpnn *m, const lap_plan &P, float *hc, int F, hipStream_t s) {
    spmm<float>(P, F, hc, 2 * F, m->tmp.get(), F, nullptr, s);
    hipLaunchKernelGGL(k_agg, dim3(egrid((size_t)P.n * F)), dim3(kBlock), 0, s, P.g, P.dinv<float>(), F, hc, 2 * F,
                       m->tmp.get(), F, hc + F, 2 * F);
}

// gh (n x F) = left half of ghc + A D^{-1} (right half)
void aggregate_t(lap_mpnn *m, const lap_plan &P, const float *ghc, int F, hipStream_t s) {
    float *u = m->gh.get();  // used as the scaled input, then overwritten
    hipLaunchKernelGGL(k_aggt_pre, dim3(egrid((size_t)P.n * F)), dim3(kBlock), 0, s, P.g, P.dinv<float>(), F,
                       ghc + F, 2 * F, u);
    spmm<float>(P, F, u, F, m->tmp.get(), F, nullptr, s);
    hipLaunchKernelGGL(k_aggt_post, dim3(egrid((size_t)P.n * F)), dim3(kBlock), 0, s, P.g, F, ghc, 2 * F,
                       m->tmp.get(), m->gh.get());
}

// column sums of x (n x F, ld) into out (F floats)
void colsum(lap_mpnn *m, int n, const float *x, int ld, int F, float *out, hipStream_t s) {
    ts_tn<float>(n, m->ones.get(), 1, 1, x, ld, F, out, 1, nullptr, 0, 1.f, m->bs, s);
}

}  // namespace

void mpnn_init(lap_mpnn *m, const lap_mpnn_config &cfg) {
    LAP_REQUIRE(cfg.layers >= 0 && cfg.layers <= 8, LAP_EINVAL, "layers must be in [0, 8]");
    LAP_REQUIRE(cfg.hidden >= 1 && cfg.hidden <= kMpnnMaxCols, LAP_EINVAL, "hidden must be in [1, 32]");
    LAP_REQUIRE(cfg.random_channels >= 0 && cfg.random_channels <= 16, LAP_EINVAL,
                "random_channels must be in [0, 16]");
    LAP_REQUIRE(cfg.out_cols >= 1 && cfg.out_cols < kMpnnMaxCols, LAP_EINVAL, "out_cols must be in [1, 31]");
    m->cfg = cfg;
    LAP_HIP(hipGetDevice(&m->device));
    const int L = cfg.layers;
    long long at = 0;
    for (int l = 0; l <= L; ++l) {
        const int r = 2 * in_width(m, l), c = l < L ? cfg.hidden : cfg.out_cols;
        m->wr.push_back(r);
        m->wc.push_back(c);
        m->woff.push_back(at);
        at += (long long)r * c;
        m->boff.push_back(at);
        at += c;
    }
    m->nparams = at;
    // Glorot-uniform weights from SplitMix64 (counter = flat index), zero biases
    std::vector<float> h((size_t)at, 0.f);
    for (int l = 0; l <= L; ++l) {
        const double a = std::sqrt(6.0 / (m->wr[l] + m->wc[l]));
        for (long long t = 0; t < (long long)m->wr[l] * m->wc[l]; ++t) {
            const unsigned long long i = (unsigned long long)(m->woff[l] + t);
            unsigned long long z = cfg.seed + (i + 1ull) * 0x9e3779b97f4a7c15ull;
            z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
            z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
            z = z ^ (z >> 31);
            const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
            h[(size_t)(m->woff[l] + t)] = (float)(a * u);
        }
    }
    m->params.alloc(at);
    m->grad.alloc(at);
    m->adam_m.alloc(at);
    m->adam_v.alloc(at);
    LAP_HIP(hipMemcpy(m->params.get(), h.data(), sizeof(float) * at, hipMemcpyHostToDevice));
    LAP_HIP(hipMemset(m->adam_m.get(), 0, sizeof(float) * at));
    LAP_HIP(hipMemset(m->adam_v.get(), 0, sizeof(float) * at));
    m->small.alloc(4096);
    m->loss.alloc(1);
    m->bs.ensure();
    ts_prepare<float>();
}

void mpnn_forward(lap_mpnn *m, const lap_plan &P, uint64_t seed, hipStream_t s) {
    const int n = P.n, L = m->cfg.layers, H = m->cfg.hidden, p = m->cfg.out_cols, R = m->cfg.random_channels;
    ensure_work(m, n);
    const int F0 = 3 + R;
    float *h0 = m->hc[0].get();
    hipLaunchKernelGGL(k_feat, dim3(egrid(n)), dim3(kBlock), 0, s, P.g, P.weighted ? P.weights<float>().csr : nullptr,
                       P.d_iperm.get(), R, (unsigned long long)seed, h0, 2 * F0);
    // f2 = mean neighbour log-degree: D^{-1} A applied to column 1
    spmm<float>(P, 1, h0 + 1, 2 * F0, m->tmp.get(), 1, nullptr, s);
    hipLaunchKernelGGL(k_agg, dim3(egrid(n)), dim3(kBlock), 0, s, P.g, P.dinv<float>(), 1, h0 + 1, 2 * F0, m->tmp.get(),
                       1, h0 + 2, 2 * F0);
    const int ldy = kMpnnMaxCols;
    for (int l = 0; l <= L; ++l) {
        const int F = in_width(m, l);
        float *hc = m->hc[l].get();
        aggregate(m, P, hc, F, s);
        const float *W = m->params.get() + m->woff[l];
        const float *b = m->params.get() + m->boff[l];
        if (l < L) {
            float *z = m->zp[l].get();
            ts_nn<float>(n, hc, 2 * F, 2 * F, W, 2 * F, H, z, H, nullptr, 0, 1.f, 0.f, s);
            hipLaunchKernelGGL(k_bias_act, dim3(egrid((size_t)n * H)), dim3(kBlock), 0, s, n, H, z, H, b, 1,
                               m->hc[l + 1].get(), 2 * H);
        } else {
            float *y = m->yx.get();
            ts_nn<float>(n, hc, 2 * F, 2 * F, W, 2 * F, p, y, ldy, nullptr, 0, 1.f, 0.f, s);
            hipLaunchKernelGGL(k_bias_act, dim3(egrid((size_t)n * p)), dim3(kBlock), 0, s, n, p, y, ldy, b, 0,
                               nullptr, 0);
        }
    }
    // project off the constant vector
    float *cs = m->small.get() + 3072;
    colsum(m, n, m->yx.get(), ldy, p, cs, s);
    hipLaunchKernelGGL(k_center, dim3(egrid((size_t)n * p)), dim3(kBlock), 0, s, n, p, m->yx.get(), ldy, cs);
    LAP_HIP(hipGetLastError());
}

double mpnn_loss_grad(lap_mpnn *m, const lap_plan &P, uint64_t seed, const double *X, int kx, hipStream_t s) {
    const int n = P.n, L = m->cfg.layers, H = m->cfg.hidden, p = m->cfg.out_cols;
    LAP_REQUIRE(kx >= 1 && p + kx <= kMpnnMaxCols, LAP_EINVAL, "need 1 <= kx and out_cols + kx <= 32");
    LAP_REQUIRE(P.ncomp == 1, LAP_EUNSUPPORTED, "training needs a connected graph");
    mpnn_forward(m, P, seed, s);
    const int ldy = kMpnnMaxCols;
    float *yx = m->yx.get();
    hipLaunchKernelGGL(k_load_x, dim3(egrid((size_t)n * kx)), dim3(kBlock), 0, s, n, kx, X, P.d_perm.get(), yx, ldy,
                       p);
    float *SC = m->small.get();          // p x (p + kx)
    float *coef = m->small.get() + 1024;  // (p + kx) x p
    float *cs = m->small.get() + 3072;
    float *WT = m->small.get();  // reused after the loss (transposed weights, up to 2 x 32 x 32)
    ts_tn<float>(n, yx, ldy, p, yx, ldy, p + kx, SC, p, nullptr, 0, 1.f, m->bs, s);
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(kBlock), 0, s, p, kx, SC, coef, m->loss.get());
    float *gy = m->gy.get();
    ts_nn<float>(n, yx, ldy, p + kx, coef, p + kx, p, gy, p, nullptr, 0, 1.f, 0.f, s);
    colsum(m, n, gy, p, p, cs, s);
    hipLaunchKernelGGL(k_center, dim3(egrid((size_t)n * p)), dim3(kBlock), 0, s, n, p, gy, p, cs);
    // output layer
    float *G = m->grad.get();
    {
        const int F = in_width(m, L);
        const float *hc = m->hc[L].get();
        ts_tn<float>(n, hc, 2 * F, 2 * F, gy, p, p, G + m->woff[L], 2 * F, nullptr, 0, 1.f, m->bs, s);
        colsum(m, n, gy, p, p, G + m->boff[L], s);
        if (L > 0) {
            hipLaunchKernelGGL(k_transpose, dim3(egrid(2 * F * p)), dim3(kBlock), 0, s, 2 * F, p,
                               m->params.get() + m->woff[L], WT);
            ts_nn<float>(n, gy, p, p, WT, p, 2 * F, m->ghc.get(), 2 * F, nullptr, 0, 1.f, 0.f, s);
            aggregate_t(m, P, m->ghc.get(), F, s);
        }
    }
    for (int l = L - 1; l >= 0; --l) {
        const int F = in_width(m, l);
        float *gz = m->gh.get();  // n x H, becomes dL/dZ
        hipLaunchKernelGGL(k_relu_bwd, dim3(egrid((size_t)n * H)), dim3(kBlock), 0, s, (size_t)n * H, m->zp[l].get(),
                           gz);
        const float *hc = m->hc[l].get();
        ts_tn<float>(n, hc, 2 * F, 2 * F, gz, H, H, G + m->woff[l], 2 * F, nullptr, 0, 1.f, m->bs, s);
        colsum(m, n, gz, H, H, G + m->boff[l], s);
        if (l > 0) {
            hipLaunchKernelGGL(k_transpose, dim3(egrid(2 * F * H)), dim3(kBlock), 0, s, 2 * F, H,
                               m->params.get() + m->woff[l], WT);
            ts_nn<float>(n, gz, H, H, WT, H, 2 * F, m->ghc.get(), 2 * F, nullptr, 0, 1.f, 0.f, s);
            aggregate_t(m, P, m->ghc.get(), F, s);
        }
    }
    LAP_HIP(hipGetLastError());
    double loss = 0.0;
    LAP_HIP(hipMemcpyAsync(&loss, m->loss.get(), sizeof(double), hipMemcpyDeviceToHost, s));
    LAP_HIP(hipStreamSynchronize(s));
    LAP_REQUIRE(std::isfinite(loss), LAP_EDEVICE, "the Gram matrix of the network's output is singular");
    return loss;
}

void mpnn_adam(lap_mpnn *m, float lr, hipStream_t s) {
    ++m->step;
    // Adam (Kingma & Ba, beta1 0.9, beta2 0.999, eps 1e-8).  The bias
    // corrections 1 - beta^t are formed in double: in single precision
    // 1 - 0.999^t loses about five digits to cancellation for small t.
    const double b1 = 0.9, b2 = 0.999;
    const double bc1 = 1.0 - std::pow(b1, (double)m->step), bc2 = 1.0 - std::pow(b2, (double)m->step);
    hipLaunchKernelGGL(k_adam, dim3(egrid(m->nparams)), dim3(kBlock), 0, s, m->nparams, m->params.get(),
                       m->grad.get(), m->adam_m.get(), m->adam_v.get(), lr, (float)b1, (float)b2, (float)(1.0 - b1),
                       (float)(1.0 - b2), 1e-8f, (float)(1.0 / bc1), (float)(1.0 / bc2));
    LAP_HIP(hipGetLastError());
}

void mpnn_output(lap_mpnn *m, const lap_plan &P, double *V0, hipStream_t s) {
    const int n = P.n, p = m->cfg.out_cols;
    hipLaunchKernelGGL(k_store_v, dim3(egrid((size_t)n * p)), dim3(kBlock), 0, s, n, p, m->yx.get(), kMpnnMaxCols,
                       P.d_perm.get(), V0);
    LAP_HIP(hipGetLastError());
}

}  // namespace lapeig
