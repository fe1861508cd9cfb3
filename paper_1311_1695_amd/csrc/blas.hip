// Outer-iteration kernels of Jacobi-Davidson, all in double precision:
// orthogonalization of the new direction (Algorithm 2 step 2), the border of
// H = V'GV (step 4), the eigenpairs of H (step 5), the Ritz vector and its
// residual (step 6), the certificate of a converged pair (exit test of
// Section 4 with the quotient of eq. (1)), restart and deflation.
//
// Storage: B = [X | V] is n x (kcap + m_max) column-major (ld = n): the
// locked eigenvectors X in columns [0, nx), the search basis V in
// [nx, nx + m).  W = G V is n x m_max column-major.  H is m_max x m_max.
#include "lapeig_dev.h"
#include "jd_kernels.h"

namespace lapeig {

namespace {

// ---------------------------------------------------------------------------
// Classical Gram-Schmidt, applied twice ("twice is enough"), of one vector
// against the nb = nx + m orthonormal columns of B.
//   pass 1: v = src (converted to double);     c = B'v,  n0 = ||v||^2
//   pass 2: v -= B c;                          c = B'v
//   pass 3: v -= B c;                          n1 = ||v||^2
// Each pass leaves one row of partial sums per workgroup and the next
// launch folds them (every workgroup the same totals, in one fixed order);
// the last pass's rows are folded by the launch that scales v (norm_scale).
// ---------------------------------------------------------------------------
template <typename S, int NV>
__global__ __launch_bounds__(kBlock) void k_orth1(double *__restrict__ part_out, int n, const double *__restrict__ B,
                                                  int nb, const S *__restrict__ src, double *__restrict__ v) {
    double acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double vi = (double)src[i];
        v[i] = vi;
#pragma unroll
        for (int j = 0; j < NV - 1; ++j)
            if (j < nb) acc[j] += B[(size_t)j * n + i] * vi;
        acc[NV - 1] += vi * vi;
    }
    // pack the norm right after the nb coefficients
    double packed[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) packed[j] = j < nb ? acc[j] : (j == nb ? acc[NV - 1] : 0.0);
    write_partials<double, NV>(packed, nb + 1, part_out);
}

template <int NV>
__global__ __launch_bounds__(kBlock) void k_orth2(const double *__restrict__ part_in, int nb_in,
                                                  double *__restrict__ part_out, int n, const double *__restrict__ B,
                                                  int nb, double *__restrict__ v, JDStatus *st, int first, int last) {
    __shared__ double c[NV];
    fold_partials<double, NV>(part_in, nb_in, nb + first, c);
    if (first && blockIdx.x == 0 && threadIdx.x == 0) st->orth_n0 = sqrt(c[nb]);
    double acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double vi = v[i];
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NV; ++j)
            if (j < nb) s += B[(size_t)j * n + i] * c[j];
        vi -= s;
        v[i] = vi;
        if (!last) {
#pragma unroll
            for (int j = 0; j < NV; ++j)
                if (j < nb) acc[j] += B[(size_t)j * n + i] * vi;
        } else {
            acc[0] += vi * vi;
        }
    }
    if (!last) {
        write_partials<double, NV>(acc, nb, part_out);
    } else {
        double a1[1] = {acc[0]};
        write_partials<double, 1>(a1, 1, part_out);
    }
}

// The norm of the orthogonalized v from the last pass's partial rows:
// n1 = ||v||, the direction is degenerate (it lay in span(B), rounding noise
// is left) when n1 <= 1e-12 n0, and the scale is 1/n1 (0 if degenerate).
// Every workgroup computes the same values; the first records them in st.
__device__ __forceinline__ double norm_scale(const double *__restrict__ rows, int nrows, JDStatus *st) {
    __shared__ double t[1];
    fold_partials<double, 1>(rows, nrows, 1, t);
    const double n1 = sqrt(t[0]);
    const bool degenerate = !(n1 > 1e-12 * st->orth_n0);
    const double sc = degenerate ? 0.0 : 1.0 / n1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->orth_n1 = n1;
        st->degenerate = degenerate;
        st->inv_norm = sc;
    }
    return sc;
}

// V[:, m] = v / ||v||,  W[:, m] = G V[:, m]  (one MVP, step 3)
template <bool Wt>
__global__ __launch_bounds__(kBlock) void k_spmv_normalize(const double *__restrict__ norm_rows, int norm_nrows,
                                                           JDStatus *st, Graph g, Weights<double> w,
                                                           const double *__restrict__ v,
                                                           double *__restrict__ vcol,
                                                           double *__restrict__ wcol) {
    const double s = norm_scale(norm_rows, norm_nrows, st);
    // a degenerate direction (s = 0, possibly from a non-finite input) leaves
    // exact zero columns, never 0 * inf or 0 * NaN
    for_each_row<double, Wt, false>(g, w, v, [&](int i, double xi, double yi, double) {
        vcol[i] = s != 0.0 ? xi * s : 0.0;
        wcol[i] = s != 0.0 ? yi * s : 0.0;
    });
}

// H(j, m) = H(m, j) = V[:, j]' W[:, m] for j <= m (step 4)
template <int NV>
__global__ __launch_bounds__(kBlock) void k_hborder(int n, const double *__restrict__ V, int m,
                                                    const double *__restrict__ wcol, double *H,
                                                    int ldh, double *partial, unsigned *counter) {
    double acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double wi = wcol[i];
#pragma unroll
        for (int j = 0; j < NV; ++j)
            if (j <= m) acc[j] += V[(size_t)j * n + i] * wi;
    }
    __shared__ double out[NV];
    if (grid_reduce<double, NV>(acc, m + 1, partial, counter, out)) {
        for (int j = threadIdx.x; j <= m; j += blockDim.x) {
            H[(size_t)m * ldh + j] = out[j];
            H[(size_t)j * ldh + m] = out[j];
        }
    }
}

// The same border as partial rows (m + 1 <= NV values per workgroup), which
// the Rayleigh-Ritz kernel folds.
template <int NV>
__global__ __launch_bounds__(kBlock) void k_hborder_part(double *__restrict__ part_out, int n,
                                                         const double *__restrict__ V, int m,
                                                         const double *__restrict__ wcol) {
    double acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double wi = wcol[i];
#pragma unroll
        for (int j = 0; j < NV; ++j)
            if (j <= m) acc[j] += V[(size_t)j * n + i] * wi;
    }
    write_partials<double, NV>(acc, m + 1, part_out);
}

// Makes the payload written to *hm visible to the host, then the sequence
// number the host waits for (host-coherent memory; one thread calls it).
__device__ __forceinline__ void publish(HostMirror *hm, unsigned seq) {
    __threadfence_system();
    __hip_atomic_store(&hm->seq, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// 1/x and 1/sqrt(x) (x > 0 finite) from the hardware FP64 estimates, each
// refined by two Newton steps (r <- r(2 - xr), y <- y(3 - xy^2)/2), which
// square the relative error twice and end within about an ulp.
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}
__device__ __forceinline__ double rsq_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    y = y * fma(-hx * y, y, 1.5);
    return y;
}

// Value of x in lane l of the wavefront (l wave-uniform).
__device__ __forceinline__ double lane_val(double x, int l) {
    const unsigned long long v = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ int lane_val(int x, int l) { return __builtin_amdgcn_readlane(x, l); }

constexpr int kArrowMax = 32;  // largest arrowhead of the secular-equation path

// ---------------------------------------------------------------------------
// Eigenpairs of an arrowhead matrix A = [diag(d) b; b' c] (m x m, n = m - 1
// poles), the form the projected matrix takes in every Rayleigh-Ritz step of
// single-vector JD: in the previous Ritz basis after an expansion, and after
// a restart or a lock, which leave H diagonal.  Its eigenvalues are the
// roots of the secular equation g(l) = c - l - sum_i b_i^2 / (d_i - l) = 0,
// which interlace the poles d_i; one lane finds one root.
//   1. sort the poles; deflate borders |b_i| <= tol (pair (d_i, e_i)) and
//      poles closer than tol (a plane rotation moves the border weight onto
//      one of the two), tol = 8 eps max(|d|, |c|, ||b||);
//   2. each root in coordinates shifted to its nearer pole o (tau = l - d_o,
//      differences of poles taken first): iterate on the model
//      g(x) ~ r(t) + r'(t)(x - t) + b_o^2 / x (the pole o exact, the rest of
//      g linear), whose zero is the root of a quadratic, inside a bracket
//      kept by the sign of g (bisection when the model root leaves it); stop
//      when |g| is at its rounding level;
//   3. recompute the border from the roots (Gu and Eisenstat),
//      b_i^2 = -prod_k (d_i - l_k) / prod_{j != i} (d_i - d_j), taken as a
//      product of bounded ratios, so that the eigenvectors
//      (b_i / (l_k - d_i) ..., 1) come out orthogonal to working precision;
//   4. undo the rotations and the sort; Y = Z X.
// One wavefront, m <= kArrowMax.  The poles, borders, roots and shifts stay
// in the registers of the lane that owns them and are read across lanes.
// zid: Z is the identity.  Returns false, having written nothing, when a
// root does not converge (the caller then runs Jacobi on the same A).
__device__ bool arrow_rr(int m, int me, double *A, const double *Z, bool zid, double *theta, double *Y, int ldy) {
    constexpr double kEps = 2.220446049250313e-16;
    __shared__ double ds[kWave], bs[kWave], kdl[kWave], kbl[kWave], rc[kWave], rs[kWave];
    __shared__ double dors[kWave + 1], rts[kWave + 1], bhs[kWave];
    __shared__ int pms[kWave], ips[kWave], kixs[kWave], ri[kWave];
    __shared__ int nrot_s;
    const int lane = lane_id();
    const int n = m - 1;
    // 1. poles, border, corner; the rank of each pole (ties by index)
    double di = 0.0, bi = 0.0;
    if (lane < n) {
        di = A[lane * me + lane];
        bi = A[lane * me + n];
    }
    const double c = A[n * me + n];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
        const double dj = lane_val(di, j);
        rank += (dj < di) || (dj == di && j < lane);
    }
    if (lane < n) {
        ds[rank] = di;
        bs[rank] = bi;
        pms[rank] = lane;
        ips[lane] = rank;
    }
    double amax = fabs(di), b2 = bi * bi;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        amax = fmax(amax, __shfl_xor(amax, o, kWave));
        b2 += __shfl_xor(b2, o, kWave);
    }
    const double bn = sqrt(b2);
    const double tol = 8.0 * kEps * fmax(fmax(amax, fabs(c)), bn);
    __syncthreads();
    // lane s holds the s-th smallest pole and its border
    const double dsl = lane < n ? ds[lane] : 0.0;
    double bsl = lane < n ? bs[lane] : 0.0;
    // close poles: rotate (i, i + 1) so that b_i = 0, in order of i.  Values
    // change only after a rotation, so if no pair qualifies as it stands the
    // ordered pass would do nothing: test all pairs at once first.
    const double dnext = __shfl_down(dsl, 1, kWave), bnext = __shfl_down(bsl, 1, kWave);
    const bool close = lane + 1 < n && fabs(bsl) > tol && fabs(bnext) > tol && dnext - dsl <= tol;
    int nr = 0;
    if (__ballot(close) != 0) {
        if (lane == 0) {
            int cnt = 0;
            for (int i = 0; i + 1 < n; ++i) {
                const double x = bs[i], y = bs[i + 1];
                if (fabs(x) > tol && fabs(y) > tol && ds[i + 1] - ds[i] <= tol) {
                    const double r = sqrt(fma(x, x, y * y));
                    rc[cnt] = y / r;
                    rs[cnt] = x / r;
                    ri[cnt] = i;
                    ++cnt;
                    bs[i] = 0.0;
                    bs[i + 1] = r;
                }
            }
            nrot_s = cnt;
        }
        __syncthreads();
        nr = nrot_s;
        bsl = lane < n ? bs[lane] : 0.0;
    }
    // the kept poles (|b| > tol), compacted: lane j < nk holds the j-th
    const bool keep = lane < n && fabs(bsl) > tol;
    const unsigned long long kmask = __ballot(keep);
    const int nk = __popcll(kmask);
    if (keep) {
        const int pos = __popcll(kmask & ((1ull << lane) - 1ull));
        kdl[pos] = dsl;
        kbl[pos] = bsl;
        kixs[pos] = lane;
    }
    __syncthreads();
    const double kd = lane < nk ? kdl[lane] : 0.0, kb = lane < nk ? kbl[lane] : 0.0;
    // 2. the nk + 1 roots of the secular equation of the kept part, in
    // coordinates shifted to the nearer pole o.  Root g is found by the G
    // lanes of group g (G = 8, 4 or 2 as nk + 1 <= 8, 16 or 32); lane `sub` of
    // a group takes the poles j = sub, sub + G, ... and the group adds its
    // sums by a butterfly, so all G lanes hold the same totals and take the
    // same steps.
    const int nroot = nk + 1;
    const int lg = nroot <= 8 ? 3 : (nroot <= 16 ? 2 : 1);
    const int G = 1 << lg;
    const int g = lane >> lg, sub = lane & (G - 1);
    auto group_sum = [&](double v) {
        v += lane_xor<1>(v);
        if (G >= 4) v += lane_xor<2>(v);
        if (G >= 8) v += lane_xor<4>(v);
        return v;
    };
    bool ok = true;
    int og = -1;
    double tg = c, dorg = 0.0;
    if (nk > 0 && g <= nk) {
        const double kdg = g < nk ? kdl[g] : 0.0, kdgm = g >= 1 ? kdl[g - 1] : 0.0;
        if (g == 0) {
            og = 0;
        } else if (g == nk) {
            og = nk - 1;
        } else {
            const double mid = 0.5 * (kdgm + kdg);
            double s = 0.0;
            for (int j = sub; j < nk; j += G) s += kbl[j] * kbl[j] * rcp_nr(kdl[j] - mid);
            const double gm = (c - mid) - group_sum(s);
            og = gm > 0.0 ? g : g - 1;
        }
        dorg = kdl[og];
        const double bo2 = kbl[og] * kbl[og];
        const double c0 = c - dorg;
        const double outer = bn + fabs(c0) + tol;
        double tlo = g >= 1 ? kdgm - dorg : -outer;
        double thi = g < nk ? kdg - dorg : outer;
        // start: the zero of the model at t = 0, -b_o^2 / r(0)
        double s0 = 0.0;
        for (int j = sub; j < nk; j += G)
            if (j != og) s0 += kbl[j] * kbl[j] * rcp_nr(kdl[j] - dorg);
        const double r0 = c0 - group_sum(s0);
        double t = r0 != 0.0 ? -bo2 / r0 : 0.5 * (tlo + thi);
        if (!(tlo < t && t < thi) || t == 0.0) t = 0.5 * (tlo + thi);
        ok = false;
        for (int it = 0; it < 80; ++it) {
            double R = 0.0, Rd = 0.0, Ab = 0.0;
            for (int j = sub; j < nk; j += G) {
                const double r = rcp_nr((kdl[j] - dorg) - t);
                const double sj = j != og ? kbl[j] * kbl[j] * r : 0.0;
                R += sj;
                Rd += sj * r;
                Ab += fabs(sj);
            }
            R = group_sum(R);
            Rd = group_sum(Rd);
            Ab = group_sum(Ab);
            const double rt_ = c0 - t - R, rdt = -1.0 - Rd;
            const double bt = bo2 * rcp_nr(t);
            const double gv = rt_ + bt;
            if (fabs(gv) <= 8.0 * kEps * (fabs(c0) + fabs(t) + Ab + fabs(bt))) { ok = true; break; }
            if (gv > 0.0) tlo = t; else thi = t;
            if (thi - tlo <= 4.0 * kEps * fmax(fabs(tlo), fabs(thi))) { ok = true; break; }
            const double beta = rdt, alpha = rt_ - t * rdt;
            const double disc = alpha * alpha - 4.0 * beta * bo2;
            double tn = 0.5 * (tlo + thi);
            if (disc >= 0.0) {
                const double q = -0.5 * (alpha + copysign(sqrt(disc), alpha));
                const double x1 = beta != 0.0 ? q * rcp_nr(beta) : tn, x2 = q != 0.0 ? bo2 * rcp_nr(q) : tn;
                const bool in1 = tlo < x1 && x1 < thi, in2 = tlo < x2 && x2 < thi;
                if (in1 && in2) tn = fabs(x1 - t) <= fabs(x2 - t) ? x1 : x2;
                else if (in1) tn = x1;
                else if (in2) tn = x2;
            }
            if (fabs(tn - t) <= 2.0 * kEps * fabs(t)) { ok = true; break; }
            t = tn;
            if (t == 0.0) break;
        }
        tg = t;
    }
    if (__ballot(!ok) != 0) return false;
    // back to one root per lane: lane k <= nk takes group k's root
    const int src = (lane <= nk ? lane : 0) << lg;
    const int o = __shfl(og, src, kWave);
    const double dor = __shfl(dorg, src, kWave), t = __shfl(tg, src, kWave);
    if (lane <= nk) {
        dors[lane] = dor;
        rts[lane] = t;
    }
    __syncthreads();
    // 3. the border from the roots (lane i < nk); with nk > 0 every root has
    // a pole, and l_k - d_i = t_k - (d_i - d_{o_k}) = -((d_i - d_{o_k}) - t_k)
    if (lane < nk) {
        const int i = lane;
        double pr = -((kd - dor) - t) * ((kd - dors[i + 1]) - rts[i + 1]);
#pragma unroll 4
        for (int j = 0; j < nk; ++j) {
            // roots j (below i) and j + 1 (above)
            const double num = j < i ? (kd - dors[j]) - rts[j] : (kd - dors[j + 1]) - rts[j + 1];
            const double den = j == i ? 1.0 : kd - kdl[j];
            pr *= j == i ? 1.0 : num * rcp_nr(den);
        }
        bhs[i] = copysign(sqrt(fmax(pr, 0.0)), kb);
    }
    __syncthreads();
    // the deflated lanes' sorted row: the (lane - nk - 1)-th row not kept
    int row = n;
    for (int i = 0, cnt = lane - (nk + 1); cnt >= 0 && i < n; ++i)
        if (!((kmask >> i) & 1ull)) {
            if (cnt == 0) { row = i; break; }
            --cnt;
        }
    const double ldefl = __shfl(dsl, row < n ? row : 0, kWave);
    // 4. eigenvector p (lane p < m) in the sorted coordinates (rows 0..n-1
    // the sorted poles, row n the corner), one column per lane, into A (no
    // longer needed): roots p <= nk take (b_j / (l_p - d_j) ..., 1)
    // normalized; the deflated poles, in sorted order after the roots, their
    // unit vectors.
    double *X = A;
    double lam = 0.0;
    if (lane < m) {
        const int p = lane;
        for (int r = 0; r < n; ++r) X[r * me + p] = 0.0;
        if (p <= nk) {
            lam = o >= 0 ? dor + t : t;
            double nrm = 1.0;
#pragma unroll 4
            for (int j = 0; j < nk; ++j) {
                const double v = -bhs[j] * rcp_nr((kdl[j] - dor) - t);
                X[kixs[j] * me + p] = v;
                nrm = fma(v, v, nrm);
            }
            const double inv = rsq_nr(nrm);
#pragma unroll 4
            for (int j = 0; j < nk; ++j) X[kixs[j] * me + p] *= inv;
            X[n * me + p] = inv;
        } else {
            X[row * me + p] = 1.0;
            X[n * me + p] = 0.0;
            lam = ldefl;
        }
        // undo the rotations (last first) on the rows
        for (int q = nr - 1; q >= 0; --q) {
            const int i = ri[q];
            const double cq = rc[q], sq = rs[q];
            const double xi = X[i * me + p], xj = X[(i + 1) * me + p];
            X[i * me + p] = cq * xi + sq * xj;
            X[(i + 1) * me + p] = -sq * xi + cq * xj;
        }
    }
    // ascending order (ties by index)
    int lr = 0;
    for (int q = 0; q < m; ++q) {
        const double lq = lane_val(lam, q);
        lr += (lq < lam) || (lq == lam && q < lane);
    }
    if (lane < m) theta[lr] = lam;
    __syncthreads();
    // Y(:, rank_c) = Z X(original rows, c); sorted row s is original row pm_s.
    // Lane l computes rows (l >> 5) + 2i of column l & 31.
    const int cc = lane & 31;
    const int rk = __shfl(lr, cc, kWave);
    if (cc < m) {
        for (int r = lane >> 5; r < m; r += 2) {
            double y;
            if (zid) {
                y = X[(r < n ? ips[r] : n) * me + cc];
            } else {
                const double *zr = Z + r * me;
                y = zr[n] * X[n * me + cc];
#pragma unroll 4
                for (int s = 0; s < n; ++s) y = fma(zr[pms[s]], X[s * me + cc], y);
            }
            Y[(size_t)rk * ldy + r] = y;
        }
    }
    return true;
}

// ---------------------------------------------------------------------------
// All eigenpairs of the small symmetric H (step 5) in one workgroup:
// cyclic Jacobi in the round-robin (tournament) ordering, so the m/2
// rotations of a round act on disjoint index pairs and run in parallel.
// Rotation as in Golub & Van Loan (symmetric Schur 2x2).  Off-diagonal
// entries below eps ||H||_F / m are skipped; sweeps stop when none is left.
// Output: theta ascending (ties by index), Y column-major (ld = ldy).
// ---------------------------------------------------------------------------
constexpr int kRRMax = 96;  // 2 * 96^2 doubles of LDS (147 KB) at most
// Threads of the Rayleigh-Ritz launch above 32 columns: two wavefronts per
// SIMD hide each other's LDS latency in the rounds (m = 60: 1.68 -> 1.10 ms
// against four wavefronts), and the register budget of 2 per SIMD leaves
// the one-wavefront arrowhead path unspilled.
constexpr int kRRThreads = 512;
// Rotation items per thread: (me / 2)^2 blocks of A and me (me / 2) items of
// Z over the launch (kRRThreads, or one wavefront for me <= 32)
constexpr int kRRItemsA = 5, kRRItemsZ = 9;
static_assert((kRRMax / 2) * (kRRMax / 2) <= kRRItemsA * kRRThreads && 16 * 16 <= kRRItemsA * kWave,
              "A items per thread");
static_assert(kRRMax * (kRRMax / 2) <= kRRItemsZ * kRRThreads && 32 * 16 <= kRRItemsZ * kWave,
              "Z items per thread");

// The last column of H from the border kernel's partial rows (brows <= 4 x 64
// rows, stride bld, m <= kDeferBorderMax values wanted) in one wavefront:
// lane l adds rows l, l + 64, ... in that order, then a fixed butterfly.
__device__ void fold_border_rows(const double *__restrict__ bpart, int brows, int bld, int m, double *hcol) {
    double acc[kDeferBorderMax];
#pragma unroll
    for (int c = 0; c < kDeferBorderMax; ++c) acc[c] = 0.0;
#pragma unroll
    for (int q = 0; q < kDeferRows / kWave; ++q) {
        const int r = lane_id() + q * kWave;
        if (r < brows) {
#pragma unroll
            for (int c = 0; c < kDeferBorderMax; ++c)
                if (c < m) acc[c] += bpart[(size_t)r * bld + c];
        }
    }
    const int idx = wave_reduce_scatter<double, kDeferBorderMax>(acc);
    if ((lane_id() & (kWave / kDeferBorderMax - 1)) == 0 && idx < m) hcol[idx] = acc[0];
}

// One 2x2 block of a Jacobi round, A(pk, pl) with pair k's rows and pair l's
// columns: the row rotation of k, then the column rotation of l (the same
// operations in the same order as a rows pass followed by a columns pass);
// on the rotated pair's own block (k == l) the off-diagonal entries are 0.
__device__ __forceinline__ void rotate_block(double sk, double ck, double sl, double cl, bool own, double &apr,
                                             double &apc, double &aqr, double &aqc) {
    if (sk != 0.0) {
        const double npr = ck * apr - sk * aqr, nqr = sk * apr + ck * aqr;
        const double npc = ck * apc - sk * aqc, nqc = sk * apc + ck * aqc;
        apr = npr; aqr = nqr; apc = npc; aqc = nqc;
    }
    if (sl != 0.0) {
        const double npr = cl * apr - sl * apc, npc = sl * apr + cl * apc;
        const double nqr = cl * aqr - sl * aqc, nqc = sl * aqr + cl * aqc;
        apr = npr; apc = npc; aqr = nqr; aqc = nqc;
    }
    if (own) { apc = 0.0; aqr = 0.0; }
}

__global__ __launch_bounds__(kRRThreads) void k_rr_eig(int m, double *Hin, int ldh, double *__restrict__ theta,
                                                   double *__restrict__ Y, int ldy, int mprev, JDStatus *st,
                                                   const double *__restrict__ bpart, int brows, int bld) {
    extern __shared__ double lds[];
    const int me = (m + 1) & ~1;  // even size; index m is a dummy when m is odd
    double *A = lds;              // me x me, row-major
    double *Z = A + me * me;      // me x me, row-major accumulator of rotations
    __shared__ double cs[kRRMax / 2], sn[kRRMax / 2];
    __shared__ int pp[kRRMax / 2], qq[kRRMax / 2];
    __shared__ int rotates[2];  // some pair of the round rotates (by round parity)
    __shared__ double fro2;
    __shared__ double hcol[kDeferBorderMax];  // the last column of H, when folded here
    const int tid = threadIdx.x;
    // warm start: H = [H1 H12; H12' H22] with H1 = Yp diag(theta) Yp' from the
    // previous call (theta and Y still hold it): start from
    // [diag(theta) Yp'H12; H12'Yp H22] and accumulate onto Z = diag(Yp, I)
    const bool warm = mprev >= 1 && mprev < m;
    const int mp = warm ? mprev : 0;
    if (blockDim.x == kWave) {
        // me <= 32, one wavefront: lane l builds column l & 31, rows (l >> 5) + 2q.
        // The loads of Yp, theta and H are issued together with those of the
        // border's partial rows, before anything waits on them.  With border
        // rows, row and column m - 1 of H come from the fold instead of Hin.
        const int j = tid & 31, i0 = tid >> 5;
        const bool bcol = bpart != nullptr;
        double zr[16], ar[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int i = i0 + 2 * q;
            double z = i == j ? 1.0 : 0.0, a = 0.0;
            if (i < me && j < me) {
                const bool inh = i < m && j < m && !(bcol && (i == m - 1 || j == m - 1));
                if (warm) {
                    if (i < mp && j < mp) z = Y[(size_t)j * ldy + i];
                    else if (i < mp && j < m && inh) z = Hin[(size_t)j * ldh + i];  // H12, staged in Z
                    if (i == j && i < mp) a = theta[i];
                    else if (i >= mp && j >= mp && inh) a = Hin[(size_t)j * ldh + i];
                } else if (inh) {
                    a = Hin[(size_t)j * ldh + i];
                }
            }
            zr[q] = z;
            ar[q] = a;
        }
        if (bcol) {
            // the new last column of H from the border kernel's partial rows
            // (m <= kDeferBorderMax values, brows <= 4 x 64 rows): lane l adds
            // rows l, l + 64, ..., then a fixed butterfly
            fold_border_rows(bpart, brows, bld, m, hcol);
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int i = i0 + 2 * q;
            if (i < me && j < me) {
                double z = zr[q], a = ar[q];
                if (bcol && i < m && j < m && (i == m - 1 || j == m - 1)) {
                    const double h = hcol[i == m - 1 ? j : i];
                    if (warm && i < mp) z = h;                    // H12
                    else if (!warm || (i >= mp && j >= mp)) a = h;  // H, H22
                }
                Z[i * me + j] = z;
                A[i * me + j] = a;
            }
        }
        __syncthreads();
        if (warm) {
            // A12 = Yp' H12 from LDS, then Z's upper-right block back to zero
            for (int t = tid; t < mp * (m - mp); t += blockDim.x) {
                const int i = t % mp, c = mp + t / mp;
                double v = 0.0;
                for (int r = 0; r < mp; ++r) v += Z[r * me + i] * Z[r * me + c];
                A[i * me + c] = v;
                A[c * me + i] = v;
            }
            __syncthreads();
            for (int t = tid; t < mp * (me - mp); t += blockDim.x) Z[(t % mp) * me + mp + t / mp] = 0.0;
            __syncthreads();
        }
    } else {
        // me > 32 (no border rows: those come only with m <= kDeferBorderMax)
        if (warm) {
            for (int t = tid; t < me * me; t += blockDim.x) {
                const int i = t / me, j = t % me;
                Z[t] = (i < mp && j < mp) ? Y[(size_t)j * ldy + i] : (i == j ? 1.0 : 0.0);
                A[t] = (i == j && i < mp) ? theta[i]
                                          : ((i >= mp && j >= mp && i < m && j < m) ? Hin[(size_t)j * ldh + i] : 0.0);
            }
            __syncthreads();
            for (int t = tid; t < mp * (m - mp); t += blockDim.x) {
                const int i = t % mp, c = mp + t / mp;
                double v = 0.0;
                for (int r = 0; r < mp; ++r) v += Z[r * me + i] * Hin[(size_t)c * ldh + r];
                A[i * me + c] = v;
                A[c * me + i] = v;
            }
        } else {
            for (int t = tid; t < me * me; t += blockDim.x) {
                const int i = t / me, j = t % me;
                A[t] = (i < m && j < m) ? Hin[(size_t)j * ldh + i] : 0.0;
                Z[t] = (i == j) ? 1.0 : 0.0;
            }
        }
        __syncthreads();
    }
    // H's folded border back to global memory, after everything else
    auto flush_border = [&]() {
        if (bpart && tid < m) {
            Hin[(size_t)(m - 1) * ldh + tid] = hcol[tid];
            Hin[(size_t)tid * ldh + (m - 1)] = hcol[tid];
        }
    };
    // arrowhead (the leading m-1 block exactly diagonal, as it is by
    // construction after a warm start from m - 1): the secular-equation path
    if (blockDim.x == kWave && m >= 2 && m <= kArrowMax) {
        bool offd = false;
        if (!(warm && mp == m - 1))
            for (int t = tid; t < (m - 1) * (m - 1); t += blockDim.x) {
                const int i = t / (m - 1), j = t % (m - 1);
                offd |= i != j && A[i * me + j] != 0.0;
            }
        if (__ballot(offd) == 0 && arrow_rr(m, me, A, Z, !warm, theta, Y, ldy)) {
            flush_border();
            if (tid == 0 && st) st->rr_sweeps = -1;  // the secular-equation path
            return;
        }
        __syncthreads();
    }
    {
        __shared__ double wsum[kRRThreads / kWave];
        double f = 0.0;
        for (int t = tid; t < me * me; t += blockDim.x) f += A[t] * A[t];
        f = wave_sum(f);
        if (lane_id() == 0) wsum[wave_id()] = f;
        __syncthreads();
        if (tid == 0) {
            double g = 0.0;
            for (int w = 0; w < (int)blockDim.x / kWave; ++w) g += wsum[w];
            fro2 = g;
        }
        __syncthreads();
    }
    const double tol = 2.220446049250313e-16 * sqrt(fro2) / (double)me;
    const int half = me / 2, m1 = me - 1;
    // The items of every round are the same: this thread's 2x2 blocks of A
    // (pair k rows, pair l columns) and (row, pair) items of Z, taken once
    // here, packed as (k << 8) | l and (row << 8) | k
    const int nA = half * half, nZ = me * half, bd = (int)blockDim.x;
    int itA[kRRItemsA], itZ[kRRItemsZ];
    int na = 0, nz = 0;
#pragma unroll
    for (int j = 0; j < kRRItemsA; ++j) {
        const int e = tid + j * bd;
        itA[j] = e < nA ? ((e / half) << 8) | (e % half) : 0;
        na += e < nA;
    }
#pragma unroll
    for (int j = 0; j < kRRItemsZ; ++j) {
        const int e = tid + j * bd;
        itZ[j] = e < nZ ? ((e / half) << 8) | (e % half) : 0;
        nz += e < nZ;
    }
    int sweeps = 0;
    for (; sweeps < 60 && me > 1; ++sweeps) {
        // A sweep rotates exactly the pairs with |a_pq| > tol, so when no
        // off-diagonal entry exceeds tol it would change nothing: stop here
        // instead of running it.
        {
            __shared__ double wmax[kRRThreads / kWave];
            double mx = 0.0;
            for (int t = tid; t < me * me; t += blockDim.x)
                if (t / me < t % me) mx = fmax(mx, fabs(A[t]));
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, kWave));
            if (lane_id() == 0) wmax[wave_id()] = mx;
            __syncthreads();
            double g = 0.0;
            for (int w = 0; w < (int)blockDim.x / kWave; ++w) g = fmax(g, wmax[w]);
            __syncthreads();
            if (!(g > tol)) break;
        }
        for (int round = 0; round < me - 1; ++round) {
            // tournament pairing: position 0 fixed, the others rotate
            if (tid < kWave) {  // the pairs of a round (half <= 48) sit in the first wavefront
                bool rot = false;
                if (tid < half) {
                    auto player = [&](int pos) {
                        if (pos == 0) return 0;
                        const int x = pos - 1 + round;  // < 2 (me - 1)
                        return 1 + (x >= m1 ? x - m1 : x);
                    };
                    int a = player(tid), b = player(me - 1 - tid);
                    int p = a < b ? a : b, q = a < b ? b : a;
                    double c = 1.0, s = 0.0;
                    const double apq = A[p * me + q], app = A[p * me + p], aqq = A[q * me + q];
                    // (entries below the smallest normal are left alone: the
                    // hardware reciprocal estimate does not take them)
                    if (fabs(apq) > fmax(tol, 2.2250738585072014e-308)) {
                        // tau = (aqq - app) / (2 apq), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
                        // c = 1 / sqrt(1 + t^2), s = t c; for |tau| > 1e150, t = 1 / (2 tau)
                        // to double precision (and tau^2 would overflow)
                        const double tau = (aqq - app) * rcp_nr(2.0 * apq);
                        const double at = fabs(tau);
                        const double w = fma(tau, tau, 1.0);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) *
                                         (at > 1e150 ? 0.5 * rcp_nr(at) : rcp_nr(at + w * rsq_nr(w)));
                        c = rsq_nr(fma(t, t, 1.0));
                        s = t * c;
                        rot = true;
                    }
                    pp[tid] = p; qq[tid] = q; cs[tid] = c; sn[tid] = s;
                }
                const bool any = __ballot(rot) != 0;
                if (tid == 0) rotates[round & 1] = any;
            }
            __syncthreads();
            if (!rotates[round & 1]) continue;  // nothing to rotate: no update, no second barrier
            // A <- J'AJ.  The pairs of a round are disjoint, so A falls into
            // independent 2x2 blocks (pair k rows, pair l columns); each item
            // applies the row rotation of k and then the column rotation of l
            // to its block, the same operations in the same order as a rows
            // pass followed by a columns pass.  Z <- ZJ likewise by (row, pair).
            // Items e = tid, tid + blockDim.x, ... in pairs: both items'
            // parameters and entries are read before either is computed, so
            // a thread waits for LDS once per pair of items.
#pragma unroll
            for (int j = 0; j < kRRItemsA; j += 2) {
                if (j >= na) break;
                const bool two = j + 1 < na;
                const int ka = itA[j] >> 8, la = itA[j] & 255;
                const int kb = two ? itA[j + 1] >> 8 : ka, lb = two ? itA[j + 1] & 255 : la;
                const double ska = sn[ka], sla = sn[la], cka = cs[ka], cla = cs[la];
                const double skb = sn[kb], slb = sn[lb], ckb = cs[kb], clb = cs[lb];
                const int pa = pp[ka], qa = qq[ka], ra = pp[la], ca = qq[la];
                const int pb = pp[kb], qb = qq[kb], rb = pp[lb], cb = qq[lb];
                double a0 = A[pa * me + ra], a1 = A[pa * me + ca], a2 = A[qa * me + ra], a3 = A[qa * me + ca];
                double b0 = A[pb * me + rb], b1 = A[pb * me + cb], b2 = A[qb * me + rb], b3 = A[qb * me + cb];
                if (!(ska == 0.0 && sla == 0.0)) {
                    rotate_block(ska, cka, sla, cla, ka == la, a0, a1, a2, a3);
                    A[pa * me + ra] = a0; A[pa * me + ca] = a1; A[qa * me + ra] = a2; A[qa * me + ca] = a3;
                }
                if (two && !(skb == 0.0 && slb == 0.0)) {
                    rotate_block(skb, ckb, slb, clb, kb == lb, b0, b1, b2, b3);
                    A[pb * me + rb] = b0; A[pb * me + cb] = b1; A[qb * me + rb] = b2; A[qb * me + cb] = b3;
                }
            }
#pragma unroll
            for (int j = 0; j < kRRItemsZ; j += 2) {
                if (j >= nz) break;
                const bool two = j + 1 < nz;
                const int ia = itZ[j] >> 8, ka = itZ[j] & 255;
                const int ib = two ? itZ[j + 1] >> 8 : ia, kb = two ? itZ[j + 1] & 255 : ka;
                const double ska = sn[ka], cka = cs[ka], skb = sn[kb], ckb = cs[kb];
                const int pa = pp[ka], qa = qq[ka], pb = pp[kb], qb = qq[kb];
                const double zpa = Z[ia * me + pa], zqa = Z[ia * me + qa];
                const double zpb = Z[ib * me + pb], zqb = Z[ib * me + qb];
                if (ska != 0.0) {
                    Z[ia * me + pa] = cka * zpa - ska * zqa;
                    Z[ia * me + qa] = ska * zpa + cka * zqa;
                }
                if (two && skb != 0.0) {
                    Z[ib * me + pb] = ckb * zpb - skb * zqb;
                    Z[ib * me + qb] = skb * zpb + ckb * zqb;
                }
            }
            __syncthreads();
        }
    }
    // rank sort of the m real diagonal entries (the dummy index is excluded)
    for (int i = tid; i < m; i += blockDim.x) {
        const double di = A[i * me + i];
        int rank = 0;
        for (int j = 0; j < m; ++j) {
            const double dj = A[j * me + j];
            rank += (dj < di) || (dj == di && j < i);
        }
        theta[rank] = di;
        for (int r = 0; r < m; ++r) Y[(size_t)rank * ldy + r] = Z[r * me + i];
    }
    flush_border();
    if (tid == 0 && st) st->rr_sweeps = sweeps;
}

// u = V y, Gu ~= W y, r = W y - theta u (step 6); also u into column `qcol`
// of the row-major PCG projector Q (type T, ld = ldq).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ritz(int n, const double *__restrict__ V,
                                                 const double *__restrict__ W, int m,
                                                 const double *__restrict__ Y, const double *__restrict__ theta,
                                                 double *__restrict__ u, double *__restrict__ r,
                                                 T *__restrict__ Q, int ldq, int qcol, double *partial,
                                                 unsigned *counter, JDStatus *st, HostMirror *hm, unsigned seq) {
    __shared__ double y[kRRMax];
    for (int j = threadIdx.x; j < m; j += blockDim.x) y[j] = Y[j];
    __syncthreads();
    const double th = theta[0];
    double acc[2] = {0.0, 0.0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double ui = 0.0, gi = 0.0;
        for (int j = 0; j < m; ++j) {
            ui += V[(size_t)j * n + i] * y[j];
            gi += W[(size_t)j * n + i] * y[j];
        }
        const double ri = gi - th * ui;
        u[i] = ui;
        r[i] = ri;
        Q[(size_t)i * ldq + qcol] = (T)ui;
        acc[0] += ri * ri;
        acc[1] += ui * ui;
    }
    __shared__ double out[2];
    if (grid_reduce<double, 2>(acc, 2, partial, counter, out)) {
        if (threadIdx.x == 0) {
            const double un = sqrt(out[1]);
            const double rn = sqrt(out[0]) / un;
            st->theta = th;
            st->unorm = un;
            st->rnorm = rn;
            if (hm) {
                hm->theta = th;
                hm->unorm = un;
                hm->rnorm = rn;
                hm->degenerate = st->degenerate;
                publish(hm, seq);
            }
        }
    }
}

// Certificate, part 1: Gu with a fresh product and the Rayleigh quotient by
// eq. (1): theta = (1/2) sum_ij A_ij (u_i - u_j)^2 / u'u.
template <bool Wt>
__global__ __launch_bounds__(kBlock) void k_cert1(Graph g, Weights<double> w, const double *__restrict__ u,
                                                  double *__restrict__ gu, double *partial,
                                                  unsigned *counter, JDStatus *st) {
    double acc[2] = {0.0, 0.0};
    for_each_row<double, Wt, true>(g, w, u, [&](int i, double xi, double yi, double qi) {
        gu[i] = yi;
        acc[0] += qi;
        acc[1] += xi * xi;
    });
    __shared__ double out[2];
    if (grid_reduce<double, 2>(acc, 2, partial, counter, out)) {
        if (threadIdx.x == 0) {
            st->cert_unorm2 = out[1];
            st->cert_theta = 0.5 * out[0] / out[1];
        }
    }
}

// Certificate, part 2: ||G u - theta u|| / ||u||.
__global__ __launch_bounds__(kBlock) void k_cert2(int n, const double *__restrict__ u,
                                                  const double *__restrict__ gu, double *partial,
                                                  unsigned *counter, JDStatus *st, HostMirror *hm, unsigned seq) {
    const double th = st->cert_theta;
    double acc[1] = {0.0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double d = gu[i] - th * u[i];
        acc[0] += d * d;
    }
    __shared__ double out[1];
    if (grid_reduce<double, 1>(acc, 1, partial, counter, out)) {
        if (threadIdx.x == 0) {
            const double cr = sqrt(out[0] / st->cert_unorm2);
            st->cert_rnorm = cr;
            if (hm) {
                hm->cert_theta = th;
                hm->cert_rnorm = cr;
                publish(hm, seq);
            }
        }
    }
}

// In-place basis rotation, row by row: for each matrix job,
//   out[:, j] = (M Y)[:, c0 + j] * (j == 0 ? scale0 : 1),  j < nc,
// where M = in[:, 0..m) and out may overlap in (each row is read before it
// is written, by the same thread).  Used for restarts (keep the Ritz vectors
// of the m_min smallest Ritz values) and deflation (lock u = V y_1, keep V y_j).
struct RotJob {
    const double *in;
    double *out;
    int c0, nc;
    const double *scale0;  // device scalar applied to output column 0, or null
};

template <int MM>
__global__ __launch_bounds__(kBlock) void k_rotate(int n, int m, const double *__restrict__ Y, int ldy,
                                                   RotJob j0, RotJob j1) {
    __shared__ double Ys[MM * MM];
    // zero padding: rows c >= m of each column multiply zero inputs
    for (int t = threadIdx.x; t < MM * MM; t += blockDim.x) {
        const int col = t / MM, c = t % MM;
        Ys[t] = (col < m && c < m) ? Y[(size_t)col * ldy + c] : 0.0;
    }
    __syncthreads();
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        for (int job = 0; job < 2; ++job) {
            const RotJob &J = job ? j1 : j0;
            if (!J.in || J.nc <= 0) continue;
            // the whole input row is read before any output of the row is written
            double row[MM];
#pragma unroll
            for (int c = 0; c < MM; ++c) row[c] = c < m ? J.in[(size_t)c * n + i] : 0.0;
            const double sc = J.scale0 ? *J.scale0 : 1.0;
#pragma unroll 1
            for (int o = 0; o < J.nc; ++o) {
                const double *yc = Ys + (J.c0 + o) * MM;
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < MM; ++c) s += row[c] * yc[c];
                J.out[(size_t)o * n + i] = o == 0 ? s * sc : s;
            }
        }
    }
}

// H = diag(theta[off .. off+cnt)) (after a restart or a deflation)
__global__ void k_hdiag(double *H, int ldh, int cnt, const double *theta, int off) {
    for (int t = threadIdx.x; t < ldh * ldh; t += blockDim.x) {
        const int i = t / ldh, j = t % ldh;
        H[t] = (i == j && i < cnt) ? theta[off + i] : 0.0;
    }
}

// Zero eigenvectors (Section 2): normalized indicator of each component.
template <typename T>
__global__ void k_zero_space(int n, int nz, const int *__restrict__ comp, const double *__restrict__ inv_sqrt_size,
                             double *__restrict__ B, T *__restrict__ Q, int ldq) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int c = comp[i];
        for (int j = 0; j < nz; ++j) {
            const double val = (c == j) ? inv_sqrt_size[j] : 0.0;
            B[(size_t)j * n + i] = val;
            Q[(size_t)i * ldq + j] = (T)val;
        }
    }
}

// Start vector: SplitMix64 (Steele, Lea & Flood 2014) used as a counter-based
// generator: entry i of column `colidx` takes output number colidx*n + (the
// caller's index of plan row i) of the stream `seed`, mapped to [-1, 1).
__device__ __forceinline__ double splitmix_unit(unsigned long long seed, unsigned long long idx) {
    unsigned long long z = seed + (idx + 1ULL) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

__global__ void k_random(int n, unsigned long long seed, long long colidx, const int *__restrict__ iperm,
                         double *__restrict__ v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        v[i] = splitmix_unit(seed, (unsigned long long)colidx * (unsigned long long)n + iperm[i]);
}

__global__ __launch_bounds__(kBlock) void k_scale_copy(const double *__restrict__ norm_rows, int norm_nrows,
                                                       JDStatus *st, int n, const double *__restrict__ v,
                                                       double *__restrict__ out) {
    const double sc = norm_scale(norm_rows, norm_nrows, st);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        out[i] = sc != 0.0 ? v[i] * sc : 0.0;
}

inline int vec_grid(int n) {
    int g = (n + kBlock - 1) / kBlock;
    const int cap = 4 * device_cu_count();
    return g < 1 ? 1 : (g > cap ? cap : g);
}

// Output of the eigenvectors: column j = column order[j] of X (plan order,
// element (i, c) at X[i sr + c sc]) in the caller's vertex order, with the
// sign that makes its largest-magnitude entry positive (ties: the lowest
// caller index).  Two launches over (chunk of rows, column): the first
// leaves each chunk's (max |x|, its first index), the second folds a
// column's chunks (max with the lowest index on ties, the same in any order)
// and writes its rows.

// (value, index) of the workgroup: the largest value, the lowest index on ties
__device__ __forceinline__ void argmax_block(double &bv, int &bi) {
    __shared__ double sv[kBlock];
    __shared__ int si[kBlock];
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            const double ov = sv[threadIdx.x + h];
            const int oi = si[threadIdx.x + h];
            if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                sv[threadIdx.x] = ov;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    bv = sv[0];
    bi = si[0];
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_final_max(int n, int rows_per, const double *__restrict__ X,
                                                      long long sr, long long sc, const int *__restrict__ order,
                                                      const int *__restrict__ perm, double *__restrict__ part) {
    const int j = blockIdx.y, ch = blockIdx.x;
    const long long c = order[j];
    const int i0 = ch * rows_per, i1 = min(n, i0 + rows_per);
    double bv = -1.0;
    int bi = n;
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const double v = fabs(X[(long long)perm[i] * sr + c * sc]);
        if (v > bv) { bv = v; bi = i; }  // i increases: the first maximum stays
    }
    argmax_block(bv, bi);
    if (threadIdx.x == 0) {
        part[((size_t)j * gridDim.x + ch) * 2] = bv;
        part[((size_t)j * gridDim.x + ch) * 2 + 1] = (double)bi;
    }
}

__global__ __launch_bounds__(kBlock) void k_final_write(int n, int rows_per, const double *__restrict__ X,
                                                        long long sr, long long sc, const int *__restrict__ order,
                                                        const int *__restrict__ perm,
                                                        const double *__restrict__ part, double *__restrict__ out) {
    const int j = blockIdx.y, ch = blockIdx.x, nch = gridDim.x;
    const long long c = order[j];
    double bv = -1.0;
    int bi = n;
    for (int q = threadIdx.x; q < nch; q += blockDim.x) {
        const double v = part[((size_t)j * nch + q) * 2];
        const int i = (int)part[((size_t)j * nch + q) * 2 + 1];
        if (v > bv || (v == bv && i < bi)) { bv = v; bi = i; }
    }
    argmax_block(bv, bi);
    const double sign = (bi < n && X[(long long)perm[bi] * sr + c * sc] < 0.0) ? -1.0 : 1.0;
    const int i0 = ch * rows_per, i1 = min(n, i0 + rows_per);
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x)
        out[(size_t)j * n + i] = sign * X[(long long)perm[i] * sr + c * sc];
}

}  // namespace

// ------------------------------------------------------------------ launchers

// Grid of the kernels whose sums are deferred: at most kDeferRows
// workgroups, so that a fold reads at most that many partial rows.
inline int defer_grid(int n) {
    const int g = (n + kBlock - 1) / kBlock;
    return g < 1 ? 1 : (g > kDeferRows ? kDeferRows : g);
}

// Grid of the Gram-Schmidt passes: streaming kernels that large vectors
// want spread over more workgroups than a deferred fold of kDeferRows rows
// allows; their partial rows (two workgroups per compute unit at most) are
// folded by the next pass and the norm's consumer in every workgroup.
inline int orth_grid(int n) {
    const int g = (n + kBlock - 1) / kBlock, cap = std::max(kDeferRows, 2 * device_cu_count());
    return g < 1 ? 1 : (g > cap ? cap : g);
}

template <typename S, int NV>
static void orth_nv(int n, const double *B, int nb, const S *src, double *v, ReduceScratch &rs, JDStatus *st,
                    hipStream_t s) {
    const int grid = orth_grid(n);
    rs.ensure_deferred();
    double *pa = rs.dpart.get(), *pb = pa + (size_t)rs.darea * 64;
    hipLaunchKernelGGL((k_orth1<S, NV>), dim3(grid), dim3(kBlock), 0, s, pa, n, B, nb, src, v);
    hipLaunchKernelGGL((k_orth2<NV>), dim3(grid), dim3(kBlock), 0, s, pa, grid, pb, n, B, nb, v, st, 1, 0);
    hipLaunchKernelGGL((k_orth2<NV>), dim3(grid), dim3(kBlock), 0, s, pb, grid, pa, n, B, nb, v, st, 0, 1);
    rs.norm_rows = pa;
    rs.norm_nrows = grid;
    LAP_HIP(hipGetLastError());
}

template <typename S>
void jd_orth(int n, const double *B, int nb, const S *src, double *v, ReduceScratch &rs, JDStatus *st,
             hipStream_t s) {
    LAP_REQUIRE(nb + 1 <= 64, LAP_EUNSUPPORTED, "basis wider than 63 columns");
    if (nb + 1 <= 16) orth_nv<S, 16>(n, B, nb, src, v, rs, st, s);
    else if (nb + 1 <= 32) orth_nv<S, 32>(n, B, nb, src, v, rs, st, s);
    else orth_nv<S, 64>(n, B, nb, src, v, rs, st, s);
}
template void jd_orth<float>(int, const double *, int, const float *, double *, ReduceScratch &, JDStatus *, hipStream_t);
template void jd_orth<double>(int, const double *, int, const double *, double *, ReduceScratch &, JDStatus *, hipStream_t);

void jd_expand(const lap_plan &P, const double *v, double *vcol, double *wcol, JDStatus *st,
               const ReduceScratch &rs, hipStream_t s) {
    LAP_REQUIRE(rs.norm_rows != nullptr, LAP_EDEVICE, "expansion without an orthogonalized vector");
    const int grid = row_grid(P.g, 1 << 20);
    if (P.weighted)
        hipLaunchKernelGGL((k_spmv_normalize<true>), dim3(grid), dim3(kBlock), 0, s, rs.norm_rows, rs.norm_nrows,
                           st, P.g, P.weights<double>(), v, vcol, wcol);
    else
        hipLaunchKernelGGL((k_spmv_normalize<false>), dim3(grid), dim3(kBlock), 0, s, rs.norm_rows,
                           rs.norm_nrows, st, P.g, P.weights<double>(), v, vcol, wcol);
    LAP_HIP(hipGetLastError());
}

void jd_hborder(int n, const double *V, int m, const double *wcol, double *H, int ldh, ReduceScratch &rs,
                hipStream_t s) {
    LAP_REQUIRE(m + 1 <= 64, LAP_EUNSUPPORTED, "search space wider than 64 columns");
    rs.border_rows = nullptr;
    if (m + 1 <= kDeferBorderMax) {
        // partial rows only; the Rayleigh-Ritz launch folds them into H
        const int grid = defer_grid(n);
        rs.ensure_deferred();
        double *pb = rs.dpart.get() + (size_t)rs.darea * 64;
        if (m + 1 <= 16)
            hipLaunchKernelGGL((k_hborder_part<16>), dim3(grid), dim3(kBlock), 0, s, pb, n, V, m, wcol);
        else
            hipLaunchKernelGGL((k_hborder_part<32>), dim3(grid), dim3(kBlock), 0, s, pb, n, V, m, wcol);
        LAP_HIP(hipGetLastError());
        rs.border_rows = pb;
        rs.border_nrows = grid;
        rs.border_ld = m + 1 <= 16 ? 16 : 32;
        return;
    }
    const int grid = vec_grid(n);
    rs.ensure(grid, 64);
    if (m + 1 <= 16)
        hipLaunchKernelGGL((k_hborder<16>), dim3(grid), dim3(kBlock), 0, s, n, V, m, wcol, H, ldh, rs.partial.get(),
                           rs.counter.get());
    else if (m + 1 <= 32)
        hipLaunchKernelGGL((k_hborder<32>), dim3(grid), dim3(kBlock), 0, s, n, V, m, wcol, H, ldh, rs.partial.get(),
                           rs.counter.get());
    else
        hipLaunchKernelGGL((k_hborder<64>), dim3(grid), dim3(kBlock), 0, s, n, V, m, wcol, H, ldh, rs.partial.get(),
                           rs.counter.get());
    LAP_HIP(hipGetLastError());
}

void jd_rr(int m, double *H, int ldh, double *theta, double *Y, int ldy, JDStatus *st, hipStream_t s,
           int mprev, const ReduceScratch *border, bool wide) {
    const double *bpart = border ? border->border_rows : nullptr;
    LAP_REQUIRE(!bpart || m <= kDeferBorderMax, LAP_EDEVICE, "border partial rows for too large an H");
    LAP_REQUIRE(!bpart || !wide, LAP_EDEVICE, "border partial rows are folded by the one-wavefront launch only");
    LAP_REQUIRE(m >= 1 && m <= kRRMax, LAP_EUNSUPPORTED, "projected matrix larger than 96");
    const int me = (m + 1) & ~1;
    const size_t lds = 2 * (size_t)me * me * sizeof(double);
    static bool attr_set = false;
    if (!attr_set) {
        LAP_HIP(hipFuncSetAttribute((const void *)k_rr_eig, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    2 * kRRMax * kRRMax * (int)sizeof(double)));
        attr_set = true;
    }
    // up to 32 columns a single wavefront does it (every barrier of the
    // round-by-round rotations is then nearly free), above it kRRThreads
    const int threads = me <= 32 && !wide ? kWave : kRRThreads;
    hipLaunchKernelGGL(k_rr_eig, dim3(1), dim3(threads), lds, s, m, H, ldh, theta, Y, ldy, mprev, st, bpart,
                       bpart ? border->border_nrows : 0, bpart ? border->border_ld : 0);
    LAP_HIP(hipGetLastError());
}

template <typename T>
void jd_ritz(int n, const double *V, const double *W, int m, const double *Y, const double *theta, double *u,
             double *r, T *Q, int ldq, int qcol, ReduceScratch &rs, JDStatus *st, hipStream_t s, HostMirror *hm,
             unsigned seq) {
    const int grid = vec_grid(n);
    rs.ensure(grid, 2);
    hipLaunchKernelGGL((k_ritz<T>), dim3(grid), dim3(kBlock), 0, s, n, V, W, m, Y, theta, u, r, Q, ldq, qcol,
                       rs.partial.get(), rs.counter.get(), st, hm, seq);
    LAP_HIP(hipGetLastError());
}
template void jd_ritz<float>(int, const double *, const double *, int, const double *, const double *, double *,
                             double *, float *, int, int, ReduceScratch &, JDStatus *, hipStream_t, HostMirror *, unsigned);
template void jd_ritz<double>(int, const double *, const double *, int, const double *, const double *, double *,
                              double *, double *, int, int, ReduceScratch &, JDStatus *, hipStream_t, HostMirror *, unsigned);

void jd_certify(const lap_plan &P, const double *u, double *gu, ReduceScratch &rs, JDStatus *st, hipStream_t s,
                HostMirror *hm, unsigned seq) {
    const int grid = row_grid(P.g, 4 * device_cu_count());
    rs.ensure(std::max(grid, vec_grid(P.n)), 2);
    if (P.weighted)
        hipLaunchKernelGGL((k_cert1<true>), dim3(grid), dim3(kBlock), 0, s, P.g, P.weights<double>(), u, gu,
                           rs.partial.get(), rs.counter.get(), st);
    else
        hipLaunchKernelGGL((k_cert1<false>), dim3(grid), dim3(kBlock), 0, s, P.g, P.weights<double>(), u, gu,
                           rs.partial.get(), rs.counter.get(), st);
    hipLaunchKernelGGL(k_cert2, dim3(vec_grid(P.n)), dim3(kBlock), 0, s, P.n, u, gu, rs.partial.get(),
                       rs.counter.get(), st, hm, seq);
    LAP_HIP(hipGetLastError());
}

void jd_rotate(int n, int m, const double *Y, int ldy, const double *vin, double *vout, int vc0, int vnc,
               const double *vscale0, const double *win, double *wout, int wc0, int wnc, hipStream_t s) {
    RotJob a{vin, vout, vc0, vnc, vscale0};
    RotJob b{win, wout, wc0, wnc, nullptr};
    const int grid = vec_grid(n);
    if (m <= 16)
        hipLaunchKernelGGL((k_rotate<16>), dim3(grid), dim3(kBlock), 0, s, n, m, Y, ldy, a, b);
    else if (m <= 32)
        hipLaunchKernelGGL((k_rotate<32>), dim3(grid), dim3(kBlock), 0, s, n, m, Y, ldy, a, b);
    else if (m <= 64)
        hipLaunchKernelGGL((k_rotate<64>), dim3(grid), dim3(kBlock), 0, s, n, m, Y, ldy, a, b);
    else
        throw Failure{LAP_EUNSUPPORTED, "rotation of more than 64 columns"};
    LAP_HIP(hipGetLastError());
}

void jd_hdiag(double *H, int ldh, int cnt, const double *theta, int off, hipStream_t s) {
    hipLaunchKernelGGL(k_hdiag, dim3(1), dim3(kBlock), 0, s, H, ldh, cnt, theta, off);
    LAP_HIP(hipGetLastError());
}

template <typename T>
void jd_zero_space(int n, int nz, const int *comp, const double *inv_sqrt_size, double *B, T *Q, int ldq,
                   hipStream_t s) {
    hipLaunchKernelGGL((k_zero_space<T>), dim3(vec_grid(n)), dim3(kBlock), 0, s, n, nz, comp, inv_sqrt_size, B,
                       Q, ldq);
    LAP_HIP(hipGetLastError());
}
template void jd_zero_space<float>(int, int, const int *, const double *, double *, float *, int, hipStream_t);
template void jd_zero_space<double>(int, int, const int *, const double *, double *, double *, int, hipStream_t);

void jd_scale_copy(int n, const double *v, double *out, JDStatus *st, const ReduceScratch &rs, hipStream_t s) {
    LAP_REQUIRE(rs.norm_rows != nullptr, LAP_EDEVICE, "scaling without an orthogonalized vector");
    hipLaunchKernelGGL(k_scale_copy, dim3(vec_grid(n)), dim3(kBlock), 0, s, rs.norm_rows, rs.norm_nrows, st, n, v,
                       out);
    LAP_HIP(hipGetLastError());
}

void jd_random(int n, uint64_t seed, long long colidx, const int *iperm, double *v, hipStream_t s) {
    hipLaunchKernelGGL(k_random, dim3(vec_grid(n)), dim3(kBlock), 0, s, n, (unsigned long long)seed, colidx,
                       iperm, v);
    LAP_HIP(hipGetLastError());
}

// Row chunks of the output launches: at least 2048 rows, at most 256 chunks.
int final_chunks(int n) {
    int c = (n + 2047) / 2048;
    return c < 1 ? 1 : (c > 256 ? 256 : c);
}

void jd_finalize(int n, int nconv, const double *X, long long sr, long long sc, const int *order_dev,
                 const int *perm_dev, double *out_dev, double *part, hipStream_t s) {
    if (nconv <= 0) return;
    const int nch = final_chunks(n);
    const int rows_per = (n + nch - 1) / nch;
    hipLaunchKernelGGL(k_final_max, dim3(nch, nconv), dim3(kBlock), 0, s, n, rows_per, X, sr, sc, order_dev,
                       perm_dev, part);
    hipLaunchKernelGGL(k_final_write, dim3(nch, nconv), dim3(kBlock), 0, s, n, rows_per, X, sr, sc, order_dev,
                       perm_dev, part, out_dev);
    LAP_HIP(hipGetLastError());
}

}  // namespace lapeig
