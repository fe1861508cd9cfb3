// The FSAI preconditioner: the factorized sparse approximate inverse of
// Kolotilina and Yeremin, the kind of "approximate inverse preconditioner"
// that the paper's Conclusion proposes for parallel machines, applied as a
// product of sparse matrices instead of IC(0)'s sequential triangular
// solves.  P = Z'Z ~ S^{-1} with S = G + tau D and Z lower triangular in the
// plan's vertex order (decreasing degree): row v of Z lives on
// P_v = {u in N(v) : u < v} and v itself, and solves the local system
//     S[P_v, P_v] g = e_v,   Z[v, P_v] = g / sqrt(g_v).
// With S[P_v, P_v] = R R' (Cholesky) and v the last index of P_v, that row
// is the last column of R^{-T}: z = R^{-T} e_last (since g = R^{-T} R^{-1}
// e_last = R^{-T} e_last / R_last,last and g_v = 1 / R_last,last^2).  tau
// (1e-8) keeps every local system definite when P_v is a whole connected
// component; a vertex without edges gets Z_vv = 1.
//
// In plan order the lower neighbours of v are those of higher degree, so
// |P_v| stays small even for hub rows (at most 76 on the 1.03M-vertex
// collaboration graph, 5.7 on average).  The factor is built once per plan
// on the host, rows split across threads, and uploaded in FP64 and FP32;
// every application runs on the device (pcg.hip).
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "lapeig_internal.h"

namespace lapeig {

namespace {

// weight of edge (a, b) in the plan-order CSR (0 when absent)
inline double edge_weight(const std::vector<int> &rp, const std::vector<int> &cl, const std::vector<double> &w,
                          bool weighted, int a, int b) {
    auto first = cl.begin() + rp[a], last = cl.begin() + rp[a + 1];
    auto it = std::lower_bound(first, last, b);
    if (it == last || *it != b) return 0.0;
    return weighted ? w[it - cl.begin()] : 1.0;
}

struct RowScratch {
    std::vector<double> R, z;
    std::vector<int> Pv;
};

// Row v of Z into zrow (|P_v| values, P_v ascending, v last).  Returns false
// when a local pivot is not positive (then a Jacobi row is written).
bool fsai_row(const lap_plan &P, const std::vector<double> &deg, int v, double tau, RowScratch &sc, double *zrow) {
    const auto &rp = P.h_rowptr;
    const auto &cl = P.h_col;
    const auto &w = P.h_w;
    sc.Pv.clear();
    for (int e = rp[v]; e < rp[v + 1] && cl[e] < v; ++e) sc.Pv.push_back(cl[e]);
    sc.Pv.push_back(v);
    const int m = (int)sc.Pv.size();
    if (deg[v] <= 0.0) {  // an isolated vertex
        zrow[m - 1] = 1.0;
        return true;
    }
    sc.R.assign((size_t)m * m, 0.0);
    double *R = sc.R.data();  // lower triangle, column-major
    for (int b = 0; b < m; ++b)
        for (int a = b; a < m; ++a)
            R[a + (size_t)b * m] = a == b ? (1.0 + tau) * deg[sc.Pv[a]]
                                          : -edge_weight(rp, cl, w, P.weighted, sc.Pv[a], sc.Pv[b]);
    // Cholesky, left-looking by columns
    for (int j = 0; j < m; ++j) {
        for (int k = 0; k < j; ++k) {
            const double rjk = R[j + (size_t)k * m];
            for (int a = j; a < m; ++a) R[a + (size_t)j * m] -= R[a + (size_t)k * m] * rjk;
        }
        const double d = R[j + (size_t)j * m];
        if (!(d > 0.0)) {
            for (int a = 0; a < m; ++a) zrow[a] = 0.0;
            zrow[m - 1] = 1.0 / std::sqrt(deg[v]);
            return false;
        }
        const double sd = std::sqrt(d);
        R[j + (size_t)j * m] = sd;
        for (int a = j + 1; a < m; ++a) R[a + (size_t)j * m] /= sd;
    }
    // z = R^{-T} e_{m-1}:  R' z = e_last, back substitution
    for (int i = m - 1; i >= 0; --i) {
        double s = i == m - 1 ? 1.0 : 0.0;
        for (int k = i + 1; k < m; ++k) s -= R[k + (size_t)i * m] * zrow[k];
        zrow[i] = s / R[i + (size_t)i * m];
    }
    return true;
}

}  // namespace

void fsai_ensure(lap_plan *P) {
    if (P->fsai_ready) return;
    const int n = P->n;
    const auto &rp = P->h_rowptr;
    const auto &cl = P->h_col;
    const size_t nnz = cl.size();
    std::vector<double> deg(n);
    for (int v = 0; v < n; ++v) {
        double d = 0.0;
        if (P->weighted) for (int e = rp[v]; e < rp[v + 1]; ++e) d += P->h_w[e];
        else d = rp[v + 1] - rp[v];
        deg[v] = d;
    }
    std::vector<int> mid(n);
    for (int v = 0; v < n; ++v)
        mid[v] = (int)(std::lower_bound(cl.begin() + rp[v], cl.begin() + rp[v + 1], v) - cl.begin());
    std::vector<double> zv(std::max<size_t>(nnz, 1), 0.0), zd(n, 0.0);
    const double tau = kFsaiTau;
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 20000) nt = 1;
    std::vector<int> maxrow(nt, 0), bad(nt, 0);
    auto work = [&](unsigned t) {
        RowScratch sc;
        std::vector<double> zrow;
        for (int v = (int)t; v < n; v += (int)nt) {
            const int m = mid[v] - rp[v] + 1;
            zrow.assign(m, 0.0);
            if (!fsai_row(*P, deg, v, tau, sc, zrow.data())) ++bad[t];
            maxrow[t] = std::max(maxrow[t], m);
            for (int a = 0; a < m - 1; ++a) zv[rp[v] + a] = zrow[a];  // row v of Z, lower part of row v
            zd[v] = zrow[m - 1];
        }
    };
    if (nt == 1) {
        work(0);
    } else {
        std::vector<std::thread> pool;
        for (unsigned t = 0; t < nt; ++t) pool.emplace_back(work, t);
        for (auto &th : pool) th.join();
    }
    // the transposed entries: Z(v, u) for u < v also sits in row u's upper part
    auto place = [&](unsigned t) {
        for (int u = (int)t; u < n; u += (int)nt)
            for (int e = mid[u]; e < rp[u + 1]; ++e) {
                const int v = cl[e];
                const int f = (int)(std::lower_bound(cl.begin() + rp[v], cl.begin() + mid[v], u) - cl.begin());
                zv[e] = zv[f];
            }
    };
    if (nt == 1) {
        place(0);
    } else {
        std::vector<std::thread> pool;
        for (unsigned t = 0; t < nt; ++t) pool.emplace_back(place, t);
        for (auto &th : pool) th.join();
    }
    int mr = 0;
    for (unsigned t = 0; t < nt; ++t) mr = std::max(mr, maxrow[t]);
    auto up = [](auto &buf, const auto &h) {
        using E = typename std::decay_t<decltype(h)>::value_type;
        buf.alloc(h.size());
        LAP_HIP(hipMemcpy(buf.get(), h.data(), sizeof(E) * h.size(), hipMemcpyHostToDevice));
    };
    up(P->d_fsai_mid, mid);
    up(P->d_fsai_zv64, zv);
    up(P->d_fsai_zd64, zd);
    std::vector<float> zv32(zv.begin(), zv.end()), zd32(zd.begin(), zd.end());
    up(P->d_fsai_zv32, zv32);
    up(P->d_fsai_zd32, zd32);
    P->fsai_tau = tau;
    P->fsai_max_row = mr;
    P->fsai_ready = true;
}

}  // namespace lapeig
