// Plan creation: host-side validation of the Laplacian, degree renumbering,
// row classification, sliced layout, connected components, and upload.
#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <numeric>

#include "lapeig_internal.h"

namespace lapeig {

namespace {

std::string row_msg(const char *what, long long row) {
    return std::string(what) + " (row " + std::to_string(row) + ")";
}

}  // namespace

// Section 2: G = D - A with A the weighted adjacency of a simple undirected
// graph with positive weights and D the generalized degrees.  Everything is
// checked before the first HIP call.
void validate_laplacian(const lap_csr *L) {
    LAP_REQUIRE(L != nullptr, LAP_EINVAL, "lap_csr is NULL");
    LAP_REQUIRE(L->n >= 1, LAP_EINVAL, "n must be >= 1");
    LAP_REQUIRE(L->nnz >= 0, LAP_EINVAL, "nnz must be >= 0");
    LAP_REQUIRE(L->rowptr && (L->nnz == 0 || (L->col && L->val)), LAP_EINVAL,
                "rowptr/col/val must be non-NULL");
    const int n = L->n;
    const int32_t *rp = L->rowptr, *cl = L->col;
    const double *v = L->val;
    LAP_REQUIRE(rp[0] == 0, LAP_ENOTLAPLACIAN, "rowptr[0] must be 0");
    LAP_REQUIRE(rp[n] == L->nnz, LAP_ENOTLAPLACIAN, "rowptr[n] must equal nnz");
    bool integral = true;
    for (int i = 0; i < n; ++i) {
        LAP_REQUIRE(rp[i + 1] >= rp[i], LAP_ENOTLAPLACIAN, row_msg("rowptr decreases", i));
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            LAP_REQUIRE(cl[p] >= 0 && cl[p] < n, LAP_ENOTLAPLACIAN, row_msg("column out of range", i));
            LAP_REQUIRE(p == rp[i] || cl[p] > cl[p - 1], LAP_ENOTLAPLACIAN,
                        row_msg("columns not strictly increasing (unsorted or duplicate)", i));
            LAP_REQUIRE(std::isfinite(v[p]), LAP_ENOTLAPLACIAN, row_msg("non-finite value", i));
            if (cl[p] != i)
                LAP_REQUIRE(v[p] < 0.0, LAP_ENOTLAPLACIAN,
                            row_msg("off-diagonal value must be negative (a positive edge weight)", i));
            if (v[p] != std::floor(v[p])) integral = false;
        }
    }
    for (int i = 0; i < n; ++i) {
        double off = 0.0, diag = 0.0, mag = 0.0;
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            int j = cl[p];
            if (j == i) { diag = v[p]; continue; }
            off += v[p];
            mag += std::fabs(v[p]);
            // symmetric pattern and values: find (j, i)
            const int32_t *b = cl + rp[j], *e = cl + rp[j + 1];
            const int32_t *f = std::lower_bound(b, e, i);
            LAP_REQUIRE(f != e && *f == i, LAP_ENOTLAPLACIAN, row_msg("pattern not symmetric", i));
            LAP_REQUIRE(v[f - cl] == v[p], LAP_ENOTLAPLACIAN, row_msg("values not symmetric", i));
        }
        if (integral) {
            LAP_REQUIRE(diag == -off, LAP_ENOTLAPLACIAN,
                        row_msg("diagonal is not minus the sum of the off-diagonal values", i));
        } else {
            LAP_REQUIRE(std::fabs(diag + off) <= 1e-12 * std::max(mag, 1e-300) || (mag == 0.0 && diag == 0.0),
                        LAP_ENOTLAPLACIAN,
                        row_msg("diagonal is not minus the sum of the off-diagonal values", i));
        }
    }
}

namespace {

template <typename T>
void upload(DevBuf<T> &dst, const std::vector<T> &src) {
    dst.alloc(src.size());
    if (!src.empty())
        LAP_HIP(hipMemcpy(dst.get(), src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
}

}  // namespace

void build_plan(const lap_csr *L, hipStream_t stream, lap_plan *P, bool hub_order, int long_threshold,
                int huge_threshold) {
    validate_laplacian(L);
    const int n = L->n;
    const int32_t *rp = L->rowptr, *cl = L->col;
    const double *v = L->val;

    // degree (number of neighbours) and weightedness
    std::vector<int> deg(n);
    bool weighted = false;
    long long nnz_a = 0;
    for (int i = 0; i < n; ++i) {
        int d = 0;
        for (int p = rp[i]; p < rp[i + 1]; ++p)
            if (cl[p] != i) {
                ++d;
                if (v[p] != -1.0) weighted = true;
            }
        deg[i] = d;
        nnz_a += d;
    }
    LAP_REQUIRE(nnz_a < (1LL << 31) - 64LL * n, LAP_EUNSUPPORTED, "graph too large for int32 offsets");

    // Renumber by decreasing degree, so that every row class is a prefix.
    // Inside one degree, vertices with the same first neighbour in that order
    // (on power-law graphs nearly always their largest hub) are placed side by
    // side: a hub's neighbour list then falls into runs of consecutive
    // positions and the 64 lanes of a slice gather from fewer cache lines.
    // The key is formed twice, the second time against the refined order;
    // remaining ties go by the caller's index (all ties, without hub_order).
    std::vector<int> iperm(n), perm(n), first(n);
    std::iota(iperm.begin(), iperm.end(), 0);
    std::stable_sort(iperm.begin(), iperm.end(), [&](int a, int b) { return deg[a] > deg[b]; });
    for (int pass = 0; pass < (hub_order ? 2 : 0); ++pass) {
        for (int p = 0; p < n; ++p) perm[iperm[p]] = p;
        for (int i = 0; i < n; ++i) {
            int f = n;
            for (int e = rp[i]; e < rp[i + 1]; ++e)
                if (cl[e] != i) f = std::min(f, perm[cl[e]]);
            first[i] = f;
        }
        std::sort(iperm.begin(), iperm.end(), [&](int a, int b) {
            if (deg[a] != deg[b]) return deg[a] > deg[b];
            if (first[a] != first[b]) return first[a] < first[b];
            return a < b;
        });
    }
    for (int p = 0; p < n; ++p) perm[iperm[p]] = p;

    // CSR of A in plan order, columns ascending
    std::vector<int> prow(n + 1, 0);
    for (int p = 0; p < n; ++p) prow[p + 1] = prow[p] + deg[iperm[p]];
    std::vector<int> pcol(nnz_a);
    std::vector<double> pw(weighted ? nnz_a : 0);
    {
        std::vector<std::pair<int, double>> tmp;
        for (int p = 0; p < n; ++p) {
            int i = iperm[p];
            tmp.clear();
            for (int e = rp[i]; e < rp[i + 1]; ++e)
                if (cl[e] != i) tmp.emplace_back(perm[cl[e]], -v[e]);
            std::sort(tmp.begin(), tmp.end());
            for (size_t t = 0; t < tmp.size(); ++t) {
                pcol[prow[p] + t] = tmp[t].first;
                if (weighted) pw[prow[p] + t] = tmp[t].second;
            }
        }
    }
    // connected components (plan order), breadth-first
    std::vector<int> comp(n, -1), queue(n);
    int ncomp = 0;
    std::vector<int> csize;
    for (int s = 0; s < n; ++s) {
        if (comp[s] >= 0) continue;
        int head = 0, tail = 0;
        queue[tail++] = s;
        comp[s] = ncomp;
        while (head < tail) {
            int i = queue[head++];
            for (int e = prow[i]; e < prow[i + 1]; ++e)
                if (comp[pcol[e]] < 0) { comp[pcol[e]] = ncomp; queue[tail++] = pcol[e]; }
        }
        csize.push_back(tail);
        ++ncomp;
    }

    // Jacobi preconditioner D^{-1} (generalized degrees)
    std::vector<double> dinv(n);
    for (int p = 0; p < n; ++p) {
        double d = 0.0;
        if (weighted) for (int e = prow[p]; e < prow[p + 1]; ++e) d += pw[e];
        else d = prow[p + 1] - prow[p];
        dinv[p] = d > 0.0 ? 1.0 / d : 1.0;
    }

    // ---- first HIP calls
    LAP_HIP(hipGetDevice(&P->device));
    P->n = n;
    P->nnz_a = nnz_a;
    P->weighted = weighted;
    P->stream = stream;
    P->max_degree = n ? deg[iperm[0]] : 0;
    P->perm = perm;
    P->iperm = iperm;
    P->comp = comp;
    P->comp_size = csize;
    P->ncomp = ncomp;
    upload(P->d_perm, perm);
    upload(P->d_iperm, iperm);
    upload(P->d_comp, comp);
    upload(P->d_rowptr, prow);
    upload(P->d_col, pcol);
    upload(P->d_dinv64, dinv);
    std::vector<float> dinv32(dinv.begin(), dinv.end());
    upload(P->d_dinv32, dinv32);
    if (weighted) {
        upload(P->d_w64, pw);
        std::vector<float> pw32(pw.begin(), pw.end());
        upload(P->d_w32, pw32);
    }
    P->g.n = n;
    P->g.rowptr = P->d_rowptr.get();
    P->g.col = P->d_col.get();
    // the plan-order CSR stays on the host, so the row-class layout can be rebuilt
    P->h_rowptr = std::move(prow);
    P->h_col = std::move(pcol);
    P->h_w = std::move(pw);
    build_layout(P, long_threshold, huge_threshold);
}

// Row classes for the given thresholds (rows are in decreasing degree, so
// each class is a prefix): the 64-row column-major slices of the short rows
// and the kChunk-edge chunks of the long ones, uploaded to the device.
// Solver work areas captured with the old layout are dropped.
void build_layout(lap_plan *P, int long_threshold, int huge_threshold) {
    LAP_REQUIRE(long_threshold >= 1 && huge_threshold >= long_threshold, LAP_EINVAL,
                "row-class thresholds must satisfy 1 <= long <= huge");
    const int n = P->n;
    const bool weighted = P->weighted;
    const std::vector<int> &prow = P->h_rowptr, &pcol = P->h_col;
    const std::vector<double> &pw = P->h_w;
    auto deg = [&](int r) { return prow[r + 1] - prow[r]; };
    int n_long = 0, n_huge = 0;
    while (n_long < n && deg(n_long) > long_threshold) ++n_long;
    while (n_huge < n && deg(n_huge) > huge_threshold) ++n_huge;
    // The slices start at a multiple of 32 rows, so that a slice's 64 values
    // of any vector (FP32 or FP64) fill whole 128-byte lines: the up to 31
    // rows that this moves into the long class are summed a wavefront per row.
    n_long = std::min(n, (n_long + 31) & ~31);

    // 64-row column-major slices for rows [n_long, n)
    const int nslices = (n - n_long + kWave - 1) / kWave;
    std::vector<int> soff(nslices + 1, 0);
    for (int s = 0; s < nslices; ++s) soff[s + 1] = soff[s] + deg(n_long + s * kWave) * kWave;
    std::vector<int> scol(soff[nslices]);
    std::vector<double> sw(weighted ? soff[nslices] : 0);
    for (int s = 0; s < nslices; ++s) {
        const int r0 = n_long + s * kWave;
        const int width = (soff[s + 1] - soff[s]) / kWave;
        for (int l = 0; l < kWave; ++l) {
            const int r = r0 + l;
            const int d = r < n ? deg(r) : 0;
            for (int t = 0; t < width; ++t) {
                const size_t at = (size_t)soff[s] + (size_t)t * kWave + l;
                if (t < d) {
                    scol[at] = pcol[prow[r] + t];
                    if (weighted) sw[at] = pw[prow[r] + t];
                } else {  // padding: the row itself contributes w (x_r - x_r) = 0
                    scol[at] = r < n ? r : n - 1;
                    if (weighted) sw[at] = 0.0;
                }
            }
        }
    }
    // long rows in chunks of kChunk edges (the block product splits them)
    std::vector<int> coff(n_long + 1, 0), crow;
    for (int r = 0; r < n_long; ++r) {
        const int nc = std::max(1, (deg(r) + kChunk - 1) / kChunk);  // a row of degree 0 still gets its chunk
        coff[r + 1] = coff[r] + nc;
        for (int c = 0; c < nc; ++c) crow.push_back(r);
    }

    P->jd_cache.reset();
    P->jdb_cache.reset();
    LAP_HIP(hipDeviceSynchronize());  // no launch may still read the old layout
    upload(P->d_sell_off, soff);
    upload(P->d_sell_col, scol);
    upload(P->d_chunk_off, coff);
    upload(P->d_chunk_row, crow);
    if (weighted) {
        upload(P->d_sellw64, sw);
        std::vector<float> sw32(sw.begin(), sw.end());
        upload(P->d_sellw32, sw32);
    }
    P->long_threshold = long_threshold;
    P->huge_threshold = huge_threshold;
    P->g.n_huge = n_huge;
    P->g.n_long = n_long;
    P->g.nslices = nslices;
    // When the grid holds only a few units per SIMD, the widest slices would
    // finish last; their rows are then visited eight lanes per row.  Larger
    // graphs stride many units through every wavefront, which evens the load.
    int mid = 0;
    if ((long long)(n_long - n_huge) + nslices <= 16LL * device_cu_count())
        while (mid < nslices && soff[mid + 1] - soff[mid] > kMidWidth * kWave) ++mid;  // widest slices lead
    P->g.nslices_mid = mid;
    P->g.sell_off = P->d_sell_off.get();
    P->g.sell_col = P->d_sell_col.get();
    P->g.nchunks = (int)crow.size();
    int n_multi = 0;  // rows in decreasing degree: the chunked ones lead
    while (n_multi < n_long && deg(n_multi) > kChunk) ++n_multi;
    P->g.n_multi = n_multi;
    P->g.chunk_row = P->d_chunk_row.get();
    P->g.chunk_off = P->d_chunk_off.get();
    // partial sums of chunked rows for block products of up to 64 double columns
    P->chunk_part.alloc(std::max<size_t>(crow.size(), 1) * 64 * sizeof(double));
}

bool fault_enabled(const char *name) {
    const char *v = std::getenv("LAPEIG_FAULT");
    if (!v) return false;
    const std::string all(v), want(name);
    size_t pos = 0;
    while (pos <= all.size()) {
        const size_t end = std::min(all.find(',', pos), all.size());
        if (all.compare(pos, end - pos, want) == 0) return true;
        pos = end + 1;
    }
    return false;
}

double fault_breakdown_shift(const lap_plan &P) {
    double dmax = 0.0;
    for (int i = 0; i < P.n; ++i) {
        double d = 0.0;
        for (int e = P.h_rowptr[i]; e < P.h_rowptr[i + 1]; ++e) d += P.h_w.empty() ? 1.0 : P.h_w[e];
        dmax = std::max(dmax, d);
    }
    return 4.0 * dmax + 1.0;  // above 2 max_i d_i >= lambda_max (Gershgorin)
}

int device_cu_count() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

}  // namespace lapeig
