/*
 * lapeig_oracle.c -- plain FP64 CPU oracle for the smallest eigenpairs of a
 * graph Laplacian G = D - A by the Jacobi-Davidson method.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this file.  The GPU library
 * never links it and shares no code, header or table with it.
 *
 * Everything here is deliberately plain: serial loops in double precision,
 * no blocking, no fusion, no reordering of the paper's steps, so that each
 * function can be read against the passage it cites:
 *
 *   orc_spmv            y = G x, with G = D - A as defined in Section 2
 *   orc_quadform        x'Gx = 1/2 sum_ij A_ij (x_i - x_j)^2, eq. (1)
 *   orc_components      connected components; the multiplicity of the
 *                       zero eigenvalue equals their number (Section 2)
 *   orc_dense_eig       cyclic Jacobi for small symmetric matrices: the
 *                       projected matrix H of Algorithm 2 step 5 and the
 *                       brute-force spectrum of tiny graphs
 *   orc_mgs             modified Gram-Schmidt, Algorithm 2 step 2
 *   orc_ic0_*           incomplete Cholesky with no fill-in, the
 *                       preconditioner of Section 4
 *   orc_fsai_*          factorized sparse approximate inverse, the
 *                       approximate-inverse preconditioner that the
 *                       Conclusion proposes for parallel machines
 *   orc_pcg_correction  PCG on the projected correction equation,
 *                       Algorithm 2 step 8 with M = (I-QQ')P(I-QQ')
 *                       (comments on Algorithm 2; eq. JDsismorethanone)
 *   orc_jd              Algorithm 2 with deflation against converged
 *                       vectors and the m_min/m_max restart (Section 3.2)
 *   orc_start_value     SplitMix64 counter-based start vectors
 *   orc_dacg            Algorithm 3: DACG, the eigenpairs one by one by a
 *                       deflated preconditioned nonlinear CG on the
 *                       Rayleigh quotient (Section 3.3)
 *
 * Readings of points the paper leaves open are marked READING in the code.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))

typedef struct {
    int n;
    const int *rowptr; /* n+1 */
    const int *col;    /* nnz, sorted per row, diagonal included */
    const double *val; /* nnz: G's entries */
} orc_lap;

/* ------------------------------------------------------------------ */
/* Small vector helpers (plain loops)                                  */
/* ------------------------------------------------------------------ */

static double dot(int n, const double *a, const double *b) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static double nrm2(int n, const double *a) { return sqrt(dot(n, a, a)); }

static void axpy(int n, double alpha, const double *x, double *y) {
    for (int i = 0; i < n; ++i) y[i] += alpha * x[i];
}

static void scal(int n, double alpha, double *x) {
    for (int i = 0; i < n; ++i) x[i] *= alpha;
}

/* ------------------------------------------------------------------ */
/* Laplacian products (Section 2)                                      */
/* ------------------------------------------------------------------ */

/* y = G x, straight from the stored entries of G. */
ORC_API void orc_spmv(int n, const int *rowptr, const int *col, const double *val,
                      const double *x, double *y) {
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) s += val[p] * x[col[p]];
        y[i] = s;
    }
}

static void lap_apply(const orc_lap *L, const double *x, double *y) {
    orc_spmv(L->n, L->rowptr, L->col, L->val, x, y);
}

/* eq. (1): x'Gx = 1/2 sum_{i,j} A_ij (x_i - x_j)^2, where A_ij = -G_ij
 * off the diagonal.  Summing over both orientations of every edge and
 * halving is the formula as written. */
ORC_API double orc_quadform(int n, const int *rowptr, const int *col, const double *val,
                            const double *x) {
    double s = 0.0;
    for (int i = 0; i < n; ++i)
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int j = col[p];
            if (j == i) continue;
            double d = x[i] - x[j];
            s += (-val[p]) * d * d;
        }
    return 0.5 * s;
}

/* Connected components by breadth-first search.  label[i] in [0, ncomp),
 * numbered in order of their smallest vertex.  Returns ncomp. */
ORC_API int orc_components(int n, const int *rowptr, const int *col, int *label) {
    int *queue = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) label[i] = -1;
    int ncomp = 0;
    for (int s = 0; s < n; ++s) {
        if (label[s] >= 0) continue;
        int head = 0, tail = 0;
        queue[tail++] = s;
        label[s] = ncomp;
        while (head < tail) {
            int i = queue[head++];
            for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
                int j = col[p];
                if (label[j] < 0) { label[j] = ncomp; queue[tail++] = j; }
            }
        }
        ++ncomp;
    }
    free(queue);
    return ncomp;
}

/* ------------------------------------------------------------------ */
/* Dense symmetric eigenproblem: cyclic Jacobi (Golub & Van Loan,      */
/* "Matrix Computations", the symmetric Schur 2x2 step swept over all  */
/* off-diagonal pairs).  Used for H in Algorithm 2 step 5 ("eigensolution*/
/* of the usually very small matrix H") and for brute force on tiny    */
/* graphs.                                                             */
/* ------------------------------------------------------------------ */

/* A: n x n row-major symmetric, overwritten.  evals ascending; evecs n x n
 * column-major (evecs[i + j*n] = component i of eigenvector j).  Returns
 * the number of sweeps, or -1 when it did not converge. */
ORC_API int orc_dense_eig(int n, double *A, double *evals, double *evecs) {
    double *Vm = (double *)calloc((size_t)n * n, sizeof(double));
    for (int i = 0; i < n; ++i) Vm[i * n + i] = 1.0; /* row-major accumulator */
    double fro = 0.0;
    for (int i = 0; i < n * n; ++i) fro += A[i] * A[i];
    fro = sqrt(fro);
    double tol = 1e-3 * 2.220446049250313e-16 * fro;
    int sweep, ok = 0;
    for (sweep = 0; sweep < 100; ++sweep) {
        int rotated = 0;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (fabs(apq) <= tol) continue;
                rotated = 1;
                double app = A[p * n + p], aqq = A[q * n + q];
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                /* A <- J' A J with J the rotation in the (p, q) plane */
                for (int k = 0; k < n; ++k) {
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                A[p * n + q] = 0.0;
                A[q * n + p] = 0.0;
                for (int k = 0; k < n; ++k) {
                    double vkp = Vm[k * n + p], vkq = Vm[k * n + q];
                    Vm[k * n + p] = c * vkp - s * vkq;
                    Vm[k * n + q] = s * vkp + c * vkq;
                }
            }
        if (!rotated) { ok = 1; break; }
    }
    /* selection sort ascending, carrying vectors */
    int *idx = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) idx[i] = i;
    for (int i = 0; i < n; ++i) {
        int best = i;
        for (int j = i + 1; j < n; ++j)
            if (A[idx[j] * n + idx[j]] < A[idx[best] * n + idx[best]]) best = j;
        int tmp = idx[i]; idx[i] = idx[best]; idx[best] = tmp;
    }
    for (int j = 0; j < n; ++j) {
        evals[j] = A[idx[j] * n + idx[j]];
        for (int i = 0; i < n; ++i) evecs[i + (size_t)j * n] = Vm[i * n + idx[j]];
    }
    free(idx);
    free(Vm);
    return ok ? sweep : -1;
}

/* ------------------------------------------------------------------ */
/* Algorithm 2 step 2: modified Gram-Schmidt of v against the q        */
/* orthonormal columns of Q (n x q column-major).  READING: one extra  */
/* pass when the norm drops below 1/sqrt(2) of its value before the    */
/* pass ("twice is enough").  Returns the final norm; v not normalized.*/
/* ------------------------------------------------------------------ */
ORC_API double orc_mgs(int n, int q, const double *Q, double *v) {
    for (int pass = 0; pass < 2; ++pass) {
        double before = nrm2(n, v);
        for (int j = 0; j < q; ++j) {
            const double *qj = Q + (size_t)j * n;
            axpy(n, -dot(n, qj, v), qj, v);
        }
        double after = nrm2(n, v);
        if (after >= before / sqrt(2.0)) return after;
    }
    return nrm2(n, v);
}

/* ------------------------------------------------------------------ */
/* IC(0): incomplete Cholesky with no fill-in (Section 4).  G ~ K K'   */
/* with K lower triangular on the pattern of G's lower triangle.       */
/* READING: a pivot below 1e-10 * G_ii is replaced by G_ii (1 for an   */
/* isolated vertex); the number of replacements is returned.           */
/* ------------------------------------------------------------------ */
typedef struct {
    int n;
    int *rowptr; /* row i: strictly-lower entries ascending, then the diagonal */
    int *col;
    double *val;
} orc_ic0;

ORC_API orc_ic0 *orc_ic0_create(int n, const int *rowptr, const int *col, const double *val,
                                int *nfloor_out) {
    orc_ic0 *K = (orc_ic0 *)calloc(1, sizeof(orc_ic0));
    K->n = n;
    K->rowptr = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    int cnt = 0;
    K->rowptr[0] = 0;
    for (int i = 0; i < n; ++i) {
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p)
            if (col[p] < i) ++cnt;
        ++cnt; /* diagonal */
        K->rowptr[i + 1] = cnt;
    }
    K->col = (int *)malloc(sizeof(int) * (size_t)(cnt > 0 ? cnt : 1));
    K->val = (double *)malloc(sizeof(double) * (size_t)(cnt > 0 ? cnt : 1));
    int *pos = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) pos[i] = -1;
    int nfloor = 0;
    for (int i = 0; i < n; ++i) {
        int w = K->rowptr[i];
        double gii = 0.0;
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            if (col[p] < i) { K->col[w] = col[p]; K->val[w] = val[p]; pos[col[p]] = w; ++w; }
            else if (col[p] == i) gii = val[p];
        }
        int dpos = w;
        K->col[dpos] = i;
        /* off-diagonal entries of row i, in ascending column order */
        for (int e = K->rowptr[i]; e < dpos; ++e) {
            int k = K->col[e];
            double s = K->val[e];
            /* subtract sum_{j<k} K_ij K_kj over the shared pattern */
            for (int f = K->rowptr[k]; f < K->rowptr[k + 1] - 1; ++f) {
                int j = K->col[f];
                if (pos[j] >= 0 && j < k) s -= K->val[pos[j]] * K->val[f];
            }
            K->val[e] = s / K->val[K->rowptr[k + 1] - 1];
        }
        double d = gii;
        for (int e = K->rowptr[i]; e < dpos; ++e) d -= K->val[e] * K->val[e];
        if (!(d >= 1e-10 * gii) || d <= 0.0) {
            d = gii > 0.0 ? gii : 1.0;
            ++nfloor;
        }
        K->val[dpos] = sqrt(d);
        for (int e = K->rowptr[i]; e < dpos; ++e) pos[K->col[e]] = -1;
    }
    free(pos);
    if (nfloor_out) *nfloor_out = nfloor;
    return K;
}

ORC_API void orc_ic0_destroy(orc_ic0 *K) {
    if (!K) return;
    free(K->rowptr); free(K->col); free(K->val); free(K);
}

/* z = (K K')^{-1} r: forward substitution with K, back substitution with K'. */
ORC_API void orc_ic0_apply(const orc_ic0 *K, const double *r, double *z) {
    int n = K->n;
    for (int i = 0; i < n; ++i) {
        double s = r[i];
        int d = K->rowptr[i + 1] - 1;
        for (int e = K->rowptr[i]; e < d; ++e) s -= K->val[e] * z[K->col[e]];
        z[i] = s / K->val[d];
    }
    for (int i = n - 1; i >= 0; --i) {
        int d = K->rowptr[i + 1] - 1;
        z[i] /= K->val[d];
        for (int e = K->rowptr[i]; e < d; ++e) z[K->col[e]] -= K->val[e] * z[i];
    }
}

/* ------------------------------------------------------------------ */
/* FSAI, the factorized sparse approximate inverse of Kolotilina and   */
/* Yeremin (as reviewed by Benzi): the "approximate inverse            */
/* preconditioner" that the Conclusion proposes, applied as a product  */
/* of sparse matrices.  P = Z'Z ~ S^{-1}, Z lower triangular in a      */
/* vertex order (pos[v] = position of vertex v; NULL = natural order). */
/* Row v of Z lives on P_v = {v} and the neighbours u of v with        */
/* pos[u] < pos[v]; its values solve the local system                  */
/*     S[P_v, P_v] g = e_v,   Z[v, P_v] = g / sqrt(g_v),               */
/* with S = G + tau D, so that (Z S Z')_vv = 1 and (Z S)_vu = 0 for    */
/* u in P_v, u != v.                                                   */
/* READING: tau (1e-8 in the solvers) keeps every local system         */
/* definite when P_v is a whole connected component (G alone is        */
/* singular there); a vertex with no edge gets Z_vv = 1.               */
/* ------------------------------------------------------------------ */
typedef struct {
    int n;
    int *rowptr; /* row v of Z (vertex index), entries in ascending column */
    int *col;
    double *val;
} orc_fsai;

/* G(a, b) from the CSR (columns sorted): binary search in row a. */
static double lap_entry(int n, const int *rowptr, const int *col, const double *val, int a, int b) {
    (void)n;
    int lo = rowptr[a], hi = rowptr[a + 1] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (col[mid] == b) return val[mid];
        if (col[mid] < b) lo = mid + 1; else hi = mid - 1;
    }
    return 0.0;
}

/* Solve the symmetric positive definite m x m system A g = b in place
 * (A column-major, overwritten by its Cholesky factor; b by g).
 * Returns 0, or -1 if a pivot is not positive. */
static int dense_spd_solve(int m, double *A, double *b) {
    for (int j = 0; j < m; ++j) {
        double d = A[j + (size_t)j * m];
        for (int k = 0; k < j; ++k) d -= A[j + (size_t)k * m] * A[j + (size_t)k * m];
        if (!(d > 0.0)) return -1;
        d = sqrt(d);
        A[j + (size_t)j * m] = d;
        for (int i = j + 1; i < m; ++i) {
            double s = A[i + (size_t)j * m];
            for (int k = 0; k < j; ++k) s -= A[i + (size_t)k * m] * A[j + (size_t)k * m];
            A[i + (size_t)j * m] = s / d;
        }
    }
    for (int i = 0; i < m; ++i) { /* L y = b */
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= A[i + (size_t)k * m] * b[k];
        b[i] = s / A[i + (size_t)i * m];
    }
    for (int i = m - 1; i >= 0; --i) { /* L' g = y */
        double s = b[i];
        for (int k = i + 1; k < m; ++k) s -= A[k + (size_t)i * m] * b[k];
        b[i] = s / A[i + (size_t)i * m];
    }
    return 0;
}

ORC_API orc_fsai *orc_fsai_create(int n, const int *rowptr, const int *col, const double *val,
                                  const int *pos, double tau) {
    orc_fsai *Z = (orc_fsai *)calloc(1, sizeof(orc_fsai));
    Z->n = n;
    Z->rowptr = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    Z->rowptr[0] = 0;
    int cnt = 0;
    for (int v = 0; v < n; ++v) {
        int pv = pos ? pos[v] : v;
        for (int p = rowptr[v]; p < rowptr[v + 1]; ++p) {
            int u = col[p];
            if (u != v && (pos ? pos[u] : u) < pv) ++cnt;
        }
        ++cnt; /* v itself */
        Z->rowptr[v + 1] = cnt;
    }
    Z->col = (int *)malloc(sizeof(int) * (size_t)cnt);
    Z->val = (double *)malloc(sizeof(double) * (size_t)cnt);
    for (int v = 0; v < n; ++v) {
        int pv = pos ? pos[v] : v;
        int w = Z->rowptr[v];
        /* P_v in ascending vertex index (the CSR columns are sorted) */
        for (int p = rowptr[v]; p < rowptr[v + 1]; ++p) {
            int u = col[p];
            if (u == v) { Z->col[w++] = v; continue; }
            if ((pos ? pos[u] : u) < pv) Z->col[w++] = u;
        }
        if (w == Z->rowptr[v]) Z->col[w++] = v; /* a row without its diagonal entry */
        int m = Z->rowptr[v + 1] - Z->rowptr[v];
        const int *P = Z->col + Z->rowptr[v];
        double *A = (double *)malloc(sizeof(double) * (size_t)m * m);
        double *g = (double *)malloc(sizeof(double) * (size_t)m);
        int iv = -1;
        for (int a = 0; a < m; ++a) {
            if (P[a] == v) iv = a;
            g[a] = 0.0;
            for (int b = 0; b < m; ++b) {
                double e = lap_entry(n, rowptr, col, val, P[a], P[b]);
                if (a == b) e *= 1.0 + tau; /* S = G + tau D on the diagonal */
                A[a + (size_t)b * m] = e;
            }
        }
        g[iv] = 1.0;
        double *Zv = Z->val + Z->rowptr[v];
        if (m == 1 && !(A[0] > 0.0)) {
            Zv[0] = 1.0; /* no edge: identity row */
        } else if (dense_spd_solve(m, A, g) == 0 && g[iv] > 0.0) {
            double sc = 1.0 / sqrt(g[iv]);
            for (int a = 0; a < m; ++a) Zv[a] = g[a] * sc;
        } else {
            /* not reached for tau > 0 on a Laplacian; keep a Jacobi row */
            for (int a = 0; a < m; ++a) Zv[a] = 0.0;
            double d = lap_entry(n, rowptr, col, val, v, v);
            Zv[iv] = d > 0.0 ? 1.0 / sqrt(d) : 1.0;
        }
        free(A);
        free(g);
    }
    return Z;
}

ORC_API void orc_fsai_destroy(orc_fsai *Z) {
    if (!Z) return;
    free(Z->rowptr); free(Z->col); free(Z->val); free(Z);
}

ORC_API int orc_fsai_nnz(const orc_fsai *Z) { return Z->rowptr[Z->n]; }

/* Z in CSR (rowptr n+1, col and val nnz), vertex indices. */
ORC_API void orc_fsai_export(const orc_fsai *Z, int *rowptr, int *col, double *val) {
    memcpy(rowptr, Z->rowptr, sizeof(int) * (size_t)(Z->n + 1));
    memcpy(col, Z->col, sizeof(int) * (size_t)Z->rowptr[Z->n]);
    memcpy(val, Z->val, sizeof(double) * (size_t)Z->rowptr[Z->n]);
}

/* z = Z'(Z r) */
ORC_API void orc_fsai_apply(const orc_fsai *Z, const double *r, double *z) {
    int n = Z->n;
    double *y = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int v = 0; v < n; ++v) {
        double s = 0.0;
        for (int e = Z->rowptr[v]; e < Z->rowptr[v + 1]; ++e) s += Z->val[e] * r[Z->col[e]];
        y[v] = s;
    }
    for (int i = 0; i < n; ++i) z[i] = 0.0;
    for (int v = 0; v < n; ++v)
        for (int e = Z->rowptr[v]; e < Z->rowptr[v + 1]; ++e) z[Z->col[e]] += Z->val[e] * y[v];
    free(y);
}

#define ORC_FSAI_TAU 1e-8

/* ------------------------------------------------------------------ */
/* Preconditioner P (Section 4 uses IC(0); the Jacobi choice D^{-1} is */
/* the one the GPU path applies by default; FSAI per the Conclusion).  */
/* ------------------------------------------------------------------ */
enum { ORC_PREC_NONE = 0, ORC_PREC_JACOBI = 1, ORC_PREC_IC0 = 2, ORC_PREC_FSAI = 3 };

typedef struct {
    int kind;
    const orc_ic0 *ic0;
    double *dinv;
    const orc_fsai *fsai;
} orc_prec;

static void prec_apply(const orc_prec *P, int n, const double *r, double *z) {
    if (P->kind == ORC_PREC_IC0) orc_ic0_apply(P->ic0, r, z);
    else if (P->kind == ORC_PREC_JACOBI) for (int i = 0; i < n; ++i) z[i] = P->dinv[i] * r[i];
    else if (P->kind == ORC_PREC_FSAI) orc_fsai_apply(P->fsai, r, z);
    else memcpy(z, r, sizeof(double) * (size_t)n);
}

static double *diag_inverse(const orc_lap *L) {
    double *d = (double *)malloc(sizeof(double) * (size_t)L->n);
    for (int i = 0; i < L->n; ++i) {
        double g = 0.0;
        for (int p = L->rowptr[i]; p < L->rowptr[i + 1]; ++p)
            if (L->col[p] == i) g = L->val[p];
        d[i] = g > 0.0 ? 1.0 / g : 1.0;
    }
    return d;
}

/* x <- (I - Q Q') x for Q with orthonormal columns (one classical pass). */
static void project_out(int n, int q, const double *Q, double *x) {
    for (int j = 0; j < q; ++j) {
        const double *qj = Q + (size_t)j * n;
        axpy(n, -dot(n, qj, x), qj, x);
    }
}

/* ------------------------------------------------------------------ */
/* Algorithm 2 step 8: solve                                           */
/*   (I-QQ')(G - theta I)(I-QQ') t = -r,   t orthogonal to Q,          */
/* by PCG with the projected preconditioner M = (I-QQ')P(I-QQ')        */
/* (comments on Algorithm 2).  Q = [x_1 .. x_{j-1} u] as in eq.        */
/* (JDsismorethanone).  READING: t_0 = 0; stop when the residual norm  */
/* is <= rtol * ||r||, after itmax iterations, or when p'Ap <= 0 (the  */
/* operator is indefinite; the last t is returned, or M(-r) if no step */
/* was taken).  Returns the number of operator applications (MVPs).    */
/* ------------------------------------------------------------------ */
static int pcg_correction(const orc_lap *L, double theta, int q, const double *Q,
                          const double *r, const orc_prec *P, int itmax, double rtol,
                          double *t, int *breakdown) {
    int n = L->n;
    double *res = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *s = (double *)malloc(sizeof(double) * (size_t)n);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
    for (int i = 0; i < n; ++i) { t[i] = 0.0; res[i] = -r[i]; }
    project_out(n, q, Q, res);
    /* z = M res = (I-QQ') P (I-QQ') res */
    memcpy(tmp, res, sizeof(double) * (size_t)n);
    project_out(n, q, Q, tmp);
    prec_apply(P, n, tmp, z);
    project_out(n, q, Q, z);
    memcpy(p, z, sizeof(double) * (size_t)n);
    double rho = dot(n, res, z);
    double r0 = nrm2(n, r);
    int it, mvp = 0;
    if (breakdown) *breakdown = 0;
    for (it = 1; it <= itmax; ++it) {
        /* s = (I-QQ')(G - theta I)(I-QQ') p */
        memcpy(tmp, p, sizeof(double) * (size_t)n);
        project_out(n, q, Q, tmp);
        lap_apply(L, tmp, s);
        axpy(n, -theta, tmp, s);
        project_out(n, q, Q, s);
        ++mvp;
        double pAp = dot(n, p, s);
        if (!(pAp > 0.0)) {
            if (breakdown) *breakdown = 1;
            if (it == 1) memcpy(t, z, sizeof(double) * (size_t)n);
            break;
        }
        double alpha = rho / pAp;
        axpy(n, alpha, p, t);
        axpy(n, -alpha, s, res);
        if (nrm2(n, res) <= rtol * r0) break;
        memcpy(tmp, res, sizeof(double) * (size_t)n);
        project_out(n, q, Q, tmp);
        prec_apply(P, n, tmp, z);
        project_out(n, q, Q, z);
        double rho_new = dot(n, res, z);
        double beta = rho_new / rho;
        rho = rho_new;
        for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    free(res); free(z); free(p); free(s); free(tmp);
    return mvp;
}

/* Public wrapper: precond 0 = none, 1 = Jacobi (D^{-1}), 2 = IC(0),
 * 3 = FSAI in the order pos (NULL: natural order).
 * Q: n x q column-major orthonormal; r, t: n.  Returns MVPs. */
ORC_API int orc_pcg_correction_ex(int n, const int *rowptr, const int *col, const double *val,
                                  double theta, int q, const double *Q, const double *r,
                                  int precond, const int *pos, int itmax, double rtol, double *t,
                                  int *breakdown) {
    orc_lap L = {n, rowptr, col, val};
    orc_prec P = {precond, NULL, NULL, NULL};
    int nfloor = 0;
    orc_ic0 *K = NULL;
    orc_fsai *Z = NULL;
    if (precond == ORC_PREC_IC0) { K = orc_ic0_create(n, rowptr, col, val, &nfloor); P.ic0 = K; }
    if (precond == ORC_PREC_JACOBI) P.dinv = diag_inverse(&L);
    if (precond == ORC_PREC_FSAI) { Z = orc_fsai_create(n, rowptr, col, val, pos, ORC_FSAI_TAU); P.fsai = Z; }
    int mvp = pcg_correction(&L, theta, q, Q, r, &P, itmax, rtol, t, breakdown);
    orc_ic0_destroy(K);
    orc_fsai_destroy(Z);
    free(P.dinv);
    return mvp;
}

ORC_API int orc_pcg_correction(int n, const int *rowptr, const int *col, const double *val,
                               double theta, int q, const double *Q, const double *r,
                               int precond, int itmax, double rtol, double *t,
                               int *breakdown) {
    return orc_pcg_correction_ex(n, rowptr, col, val, theta, q, Q, r, precond, NULL, itmax, rtol, t,
                                 breakdown);
}

/* ------------------------------------------------------------------ */
/* Start vectors: SplitMix64 (Steele, Lea & Flood 2014, as published   */
/* by Vigna), used counter-style: value i of the stream for `seed` is  */
/* the SplitMix64 output mix(seed + (i+1) * 0x9e3779b97f4a7c15),       */
/* mapped to [-1, 1) through its top 53 bits.                          */
/* ------------------------------------------------------------------ */
ORC_API double orc_start_value(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

/* ------------------------------------------------------------------ */
/* Algorithm 2 (Jacobi-Davidson) for the k smallest eigenpairs.        */
/* ------------------------------------------------------------------ */
typedef struct {
    int m_min, m_max;   /* restart sizes, Section 4: 5 and 10 */
    int itmax;          /* PCG iterations per correction, Section 4: 20 */
    double rtol_pcg;    /* delta_PCG, Section 4: 1e-2 */
    int kmax;           /* outer iteration limit; <= 0 means 1000 k */
    int precond;        /* ORC_PREC_*; Section 4 uses IC(0) */
    int criterion;      /* 0: ||r|| <= tol min(theta,1); 1: ||r|| < tol theta (Section 4) */
    uint64_t seed;      /* start-vector stream */
    const int *fsai_pos; /* vertex order of FSAI (NULL: natural order) */
} orc_jd_opts;

typedef struct {
    int nconv, ncomp, outer, inner, nfloor, status;
    long long mvp;
} orc_jd_info;

static int converged(double rnorm, double theta, double tol, int criterion) {
    if (criterion == 1) return rnorm < tol * theta;
    double scale = theta < 1.0 ? theta : 1.0;
    return rnorm <= tol * scale;
}

/* Columns cols[0..nc) of Vin * Y  ->  Vout (n x nc), Y m x m column-major. */
static void basis_times(int n, int m, const double *Vin, const double *Y, int c0, int nc,
                        double *Vout) {
    for (int j = 0; j < nc; ++j) {
        double *o = Vout + (size_t)j * n;
        for (int i = 0; i < n; ++i) o[i] = 0.0;
        for (int l = 0; l < m; ++l) axpy(n, Y[l + (size_t)(c0 + j) * m], Vin + (size_t)l * n, o);
    }
}

/* evals: k ascending; evecs: n x k column-major; res: k residual norms
 * ||G x - theta x|| (nullable).  Returns 0, or 1 when kmax was reached
 * (the first info->nconv pairs are then certified). */
ORC_API int orc_jd(int n, const int *rowptr, const int *col, const double *val, int k,
                   double tol, const orc_jd_opts *o, double *evals, double *evecs,
                   double *res, orc_jd_info *info) {
    orc_lap L = {n, rowptr, col, val};
    int m_min = o->m_min, m_max = o->m_max;
    int kmax = o->kmax > 0 ? o->kmax : 1000 * k;
    memset(info, 0, sizeof(*info));

    double *X = (double *)calloc((size_t)n * (size_t)(k + 1), sizeof(double));
    double *lam = (double *)calloc((size_t)(k + 1), sizeof(double));
    double *rlock = (double *)calloc((size_t)(k + 1), sizeof(double));
    int nx = 0;

    /* Zero eigenpairs (Section 2): G e_C = 0 for the indicator of every
     * connected component C, and the multiplicity of 0 is their number.
     * READING: k counts these pairs; they are locked before the iteration. */
    int *label = (int *)malloc(sizeof(int) * (size_t)n);
    int ncomp = orc_components(n, rowptr, col, label);
    info->ncomp = ncomp;
    for (int c = 0; c < ncomp && nx < k; ++c) {
        double *x = X + (size_t)nx * n;
        int cnt = 0;
        for (int i = 0; i < n; ++i) if (label[i] == c) ++cnt;
        for (int i = 0; i < n; ++i) x[i] = label[i] == c ? 1.0 / sqrt((double)cnt) : 0.0;
        lam[nx] = 0.0;
        double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
        lap_apply(&L, x, tmp);
        rlock[nx] = nrm2(n, tmp);
        free(tmp);
        ++nx;
    }
    free(label);

    orc_prec P = {o->precond, NULL, NULL, NULL};
    orc_ic0 *K = NULL;
    orc_fsai *Zf = NULL;
    if (o->precond == ORC_PREC_IC0) { K = orc_ic0_create(n, rowptr, col, val, &info->nfloor); P.ic0 = K; }
    if (o->precond == ORC_PREC_JACOBI) P.dinv = diag_inverse(&L);
    if (o->precond == ORC_PREC_FSAI) { Zf = orc_fsai_create(n, rowptr, col, val, o->fsai_pos, ORC_FSAI_TAU); P.fsai = Zf; }

    double *V = (double *)calloc((size_t)n * m_max, sizeof(double));
    double *W = (double *)calloc((size_t)n * m_max, sizeof(double));
    double *V2 = (double *)calloc((size_t)n * m_max, sizeof(double));
    double *W2 = (double *)calloc((size_t)n * m_max, sizeof(double));
    double *H = (double *)calloc((size_t)m_max * m_max, sizeof(double));
    double *Hs = (double *)calloc((size_t)m_max * m_max, sizeof(double));
    double *Theta = (double *)calloc((size_t)m_max, sizeof(double));
    double *Y = (double *)calloc((size_t)m_max * m_max, sizeof(double));
    double *v = (double *)calloc((size_t)n, sizeof(double));
    double *u = (double *)calloc((size_t)n, sizeof(double));
    double *r = (double *)calloc((size_t)n, sizeof(double));
    double *Lu = (double *)calloc((size_t)n, sizeof(double));
    double *t = (double *)calloc((size_t)n, sizeof(double));
    double *Q = (double *)calloc((size_t)n * (size_t)(k + 1), sizeof(double));
    int m = 0;
    uint64_t start_col = 0;
    int status = 1;
    int it = 0;

    /* "Choose unitary starting vector" (Algorithm 2).  READING: seeded
     * uniform entries; made unit length by step 2-3 of the first pass. */
    for (int i = 0; i < n; ++i) v[i] = orc_start_value(o->seed, start_col * (uint64_t)n + i);
    ++start_col;

    if (nx >= k) { status = 0; goto done; }

    while (it < kmax) {
        ++it;
        /* step 2: orthogonalize v against the converged vectors (READING: the
         * deflation of eq. JDsismorethanone keeps V orthogonal to them) and
         * against V by modified Gram-Schmidt; step 3: normalize. */
        double vn0 = nrm2(n, v);
        double vn = orc_mgs(n, nx, X, v);
        vn = orc_mgs(n, m, V, v);
        if (!(vn > 1e-12 * vn0)) {
            /* the correction lay in span[X V]: take a fresh start vector */
            for (int i = 0; i < n; ++i) v[i] = orc_start_value(o->seed, start_col * (uint64_t)n + i);
            ++start_col;
            orc_mgs(n, nx, X, v);
            vn = orc_mgs(n, m, V, v);
        }
        scal(n, 1.0 / vn, v);
        /* step 3: w = G v (one MVP) */
        double *vcol = V + (size_t)m * n, *wcol = W + (size_t)m * n;
        memcpy(vcol, v, sizeof(double) * (size_t)n);
        lap_apply(&L, vcol, wcol);
        info->mvp += 1;
        /* step 4: border H with V'w and v'w */
        for (int i = 0; i < m; ++i) {
            double h = dot(n, V + (size_t)i * n, wcol);
            H[i * m_max + m] = h;
            H[m * m_max + i] = h;
        }
        H[m * m_max + m] = dot(n, vcol, wcol);
        ++m;

        for (;;) {
            /* step 5: all eigenpairs of H, ascending (the smallest is used) */
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < m; ++j) Hs[i * m + j] = H[i * m_max + j];
            orc_dense_eig(m, Hs, Theta, Y);
            /* step 6: u = V y, r = G u - theta u with G u = W y */
            double theta = Theta[0];
            for (int i = 0; i < n; ++i) { u[i] = 0.0; r[i] = 0.0; }
            for (int l = 0; l < m; ++l) {
                axpy(n, Y[l], V + (size_t)l * n, u);
                axpy(n, Y[l], W + (size_t)l * n, r);
            }
            axpy(n, -theta, u, r);
            double rn = nrm2(n, r);
            /* step 7: exit test.  READING: a pair that passes on r = Wy - theta u
             * is certified with a fresh product G u and the Rayleigh quotient
             * of eq. (1) before it is accepted. */
            if (!converged(rn, theta, tol, o->criterion)) break;
            double un = nrm2(n, u);
            scal(n, 1.0 / un, u);
            lap_apply(&L, u, Lu);
            info->mvp += 1;
            double th = orc_quadform(n, rowptr, col, val, u);
            double rc = 0.0;
            for (int i = 0; i < n; ++i) { double d = Lu[i] - th * u[i]; rc += d * d; }
            rc = sqrt(rc);
            if (!converged(rc, th, tol, o->criterion)) break;
            /* lock (theta, u): deflation for the next eigenvalue, eq.
             * (JDsismorethanone).  READING: the remaining Ritz vectors are kept
             * as the new basis, H becomes their Ritz values. */
            memcpy(X + (size_t)nx * n, u, sizeof(double) * (size_t)n);
            lam[nx] = th;
            rlock[nx] = rc;
            ++nx;
            if (nx >= k) { status = 0; goto done; }
            basis_times(n, m, V, Y, 1, m - 1, V2);
            basis_times(n, m, W, Y, 1, m - 1, W2);
            { double *s = V; V = V2; V2 = s; s = W; W = W2; W2 = s; }
            --m;
            memset(H, 0, sizeof(double) * (size_t)m_max * m_max);
            for (int i = 0; i < m; ++i) H[i * m_max + i] = Theta[i + 1];
            if (m == 0) break;
        }
        if (m == 0) {
            for (int i = 0; i < n; ++i) v[i] = orc_start_value(o->seed, start_col * (uint64_t)n + i);
            ++start_col;
            continue;
        }
        double theta = Theta[0];
        /* restart: when H would outgrow m_max keep m_min columns.  READING:
         * the m_min Ritz vectors of smallest Ritz value (thick restart). */
        if (m == m_max) {
            basis_times(n, m, V, Y, 0, m_min, V2);
            basis_times(n, m, W, Y, 0, m_min, W2);
            { double *s = V; V = V2; V2 = s; s = W; W = W2; W2 = s; }
            memset(H, 0, sizeof(double) * (size_t)m_max * m_max);
            for (int i = 0; i < m_min; ++i) H[i * m_max + i] = Theta[i];
            m = m_min;
        }
        /* step 8: correction equation with Q = [x_1 .. x_{j-1} u] */
        memcpy(Q, X, sizeof(double) * (size_t)n * nx);
        double un = nrm2(n, u);
        for (int i = 0; i < n; ++i) Q[(size_t)nx * n + i] = u[i] / un;
        int br = 0;
        int its = pcg_correction(&L, theta, nx + 1, Q, r, &P, o->itmax, o->rtol_pcg, t, &br);
        info->inner += its;
        info->mvp += its;
        memcpy(v, t, sizeof(double) * (size_t)n);
    }
done:
    info->outer = it;
    info->nconv = nx < k ? nx : k;
    info->status = status;
    /* sort the locked pairs ascending (READING: JD may lock out of order) */
    {
        int *idx = (int *)malloc(sizeof(int) * (size_t)(nx > 0 ? nx : 1));
        for (int i = 0; i < nx; ++i) idx[i] = i;
        for (int i = 0; i < nx; ++i) {
            int b = i;
            for (int j = i + 1; j < nx; ++j) if (lam[idx[j]] < lam[idx[b]]) b = j;
            int s = idx[i]; idx[i] = idx[b]; idx[b] = s;
        }
        int nout = nx < k ? nx : k;
        for (int j = 0; j < nout; ++j) {
            evals[j] = lam[idx[j]];
            memcpy(evecs + (size_t)j * n, X + (size_t)idx[j] * n, sizeof(double) * (size_t)n);
            if (res) res[j] = rlock[idx[j]];
        }
        free(idx);
    }
    orc_ic0_destroy(K);
    orc_fsai_destroy(Zf);
    free(P.dinv);
    free(X); free(lam); free(rlock); free(V); free(W); free(V2); free(W2); free(H); free(Hs);
    free(Theta); free(Y); free(v); free(u); free(r); free(Lu); free(t); free(Q);
    return status;
}

/* ------------------------------------------------------------------ */
/* Algorithm 3 (DACG): the eigenpairs one after the other, each by      */
/* minimizing the Rayleigh quotient q(x) = x'Gx / x'x over the vectors  */
/* orthogonal to those already computed (the columns of U), with a      */
/* preconditioned nonlinear conjugate gradient (the DACG of Bergamaschi,*/
/* Gambolati and Pini that the paper cites):                           */
/*   q_k = x_k'G x_k / x_k'x_k,  g_k = 2 (G x_k - q_k x_k) / x_k'x_k   */
/*   h_k = P g_k;  beta_k = g_k'h_k / g_{k-1}'h_{k-1}  (beta_0 = 0)    */
/*   p_k = (I - UU') h_k + beta_k p_{k-1}    (deflated direction)       */
/*   x_{k+1} = x_k - alpha_k p_k, alpha_k minimizing q on span{x, p}:   */
/*   the smaller eigenpair of the 2 x 2 pencil ([x p]'G[x p], [x p]'[x p]) */
/* Per iteration: one product (G p; G x follows by the same update),    */
/* one preconditioner application, one deflation of the direction       */
/* (the three costs the comments on Algorithm 3 list).                  */
/* READINGS: the zero pairs (component indicators) are locked first, as */
/* in JD; the stopping test is JD's certificate ||G x - q x|| <=        */
/* tol min(q, 1) ||x|| (it implies the paper's ||Gx - qx|| / q <= tol   */
/* for unit x); x_0 is the seeded start vector made orthogonal to U;    */
/* itmax limits the iterations of each pair (then status 1 and the      */
/* certified prefix).                                                   */
/* ------------------------------------------------------------------ */
typedef struct {
    int itmax;          /* iterations per pair; <= 0 means 20000 */
    int precond;        /* ORC_PREC_* */
    uint64_t seed;
    const int *fsai_pos;
} orc_dacg_opts;

ORC_API int orc_dacg(int n, const int *rowptr, const int *col, const double *val, int k, double tol,
                     const orc_dacg_opts *o, double *evals, double *evecs, double *res, orc_jd_info *info) {
    orc_lap L = {n, rowptr, col, val};
    int itmax = o->itmax > 0 ? o->itmax : 20000;
    memset(info, 0, sizeof(*info));
    double *U = (double *)calloc((size_t)n * (size_t)(k > 0 ? k : 1), sizeof(double));
    int nu = 0;
    int *label = (int *)malloc(sizeof(int) * (size_t)n);
    int ncomp = orc_components(n, rowptr, col, label);
    info->ncomp = ncomp;
    for (int c = 0; c < ncomp && nu < k; ++c) {
        double *x = U + (size_t)nu * n;
        int cnt = 0;
        for (int i = 0; i < n; ++i) if (label[i] == c) ++cnt;
        for (int i = 0; i < n; ++i) x[i] = label[i] == c ? 1.0 / sqrt((double)cnt) : 0.0;
        evals[nu] = 0.0;
        if (res) {
            double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
            lap_apply(&L, x, tmp);
            res[nu] = nrm2(n, tmp);
            free(tmp);
        }
        ++nu;
    }
    free(label);
    orc_prec P = {o->precond, NULL, NULL, NULL};
    orc_ic0 *K = NULL;
    orc_fsai *Zf = NULL;
    if (o->precond == ORC_PREC_IC0) { K = orc_ic0_create(n, rowptr, col, val, &info->nfloor); P.ic0 = K; }
    if (o->precond == ORC_PREC_JACOBI) P.dinv = diag_inverse(&L);
    if (o->precond == ORC_PREC_FSAI) { Zf = orc_fsai_create(n, rowptr, col, val, o->fsai_pos, ORC_FSAI_TAU); P.fsai = Zf; }
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *gx = (double *)malloc(sizeof(double) * (size_t)n);
    double *g = (double *)malloc(sizeof(double) * (size_t)n);
    double *h = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *gp = (double *)malloc(sizeof(double) * (size_t)n);
    int status = 0;
    uint64_t start_col = 0;
    while (nu < k) {
        /* x_0: seeded, orthogonal to U (step 1) */
        for (int i = 0; i < n; ++i) x[i] = orc_start_value(o->seed, start_col * (uint64_t)n + i);
        ++start_col;
        orc_mgs(n, nu, U, x);
        scal(n, 1.0 / nrm2(n, x), x);
        lap_apply(&L, x, gx);
        ++info->mvp;
        double gh_prev = 0.0;
        int it, done = 0;
        for (it = 0; it < itmax; ++it) {
            double f = dot(n, x, x), c = dot(n, x, gx);
            double q = c / f;
            /* residual, and the stopping test (step 3) */
            double rn2 = 0.0;
            for (int i = 0; i < n; ++i) { double r = gx[i] - q * x[i]; rn2 += r * r; g[i] = 2.0 * r / f; }
            double scale = q < 1.0 ? q : 1.0;
            if (sqrt(rn2 / f) <= tol * scale) { done = 1; break; }
            /* preconditioned gradient, conjugate direction, deflation (step 2) */
            prec_apply(&P, n, g, h);
            double gh = dot(n, g, h);
            double beta = it == 0 ? 0.0 : gh / gh_prev;
            gh_prev = gh;
            project_out(n, nu, U, h);
            for (int i = 0; i < n; ++i) p[i] = h[i] + (it == 0 ? 0.0 : beta * p[i]);
            /* the line search: the smaller eigenpair of the 2 x 2 pencil */
            lap_apply(&L, p, gp);
            ++info->mvp;
            double a = dot(n, p, gp), b = dot(n, x, gp), d = dot(n, p, p), e = dot(n, x, p);
            double A2 = f * d - e * e, B2 = a * f + c * d - 2.0 * b * e, C2 = c * a - b * b;
            double disc = B2 * B2 - 4.0 * A2 * C2;
            if (disc < 0.0) disc = 0.0;
            double mu = 2.0 * C2 / (B2 + sqrt(disc));
            double den1 = a - mu * d, den2 = b - mu * e;
            double alpha = fabs(den1) >= fabs(den2) ? den2 / den1 : (c - mu * f) / den2;
            axpy(n, -alpha, p, x);
            axpy(n, -alpha, gp, gx);
        }
        info->inner += it;
        info->outer += 1;
        if (!done) { status = 1; break; }
        /* step 4: lock u_j = x / ||x||, certified with a fresh product */
        double xn = nrm2(n, x);
        double *u = U + (size_t)nu * n;
        for (int i = 0; i < n; ++i) u[i] = x[i] / xn;
        lap_apply(&L, u, gx);
        ++info->mvp;
        double theta = dot(n, u, gx);
        double rn2 = 0.0;
        for (int i = 0; i < n; ++i) { double r = gx[i] - theta * u[i]; rn2 += r * r; }
        evals[nu] = theta;
        if (res) res[nu] = sqrt(rn2);
        ++nu;
    }
    info->nconv = nu;
    info->status = status;
    /* ascending order (the sequential minimization yields it, up to clusters) */
    for (int i = 0; i < nu; ++i) {
        int bsel = i;
        for (int j = i + 1; j < nu; ++j) if (evals[j] < evals[bsel]) bsel = j;
        if (bsel != i) {
            double t = evals[i]; evals[i] = evals[bsel]; evals[bsel] = t;
            if (res) { t = res[i]; res[i] = res[bsel]; res[bsel] = t; }
            for (int r = 0; r < n; ++r) {
                t = U[(size_t)i * n + r]; U[(size_t)i * n + r] = U[(size_t)bsel * n + r]; U[(size_t)bsel * n + r] = t;
            }
        }
    }
    memcpy(evecs, U, sizeof(double) * (size_t)n * (size_t)nu);
    orc_ic0_destroy(K);
    orc_fsai_destroy(Zf);
    free(P.dinv);
    free(U); free(x); free(gx); free(g); free(h); free(p); free(gp);
    return status;
}
