/*
 * lapeig.h -- C ABI of the MI355X (gfx950) Jacobi-Davidson solver for the
 * smallest eigenpairs of a graph Laplacian G = D - A.
 *
 * The problem (Section 2 of Bergamaschi, Bozzo & Franceschet, "Computing the
 * smallest eigenpairs of the graph Laplacian"): G is the weighted Laplacian
 * of a simple undirected graph with positive edge weights, D the diagonal of
 * generalized degrees.  G is symmetric positive semidefinite, G e = 0, and
 * the multiplicity of the eigenvalue 0 is the number of connected
 * components.  The method (Section 3.2, Algorithm 2) is Jacobi-Davidson:
 * Rayleigh-Ritz on a search space V, Newton-type corrections from the
 * projected correction equation solved inexactly by PCG, deflation against
 * the converged vectors, and restarts between m_min and m_max columns.
 *
 * Conventions shared by every entry point
 *   - Every function returns lap_status: 0 (LAP_OK) or a negative code.
 *     lap_last_error() returns a thread-local message for the last failure.
 *   - Input validation happens on the host before any HIP call, so bad
 *     arguments are reported without touching the GPU.
 *   - "device" pointers are HIP device allocations on the plan's device;
 *     "host" pointers are ordinary host memory.  The caller owns every
 *     buffer it passes; no pointer is retained after the call returns,
 *     except that a plan keeps its own device copies of the matrix.
 *   - A plan is not thread-safe; distinct plans are independent.
 *   - Block vectors passed to lap_spmv are n x b ROW-major ("interleaved":
 *     element (i, c) at X[i*b + c]); the orthogonalization and PCG entry
 *     points take n x b COLUMN-major blocks (element (i, c) at X[i + c*n]).
 */
#ifndef LAPEIG_H
#define LAPEIG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LAP_OK = 0,
    LAP_EINVAL = -1,          /* bad argument (size, pointer, option) */
    LAP_ENOTLAPLACIAN = -2,   /* the CSR is not the Laplacian of a simple weighted graph */
    LAP_ENOMEM = -3,          /* device or host allocation failed */
    LAP_EDEVICE = -4,         /* a HIP runtime call failed */
    LAP_ENOCONV = -5,         /* eigensolver hit its outer-iteration limit */
    LAP_EUNSUPPORTED = -6     /* valid request this build does not support */
} lap_status;

typedef enum { LAP_F32 = 0, LAP_F64 = 1 } lap_dtype;

/* Arithmetic of lap_eigs.  FP64: every step in double precision.  MIXED:
 * the Laplacian products inside PCG and the whole inner PCG run in single
 * precision with single-precision accumulation; the outer products W = G V,
 * orthogonalization, Rayleigh-Ritz, Rayleigh quotients and the certifying
 * residual stay in double precision, so the answer is certified in FP64. */
typedef enum { LAP_PREC_FP64 = 0, LAP_PREC_MIXED = 1 } lap_precision;

/* The Laplacian G itself (diagonal included), host memory, CSR with int32
 * indices.  Requirements, checked by lap_plan_create: n >= 1; rowptr[0] = 0,
 * rowptr nondecreasing, rowptr[n] = nnz; columns strictly increasing in each
 * row and in [0, n); values finite; off-diagonal values < 0 (the negated
 * edge weights); G symmetric in pattern and value; each diagonal value
 * equal to minus the sum of its row's off-diagonal values (exactly for
 * integer data, else to 1e-12 relative). */
typedef struct {
    int32_t n;
    int32_t nnz;
    const int32_t *rowptr;   /* n + 1 */
    const int32_t *col;      /* nnz */
    const double *val;       /* nnz */
} lap_csr;

typedef struct lap_plan lap_plan;

/* Solver options.  lap_eigs_default_opts fills the paper's parameters
 * (Section 4): m_min = 5, m_max = 10, ITMAX = 20, delta_PCG = 1e-2. */
typedef struct {
    int m_min;           /* basis size kept at a restart */
    int m_max;           /* basis size that triggers a restart */
    int itmax;           /* PCG iterations per correction equation */
    double rtol_pcg;     /* PCG stops at ||res|| <= rtol_pcg * ||r|| */
    int kmax;            /* outer-iteration limit; <= 0 means 1000 * k */
    int precision;       /* lap_precision */
    int block;           /* corrections per outer iteration: 1 is Algorithm 2 */
    uint64_t seed;       /* SplitMix64 stream for start vectors */
    const double *init;  /* optional start block, n x init_cols column-major, caller's
                            vertex order; NULL for a seeded random start.  The solver
                            orthogonalizes it, so any columns will do; columns with a
                            non-finite entry, or inside the span of what is already in
                            the basis, are skipped (info->warm_start_used counts the
                            others) and the seeded random start takes over.  The answer
                            is certified either way and only the iteration count changes */
    int init_cols;
    int init_on_device;  /* 0: init is host memory; 1: device memory */
    int precond;         /* lap_precond: P of the preconditioner M = (I-QQ')P(I-QQ') */
} lap_eigs_opts;

/* The preconditioner P of the correction equation (comments on Algorithm 2).
 * The paper uses IC(0) (Section 4), whose triangular solves are sequential;
 * its Conclusion proposes approximate-inverse preconditioners, applied as
 * products of sparse matrices, for parallel machines.
 *   LAP_PRECOND_JACOBI: P = D^{-1} (the default).
 *   LAP_PRECOND_FSAI:   P = Z'Z, the factorized sparse approximate inverse
 *     (Kolotilina & Yeremin) of G + 1e-8 D: Z lower triangular in the plan's
 *     vertex order with the pattern of G's lower triangle, row v solving
 *     (G + 1e-8 D)[P_v, P_v] g = e_v, Z[v, P_v] = g / sqrt(g_v).  Built once
 *     per plan on first use (host, multi-threaded) and kept on the device in
 *     FP64 and FP32; each application is two sparse products.  Single-vector
 *     solver only (block and batched solves return LAP_EUNSUPPORTED). */
typedef enum { LAP_PRECOND_JACOBI = 0, LAP_PRECOND_FSAI = 1 } lap_precond;

typedef struct {
    int nconv;           /* certified pairs returned (the first nconv entries) */
    int ncomp;           /* connected components = multiplicity of eigenvalue 0 */
    int outer;           /* outer iterations: correction equations solved (steps that
                            only load the caller's start block are not counted) */
    int inner;           /* PCG iterations, summed over the columns */
    long long mvp;       /* Laplacian-vector products; a b-column product counts b */
    double seconds;      /* wall time of the call */
    int warm_start_used; /* columns of opts.init that entered the search space; 0 when no
                            start block was given or none was usable (every column
                            non-finite or inside the span of the deflated vectors), in
                            which case the seeded random start took their place */
} lap_eigs_info;

void lap_eigs_default_opts(lap_eigs_opts *opts);

/* Validate G on the host, then copy it to the current HIP device in the
 * solver's layout (vertices renumbered by decreasing degree; rows of degree
 * above a threshold stored as CSR, the rest as 64-row column-major slices).
 * stream: hipStream_t used by the plan's own work (NULL = default stream).
 * Errors: LAP_EINVAL (null pointers, n < 1), LAP_ENOTLAPLACIAN (first bad
 * row named in lap_last_error), LAP_ENOMEM / LAP_EDEVICE. */
lap_status lap_plan_create(const lap_csr *L, void *stream, lap_plan **out);

/* Vertex order inside one degree of the plan (the degree classes always come
 * in decreasing degree, so the row classes stay prefixes).  HUB (what
 * lap_plan_create uses): vertices whose first neighbour in plan order is the
 * same (on power-law graphs nearly always their largest hub) sit side by
 * side, so a slice's lanes gather from fewer cache lines.  CALLER: the
 * caller's vertex order, for callers that bring their own locality order
 * (for example reverse Cuthill-McKee) to compare against it. */
typedef enum { LAP_PLAN_ORDER_HUB = 0, LAP_PLAN_ORDER_CALLER = 1 } lap_plan_order;

/* lap_plan_create with the order inside a degree chosen by `order` (a
 * lap_plan_order); LAP_EINVAL for any other value, before any device work.
 * Results of every entry point are the same up to the rounding of sums taken
 * in another order. */
lap_status lap_plan_create_ex(const lap_csr *L, void *stream, int order, lap_plan **out);
void lap_plan_destroy(lap_plan *plan);

/* Row classes of the Laplacian product (an engineering choice; the paper
 * fixes no data layout).  Rows, in decreasing degree, of degree above
 * huge_threshold are evaluated by a workgroup each, above long_threshold by
 * a wavefront each, the rest in 64-row column-major slices; a plan starts
 * with long = 32, huge = 512.  Results do not depend on the layout except
 * through the order of floating-point additions within a row.
 *   lap_plan_set_layout: rebuild the layout for the given thresholds
 *     (1 <= long_threshold <= huge_threshold, else LAP_EINVAL).  Blocks
 *     until the device is idle; work areas that solves cached in the plan
 *     are released.
 *   lap_plan_layout: the current thresholds (host out-parameters).
 *   lap_plan_autotune: time a kernel for a grid of thresholds and keep the
 *     fastest layout.  target LAP_TUNE_PRODUCT: the product itself (FP32 or
 *     FP64, b columns, b in [1, 64]), as lap_spmv uses it; LAP_TUNE_PCG: one
 *     iteration launch of the projected PCG that lap_eigs runs per
 *     correction equation (b = 1; FP32 for LAP_PREC_MIXED, FP64 for
 *     LAP_PREC_FP64), whose per-row work favours other thresholds.
 *     cache_path (or NULL): a JSON file of earlier choices keyed by device,
 *     target, b, precision, n, nnz and a log2 histogram of row degrees; a
 *     matching entry is applied without timing, a new choice is added (the
 *     file is rewritten through a temporary and a rename).  info (or NULL)
 *     receives the choice and the time per product of the chosen and of the
 *     initial layout.  Takes from milliseconds to a few seconds. */
typedef enum { LAP_TUNE_PRODUCT = 0, LAP_TUNE_PCG = 1 } lap_tune_target;

typedef struct {
    int32_t long_threshold;
    int32_t huge_threshold;
    double best_us;        /* microseconds per timed launch, chosen layout */
    double default_us;     /* the same at long 32, huge 512 (0 when from the cache) */
    int32_t candidates;    /* layouts timed (0 when taken from the cache) */
    int32_t from_cache;    /* 1 when the choice came from cache_path */
} lap_tune_info;

lap_status lap_plan_set_layout(lap_plan *plan, int32_t long_threshold, int32_t huge_threshold);
lap_status lap_plan_layout(const lap_plan *plan, int32_t *long_threshold, int32_t *huge_threshold);
lap_status lap_plan_autotune(lap_plan *plan, lap_tune_target target, lap_dtype dtype, int32_t b,
                             const char *cache_path, lap_tune_info *info);

/* Size of the plan's matrix and its vertex renumbering: perm[i] is the
 * solver's internal index of the caller's vertex i (host array of n). */
int32_t lap_plan_n(const lap_plan *plan);
lap_status lap_plan_perm(const lap_plan *plan, int32_t *perm);

/* The k smallest eigenpairs of G (Algorithm 2 and its deflation for
 * lambda_2, lambda_3, ..., eq. JDsismorethanone).  k counts the zero
 * eigenvalues (one per connected component, whose eigenvectors are the
 * normalized component indicators); 1 <= k < n, tol > 0.
 * A pair is returned only after an FP64 certificate with a fresh product:
 *   ||G u - theta u|| <= tol * min(theta, 1),  ||u|| = 1,
 * theta the Rayleigh quotient of eq. (1).
 * evals: host, k, ascending.  evecs: n x k column-major in the caller's
 * vertex order, host (evecs_on_device = 0) or device (1), or NULL.
 * res: host, k residual norms, or NULL.  info: or NULL.
 * Eigenvector signs are fixed so that each vector's entry of largest
 * magnitude (lowest index on ties) is positive.  Returns LAP_ENOCONV when
 * kmax is reached; info->nconv pairs are then valid.  Synchronizes the
 * plan's stream before returning. */
lap_status lap_eigs(lap_plan *plan, int k, double tol, const lap_eigs_opts *opts,
                    double *evals, double *evecs, int evecs_on_device, double *res,
                    lap_eigs_info *info);

/* The k smallest eigenpairs by DACG (Algorithm 3): one pair after the
 * other, each minimizing the Rayleigh quotient over the vectors orthogonal
 * to the pairs already found, by a nonlinear conjugate gradient
 * preconditioned with D^{-1}, the search direction deflated against the
 * found pairs, the step minimizing the quotient on span{x, p}.  Same
 * arguments, outputs, certificate and zero-pair handling as lap_eigs; it
 * works in double precision whatever opts->precision says.  opts->kmax
 * limits the iterations of each pair (<= 0: 20000; then LAP_ENOCONV and the
 * certified prefix), opts->seed picks the start vectors, opts->precond
 * must be LAP_PRECOND_JACOBI (else LAP_EUNSUPPORTED); block and init are
 * ignored.  info->outer counts the pairs DACG computed, info->inner its
 * iterations, info->mvp the Laplacian products.  Its iteration count grows
 * with lambda_j / (lambda_{j+1} - lambda_j) (eq. xi), so it suits few,
 * well-separated pairs; k <= 62. */
lap_status lap_eigs_dacg(lap_plan *plan, int k, double tol, const lap_eigs_opts *opts, double *evals,
                         double *evecs, int evecs_on_device, double *res, lap_eigs_info *info);

/* The k smallest eigenpairs by the Implicitly Restarted Lanczos Method on
 * the inverse (Section 3.1, Algorithm 1 right): Lanczos on G^+ (G inverted
 * on the complement of its zero space), each step solving G w = v_j by the
 * projected PCG of lap_pcg (theta = 0, Q = the zero space, the two-launch
 * form, to ||v_j - G w|| <= rtol_inner ||v_j||), full reorthogonalization,
 * and thick restarts that keep the wanted Ritz vectors and the last Lanczos
 * vector (with exact shifts the space of Sorensen's implicit restart),
 * until the wanted Ritz values of G^+ -- the reciprocals of the smallest
 * nonzero eigenvalues -- hold the certificate of lap_eigs.
 *   m: Krylov size (0: max(3 w, w + 6), w = k minus the zero pairs; the
 *      paper: about three times the wanted pairs); zero space + m + 1 <= 63.
 *   rtol_inner <= 0: 1e-12 (the paper: proportional to the accuracy wanted;
 *      a residual of G^+ is amplified by up to ||G|| in the residual of G).
 *   itmax_inner <= 0: 1000 PCG iterations per step.
 *   opts (or NULL): seed (the start vector), precond (Jacobi or FSAI),
 *      kmax (restart limit; <= 0: 1000; then LAP_ENOCONV with the zero
 *      pairs only).  Other fields are ignored; double precision.
 * Outputs as lap_eigs; info->outer = Lanczos steps (inner solves),
 * info->inner = PCG iterations, info->mvp = all Laplacian products. */
lap_status lap_eigs_irlm(lap_plan *plan, int k, double tol, int m, double rtol_inner, int itmax_inner,
                         const lap_eigs_opts *opts, double *evals, double *evecs, int evecs_on_device,
                         double *res, lap_eigs_info *info);

/* One-shot convenience: plan, solve, destroy. */
lap_status lap_eigs_csr(const lap_csr *L, int k, double tol, const lap_eigs_opts *opts,
                        double *evals, double *evecs, double *res, lap_eigs_info *info);

/* Y = G X - X diag(shift): the matrix-vector product (MVP) of Section 3
 * on b columns.  X, Y: device, n x b row-major of dtype (float or double);
 * shift: host array of b doubles or NULL (no shift).  flags: 0 when X and Y
 * are in the caller's vertex order, LAP_ORDER_PLAN when they are already in
 * the plan's internal order (no renumbering passes).  Asynchronous on
 * stream.  Supported b: 1..64. */
#define LAP_ORDER_PLAN 1
#define LAP_PCG_FSAI 2   /* lap_pcg flag: P = the plan's FSAI factor instead of D^{-1} */
lap_status lap_spmv(lap_plan *plan, lap_dtype dtype, int b, const void *X, void *Y,
                    const double *shift, int flags, void *stream);

/* lap_spmv without any device allocation, for callers that cannot allocate:
 * code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, semantics and results (bit for bit) as
 * lap_spmv.  Its scratch -- the renumbered copies of X and Y when flags lacks
 * LAP_ORDER_PLAN, the shifts, and the partial sums of the hub rows of a
 * block product -- lives in one fixed 64 MiB device array that each GPU the
 * library runs on holds until the process ends; a call whose scratch would
 * exceed it (about 2 n b element bytes in the caller's order, for example
 * n b > 4M in FP64) returns LAP_EINVAL.  The plan must live on the current
 * device (else LAP_EINVAL).  All calls on one GPU share that array: calls
 * that overlap in time on one GPU (several streams or threads) race.  A
 * shift is copied to the device on the stream (hipMemcpyAsync from host
 * memory).  Asynchronous on stream. */
lap_status lap_spmv_noalloc(lap_plan *plan, lap_dtype dtype, int b, const void *X, void *Y,
                            const double *shift, int flags, void *stream);

/* Block orthogonalization (Algorithm 2 step 2, double precision):
 * W <- an orthonormal basis of (I - Q Q') W, by classical Gram-Schmidt
 * applied twice against Q, then twice within W column by column; columns
 * whose norm falls below 1e-12 of their norm before the pass are replaced
 * by zero columns and not counted.  Q: device n x q column-major with
 * orthonormal columns (q >= 0); W: device n x b column-major, in/out.
 * rank_out: host int, the number of nonzero columns kept, compacted to the
 * front of W.  dtype must be LAP_F64.  Synchronizes stream. */
lap_status lap_orth(lap_dtype dtype, int n, int q, const double *Q, int b, double *W,
                    int *rank_out, void *stream);

/* All eigenpairs of a small symmetric matrix: the projected matrix H of
 * Algorithm 2 step 5 (Rayleigh-Ritz), in one workgroup.  When m <= 32 and
 * the leading (m-1) x (m-1) block is exactly diagonal (an arrowhead, the
 * form H has in single-vector JD after an expansion, a restart or a lock),
 * from the secular equation, one root per lane; otherwise, or if a root
 * does not converge, by cyclic Jacobi.
 * H: device, m x m column-major, symmetric (both triangles are read; H is
 * not modified).  theta: device, m doubles, ascending.  Y: device, m x m
 * column-major, orthonormal eigenvectors (column j belongs to theta[j]).
 * The caller owns all three.  sweeps_out: host int or NULL; if given, the
 * call synchronizes stream and stores -1 when the secular-equation path
 * solved H, otherwise the number of Jacobi sweeps.  1 <= m <= 96 (else
 * LAP_EINVAL); non-finite entries of H give unspecified output.
 * Asynchronous on stream when sweeps_out is NULL. */
lap_status lap_sym_eig(int m, const double *H, double *theta, double *Y, int *sweeps_out, void *stream);

/* PCG on the projected correction equations (Algorithm 2 step 8):
 *   (I - QQ')(G - theta_c I)(I - QQ') t_c = -r_c,  t_c orthogonal to Q,
 * for each column c < b, with the preconditioner M = (I-QQ')P(I-QQ') and
 * P = D^{-1} (Jacobi) or the FSAI factor (flag LAP_PCG_FSAI).  t_0 = 0; column c stops when its residual norm is
 * <= rtol * ||r_c||, after itmax iterations, or when p'(G - theta_c I)p
 * <= 0 (then the current t_c, or M(-r_c) if no step was taken).
 * theta: host, b doubles.  Q: device n x q column-major orthonormal, in the
 * caller's vertex order unless flags has LAP_ORDER_PLAN (same for R, T).
 * R: device n x b column-major (r_c); T: device n x b column-major output.
 * dtype: arithmetic of the iteration (LAP_F32 or LAP_F64; inputs and
 * outputs stay double).  iters_out: host, b ints (PCG iterations per
 * column) or NULL.  flags: LAP_ORDER_PLAN as for lap_spmv, LAP_PCG_FSAI for
 * P = Z'Z (LAP_PRECOND_FSAI).  Synchronizes stream.  Supported q <= 62, b <= 32. */
lap_status lap_pcg(lap_plan *plan, lap_dtype dtype, int b, const double *theta,
                   const double *Q, int q, const double *R, double *T, int itmax,
                   double rtol, int *iters_out, int flags, void *stream);

/* Consumers of the smallest eigenpairs (Section 2).
 *
 * lap_fiedler_bisect: spectral bisection with prescribed sizes.  Relaxing the
 *   +-1/2 entries of the minimum-cut problem to real ones gives the minimum
 *   n1 n2 lambda_2 / n at x = (n1 - n2)/(2n) e + sqrt(n1 n2/n) v_2, so the
 *   first side is the set of the n1 vertices where the Fiedler vector v_2 is
 *   smallest (equal entries taken by increasing vertex index).
 *   fiedler: device, n doubles, caller order (the second column lap_eigs
 *   returns on a connected graph; any finite vector is accepted).
 *   part: device, n int32, caller order: 0 on the first side, 1 on the other.
 *   cut: host double or NULL: the sum of the weights of the edges between
 *   the sides (x'Gx for x = +-1/2, eq. (1)), which is >= n1 n2 lambda_2 / n.
 *   0 <= n1 <= n; a non-finite entry gives LAP_EINVAL.  Synchronizes stream.
 *
 * lap_pinv_apply: the approximations of the pseudo-inverse G^+ used for
 *   current-flow betweenness, from k computed pairs:
 *     sigma = 0:  Y = T^(k) X = sum_j (1/lambda_j) v_j v_j' X
 *     sigma > 0:  Y = S^(k) X = X/sigma - (1/sigma) sum_{lambda_j = 0} v_j v_j' X
 *                                + sum_{lambda_j > 0} (1/lambda_j - 1/sigma) v_j v_j' X
 *   with j over the k pairs; the zero pairs (one per connected component)
 *   take the place of v_1 = e/sqrt(n).  evals: host, k values >= 0 (zero
 *   exactly for the zero pairs, as lap_eigs returns them); evecs: device
 *   n x k column-major, orthonormal; X, Y: device n x b column-major (Y must
 *   not overlap X).  1 <= k <= 64.  Synchronizes stream. */
lap_status lap_fiedler_bisect(lap_plan *plan, const double *fiedler, int n1, int32_t *part, double *cut,
                              void *stream);
lap_status lap_pinv_apply(int n, int k, const double *evals, const double *evecs, double sigma, int b,
                          const double *X, double *Y, void *stream);

/* Many independent graphs at once (the batched form of Algorithm 2): one
 * persistent launch, captured in a hipGraph, in which each 1024-thread
 * workgroup runs the whole single-vector solver for one graph with all its
 * reductions in LDS, taking graphs largest first from a device queue; the
 * row classes of its product are autotuned per batch (lap_batch_autotune).
 * Each graph is validated as in lap_plan_create and must be connected
 * (LAP_EUNSUPPORTED otherwise); 1 <= k <= 8, m_max <= 16, block = 1.
 * lap_batch_create validates, renumbers and uploads the graphs (host
 * arrays); the handle owns the device copies.  lap_batch_eigs solves all
 * graphs for the k smallest pairs each:
 *   evals: host, nb x k (graph g's values at g*k, ascending);
 *   evecs: host or NULL, graph g's n_g x k column-major block at offset
 *          k * (n_0 + ... + n_{g-1}), in the caller's vertex order
 *          (lap_batch_eigs_ex: host when evecs_on_device = 0, device
 *          memory of the batch's GPU when 1);
 *   res:   host or NULL, nb x k certified residual norms;
 *   infos: host or NULL, nb entries.
 * Pairs a graph did not certify within kmax are NaN (evals, res) and zero
 * vectors; the call then returns LAP_ENOCONV.  Synchronizes before it
 * returns. */
typedef struct lap_batch lap_batch;
lap_status lap_batch_create(const lap_csr *Ls, int nb, lap_batch **out);
void lap_batch_destroy(lap_batch *batch);
int32_t lap_batch_total_n(const lap_batch *batch);

/* Row classes of the batched product: rows whose degree is above a threshold
 * get a wavefront each, the others a thread each.  lap_batch_autotune times
 * one product pass over all graphs of the batch for each candidate threshold
 * (4, 8, ..., 256, and none long) in the given lap_precision's arithmetic and
 * keeps the fastest for that precision; lap_batch_eigs does this by itself
 * on its first call in a precision.  long_threshold / seconds (either may be
 * NULL): the chosen threshold and the seconds per pass it measured.
 * lap_batch_layout: the threshold in use for a precision and whether it was
 * tuned (1) or is the default 32 (0).  Errors: LAP_EINVAL (NULL batch or
 * outputs, unknown precision), LAP_EDEVICE. */
lap_status lap_batch_autotune(lap_batch *batch, int precision, int32_t *long_threshold, double *seconds);
lap_status lap_batch_layout(const lap_batch *batch, int precision, int32_t *long_threshold, int32_t *tuned);
lap_status lap_batch_eigs(lap_batch *batch, int k, double tol, const lap_eigs_opts *opts, double *evals,
                          double *evecs, double *res, lap_eigs_info *infos, void *stream);
lap_status lap_batch_eigs_ex(lap_batch *batch, int k, double tol, const lap_eigs_opts *opts, double *evals,
                             double *evecs, int evecs_on_device, double *res, lap_eigs_info *infos,
                             void *stream);
lap_status lap_eigs_batch(const lap_csr *Ls, int nb, int k, double tol, const lap_eigs_opts *opts,
                          double *evals, double *evecs, double *res, lap_eigs_info *infos, void *stream);

/* Learned start block (an engineering addition: the paper starts from a
 * single unit vector, Algorithm 2).  A small message-passing network over
 * the plan's graph proposes out_cols start vectors; lap_eigs takes them as
 * opts.init, and its FP64 certificate decides the answer as always.
 *   features of vertex i: 1, log(1 + d_i), the mean of log(1 + d_j) over
 *     its neighbours (weighted), and random_channels values sqrt(3) u with
 *     u the SplitMix64 uniform variate in [-1, 1) of counter
 *     i * random_channels + c under feature_seed (i the caller's index);
 *   layers hidden layers h' = ReLU([h | D^{-1}A h] W + b), width hidden;
 *   output Y = [h | D^{-1}A h] W_o + b_o (out_cols columns), minus its
 *     column means (the component of the zero eigenvector; connected
 *     graphs).
 * Parameters are FP32, one flat vector: per layer W (column-major,
 * 2 F_in x F_out) then b, output layer last; lap_mpnn_create draws W
 * Glorot-uniform from SplitMix64 under cfg->seed, b = 0.
 * Training minimizes loss = 1 - trace(S^{-1} C C')/kx, S = Yh'Yh,
 * C = Yh'X, for orthonormal eigenvectors X (n x kx, orthogonal to the
 * constant vector): the mean squared cosine of the principal angles
 * between span X and span Yh, complemented.  Limits: 1 <= hidden <= 32,
 * 0 <= layers <= 8, 0 <= random_channels <= 16, 1 <= out_cols,
 * out_cols + kx <= 32; loss and training need a connected graph.
 *   lap_mpnn_infer: V0 (device, n x out_cols column-major, caller order).
 *   lap_mpnn_loss_grad: X device (n x kx column-major, caller order);
 *     loss (host double); grad (host, num_params floats) or NULL.
 *   lap_mpnn_train_step: the same, then one Adam step (beta 0.9 / 0.999,
 *     eps 1e-8) with learning rate lr.
 * All three run on stream and synchronize it before returning. */
typedef struct {
    int32_t layers;
    int32_t hidden;
    int32_t random_channels;
    int32_t out_cols;
    uint64_t seed;
} lap_mpnn_config;
typedef struct lap_mpnn lap_mpnn;

lap_status lap_mpnn_create(const lap_mpnn_config *cfg, lap_mpnn **out);

/* Keeping a trained network (checkpoint of the warm-start network and of its
 * optimizer).  lap_mpnn_save writes a versioned file: the line "LAPEIG-MPNN",
 * a one-line JSON header {"format": 1, "layers", "hidden", "random_channels",
 * "out_cols", "seed", "num_params", "adam_step", "payload_bytes", "dtype":
 * "float32-le", "fnv1a64"}, then the parameters and Adam's two moment
 * vectors (num_params float32 values each, little-endian, the flat order of
 * lap_mpnn_get_params); it writes path.tmp and renames it over path.
 * lap_mpnn_load checks the whole file on the host before any HIP call
 * (magic, format, configuration limits, num_params against the
 * configuration, payload size, FNV-1a checksum of the payload, finite
 * values) and then creates the network on the current device with those
 * parameters and that Adam state, so training resumes where it stopped.
 * Errors: LAP_EINVAL (NULL arguments, unreadable or malformed file, failed
 * write), LAP_EUNSUPPORTED (a newer format), LAP_ENOMEM / LAP_EDEVICE. */
lap_status lap_mpnn_save(const lap_mpnn *net, const char *path);
lap_status lap_mpnn_load(const char *path, lap_mpnn **out);
void lap_mpnn_destroy(lap_mpnn *net);
int64_t lap_mpnn_num_params(const lap_mpnn *net);
/* The configuration a network was created (or loaded) with; LAP_EINVAL on NULL. */
lap_status lap_mpnn_get_config(const lap_mpnn *net, lap_mpnn_config *cfg);
lap_status lap_mpnn_get_params(const lap_mpnn *net, float *params);
lap_status lap_mpnn_set_params(lap_mpnn *net, const float *params); /* also resets Adam */
lap_status lap_mpnn_infer(lap_mpnn *net, lap_plan *plan, uint64_t feature_seed, double *V0, void *stream);
lap_status lap_mpnn_loss_grad(lap_mpnn *net, lap_plan *plan, uint64_t feature_seed, const double *X, int kx,
                              double *loss, float *grad, void *stream);
lap_status lap_mpnn_train_step(lap_mpnn *net, lap_plan *plan, uint64_t feature_seed, const double *X, int kx,
                               float lr, double *loss, void *stream);

const char *lap_status_string(lap_status s);
const char *lap_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LAPEIG_H */
