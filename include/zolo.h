/*
 * zolo.h -- C ABI of the MI355X (gfx950) Zolotarev spectrum-filter eigensolver.
 *
 * Problem (Li & Yang, Sec. 1, eq. IGEVP): for a sparse Hermitian definite
 * pencil (A, B) and an interval (a, b), find all (lambda, x) with
 * A x = lambda B x and a < lambda < b.  The solver is subspace iteration
 * (Algorithm 1) with the rational filter
 *     R_ab(x) = (Z_2r2(Zhat_2r1(T(x); l1); l2) + 1) / 2      (eq. Rab / R2)
 * applied by the hybrid algorithm (Algorithm 2): r1 sparse LDL^T
 * factorizations of A - sigma_hat_j B build the operator G of eq. (solve),
 * and shift-invariant block GMRES on G solves the outer shifts of eq. (solve2).
 *
 * Conventions for every call below.
 *  - Errors never abort: a call returns a zolo_status and zolo_last_error()
 *    gives a thread-local message for the last failing call.
 *  - Host arrays passed in are copied during the call; the caller keeps them.
 *  - Handles (ctx, pencil, factors, result) are owned by the library until
 *    their *_free / *_destroy call.
 *  - "d_" arguments are device pointers owned by the caller (for instance
 *    PyTorch tensors on the context's device); dense blocks are row-major
 *    N x p with leading dimension ld >= p (element stride between rows).
 *    Real pencils use double; complex Hermitian pencils use interleaved
 *    complex128 (re, im).
 *  - stream: a hipStream_t passed as void*; NULL means the default stream.
 *    Device entry points enqueue on that stream and synchronise it before
 *    returning, so outputs are ready when the call returns.
 *  - Indices of the CSR inputs are 0-based, rows sorted by column, A and B
 *    share one pattern stored in full (both triangles).
 */
#ifndef ZOLO_H
#define ZOLO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ZOLO_OK = 0,
  ZOLO_EINVAL = 1,     /* invalid argument (sizes, pointers, gap order, CSR) */
  ZOLO_ENOTHERM = 2,   /* A or B not Hermitian, or patterns differ           */
  ZOLO_ENOMEM = 3,     /* device or host allocation failed                  */
  ZOLO_ENOCONV = 4,    /* GMRES or subspace iteration missed its tolerance  */
  ZOLO_EGAP = 5,       /* a Ritz value fell inside a stated eigengap         */
  ZOLO_ESUBSPACE = 6,  /* subspace too small for the count found             */
  ZOLO_EDEVICE = 7,    /* HIP runtime error                                  */
  ZOLO_EBREAKDOWN = 8, /* zero pivot in a factorization or Gram matrix       */
  ZOLO_ETIMEOUT = 9    /* zolo_wait: the query has not finished in time      */
} zolo_status;

typedef enum { ZOLO_REAL64 = 0, ZOLO_COMPLEX128 = 1 } zolo_scalar;
typedef enum { ZOLO_PREC_FP64 = 0, ZOLO_PREC_MIXED = 1 } zolo_precision;

#define ZOLO_MAX_R 16

/*
 * Coefficient set of the filter (Algorithm 2, lines 2-4; Remark after
 * Proposition 2 for the hatted names).  Filled by zolo_filter_plan.
 *   Moebius map T(x) = gamma (x - alpha)/(x - beta)          (eq. mo, eq. req)
 *   inner function g(x) = Zhat_2r1(T(x); l1)
 *     = M_hat [c0 + sum_j (w_hat_j/(x - sigma_hat_j) + conj(w_hat_j)/(x - conj(sigma_hat_j)))]
 *                                                             (Proposition 2)
 *   outer Z_2r2(g; l2) = (M/2) sum_j a_j (1/(g + i sqrt c_j) + 1/(g - i sqrt c_j))
 *                                                             (Corollary 1)
 */
typedef struct {
  int r1, r2;
  double a_minus, a_plus, b_minus, b_plus;
  double l1, l2;
  double alpha, beta, gamma;
  double M_hat, c0, delta1;
  double sigma_hat_re[ZOLO_MAX_R], sigma_hat_im[ZOLO_MAX_R];
  double w_hat_re[ZOLO_MAX_R], w_hat_im[ZOLO_MAX_R];
  double a_hat[ZOLO_MAX_R], c_hat[ZOLO_MAX_R]; /* c_hat_{2j-1}, j = 1..r1 */
  double M;
  double a[ZOLO_MAX_R], c[ZOLO_MAX_R];         /* c_{2j-1} of Z_2r2(.; l2) */
  double delta_S, delta0;                      /* composite error; delta0 = delta_S/2 */
  int kind;  /* ZOLO_FILTER_*: 0 the composite Zolotarev filter (outer stage by
                multi-shift GMRES); otherwise a one-stage filter applied as
                R(B^-1 A) V = s0 V + s1 G V with G as above */
} zolo_filter_coeffs;

/* Filters (Sec. 2.2): the paper's composite Zolotarev filter, and the
 * comparison filters of its Figs. 2-3, applied with one factorization per
 * conjugate pair of poles on the same kernels. */
enum {
  ZOLO_FILTER_HYBRID = 0,     /* (Z_2r2(Zhat_2r1(T(x))) + 1)/2, Algorithm 2       */
  ZOLO_FILTER_ZOLO = 1,       /* (Zhat_2r(T(x)) + 1)/2: the inner function alone  */
  ZOLO_FILTER_TRAPEZOID = 2,  /* contour integral, trapezoidal rule (CITZ)        */
  ZOLO_FILTER_GAUSS = 3       /* contour integral, Gauss-Legendre rule (CIGQ)     */
};

typedef struct {
  double a_minus, a_plus, b_minus, b_plus; /* eigengaps; a_minus may be -INF or b_plus +INF;
                              all four NaN: estimated by inertia counts on the device */
  int r1;                  /* number of factorizations (inner order); 0 = fewest
                              (<= 4) giving an outer modulus l2 >= 0.2, and no more
                              than the free device memory holds                    */
  int r2;                  /* outer order; 0 = smallest r2 with delta0 <= filter_eps */
  double filter_eps;       /* target delta0 when r2 == 0 (Remark after Algorithm 2) */
  int n_ss;                /* subspace size; 0 = ceil(1.5 n_lambda_est)             */
  int max_subspace_iter;   /* Algorithm 1 iterations                                */
  int max_gmres_iter;      /* block GMRES steps per filter application (all cycles) */
  double tol_resid;        /* ||Ax - lam Bx|| / ((||A|| + |lam| ||B||) ||x||)        */
  double tol_gmres;        /* per shift and column, relative LS residual            */
  int precision;           /* zolo_precision                                        */
  uint64_t seed;           /* start block when none is passed                       */
  int max_refine;          /* mixed precision: refinement steps per pole solve      */
  double tol_refine;       /* mixed precision: inner relative residual target at the
                              first GMRES step; step k relaxes it to
                              min(1e-2, tol_refine / outer residual of step k-1)     */
  int block_cols;          /* > 0: apply the filter to column sub-blocks of at most
                              this many columns (block GMRES per sub-block; the
                              Krylov basis then holds block_cols columns), 0 = all */
  int filter_kind;         /* ZOLO_FILTER_*; for the comparison filters r1 is the
                              number of factorizations (poles per half-plane)      */
  int gmres_restart;       /* block GMRES restarts every this many steps (collinear
                              residuals, see zolo_filter_apply); the basis holds
                              that many blocks.  0 = no restart (max_gmres_iter)   */
  int reuse_subspace;      /* serving only (zolo_submit), default 0.  1: the server
                              keeps this query's eigenpairs resident, and answers it
                              from the resident eigenpairs of an earlier query for
                              the same result (pencil, interval, filter, tolerances
                              and limits alike, subspace no larger) when their
                              residuals, recomputed now, meet tol_resid
                              (stats.subspace_reused); else it runs as usual       */
} zolo_opts;

typedef struct {
  int n_iter;              /* subspace iterations                                   */
  int n_gmres_total;       /* GMRES steps summed over iterations                    */
  int n_gmres_last;
  long long n_solv;        /* RHS solves: r1 * n_ss * n_gmres (x2 complex pencils)  */
  long long n_refine;      /* extra FP32 solves (mixed)                             */
  int refine_sweeps_max;   /* mixed: most corrections one pole refinement took      */
  int refine_missed;       /* mixed: refinements stopped above their target
                              (max_refine reached, or a sweep gained < 2x)          */
  double refine_worst;     /* mixed: largest relative residual such a refinement left */
  int n_found;
  double max_resid;        /* spec residual over returned pairs               */
  double e_lambda_x;       /* eq. (relerr)                                          */
  double b_orth;           /* max |X^H B X - I|                                     */
  double t_plan, t_symbolic, t_factor, t_iter, t_total;   /* seconds              */
  double gmres_resid;      /* worst final LS residual                               */
  double norm_a, norm_b;   /* infinity norms used in the residual                   */
  int r1, r2;
  double l1, l2, delta0;
  long long factor_bytes;  /* device bytes of all factors                           */
  long long nnz_l;         /* entries of one factor (panel + diagonal-block inverse) */
  double factor_flops;     /* per pole                                              */
  long long inertia_count; /* eigenvalues in (a, b) by inertia (eigengaps estimated),
                              -1 when the caller gave the gaps                      */
  double t_gaps;           /* seconds spent estimating the eigengaps                */
  double a_minus, a_plus, b_minus, b_plus;  /* the eigengaps the filter used        */
  int factors_reused;      /* 1: resident factors of an earlier query were used     */
  int n_restart;           /* block GMRES restarts summed over iterations           */
  int precision_fallback;  /* 1: ZOLO_PREC_MIXED was asked, but the complex64 factors'
                              refinement diverged (poles too close to the spectrum)
                              and the query ran again with FP64 factors            */
  int subspace_reused;     /* serving: 1 when the eigenpairs are a resident subspace
                              of an earlier query for the same result; max_resid is
                              then recomputed and t_total is the check's time       */
} zolo_stats;

typedef struct zolo_ctx zolo_ctx;
typedef struct zolo_pencil zolo_pencil;
typedef struct zolo_factors zolo_factors;
typedef struct zolo_result zolo_result;

/* Thread-local message of the last failing call ("" if none). */
const char* zolo_last_error(void);
const char* zolo_version(void);

/* Defaults: r1 = 2, r2 = 0 (auto), filter_eps = 1e-10, tol_resid = 1e-8,
 * tol_gmres = 1e-10, max_subspace_iter = 6, max_gmres_iter = 60,
 * gmres_restart = 30, FP64, the composite filter. */
zolo_status zolo_opts_default(zolo_opts* out);

/* Context on one HIP device: selects the device, creates nothing else.
 * Device memory released by the library (factors, workspaces, results) is
 * kept in a process-wide cache and reused by later allocations of about the
 * same size; destroying a context returns the cached blocks to HIP. */
zolo_status zolo_ctx_create(int hip_device, zolo_ctx** out);
void zolo_ctx_destroy(zolo_ctx* ctx);
/* Device-memory budget of the context's device (bytes; 0 = none, the
 * default).  Every device allocation of the library (factors, solve programs,
 * Krylov bases, results) counts against it while it is held; one that would
 * exceed it fails with ZOLO_ENOMEM and a message, before any hipMalloc.
 * zolo_ctx_hbm_in_use reports the bytes currently held. */
zolo_status zolo_ctx_set_hbm_budget(zolo_ctx* ctx, size_t bytes);
zolo_status zolo_ctx_hbm_in_use(const zolo_ctx* ctx, size_t* bytes);

/*
 * Upload a pencil (host CSR) and run nested dissection + symbolic analysis on
 * the host (multifrontal method, Sec. 2.3: the pre-factorization phase).
 * grid (may be NULL): {nx, ny, nz} when the rows are the points x + nx*y +
 * nx*ny*z of a box grid whose stencil couples only neighbours within distance
 * one; then separators are grid planes.  Otherwise a graph bisection by
 * breadth-first level structures is used.  leaf_size: largest subdomain
 * left undissected (0 = default 64).
 * Errors: ZOLO_EINVAL (bad CSR), ZOLO_ENOTHERM (A or B not Hermitian).
 */
zolo_status zolo_pencil_create(zolo_ctx* ctx, int64_t n, const int64_t* rowptr, const int32_t* colind,
                               const void* a_vals, const void* b_vals, int scalar, const int32_t* grid,
                               int leaf_size, zolo_pencil** out);
void zolo_pencil_free(zolo_pencil* p);
/* Symbolic figures: fronts, levels, entries of one factor, flops per pole. */
zolo_status zolo_pencil_info(const zolo_pencil* p, int64_t* n_fronts, int64_t* n_levels, int64_t* nnz_l,
                             double* flops_per_pole, int64_t* max_front);
/*
 * Host only (no device needed): nested dissection + symbolic analysis of a
 * CSR pattern, as zolo_pencil_create runs it.  perm (may be NULL): n entries,
 * perm[new] = old.  info (may be NULL): 8 entries = {fronts, levels,
 * panel entries (sum k*ns), inverse entries (sum ns^2), update entries
 * (sum nb^2), largest front, struct entries (sum nb), flops per pole}.
 */
zolo_status zolo_symbolic(int64_t n, const int64_t* rowptr, const int32_t* colind, const int32_t* grid, int leaf_size,
                          int32_t* perm, double* info);
/* Nested-dissection permutation: perm[new] = old (host array of n). */
/* Entries (scalars of the factor type) of one pole's numeric factorization,
 * from the symbolic analysis: out[0] panels, out[1] L11^-1 blocks, out[2] the
 * update-block pool (level-scoped), out[3] all update blocks together,
 * out[4], out[5] per-level temporaries (inverse doubling, solve panels).
 * LU (complex Hermitian pencils) doubles out[0], out[1], out[4], out[5]. */
zolo_status zolo_pencil_memory(const zolo_pencil* p, int64_t* out);
/* Algorithmic real flops of one pole from the symbolic analysis (complex
 * arithmetic, 8 real flops per complex multiply-add; LU twice LDL^T):
 * out[0] the elimination of every front (LDL^T: sum of 8 (k^3 - nb^3) / 6 over
 * fronts of k rows with nb update rows), out[1] the same with the L11^-1
 * blocks the solves use, out[2] a forward plus backward solve per right-hand
 * side column (16 nnz(L)). */
zolo_status zolo_pencil_flops(const zolo_pencil* p, double* out);
zolo_status zolo_pencil_perm(const zolo_pencil* p, int32_t* perm);

/*
 * Filter coefficients from the eigengaps (Algorithm 2, lines 2-4): Moebius
 * map, inner Zhat_2r1(.; l1) poles/weights, l2 and the outer Z_2r2(.; l2).
 * r2 == 0 selects the smallest r2 <= 16 with delta0 <= eps (Remark).
 * Host only.  Errors: ZOLO_EINVAL (gaps not ordered, r out of range).
 */
/* Coefficients of any filter kind (ZOLO_FILTER_*) with r factorizations: the
 * composite (r1 = r, r2 by the Remark), Zolo(r) (the inner function alone, from
 * the eigengaps), or a contour rule on the circle through a and b with r poles
 * in the upper half-plane (2r in all).  Host only; errors: ZOLO_EINVAL. */
zolo_status zolo_filter_plan_kind(int kind, double a, double b, double a_minus, double a_plus, double b_minus,
                                  double b_plus, int r, double eps, zolo_filter_coeffs* out);
zolo_status zolo_filter_plan(double a_minus, double a_plus, double b_minus, double b_plus, int r1, int r2,
                             double eps, zolo_filter_coeffs* out);

/*
 * Numeric factorization of K_j = A - sigma_hat_j B, j = 1..r1 (Algorithm 2,
 * lines 5-6), without pivoting in the nested-dissection order: complex-
 * symmetric LDL^T for real pencils, LU = L D U for complex Hermitian pencils
 * (whose conjugate poles are solved with K_j^-H).  Poles are factored
 * concurrently on streams of their own and joined to `stream`.
 * precision ZOLO_PREC_MIXED stores complex64 factors (FP32 accumulation).
 * Errors: ZOLO_EBREAKDOWN (zero pivot), ZOLO_ENOMEM, ZOLO_EDEVICE.
 */
zolo_status zolo_factor(zolo_ctx* ctx, zolo_pencil* p, const zolo_filter_coeffs* co, int precision,
                        void* stream, zolo_factors** out);
void zolo_factors_free(zolo_factors* f);

/* Sylvester inertia (Sec. 1: the number of eigenvalues of the pencil in an
 * interval, which sizes the subspace; Alg. 2 line 1: the eigengaps):
 * counts[k] = number of eigenvalues of (A, B) below sigmas[k], for
 * 1 <= nshift <= ZOLO_MAX_R real shifts (host arrays).  Each shift is an
 * unpivoted LDL^T (complex Hermitian pencils: L D L^H) of A - sigma_k B in the
 * nested-dissection order on the device, counting negative pivots; the shifts
 * are factored concurrently.  Blocking.  Errors: ZOLO_EBREAKDOWN (a zero pivot:
 * the shift is numerically an eigenvalue), ZOLO_ENOMEM, ZOLO_EINVAL. */
zolo_status zolo_inertia(zolo_ctx* ctx, zolo_pencil* p, const double* sigmas, int nshift, int64_t* counts,
                         void* stream);

/* d_Y = A d_X or B d_X (which = 0 for A, 1 for B); N x p row-major blocks in
 * the ORIGINAL ordering, double for real pencils, complex128 for complex ones. */
zolo_status zolo_spmm(zolo_pencil* p, int which, const void* d_X, int64_t ldx, int ncols, void* d_Y, int64_t ldy,
                      void* stream);

/* Residual norms of approximate eigenpairs (x_c, lam_c) of the pencil, the
 * accuracy measure of an eigenpair of eq. (IGEVP) (Sec. 1):
 *   d_out[c] = ||A x_c - lam_c B x_c||_2 / ((||A||_inf + |lam_c| ||B||_inf) ||x_c||_2)
 * for c < ncols <= 512.  d_X: N x ncols row-major (ld ldx >= ncols), original
 * ordering, the pencil's scalar type; d_lambda, d_out: ncols doubles, device.
 * Caller-owned buffers; the library allocates (and on return releases) its
 * partial sums, so the call blocks until the norms are written.  A zero-norm
 * column gives 0 (zero residual) or +inf.  Errors: ZOLO_EINVAL (null
 * pointers, ld < ncols, ncols above the limit), ZOLO_ENOMEM. */
zolo_status zolo_residuals(zolo_pencil* p, const void* d_X, int64_t ldx, int ncols, const double* d_lambda,
                           double* d_out, void* stream);

/* zolo_residuals for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same norms from the same kernels, with the partial sums in a static
 * device array of the library (4 MiB per GPU, held until the process ends;
 * its address is looked up when a context is created on the device).  No
 * hipMalloc/hipFree and no host synchronization: the norms are ready when
 * `stream` reaches them.  Limit: ncols <= 512 (ZOLO_EINVAL beyond, with a
 * message).  All calls on one GPU share the array, so calls that overlap on
 * one GPU (other streams or threads) race and must be serialized by the
 * caller.  Errors: as zolo_residuals, and ZOLO_EDEVICE if the array's
 * address cannot be obtained. */
zolo_status zolo_residuals_noalloc(zolo_pencil* p, const void* d_X, int64_t ldx, int ncols, const double* d_lambda,
                                   double* d_out, void* stream);

/* d_X (complex128, N x p) = K_j^-1 d_T for pole j (0-based) (eq. solve).
 * Real pencils: j < r1, d_T real.  Complex Hermitian pencils: d_T complex128,
 * j < r1 gives K_j^-1 and r1 <= j < 2 r1 gives K_{j-r1}^-H
 * = (A - conj(sigma_hat) B)^-1.  Original ordering.  In mixed precision the
 * FP32 factor is refined against FP64 residuals until tol_refine. */
zolo_status zolo_pole_solve(zolo_factors* f, int j, const double* d_T, int64_t ldt, int ncols, void* d_X,
                            int64_t ldx, void* stream);

/* d_W = G d_V with G = Zhat(T(B^-1 A); l1) applied through the factors
 * (eq. solve, Proposition 2).  Blocks of the pencil's scalar type (double or
 * complex128), original ordering. */
zolo_status zolo_apply_G(zolo_factors* f, const double* d_V, int64_t ldv, int ncols, double* d_W, int64_t ldw,
                         void* stream);

/* Per-call statistics of zolo_filter_apply. */
typedef struct {
  int n_gmres;             /* block GMRES steps                                  */
  double worst_resid;      /* max over shifts and columns of the relative LS residual */
  int breakdown;           /* 1 if the block Krylov space was exhausted          */
  int restarts;            /* restart cycles                                     */
} zolo_filter_stats;

/*
 * d_Y = R_ab(B^-1 A) d_V (Algorithm 2, lines 8-9): multi-shift block GMRES
 * on G with the outer shifts +- i sqrt(c_j) (eq. solve2, Corollary 1), then
 * Y = V/2 + sum_j (M a_j / 4) [(G + i sqrt c_j)^-1 + (G - i sqrt c_j)^-1] V.
 * Real pencils solve only the + shifts (the - solutions are their
 * conjugates); complex Hermitian pencils solve both.  Blocks of the pencil's
 * scalar type.  tol_gmres <= 0 and max_iter <= 0 take the defaults.  Returns
 * ZOLO_ENOCONV (with d_Y filled by the best iterate) if max_iter steps do
 * not reach tol_gmres.
 * restart > 0 (and < max_iter): the basis holds restart blocks; after each
 * cycle the shift with the largest residual (the base) takes its
 * minimal-residual update and every other shift the update that keeps its
 * residual a multiple of the base's residual block (collinear restarts for
 * shifted systems, Frommer and Glaessner 1998, in block form), so the next
 * cycle again serves all shifts from one basis.  Real pencils continue on the
 * 2 ncols real columns [Re R, Im R] of the complex base residual R (twice the
 * pole solves per step after the first restart).
 * Factors of a comparison filter (coefficients of kind != ZOLO_FILTER_HYBRID)
 * apply their one-stage R instead, with no GMRES (tolerances ignored, st
 * zeroed): Zolo(r) gives (G V + V)/2, the contour rules G V.
 */
zolo_status zolo_filter_apply(zolo_factors* f, const double* d_V, int64_t ldv, int ncols, double* d_Y,
                              int64_t ldy, double tol_gmres, int max_iter, int restart, zolo_filter_stats* st,
                              void* stream);

/*
 * Eigenpairs of (A, B) in (a, b) (Algorithm 1 with Algorithm 2).
 * n_lambda_est: estimated count (footnote of Sec. 1); opts may be NULL.
 * d_Q0 (may be NULL): N x n_ss start block (row-major, ld n_ss) in the
 * original ordering, of the pencil's scalar type (double or complex128);
 * NULL draws a Gaussian block from opts->seed.  ZOLO_PREC_MIXED factors in
 * complex64 (both pencil types) and refines every pole solve against FP64
 * residuals.
 * The result holds Ritz pairs with a < theta < b and residual <= tol_resid;
 * its vectors are complex128 for complex pencils.  An interval with no
 * eigenvalue returns count 0 once two filtered iterations select none.
 * Errors: ZOLO_EGAP (best results and stats still filled: a Ritz value
 * converged inside a stated eigengap, so the gaps given are wrong),
 * ZOLO_ENOCONV (best results and stats still filled),
 * ZOLO_ESUBSPACE (found >= n_ss - 1 and the inertia count of (a, b) differs), ZOLO_EINVAL.
 */
zolo_status zolo_solve(zolo_ctx* ctx, zolo_pencil* p, double a, double b, int n_lambda_est, const zolo_opts* opts,
                       const double* d_Q0, void* stream, zolo_result** out);
/*
 * Spectrum slicing (Sec. 1; the independent intervals are the parallel work of
 * Sec. 3.2): all eigenpairs of (A, B) in (lo, hi), computed as n_slices
 * adjacent slices of about equal width, each one Algorithm 1 query with its
 * eigengaps, count and r1 estimated by inertia (opts' gaps and n_ss are
 * ignored; its r1, precision, tolerances and block_cols apply).  Inner slice
 * ends are moved off eigenvalues by inertia before the queries run.  The
 * result joins the slices' pairs in ascending order (stats: sums of the
 * slices' counts and times, worst residuals).  Errors: as zolo_solve, ZOLO_EGAP
 * when no slice end can be placed away from the eigenvalues, ZOLO_ENOCONV
 * (result filled) when the pairs found differ from the inertia count.
 */
zolo_status zolo_slice(zolo_ctx* ctx, zolo_pencil* p, double lo, double hi, int n_slices, const zolo_opts* opts,
                       void* stream, zolo_result** out);
int64_t zolo_result_count(const zolo_result* r);
/* ascending eigenvalues, host array of zolo_result_count entries, owned by r */
const double* zolo_result_eigenvalues(const zolo_result* r);
/* copy the B-orthonormal eigenvectors (N x count, row-major, ld) to a device buffer */
zolo_status zolo_result_copy_vectors(const zolo_result* r, void* d_dst, int64_t ld, void* stream);
/* the same to a host buffer (blocking copy over PCIe) */
zolo_status zolo_result_copy_vectors_host(const zolo_result* r, void* h_dst, int64_t ld);
/* the result's own device copy of the eigenvectors (N x count row-major, ld
 * returned in *ld = count; double, or interleaved complex128 for complex
 * pencils); owned by r and valid until zolo_result_free; NULL when count = 0 */
const void* zolo_result_device_vectors(const zolo_result* r, int64_t* ld);
zolo_status zolo_result_stats(const zolo_result* r, zolo_stats* out);
void zolo_result_free(zolo_result* r);

/*
 * Kernel-class timing for measurement: when enabled, every launch of the
 * library is bracketed by HIP events on the stream it is launched on, and
 * the algorithmic work of the launch (flops, and the bytes the operation
 * must move at least once) is accumulated per class.  Enabling resets the
 * counters.  Not thread safe; for benchmarks.
 */
enum {
  ZOLO_PROF_SPMM = 0,          /* CSR products B V, A Y, B Y                     */
  ZOLO_PROF_GEMM_FACTOR = 1,   /* front trailing / Schur / inverse updates        */
  ZOLO_PROF_GEMM_SOLVE = 2,    /* supernodal solve products                       */
  ZOLO_PROF_GEMM_KRYLOV = 3,   /* CGS2, CholQR, assembly, Rayleigh-Ritz products  */
  ZOLO_PROF_FRONT_OTHER = 4,   /* assembly, extend-add, diagonal blocks, panels   */
  ZOLO_PROF_SOLVE_GATHER = 5,  /* row gathers / extend-adds of the solves         */
  ZOLO_PROF_HLS = 6,           /* shifted Hessenberg least squares                */
  ZOLO_PROF_RR = 7,            /* reduced eigenproblem                            */
  ZOLO_PROF_ELEMWISE = 8,      /* G combine, reductions                           */
  ZOLO_PROF_COUNT = 9
};
typedef struct {
  long long launches;
  double ms;      /* summed event time                      */
  double flops;   /* algorithmic flops of those launches    */
  double bytes;   /* algorithmic bytes of those launches    */
} zolo_kernel_profile;
zolo_status zolo_profile_enable(int on);
zolo_status zolo_profile_query(int cls, zolo_kernel_profile* out);

/*
 * Serving: a request loop over resident pencils (not in the paper; it runs
 * Algorithm 1 per query as zolo_solve does).
 *
 *  - zolo_server_create starts `slots` worker threads on the context's
 *    device, each with its own HIP stream, so up to `slots` queries run on the
 *    GPU at once and their kernels overlap.
 *  - Admission: a query's device memory is estimated before it starts
 *    (factors of its r1 poles from the pencil's symbolic analysis, the block
 *    Krylov basis of max_gmres_iter steps, subspace and solve buffers); queued
 *    queries start in arrival order while the estimates of the running ones,
 *    the resident factorizations that cannot be evicted, plus the next stay
 *    within hbm_budget_bytes (0 = 60% of the free device memory at
 *    creation).  A query whose estimate alone exceeds the budget fails with
 *    ZOLO_ENOMEM.
 *  - Batching: queued queries asking for the same result (same pencil,
 *    interval, eigengaps, r1, r2, precision, tolerances and limits) are
 *    answered by one run, with the start block of the member with the
 *    largest subspace; each receives a copy of its eigenpairs.
 *  - Residency: a query's factorization stays on the device after it
 *    finishes and serves later queries of the same filter (pencil, eigengaps,
 *    r1, r2, filter_eps, precision), one query at a time; resident
 *    factorizations count against the budget and the least recently used
 *    idle ones are freed when a query needs their memory.
 *    zolo_server_get_info reports them (hits: runs that reused one).
 *  - zolo_submit copies opts and the optional host start block (N x n_ss
 *    row-major, n_ss = opts->n_ss or ceil(1.5 n_lambda_est); NULL draws it
 *    from opts->seed) and returns at once.  The pencil must outlive the query,
 *    and, since resident factorizations and subspaces refer to it, either the
 *    server or a zolo_server_drop_pencil call for it.
 *  - zolo_server_drop_pencil waits until no queued or running query uses the
 *    pencil and frees its resident factorizations and subspaces; afterwards
 *    the pencil may be freed (queries submitted on it later make new ones).
 *  - zolo_wait returns the query's status and hands over its result (freed
 *    by the caller with zolo_result_free); timeout_ms < 0 waits forever; on
 *    ZOLO_ETIMEOUT nothing is handed over and the query keeps running.
 *  - zolo_server_destroy lets running and queued queries finish first; every
 *    query handle of the server must be freed before it.  Functions of one
 *    server may be called from several threads.
 */
typedef struct zolo_server zolo_server;
typedef struct zolo_query zolo_query;
typedef struct {
  double t_submit, t_start, t_end;  /* seconds on a monotonic clock            */
  int batch;                        /* queries in the joint run (1 = alone)    */
  long long est_bytes;              /* admission estimate of the joint run     */
  int done;                         /* 1 once the result is ready              */
} zolo_query_info;
zolo_status zolo_server_create(zolo_ctx* ctx, int slots, size_t hbm_budget_bytes, zolo_server** out);
zolo_status zolo_submit(zolo_server* srv, zolo_pencil* p, double a, double b, int n_lambda_est, const zolo_opts* opts,
                        const double* h_Q0, zolo_query** out);
zolo_status zolo_wait(zolo_query* q, int timeout_ms, zolo_result** out);
zolo_status zolo_query_get_info(const zolo_query* q, zolo_query_info* out);
typedef struct {
  long long budget_bytes;           /* admission budget                       */
  long long running_bytes;          /* estimates of the queries running now   */
  int resident_factors;             /* factorizations kept after their query  */
  long long resident_bytes;
  long long factor_hits;            /* runs that used a resident factorization */
  long long factor_misses;          /* runs that factored                     */
  int queued;
  long long subspace_hits;          /* queries answered from a resident subspace
                                       (eigenpairs of an earlier query for the
                                       same result, residuals recomputed)      */
  int resident_subspaces;
} zolo_server_info;
zolo_status zolo_server_get_info(zolo_server* srv, zolo_server_info* out);
zolo_status zolo_server_drop_pencil(zolo_server* srv, zolo_pencil* p);
/* frees a query handle; waits for the query if it is still queued or running */
void zolo_query_free(zolo_query* q);
void zolo_server_destroy(zolo_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* ZOLO_H */
