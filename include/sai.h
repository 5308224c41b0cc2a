/*
 * sai.h - C ABI of the MI355X (gfx950) SMW-split sparse approximate inverse solver.
 *
 * Method: Jia & Zhang, "An Approach to Making SPAI and PSAI Preconditioning
 * Effective for Large Irregular Sparse Linear Systems" (arXiv:1211.6866).
 * The problem is A x = b with A a real nonsingular n x n sparse matrix
 * (Section 1, (eq:Axb)).  A few irregular (relatively dense) columns of A are
 * split off, A = A~ + U V^T (Section 3, (split)); one sparse approximate
 * inverse M of the regular sparse A~ is built from n independent column
 * least-squares problems (Section 2, (subprob), (lsprob)); the s+1 systems
 * A~ [y, W] = [b, U] are solved by M-preconditioned Krylov iterations under the
 * stopping rules of the Section 4 theorem ((stopb), (stopU2), c = 1); and
 * x = y - W (I + V^T W)^{-1} V^T y is recovered (Procedure *, (update1)).
 *
 * Conventions for every entry point:
 *  - Pointers are DEVICE pointers unless the argument is documented "host".
 *    The caller owns every buffer it passes in; the library never keeps a
 *    pointer to a caller buffer after the call returns.
 *  - `stream` is a hipStream_t passed as void*; all device work is enqueued
 *    on it.  Every call returns after the work that fills its host outputs
 *    has completed (it synchronises the stream at least once).
 *  - Sparse matrices are CSR with int32 row pointers and column indices
 *    (nnz < 2^31), sorted strictly increasing within each row, and float64
 *    values.
 *  - Multi-right-hand-side blocks ("blocks") are n x k, ROW-major (the k
 *    values of one row are contiguous, leading dimension k), float64.
 *  - Device memory the library needs (handles, workspaces) is obtained from
 *    the optional allocator given to sai_split (NULL: hipMalloc/hipFree) and
 *    released through it; the allocator must return 256-byte aligned memory
 *    usable on `stream`.
 *  - Return value: SAI_OK or one of the error codes below.  On an error no
 *    output handle is created; host statistics may be partially filled.
 *    sai_strerror() names a code.  The last error message of the calling
 *    thread is available from sai_last_error().
 */
#ifndef SAI_H
#define SAI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SAI_OK = 0,
  SAI_EINVAL = 1,      /* malformed input (CSR not square/sorted/in range, NaN/Inf, bad option) */
  SAI_EZERODIAG = 2,   /* an irregular column has no diagonal entry (the paper permutes rows first) */
  SAI_ESINGULAR = 3,   /* I + V^T W (or a column LS block) is numerically singular */
  SAI_ENOCONV = 4,     /* maxit reached before the stopping rule held; outputs are still written */
  SAI_EBREAKDOWN = 5,  /* BiCGStab broke down twice on one column; outputs are still written */
  SAI_ENOMEM = 6,      /* an allocation failed */
  SAI_EHIP = 7,        /* a HIP runtime call failed */
  SAI_ETOOBIG = 8      /* a size exceeds a documented kernel limit */
};

typedef void* (*sai_alloc_fn)(void* ctx, size_t bytes, void* stream);
typedef void (*sai_free_fn)(void* ctx, void* ptr, void* stream);
typedef struct {
  sai_alloc_fn alloc; /* NULL: hipMalloc */
  sai_free_fn free;   /* NULL: hipFree */
  void* ctx;
} sai_allocator;

typedef struct sai_split_s sai_split_t;
typedef struct sai_precond_s sai_precond_t;

/* ------------------------------------------------------------------ split --
 * Procedure * step 1 and Section 4 (first and second issues):
 *   p = floor(nnz(A)/n); column j is irregular iff nnz(A(:,j)) > dense_factor*p
 *   (the paper uses 10p); each irregular column keeps its diagonal and the
 *   keep-1 off-diagonal entries nearest to the diagonal (ties: smaller row)
 *   or, with SAI_KEEP_LARGEST, of largest magnitude (ties: smaller row);
 *   keep = p by default (p_hat = p).  U holds the dropped entries, its column
 *   d belonging to the d-th irregular column j_d in ascending order, and
 *   V = (e_{j_1} .. e_{j_s}).  A~ = A - U V^T is formed by copying values.
 * Inputs: A in CSR (device).  Output: *out, a handle owning copies of A~ (CSR
 * and CSC), U (row-ordered CSR with column index d), the j_d and A's sparsity
 * structure (for gradients).  Errors: SAI_EINVAL, SAI_EZERODIAG, SAI_ENOMEM,
 * SAI_EHIP. */
enum { SAI_KEEP_NEAREST = 0, SAI_KEEP_LARGEST = 1 };
typedef struct {
  double dense_factor; /* 10 */
  int32_t keep;        /* <= 0: p */
  int32_t rule;        /* SAI_KEEP_NEAREST | SAI_KEEP_LARGEST */
  /* Optional override of the count rule (host array, not kept after the call):
   * when non-NULL, the s_given columns it lists (strictly ascending, in
   * [0, n)) are the irregular ones whatever their counts; s_given = 0 gives
   * A~ = A.  NULL: columns are classified by dense_factor * p.  Errors:
   * SAI_EINVAL for an unsorted, repeated or out-of-range entry or s_given < 0. */
  const int32_t* host_dense_cols;
  int32_t s_given;
} sai_split_opts;

int sai_split(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
              const double* val, const sai_split_opts* opts, const sai_allocator* alloc,
              void* stream, sai_split_t** out);

/* Read-only views into a split handle (device pointers valid until
 * sai_split_destroy).  U is stored by rows: entries u_row_ptr[i]..u_row_ptr[i+1]
 * of row i have column u_col (an index d in [0, s)) and value u_val. */
typedef struct {
  int32_t n, s, p, keep;
  int64_t nnz_a, nnz_t, nnz_u;
  const int32_t* t_row_ptr;  /* n+1 */
  const int32_t* t_col_idx;  /* nnz_t */
  const double* t_val;       /* nnz_t */
  const int32_t* t_col_ptr;  /* n+1, CSC of A~ (= CSR of A~^T) */
  const int32_t* t_row_idx;  /* nnz_t */
  const double* t_cval;      /* nnz_t */
  const int32_t* dense_cols; /* s, ascending */
  const int32_t* u_row_ptr;  /* n+1 */
  const int32_t* u_col;      /* nnz_u */
  const double* u_val;       /* nnz_u */
} sai_split_info;
int sai_split_get_info(const sai_split_t* h, sai_split_info* info /* host */);
void sai_split_destroy(sai_split_t* h);

/* ------------------------------------------------------------------ build --
 * Builds M ~ A~^{-1} column by column (Section 2, (miniz) -> (subprob) ->
 * (lsprob)): for pattern J_k, I_k = nonzero rows of A~(:,J_k), m_k(J_k) is the
 * least-squares solution of A~(I_k,J_k) m = e_k(I_k), computed by Householder
 * QR and back-substitution.  Patterns:
 *   SAI_PAT_A    J_k = P(A~(:,k))
 *   SAI_PAT_A2   J_k = P(|A~|^2 e_k), structural (Section 2.2, BPSAI envelope, l = 2)
 *   SAI_PAT_SPAI SPAI augmentation (Section 2.1, (candi), (rhoj)) from
 *                P(A~(:,k)) (or {k}), spai_steps steps of spai_per_step indices,
 *                stopping when ||A~ m_k - e_k|| <= delta.  The pattern search
 *                always runs in float64; the final solve in `precision`.
 *   SAI_PAT_PSAI_TOL  PSAI(tol) (Section 2.2): from S = {k}, loops l = 0 ..
 *                psai_lmax add the structural power pattern P(|A~|^(l+1) e_k) to
 *                S, solve on S, drop |m_jk| <= delta / (|S| ||A~||_1) (tolk,
 *                the largest entry kept), and stop once ||A~ m_k - e_k|| <= delta
 *                (the residual before that drop).  Runs in float64; the kept
 *                values are stored in `precision` without a re-solve; `drop`
 *                and `tau` are not used.
 * Dropping after the solve (Section 2.2, (tolk)): SAI_DROP_ABS drops
 * |m_jk| <= tau, SAI_DROP_TOLK drops |m_jk| <= delta/(|J_k| ||A~||_1); the
 * largest entry of each column is always kept; no re-solve.
 * precision: SAI_FP32 builds M in float32 ("mixed"), SAI_FP64 in float64.
 * Errors: SAI_EINVAL, SAI_ESINGULAR (a column block without full column rank),
 * SAI_ETOOBIG (|J_k| > 512 or |I_k| > 8192; in the SPAI and PSAI(tol) searches
 * also more than 65536 gathered row or candidate entries for a column that
 * goes past its first solve; columns within the limits of the fast kernels
 * (|J_k| <= 128, |I_k| <= 2048 and 8192 entries in the searches) run there,
 * the others in a second pass with these larger limits), SAI_ENOMEM, SAI_EHIP. */
enum { SAI_PAT_A = 0, SAI_PAT_A2 = 1, SAI_PAT_SPAI = 2, SAI_PAT_PSAI_TOL = 3 };
enum { SAI_DROP_NONE = 0, SAI_DROP_ABS = 1, SAI_DROP_TOLK = 2 };
enum { SAI_INIT_PATTERN_A = 0, SAI_INIT_DIAG = 1 };
enum { SAI_FP32 = 0, SAI_FP64 = 1 };
typedef struct {
  int32_t pattern;
  int32_t drop;
  double tau;           /* SAI_DROP_ABS threshold, 1e-3 */
  double delta;         /* SPAI stop / SAI_DROP_TOLK, 0.4 */
  int32_t spai_steps;   /* 3 */
  int32_t spai_per_step;/* 5 */
  int32_t spai_init;    /* SAI_INIT_PATTERN_A | SAI_INIT_DIAG */
  int32_t precision;    /* SAI_FP32 | SAI_FP64 */
  int32_t keep_lists;   /* nonzero: keep J_k, I_k, pre-drop m_k and res_k for inspection */
  int32_t psai_lmax;    /* SAI_PAT_PSAI_TOL: last loop index l_max, in [0, 64]; 10 */
} sai_build_opts;

typedef struct {
  int32_t n;
  int64_t nnz_m;          /* after dropping */
  int64_t nnz_m_full;     /* sum |J_k| before dropping */
  int64_t sum_i;          /* sum |I_k| */
  int32_t max_i, max_j;
  int32_t n_c;            /* columns with res_k > delta */
  double spar;            /* nnz(M) / nnz(A~) */
  int64_t bucket_cols[16]; /* columns per LS kernel variant (in the order of the
                             precision's variant table, the global-memory kernel
                             last; unused slots 0) */
  float t_pattern_ms, t_ls_ms, t_assemble_ms, t_total_ms;
  int32_t s, p;           /* of the split: irregular columns, floor(nnz(A)/n) */
  int32_t l_m;            /* most loops a column used (Table 5's l_m): PSAI(tol)
                             loops run (1 .. psai_lmax + 1); SPAI augmentation
                             steps taken (0 .. spai_steps); 0 for static patterns */
  int64_t drop_flips;     /* entries whose keep/drop decision the build precision
                             cannot settle: | |m_jk| - tol_k | <= eta ||m_k|| /
                             (1 - eta) with eta = 1e-4 (SAI_FP32) or 1e-12
                             (SAI_FP64), the always-kept largest entry excluded;
                             0 without a drop after the solve.  If every column
                             is within eta ||m'_k|| of an exact column m'_k, the
                             exact dropping can differ only on these entries. */
} sai_build_stats;

int sai_build(const sai_split_t* sp, const sai_build_opts* opts, void* stream,
              sai_precond_t** out, sai_build_stats* stats /* host, may be NULL */);

/* Views into a preconditioner handle.  M in CSC (column k = m_k; = CSR of M^T)
 * and CSR; values are float or double per `precision`.  When built with
 * keep_lists: j_ptr/j_idx (int64 offsets, int32 entries) hold J_k, i_ptr/i_idx
 * hold I_k, m_full holds m_k on J_k before dropping (same value type), res
 * the LS residual norms ||A~ m_k - e_k|| (float64, before dropping); otherwise
 * those are NULL.  For SAI_PAT_PSAI_TOL, J_k and m_full are the final (dropped)
 * pattern and values and res the residual of the last solve before its drop. */
typedef struct {
  int32_t n, precision;
  int64_t nnz;
  const int32_t* col_ptr;
  const int32_t* row_idx;
  const void* cval;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const void* val;
  const int64_t* j_ptr;
  const int32_t* j_idx;
  const int64_t* i_ptr;
  const int32_t* i_idx;
  const void* m_full;
  const double* res;
} sai_precond_info;
int sai_precond_get_info(const sai_precond_t* h, sai_precond_info* info /* host */);
void sai_precond_destroy(sai_precond_t* h);

/* ----------------------------------------------------------------- gather --
 * The gather step on its own (Section 2, (lsprob): the dense block
 * A~(I_k, J_k) of every column's least-squares problem, with I_k the nonzero
 * rows of A~(:, J_k)).  The column solvers of sai_build gather these blocks
 * internally; these calls write them out, for inspection and for other
 * solvers.  `pc` must have been built with keep_lists (its J_k and I_k are
 * used); otherwise SAI_EINVAL.
 * sai_gather_offsets: blk_off (device, n + 1 int64) = exclusive prefix sums of
 * |I_k| |J_k|; *total (host, may be NULL) = blk_off[n].
 * sai_gather: writes block k column-major (element (r, c) = A~(I_k[r], J_k[c]),
 * leading dimension |I_k|) at element offset blk_off[k] of `blocks` (device,
 * blk_off[n] elements of float for SAI_FP32 or double for SAI_FP64, owned by
 * the caller).  Values are copies (rounded to float for SAI_FP32). */
int sai_gather_offsets(const sai_precond_t* pc, int64_t* blk_off, int64_t* total /* host */,
                       void* stream);
int sai_gather(const sai_split_t* sp, const sai_precond_t* pc, int32_t precision,
               const int64_t* blk_off, void* blocks, void* stream);

/* ----------------------------------------------------------------- krylov --
 * Solves A~ X = R (transpose = 0) or A~^T X = R (transpose = 1, with M^T as
 * preconditioner) for the k columns of the block R independently, right-
 * preconditioned, x_0 = 0 (Section 3 (regprob), (auxi); Section 5 solver
 * settings).  Column c stops when its true residual norm is < thr[c] (host
 * array of k absolute thresholds; the Section 4 theorem gives them, see
 * sai_solve).  Methods: SAI_BICGSTAB (van der Vorst, r_hat = r_0; one restart
 * with r_hat = r on breakdown; residual replacement when a recursive residual
 * passes but the true one does not) or SAI_GMRES (GMRES(restart), restart in
 * [1, 64]; Arnoldi with Givens rotations, x updated and the true residual
 * checked at the end of each cycle; a column leaves a cycle early when its
 * rotated residual estimate passes thr[c]).  GMRES runs the k columns in
 * lockstep (shared sparse products, Gram-Schmidt twice) once n k >= 32768, else
 * one workgroup per column (modified Gram-Schmidt); the two round differently.
 * iters/status: host arrays of k entries (may be NULL); status per column is
 * 0 converged, 1 maxit, 2 breakdown.  Returns SAI_ENOCONV / SAI_EBREAKDOWN if
 * any column ended that way (X is written in every case).  Any k >= 1: up to
 * 64 columns run as one lockstep solve, wider blocks in groups of 64 columns
 * one after the other (sai_solve and sai_backward pass s + 1 columns, so s is
 * not limited by the solver; the allocation-free SMW below takes s <= 64). */
enum { SAI_BICGSTAB = 0, SAI_GMRES = 1 };
enum { SAI_C_ONE = 0, SAI_C_ONE_THEN_REFINE = 1 };
typedef struct {
  int32_t method;   /* SAI_BICGSTAB | SAI_GMRES */
  int32_t restart;  /* GMRES(m): 30 */
  double eps;       /* 1e-8 */
  int32_t maxit;    /* 500 */
  int32_t c_mode;   /* SAI_C_ONE (paper) | SAI_C_ONE_THEN_REFINE */
  int32_t equilibrate; /* sai_solve only; 0: b as given; 1: Section 4's scaling:
                          solve A (alpha x) = alpha b with alpha = rho / ||b||,
                          rho = ||A||_F / sqrt(n) (the root-mean-square column norm
                          of A), so that ||alpha b|| is comparable to the column
                          norms and hence to the ||u_j||; x is scaled back.  rr is
                          the same relative residual. */
} sai_solve_opts;

int sai_krylov(const sai_split_t* sp, const sai_precond_t* pc, int32_t transpose, int32_t k,
               const double* R, double* X, const double* thr /* host, k */,
               const sai_solve_opts* opts, void* stream, int32_t* iters /* host */,
               int32_t* status /* host */);

/* -------------------------------------------------------------------- smw --
 * Procedure * step 3, (update1) / (composi): Y = [y_hat, W_hat] is an
 * n x (s+1) block (row-major); forms K = I + W_hat(j_d, :), solves
 * K z = y_hat(j_d) by LU with partial pivoting in float64 and writes
 * x = y_hat - W_hat z; c = ||z|| (host, may be NULL).  Errors: SAI_ESINGULAR
 * (a zero pivot; by Theorem 3.1 A is then singular). */
int sai_smw(const sai_split_t* sp, const double* Y, double* x, double* c /* host */,
            void* stream);

/* sai_smw for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * recovery and results as sai_smw, with no hipMalloc, hipFree or allocating
 * library call.  Its workspace (K, z and the pivot flag, 33,536 bytes) is a
 * file-scope device array that each GPU holds until the process ends; every
 * call on one GPU shares it, so calls that overlap on one GPU race.  Arguments
 * as for sai_smw (Y, x device; c host, may be NULL).  Errors: SAI_ETOOBIG for
 * s > 64, SAI_ESINGULAR for a zero pivot, SAI_EINVAL for a NULL argument. */
int sai_smw_noalloc(const sai_split_t* sp, const double* Y, double* x, double* c /* host */,
                    void* stream);

/* rr = ||b - A x|| / ||b|| with A = A~ + U V^T (rrnorm), in float64. */
int sai_residual(const sai_split_t* sp, const double* b, const double* x,
                 double* rr /* host */, void* stream);

/* ------------------------------------------------------------------ solve --
 * Procedure * end to end for one right-hand side b (device, n): solves
 * A~ [y, W] = [b, U] with thresholds (eps/2)||b|| for y (stopb) and
 * eps ||b|| / (2 sqrt(s) c) for each w_j (stopU2) with c = 1, recovers x
 * (device, n) and computes rr.  With SAI_C_ONE_THEN_REFINE, if rr >= eps and
 * c > 1 the s auxiliary solves are continued to the thresholds with the
 * computed c and x is recovered again. */
typedef struct {
  int32_t s;
  int32_t status;       /* SAI_OK / SAI_ENOCONV / SAI_EBREAKDOWN */
  int32_t iters_max;    /* max over the s+1 systems */
  int32_t* iters;       /* host array of s+1 entries to fill, or NULL */
  double rr, a, c;      /* rr, a = rr/eps, c = ||(I + V^T W)^{-1} V^T y|| */
  float t_solve_ms, t_smw_ms, t_check_ms;
} sai_solve_stats;

int sai_solve(const sai_split_t* sp, const sai_precond_t* pc, const double* b, double* x,
              const sai_solve_opts* opts, void* stream, sai_solve_stats* stats /* host */);

/* sai_solve, with the s+1 Krylov solutions Y = [y, W] (device, n x (s+1),
 * row-major, caller-owned; W approximates A~^{-1} U, y the solution of
 * A~ y = b, of the scaled b under `equilibrate`) written to Y instead of a
 * workspace, for sai_backward_y.  Errors as sai_solve; SAI_EINVAL for a NULL Y. */
int sai_solve_y(const sai_split_t* sp, const sai_precond_t* pc, const double* b, double* x,
                double* Y, const sai_solve_opts* opts, void* stream,
                sai_solve_stats* stats /* host */);

/* --------------------------------------------------------------- backward --
 * Gradient of a scalar loss L(x), x = A^{-1} b, given grad_x = dL/dx (device,
 * n).  Derived from Theorem 3.1 applied to A^T = A~^T + V U^T: solves
 * A~^T [eta, Z] = [grad_x, V] with M^T as right preconditioner under the
 * same stopping rules (column 0: (eps/2)||grad_x||; columns e_{j_d}:
 * eps ||grad_x|| / (2 sqrt(s))), then lambda = eta - Z (I + U^T Z)^{-1} U^T eta.
 * With SAI_C_ONE_THEN_REFINE, if c' = ||(I + U^T Z)^{-1} U^T eta|| > 1 the s
 * auxiliary solves are continued to eps ||grad_x|| / (2 sqrt(s) c') (the unit
 * right-hand sides e_{j_d} are not scaled like grad_x, so c = 1 can leave the
 * adjoint residual well above eps) and lambda is formed again; stats->c = c'.
 * Writes grad_b = lambda (device, n) and grad_a_val[e] = -lambda_i x_j for the
 * e-th stored entry (i, j) of the A given to sai_split (device, nnz(A), A's
 * CSR order).  Either output may be NULL. */
int sai_backward(const sai_split_t* sp, const sai_precond_t* pc, const double* x,
                 const double* grad_x, double* grad_b, double* grad_a_val,
                 const sai_solve_opts* opts, void* stream, sai_solve_stats* stats /* host */);

/* The same gradients from the forward solve's W (Y of sai_solve_y on this split
 * and preconditioner; only Y[:, 1..s] is read; Y may be NULL when s = 0), with
 * one system with A~^T per pass instead of s+1.  Theorem 3.1's
 * A^{-1} = A~^{-1} - W K^{-1} V^T A~^{-1}, K = I + V^T W, transposes to
 * A^{-T} = A~^{-T} (I - V K^{-T} W^T).  Pass p solves A~^T d = r - V z,
 * K^T z = W^T r, with M^T as right preconditioner and adds d to lambda; r is
 * grad_x in the first pass, then the true residual grad_x - A~^T lambda -
 * V (U^T lambda) (float64).  The passes stop once that residual is below
 * eps ||grad_x||, at most 4.  After a pass it is (I + V W^T) r_s - V R^T d
 * (r_s the solve's residual, R = U - A~ W the forward's auxiliary residuals,
 * d the pass's solution); the second term usually keeps the first pass above
 * eps and the next pass removes it.  The first solve stops at
 * (eps/2)||grad_x||, each later one at (eps/2)||grad_x|| / a with
 * a = max(1, ||(I + V W^T) r_s|| / ||r_s||) of the pass before.  stats: iters[0]
 * = the iterations of all passes (iters[1..s] = 0), rr = the final adjoint
 * residual ||grad_x - A^T lambda|| / ||grad_x||, c = ||z|| of the first pass,
 * t_check_ms = the residual checks, t_smw_ms = the corrections; c_mode and
 * equilibrate are not used.  Outputs as sai_backward (written also when the
 * status is not SAI_OK).  Errors: SAI_ENOCONV when 4 passes leave the residual
 * at or above eps, SAI_EBREAKDOWN, SAI_ESINGULAR for a zero pivot of K^T,
 * SAI_EINVAL for a NULL argument (Y with s > 0) or a non-finite grad_x. */
int sai_backward_y(const sai_split_t* sp, const sai_precond_t* pc, const double* x,
                   const double* Y, const double* grad_x, double* grad_b, double* grad_a_val,
                   const sai_solve_opts* opts, void* stream, sai_solve_stats* stats /* host */);

/* -------------------------------------------------------------- profiling --
 * While enabled, the library records a pair of HIP events on the launch stream
 * around each of its kernel launches and accumulates, per kernel name, the
 * number of launches and their total elapsed time.  sai_profile_enable(1)
 * records every kernel, sai_profile_enable(2) only the sparse products, column
 * solvers, SPAI search and GMRES (less event overhead), sai_profile_enable(3)
 * only the kernels whose name starts with the prefix given to
 * sai_profile_only (host string, copied; "" matches every name), 0 stops;
 * enabling resets the totals; sai_profile_get resolves pending events (it
 * waits for them) and returns entry i (0 <= i < sai_profile_count()).  Not
 * thread-safe with respect to concurrent launches from several host threads. */
int sai_profile_enable(int32_t on);
int sai_profile_only(const char* prefix /* host */);
int sai_profile_count(void);
int sai_profile_get(int32_t i, char* name /* host, name_cap bytes */, int32_t name_cap,
                    int64_t* launches /* host */, double* total_ms /* host */);

/* ---------------------------------------------------------------- tuning --
 * Launch-shape knobs of the kernels (gather batch sizes, grid shapes, workgroup
 * sizes; names in upper case, e.g. "SPMM_M", "XMAP", "SGRID", "NARROW_MIN",
 * "PSAI_NT").  A knob's value is taken from the environment variable
 * SAI_TUNE_<name> if set, else from sai_tune_set, else the built-in default.
 * They change speed, not results beyond the order of floating-point sums
 * (every setting is deterministic).  The Python package's autotuner measures
 * the variants on one device and stores its choices in a JSON file that the
 * binding passes to sai_tune_set at load.  sai_tune_get reports the value a
 * kernel would use (dflt when none is set).  Errors: SAI_EINVAL (a name that
 * is empty, longer than 63 characters or not [A-Z0-9_]).  Process-wide,
 * thread-safe; a value takes effect at the next launch. */
int sai_tune_set(const char* name /* host */, int32_t value);
int sai_tune_get(const char* name /* host */, int32_t dflt, int32_t* value /* host */);
int sai_tune_clear(void);

/* ------------------------------------------------------------------ misc --*/
const char* sai_strerror(int code);
const char* sai_last_error(void);
/* Device-to-device copy on `stream` (used by bindings to export handle views). */
int sai_memcpy_d2d(void* dst, const void* src, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SAI_H */
