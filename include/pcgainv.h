/*
 * pcgainv.h -- C ABI of the MI355X PCG-AINV solver for the five-point
 * elliptic sea-surface system.
 *
 * Method: preconditioned conjugate gradient (Algorithm 1 of Cuomo, De Michele,
 * Farina, Chinnici, "A PCG implementation of an elliptic kernel in an ocean
 * global circulation model based on GPU libraries") with the factored
 * approximate inverse P = Z D^-1 Z^T ~ A^-1 (Sec. 3-4), where Z is unit upper
 * triangular and is computed by A-orthogonalisation with a drop tolerance
 * (the AINV of the paper's ref. [book4-14]; the threshold variant is the
 * "drop tolerance" Bridson class discussed in Sec. 5).
 *
 * Conventions shared by every call
 *   - All functions return an int status: PCGA_OK (0), PCGA_NOCONV (1, a
 *     result is still produced), or a negative error code.  No function
 *     aborts or throws across the ABI; pcga_strerror() names the code and
 *     pcga_last_error() gives a message for the calling thread.
 *   - Host pointers are plain C arrays owned by the caller.  Device pointers
 *     are HIP device addresses on the current device, owned by the caller.
 *   - The library never allocates device memory.  The caller provides one
 *     device workspace per solver (size from pcga_workspace_bytes) and
 *     keeps it alive until pcga_solver_destroy.  The library allocates only
 *     small host and pinned-host buffers of its own.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream.  All device work of a solver is ordered on its stream.
 *
 * Grid and storage (the natural ordering of Sec. 3: west->east, then
 * south->north).  Cell (i, j), 0 <= i < nx, 0 <= j < ny, has index
 * k = j*nx + i.  The operator is the symmetric positive definite negation of
 * eq. (10): A[k,k] = sum of the cell's face coefficients, A[k,nbr] = -c_face.
 * It is passed in "A5" form: three arrays of n = nx*ny doubles,
 *   diag[k] = A[k,k],  ae[k] = A[k, east(k)],  an[k] = A[k, k+nx],
 * where east(k) of a cell with i = nx-1 is the cell with i = 0 of the same
 * row when PCGA_PERIODIC_X is set (east-west periodic globe), and does not
 * exist otherwise (then ae[k] must be 0).  an[k] of the last row must be 0.
 * Land cells are identity rows (diag 1, no couplings) with zero right-hand
 * side.
 */
#ifndef PCGAINV_H
#define PCGAINV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PCGA_OK 0
#define PCGA_NOCONV 1       /* maxit / max_outer reached; x and history valid */
#define PCGA_EINVAL (-1)    /* bad shape, pointer, flag or non-5-point input  */
#define PCGA_EBREAKDOWN (-2)/* pivot p_i <= 0 in setup, or (d,q) <= 0 / rho <= 0 */
#define PCGA_ENAN (-3)      /* NaN or Inf met in the iteration               */
#define PCGA_EHIP (-4)      /* HIP runtime error; see pcga_last_error()       */
#define PCGA_ENOMEM (-5)    /* workspace too small or host allocation failed  */

#define PCGA_PERIODIC_X 1u

/* precision of a solver */
#define PCGA_FP64 0         /* A, Z, vectors and scalars in FP64              */
#define PCGA_MIXED 1        /* FP32 inner PCG (Z, D^-1, vectors; the FP64     */
                            /* operator applied to FP32 vectors), FP64        */
                            /* scalars, residual, solution and refinement     */
#define PCGA_MIXED_A32 2    /* as PCGA_MIXED with the inner operator in FP32  */
                            /* too (coefficients rounded, q = A d summed in   */
                            /* FP32): every inner datum FP32; FP64 kept for   */
                            /* the residual, the solution and alpha/beta      */

typedef struct pcga_a5 {
    int32_t nx, ny;
    uint32_t flags;         /* PCGA_PERIODIC_X or 0 */
    const double *diag, *ae, *an;  /* host, n = nx*ny each, caller-owned */
} pcga_a5_t;

/* A general sparse SPD operator in CSR, for matrices that do not come from
 * the grid (the comparison of Sec. 5 also uses one): n rows; rowptr[n+1]
 * (rowptr[0] = 0, non-decreasing); col[rowptr[n]] with the columns of each
 * row strictly ascending; val[rowptr[n]].  The diagonal must be present and
 * positive, every value finite, and A symmetric entry by entry (A[i,j] ==
 * A[j,i] bitwise); the calls check this and return PCGA_EINVAL otherwise.
 * Host arrays, caller-owned.  n <= 2^31 - 1. */
typedef struct pcga_csr {
    int64_t n;
    const int64_t *rowptr;
    const int32_t *col;
    const double *val;
} pcga_csr_t;

typedef struct pcga_ainv pcga_ainv_t;       /* opaque host (Z, D) */
typedef struct pcga_solver pcga_solver_t;   /* opaque device solver */

const char *pcga_strerror(int status);
const char *pcga_last_error(void);

/* Streams for callers that run several solvers or batches concurrently
 * (for instance continuous batching of time-step solves).
 * pcga_stream_create makes a stream on the calling thread's current device,
 * non-blocking with respect to the null stream, at the default priority.
 * The HIP runtime gives a process a fixed number of hardware queues
 * (GPU_MAX_HW_QUEUES) and binds each new stream to the queue that has the
 * fewest streams; work on two streams bound to one queue runs one after the
 * other.  Streams made together, after the process's other streams, thus
 * land on distinct queues (up to the queue count), which streams taken from
 * a framework's pool need not do.  The caller owns the stream (*stream;
 * NULL on error) and passes it where a call takes `stream`.
 * pcga_stream_destroy waits for the stream's work, then destroys it; every
 * solver or batch made on it must be destroyed first (NULL: no-op).
 * Errors: EINVAL (stream NULL), EHIP. */
int pcga_stream_create(void **stream);
int pcga_stream_destroy(void *stream);

/* ---- preconditioner setup (host, FP64) ---------------------------------
 * pcga_ainv_setup: A-orthogonalisation of A with drop tolerance `drop_tol`
 * (Sec. 3-5; ref. [book4-14]).  Z := I; for i = 0..n-1 (natural order):
 * p_i = a_i^T z_i (row i of A, columns ascending); every later column z_j
 * with c_j = a_i^T z_j != 0 is updated z_j <- z_j - (c_j/p_i) z_i, after
 * which its touched off-diagonal entries with |z| < drop_tol or z == 0 are
 * removed (an entry equal to drop_tol is kept).  D = diag(p).
 * drop_tol = 0 gives the exact inverse factor; drop_tol = +inf gives Z = I,
 * D = diag(A) (the diagonal preconditioner of eq. (11)-(12)).
 * Deterministic: unfused FP64 in a fixed operation order.
 * Errors: EINVAL (shape/flags/negative tol/A5 edge rules), EBREAKDOWN
 * (p_i <= 0: A is not an M/H-matrix), ENOMEM.  On error *out is NULL.
 */
int pcga_ainv_setup(const pcga_a5_t *A, double drop_tol, pcga_ainv_t **out);

/* pcga_ainv_setup_fill: the fixed-fill form, the second Bridson class of
 * Sec. 5 (a set number of nonzeros in each row of the lower factor Z^T, i.e.
 * each column of Z).  The same A-orthogonalisation as pcga_ainv_setup, with
 * drop_tol applied after every update as there (0 disables it); in addition,
 * when column z_j has received all its updates it keeps only its `max_fill`
 * off-diagonal entries of largest magnitude (equal magnitudes: the larger
 * row, nearer the diagonal, first), and p_j is formed from the capped
 * column.  max_fill = 0 gives Z = I, D = diag(A); a cap above the longest
 * column of the threshold factor gives that factor bitwise.  Every row of Z^T
 * then has at most max_fill off-diagonal entries.  Deterministic.
 * Errors: EINVAL (as pcga_ainv_setup, or max_fill < 0), EBREAKDOWN, ENOMEM.
 * On error *out is NULL (when out is not). */
int pcga_ainv_setup_fill(const pcga_a5_t *A, double drop_tol, int32_t max_fill,
                         pcga_ainv_t **out);

/* pcga_fsai_band_setup: the paper's own preconditioner (Sec. 3, six-step
 * scheme; Propositions 2-3): the factored approximate inverse of T, the part
 * of A with |col - row| <= 1 in natural ordering (east-west couplings inside
 * each grid row), with band q: column z_j keeps rows j-q .. j (entries with
 * j > i + q are the negligible set) and is computed by T-orthogonalisation on
 * that pattern; D = diag(p).  The result is used like an AINV factor
 * (P = Z D^-1 Z^T).  q = 0 gives Jacobi.  Errors: EINVAL (A5 rules, q outside
 * 0..4096), EBREAKDOWN (a pivot <= 0), ENOMEM. */
int pcga_fsai_band_setup(const pcga_a5_t *A, int32_t q, pcga_ainv_t **out);

/* Sizes of a setup result: n and the number of stored off-diagonal entries
 * of Z (the unit diagonal is implicit). */
/* pcga_ainv_setup_csr: the same A-orthogonalisation on a CSR operator (the
 * rows of A in their stored, ascending column order): Z, D with
 * Z D^-1 Z^T ~ A^-1.  max_fill >= 0 keeps at most that many off-diagonal
 * entries per column of Z (the fixed-fill class of Sec. 5), < 0 no cap.
 * Errors: EINVAL (A fails the CSR checks, drop_tol < 0), EBREAKDOWN,
 * ENOMEM. */
int pcga_ainv_setup_csr(const pcga_csr_t *A, double drop_tol, int32_t max_fill,
                        pcga_ainv_t **out);

int pcga_ainv_info(const pcga_ainv_t *F, int64_t *n, int64_t *nnz_off);

/* Export Z (strict upper part) in CSC with rows ascending in each column:
 * colptr[n+1], rowidx[nnz_off], val[nnz_off]; and D[n].  Any pointer may be
 * NULL to skip that array. */
int pcga_ainv_export(const pcga_ainv_t *F, int64_t *colptr, int32_t *rowidx,
                     double *val, double *D);

/* Build (Z, D) from caller-given CSC data (strict upper part of a unit upper
 * triangular Z, rows ascending per column, plus D > 0).  Lets a caller use a
 * factor computed elsewhere, e.g. the paper's banded factor of T. */
int pcga_ainv_import(int64_t n, const int64_t *colptr, const int32_t *rowidx,
                     const double *val, const double *D, pcga_ainv_t **out);

int pcga_ainv_free(pcga_ainv_t *F);

/* pcga_layout_info: host-only inspection of the sliced-ELL layouts a solver
 * would build from F at target width slice_width (0: the FP64 default, else
 * 1..64); no device is needed.  out[12] receives, for Z^T (out[0..5]) and Z
 * (out[6..11]): slices, slices stored with an offset table, the widest such
 * slice in entry steps (at most 64: a table sits in one wavefront register),
 * the widest slice, stored entries (with padding), and index bytes (2 or 4).
 * Errors: EINVAL (NULL, bad width, or a layout that breaks its invariants),
 * ENOMEM. */
int pcga_layout_info(const pcga_ainv_t *F, int32_t slice_width, int64_t *out);

/* ---- device solver ------------------------------------------------------
 * pcga_workspace_bytes: device bytes needed for (A, F, precision).
 * pcga_solver_create: validate, lay A and (Z, D) out in the workspace
 * (row-major A5 arrays; Z^T and Z in sliced ELL with per-slice lanes per
 * row), and bind the stream.  The solver keeps no pointer to A or F.
 * The workspace must be 256-byte aligned.  A base on a 16 MiB boundary is
 * recommended for FP64.  The part of the workspace kept in the 256 MiB
 * memory-side cache nearly fills it, so its starting address matters: at
 * 1442x1021 an FP64 iteration measured 96-98 us from such a base and
 * 102-106 us from some other 1 MiB multiples.
 * Errors: EINVAL, ENOMEM (bytes too small), EHIP.
 */
int pcga_workspace_bytes(const pcga_a5_t *A, const pcga_ainv_t *F, int precision,
                         size_t *bytes);
int pcga_solver_create(const pcga_a5_t *A, const pcga_ainv_t *F, int precision,
                       void *dev_workspace, size_t bytes, void *stream,
                       pcga_solver_t **out);
int pcga_solver_destroy(pcga_solver_t *S);

/* A solver for a CSR operator (see pcga_csr_t): A is laid out in the same
 * sliced ELL as Z (its diagonal among the entries, 32-bit columns or
 * per-slice offset tables), and each iteration's first kernel forms
 * d = s + beta d at every row it gathers while it computes q = A d.
 * precision must be PCGA_FP64; slice_width as in pcga_solver_create_ex (0:
 * default).  The solve calls (pcga_pcg_solve, pcga_pcg_solve_noalloc),
 * pcga_apply_a, pcga_apply_prec, pcga_profile_iteration, pcga_solver_info,
 * pcga_solver_tune, pcga_solver_set_grids (g_stencil then sets the operator
 * kernel's workgroups), pcga_ts_eta and pcga_ts_guess work on it;
 * pcga_step_stencil, pcga_ts_rhs and batches need the five-point operator
 * and return PCGA_EINVAL.  Errors as pcga_solver_create. */
int pcga_workspace_bytes_csr(const pcga_csr_t *A, const pcga_ainv_t *F, int precision,
                             int32_t slice_width, size_t *bytes);
int pcga_solver_create_csr(const pcga_csr_t *A, const pcga_ainv_t *F, int precision,
                           int32_t slice_width, void *ws, size_t bytes, void *stream,
                           pcga_solver_t **out);
/* The same with the sliced-ELL target width (1..64; 0: the default, 24 for
 * PCGA_FP64 and PCGA_MIXED): a slice
 * starts with one lane per row and doubles its lanes per row (halving its
 * rows) until its longest row needs at most slice_width entry steps (or one
 * row has all 64 lanes).  Results are the same method; the summation order
 * inside a row, and so the rounding, depends on the width.  An autotuner
 * picks it by timing (paper_1210_1878_amd/autotune.py). */
int pcga_workspace_bytes_ex(const pcga_a5_t *A, const pcga_ainv_t *F, int precision,
                            int32_t slice_width, size_t *bytes);
int pcga_solver_create_ex(const pcga_a5_t *A, const pcga_ainv_t *F, int precision,
                          int32_t slice_width, void *dev_workspace, size_t bytes, void *stream,
                          pcga_solver_t **out);

/* Solver facts: n, nnz_off, precision, the modelled device bytes one PCG
 * iteration must move (each array once; FP64: 144 n + (8 + b) nnz_pad, mixed
 * inner: 84 n + (4 + b) nnz_pad, with the FP64 coefficients read by the
 * stencil; nnz_pad = stored sliced-ELL entries of Z^T
 * plus Z, b = index bytes) and b itself: 2 when every stored entry of Z lies
 * within 65535 rows of its row (16-bit distances), else 4 (32-bit columns);
 * formats[0], formats[1]: how Z^T and Z are stored and read (bit 0: 16-bit
 * distances; bit 1: indices, bit 2: values read with non-temporal loads,
 * chosen so that the rest of an iteration's data fits the 256 MiB
 * memory-side cache; formats[0] only: bit 3, the solution x read and
 * written with non-temporal loads and stores, bit 4, the update
 * x += alpha d of Algorithm 1 applied by the next iteration's five-point
 * kernel instead of the Z^T kernel, which then reads neither d nor x: the
 * FP64 solves and the FP32 inner iterations of the mixed solves of a
 * five-point operator with a sliced-ELL Z, where the bytes above count one
 * vector pass less, 136 n and 80 n; formats[1] only: bit 5, the values of
 * Z's table steps read from Z^T's value array, FP64); formats[2]:
 * q when every entry of Z lies within q <= 8
 * rows above the diagonal (e.g. the banded factor of T), which the solve
 * then applies from diagonals (no index arrays, no gathers), else 0.  Any
 * output pointer may be NULL. */
int pcga_solver_info(const pcga_solver_t *S, int64_t *n, int64_t *nnz_off,
                     int32_t *precision, double *bytes_per_iter, int32_t *index_bytes,
                     int32_t *formats);

/* Launch tuning (set by the autotuner): iterations per chunk (even,
 * 2..512), whether chunks are replayed through a captured HIP graph (1) or
 * launched directly (0), and the maximum number of workgroups per kernel
 * (8..2048; 0 selects the default, 1280 for PCGA_FP64 and 1536 for
 * PCGA_MIXED; each workgroup streams one contiguous range of the grid).
 * Takes effect at the next solve.  Results of a solve are bitwise
 * reproducible for fixed settings. */
int pcga_solver_tune(pcga_solver_t *S, int32_t chunk, int32_t use_graph, int32_t max_blocks);
/* Workgroups per launch of each kernel of an iteration, for kernels whose
 * register use allows a different occupancy than the others: g_stencil for
 * the five-point kernels (also the residual passes), g_zt for the Z^T sweep,
 * g_z for the Z sweep; each 1..2048, or 0 for the max_blocks of
 * pcga_solver_tune.  Each count is capped by the work there is (a workgroup
 * per 256 cells, or per four slices).  Results depend on the counts only
 * through the order in which per-workgroup partial sums are added.  Errors:
 * EINVAL, EHIP. */
int pcga_solver_set_grids(pcga_solver_t *S, int32_t g_stencil, int32_t g_zt, int32_t g_z);

/* ---- solves --------------------------------------------------------------
 * pcga_pcg_solve: Algorithm 1 with s = Z D^-1 Z^T r and the direction update
 * d_{k+1} = s_{k+1} + beta_k d_k.  b_dev, x_dev: n FP64 device values; x_dev
 * holds x0 on entry and x on return.  Stops when ||r_k||/||b|| <= tol
 * (recursive residual, 2-norm) or k = maxit (maxit < 0 means n).
 * hist_host (capacity hist_cap, may be NULL) receives ||r_k||/||b|| for
 * k = 0..iters (truncated to hist_cap); *hist_len = iters + 1.
 * *true_relres = ||b - A x||/||b|| recomputed in FP64 (NULL to skip).
 * ||b|| = 0 gives x = 0, iters = 0, hist = {0}.
 * Returns OK, NOCONV, EBREAKDOWN, ENAN, EINVAL (wrong precision), EHIP.
 * Requires a PCGA_FP64 solver.  The call returns after the solve finished.
 */
int pcga_pcg_solve(pcga_solver_t *S, const double *b_dev, double *x_dev, double tol,
                   int32_t maxit, int32_t *iters, double *hist_host, int32_t hist_cap,
                   int32_t *hist_len, double *true_relres);

/* pcga_pcg_solve_noalloc: pcga_pcg_solve for callers that cannot allocate
 * device memory while they run (serving loops that must not allocate, code
 * next to a stream capture, harnesses that forbid allocation).  Same
 * arguments, method, results and status codes as pcga_pcg_solve, and the
 * same kernels; it allocates nothing and captures no graph: the kernels are
 * launched directly, and the solve's vectors (r, s, d, q, t), partial sums
 * and control block live in one static device array of the library,
 * PCGA_NOALLOC_MAX_BYTES per device (held from the library's load until the
 * process ends), instead of the solver's workspace.  x_dev is the iterate
 * itself (it must not alias b_dev).  The solver's operator and factor are
 * read from its workspace as usual.
 * Limit: a grid needs about 56 n bytes of the array (seven FP64 vectors plus
 * about 130 KB of partial sums and control block), so n up to about 1.19 M
 * cells; a larger grid returns PCGA_ENOMEM with a message and no device work.
 * Every call on one device uses that device's array, which keeps the last
 * call's contents (each solve initialises what it reads): calls that overlap
 * on one device, from several threads or streams, race.  Returns as
 * pcga_pcg_solve, plus ENOMEM for a grid beyond the limit. */
#define PCGA_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int pcga_pcg_solve_noalloc(pcga_solver_t *S, const double *b_dev, double *x_dev, double tol,
                           int32_t maxit, int32_t *iters, double *hist_host, int32_t hist_cap,
                           int32_t *hist_len, double *true_relres);

/* pcga_pcg_solve_mixed: FP64 iterative refinement.  Outer step o: r = b - A x
 * in FP64; stop if ||r||/||b|| <= tol; else solve A e = r with the FP32
 * inner PCG (FP32 Z, D^-1 and vectors; q = A d with the FP64 coefficients,
 * rounded to FP32; FP64 alpha/beta/rho and dot sums)
 * to relative residual inner_tol (at most inner_maxit iterations, < 0: n),
 * then x += e in FP64.  At most max_outer corrections.  hist_host receives
 * the outer true residuals ||b - A x_o||/||b||, o = 0..*outer.
 * Requires a PCGA_MIXED solver. */
int pcga_pcg_solve_mixed(pcga_solver_t *S, const double *b_dev, double *x_dev,
                         double tol, double inner_tol, int32_t max_outer,
                         int32_t inner_maxit, int32_t *outer, int32_t *inner_total,
                         double *hist_host, int32_t hist_cap, int32_t *hist_len,
                         double *true_relres);

/* pcga_pcg_solve_mixed_ex: pcga_pcg_solve_mixed with a choice of refinement.
 * refine = PCGA_REFINE_RESTART: as pcga_pcg_solve_mixed (every inner PCG
 *   starts from e = 0, d = s).
 * refine = PCGA_REFINE_KEEP: the inner direction is kept across corrections
 *   (reliable updates, Sleijpen and van der Vorst 1996).  Each inner run
 *   stops once its FP32 recursive residual has dropped by the factor
 *   max(inner_tol, tol / rel_o) (rel_o = ||b - A x_o|| / ||b||); its
 *   correction is added to x in FP64, r is replaced by the FP64 b - A x, and
 *   the next run continues from the last direction: d = s + (rho_new /
 *   rho_old) d instead of d = s.  In exact arithmetic this is one PCG run
 *   of Algorithm 1 whose residual is recomputed at each correction; the
 *   FP64 parts are those of the restarted form.  inner_tol must be in
 *   (0, 1); 0.1 is the usual choice (about one correction per decade).
 *   *outer counts corrections, hist_host receives the true residual before
 *   each of them and at the end.
 * Other arguments, results and errors as pcga_pcg_solve_mixed; EINVAL for an
 * unknown refine value. */
#define PCGA_REFINE_RESTART 0
#define PCGA_REFINE_KEEP 1
int pcga_pcg_solve_mixed_ex(pcga_solver_t *S, const double *b_dev, double *x_dev, double tol,
                            double inner_tol, int32_t max_outer, int32_t inner_maxit,
                            int32_t refine, int32_t *outer, int32_t *inner_total,
                            double *hist_host, int32_t hist_cap, int32_t *hist_len,
                            double *true_relres);

/* ---- single steps of the hot path (for parity tests and profiling) -------
 * y = A x (FP64, the five-point product of eq. (10)). */
int pcga_apply_a(pcga_solver_t *S, const double *x_dev, double *y_dev);
/* t = D^-1 Z^T r and s = Z t, in the solver's inner precision (FP64 data for
 * PCGA_FP64; FP32 data with FP64 input/output for PCGA_MIXED). */
int pcga_apply_prec(pcga_solver_t *S, const double *r_dev, double *t_dev, double *s_dev);

/* One launch of the fused first kernel of an iteration (Algorithm 1's
 * direction update and operator product): d_new = s + beta d, q = A d_new
 * (the five-point product of eq. (10), FP64 coefficients) and (d_new, q),
 * summed over the launch's workgroups as the next kernel of an iteration
 * sums it.  s_dev, d_dev: n FP64 device values in; dnew_dev, q_dev: n FP64
 * device values out (caller-owned, not aliasing the inputs); *dq: host.  In
 * the solver's inner precision: a PCGA_MIXED solver rounds s and d to FP32,
 * runs the FP32 kernel (d_new in FP32; A d_new formed in FP64 and rounded to
 * FP32) and returns its FP32 results widened to FP64.  beta >= 0 and finite
 * (beta = 0: d_new = s).  Uses the solver's control block and, for
 * PCGA_MIXED, its inner vectors: the solver stays usable.  Errors: EINVAL,
 * EHIP. */
int pcga_step_stencil(pcga_solver_t *S, const double *s_dev, const double *d_dev, double beta,
                      double *dnew_dev, double *q_dev, double *dq);

/* Average device time in milliseconds of each kernel of one PCG iteration,
 * ms_out[0] = d-update + five-point product + (d,q); ms_out[1] = residual and
 * solution update + D^-1 Z^T r; ms_out[2] = Z t + (s,r) (0 with the
 * diagonal preconditioner, whose second kernel also applies D^-1); ms_out[3]
 * = one whole iteration.  Starts from the prologue of a solve from x0 = 0; no
 * stopping test fires.  mode 0: each kernel launched `reps` (1..100000)
 * times back to back between two HIP events (data a kernel re-reads may stay
 * cached between its launches).  mode 1: `reps` whole iterations with a HIP
 * event between every two kernels, so that each kernel meets the cache state
 * of a solve (the times include the events' own cost, a few microseconds).
 * ms_out[3]: `reps` whole iterations between two events, launched as a solve
 * launches them (from a captured graph when the solver uses graphs).  FP64
 * kernels for PCGA_FP64, the FP32 inner kernels for PCGA_MIXED.  For
 * benchmarks: the solver's vectors are left in an unspecified state, the
 * solver stays usable. */
int pcga_profile_iteration(pcga_solver_t *S, const double *b_dev, int32_t reps, int32_t mode,
                           double *ms_out);

/* ---- the time step around the solve ----------------------------------------
 * The elliptic solve is one stage of the sea-surface time step (Sec. 2,
 * eq. (1)-(2)).  These passes produce a step's right-hand side and first
 * guess and advance the sea-surface height, on the solver's grid (nx, ny,
 * periodicity) and stream; all pointers are device arrays of n = nx*ny FP64
 * values owned by the caller.  They are queued on the solver's stream and
 * return without waiting for it.  Errors: EINVAL (NULL pointer, bad dt),
 * EHIP.
 *
 * pcga_ts_rhs: the right-hand side of eq. (8),
 *   b = -(delta_i(e2 Mu) - delta_j(e1 Mv)),
 * negated like the operator (the system solved is the negation of
 * eq. (10)).  delta_i f(i,j) = f(i+1/2,j) - f(i-1/2,j) and likewise delta_j.
 * e2u[k], mu[k]: metric factor e2 and transport Mu on the east face of cell
 * k; e1v[k], mv[k]: e1 and Mv on its north face.  Closed faces (zero flux):
 * the west face of i = 0 and the east face of i = nx-1 unless the grid is
 * periodic (then they are one face, stored at i = nx-1), the south face of
 * j = 0 and the north face of j = ny-1 (values stored there are ignored).
 * Transports on faces that touch land must be zero (land rows then get
 * b = 0, as the solve requires). */
int pcga_ts_rhs(pcga_solver_t *S, const double *e2u, const double *mu, const double *e1v,
                const double *mv, double *b);
/* pcga_ts_eta: eq. (1), eta_next = eta_prev - 2 dt D cell by cell (eta_prev
 * = eta^{n-1}, D = D^n; eta_next may alias eta_prev).  dt >= 0. */
int pcga_ts_eta(pcga_solver_t *S, const double *eta_prev, const double *D, double dt,
                double *eta_next);
/* pcga_ts_guess: the first guess x0 of Algorithm 1 from the solutions of the
 * two previous steps, x0 = a D1 + c D2 (D2 is not read, and may be NULL,
 * when c = 0); x0 may alias D1 or D2.  The paper writes x0 = 2 D^{t-1}. */
int pcga_ts_guess(pcga_solver_t *S, const double *D1, const double *D2, double a, double c,
                  double *x0);

/* ---- batched solves (ensembles and continuous batching) -------------------
 * A batch advances many independent solves with one launch of each iteration
 * kernel for all of them.  An item (slot) is a PCGA_MIXED solver (its resident
 * operator, D^-1 and Z) with nrhs right-hand sides (1, 2 or 4, solved
 * together: A and Z are read once for all of them), each solved by the
 * method of pcga_pcg_solve_mixed (FP32 inner PCG, FP64 refinement).  Items
 * may be added and removed between pcga_batch_run calls; work of items added
 * while others run overlaps on the device.  An item's result does not depend
 * on the other items (its reductions use a block count fixed by its grid).
 *
 * Memory: the batch's control data lives in caller-provided device memory
 * (pcga_batch_scratch_bytes), each item's vectors in its own caller-provided
 * device workspace (pcga_batch_item_bytes); the library allocates none.
 * Every solver and workspace must stay alive while its item is in the batch.
 * All work runs on the batch's stream; the calls return after their device
 * work finished.  Errors: EINVAL, ENOMEM (scratch / workspace too small, no
 * free slot, batch too large), EHIP. */
typedef struct pcga_batch pcga_batch_t;

int pcga_batch_scratch_bytes(int32_t max_slots, size_t *bytes);
int pcga_batch_item_bytes(const pcga_solver_t *S, int32_t nrhs, size_t *bytes);
int pcga_batch_create(int32_t max_slots, void *scratch_dev, size_t scratch_bytes, void *stream,
                      pcga_batch_t **out);
int pcga_batch_destroy(pcga_batch_t *B);

/* Add an item: b_dev[r], x0_dev[r] (n FP64 device values each, r < nrhs) are
 * copied into the item workspace at once; x_out_dev[r] receive the solutions
 * at pcga_batch_remove.  Tolerances as in pcga_pcg_solve_mixed
 * (inner_maxit < 0 means n).  *slot receives the item's slot number. */
int pcga_batch_add(pcga_batch_t *B, pcga_solver_t *S, int32_t nrhs, const double *const *b_dev,
                   const double *const *x0_dev, double *const *x_out_dev, void *item_ws,
                   size_t item_bytes, double tol, double inner_tol, int32_t max_outer,
                   int32_t inner_maxit, int32_t *slot);
/* pcga_batch_add_ex: pcga_batch_add with the refinement of
 * pcga_pcg_solve_mixed_ex (refine = PCGA_REFINE_RESTART or
 * PCGA_REFINE_KEEP; for KEEP, inner_tol in (0, 1) is the residual reduction
 * of one inner run).  A slot's right-hand sides share its corrections: an
 * inner run ends when every active right-hand side has met its own stop, and
 * one that met it earlier rests (alpha = 0) with its direction and last rho
 * kept until the correction. */
int pcga_batch_add_ex(pcga_batch_t *B, pcga_solver_t *S, int32_t nrhs, const double *const *b_dev,
                      const double *const *x0_dev, double *const *x_out_dev, void *item_ws,
                      size_t item_bytes, double tol, double inner_tol, int32_t max_outer,
                      int32_t inner_maxit, int32_t refine, int32_t *slot);

/* Run up to `chunks` chunks of iterations (stops early once every item is
 * done); *active receives the number of items not yet done. */
int pcga_batch_run(pcga_batch_t *B, int32_t chunks, int32_t *active);

/* Asynchronous form of pcga_batch_run, for callers that advance several
 * batches (each on its own stream) from one thread.  pcga_batch_launch
 * enqueues `chunks` chunks and the control-block snapshot on the batch's
 * stream and returns at once.  pcga_batch_wait then waits for them (block =
 * 1) or only checks (block = 0): *ready = 1 once they have finished (then
 * *active is set as by pcga_batch_run and the snapshot that pcga_batch_query
 * reads is current), 0 while they run.  While a launch is in flight,
 * pcga_batch_launch, _add, _remove, _query and _set_chunk on that batch
 * return PCGA_EINVAL.  Errors: EINVAL, EHIP. */
int pcga_batch_launch(pcga_batch_t *B, int32_t chunks);
int pcga_batch_wait(pcga_batch_t *B, int32_t block, int32_t *ready, int32_t *active);

/* Item results as of the last pcga_batch_run: done flag, status (PCGA_OK,
 * PCGA_NOCONV, PCGA_EBREAKDOWN, PCGA_ENAN), outer steps, inner iterations,
 * and true_relres[r] = ||b_r - A x_r|| / ||b_r|| (FP64) for r < nrhs. */
int pcga_batch_query(pcga_batch_t *B, int32_t slot, int32_t *done, int32_t *status,
                     int32_t *outer, int32_t *inner_total, double *true_relres);

/* Write the item's solutions to its x_out_dev vectors and free the slot. */
int pcga_batch_remove(pcga_batch_t *B, int32_t slot);

/* Iterations per captured chunk (even, 2..512). */
int pcga_batch_set_chunk(pcga_batch_t *B, int32_t chunk);
/* Workgroups per launch of the batch's kernels: a multiple of 8 in 8..2048
 * (default 2048; each workgroup takes the batch's logical blocks in turn).
 * A smaller grid leaves CUs to other streams' kernels (e.g. another batch on
 * the same device).  Results do not depend on it.  EINVAL while a launch is
 * in flight or for a bad value.  Takes effect at the next launch. */
int pcga_batch_set_grid(pcga_batch_t *B, int32_t grid);

#ifdef __cplusplus
}
#endif
#endif /* PCGAINV_H */
