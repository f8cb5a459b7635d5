/*
 * oracle.c -- plain FP64 CPU reference of the PCG-AINV solver.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the device path and must never be used as a fallback for it.
 *
 * Everything here is written for readability, not speed: sequential sums in
 * index order, unfused multiply-then-add (built with -ffp-contract=off), one
 * thread.
 *
 * Contents
 *   ora_spmv        y = A x for the 5-point operator of eq. (10).
 *   ora_csr_*       the same setup, product and Algorithm 1 for a general
 *                   sparse SPD matrix in CSR (a matrix that does not come
 *                   from the grid, as in the comparison of Sec. 5).
 *   ora_ainv_*      approximate inverse A^-1 ~ Z D^-1 Z^T by
 *                   A-orthogonalisation with a drop tolerance (the AINV of
 *                   the paper's ref. [book4-14]; the threshold variant is the
 *                   "drop tolerance" Bridson class of Sec. 5).
 *   ora_ainv_setup_fill  the same with at most `fill` off-diagonal entries
 *                   kept in each column of Z (the fixed-fill Bridson class
 *                   of Sec. 5).
 *   ora_prec_apply  s = Z D^-1 Z^T r (Algorithm 1, preconditioning step).
 *   ora_pcg         Algorithm 1 (FSAI/AINV-PCG), FP64.
 *   ora_pcg_mixed   FP64 iterative refinement around an FP32 inner PCG
 *                   (restarted, or with the direction kept: ora_pcg_mixed_opt).
 *   ora_fsai_band   the paper's own banded factor of T (Sec. 3, six-step
 *                   pattern scheme, Propositions 2-3).
 *   ora_ts_*        the surrounding time step: the right-hand side of eq. (8)
 *                   from face transports, the sea-surface update of eq. (1),
 *                   and the first guess of Algorithm 1 from earlier solutions.
 *
 * Operator storage ("A5", all row-major over the nx*ny grid, k = j*nx + i):
 *   diag[k] = A[k,k], ae[k] = A[k,east(k)], an[k] = A[k,k+nx];
 *   east(k) wraps to i = 0 when `periodic` is set.
 *
 * Readings of the paper taken here (listed again in the design notes):
 *   - Algorithm 1 updates the direction with the preconditioned residual,
 *     d_{k+1} = s_{k+1} + beta_k d_k (the printed r_{k+1} would bypass the
 *     preconditioner entirely).
 *   - The stopping test is ||r_k||_2 / ||b||_2 > tol on the recursively
 *     updated residual, with k < maxit (Algorithm 1's loop condition).
 *   - Drop rule: after each column update, every off-diagonal entry that was
 *     touched and has |z| < tau, or is exactly zero, is removed.  The unit
 *     diagonal is never dropped; an entry equal to tau is kept.
 *   - Fixed fill: the count is applied to a finished column, before its pivot
 *     p_i is formed, so p_i and every later update use the capped column.
 *
 * Evaluation-order builds.  Algorithm 1 fixes what each inner product is,
 * not the order in which its terms are added.  The default build adds them
 * in index order.  Built with -DORA_DOT_ORDER=1 it adds them in reverse
 * order, with -DORA_DOT_ORDER=2 in 1024 contiguous blocks whose sums are then
 * added in order (the shape of a reduction over workgroups); built with
 * contraction on (-ffp-contract=fast) multiply-adds are fused.  These builds
 * compute the same method and differ only in rounding; the tests use them to
 * measure how far rounding order alone moves the iterates and the stopping
 * iteration of a given problem.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_OK 0
#define ORA_NOCONV 1
#define ORA_EINVAL (-1)
#define ORA_EBREAKDOWN (-2)
#define ORA_ENOMEM (-3)

/* ------------------------------------------------------------------------ */
/* Row k of A as (column, value) pairs sorted by column.  Zero couplings     */
/* (land, domain edges) are omitted.  Returns the count (<= 5).              */
/* ------------------------------------------------------------------------ */
static int a_row(int64_t nx, int64_t ny, int periodic, const double *diag,
                 const double *ae, const double *an, int64_t k, int64_t *cols,
                 double *vals) {
    int64_t i = k % nx, j = k / nx;
    int64_t c[5];
    double v[5];
    int m = 0;
    if (j > 0 && an[k - nx] != 0.0) { c[m] = k - nx; v[m] = an[k - nx]; m++; }
    if (i > 0) {
        if (ae[k - 1] != 0.0) { c[m] = k - 1; v[m] = ae[k - 1]; m++; }
    } else if (periodic) {
        int64_t w = k + nx - 1;
        if (ae[w] != 0.0) { c[m] = w; v[m] = ae[w]; m++; }
    }
    c[m] = k; v[m] = diag[k]; m++;
    if (i < nx - 1) {
        if (ae[k] != 0.0) { c[m] = k + 1; v[m] = ae[k]; m++; }
    } else if (periodic) {
        if (ae[k] != 0.0) { c[m] = k - nx + 1; v[m] = ae[k]; m++; }
    }
    if (j < ny - 1 && an[k] != 0.0) { c[m] = k + nx; v[m] = an[k]; m++; }
    /* insertion sort by column (the periodic wraps break natural order) */
    for (int a = 1; a < m; a++) {
        int64_t cc = c[a];
        double vv = v[a];
        int b = a - 1;
        while (b >= 0 && c[b] > cc) { c[b + 1] = c[b]; v[b + 1] = v[b]; b--; }
        c[b + 1] = cc;
        v[b + 1] = vv;
    }
    for (int a = 0; a < m; a++) { cols[a] = c[a]; vals[a] = v[a]; }
    return m;
}

/* y = A x, each row summed in increasing column order. */
void ora_spmv(int64_t nx, int64_t ny, int periodic, const double *diag,
              const double *ae, const double *an, const double *x, double *y) {
    int64_t n = nx * ny;
    int64_t cols[5];
    double vals[5];
    for (int64_t k = 0; k < n; k++) {
        int m = a_row(nx, ny, periodic, diag, ae, an, k, cols, vals);
        double s = 0.0;
        for (int t = 0; t < m; t++) {
            double p = vals[t] * x[cols[t]];
            s = s + p;
        }
        y[k] = s;
    }
}

/* Check the A5 input: positive diagonal, zero couplings across
 * non-periodic east edge and the north edge, nx >= 3 when periodic. */
static int check_a5(int64_t nx, int64_t ny, int periodic, const double *diag,
                    const double *ae, const double *an) {
    if (nx < 1 || ny < 1) return ORA_EINVAL;
    if (periodic && nx < 3) return ORA_EINVAL;
    for (int64_t j = 0; j < ny; j++)
        for (int64_t i = 0; i < nx; i++) {
            int64_t k = j * nx + i;
            if (!(diag[k] > 0.0)) return ORA_EINVAL;
            if (!periodic && i == nx - 1 && ae[k] != 0.0) return ORA_EINVAL;
            if (j == ny - 1 && an[k] != 0.0) return ORA_EINVAL;
        }
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* A general sparse SPD operator in CSR (Sec. 5 compares the preconditioners */
/* also on a matrix that does not come from the grid): rowptr[n+1],           */
/* col/val[rowptr[n]], columns strictly ascending within each row, the        */
/* diagonal present and positive, A symmetric entry by entry.                 */
/* ------------------------------------------------------------------------ */
static int check_csr(int64_t n, const int64_t *rowptr, const int64_t *col,
                     const double *val) {
    if (n < 1 || !rowptr || rowptr[0] != 0) return ORA_EINVAL;
    for (int64_t k = 0; k < n; k++) {
        int have_diag = 0;
        if (rowptr[k + 1] < rowptr[k]) return ORA_EINVAL;
        for (int64_t a = rowptr[k]; a < rowptr[k + 1]; a++) {
            if (col[a] < 0 || col[a] >= n) return ORA_EINVAL;
            if (a > rowptr[k] && col[a] <= col[a - 1]) return ORA_EINVAL;
            if (!isfinite(val[a])) return ORA_EINVAL;
            if (col[a] == k) {
                if (!(val[a] > 0.0)) return ORA_EINVAL;
                have_diag = 1;
            }
            /* the mirror entry (col[a], k) with the same value */
            int64_t lo = rowptr[col[a]], hi = rowptr[col[a] + 1];
            while (lo < hi) {
                int64_t mid = (lo + hi) / 2;
                if (col[mid] < k) lo = mid + 1; else hi = mid;
            }
            if (lo == rowptr[col[a] + 1] || col[lo] != k || val[lo] != val[a]) return ORA_EINVAL;
        }
        if (!have_diag) return ORA_EINVAL;
    }
    return ORA_OK;
}

/* The operator of a solve: the five-point A5 storage or a CSR matrix. */
typedef struct {
    int64_t n;
    int csr;
    int64_t nx, ny;
    int periodic;
    const double *diag, *ae, *an;
    const int64_t *rowptr, *col;
    const double *val;
    int64_t maxrow;   /* longest row */
} ora_op;

static ora_op op_a5(int64_t nx, int64_t ny, int periodic, const double *diag,
                    const double *ae, const double *an) {
    ora_op A;
    memset(&A, 0, sizeof(A));
    A.n = nx * ny;
    A.nx = nx;
    A.ny = ny;
    A.periodic = periodic;
    A.diag = diag;
    A.ae = ae;
    A.an = an;
    A.maxrow = 5;
    return A;
}

static ora_op op_csr(int64_t n, const int64_t *rowptr, const int64_t *col,
                     const double *val) {
    ora_op A;
    memset(&A, 0, sizeof(A));
    A.n = n;
    A.csr = 1;
    A.rowptr = rowptr;
    A.col = col;
    A.val = val;
    A.maxrow = 1;
    for (int64_t k = 0; k < n; k++)
        if (rowptr[k + 1] - rowptr[k] > A.maxrow) A.maxrow = rowptr[k + 1] - rowptr[k];
    return A;
}

/* Row k as (column, value) pairs sorted by column (capacity A->maxrow). */
static int op_row(const ora_op *A, int64_t k, int64_t *cols, double *vals) {
    if (!A->csr) return a_row(A->nx, A->ny, A->periodic, A->diag, A->ae, A->an, k, cols, vals);
    int m = 0;
    for (int64_t a = A->rowptr[k]; a < A->rowptr[k + 1]; a++) {
        cols[m] = A->col[a];
        vals[m] = A->val[a];
        m++;
    }
    return m;
}

/* y = A x, each row summed in increasing column order. */
static void op_apply(const ora_op *A, const double *x, double *y) {
    if (!A->csr) {
        ora_spmv(A->nx, A->ny, A->periodic, A->diag, A->ae, A->an, x, y);
        return;
    }
    for (int64_t k = 0; k < A->n; k++) {
        double s = 0.0;
        for (int64_t a = A->rowptr[k]; a < A->rowptr[k + 1]; a++) {
            double p = A->val[a] * x[A->col[a]];
            s = s + p;
        }
        y[k] = s;
    }
}

void ora_csr_spmv(int64_t n, const int64_t *rowptr, const int64_t *col, const double *val,
                  const double *x, double *y) {
    ora_op A = op_csr(n, rowptr, col, val);
    op_apply(&A, x, y);
}

/* ------------------------------------------------------------------------ */
/* AINV by A-orthogonalisation with a drop tolerance.                        */
/*                                                                          */
/* Z is unit upper triangular; column z_j holds its off-diagonal entries     */
/* (rows < j) sorted by row.  Right-looking form: at step i, z_i is final;   */
/* p_i = a_i^T z_i, and every later column z_j with c_j = a_i^T z_j != 0 is  */
/* updated z_j <- z_j - (c_j / p_i) z_i, then its touched small entries are  */
/* dropped.  a_i^T z sums over row i of A in increasing column order.        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t *r;
    double *v;
    int64_t len, cap;
} ora_col;

typedef struct {
    int64_t *j;
    int64_t len, cap;
} ora_list;

typedef struct {
    int64_t n;
    ora_col *z;
    double *D;
    int64_t nnz_off;
} ora_ainv;

/* value of column z_j (unit diagonal implicit) at row r */
static double zval(const ora_col *zj, int64_t j, int64_t r) {
    if (r == j) return 1.0;
    if (r > j) return 0.0;
    int64_t lo = 0, hi = zj->len;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (zj->r[mid] < r) lo = mid + 1; else hi = mid;
    }
    if (lo < zj->len && zj->r[lo] == r) return zj->v[lo];
    return 0.0;
}

static int list_push(ora_list *L, int64_t j) {
    if (L->len == L->cap) {
        int64_t nc = L->cap ? 2 * L->cap : 4;
        int64_t *p = (int64_t *)realloc(L->j, (size_t)nc * sizeof(int64_t));
        if (!p) return ORA_ENOMEM;
        L->j = p;
        L->cap = nc;
    }
    L->j[L->len++] = j;
    return ORA_OK;
}

void ora_ainv_free(void *h) {
    ora_ainv *F = (ora_ainv *)h;
    if (!F) return;
    if (F->z) {
        for (int64_t j = 0; j < F->n; j++) { free(F->z[j].r); free(F->z[j].v); }
        free(F->z);
    }
    free(F->D);
    free(F);
}

/* Fixed fill (the second Bridson class of Sec. 5, a set number of nonzeros
 * in each row of the lower factor Z^T, i.e. each column of Z): keep the
 * `fill` off-diagonal entries of z_i of largest magnitude.  Equal magnitudes
 * are ranked by row, the larger row (nearer the diagonal) first.  The kept
 * entries stay in increasing row order.  Plain selection by repeated scans:
 * the columns are short. */
static int keep_largest(ora_col *z, int64_t fill) {
    if (z->len <= fill) return ORA_OK;
    char *keep = (char *)calloc((size_t)z->len, 1);
    if (!keep) return ORA_ENOMEM;
    for (int64_t k = 0; k < fill; k++) {
        int64_t best = -1;
        for (int64_t a = 0; a < z->len; a++) {
            if (keep[a]) continue;
            if (best < 0 || fabs(z->v[a]) > fabs(z->v[best]) ||
                (fabs(z->v[a]) == fabs(z->v[best]) && z->r[a] > z->r[best]))
                best = a;
        }
        keep[best] = 1;
    }
    int64_t w = 0;
    for (int64_t a = 0; a < z->len; a++) {
        if (!keep[a]) continue;
        z->r[w] = z->r[a];
        z->v[w] = z->v[a];
        w++;
    }
    z->len = w;
    free(keep);
    return ORA_OK;
}

/* The method on any operator: Z, D of A ~ (Z D^-1 Z^T)^-1, see above. */
static int ainv_core(const ora_op *A, double tau, int64_t fill, void **out,
                     int64_t *nnz_off, int64_t *breakdown_row) {
    int st = ORA_OK;
    int64_t n = A->n;
    int64_t *cols = (int64_t *)malloc((size_t)A->maxrow * sizeof(int64_t));
    double *vals = (double *)malloc((size_t)A->maxrow * sizeof(double));
    ora_ainv *F = (ora_ainv *)calloc(1, sizeof(ora_ainv));
    ora_list *rows = (ora_list *)calloc((size_t)n, sizeof(ora_list));
    int64_t *seen = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *cand = NULL;
    int64_t ccap = 0;
    int64_t *mr = NULL;
    double *mv = NULL;
    int64_t mcap = 0;
    if (!F || !cols || !vals || !rows || !seen) { st = ORA_ENOMEM; goto done; }
    F->n = n;
    F->z = (ora_col *)calloc((size_t)n, sizeof(ora_col));
    F->D = (double *)malloc((size_t)n * sizeof(double));
    if (!F->z || !F->D) { st = ORA_ENOMEM; goto done; }
    for (int64_t j = 0; j < n; j++) seen[j] = -1;

    for (int64_t i = 0; i < n; i++) {
        int m = op_row(A, i, cols, vals);
        ora_col *zi = &F->z[i];
        /* every update of z_i has been applied (only steps < i touch it) */
        if (fill >= 0) {
            st = keep_largest(zi, fill);
            if (st) goto done;
        }

        /* p_i = a_i^T z_i */
        double p = 0.0;
        for (int t = 0; t < m; t++) {
            double zv = zval(zi, i, cols[t]);
            if (zv != 0.0) { double pr = vals[t] * zv; p = p + pr; }
        }
        if (!(p > 0.0)) {
            if (breakdown_row) *breakdown_row = i;
            st = ORA_EBREAKDOWN;
            goto done;
        }
        F->D[i] = p;

        /* Columns j > i that may have a nonzero at a column of row i of A:
         * the unit diagonals j = cols[t] and every j listed at those rows. */
        int64_t nc = 0;
        for (int t = 0; t < m; t++) {
            int64_t c = cols[t];
            int64_t extra = 1 + rows[c].len;
            if (nc + extra > ccap) {
                int64_t nca = 2 * (nc + extra) + 16;
                int64_t *q = (int64_t *)realloc(cand, (size_t)nca * sizeof(int64_t));
                if (!q) { st = ORA_ENOMEM; goto done; }
                cand = q;
                ccap = nca;
            }
            if (c > i && seen[c] != i) { seen[c] = i; cand[nc++] = c; }
            for (int64_t a = 0; a < rows[c].len; a++) {
                int64_t j = rows[c].j[a];
                if (j > i && seen[j] != i) { seen[j] = i; cand[nc++] = j; }
            }
        }

        for (int64_t a = 0; a < nc; a++) {
            int64_t j = cand[a];
            ora_col *zj = &F->z[j];
            double cj = 0.0;
            for (int t = 0; t < m; t++) {
                double zv = zval(zj, j, cols[t]);
                if (zv != 0.0) { double pr = vals[t] * zv; cj = cj + pr; }
            }
            if (cj == 0.0) continue;
            double mult = cj / p;

            /* z_j <- z_j - mult * z_i, where z_i = (off-diagonals, 1 at row i).
             * Merge the two row-sorted lists; rows of z_i are all <= i < j. */
            int64_t need = zj->len + zi->len + 1;
            if (need > mcap) {
                int64_t nm = 2 * need;
                int64_t *q1 = (int64_t *)realloc(mr, (size_t)nm * sizeof(int64_t));
                if (!q1) { st = ORA_ENOMEM; goto done; }
                mr = q1;
                double *q2 = (double *)realloc(mv, (size_t)nm * sizeof(double));
                if (!q2) { st = ORA_ENOMEM; goto done; }
                mv = q2;
                mcap = nm;
            }
            int64_t pa = 0, pb = 0, out_len = 0;
            int64_t nb_i = zi->len + 1;  /* z_i entries incl. the diagonal */
            while (pa < zj->len || pb < nb_i) {
                int64_t rb = (pb < zi->len) ? zi->r[pb] : (pb == zi->len ? i : INT64_MAX);
                int64_t ra = (pa < zj->len) ? zj->r[pa] : INT64_MAX;
                if (ra < rb) {
                    mr[out_len] = ra;
                    mv[out_len] = zj->v[pa];
                    out_len++;
                    pa++;
                } else {
                    double vb = (pb < zi->len) ? zi->v[pb] : 1.0;
                    double old = (ra == rb) ? zj->v[pa] : 0.0;
                    double prod = mult * vb;
                    double nv = old - prod;
                    int fresh = (ra != rb);
                    if (ra == rb) pa++;
                    pb++;
                    /* drop rule on the touched entry */
                    if (nv == 0.0 || fabs(nv) < tau) continue;
                    mr[out_len] = rb;
                    mv[out_len] = nv;
                    out_len++;
                    if (fresh) {
                        st = list_push(&rows[rb], j);
                        if (st) goto done;
                    }
                }
            }
            if (out_len > zj->cap) {
                int64_t *q1 = (int64_t *)realloc(zj->r, (size_t)out_len * sizeof(int64_t));
                if (!q1) { st = ORA_ENOMEM; goto done; }
                zj->r = q1;
                double *q2 = (double *)realloc(zj->v, (size_t)out_len * sizeof(double));
                if (!q2) { st = ORA_ENOMEM; goto done; }
                zj->v = q2;
                zj->cap = out_len;
            }
            memcpy(zj->r, mr, (size_t)out_len * sizeof(int64_t));
            memcpy(zj->v, mv, (size_t)out_len * sizeof(double));
            zj->len = out_len;
        }
    }
    {
        int64_t tot = 0;
        for (int64_t j = 0; j < n; j++) tot += F->z[j].len;
        F->nnz_off = tot;
        if (nnz_off) *nnz_off = tot;
    }
done:
    for (int64_t r = 0; rows && r < n; r++) free(rows[r].j);
    free(rows);
    free(seen);
    free(cand);
    free(mr);
    free(mv);
    free(cols);
    free(vals);
    if (st) { ora_ainv_free(F); return st; }
    *out = F;
    return ORA_OK;
}

/* Returns ORA_OK and a handle, or ORA_EBREAKDOWN (p_i <= 0) / ORA_EINVAL /
 * ORA_ENOMEM.  fill < 0: no cap on the entries per column. */
int ora_ainv_setup_fill(int64_t nx, int64_t ny, int periodic, const double *diag,
                        const double *ae, const double *an, double tau, int64_t fill,
                        void **out, int64_t *nnz_off, int64_t *breakdown_row) {
    *out = NULL;
    if (breakdown_row) *breakdown_row = -1;
    int st = check_a5(nx, ny, periodic, diag, ae, an);
    if (st) return st;
    if (!(tau >= 0.0)) return ORA_EINVAL;
    ora_op A = op_a5(nx, ny, periodic, diag, ae, an);
    return ainv_core(&A, tau, fill, out, nnz_off, breakdown_row);
}

int ora_ainv_setup(int64_t nx, int64_t ny, int periodic, const double *diag,
                   const double *ae, const double *an, double tau, void **out,
                   int64_t *nnz_off, int64_t *breakdown_row) {
    return ora_ainv_setup_fill(nx, ny, periodic, diag, ae, an, tau, -1, out, nnz_off,
                               breakdown_row);
}

/* The same A-orthogonalisation on a CSR matrix (see check_csr). */
int ora_ainv_setup_csr(int64_t n, const int64_t *rowptr, const int64_t *col,
                       const double *val, double tau, int64_t fill, void **out,
                       int64_t *nnz_off, int64_t *breakdown_row) {
    *out = NULL;
    if (breakdown_row) *breakdown_row = -1;
    int st = check_csr(n, rowptr, col, val);
    if (st) return st;
    if (!(tau >= 0.0)) return ORA_EINVAL;
    ora_op A = op_csr(n, rowptr, col, val);
    return ainv_core(&A, tau, fill, out, nnz_off, breakdown_row);
}

/* Export Z (strictly upper part) in CSC: colptr[n+1], rowidx/val[nnz_off],
 * rows ascending inside each column; D[n]. */
void ora_ainv_export(const void *h, int64_t *colptr, int64_t *rowidx,
                     double *val, double *D) {
    const ora_ainv *F = (const ora_ainv *)h;
    int64_t pos = 0;
    for (int64_t j = 0; j < F->n; j++) {
        colptr[j] = pos;
        for (int64_t a = 0; a < F->z[j].len; a++) {
            rowidx[pos] = F->z[j].r[a];
            val[pos] = F->z[j].v[a];
            pos++;
        }
        D[j] = F->D[j];
    }
    colptr[F->n] = pos;
}

/* ------------------------------------------------------------------------ */
/* Preconditioner apply s = Z D^-1 Z^T r  (Algorithm 1, line 3 / line 7).     */
/* Z given in CSC (strict upper part; unit diagonal implicit).               */
/*   t_j = (sum_{k<j} Z[k,j] r_k  +  r_j) / D_j       (k ascending)          */
/*   s_k = t_k + sum_{j>k} Z[k,j] t_j                 (j ascending)          */
/* ------------------------------------------------------------------------ */
void ora_zt_apply(int64_t n, const int64_t *colptr, const int64_t *rowidx,
                  const double *val, const double *D, const double *r,
                  double *t) {
    for (int64_t j = 0; j < n; j++) {
        double acc = 0.0;
        for (int64_t a = colptr[j]; a < colptr[j + 1]; a++) {
            double p = val[a] * r[rowidx[a]];
            acc = acc + p;
        }
        acc = acc + r[j];
        t[j] = acc / D[j];
    }
}

void ora_z_apply(int64_t n, const int64_t *colptr, const int64_t *rowidx,
                 const double *val, const double *t, double *s) {
    for (int64_t k = 0; k < n; k++) s[k] = 0.0;
    for (int64_t j = 0; j < n; j++) {
        s[j] = s[j] + t[j];  /* diagonal term: no earlier column touches row j
                                after this, since rows of z_j are < j */
        for (int64_t a = colptr[j]; a < colptr[j + 1]; a++) {
            double p = val[a] * t[j];
            s[rowidx[a]] = s[rowidx[a]] + p;
        }
    }
}

void ora_prec_apply(int64_t n, const int64_t *colptr, const int64_t *rowidx,
                    const double *val, const double *D, const double *r,
                    double *s, double *tmp) {
    ora_zt_apply(n, colptr, rowidx, val, D, r, tmp);
    ora_z_apply(n, colptr, rowidx, val, tmp, s);
}

#ifndef ORA_DOT_ORDER
#define ORA_DOT_ORDER 0
#endif

static double dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
#if ORA_DOT_ORDER == 1
    for (int64_t k = n - 1; k >= 0; k--) { double p = a[k] * b[k]; s = s + p; }
#elif ORA_DOT_ORDER == 2
    const int64_t nblk = 1024;
    for (int64_t g = 0; g < nblk; g++) {
        double part = 0.0;
        for (int64_t k = g * n / nblk; k < (g + 1) * n / nblk; k++) {
            double p = a[k] * b[k];
            part = part + p;
        }
        s = s + part;
    }
#else
    for (int64_t k = 0; k < n; k++) { double p = a[k] * b[k]; s = s + p; }
#endif
    return s;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 (PCG with P = Z D^-1 Z^T), FP64.                              */
/*  x: in x0, out x.  hist: capacity maxit+1, hist[k] = ||r_k||/||b||.       */
/*  alphas/betas (optional, capacity maxit): the CG scalars per iteration.    */
/*  Returns ORA_OK (converged), ORA_NOCONV, ORA_EBREAKDOWN, ORA_ENOMEM.       */
/* ------------------------------------------------------------------------ */
static int pcg_core(const ora_op *A, const int64_t *colptr,
                    const int64_t *rowidx, const double *val, const double *D,
                    const double *b, double *x, double tol, int64_t maxit,
                    int64_t *iters, double *hist, double *alphas, double *betas) {
    int64_t n = A->n;
    double *r = (double *)malloc((size_t)n * sizeof(double));
    double *s = (double *)malloc((size_t)n * sizeof(double));
    double *d = (double *)malloc((size_t)n * sizeof(double));
    double *q = (double *)malloc((size_t)n * sizeof(double));
    double *tmp = (double *)malloc((size_t)n * sizeof(double));
    int st = ORA_OK;
    if (!r || !s || !d || !q || !tmp) { st = ORA_ENOMEM; goto out; }

    *iters = 0;
    double nb = sqrt(dot(n, b, b));
    if (nb == 0.0) {
        for (int64_t k = 0; k < n; k++) x[k] = 0.0;
        hist[0] = 0.0;
        goto out;
    }
    op_apply(A, x, q);
    for (int64_t k = 0; k < n; k++) r[k] = b[k] - q[k];
    ora_prec_apply(n, colptr, rowidx, val, D, r, s, tmp);
    for (int64_t k = 0; k < n; k++) d[k] = s[k];
    double rho = dot(n, s, r);
    int64_t it = 0;
    hist[0] = sqrt(dot(n, r, r)) / nb;
    while (hist[it] > tol && it < maxit) {
        op_apply(A, d, q);
        double dq = dot(n, d, q);
        if (!(dq > 0.0) || !(rho > 0.0)) { st = ORA_EBREAKDOWN; break; }
        double alpha = rho / dq;
        if (alphas) alphas[it] = alpha;
        for (int64_t k = 0; k < n; k++) { double p = alpha * d[k]; x[k] = x[k] + p; }
        for (int64_t k = 0; k < n; k++) { double p = alpha * q[k]; r[k] = r[k] - p; }
        it++;
        hist[it] = sqrt(dot(n, r, r)) / nb;
        if (hist[it] <= tol) break;
        ora_prec_apply(n, colptr, rowidx, val, D, r, s, tmp);
        double rho_new = dot(n, s, r);
        if (!(rho_new > 0.0)) { st = ORA_EBREAKDOWN; break; }
        double beta = rho_new / rho;
        if (betas) betas[it - 1] = beta;
        rho = rho_new;
        for (int64_t k = 0; k < n; k++) { double p = beta * d[k]; d[k] = s[k] + p; }
    }
    *iters = it;
    if (st == ORA_OK && !(hist[it] <= tol)) st = ORA_NOCONV;
out:
    free(r); free(s); free(d); free(q); free(tmp);
    return st;
}

int ora_pcg(int64_t nx, int64_t ny, int periodic, const double *diag,
            const double *ae, const double *an, const int64_t *colptr,
            const int64_t *rowidx, const double *val, const double *D,
            const double *b, double *x, double tol, int64_t maxit,
            int64_t *iters, double *hist, double *alphas, double *betas) {
    ora_op A = op_a5(nx, ny, periodic, diag, ae, an);
    return pcg_core(&A, colptr, rowidx, val, D, b, x, tol, maxit, iters, hist, alphas, betas);
}

/* Algorithm 1 on a CSR matrix (see check_csr; not re-checked here). */
int ora_pcg_csr(int64_t n, const int64_t *rowptr, const int64_t *col, const double *aval,
                const int64_t *colptr, const int64_t *rowidx, const double *val,
                const double *D, const double *b, double *x, double tol, int64_t maxit,
                int64_t *iters, double *hist, double *alphas, double *betas) {
    ora_op A = op_csr(n, rowptr, col, aval);
    return pcg_core(&A, colptr, rowidx, val, D, b, x, tol, maxit, iters, hist, alphas, betas);
}

/* ------------------------------------------------------------------------ */
/* Mixed precision: FP64 outer refinement around an FP32 inner PCG.          */
/*   outer: r = b - A x (FP64); stop if ||r||/||b|| <= tol;                  */
/*          solve A e = r with FP32 data (Z, D and vectors rounded to float)  */
/*          to relative tolerance inner_tol; x += e in FP64.                 */
/*   inner: CG scalars and dot sums in FP64, vector updates in FP32; q = A d  */
/*          sums the FP64 coefficients times the FP32 d in FP64 and rounds   */
/*          q to float (rounded coefficients would cap each outer step's     */
/*          reduction on fine grids).                                         */
/*   a32 != 0: the operator too in FP32 for the inner solve (its            */
/*          coefficients rounded to float, q = A d summed in float): every   */
/*          inner datum in FP32, FP64 kept for the residual, the solution    */
/*          and the CG scalars.                                              */
/* keep != 0: the direction is kept across corrections (reliable updates:  */
/*          Sleijpen and van der Vorst, 1996).  After each correction the    */
/*          inner solve continues from the new residual with the previous   */
/*          direction, d = s + (rho_new/rho_old) d, instead of d = s; in     */
/*          exact arithmetic the iterates are those of one PCG run, with the */
/*          residual replaced by the true FP64 one at every correction.     */
/*          The inner stop of outer step o is max(inner_tol, tol/rel_o),    */
/*          rel_o = ||r_o||/||b||: a segment stops early when the remaining  */
/*          reduction is below inner_tol.                                   */
/* outer_hist[o] = ||b - A x_o||/||b|| (capacity max_outer+1).               */
/* ------------------------------------------------------------------------ */
static void spmv32(int64_t nx, int64_t ny, int periodic, const double *diag,
                   const double *ae, const double *an, const float *x, float *y, int a32) {
    int64_t n = nx * ny;
    int64_t cols[5];
    double vals[5];
    for (int64_t k = 0; k < n; k++) {
        int m = a_row(nx, ny, periodic, diag, ae, an, k, cols, vals);
        if (a32) {
            float s = 0.0f;
            for (int t = 0; t < m; t++) {
                float p = (float)vals[t] * x[cols[t]];
                s = s + p;
            }
            y[k] = s;
            continue;
        }
        double s = 0.0;
        for (int t = 0; t < m; t++) {
            double p = vals[t] * (double)x[cols[t]];
            s = s + p;
        }
        y[k] = (float)s;
    }
}

static double dot32(int64_t n, const float *a, const float *b) {
    double s = 0.0;
    for (int64_t k = 0; k < n; k++) { double p = (double)a[k] * (double)b[k]; s = s + p; }
    return s;
}

static void prec32(int64_t n, const int64_t *colptr, const int64_t *rowidx,
                   const float *val, const float *D, const float *r, float *s,
                   float *t) {
    for (int64_t j = 0; j < n; j++) {
        float acc = 0.0f;
        for (int64_t a = colptr[j]; a < colptr[j + 1]; a++) {
            float p = val[a] * r[rowidx[a]];
            acc = acc + p;
        }
        acc = acc + r[j];
        t[j] = acc / D[j];
    }
    for (int64_t k = 0; k < n; k++) s[k] = 0.0f;
    for (int64_t j = 0; j < n; j++) {
        s[j] = s[j] + t[j];
        for (int64_t a = colptr[j]; a < colptr[j + 1]; a++) {
            float p = val[a] * t[j];
            s[rowidx[a]] = s[rowidx[a]] + p;
        }
    }
}

int ora_pcg_mixed_opt(int64_t nx, int64_t ny, int periodic, const double *diag,
                      const double *ae, const double *an, const int64_t *colptr,
                      const int64_t *rowidx, const double *val, const double *D,
                      const double *b, double *x, double tol, double inner_tol,
                      int64_t max_outer, int64_t inner_maxit, int64_t *outer,
                      int64_t *inner_total, double *outer_hist, int a32, int keep) {
    int64_t n = nx * ny;
    int64_t nnz = colptr[n];
    double *r64 = (double *)malloc((size_t)n * sizeof(double));
    double *y64 = (double *)malloc((size_t)n * sizeof(double));
    float *val32 = (float *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(float));
    float *D32 = (float *)malloc((size_t)n * sizeof(float));
    float *e = (float *)malloc((size_t)n * sizeof(float));
    float *r = (float *)malloc((size_t)n * sizeof(float));
    float *s = (float *)malloc((size_t)n * sizeof(float));
    float *d = (float *)malloc((size_t)n * sizeof(float));
    float *q = (float *)malloc((size_t)n * sizeof(float));
    float *t = (float *)malloc((size_t)n * sizeof(float));
    int st = ORA_OK;
    *outer = 0;
    *inner_total = 0;
    if (!r64 || !y64 || !val32 || !D32 || !e || !r || !s || !d || !q || !t) {
        st = ORA_ENOMEM;
        goto out;
    }
    for (int64_t a = 0; a < nnz; a++) val32[a] = (float)val[a];
    for (int64_t k = 0; k < n; k++) D32[k] = (float)D[k];

    double nb = sqrt(dot(n, b, b));
    if (nb == 0.0) {
        for (int64_t k = 0; k < n; k++) x[k] = 0.0;
        outer_hist[0] = 0.0;
        goto out;
    }
    int64_t o = 0;
    double rho = 0.0;   /* last rho of the inner run (kept across corrections) */
    for (;;) {
        ora_spmv(nx, ny, periodic, diag, ae, an, x, y64);
        for (int64_t k = 0; k < n; k++) r64[k] = b[k] - y64[k];
        outer_hist[o] = sqrt(dot(n, r64, r64)) / nb;
        if (outer_hist[o] <= tol) break;
        if (o == max_outer) { st = ORA_NOCONV; break; }

        /* inner FP32 PCG for A e = r, e0 = 0 */
        for (int64_t k = 0; k < n; k++) { r[k] = (float)r64[k]; e[k] = 0.0f; }
        double nr = sqrt(dot32(n, r, r));
        prec32(n, colptr, rowidx, val32, D32, r, s, t);
        double rho_new = dot32(n, s, r);
        if (keep && o > 0) {
            /* continue the previous inner run: its last rho divides */
            if (!(rho_new > 0.0)) { st = ORA_EBREAKDOWN; goto out; }
            float bf = (float)(rho_new / rho);
            for (int64_t k = 0; k < n; k++) { float p = bf * d[k]; d[k] = s[k] + p; }
        } else {
            for (int64_t k = 0; k < n; k++) d[k] = s[k];
        }
        rho = rho_new;
        double itol = inner_tol;
        if (keep && tol / outer_hist[o] > itol) itol = tol / outer_hist[o];
        double rel = 1.0;
        int64_t it = 0;
        while (rel > itol && it < inner_maxit) {
            spmv32(nx, ny, periodic, diag, ae, an, d, q, a32);
            double dq = dot32(n, d, q);
            if (!(dq > 0.0) || !(rho > 0.0)) { st = ORA_EBREAKDOWN; goto out; }
            double alpha = rho / dq;
            float af = (float)alpha;
            for (int64_t k = 0; k < n; k++) { float p = af * d[k]; e[k] = e[k] + p; }
            for (int64_t k = 0; k < n; k++) { float p = af * q[k]; r[k] = r[k] - p; }
            it++;
            rel = sqrt(dot32(n, r, r)) / nr;
            if (rel <= itol) break;
            prec32(n, colptr, rowidx, val32, D32, r, s, t);
            rho_new = dot32(n, s, r);
            if (!(rho_new > 0.0)) { st = ORA_EBREAKDOWN; goto out; }
            double beta = rho_new / rho;
            rho = rho_new;
            float bf = (float)beta;
            for (int64_t k = 0; k < n; k++) { float p = bf * d[k]; d[k] = s[k] + p; }
        }
        *inner_total += it;
        for (int64_t k = 0; k < n; k++) x[k] = x[k] + (double)e[k];
        o++;
    }
    *outer = o;
out:
    free(r64); free(y64); free(val32); free(D32); free(e); free(r); free(s);
    free(d); free(q); free(t);
    return st;
}

int ora_pcg_mixed_ex(int64_t nx, int64_t ny, int periodic, const double *diag,
                     const double *ae, const double *an, const int64_t *colptr,
                     const int64_t *rowidx, const double *val, const double *D,
                     const double *b, double *x, double tol, double inner_tol,
                     int64_t max_outer, int64_t inner_maxit, int64_t *outer,
                     int64_t *inner_total, double *outer_hist, int a32) {
    return ora_pcg_mixed_opt(nx, ny, periodic, diag, ae, an, colptr, rowidx, val, D, b, x, tol,
                             inner_tol, max_outer, inner_maxit, outer, inner_total, outer_hist,
                             a32, 0);
}

int ora_pcg_mixed(int64_t nx, int64_t ny, int periodic, const double *diag,
                  const double *ae, const double *an, const int64_t *colptr,
                  const int64_t *rowidx, const double *val, const double *D,
                  const double *b, double *x, double tol, double inner_tol,
                  int64_t max_outer, int64_t inner_maxit, int64_t *outer,
                  int64_t *inner_total, double *outer_hist) {
    return ora_pcg_mixed_ex(nx, ny, periodic, diag, ae, an, colptr, rowidx, val, D, b, x, tol,
                            inner_tol, max_outer, inner_maxit, outer, inner_total, outer_hist, 0);
}

/* y = A x in the inner precision of the mixed solve (a32 as above), for pins. */
void ora_spmv32(int64_t nx, int64_t ny, int periodic, const double *diag, const double *ae,
                const double *an, const float *x, float *y, int a32) {
    spmv32(nx, ny, periodic, diag, ae, an, x, y, a32);
}

/* ------------------------------------------------------------------------ */
/* The paper's banded FSAI of T (Sec. 3, six-step scheme).                    */
/* T keeps the entries of A with |col - row| <= 1 (in natural ordering this  */
/* is the east-west tridiagonal part; the periodic wrap lies outside the     */
/* band).  The unit upper factor keeps, in column j, rows j-q .. j-1 only    */
/* (entries with col > row + q are the negligible set S), and is computed by  */
/* T-orthogonalisation restricted to that pattern: for i = j-q .. j-1        */
/* (ascending), z_j <- z_j - (t_i^T z_j / p_i) z_i, with the update kept on   */
/* the band of z_j.  p_j = t_j^T z_j.                                        */
/* Output: Z band as val[j*q + (q-1-m)] = Z[j-1-m, j] for m = 0..q-1         */
/* (zero where j-1-m < 0), D[n].  Returns ORA_EBREAKDOWN if some p_j <= 0.    */
/* ------------------------------------------------------------------------ */
int ora_fsai_band(int64_t nx, int64_t ny, int periodic, const double *diag,
                  const double *ae, const double *an, int64_t q, double *zband,
                  double *D) {
    (void)an;
    int64_t n = nx * ny;
    if (q < 0) return ORA_EINVAL;
    /* tridiagonal entries of T: tdiag[k] = A[k,k], toff[k] = A[k,k+1] */
    double *zj = (double *)malloc((size_t)(q + 1) * sizeof(double));
    if (!zj) return ORA_ENOMEM;
    int st = ORA_OK;
    for (int64_t j = 0; j < n; j++) {
        /* z_j restricted to rows j-q..j: zj[m] is the entry at row j-q+m */
        for (int64_t m = 0; m <= q; m++) zj[m] = 0.0;
        zj[q] = 1.0;
        int64_t lo = j - q < 0 ? 0 : j - q;
        for (int64_t i = lo; i < j; i++) {
            /* c = t_i^T z_j over row i of T (cols i-1, i, i+1 inside band) */
            double c = 0.0;
            for (int64_t col = i - 1; col <= i + 1; col++) {
                if (col < 0 || col >= n || col < j - q || col > j) continue;
                double tv;
                if (col == i) tv = diag[i];
                else if (col == i + 1) tv = ((i % nx) != nx - 1) ? ae[i] : 0.0;
                else tv = ((col % nx) != nx - 1) ? ae[col] : 0.0;
                double zv = zj[col - (j - q)];
                if (zv != 0.0) { double p = tv * zv; c = c + p; }
            }
            if (c == 0.0) continue;
            double mult = c / D[i];
            /* z_i's band entries (rows i-q..i) that fall in rows j-q..j */
            for (int64_t rr = (i - q > lo ? i - q : lo); rr <= i; rr++) {
                double zi_r = (rr == i) ? 1.0 : zband[i * q + (q - 1 - (i - 1 - rr))];
                double p = mult * zi_r;
                zj[rr - (j - q)] = zj[rr - (j - q)] - p;
            }
        }
        /* p_j = t_j^T z_j */
        double p = 0.0;
        for (int64_t col = j - 1; col <= j + 1; col++) {
            if (col < 0 || col >= n || col < j - q || col > j) continue;
            double tv;
            if (col == j) tv = diag[j];
            else tv = ((col % nx) != nx - 1) ? ae[col] : 0.0;
            double zv = zj[col - (j - q)];
            if (zv != 0.0) { double pr = tv * zv; p = p + pr; }
        }
        if (!(p > 0.0)) { st = ORA_EBREAKDOWN; break; }
        D[j] = p;
        for (int64_t m = 0; m < q; m++) {
            int64_t row = j - 1 - m;
            zband[j * q + (q - 1 - m)] = (row >= 0) ? zj[row - (j - q)] : 0.0;
        }
    }
    (void)periodic;
    free(zj);
    return st;
}

/* ------------------------------------------------------------------------
 * The time step around the solve (Sec. 2 eq. (1); Sec. 3 eq. (8); the first
 * guess of Algorithm 1).
 *
 * Right-hand side, eq. (8): b_paper(i,j) = delta_i(e2 Mu) - delta_j(e1 Mv),
 * with delta_i f(i,j) = f(i+1/2,j) - f(i-1/2,j) over the cell's faces
 * (likewise delta_j).  Face values are stored at the cell to their west
 * (east faces: e2u[k], mu[k]) or south (north faces: e1v[k], mv[k]).  The
 * west face of i = 0 is the east face of i = nx-1 on a periodic grid and a
 * closed face (zero flux) otherwise; the east face of i = nx-1 on a
 * non-periodic grid, the south face of j = 0 and the north face of
 * j = ny-1 are closed.  The system solved is the negation of eq. (10)
 * (symmetric positive definite), so the stored right-hand side is
 * b = -b_paper.  Transports on faces that touch land are the caller's to
 * set to zero; land cells then get b = 0.
 * ------------------------------------------------------------------------ */
void ora_ts_rhs(int64_t nx, int64_t ny, int periodic, const double *e2u, const double *mu,
                const double *e1v, const double *mv, double *b) {
    for (int64_t j = 0; j < ny; j++) {
        for (int64_t i = 0; i < nx; i++) {
            const int64_t k = j * nx + i;
            double fe = 0.0, fw = 0.0, fn = 0.0, fs = 0.0;
            if (i < nx - 1 || periodic) fe = e2u[k] * mu[k];
            if (i > 0) {
                fw = e2u[k - 1] * mu[k - 1];
            } else if (periodic) {
                fw = e2u[k + nx - 1] * mu[k + nx - 1];
            }
            if (j < ny - 1) fn = e1v[k] * mv[k];
            if (j > 0) fs = e1v[k - nx] * mv[k - nx];
            const double bp = (fe - fw) - (fn - fs);
            b[k] = -bp;
        }
    }
}

/* Eq. (1): eta^{n+1} = eta^{n-1} - 2 dt D^n, cell by cell. */
void ora_ts_eta(int64_t n, const double *eta_prev, const double *D, double dt, double *eta_next) {
    const double s = 2.0 * dt;
    for (int64_t k = 0; k < n; k++) eta_next[k] = eta_prev[k] - s * D[k];
}

/* First guess of Algorithm 1 from the two previous solutions:
 * x0 = a D^{t-1} + c D^{t-2} (the second term left out when c = 0). */
void ora_ts_guess(int64_t n, const double *D1, const double *D2, double a, double c, double *x0) {
    for (int64_t k = 0; k < n; k++) {
        if (c == 0.0)
            x0[k] = a * D1[k];
        else
            x0[k] = a * D1[k] + c * D2[k];
    }
}
