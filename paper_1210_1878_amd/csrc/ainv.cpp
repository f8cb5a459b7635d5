// ainv.cpp -- host FP64 approximate-inverse setup (A-orthogonalisation with a
// drop tolerance), the preconditioner of Sec. 3-5 in the threshold form of
// the paper's ref. [book4-14].
//
// Left-looking organisation: column z_j is finished before z_{j+1} starts.
// For column j the steps i < j are visited in increasing order; step i
// applies z_j <- z_j - (a_i^T z_j / p_i) z_i when a_i^T z_j != 0 and then
// removes the touched off-diagonal entries with |z| < tau or z == 0.  This
// is the same sequence of floating-point operations on every column as the
// right-looking statement of the method (each column is only ever modified
// by earlier steps, in increasing order, each using a final z_i), so the
// pattern and values are fully determined by the order rules:
//   - a_i^T z sums over row i of A in increasing column order, unfused,
//     starting from +0.0 and skipping absent entries;
//   - a new entry takes the value 0.0 - m*v.
// This file must be compiled without floating-point contraction.
//
// With a fill cap the finished column is capped before its pivot; steps only
// read final columns, so this equals capping each column when it becomes the
// pivot of the right-looking statement.
//
// Candidate steps for column j are kept in a min-heap: a step i can touch
// z_j only if row i of A has a column where z_j is nonzero, i.e. i is a grid
// neighbour (or the cell itself) of some entry of z_j; for a general sparse
// A, a row that shares a column with an entry of z_j.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <new>
#include <queue>
#include <vector>

#include "pcga_host.h"

namespace pcga {

// Sorted entries of row k of A (at most 5), zero couplings omitted.
int A5View::row(int64_t k, int64_t *cols, double *vals) const {
    const int64_t i = k % nx, j = k / nx;
    struct E { int64_t c; double v; } e[5];
    int m = 0;
    const double w = (i > 0) ? ae[k - 1] : (periodic ? ae[k + nx - 1] : 0.0);
    const int64_t wc = (i > 0) ? k - 1 : k + nx - 1;
    const double east = (i < nx - 1 || periodic) ? ae[k] : 0.0;
    const int64_t ec = (i < nx - 1) ? k + 1 : k - nx + 1;
    if (j > 0 && an[k - nx] != 0.0) e[m++] = {k - nx, an[k - nx]};
    if (w != 0.0) e[m++] = {wc, w};
    e[m++] = {k, diag[k]};
    if (east != 0.0) e[m++] = {ec, east};
    if (j < ny - 1 && an[k] != 0.0) e[m++] = {k + nx, an[k]};
    std::sort(e, e + m, [](const E &a, const E &b) { return a.c < b.c; });
    for (int t = 0; t < m; t++) { cols[t] = e[t].c; vals[t] = e[t].v; }
    return m;
}

int A5View::validate() const {
    if (nx < 1 || ny < 1 || !diag || !ae || !an) return PCGA_EINVAL;
    if ((int64_t)nx * ny > (int64_t)INT32_MAX) return PCGA_EINVAL;
    if (periodic && nx < 3) return PCGA_EINVAL;
    for (int64_t j = 0; j < ny; j++) {
        for (int64_t i = 0; i < nx; i++) {
            const int64_t k = j * nx + i;
            if (!(diag[k] > 0.0) || !std::isfinite(diag[k])) return PCGA_EINVAL;
            if (!std::isfinite(ae[k]) || !std::isfinite(an[k])) return PCGA_EINVAL;
            if (!periodic && i == nx - 1 && ae[k] != 0.0) return PCGA_EINVAL;
            if (j == ny - 1 && an[k] != 0.0) return PCGA_EINVAL;
        }
    }
    return PCGA_OK;
}

// Rows of A whose stencil contains column r (A is symmetric, so these are the
// columns of row r): r itself and its grid neighbours.
int A5View::nbrs(int64_t r, int64_t *out) const {
    const int64_t i = r % nx, j = r / nx;
    int m = 0;
    out[m++] = r;
    if (i > 0) out[m++] = r - 1; else if (periodic) out[m++] = r + nx - 1;
    if (i < nx - 1) out[m++] = r + 1; else if (periodic) out[m++] = r - nx + 1;
    if (j > 0) out[m++] = r - nx;
    if (j < ny - 1) out[m++] = r + nx;
    return m;
}

int CsrView::row(int64_t k, int64_t *cols, double *vals) const {
    int m = 0;
    for (int64_t a = rowptr[k]; a < rowptr[k + 1]; a++, m++) {
        cols[m] = col[a];
        vals[m] = val[a];
    }
    return m;
}

int CsrView::nbrs(int64_t r, int64_t *out) const {
    int m = 0;
    for (int64_t a = rowptr[r]; a < rowptr[r + 1]; a++) out[m++] = col[a];
    return m;
}

int CsrView::validate() {
    if (nrows < 1 || nrows > (int64_t)INT32_MAX || !rowptr || !col || !val) return PCGA_EINVAL;
    if (rowptr[0] != 0) return PCGA_EINVAL;
    longest = 1;
    for (int64_t k = 0; k < nrows; k++) {
        if (rowptr[k + 1] < rowptr[k]) return PCGA_EINVAL;
        longest = std::max<int64_t>(longest, rowptr[k + 1] - rowptr[k]);
        bool diag = false;
        for (int64_t a = rowptr[k]; a < rowptr[k + 1]; a++) {
            const int64_t c = col[a];
            if (c < 0 || c >= nrows || !std::isfinite(val[a])) return PCGA_EINVAL;
            if (a > rowptr[k] && c <= col[a - 1]) return PCGA_EINVAL;
            if (c == k) {
                if (!(val[a] > 0.0)) return PCGA_EINVAL;
                diag = true;
            }
            // the mirror entry (c, k) with the same value
            const int32_t *b0 = col + rowptr[c], *b1 = col + rowptr[c + 1];
            const int32_t *f = std::lower_bound(b0, b1, (int32_t)k);
            if (f == b1 || *f != k || val[f - col] != val[a]) return PCGA_EINVAL;
        }
        if (!diag) return PCGA_EINVAL;
    }
    return PCGA_OK;
}

// Fixed fill (the second Bridson class of Sec. 5: a set number of nonzeros
// per row of the lower factor Z^T, i.e. per column of Z): a finished column
// keeps its `fill` off-diagonal entries of largest magnitude, the larger row
// first among equal magnitudes, and its pivot is formed from what is kept.
static void cap_column(int64_t j, int64_t fill, const std::vector<int64_t> &pattern,
                       const std::vector<double> &w, std::vector<int64_t> &live,
                       std::vector<int64_t> &off) {
    off.clear();
    for (int64_t r : pattern)
        if (r != j && live[r] == j) off.push_back(r);
    // an entry removed by the drop tolerance and inserted again by a later
    // step (possible when couplings of both signs cancel) is listed twice
    std::sort(off.begin(), off.end());
    off.erase(std::unique(off.begin(), off.end()), off.end());
    if ((int64_t)off.size() <= fill) return;
    auto first = [&](int64_t a, int64_t b) {
        const double fa = std::fabs(w[a]), fb = std::fabs(w[b]);
        return fa != fb ? fa > fb : a > b;
    };
    std::nth_element(off.begin(), off.begin() + fill, off.end(), first);
    for (size_t t = (size_t)fill; t < off.size(); t++) live[off[t]] = -1;
}

// The method on any operator view (rows of A and, by symmetry, the rows that
// share a column); the view has been validated.
template <class Op>
static int ainv_build_impl(const Op &A, double tau, int64_t fill, AinvFactor &F, int64_t *bad_row) {
    if (bad_row) *bad_row = -1;
    if (!(tau >= 0.0)) return PCGA_EINVAL;
    const int64_t n = A.n();
    try {
        F.n = n;
        F.colptr.assign(1, 0);
        F.colptr.reserve(n + 1);
        F.rowidx.clear();
        F.val.clear();
        F.D.assign(n, 0.0);

        std::vector<double> w(n, 0.0);        // values of the column being built
        std::vector<int64_t> live(n, -1);     // live[r] == j: entry r present in z_j
        std::vector<int64_t> queued(n, -1);   // queued[i] == j: step i already queued
        std::vector<int64_t> pattern;         // rows ever inserted into z_j
        std::priority_queue<int64_t, std::vector<int64_t>, std::greater<int64_t>> steps;
        std::vector<int64_t> off;             // scratch of cap_column

        std::vector<int64_t> colsv(A.maxrow()), nbv(A.maxrow());
        std::vector<double> valsv(A.maxrow());
        int64_t *cols = colsv.data(), *nb = nbv.data();
        double *vals = valsv.data();

        for (int64_t j = 0; j < n; j++) {
            pattern.clear();
            w[j] = 1.0;
            live[j] = j;
            pattern.push_back(j);
            {
                int m = A.nbrs(j, nb);
                for (int t = 0; t < m; t++)
                    if (nb[t] < j && queued[nb[t]] != j) { queued[nb[t]] = j; steps.push(nb[t]); }
            }
            while (!steps.empty()) {
                const int64_t i = steps.top();
                steps.pop();
                // c = a_i^T z_j
                const int m = A.row(i, cols, vals);
                double c = 0.0;
                for (int t = 0; t < m; t++) {
                    if (live[cols[t]] == j) {
                        const double pr = vals[t] * w[cols[t]];
                        c = c + pr;
                    }
                }
                if (c == 0.0) continue;
                const double mult = c / F.D[i];
                // z_j <- z_j - mult * z_i ; z_i = stored off-diagonals + unit at i
                const int64_t a0 = F.colptr[i], a1 = F.colptr[i + 1];
                for (int64_t a = a0; a <= a1; a++) {
                    const int64_t r = (a < a1) ? (int64_t)F.rowidx[a] : i;
                    const double v = (a < a1) ? F.val[a] : 1.0;
                    const double pr = mult * v;
                    const bool had = (live[r] == j);
                    const double nv = (had ? w[r] : 0.0) - pr;
                    if (nv == 0.0 || std::fabs(nv) < tau) {
                        if (had) live[r] = -1;
                        continue;
                    }
                    w[r] = nv;
                    if (!had) {
                        live[r] = j;
                        pattern.push_back(r);
                        int mm = A.nbrs(r, nb);
                        for (int t = 0; t < mm; t++) {
                            const int64_t s = nb[t];
                            if (s > i && s < j && queued[s] != j) { queued[s] = j; steps.push(s); }
                        }
                    }
                }
            }
            if (fill >= 0) cap_column(j, fill, pattern, w, live, off);
            // p_j = a_j^T z_j
            const int m = A.row(j, cols, vals);
            double p = 0.0;
            for (int t = 0; t < m; t++) {
                if (live[cols[t]] == j) {
                    const double pr = vals[t] * w[cols[t]];
                    p = p + pr;
                }
            }
            if (!(p > 0.0)) {
                if (bad_row) *bad_row = j;
                return PCGA_EBREAKDOWN;
            }
            F.D[j] = p;
            // store the live off-diagonal entries, rows ascending
            std::sort(pattern.begin(), pattern.end());
            for (int64_t r : pattern) {
                if (r != j && live[r] == j) {
                    F.rowidx.push_back((int32_t)r);
                    F.val.push_back(w[r]);
                }
                live[r] = -1;
            }
            F.colptr.push_back((int64_t)F.rowidx.size());
        }
    } catch (const std::bad_alloc &) {
        return PCGA_ENOMEM;
    }
    return PCGA_OK;
}

int ainv_build(const A5View &A, double tau, int64_t fill, AinvFactor &F, int64_t *bad_row) {
    if (bad_row) *bad_row = -1;
    const int st = A.validate();
    if (st) return st;
    return ainv_build_impl(A, tau, fill, F, bad_row);
}

int ainv_build(const CsrView &A, double tau, int64_t fill, AinvFactor &F, int64_t *bad_row) {
    if (bad_row) *bad_row = -1;
    CsrView V = A;
    const int st = V.validate();
    if (st) return st;
    return ainv_build_impl(V, tau, fill, F, bad_row);
}

// The paper's banded factor of T (Sec. 3, six-step pattern scheme).  T keeps
// the entries of A with |col - row| <= 1 in natural ordering: the east-west
// couplings inside each grid row (the periodic wrap lies outside the band).
// Column z_j of the unit upper factor is restricted to rows j-q .. j (the
// dropped set is {(i, j): j > i + q}) and computed by T-orthogonalisation on
// that pattern: for i = j-q .. j-1 in increasing order,
//   c = t_i^T z_j (columns i-1, i, i+1 of row i that lie in the band of z_j,
//   ascending, absent/zero entries skipped), and if c != 0:
//   z_j[r] <- z_j[r] - (c / p_i) z_i[r] for the rows r of z_i inside the band;
// then p_j = t_j^T z_j.  Unfused FP64 in this order.
int fsai_band_build(const A5View &A, int64_t q, AinvFactor &F, int64_t *bad_row) {
    if (bad_row) *bad_row = -1;
    int st = A.validate();
    if (st) return st;
    if (q < 0 || q > 4096) return PCGA_EINVAL;
    const int64_t n = A.n(), nx = A.nx;
    auto t_at = [&](int64_t row, int64_t col) -> double {   // entry of T
        if (col == row) return A.diag[row];
        if (col == row + 1) return (row % nx != nx - 1) ? A.ae[row] : 0.0;
        if (col == row - 1) return (col % nx != nx - 1) ? A.ae[col] : 0.0;
        return 0.0;
    };
    try {
        // band storage: band[j*(q+1) + m] = z_j[j - q + m], m = 0..q (m = q is the unit diagonal)
        std::vector<double> band((size_t)n * (q + 1), 0.0);
        F.n = n;
        F.D.assign(n, 0.0);
        for (int64_t j = 0; j < n; j++) {
            double *zj = &band[(size_t)j * (q + 1)];
            zj[q] = 1.0;
            const int64_t top = j - q;               // row held in zj[0]
            const int64_t lo = top < 0 ? 0 : top;
            for (int64_t i = lo; i < j; i++) {
                double c = 0.0;
                for (int64_t col = i - 1; col <= i + 1; col++) {
                    if (col < 0 || col >= n || col < top || col > j) continue;
                    const double z = zj[col - top];
                    if (z == 0.0) continue;
                    const double pr = t_at(i, col) * z;
                    c = c + pr;
                }
                if (c == 0.0) continue;
                const double mult = c / F.D[i];
                const double *zi = &band[(size_t)i * (q + 1)];   // zi[m] = z_i[i - q + m]
                for (int64_t r = (i - q > lo ? i - q : lo); r <= i; r++) {
                    const double pr = mult * zi[r - (i - q)];
                    zj[r - top] = zj[r - top] - pr;
                }
            }
            double p = 0.0;
            for (int64_t col = j - 1; col <= j + 1; col++) {
                if (col < 0 || col >= n || col < top || col > j) continue;
                const double z = zj[col - top];
                if (z == 0.0) continue;
                const double pr = t_at(j, col) * z;
                p = p + pr;
            }
            if (!(p > 0.0)) {
                if (bad_row) *bad_row = j;
                return PCGA_EBREAKDOWN;
            }
            F.D[j] = p;
        }
        F.colptr.assign(1, 0);
        F.rowidx.clear();
        F.val.clear();
        for (int64_t j = 0; j < n; j++) {
            const double *zj = &band[(size_t)j * (q + 1)];
            for (int64_t m = 0; m < q; m++) {
                const int64_t r = j - q + m;
                if (r >= 0 && zj[m] != 0.0) {
                    F.rowidx.push_back((int32_t)r);
                    F.val.push_back(zj[m]);
                }
            }
            F.colptr.push_back((int64_t)F.rowidx.size());
        }
    } catch (const std::bad_alloc &) {
        return PCGA_ENOMEM;
    }
    return PCGA_OK;
}

}  // namespace pcga
