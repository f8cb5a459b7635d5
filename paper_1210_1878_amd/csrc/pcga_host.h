// pcga_host.h -- host-side data structures of the PCG-AINV library.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "pcgainv.h"

namespace pcga {

// Read-only view of the five-point operator in A5 form (see pcgainv.h).
struct A5View {
    int64_t nx = 0, ny = 0;
    bool periodic = false;
    const double *diag = nullptr, *ae = nullptr, *an = nullptr;

    int64_t n() const { return nx * ny; }
    int64_t maxrow() const { return 5; }
    int row(int64_t k, int64_t *cols, double *vals) const;
    // rows of A with an entry in column r (by symmetry, the columns of row r)
    int nbrs(int64_t r, int64_t *out) const;
    int validate() const;
};

// Read-only view of a general sparse SPD operator in CSR (see pcgainv.h):
// rows with strictly ascending columns, the diagonal present and positive,
// symmetric entry by entry.
struct CsrView {
    int64_t nrows = 0;
    const int64_t *rowptr = nullptr;
    const int32_t *col = nullptr;
    const double *val = nullptr;
    int64_t longest = 1;   // set by validate()

    int64_t n() const { return nrows; }
    int64_t maxrow() const { return longest; }
    int row(int64_t k, int64_t *cols, double *vals) const;
    int nbrs(int64_t r, int64_t *out) const;
    int validate();
};

// Unit upper triangular Z (strict upper part in CSC, rows ascending) and D.
struct AinvFactor {
    int64_t n = 0;
    std::vector<int64_t> colptr;
    std::vector<int32_t> rowidx;
    std::vector<double> val;
    std::vector<double> D;
    int64_t nnz_off() const { return colptr.empty() ? 0 : colptr.back(); }
};

// fill < 0: no cap on the off-diagonal entries per column
int ainv_build(const A5View &A, double tau, int64_t fill, AinvFactor &F, int64_t *bad_row);
int ainv_build(const CsrView &A, double tau, int64_t fill, AinvFactor &F, int64_t *bad_row);
int fsai_band_build(const A5View &A, int64_t q, AinvFactor &F, int64_t *bad_row);

// Sliced ELL with a per-slice number of lanes per row ("SELL-L").
//   A slice is one 64-lane wavefront.  It covers `nrows = 64 >> lpr_log2`
//   consecutive rows starting at `row0`; lane l works on row
//   row0 + (l >> lpr_log2) and takes entries e = c*2^lpr_log2 + (l & (2^lpr-1))
//   for c = 0..width-1.  Entry (c, l) of slice s is stored at
//   off[s] + c*64 + l (column-major in the slice, so each step c is one
//   coalesced 64-wide load).  Padding entries have value 0 and point to the
//   lane's own row.
//   Narrow form: when every entry lies within 65535 rows of its lane's row
//   (rows past the matrix count as its last row), the column is stored as
//   the 16-bit distance |col - row| instead (dist, same positions; idx is
//   then empty); the direction is fixed per matrix (Z^T: col <= row, Z:
//   col >= row).
struct SellLayout {
    int64_t nrows_total = 0;
    std::vector<int32_t> row0;      // [nslices]
    std::vector<int32_t> meta;      // [nslices]: lpr_log2 | (width << 8)
    std::vector<int64_t> off;       // [nslices + 1] entry offsets
    std::vector<int32_t> toff;      // [nslices] start of the slice's offset table in tab, -1: none
    std::vector<int32_t> tab;       // offset tables (col - row, ascending) of table slices
    std::vector<int32_t> idx;       // [off.back()] (empty in the narrow form)
    std::vector<uint16_t> dist;     // [off.back()] (narrow form only)
    std::vector<double> val;        // [off.back()]
    bool narrow = false;
    int64_t nslices() const { return (int64_t)row0.size(); }
    int64_t entries() const { return off.empty() ? 0 : off.back(); }
};

// Most entry steps of a table slice: the kernels keep a slice's offset table
// in one wavefront register, lane c holding table[c].
constexpr int64_t kTableMax = 64;

// rows given as CSR (rowptr[m+1], col, val with columns ascending per row).
void sell_build(int64_t m, const int64_t *rowptr, const int32_t *col, const double *val,
                int target_width, SellLayout &L);

// Structural invariants the kernels rely on: per-slice entry counts match
// the widths, and every table slice is one lane per row with at most
// kTableMax steps and a table inside `tab`.
bool sell_check(const SellLayout &L);

// Switch L to the narrow form when it fits (lower: every column <= its row,
// else every column >= its row).  Returns whether it did.
bool sell_narrow(SellLayout &L, bool lower);

// Map the steps of Z's table slices onto Z^T's value array where the values
// agree bitwise (see layout.cpp); a block of 64 zeros at zero_base (after
// Z^T's entries) serves lanes whose value is +0.  a, b, k run parallel to
// z.tab.  Returns the number of mapped steps.
int64_t sell_shared_values(const SellLayout &zt, const SellLayout &z, int64_t zero_base,
                           std::vector<int32_t> &a, std::vector<int32_t> &b,
                           std::vector<int32_t> &k);

std::string &last_error();
int fail(int code, const std::string &msg);

}  // namespace pcga
