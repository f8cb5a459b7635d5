// layout.cpp -- sliced ELL with per-slice lanes per row (see SellLayout).
//
// Rows are cut into 64-lane slices greedily in natural order.  A slice starts
// with one lane per row (64 rows); if its longest row would make it wider
// than `target_width` steps, the lanes per row double (and the rows per
// slice halve) until it fits or one row owns all 64 lanes.  Ordinary ocean
// rows (about ten entries) therefore stay one-lane-per-row, while the long
// polar rows of the approximate inverse are spread over many lanes, which
// bounds the work of every wavefront.
//
// In a one-lane-per-row slice the rows' column offsets (col - row) are
// nearly the same set (the approximate inverse's pattern repeats from cell
// to cell): the slice then stores the sorted union of the offsets as a table
// and step c of every lane holds the entry at offset table[c] (0 if the row
// has none).  The kernels compute the gathered columns from the table, so no
// per-lane index has to arrive before a gather can be issued; the padding is
// that of plain ELL (1.13x at 1442x1021).

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>

#include "pcga_host.h"

namespace pcga {

void sell_build(int64_t m, const int64_t *rowptr, const int32_t *col, const double *val,
                int target_width, SellLayout &L) {
    if (target_width < 1) target_width = 1;
    L.nrows_total = m;
    L.row0.clear();
    L.meta.clear();
    L.off.assign(1, 0);
    L.toff.clear();
    L.tab.clear();
    L.idx.clear();
    L.val.clear();
    std::vector<int64_t> uni;
    int64_t R = 0;
    while (R < m) {
        int lg = 0;
        int64_t width = 0, maxlen = 0;
        for (lg = 0; lg <= 6; lg++) {
            const int64_t lpr = int64_t(1) << lg;
            const int64_t nr = 64 >> lg;
            const int64_t end = std::min(m, R + nr);
            maxlen = 0;
            for (int64_t r = R; r < end; r++) maxlen = std::max(maxlen, rowptr[r + 1] - rowptr[r]);
            width = (maxlen + lpr - 1) / lpr;
            if (width <= target_width || lg == 6) break;
        }
        const int64_t lpr = int64_t(1) << lg;
        const int64_t nr = 64 >> lg;
        const int64_t end = std::min(m, R + nr);
        // one lane per row: the union of the rows' column offsets, when it is
        // not much wider than the longest row, becomes the slice's table
        bool uniform = false;
        if (lg == 0) {
            uni.clear();
            for (int64_t r = R; r < end; r++)
                for (int64_t a = rowptr[r]; a < rowptr[r + 1]; a++) uni.push_back(col[a] - r);
            std::sort(uni.begin(), uni.end());
            uni.erase(std::unique(uni.begin(), uni.end()), uni.end());
            // the kernels hold a slice's table in one register of the
            // wavefront (lane c holds table[c]), so a table has at most 64 steps
            if ((int64_t)uni.size() <= kTableMax &&
                (int64_t)uni.size() <= maxlen + std::max<int64_t>(2, maxlen / 4)) {
                uniform = true;
                width = (int64_t)uni.size();
            }
        }
        L.row0.push_back((int32_t)R);
        L.meta.push_back((int32_t)(lg | (width << 8)));
        L.toff.push_back(uniform ? (int32_t)L.tab.size() : -1);
        if (uniform)
            for (int64_t o : uni) L.tab.push_back((int32_t)o);
        const int64_t base = L.off.back();
        L.idx.resize(base + width * 64);
        L.val.resize(base + width * 64);
        for (int64_t c = 0; c < width; c++) {
            for (int l = 0; l < 64; l++) {
                const int64_t r = R + (l >> lg);
                const int64_t pos = base + c * 64 + l;
                const int32_t own = (int32_t)std::min(r, m - 1);
                L.idx[pos] = own;
                L.val[pos] = 0.0;
                if (r >= m) continue;
                if (uniform) {
                    // the row's entry at column r + uni[c], if it has one
                    const int64_t want = r + uni[c];
                    const int32_t *b0 = col + rowptr[r], *b1 = col + rowptr[r + 1];
                    const int32_t *hit = std::lower_bound(b0, b1, (int32_t)want);
                    if (hit != b1 && *hit == want) {
                        L.idx[pos] = *hit;
                        L.val[pos] = val[hit - col];
                    }
                } else {
                    const int64_t e = c * lpr + (l & (lpr - 1));
                    if (e < rowptr[r + 1] - rowptr[r]) {
                        L.idx[pos] = col[rowptr[r] + e];
                        L.val[pos] = val[rowptr[r] + e];
                    }
                }
            }
        }
        L.off.push_back(base + width * 64);
        R += nr;
    }
}

bool sell_check(const SellLayout &L) {
    const int64_t ns = L.nslices();
    if ((int64_t)L.meta.size() != ns || (int64_t)L.toff.size() != ns ||
        (int64_t)L.off.size() != ns + 1)
        return false;
    for (int64_t s = 0; s < ns; s++) {
        const int lg = L.meta[s] & 255;
        const int64_t width = L.meta[s] >> 8;
        if (lg < 0 || lg > 6 || width < 0) return false;
        if (L.off[s + 1] - L.off[s] != width * 64) return false;
        if (L.toff[s] >= 0) {
            if (lg != 0 || width > kTableMax) return false;
            if ((int64_t)L.toff[s] + width > (int64_t)L.tab.size()) return false;
        }
    }
    return true;
}

bool sell_narrow(SellLayout &L, bool lower) {
    const int64_t m = L.nrows_total;
    std::vector<uint16_t> d(L.idx.size());
    for (int64_t s = 0; s < L.nslices(); s++) {
        const int lg = L.meta[s] & 255;
        for (int64_t pos = L.off[s]; pos < L.off[s + 1]; pos++) {
            const int l = (int)((pos - L.off[s]) % 64);
            const int64_t r = std::min<int64_t>(L.row0[s] + (l >> lg), m - 1);
            const int64_t c = L.idx[pos];
            const int64_t dist = lower ? r - c : c - r;
            if (dist < 0 || dist > 65535) return false;
            d[pos] = (uint16_t)dist;
        }
    }
    L.dist.swap(d);
    L.idx.clear();
    L.idx.shrink_to_fit();
    L.narrow = true;
    return true;
}

// Z's values are Z^T's values in another order: Z[i, i+o] = Z^T[i+o, i].
// For a table slice of Z (rows R..R+63, one lane per row) the 64 values of
// step c (offset o) are the entries at offset -o of Z^T's rows R+o..R+o+63.
// A lane whose Z^T row lies in a table slice of Z^T with -o in its table
// finds its value at that slice's step (consecutive lanes at consecutive
// positions); a lane whose value is +0 may instead read the block of 64
// zeros at zero_base (Z^T stores nothing there, or it lies in a slice
// without a table).  A step is mapped when its lanes form at most two such
// runs and every value agrees bitwise with the one Z stores (lanes past the
// last row are free): lanes l < k[c] read zt.val[a[c] + l], lanes l >= k[c]
// read zt.val[b[c] + l]; k[c] = -1: the step reads Z's own values.  a, b, k
// run parallel to z.tab.
int64_t sell_shared_values(const SellLayout &zt, const SellLayout &z, int64_t zero_base,
                           std::vector<int32_t> &a, std::vector<int32_t> &b,
                           std::vector<int32_t> &k) {
    const int64_t n = z.nrows_total;
    a.assign(z.tab.size(), 0);
    b.assign(z.tab.size(), 0);
    k.assign(z.tab.size(), -1);
    if (zt.nrows_total != n || zero_base + 64 > INT32_MAX) return 0;
    // the table slice of Z^T that holds row j with one lane per row, else -1
    std::vector<int32_t> slice_of(n, -1);
    for (int64_t s = 0; s < zt.nslices(); s++) {
        if (zt.toff[s] < 0 || (zt.meta[s] & 255) != 0) continue;
        for (int64_t r = zt.row0[s]; r < std::min<int64_t>(n, zt.row0[s] + 64); r++) slice_of[r] = (int32_t)s;
    }
    // step of offset -o in table slice s, or -1
    auto step_of = [&](int64_t s, int64_t o) -> int64_t {
        const int64_t w = zt.meta[s] >> 8;
        const int32_t *t = zt.tab.data() + zt.toff[s];
        const int32_t *p = std::lower_bound(t, t + w, (int32_t)-o);
        return (p != t + w && *p == -o) ? (int64_t)(p - t) : -1;
    };
    // per lane: where its value can be read
    constexpr int64_t kFree = INT64_MIN;       // lane past the last row (any in-bounds position)
    constexpr int64_t kZero = INT64_MIN + 1;   // +0: the zero block
    int64_t mapped = 0;
    int64_t base[64];   // position - lane, or kFree / kZero
    for (int64_t s = 0; s < z.nslices(); s++) {
        if (z.toff[s] < 0 || (z.meta[s] & 255) != 0) continue;
        const int64_t R = z.row0[s], w = z.meta[s] >> 8;
        for (int64_t c = 0; c < w; c++) {
            const int64_t ti = z.toff[s] + c;
            const int64_t o = z.tab[ti];
            bool ok = o > 0;
            for (int64_t l = 0; ok && l < 64; l++) {
                const int64_t i = R + l;
                if (i >= n) {
                    base[l] = kFree;
                    continue;
                }
                const double zv = z.val[z.off[s] + c * 64 + l];
                const int64_t j = i + o;
                int64_t p = -1;
                if (j < n && slice_of[j] >= 0) {
                    const int64_t s1 = slice_of[j], c1 = step_of(s1, o);
                    if (c1 >= 0) p = zt.off[s1] + c1 * 64 + (j - zt.row0[s1]);
                }
                const double zero = 0.0;
                if (p >= 0 && std::memcmp(&zv, &zt.val[p], sizeof(double)) == 0)
                    base[l] = p - l;
                else if (std::memcmp(&zv, &zero, sizeof(double)) == 0)
                    base[l] = kZero;
                else
                    ok = false;
            }
            if (!ok) continue;
            // at most two runs (free lanes join any run): run 1 = lanes < split
            int64_t r1 = kFree, r2 = kFree, split = 64, first1 = -1;
            for (int64_t l = 0; ok && l < 64; l++) {
                if (base[l] == kFree) continue;
                if (split == 64) {
                    if (r1 == kFree) {
                        r1 = base[l];
                        first1 = l;
                    } else if (base[l] != r1) {
                        split = l;
                        r2 = base[l];
                    }
                } else if (base[l] != r2) {
                    ok = false;
                }
            }
            if (!ok || r1 == kFree) continue;
            // a zero run reads zero_base + (lane - its first lane)
            const int64_t b1 = r1 == kZero ? zero_base - first1 : r1;
            const int64_t b2 = r2 == kFree ? b1 : (r2 == kZero ? zero_base - split : r2);
            // positions of all lanes inside [0, zero_base + 64)
            bool inb = true;
            for (int64_t l = 0; l < 64; l++) {
                const int64_t p = (l < split ? b1 : b2) + l;
                if (p < 0 || p >= zero_base + 64) inb = false;
            }
            if (!inb || b1 > INT32_MAX || b2 > INT32_MAX || b2 < INT32_MIN) continue;
            a[ti] = (int32_t)b1;
            b[ti] = (int32_t)b2;
            k[ti] = (int32_t)split;
            mapped++;
        }
    }
    return mapped;
}

}  // namespace pcga
