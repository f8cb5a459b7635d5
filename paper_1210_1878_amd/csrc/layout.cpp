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
#include <cstdint>

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

}  // namespace pcga
