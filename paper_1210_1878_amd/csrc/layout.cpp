// layout.cpp -- sliced ELL with per-slice lanes per row (see SellLayout).
//
// Rows are cut into 64-lane slices greedily in natural order.  A slice starts
// with one lane per row (64 rows); if its longest row would make it wider
// than `target_width` steps, the lanes per row double (and the rows per
// slice halve) until it fits or one row owns all 64 lanes.  Ordinary ocean
// rows (about ten entries) therefore stay one-lane-per-row, while the long
// polar rows of the approximate inverse are spread over many lanes, which
// bounds the work of every wavefront.

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
    L.idx.clear();
    L.val.clear();
    int64_t R = 0;
    while (R < m) {
        int lg = 0;
        int64_t width = 0;
        for (lg = 0; lg <= 6; lg++) {
            const int64_t lpr = int64_t(1) << lg;
            const int64_t nr = 64 >> lg;
            const int64_t end = std::min(m, R + nr);
            int64_t maxlen = 0;
            for (int64_t r = R; r < end; r++) maxlen = std::max(maxlen, rowptr[r + 1] - rowptr[r]);
            width = (maxlen + lpr - 1) / lpr;
            if (width <= target_width || lg == 6) break;
        }
        const int64_t lpr = int64_t(1) << lg;
        const int64_t nr = 64 >> lg;
        L.row0.push_back((int32_t)R);
        L.meta.push_back((int32_t)(lg | (width << 8)));
        const int64_t base = L.off.back();
        L.idx.resize(base + width * 64);
        L.val.resize(base + width * 64);
        for (int64_t c = 0; c < width; c++) {
            for (int l = 0; l < 64; l++) {
                const int64_t r = R + (l >> lg);
                const int64_t e = c * lpr + (l & (lpr - 1));
                const int64_t pos = base + c * 64 + l;
                if (r < m && e < rowptr[r + 1] - rowptr[r]) {
                    L.idx[pos] = col[rowptr[r] + e];
                    L.val[pos] = val[rowptr[r] + e];
                } else {
                    L.idx[pos] = (int32_t)std::min(r, m - 1);
                    L.val[pos] = 0.0;
                }
            }
        }
        L.off.push_back(base + width * 64);
        R += nr;
    }
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
