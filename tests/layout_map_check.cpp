// Host check of the map that lets the Z sweep read Z's values from Z^T's
// value array (sell_shared_values): every mapped step's lanes must read
// exactly the value Z stores (bitwise), and every lane's position must lie
// inside Z^T's values plus the 64-zero block that follows them.
// Usage: layout_map_check nx ny periodic drop_tol file  (file: diag, ae, an
// as float64, n each).  Prints "steps mapped mismatches out_of_bounds".
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <vector>

#include "pcga_host.h"

using namespace pcga;

int main(int argc, char **argv) {
    if (argc != 6) return 2;
    const int64_t nx = atoll(argv[1]), ny = atoll(argv[2]), n = nx * ny;
    std::vector<double> d(n), e(n), a(n);
    std::ifstream f(argv[5], std::ios::binary);
    f.read((char *)d.data(), n * 8);
    f.read((char *)e.data(), n * 8);
    f.read((char *)a.data(), n * 8);
    if (!f) return 3;
    A5View V;
    V.nx = nx;
    V.ny = ny;
    V.periodic = atoi(argv[3]) != 0;
    V.diag = d.data();
    V.ae = e.data();
    V.an = a.data();
    AinvFactor F;
    int64_t bad_row = -1;
    if (ainv_build(V, atof(argv[4]), -1, F, &bad_row)) return 4;
    // Z^T (the CSC of Z read as CSR) and Z (its transpose), as the solver lays them out
    SellLayout zt, z;
    sell_build(n, F.colptr.data(), F.rowidx.data(), F.val.data(), 32, zt);
    std::vector<int64_t> rp(n + 1, 0);
    for (int64_t q = 0; q < F.nnz_off(); q++) rp[F.rowidx[q] + 1]++;
    for (int64_t k = 0; k < n; k++) rp[k + 1] += rp[k];
    std::vector<int32_t> col(F.nnz_off());
    std::vector<double> val(F.nnz_off());
    std::vector<int64_t> pos(rp.begin(), rp.end() - 1);
    for (int64_t j = 0; j < n; j++)
        for (int64_t q = F.colptr[j]; q < F.colptr[j + 1]; q++) {
            const int64_t p = pos[F.rowidx[q]]++;
            col[p] = (int32_t)j;
            val[p] = F.val[q];
        }
    sell_build(n, rp.data(), col.data(), val.data(), 32, z);
    std::vector<int32_t> ma, mb, mk;
    const int64_t mapped = sell_shared_values(zt, z, zt.entries(), ma, mb, mk);
    std::vector<double> ext(zt.val);
    ext.resize(zt.entries() + 64, 0.0);
    int64_t steps = 0, mism = 0, oob = 0;
    for (int64_t s = 0; s < z.nslices(); s++) {
        if (z.toff[s] < 0) continue;
        const int64_t w = z.meta[s] >> 8;
        for (int64_t c = 0; c < w; c++) {
            steps++;
            const int64_t ti = z.toff[s] + c;
            if (mk[ti] < 0) continue;
            for (int64_t l = 0; l < 64; l++) {
                const int64_t p = (l < mk[ti] ? (int64_t)ma[ti] : (int64_t)mb[ti]) + l;
                if (p < 0 || p >= (int64_t)ext.size()) {
                    oob++;
                    continue;
                }
                if (z.row0[s] + l >= n) continue;
                const double zv = z.val[z.off[s] + c * 64 + l];
                if (std::memcmp(&zv, &ext[p], sizeof(double)) != 0) mism++;
            }
        }
    }
    printf("%lld %lld %lld %lld\n", (long long)steps, (long long)mapped, (long long)mism, (long long)oob);
    return 0;
}
