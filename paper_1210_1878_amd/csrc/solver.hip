// solver.hip -- C ABI of the PCG-AINV library: setup handles, workspace
// layout, and the host driver of the device iteration.
//
// A solve is: a prologue (r0 = b - A x0, t = D^-1 Z^T r0, s0 = Z t, rho0,
// d0 = s0; Algorithm 1 lines 1-4) and then chunks of `chunk` iterations,
// each replayed from a captured HIP graph (or launched directly).  Every
// kernel first reads the device `done` flag, so the iterations after
// convergence cost one empty launch each and the iteration count is exact.
// The host keeps two chunks in flight: it enqueues chunk c+1, then waits for
// chunk c's snapshot of the control block (scalars, flag, history ring).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.h"
#include "pcga_host.h"
#include "solver_internal.h"

namespace pcga {

std::string &last_error() {
    static thread_local std::string msg;
    return msg;
}

int fail(int code, const std::string &msg) {
    last_error() = msg;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(PCGA_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)

static int map_status(int s) {
    switch (s) {
        case kStOk: return PCGA_OK;
        case kStNoconv: return PCGA_NOCONV;
        case kStBreak: return PCGA_EBREAKDOWN;
        case kStNan: return PCGA_ENAN;
        default: return PCGA_EHIP;
    }
}

}  // namespace pcga

using namespace pcga;

struct pcga_ainv {
    AinvFactor F;
};

// Device memory of the allocation-free solve (pcga_pcg_solve_noalloc): 64 MiB
// per device, enough for the FP64 vectors of a grid of about 1.19 M cells.
constexpr size_t kNoallocBytes = PCGA_NOALLOC_MAX_BYTES;
static_assert(kNoallocBytes % 256 == 0, "scratch size must keep 256-byte alignment");
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

// ---------------------------------------------------------------------------
// Workspace carving: one bump pass computes the size (base == nullptr) or
// assigns the pointers.
// ---------------------------------------------------------------------------
namespace {

struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base((char *)b) {}
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

struct HostLayouts {
    SellLayout zt, z;
    SellLayout a;   // a general sparse A (CSR input); empty for the five-point operator
    // FP64: Z's table steps mapped onto Z^T's values (sell_shared_values)
    std::vector<int32_t> za, zb, zk;
    int64_t zmapped = 0;
};

int build_layouts(const AinvFactor &F, int target_width, HostLayouts &H) {
    try {
        const int64_t n = F.n;
        // rows of Z^T = columns of Z: the CSC arrays read as CSR
        sell_build(n, F.colptr.data(), F.rowidx.data(), F.val.data(), target_width, H.zt);
        // rows of Z: transpose the CSC (columns visited in increasing order,
        // so each row's columns come out ascending)
        std::vector<int64_t> rp(n + 1, 0);
        for (int64_t a = 0; a < F.nnz_off(); a++) rp[F.rowidx[a] + 1]++;
        for (int64_t k = 0; k < n; k++) rp[k + 1] += rp[k];
        std::vector<int32_t> col(F.nnz_off());
        std::vector<double> val(F.nnz_off());
        std::vector<int64_t> pos(rp.begin(), rp.end() - 1);
        for (int64_t j = 0; j < n; j++)
            for (int64_t a = F.colptr[j]; a < F.colptr[j + 1]; a++) {
                const int64_t p = pos[F.rowidx[a]]++;
                col[p] = (int32_t)j;
                val[p] = F.val[a];
            }
        sell_build(n, rp.data(), col.data(), val.data(), target_width, H.z);
        // 16-bit distances when both fit (one format per solver)
        if (sell_narrow(H.zt, true) && !sell_narrow(H.z, false)) {
            // Z^T fits but Z does not (cannot happen for a transpose pair of
            // the same pattern; kept consistent anyway): rebuild Z^T wide
            sell_build(n, F.colptr.data(), F.rowidx.data(), F.val.data(), target_width, H.zt);
        }
    } catch (const std::bad_alloc &) {
        return fail(PCGA_ENOMEM, "host allocation failed while building sliced-ELL layouts");
    }
    if (!sell_check(H.zt) || !sell_check(H.z))
        return fail(PCGA_EINVAL, "internal: sliced-ELL layout violates its invariants");
    return PCGA_OK;
}

}  // namespace


namespace {

// Assign all device pointers of S from `base` (or size them when null).
size_t carve(pcga_solver &S, void *base, const HostLayouts &H) {
    Carver C(base);
    const int64_t n = S.n;
    const bool f64 = S.precision == PCGA_FP64;
    if (!S.csr) {
        S.A64.diag = C.take<double>(n);
        S.A64.ae = C.take<double>(n);
        S.A64.an = C.take<double>(n);
    }
    if (S.precision == PCGA_MIXED_A32) {
        S.A32.diag = C.take<float>(n);
        S.A32.ae = C.take<float>(n);
        S.A32.an = C.take<float>(n);
    }
    // extra: zeros after the values (the block that Z's mapped steps read
    // for lanes whose value is zero)
    auto sell = [&](const SellLayout &L, auto &dst, auto tag, int64_t extra = 0) {
        using T = decltype(tag);
        dst.row0 = C.take<int32_t>(L.nslices());
        dst.meta = C.take<int32_t>(L.nslices());
        dst.off = C.take<int64_t>(L.nslices() + 1);
        dst.toff = C.take<int32_t>(std::max<int64_t>(L.nslices(), 1));
        dst.tab = C.take<int32_t>(std::max<int64_t>((int64_t)L.tab.size(), 1));
        if (L.narrow) {
            dst.idx = nullptr;
            dst.dist = C.take<uint16_t>(std::max<int64_t>(L.entries(), 1));
        } else {
            dst.idx = C.take<int32_t>(std::max<int64_t>(L.entries(), 1));
            dst.dist = nullptr;
        }
        dst.val = C.take<T>(std::max<int64_t>(L.entries(), 1) + extra);
        dst.nslices = (int32_t)L.nslices();
        dst.nrows = (int32_t)L.nrows_total;
    };
    if (S.csr) {
        sell(H.a, S.a64, double());
        S.bnd_a = C.take<int32_t>(kWavesPerBlock * kMaxBlocks + 1);
    }
    if (S.band_q > 0) {
        if (f64)
            S.zb64 = C.take<double>((size_t)S.band_q * n);
        else
            S.zb32 = C.take<float>((size_t)S.band_q * n);
    }
    if (f64) {
        S.dinv64 = C.take<double>(n);
        sell(H.zt, S.zt64, double(), H.zmapped > 0 ? 64 : 0);
        sell(H.z, S.z64, double());
        if (H.zmapped > 0) {
            const int64_t nt = std::max<int64_t>((int64_t)H.z.tab.size(), 1);
            S.z64.alt_a = C.take<int32_t>(nt);
            S.z64.alt_b = C.take<int32_t>(nt);
            S.z64.alt_k = C.take<int32_t>(nt);
            S.z64.alt = S.zt64.val;
        }
        S.x = C.take<double>(n);
        S.r[0] = C.take<double>(n);
        S.r[1] = C.take<double>(n);
        S.s = C.take<double>(n);
        S.d[0] = C.take<double>(n);
        S.d[1] = C.take<double>(n);
        S.q = C.take<double>(n);
        S.t = C.take<double>(n);
    } else {
        S.dinv32 = C.take<float>(n);
        sell(H.zt, S.zt32, float());
        sell(H.z, S.z32, float());
        S.e32 = C.take<float>(n);
        S.r32[0] = C.take<float>(n);
        S.r32[1] = C.take<float>(n);
        S.s32 = C.take<float>(n);
        S.d32[0] = C.take<float>(n);
        S.d32[1] = C.take<float>(n);
        S.q32 = C.take<float>(n);
        S.t32 = C.take<float>(n);
        S.tmp32 = C.take<float>(n);
        S.x64[0] = C.take<double>(n);
        S.x64[1] = C.take<double>(n);
    }
    S.bnd_zt = C.take<int32_t>(kWavesPerBlock * kMaxBlocks + 1);
    S.bnd_z = C.take<int32_t>(kWavesPerBlock * kMaxBlocks + 1);
    S.bnd_zt_b = C.take<int32_t>(kMaxBlocks + 1);
    S.bnd_z_b = C.take<int32_t>(kMaxBlocks + 1);
    S.P.dq = C.take<double>(kMaxBlocks);
    S.P.rr = C.take<double>(kMaxBlocks);
    S.P.sr = C.take<double>(kMaxBlocks);
    S.P.res = C.take<double>(3 * (size_t)kMaxBlocks);
    S.cb = C.take<CtlBlock>(1);
    return C.off + 256;
}

A5View view_of(const pcga_a5_t *A) {
    A5View V;
    V.nx = A->nx;
    V.ny = A->ny;
    V.periodic = (A->flags & PCGA_PERIODIC_X) != 0;
    V.diag = A->diag;
    V.ae = A->ae;
    V.an = A->an;
    return V;
}

int check_a5(const pcga_a5_t *A) {
    if (!A) return fail(PCGA_EINVAL, "A is NULL");
    if (A->flags & ~PCGA_PERIODIC_X) return fail(PCGA_EINVAL, "unknown flag bits in A->flags");
    A5View V = view_of(A);
    if (V.validate() != PCGA_OK)
        return fail(PCGA_EINVAL,
                    "invalid A5 operator (shape, non-positive/non-finite diagonal, or "
                    "couplings across a non-periodic edge / the last row)");
    return PCGA_OK;
}

// Default sliced-ELL target width (entry steps) by precision, as the autotuner
// picks it at 1442 x 1021 (FP64 with 1280 workgroups: 86.6-87.4 us per
// iteration at 24 against 90.3-91.7 at 32; mixed inner: 51.5 us at 24
// against 52.3 at 16).
constexpr int kTargetWidth = 24, kTargetWidthMixed = 24;
constexpr int kMaxSliceWidth = 64;
int default_width(int precision) { return precision != PCGA_FP64 ? kTargetWidthMixed : kTargetWidth; }

// Per-slice work estimate, in units of about 10 ns of one wavefront's time:
// a fixed part (headers, own-row operands, the pipeline's drain at the end of
// the slice) plus a part per entry step, which costs a slice with per-lane
// indices (index load, then gather) more than twice what it costs a table
// slice.  Fitted to per-wavefront timings of the FP64 Z^T and Z sweeps at
// 1442 x 1021 (table: 1.6 us + 0.14-0.20 us per step; per-lane: 0.6-1.2 us
// + 0.37-0.44 us per step).
std::vector<int32_t> slice_costs(const SellLayout &L) {
    std::vector<int32_t> c(L.nslices());
    for (int64_t s = 0; s < L.nslices(); s++) {
        const int32_t width = L.meta[s] >> 8;
        c[s] = L.toff[s] >= 0 ? 160 + 17 * width : 90 + 40 * width;
    }
    return c;
}

// Contiguous slice ranges for G parts (wavefronts, or workgroups of a batch
// slot) with equal estimated work.
std::vector<int32_t> balanced_bounds(const std::vector<int32_t> &cost, int G) {
    const int64_t ns = (int64_t)cost.size();
    std::vector<int32_t> b(G + 1, 0);
    int64_t total = 0;
    for (int32_t c : cost) total += c;
    int64_t acc = 0, s = 0;
    for (int L = 1; L < G; L++) {
        const int64_t target = (total * L) / G;
        while (s < ns && acc + cost[s] / 2 < target) acc += cost[s++];
        b[L] = (int32_t)s;
    }
    b[G] = (int32_t)ns;
    for (int L = 1; L <= G; L++) b[L] = std::max(b[L], b[L - 1]);
    return b;
}

// Which streams of an iteration stay resident in the memory-side cache.  The
// iteration kernels read, per iteration, the vectors (9 of n words: x or e,
// r[2], s, d[2], q, t, D^-1), the FP64 operator arrays diag, ae, an, and the
// values and indices of Z^T and Z.  The vectors are kept first (each is read
// by two or three kernels), then Z^T values, Z values, Z^T indices, Z
// indices, as long as the total fits the budget; the streams left over are
// read with non-temporal loads so that they do not evict the resident ones
// (cycling a working set larger than the cache through it would evict
// everything before its reuse).
void cache_plan(pcga_solver &S, const HostLayouts &H) {
    const double w = S.precision == PCGA_FP64 ? 8.0 : 4.0;
    const double ib = H.zt.narrow ? 2.0 : 4.0;
    const double ezt = (double)H.zt.entries(), ez = (double)H.z.entries();
    const double streams[4] = {w * ezt, w * ez, ib * ezt, ib * ez};   // kept in this order
    const double op_bytes = S.csr ? 12.0 * (double)H.a.entries() : 24.0 * (double)S.n;
    double used = 9.0 * w * (double)S.n + op_bytes;
    int kept = 0;
    while (kept < 4 && used + streams[kept] <= kResidentBudget) used += streams[kept++];
    // A resident set this close to the cache's size made the iteration time
    // depend on where the workspace lies (at 1442 x 1021, 244 MB, 91% full:
    // 96-106 us over twelve bases); the solution x, read and written once per
    // iteration and never gathered, is then streamed instead (87% full:
    // 98.0-98.9 us).
    bool nt_x = false;
    if (S.precision == PCGA_FP64 && used > kSpillFraction * kMallBytes) {
        used -= w * (double)S.n;
        nt_x = true;
    }
    // streams not kept: Z idx (kept < 4), Z^T idx (< 3), Z val (< 2), Z^T val (< 1)
    const int nar = H.zt.narrow ? kFmtNarrow : 0;
    S.fmt_zt = nar | (kept < 3 ? kFmtNtIdx : 0) | (kept < 1 ? kFmtNtVal : 0) | (nt_x ? kFmtNtX : 0);
    S.fmt_z = nar | (kept < 4 ? kFmtNtIdx : 0) | (kept < 2 ? kFmtNtVal : 0);
    // Z's mapped steps read Z^T's values (resident when kept >= 1)
    if (H.zmapped > 0 && S.precision == PCGA_FP64 && kept >= 1) S.fmt_z |= kFmtZtVal;
}

int upload_bounds(pcga_solver &S) {
    const std::vector<int32_t> bz = balanced_bounds(S.cost_zt, S.g_zt * kWavesPerBlock);
    const std::vector<int32_t> b = balanced_bounds(S.cost_z, S.g_z * kWavesPerBlock);
    const int gb = slot_blocks(S.n);
    const std::vector<int32_t> bzb = balanced_bounds(S.cost_zt, gb);
    const std::vector<int32_t> bb = balanced_bounds(S.cost_z, gb);
    hipError_t e = hipMemcpyAsync(S.bnd_zt, bz.data(), bz.size() * 4, hipMemcpyHostToDevice, S.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(S.bnd_z, b.data(), b.size() * 4, hipMemcpyHostToDevice, S.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(S.bnd_zt_b, bzb.data(), bzb.size() * 4, hipMemcpyHostToDevice, S.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(S.bnd_z_b, bb.data(), bb.size() * 4, hipMemcpyHostToDevice, S.stream);
    std::vector<int32_t> ba;
    if (S.csr) {
        ba = balanced_bounds(S.cost_a, S.g_a * kWavesPerBlock);
        if (e == hipSuccess) e = hipMemcpyAsync(S.bnd_a, ba.data(), ba.size() * 4, hipMemcpyHostToDevice, S.stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(S.stream);
    if (e != hipSuccess) return fail(PCGA_EHIP, std::string("bounds upload: ") + hipGetErrorString(e));
    return PCGA_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
// Width q of Z's band (largest j - i over stored entries Z[i, j]) when it is
// at most kMaxBand, else 0 (also 0 for Z = I).
static int band_width(const AinvFactor &F) {
    int64_t q = 0;
    for (int64_t j = 0; j < F.n; j++)
        for (int64_t a = F.colptr[j]; a < F.colptr[j + 1]; a++) {
            q = std::max<int64_t>(q, j - F.rowidx[a]);
            if (q > kMaxBand) return 0;
        }
    return (int)q;
}

// Z by diagonals: zb[(m-1) n + j] = Z[j-m, j], m = 1..q (0 where not stored).
static std::vector<double> band_diagonals(const AinvFactor &F, int q) {
    std::vector<double> zb((size_t)q * F.n, 0.0);
    for (int64_t j = 0; j < F.n; j++)
        for (int64_t a = F.colptr[j]; a < F.colptr[j + 1]; a++)
            zb[(size_t)(j - F.rowidx[a] - 1) * F.n + j] = F.val[a];
    return zb;
}

namespace {

// The operator a solver is built for: the five-point A5 arrays, or a general
// sparse SPD matrix in CSR.
struct OpDesc {
    const pcga_a5_t *a5 = nullptr;
    CsrView csr;
    bool is_csr() const { return csr.rowptr != nullptr; }
    int64_t n() const { return is_csr() ? csr.nrows : (int64_t)a5->nx * a5->ny; }
    int set_csr(const pcga_csr_t *A) {
        if (!A) return fail(PCGA_EINVAL, "A is NULL");
        csr.nrows = A->n;
        csr.rowptr = A->rowptr;
        csr.col = A->col;
        csr.val = A->val;
        if (csr.validate() != PCGA_OK) {
            csr.rowptr = nullptr;
            return fail(PCGA_EINVAL,
                        "CSR A: needs n >= 1, rowptr[0] = 0 and monotone, columns strictly "
                        "ascending in each row, a positive diagonal, finite values and "
                        "A[i,j] == A[j,i]");
        }
        return PCGA_OK;
    }
    int check() const { return is_csr() ? PCGA_OK : check_a5(a5); }
};

// Host layouts and the size-determining fields of S for (operator, F).
int prepare(const OpDesc &D, const pcga_ainv_t *F, int precision, int slice_width,
            HostLayouts &H, pcga_solver &S) {
    if (!F) return fail(PCGA_EINVAL, "NULL argument");
    if (slice_width == 0) slice_width = default_width(precision);
    if (slice_width < 1 || slice_width > kMaxSliceWidth)
        return fail(PCGA_EINVAL, "slice_width must be 0 or 1.." + std::to_string(kMaxSliceWidth));
    int st = D.check();
    if (st) return st;
    if (precision != PCGA_FP64 && precision != PCGA_MIXED && precision != PCGA_MIXED_A32)
        return fail(PCGA_EINVAL, "precision must be PCGA_FP64, PCGA_MIXED or PCGA_MIXED_A32");
    if (D.is_csr() && precision != PCGA_FP64)
        return fail(PCGA_EINVAL, "a CSR operator is solved in PCGA_FP64");
    if (F->F.n != D.n()) return fail(PCGA_EINVAL, "F does not match A");
    st = build_layouts(F->F, slice_width, H);
    if (st) return st;
    if (D.is_csr()) {
        try {
            sell_build(D.csr.nrows, D.csr.rowptr, D.csr.col, D.csr.val, slice_width, H.a);
        } catch (const std::bad_alloc &) {
            return fail(PCGA_ENOMEM, "host allocation failed while building the layout of A");
        }
        if (!sell_check(H.a)) return fail(PCGA_EINVAL, "internal: layout of A violates its invariants");
    }
    S.precision = precision;
    S.n = F->F.n;
    S.csr = D.is_csr();
    S.band_q = band_width(F->F);
    // FP64: Z's values are read from Z^T's resident copy where they agree
    // (the FP32 inner solve keeps both in the cache anyway)
    if (precision == PCGA_FP64 && S.band_q == 0 && F->F.nnz_off() > 0) {
        try {
            H.zmapped = sell_shared_values(H.zt, H.z, H.zt.entries(), H.za, H.zb, H.zk);
        } catch (const std::bad_alloc &) {
            H.zmapped = 0;
        }
    }
    return PCGA_OK;
}

int workspace_bytes_impl(const OpDesc &D, const pcga_ainv_t *F, int precision, int32_t slice_width,
                         size_t *bytes) {
    if (!bytes) return fail(PCGA_EINVAL, "NULL argument");
    HostLayouts H;
    pcga_solver S;
    int st = prepare(D, F, precision, slice_width, H, S);
    if (st) return st;
    *bytes = carve(S, nullptr, H);
    return PCGA_OK;
}

int create_impl(const OpDesc &D, const pcga_ainv_t *F, int precision, int32_t slice_width,
                void *ws, size_t bytes, void *stream, pcga_solver_t **out) {
    if (!out) return fail(PCGA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!F || !ws) return fail(PCGA_EINVAL, "NULL F or workspace");
    if (((uintptr_t)ws & 255u) != 0) return fail(PCGA_EINVAL, "workspace must be 256-byte aligned");
    HostLayouts H;
    pcga_solver *S = new (std::nothrow) pcga_solver;
    if (!S) return fail(PCGA_ENOMEM, "host allocation failed");
    int st = prepare(D, F, precision, slice_width, H, *S);
    if (st) {
        delete S;
        return st;
    }
    const int64_t n = S->n;
    S->max_blocks = precision != PCGA_FP64 ? kDefaultBlocksMixed : kDefaultBlocks;
    S->nnz_off = F->F.nnz_off();
    // the two-launch diagonal path fuses the five-point product; a CSR
    // operator runs the general three-launch iteration also for Z = I
    S->jacobi = S->nnz_off == 0 && !S->csr;
    if (S->csr) {
        S->nnz_a = D.csr.rowptr[D.csr.nrows];
    } else {
        S->nx = D.a5->nx;
        S->ny = D.a5->ny;
        S->periodic = (D.a5->flags & PCGA_PERIODIC_X) ? 1 : 0;
    }
    S->stream = (hipStream_t)stream;
    const size_t need = carve(*S, nullptr, H);
    if (bytes < need) {
        delete S;
        return fail(PCGA_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
    }
    S->ws = ws;
    S->ws_bytes = bytes;
    carve(*S, ws, H);
    if (!S->csr) {
        S->A64.nx = D.a5->nx;
        S->A64.ny = D.a5->ny;
        S->A64.periodic = S->periodic;
        S->A64.n = (int32_t)n;
        S->A64.inv_nx = 1.0 / (double)D.a5->nx;
        S->A32.nx = S->A64.nx;
        S->A32.ny = S->A64.ny;
        S->A32.periodic = S->A64.periodic;
        S->A32.n = S->A64.n;
        S->A32.inv_nx = S->A64.inv_nx;
    }
    S->sell_entries = H.zt.entries() + H.z.entries();

    auto fail_free = [&](int code) {
        if (S->snap[0]) (void)hipHostFree(S->snap[0]);
        if (S->snap[1]) (void)hipHostFree(S->snap[1]);
        if (S->ev[0]) (void)hipEventDestroy(S->ev[0]);
        if (S->ev[1]) (void)hipEventDestroy(S->ev[1]);
        delete S;
        return code;
    };
#define CR(expr)                                                                               \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail_free(fail(PCGA_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_))); \
    } while (0)

    CR(hipGetDevice(&S->device));
    // coherent: the chunk graphs' last kernel writes them directly
    CR(hipHostMalloc((void **)&S->snap[0], sizeof(CtlBlock), hipHostMallocCoherent));
    CR(hipHostMalloc((void **)&S->snap[1], sizeof(CtlBlock), hipHostMallocCoherent));
    CR(hipHostGetDevicePointer((void **)&S->snap_dev[0], S->snap[0], 0));
    CR(hipHostGetDevicePointer((void **)&S->snap_dev[1], S->snap[1], 0));
    CR(hipEventCreateWithFlags(&S->ev[0], hipEventDisableTiming));
    CR(hipEventCreateWithFlags(&S->ev[1], hipEventDisableTiming));

    hipStream_t sm = S->stream;
    const size_t nb8 = n * sizeof(double);
    // operator (FP64 always; FP32 copy for the mixed inner solve)
    if (!S->csr) {
        CR(hipMemcpyAsync((void *)S->A64.diag, D.a5->diag, nb8, hipMemcpyHostToDevice, sm));
        CR(hipMemcpyAsync((void *)S->A64.ae, D.a5->ae, nb8, hipMemcpyHostToDevice, sm));
        CR(hipMemcpyAsync((void *)S->A64.an, D.a5->an, nb8, hipMemcpyHostToDevice, sm));
    }
    if (precision == PCGA_MIXED_A32) {
        const double *src[3] = {D.a5->diag, D.a5->ae, D.a5->an};
        const float *dst[3] = {S->A32.diag, S->A32.ae, S->A32.an};
        for (int a = 0; a < 3; a++) {
            std::vector<float> f(src[a], src[a] + n);
            CR(hipMemcpyAsync((void *)dst[a], f.data(), n * 4, hipMemcpyHostToDevice, sm));
            CR(hipStreamSynchronize(sm));   // f is a temporary
        }
    }
    std::vector<double> dinv(n);
    for (int64_t k = 0; k < n; k++) dinv[k] = 1.0 / F->F.D[k];
    auto up_sell = [&](const SellLayout &L, auto &dst) -> hipError_t {
        using T = std::remove_const_t<std::remove_pointer_t<decltype(dst.val)>>;
        hipError_t e;
        e = hipMemcpyAsync((void *)dst.row0, L.row0.data(), L.row0.size() * 4, hipMemcpyHostToDevice, sm);
        if (e) return e;
        e = hipMemcpyAsync((void *)dst.meta, L.meta.data(), L.meta.size() * 4, hipMemcpyHostToDevice, sm);
        if (e) return e;
        e = hipMemcpyAsync((void *)dst.off, L.off.data(), L.off.size() * 8, hipMemcpyHostToDevice, sm);
        if (e) return e;
        if (!L.toff.empty()) {
            e = hipMemcpyAsync((void *)dst.toff, L.toff.data(), L.toff.size() * 4,
                               hipMemcpyHostToDevice, sm);
            if (e) return e;
        }
        if (!L.tab.empty()) {
            e = hipMemcpyAsync((void *)dst.tab, L.tab.data(), L.tab.size() * 4,
                               hipMemcpyHostToDevice, sm);
            if (e) return e;
        }
        if (L.entries() == 0) return hipSuccess;
        if (L.narrow)
            e = hipMemcpyAsync((void *)dst.dist, L.dist.data(), L.dist.size() * 2, hipMemcpyHostToDevice, sm);
        else
            e = hipMemcpyAsync((void *)dst.idx, L.idx.data(), L.idx.size() * 4, hipMemcpyHostToDevice, sm);
        if (e) return e;
        if constexpr (std::is_same_v<T, double>) {
            return hipMemcpyAsync((void *)dst.val, L.val.data(), L.val.size() * 8,
                                  hipMemcpyHostToDevice, sm);
        } else {
            std::vector<float> v32(L.val.begin(), L.val.end());
            e = hipMemcpyAsync((void *)dst.val, v32.data(), v32.size() * 4, hipMemcpyHostToDevice, sm);
            if (e) return e;
            return hipStreamSynchronize(sm);   // v32 is a temporary
        }
    };
    if (S->band_q > 0) {
        const std::vector<double> zb = band_diagonals(F->F, S->band_q);
        if (precision == PCGA_FP64) {
            CR(hipMemcpyAsync(S->zb64, zb.data(), zb.size() * 8, hipMemcpyHostToDevice, sm));
        } else {
            const std::vector<float> zf(zb.begin(), zb.end());
            CR(hipMemcpyAsync(S->zb32, zf.data(), zf.size() * 4, hipMemcpyHostToDevice, sm));
        }
        CR(hipStreamSynchronize(sm));   // zb / zf are temporaries
    }
    if (S->csr) CR(up_sell(H.a, S->a64));
    if (precision == PCGA_FP64) {
        CR(hipMemcpyAsync(S->dinv64, dinv.data(), nb8, hipMemcpyHostToDevice, sm));
        CR(up_sell(H.zt, S->zt64));
        CR(up_sell(H.z, S->z64));
        if (H.zmapped > 0) {
            const std::vector<double> zeros(64, 0.0);
            CR(hipMemcpyAsync((void *)(S->zt64.val + H.zt.entries()), zeros.data(), 64 * 8,
                              hipMemcpyHostToDevice, sm));
            CR(hipStreamSynchronize(sm));   // zeros is a temporary
            const size_t nt = H.z.tab.size() * 4;
            CR(hipMemcpyAsync((void *)S->z64.alt_a, H.za.data(), nt, hipMemcpyHostToDevice, sm));
            CR(hipMemcpyAsync((void *)S->z64.alt_b, H.zb.data(), nt, hipMemcpyHostToDevice, sm));
            CR(hipMemcpyAsync((void *)S->z64.alt_k, H.zk.data(), nt, hipMemcpyHostToDevice, sm));
        }
    } else {
        std::vector<float> f(n);
        for (int64_t k = 0; k < n; k++) f[k] = (float)dinv[k];
        CR(hipMemcpyAsync(S->dinv32, f.data(), n * 4, hipMemcpyHostToDevice, sm));
        CR(hipStreamSynchronize(sm));
        CR(up_sell(H.zt, S->zt32));
        CR(up_sell(H.z, S->z32));
    }
    CR(hipMemsetAsync(S->cb, 0, sizeof(CtlBlock), sm));
    CR(hipStreamSynchronize(sm));
#undef CR
    S->cost_zt = slice_costs(H.zt);
    S->cost_z = slice_costs(H.z);
    if (S->csr) {
        S->cost_a = slice_costs(H.a);
        S->a64.bounds = S->bnd_a;
    }
    S->zt64.bounds = S->zt32.bounds = S->bnd_zt;
    S->z64.bounds = S->z32.bounds = S->bnd_z;
    S->zt64.bounds_b = S->zt32.bounds_b = S->bnd_zt_b;
    S->z64.bounds_b = S->z32.bounds_b = S->bnd_z_b;
    S->grids();
    st = upload_bounds(*S);
    if (st) {
        pcga_solver_destroy(S);
        return st;
    }
    // modelled compulsory bytes per iteration (see kernels.h):
    //   stencil: s, d_old read; d_new, q written       4 n words + FP64 diag, ae, an
    //   zt: r, q, d, x, dinv read; r', x, t written; Z^T entries     8 n words + E_zt
    //   z:  t, r' read; s written; Z entries                         3 n words + E_z
    //   (an entry: its value and a 4-byte column or 2-byte distance)
    //   with x += alpha d in the stencil: the stencil also reads and writes
    //   x, the zt kernel no longer reads d and x nor writes x: 1 n word less
    const double E = (double)S->sell_entries;
    S->index_bytes = H.zt.narrow ? 2 : 4;
    cache_plan(*S, H);
    //   (the stencil reads the FP64 coefficients diag, ae, an also for the
    //   FP32 inner iteration: 24 n bytes)
    //   (a CSR operator: s, d_old read, d_new, q written and A's entries, a
    //   value and a 4-byte column each, instead of the five-point kernel's
    //   7 n words)
    if (S->csr)
        S->bytes_per_iter = 8.0 * 15.0 * n + 12.0 * (double)S->nnz_a + (8.0 + S->index_bytes) * E;
    else {
        const double words = S->x_deferred() ? 14.0 : 15.0;
        if (precision == PCGA_FP64)
            S->bytes_per_iter = 8.0 * words * n + 24.0 * n + (8.0 + S->index_bytes) * E;
        else if (precision == PCGA_MIXED_A32)
            S->bytes_per_iter = 4.0 * words * n + 12.0 * n + (4.0 + S->index_bytes) * E;
        else
            S->bytes_per_iter = 4.0 * words * n + 24.0 * n + (4.0 + S->index_bytes) * E;
    }
    *out = S;
    return PCGA_OK;
}


}  // namespace

extern "C" {

const char *pcga_strerror(int s) {
    switch (s) {
        case PCGA_OK: return "ok";
        case PCGA_NOCONV: return "not converged (iteration limit reached)";
        case PCGA_EINVAL: return "invalid argument";
        case PCGA_EBREAKDOWN: return "breakdown (non-positive pivot or curvature)";
        case PCGA_ENAN: return "NaN or Inf in the iteration";
        case PCGA_EHIP: return "HIP runtime error";
        case PCGA_ENOMEM: return "out of memory / workspace too small";
        default: return "unknown status";
    }
}

const char *pcga_last_error(void) { return last_error().c_str(); }

int pcga_stream_create(void **stream) {
    if (!stream) return fail(PCGA_EINVAL, "stream is NULL");
    *stream = nullptr;
    hipStream_t h = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&h, hipStreamNonBlocking));
    *stream = (void *)h;
    return PCGA_OK;
}

int pcga_stream_destroy(void *stream) {
    if (!stream) return PCGA_OK;
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    HIP_TRY(hipStreamDestroy((hipStream_t)stream));
    return PCGA_OK;
}

static int ainv_setup_impl(const pcga_a5_t *A, double drop_tol, int64_t fill,
                           pcga_ainv_t **out) {
    if (!out) return fail(PCGA_EINVAL, "out is NULL");
    *out = nullptr;
    int st = check_a5(A);
    if (st) return st;
    if (!(drop_tol >= 0.0)) return fail(PCGA_EINVAL, "drop_tol must be >= 0 (inf allowed)");
    pcga_ainv *h = new (std::nothrow) pcga_ainv;
    if (!h) return fail(PCGA_ENOMEM, "host allocation failed");
    int64_t bad = -1;
    st = ainv_build(view_of(A), drop_tol, fill, h->F, &bad);
    if (st) {
        delete h;
        if (st == PCGA_EBREAKDOWN)
            return fail(st, "AINV breakdown: pivot p_i <= 0 at row " + std::to_string(bad));
        return fail(st, "AINV setup failed");
    }
    *out = h;
    return PCGA_OK;
}

int pcga_ainv_setup(const pcga_a5_t *A, double drop_tol, pcga_ainv_t **out) {
    return ainv_setup_impl(A, drop_tol, -1, out);
}

int pcga_ainv_setup_fill(const pcga_a5_t *A, double drop_tol, int32_t max_fill,
                         pcga_ainv_t **out) {
    if (out) *out = nullptr;
    if (max_fill < 0) return fail(PCGA_EINVAL, "max_fill must be >= 0");
    return ainv_setup_impl(A, drop_tol, max_fill, out);
}

int pcga_fsai_band_setup(const pcga_a5_t *A, int32_t q, pcga_ainv_t **out) {
    if (!out) return fail(PCGA_EINVAL, "out is NULL");
    *out = nullptr;
    int st = check_a5(A);
    if (st) return st;
    if (q < 0 || q > 4096) return fail(PCGA_EINVAL, "band q must be 0..4096");
    pcga_ainv *h = new (std::nothrow) pcga_ainv;
    if (!h) return fail(PCGA_ENOMEM, "host allocation failed");
    int64_t bad = -1;
    st = fsai_band_build(view_of(A), q, h->F, &bad);
    if (st) {
        delete h;
        if (st == PCGA_EBREAKDOWN)
            return fail(st, "banded factor breakdown: pivot <= 0 at row " + std::to_string(bad));
        return fail(st, "banded factor setup failed");
    }
    *out = h;
    return PCGA_OK;
}

int pcga_ainv_info(const pcga_ainv_t *F, int64_t *n, int64_t *nnz_off) {
    if (!F) return fail(PCGA_EINVAL, "F is NULL");
    if (n) *n = F->F.n;
    if (nnz_off) *nnz_off = F->F.nnz_off();
    return PCGA_OK;
}

int pcga_ainv_export(const pcga_ainv_t *F, int64_t *colptr, int32_t *rowidx, double *val,
                     double *D) {
    if (!F) return fail(PCGA_EINVAL, "F is NULL");
    const AinvFactor &Z = F->F;
    if (colptr) std::memcpy(colptr, Z.colptr.data(), (Z.n + 1) * sizeof(int64_t));
    if (rowidx && Z.nnz_off()) std::memcpy(rowidx, Z.rowidx.data(), Z.nnz_off() * sizeof(int32_t));
    if (val && Z.nnz_off()) std::memcpy(val, Z.val.data(), Z.nnz_off() * sizeof(double));
    if (D) std::memcpy(D, Z.D.data(), Z.n * sizeof(double));
    return PCGA_OK;
}

int pcga_ainv_import(int64_t n, const int64_t *colptr, const int32_t *rowidx,
                     const double *val, const double *D, pcga_ainv_t **out) {
    if (!out) return fail(PCGA_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > INT32_MAX || !colptr || !D) return fail(PCGA_EINVAL, "bad n or NULL array");
    if (colptr[0] != 0) return fail(PCGA_EINVAL, "colptr[0] must be 0");
    for (int64_t j = 0; j < n; j++) {
        if (colptr[j + 1] < colptr[j]) return fail(PCGA_EINVAL, "colptr not monotone");
        if (!(D[j] > 0.0) || !std::isfinite(D[j])) return fail(PCGA_EINVAL, "D must be > 0");
        for (int64_t a = colptr[j]; a < colptr[j + 1]; a++) {
            if (!rowidx || !val) return fail(PCGA_EINVAL, "NULL rowidx/val with entries");
            if (rowidx[a] < 0 || rowidx[a] >= j) return fail(PCGA_EINVAL, "Z must be strictly upper");
            if (a > colptr[j] && rowidx[a] <= rowidx[a - 1])
                return fail(PCGA_EINVAL, "rows must ascend within a column");
            if (!std::isfinite(val[a])) return fail(PCGA_EINVAL, "non-finite value in Z");
        }
    }
    pcga_ainv *h = new (std::nothrow) pcga_ainv;
    if (!h) return fail(PCGA_ENOMEM, "host allocation failed");
    try {
        h->F.n = n;
        h->F.colptr.assign(colptr, colptr + n + 1);
        h->F.rowidx.assign(rowidx, rowidx + colptr[n]);
        h->F.val.assign(val, val + colptr[n]);
        h->F.D.assign(D, D + n);
    } catch (const std::bad_alloc &) {
        delete h;
        return fail(PCGA_ENOMEM, "host allocation failed");
    }
    *out = h;
    return PCGA_OK;
}

int pcga_ainv_free(pcga_ainv_t *F) {
    delete F;
    return PCGA_OK;
}

int pcga_layout_info(const pcga_ainv_t *F, int32_t slice_width, int64_t *out) {
    if (!F || !out) return fail(PCGA_EINVAL, "NULL argument");
    if (slice_width == 0) slice_width = kTargetWidth;
    if (slice_width < 1 || slice_width > kMaxSliceWidth)
        return fail(PCGA_EINVAL, "slice_width must be 0 or 1.." + std::to_string(kMaxSliceWidth));
    HostLayouts H;
    const int st = build_layouts(F->F, slice_width, H);
    if (st) return st;
    const SellLayout *Ls[2] = {&H.zt, &H.z};
    for (int m = 0; m < 2; m++) {
        const SellLayout &L = *Ls[m];
        int64_t ntab = 0, wtab = 0, wmax = 0;
        for (int64_t s = 0; s < L.nslices(); s++) {
            const int64_t w = L.meta[s] >> 8;
            wmax = std::max(wmax, w);
            if (L.toff[s] >= 0) {
                ntab++;
                wtab = std::max(wtab, w);
            }
        }
        out[6 * m + 0] = L.nslices();
        out[6 * m + 1] = ntab;
        out[6 * m + 2] = wtab;
        out[6 * m + 3] = wmax;
        out[6 * m + 4] = L.entries();
        out[6 * m + 5] = L.narrow ? 2 : 4;
    }
    return PCGA_OK;
}

int pcga_workspace_bytes(const pcga_a5_t *A, const pcga_ainv_t *F, int precision,
                         size_t *bytes) {
    return pcga_workspace_bytes_ex(A, F, precision, 0, bytes);
}

int pcga_solver_create(const pcga_a5_t *A, const pcga_ainv_t *F, int precision, void *ws,
                       size_t bytes, void *stream, pcga_solver_t **out) {
    return pcga_solver_create_ex(A, F, precision, 0, ws, bytes, stream, out);
}

int pcga_workspace_bytes_ex(const pcga_a5_t *A, const pcga_ainv_t *F, int precision,
                            int32_t slice_width, size_t *bytes) {
    OpDesc D;
    D.a5 = A;
    return workspace_bytes_impl(D, F, precision, slice_width, bytes);
}

int pcga_workspace_bytes_csr(const pcga_csr_t *A, const pcga_ainv_t *F, int precision,
                             int32_t slice_width, size_t *bytes) {
    OpDesc D;
    int st = D.set_csr(A);
    if (st) return st;
    return workspace_bytes_impl(D, F, precision, slice_width, bytes);
}

int pcga_solver_create_ex(const pcga_a5_t *A, const pcga_ainv_t *F, int precision,
                          int32_t slice_width, void *ws, size_t bytes, void *stream,
                          pcga_solver_t **out) {
    OpDesc D;
    D.a5 = A;
    return create_impl(D, F, precision, slice_width, ws, bytes, stream, out);
}

int pcga_ainv_setup_csr(const pcga_csr_t *A, double drop_tol, int32_t max_fill,
                        pcga_ainv_t **out) {
    if (!out) return fail(PCGA_EINVAL, "out is NULL");
    *out = nullptr;
    OpDesc D;
    int st = D.set_csr(A);
    if (st) return st;
    if (!(drop_tol >= 0.0)) return fail(PCGA_EINVAL, "drop_tol must be >= 0 (inf allowed)");
    pcga_ainv *h = new (std::nothrow) pcga_ainv;
    if (!h) return fail(PCGA_ENOMEM, "host allocation failed");
    int64_t bad = -1;
    st = ainv_build(D.csr, drop_tol, max_fill < 0 ? -1 : (int64_t)max_fill, h->F, &bad);
    if (st) {
        delete h;
        if (st == PCGA_EBREAKDOWN)
            return fail(st, "AINV breakdown: pivot p_i <= 0 at row " + std::to_string(bad));
        return fail(st, "AINV setup failed");
    }
    *out = h;
    return PCGA_OK;
}

int pcga_solver_create_csr(const pcga_csr_t *A, const pcga_ainv_t *F, int precision,
                           int32_t slice_width, void *ws, size_t bytes, void *stream,
                           pcga_solver_t **out) {
    if (out) *out = nullptr;
    OpDesc D;
    int st = D.set_csr(A);
    if (st) return st;
    return create_impl(D, F, precision, slice_width, ws, bytes, stream, out);
}

int pcga_solver_destroy(pcga_solver_t *S) {
    if (!S) return PCGA_OK;
    S->drop_graphs();
    if (S->snap[0]) (void)hipHostFree(S->snap[0]);
    if (S->snap[1]) (void)hipHostFree(S->snap[1]);
    if (S->ev[0]) (void)hipEventDestroy(S->ev[0]);
    if (S->ev[1]) (void)hipEventDestroy(S->ev[1]);
    delete S;
    return PCGA_OK;
}

int pcga_solver_info(const pcga_solver_t *S, int64_t *n, int64_t *nnz_off, int32_t *precision,
                     double *bytes_per_iter, int32_t *index_bytes, int32_t *formats) {
    if (!S) return fail(PCGA_EINVAL, "S is NULL");
    if (index_bytes) *index_bytes = S->index_bytes;
    if (formats) {
        formats[0] = S->fmt_zt | (S->x_deferred() ? kFmtXDef : 0);
        formats[1] = S->fmt_z;
        formats[2] = S->band_q;
    }
    if (n) *n = S->n;
    if (nnz_off) *nnz_off = S->nnz_off;
    if (precision) *precision = S->precision;
    if (bytes_per_iter) *bytes_per_iter = S->bytes_per_iter;
    return PCGA_OK;
}

int pcga_solver_tune(pcga_solver_t *S, int32_t chunk, int32_t use_graph, int32_t max_blocks) {
    if (!S) return fail(PCGA_EINVAL, "S is NULL");
    if (chunk < 2 || chunk > 512 || (chunk & 1))
        return fail(PCGA_EINVAL, "chunk must be even, 2..512");
    if (max_blocks == 0) max_blocks = S->precision != PCGA_FP64 ? kDefaultBlocksMixed : kDefaultBlocks;
    if (max_blocks < 8 || max_blocks > kMaxBlocks)
        return fail(PCGA_EINVAL, "max_blocks must be 0 or 8.." + std::to_string(kMaxBlocks));
    if (S->graph[0] && (chunk != S->graph_chunk || max_blocks != S->max_blocks)) S->drop_graphs();
    S->chunk = chunk;
    S->use_graph = use_graph != 0;
    S->max_blocks = max_blocks;
    S->grids();
    return upload_bounds(*S);
}

int pcga_solver_set_grids(pcga_solver_t *S, int32_t g_stencil, int32_t g_zt, int32_t g_z) {
    if (!S) return fail(PCGA_EINVAL, "S is NULL");
    const int32_t g[3] = {g_stencil, g_zt, g_z};
    for (int i = 0; i < 3; i++)
        if (g[i] < 0 || g[i] > kMaxBlocks)
            return fail(PCGA_EINVAL, "workgroup counts must be 0..." + std::to_string(kMaxBlocks));
    S->drop_graphs();
    for (int i = 0; i < 3; i++) S->g_cap[i] = g[i];
    S->grids();
    return upload_bounds(*S);
}

}  // extern "C"

// ===========================================================================
// iteration driver
// ===========================================================================
namespace {

template <typename T>
struct IterBufs {
    DevOp<double> A;   // FP64 coefficients for both the FP64 and the FP32 inner iteration
    DevSell<T> zt, z;
    const T *zb;       // banded Z by diagonals (band_q > 0)
    const T *dinv;
    T *x, *r[2], *s, *d[2], *q, *t;
    CtlBlock *cb;   // control block and partial sums of the solve
    Partials P;
};

IterBufs<double> bufs64(pcga_solver &S) {
    return {S.A64, S.zt64, S.z64, S.zb64, S.dinv64, S.x, {S.r[0], S.r[1]}, S.s, {S.d[0], S.d[1]},
            S.q, S.t, S.cb, S.P};
}
IterBufs<float> bufs32(pcga_solver &S) {
    return {S.A64, S.zt32, S.z32, S.zb32, S.dinv32, S.e32, {S.r32[0], S.r32[1]}, S.s32,
            {S.d32[0], S.d32[1]}, S.q32, S.t32, S.cb, S.P};
}

// Launch k_zt / k_z in a matrix's storage and read format (kFmt* bits).
#define PCGA_FMT_CASES(KERNEL, ...)                                      \
    switch (fmt) {                                                       \
        case 0: KERNEL(0)<<<grid, kBS, 0, st>>>(__VA_ARGS__); break;     \
        case 1: KERNEL(1)<<<grid, kBS, 0, st>>>(__VA_ARGS__); break;     \
        case 2: KERNEL(2)<<<grid, kBS, 0, st>>>(__VA_ARGS__); break;     \
        case 3: KERNEL(3)<<<grid, kBS, 0, st>>>(__VA_ARGS__); break;     \
        case 6: KERNEL(6)<<<grid, kBS, 0, st>>>(__VA_ARGS__); break;     \
        default: KERNEL(7)<<<grid, kBS, 0, st>>>(__VA_ARGS__); break;    \
    }

// xdef: the x update is left to the next stencil (k_zt then ignores kFmtNtX)
template <typename T, bool FUSED, typename... Args>
void launch_zt(const DevSell<T> &M, int fmt, bool xdef, int grid, hipStream_t st, Args... args) {
#define PCGA_K(F) k_zt<T, FUSED, F>
    if (FUSED && xdef) {
        fmt &= ~kFmtNtX;
#define PCGA_KD(F) k_zt<T, FUSED, F | kFmtXDef>
        PCGA_FMT_CASES(PCGA_KD, M, args...)
#undef PCGA_KD
    } else if (FUSED && (fmt & kFmtNtX)) {
        fmt &= ~kFmtNtX;
#define PCGA_KX(F) k_zt<T, FUSED, F | kFmtNtX>
        PCGA_FMT_CASES(PCGA_KX, M, args...)
#undef PCGA_KX
    } else {
        fmt &= ~kFmtNtX;
        PCGA_FMT_CASES(PCGA_K, M, args...)
    }
#undef PCGA_K
}

template <typename T, bool DOT, bool FIRST, typename... Args>
void launch_z(const DevSell<T> &M, int fmt, int grid, hipStream_t st, Args... args) {
    if constexpr (std::is_same_v<T, double>) {
        if (fmt & kFmtZtVal) {
            fmt &= ~kFmtZtVal;
#define PCGA_KV(F) k_z<T, DOT, FIRST, F | kFmtZtVal>
            PCGA_FMT_CASES(PCGA_KV, M, args...)
#undef PCGA_KV
            return;
        }
    }
    fmt &= ~kFmtZtVal;
#define PCGA_K(F) k_z<T, DOT, FIRST, F>
    PCGA_FMT_CASES(PCGA_K, M, args...)
#undef PCGA_K
}
#undef PCGA_FMT_CASES

// The FP32 inner iteration of a PCGA_MIXED_A32 solver applies the FP32 operator.
template <typename T>
bool a32_inner(const pcga_solver &S) {
    return std::is_same_v<T, float> && S.precision == PCGA_MIXED_A32;
}

// Where x += alpha d is left to the next iteration's stencil (which has
// d_old at hand): k_zt then reads neither d nor x (one vector pass less).
bool x_deferred(const pcga_solver &S) { return S.x_deferred(); }

// Stencil of the deferred path: XD 1 (x resident) or 2 (x streamed).
template <typename T, typename C>
void launch_stencil_xd(pcga_solver &S, const DevOp<C> &A, const IterBufs<T> &B, int p, int g_sr) {
    if (S.fmt_zt & kFmtNtX)
        k_stencil<T, false, C, 2><<<S.g_tile, kBS, 0, S.stream>>>(A, B.s, B.d[p], B.d[p ^ 1], B.q,
                                                                  B.x, B.cb, B.P, g_sr, p);
    else
        k_stencil<T, false, C, 1><<<S.g_tile, kBS, 0, S.stream>>>(A, B.s, B.d[p], B.d[p ^ 1], B.q,
                                                                  B.x, B.cb, B.P, g_sr, p);
}

// One kernel of iteration parity p: 0 stencil, 1 axpy + Z^T, 2 Z + dot.
template <typename T>
void launch_kernel(pcga_solver &S, const IterBufs<T> &B, int p, int which) {
    switch (which) {
        case 0:
            if (S.csr)
                k_spmv_sell<0><<<S.g_a, kBS, 0, S.stream>>>(S.a64, (const double *)B.s,
                                                            (const double *)B.d[p], (double *)B.d[p ^ 1],
                                                            (double *)B.q, B.cb, B.P, S.g_prec(), p);
            else if (a32_inner<T>(S)) {
                if constexpr (std::is_same_v<T, float>) {
                    if (S.jacobi)
                        k_stencil<T, true, float><<<S.g_tile, kBS, 0, S.stream>>>(
                            S.A32, B.s, B.d[p], B.d[p ^ 1], B.q, nullptr, B.cb, B.P, S.g_st, p);
                    else if (x_deferred(S))
                        launch_stencil_xd<T, float>(S, S.A32, B, p, S.g_prec());
                    else
                        k_stencil<T, false, float><<<S.g_tile, kBS, 0, S.stream>>>(
                            S.A32, B.s, B.d[p], B.d[p ^ 1], B.q, nullptr, B.cb, B.P, S.g_prec(), p);
                }
            } else if (S.jacobi)
                k_stencil<T, true><<<S.g_tile, kBS, 0, S.stream>>>(
                    B.A, B.s, B.d[p], B.d[p ^ 1], B.q, nullptr, B.cb, B.P, S.g_st, p);
            else if (x_deferred(S))
                launch_stencil_xd<T, double>(S, B.A, B, p, S.g_prec());
            else
                k_stencil<T, false><<<S.g_tile, kBS, 0, S.stream>>>(
                    B.A, B.s, B.d[p], B.d[p ^ 1], B.q, nullptr, B.cb, B.P, S.g_prec(), p);
            break;
        case 1:
            if (S.jacobi) {
                k_jacobi<T, false><<<S.g_st, kBS, 0, S.stream>>>(
                    B.dinv, B.r[p], B.q, B.d[p ^ 1], B.r[p ^ 1], B.x, B.s, (int)S.n, B.cb, B.P,
                    S.g_dq(), p);
                break;
            }
            if (S.band_q > 0) {
                k_zt_band<T, true><<<S.g_st, kBS, 0, S.stream>>>(
                    B.zb, S.band_q, B.dinv, B.r[p], B.q, B.d[p ^ 1], B.r[p ^ 1], B.x, B.t, (int)S.n,
                    B.cb, B.P, S.g_dq(), p);
                break;
            }
            launch_zt<T, true>(B.zt, S.fmt_zt, x_deferred(S), S.g_zt, S.stream, B.dinv, (const T *)B.r[p],
                               (const T *)B.q, (const T *)B.d[p ^ 1], B.r[p ^ 1], B.x, B.t, B.cb, B.P,
                               S.g_dq(), p);
            break;
        default:
            if (S.band_q > 0) {
                k_z_band<T, true, false><<<S.g_st, kBS, 0, S.stream>>>(
                    B.zb, S.band_q, B.t, B.r[p ^ 1], B.s, (int)S.n, B.cb, B.P, S.g_st, p);
                break;
            }
            launch_z<T, true, false>(B.z, S.fmt_z, S.g_z, S.stream, (const T *)B.t, (const T *)B.r[p ^ 1],
                                     B.s, B.cb, B.P, S.g_zt, p);
            break;
    }
}

template <typename T>
void launch_iters(pcga_solver &S, const IterBufs<T> &B, int count) {
    for (int it = 0; it < count; it++)
        for (int w = 0; w < S.kernels_per_iter(); w++) launch_kernel<T>(S, B, it & 1, w);
}

// r0 = b - A x0 (FP64) and the solve's control state.
void launch_residual_prologue(pcga_solver &S, CtlBlock *cb, const Partials &P, const double *x,
                              const double *b, double *r, double tol, int maxit) {
    if (S.csr)
        k_residual_sell<true, false><<<S.g_a, kBS, 0, S.stream>>>(S.a64, x, b, r, P);
    else
        k_residual<true><<<S.g_st, kBS, 0, S.stream>>>(S.A64, x, b, r, P);
    k_fin_residual<0><<<1, kBS, 0, S.stream>>>(cb, P, S.g_op(), tol, maxit);
}

void launch_true_residual(pcga_solver &S, CtlBlock *cb, const Partials &P, const double *x,
                          const double *b) {
    if (S.csr)
        k_residual_sell<false, false><<<S.g_a, kBS, 0, S.stream>>>(S.a64, x, b, nullptr, P);
    else
        k_residual<false><<<S.g_st, kBS, 0, S.stream>>>(S.A64, x, b, nullptr, P);
    k_fin_residual<1><<<1, kBS, 0, S.stream>>>(cb, P, S.g_op(), 0.0, 0);
}

void launch_refine(pcga_solver &S, bool add_e, const double *x, double *xnew, const double *b,
                   double inner_tol, int inner_maxit, bool keep = false, bool cont = false,
                   double outer_tol = 0.0) {
    if (add_e)
        k_refine<true><<<S.g_st, kBS, 0, S.stream>>>(S.A64, x, S.e32, xnew, b, S.r32[0], S.P);
    else
        k_refine<false><<<S.g_st, kBS, 0, S.stream>>>(S.A64, x, nullptr, nullptr, b, S.r32[0], S.P);
    k_fin_refine<<<1, kBS, 0, S.stream>>>(S.cb, S.P, S.g_st, inner_tol, inner_maxit, keep ? 1 : 0,
                                          cont ? 1 : 0, outer_tol);
}

// t = D^-1 Z^T r0 ; s0 = Z t ; (s0, r0) partials ; d[0] = 0 (zero_d: a run
// that continues the last one keeps its direction in d[0])
template <typename T>
int prologue_prec(pcga_solver &S, const IterBufs<T> &B, bool zero_d = true) {
    if (zero_d) k_zero<T><<<zero_grid(S.n), kBS, 0, S.stream>>>((int)S.n, B.d[0]);
    if (S.jacobi) {
        k_jacobi<T, true><<<S.g_st, kBS, 0, S.stream>>>(B.dinv, B.r[0], nullptr, nullptr, nullptr,
                                                        nullptr, B.s, (int)S.n, B.cb, B.P, 0, 0);
        HIP_TRY(hipGetLastError());
        return PCGA_OK;
    }
    if (S.band_q > 0) {
        k_zt_band<T, false><<<S.g_st, kBS, 0, S.stream>>>(B.zb, S.band_q, B.dinv, B.r[0], nullptr,
                                                          nullptr, nullptr, nullptr, B.t, (int)S.n,
                                                          B.cb, B.P, 0, 0);
        k_z_band<T, true, true><<<S.g_st, kBS, 0, S.stream>>>(B.zb, S.band_q, B.t, B.r[0], B.s,
                                                              (int)S.n, B.cb, B.P, 0, 0);
        HIP_TRY(hipGetLastError());
        return PCGA_OK;
    }
    launch_zt<T, false>(B.zt, S.fmt_zt, false, S.g_zt, S.stream, B.dinv, (const T *)B.r[0], (const T *)nullptr,
                        (const T *)nullptr, (T *)nullptr, (T *)nullptr, B.t, B.cb, B.P, 0, 0);
    launch_z<T, true, true>(B.z, S.fmt_z, S.g_z, S.stream, (const T *)B.t, (const T *)B.r[0], B.s, B.cb,
                            B.P, 0, 0);
    HIP_TRY(hipGetLastError());
    return PCGA_OK;
}

// Control state of one stand-alone k_stencil launch with a given beta: with
// beta > 0, iteration k = 1 at parity 0, rho_{k-1} = 1 and a single (s,r)
// partial equal to beta, so that the kernel forms beta / 1 = beta exactly;
// with beta = 0, iteration 0 (the kernel then takes d = s).
__global__ void k_step_state(CtlBlock *cb, Partials P, double beta) {
    cb->c.done = 0;
    cb->c.cont = 0;
    cb->c.kk[0] = beta > 0.0 ? 1 : 0;
    cb->c.rho[1] = 1.0;
    P.sr[0] = beta > 0.0 ? beta : 1.0;
}

// (d, q) of that launch, summed from its partials as the next kernel of an
// iteration sums them; left in P.res[0].
__global__ __launch_bounds__(kBS) void k_step_dq(Partials P, int g) {
    double v[1];
    sum_partials<1>(P.dq, g, v);
    if (threadIdx.x == 0) P.res[0] = v[0];
}

// The control block and the residual history of the last `span` iterations
// (ending at the iteration count), written by the device to a snapshot slot
// in pinned host memory: the last node of a chunk graph.  A copy by the
// runtime (a DMA blit after the chunk) left the device idle for about 20 us
// per chunk.
static_assert(sizeof(Ctl) % sizeof(int32_t) == 0, "Ctl is copied as 32-bit words");
__global__ __launch_bounds__(kBS) void k_snap(const CtlBlock *cb, CtlBlock *dst, int span) {
    const int words = (int)(sizeof(Ctl) / sizeof(int32_t));
    const int32_t *src = (const int32_t *)&cb->c;
    int32_t *out = (int32_t *)&dst->c;
    for (int i = threadIdx.x; i < words; i += kBS) out[i] = src[i];
    const int k = cb->c.k;
    for (int j = threadIdx.x; j < span && j <= k; j += kBS)
        dst->hist[(k - j) & (kHistRing - 1)] = cb->hist[(k - j) & (kHistRing - 1)];
}

// History entries a graph-written snapshot carries: more than a chunk adds
// between two snapshots, and enough for predicted_left's mean rate.
int snap_span(const pcga_solver &S) { return std::min(kHistRing, std::max(S.chunk + 8, 512)); }

int snapshot(pcga_solver &S, const CtlBlock *cb, int slot) {
    HIP_TRY(hipMemcpyAsync(S.snap[slot], cb, sizeof(CtlBlock), hipMemcpyDeviceToHost, S.stream));
    HIP_TRY(hipEventRecord(S.ev[slot], S.stream));
    return PCGA_OK;
}

int wait_snap(pcga_solver &S, int slot) {
    HIP_TRY(hipEventSynchronize(S.ev[slot]));
    return PCGA_OK;
}

template <typename T>
int capture_iters(pcga_solver &S, const IterBufs<T> &B, int count, int slot, hipGraphExec_t *out) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(S.stream, hipStreamCaptureModeThreadLocal));
    launch_iters<T>(S, B, count);
    k_snap<<<1, kBS, 0, S.stream>>>(B.cb, S.snap_dev[slot], snap_span(S));
    hipError_t e = hipStreamEndCapture(S.stream, &g);
    if (e != hipSuccess) return fail(PCGA_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        *out = nullptr;
        return fail(PCGA_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    return PCGA_OK;
}

// The chunk graphs (S.chunk iterations) and the tail graphs (kTailChunk),
// one of each per snapshot slot.
template <typename T>
int ensure_graph(pcga_solver &S, const IterBufs<T> &B) {
    if (S.graph[0] && S.graph_chunk == S.chunk && (S.graph_tail[0] || S.chunk <= kTailChunk))
        return PCGA_OK;
    S.drop_graphs();
    for (int slot = 0; slot < 2; slot++) {
        int st = capture_iters<T>(S, B, S.chunk, slot, &S.graph[slot]);
        if (!st && S.chunk > kTailChunk)
            st = capture_iters<T>(S, B, kTailChunk, slot, &S.graph_tail[slot]);
        if (st) {
            S.drop_graphs();
            return st;
        }
    }
    S.graph_chunk = S.chunk;
    return PCGA_OK;
}

// Iterations left until the run stops, predicted from the residual history
// of the last snapshot: the relative residual's mean decrease per iteration
// since the run's start (or over the ring's length), extrapolated to the stop
// tolerance, and the iteration cap.  Large when there is too little history
// or no decrease.  (CG's residual is not monotone: a mean over many
// iterations predicts the stop better than the last chunk's decrease.)
int64_t predicted_left(const CtlBlock *sn, int hist_span) {
    const Ctl &c = sn->c;
    const int64_t k = c.k;
    int64_t left = std::min<int64_t>((int64_t)c.maxit - k, (int64_t)1 << 40);
    const int64_t span = std::min<int64_t>(k, hist_span - 1);
    if (span < 2 || !(c.tol > 0.0)) return left;
    const double now = sn->hist[k & (kHistRing - 1)], then = sn->hist[(k - span) & (kHistRing - 1)];
    if (!(now > 0.0) || !(then > now)) return left;
    if (now <= c.tol) return 0;
    const double per_iter = std::log(now / then) / (double)span;   // < 0
    const double est = std::log(c.tol / now) / per_iter;
    if (est < (double)left) left = (int64_t)std::ceil(est);
    return left;
}

// Run chunks until the device sets `done`.  hist_out receives entries 1..k
// as they arrive; final_slot names the snapshot holding the final state.
// After the last chunk of a solve: the x update its final iteration left
// to a stencil that did not run (a no-op on the paths that update x in
// their second kernel: there the pending counter never moves).
template <typename T>
int launch_x_pending(pcga_solver &S, const IterBufs<T> &B) {
    if (!x_deferred(S)) return PCGA_OK;
    k_x_pending<T><<<zero_grid(S.n), kBS, 0, S.stream>>>((int)S.n, B.x, B.d[0], B.d[1], B.cb);
    HIP_TRY(hipGetLastError());
    return PCGA_OK;
}

template <typename T>
int run_chunks(pcga_solver &S, const IterBufs<T> &B, double *hist_out, int64_t hist_cap,
               int64_t maxit, int &final_slot, bool graph_ok = true) {
    int st;
    const bool use_graph = S.use_graph && graph_ok;
    if (use_graph) {
        st = ensure_graph<T>(S, B);
        if (st) return st;
    }
    const bool tail_ok = !use_graph || S.graph_tail[0];
    // history entries a snapshot holds (a graph writes the last snap_span)
    const int hist_span = use_graph ? snap_span(S) : kHistRing;
    auto launch = [&](int slot, int count) -> int {
        if (use_graph) {
            HIP_TRY(hipGraphLaunch(count == S.chunk ? S.graph[slot] : S.graph_tail[slot], S.stream));
            HIP_TRY(hipEventRecord(S.ev[slot], S.stream));
            return PCGA_OK;
        }
        launch_iters<T>(S, B, count);
        HIP_TRY(hipGetLastError());
        return snapshot(S, B.cb, slot);
    };
    int64_t seen = 0;
    int64_t c = 0;
    // Guards against a device-side failure to finish: the iteration count
    // must advance with every chunk, and the device stops by maxit.
    const int64_t max_launched = maxit + 4 * (int64_t)S.chunk;
    int64_t launched = S.chunk;
    int in_flight = S.chunk;   // iterations of chunk c, not yet read
    int64_t left = (int64_t)1 << 40;   // predicted after the last snapshot read (unknown: large)
    if ((st = launch(0, S.chunk))) return st;
    for (;;) {
        // chunk c is in flight; its successor is a full chunk unless the run
        // is predicted to stop before chunk c has finished or within two full
        // chunks after it (a full chunk launched past the stop runs as
        // no-op kernels, about 7 us each against 0.3 us per iteration of a
        // short chunk's host round trip)
        const int next = (tail_ok && S.chunk > kTailChunk && left - in_flight < 2 * S.chunk)
                             ? kTailChunk : S.chunk;
        if ((st = launch((c + 1) & 1, next))) return st;
        in_flight = next;
        launched += next;
        if ((st = wait_snap(S, c & 1))) return st;
        const CtlBlock *sn = S.snap[c & 1];
        const int64_t k = sn->c.k;
        if (!sn->c.done && (k <= seen || launched > max_launched)) {
            (void)wait_snap(S, (c + 1) & 1);
            return fail(PCGA_EHIP, "device iteration did not advance (k=" + std::to_string(k) + ")");
        }
        if (hist_out) {
            for (int64_t i = seen + 1; i <= k && i < hist_cap; i++)
                hist_out[i] = sn->hist[i & (kHistRing - 1)];
        }
        seen = k;
        if (sn->c.done) {
            if ((st = wait_snap(S, (c + 1) & 1))) return st;
            final_slot = c & 1;
            return PCGA_OK;
        }
        left = predicted_left(sn, hist_span);
        c++;
    }
}

int check_solve_args(const pcga_solver *S, const double *b_dev, const double *x_dev, double tol,
                     int32_t maxit, const double *hist_host, int32_t hist_cap) {
    (void)maxit;
    if (!S || !b_dev || !x_dev) return fail(PCGA_EINVAL, "NULL argument");
    if (S->precision != PCGA_FP64) return fail(PCGA_EINVAL, "an FP64 solve needs a PCGA_FP64 solver");
    if (!(tol >= 0.0)) return fail(PCGA_EINVAL, "tol must be >= 0");
    if (hist_cap < 0 || (hist_cap > 0 && !hist_host)) return fail(PCGA_EINVAL, "bad history buffer");
    return PCGA_OK;
}

// One FP64 solve (Algorithm 1) on the vectors, partials and control block of
// B.  When B.x is not x_dev, x0 is copied in and the solution out; graph_ok
// = false launches the kernels directly (no graph is captured or replayed).
int solve64(pcga_solver &R, const IterBufs<double> &B, const double *b_dev, double *x_dev,
            double tol, int32_t maxit, int32_t *iters, double *hist_host, int32_t hist_cap,
            int32_t *hist_len, double *true_relres, bool graph_ok) {
    if (maxit < 0) maxit = (int32_t)std::min<int64_t>(R.n, INT32_MAX);
    const size_t nb8 = R.n * sizeof(double);
    if (B.x != x_dev) HIP_TRY(hipMemcpyAsync(B.x, x_dev, nb8, hipMemcpyDeviceToDevice, R.stream));
    launch_residual_prologue(R, B.cb, B.P, B.x, b_dev, B.r[0], tol, maxit);
    int st = prologue_prec<double>(R, B);
    if (st) return st;
    if ((st = snapshot(R, B.cb, 0))) return st;
    if ((st = wait_snap(R, 0))) return st;
    const Ctl c0 = R.snap[0]->c;
    if (hist_cap > 0) hist_host[0] = R.snap[0]->hist[0];
    if (c0.nb == 0.0) {
        k_zero<double><<<zero_grid(R.n), kBS, 0, R.stream>>>((int)R.n, x_dev);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(R.stream));
        if (iters) *iters = 0;
        if (hist_len) *hist_len = 1;
        if (hist_cap > 0) hist_host[0] = 0.0;
        if (true_relres) *true_relres = 0.0;
        return PCGA_OK;
    }
    int slot = 0;
    if (!c0.done) {
        if ((st = run_chunks<double>(R, B, hist_host, hist_cap, maxit, slot, graph_ok))) return st;
        if ((st = launch_x_pending<double>(R, B))) return st;
    }
    const Ctl cf = R.snap[slot]->c;
    // true residual ||b - A x|| in FP64
    launch_true_residual(R, B.cb, B.P, B.x, b_dev);
    if (B.x != x_dev) HIP_TRY(hipMemcpyAsync(x_dev, B.x, nb8, hipMemcpyDeviceToDevice, R.stream));
    if ((st = snapshot(R, B.cb, 0))) return st;
    if ((st = wait_snap(R, 0))) return st;
    const Ctl ct = R.snap[0]->c;
    if (iters) *iters = cf.k;
    if (hist_len) *hist_len = cf.k + 1;
    if (true_relres) *true_relres = std::sqrt(ct.rr_true) / std::sqrt(ct.bb);
    const int rs = map_status(cf.status);
    if (rs == PCGA_EBREAKDOWN) fail(rs, "PCG breakdown: (d,q) <= 0 or rho <= 0");
    if (rs == PCGA_ENAN) fail(rs, "NaN/Inf in the PCG iteration");
    return rs;
}

// ---------------------------------------------------------------------------
// Static scratch of the allocation-free solve.  The vectors r (two buffers),
// s, d (two buffers), q, t, the partial sums and the control block of one
// solve live in the file-scope device array `scratch` (kNoallocBytes).  Each
// device the library runs on holds its own copy until the process ends; its
// address on a device is looked up once, with that device current, and only
// that address is handed to kernels and copies (the array's name is a host
// stand-in).  Calls on one device share the array: calls that overlap on one
// device race.
// ---------------------------------------------------------------------------
constexpr int kNoallocDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kNoallocDevices] = {};

int scratch_address(int dev, unsigned char **out) {
    if (dev < 0 || dev >= kNoallocDevices)
        return fail(PCGA_EINVAL, "device index beyond the static scratch's device table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PCGA_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return PCGA_OK;
}

// Bytes of static scratch a grid of n cells needs (base == nullptr), or the
// pointers of B carved from base.
size_t carve_noalloc(int64_t n, unsigned char *base, IterBufs<double> *B) {
    Carver C(base);
    IterBufs<double> tmp{};
    IterBufs<double> &V = B ? *B : tmp;
    V.r[0] = C.take<double>(n);
    V.r[1] = C.take<double>(n);
    V.s = C.take<double>(n);
    V.d[0] = C.take<double>(n);
    V.d[1] = C.take<double>(n);
    V.q = C.take<double>(n);
    V.t = C.take<double>(n);
    V.P.dq = C.take<double>(kMaxBlocks);
    V.P.rr = C.take<double>(kMaxBlocks);
    V.P.sr = C.take<double>(kMaxBlocks);
    V.P.res = C.take<double>(3 * (size_t)kMaxBlocks);
    V.cb = C.take<CtlBlock>(1);
    return C.off;
}

}  // namespace

extern "C" {

int pcga_pcg_solve(pcga_solver_t *S, const double *b_dev, double *x_dev, double tol, int32_t maxit,
                   int32_t *iters, double *hist_host, int32_t hist_cap, int32_t *hist_len,
                   double *true_relres) {
    int st = check_solve_args(S, b_dev, x_dev, tol, maxit, hist_host, hist_cap);
    if (st) return st;
    HIP_TRY(hipSetDevice(S->device));
    return solve64(*S, bufs64(*S), b_dev, x_dev, tol, maxit, iters, hist_host, hist_cap, hist_len,
                   true_relres, true);
}

int pcga_pcg_solve_noalloc(pcga_solver_t *S, const double *b_dev, double *x_dev, double tol,
                           int32_t maxit, int32_t *iters, double *hist_host, int32_t hist_cap,
                           int32_t *hist_len, double *true_relres) {
    int st = check_solve_args(S, b_dev, x_dev, tol, maxit, hist_host, hist_cap);
    if (st) return st;
    const size_t need = carve_noalloc(S->n, nullptr, nullptr);
    if (need > kNoallocBytes)
        return fail(PCGA_ENOMEM, "pcga_pcg_solve_noalloc: a grid of " + std::to_string(S->n) +
                                     " cells needs " + std::to_string(need) +
                                     " bytes of static scratch; the library holds " +
                                     std::to_string(kNoallocBytes));
    HIP_TRY(hipSetDevice(S->device));
    unsigned char *base = nullptr;
    if ((st = scratch_address(S->device, &base))) return st;
    IterBufs<double> B = bufs64(*S);
    carve_noalloc(S->n, base, &B);
    B.x = x_dev;   // the caller's vector is the iterate
    return solve64(*S, B, b_dev, x_dev, tol, maxit, iters, hist_host, hist_cap, hist_len,
                   true_relres, false);
}

}  // extern "C"

namespace {

// Restarted refinement: every inner run starts from d = s.
int mixed_restart(pcga_solver &R, const double *b_dev, double *x_dev, double tol, double inner_tol,
                  int32_t max_outer, int32_t inner_maxit, int32_t *outer, int32_t *inner_total,
                  double *hist_host, int32_t hist_cap, int32_t *hist_len, double *true_relres) {
    IterBufs<float> B = bufs32(R);
    const size_t nb8 = R.n * sizeof(double);
    HIP_TRY(hipMemcpyAsync(R.x64[0], x_dev, nb8, hipMemcpyDeviceToDevice, R.stream));
    int cur = 0, o = 0, total = 0, st = 0, result = PCGA_OK;
    double rel = 0.0;
    for (;;) {
        launch_refine(R, o > 0, R.x64[cur], R.x64[cur ^ 1], b_dev, inner_tol, inner_maxit);
        if (o > 0) cur ^= 1;
        HIP_TRY(hipGetLastError());
        if ((st = snapshot(R, R.cb, 0))) return st;
        if ((st = wait_snap(R, 0))) return st;
        const Ctl c = R.snap[0]->c;
        if (c.bb == 0.0) {
            HIP_TRY(hipMemsetAsync(x_dev, 0, nb8, R.stream));
            HIP_TRY(hipStreamSynchronize(R.stream));
            if (outer) *outer = 0;
            if (inner_total) *inner_total = 0;
            if (hist_len) *hist_len = 1;
            if (hist_cap > 0) hist_host[0] = 0.0;
            if (true_relres) *true_relres = 0.0;
            return PCGA_OK;
        }
        rel = std::sqrt(c.rr_true) / std::sqrt(c.bb);
        if (o < hist_cap) hist_host[o] = rel;
        if (c.status == kStNan || !(rel == rel) || std::isinf(rel)) {
            result = fail(PCGA_ENAN, "NaN/Inf in residual");
            break;
        }
        if (rel <= tol) { result = PCGA_OK; break; }
        if (o == max_outer) { result = PCGA_NOCONV; break; }
        // inner FP32 PCG for A e = r32, e0 = 0
        HIP_TRY(hipMemsetAsync(B.x, 0, R.n * sizeof(float), R.stream));
        if ((st = prologue_prec<float>(R, B))) return st;
        if ((st = snapshot(R, R.cb, 0))) return st;
        if ((st = wait_snap(R, 0))) return st;
        int slot = 0;
        if (!R.snap[0]->c.done) {
            if ((st = run_chunks<float>(R, B, nullptr, 0, inner_maxit, slot))) return st;
            if ((st = launch_x_pending<float>(R, B))) return st;
        }
        const Ctl ci = R.snap[slot]->c;
        const int is = map_status(ci.status);
        if (is == PCGA_EBREAKDOWN || is == PCGA_ENAN) {
            result = fail(is, "inner FP32 PCG failed (breakdown or NaN)");
            break;
        }
        total += ci.k;
        o++;
    }
    HIP_TRY(hipMemcpyAsync(x_dev, R.x64[cur], nb8, hipMemcpyDeviceToDevice, R.stream));
    HIP_TRY(hipStreamSynchronize(R.stream));
    if (outer) *outer = o;
    if (inner_total) *inner_total = total;
    if (hist_len) *hist_len = o + 1;
    if (true_relres) *true_relres = rel;
    return result;
}


// Refinement with the direction kept across corrections (reliable updates):
// each inner run stops after reducing its residual by inner_tol (or by what
// is left to reach tol); its correction is folded into x in FP64, the
// residual is replaced by the FP64 b - A x, and the next run continues with
// the last direction, d = s + (rho_new / rho_old) d.  Everything between two
// runs is queued without a host wait: the refine's finaliser sets done when
// the outer residual has reached tol, so the queued run does nothing.
int mixed_keep(pcga_solver &R, const double *b_dev, double *x_dev, double tol, double inner_tol,
               int32_t max_outer, int32_t inner_maxit, int32_t *outer, int32_t *inner_total,
               double *hist_host, int32_t hist_cap, int32_t *hist_len, double *true_relres) {
    IterBufs<float> B = bufs32(R);
    const size_t nb8 = R.n * sizeof(double);
    HIP_TRY(hipMemcpyAsync(R.x64[0], x_dev, nb8, hipMemcpyDeviceToDevice, R.stream));
    int cur = 0, o = 0, total = 0, st = 0, result = PCGA_OK;
    double rel = 0.0;
    launch_refine(R, false, R.x64[0], nullptr, b_dev, inner_tol, inner_maxit, true, false, tol);
    for (;;) {
        HIP_TRY(hipMemsetAsync(B.x, 0, R.n * sizeof(float), R.stream));   // e = 0
        if ((st = prologue_prec<float>(R, B, o == 0))) return st;
        int slot = 0;
        if ((st = run_chunks<float>(R, B, nullptr, 0, inner_maxit, slot))) return st;
        const Ctl c = R.snap[slot]->c;
        if (c.bb == 0.0) {
            HIP_TRY(hipMemsetAsync(x_dev, 0, nb8, R.stream));
            HIP_TRY(hipStreamSynchronize(R.stream));
            if (outer) *outer = 0;
            if (inner_total) *inner_total = 0;
            if (hist_len) *hist_len = 1;
            if (hist_cap > 0) hist_host[0] = 0.0;
            if (true_relres) *true_relres = 0.0;
            return PCGA_OK;
        }
        rel = std::sqrt(c.rr_true) / std::sqrt(c.bb);
        if (o < hist_cap) hist_host[o] = rel;
        if (c.status == kStNan || !(rel == rel) || std::isinf(rel)) {
            result = fail(PCGA_ENAN, "NaN/Inf in residual");
            break;
        }
        if (rel <= tol) { result = PCGA_OK; break; }
        if (o == max_outer) { result = PCGA_NOCONV; break; }
        const int is = map_status(c.status);
        if (is == PCGA_EBREAKDOWN || is == PCGA_ENAN) {
            result = fail(is, "inner FP32 PCG failed (breakdown or NaN)");
            break;
        }
        total += c.k;
        o++;
        if ((st = launch_x_pending<float>(R, B))) return st;
        // the run's last direction d_{K-1} is in d[K & 1]; the next run reads d[0]
        if (c.k & 1)
            HIP_TRY(hipMemcpyAsync(B.d[0], B.d[1], R.n * sizeof(float), hipMemcpyDeviceToDevice,
                                   R.stream));
        launch_refine(R, true, R.x64[cur], R.x64[cur ^ 1], b_dev, inner_tol, inner_maxit, true, true,
                      tol);
        cur ^= 1;
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipMemcpyAsync(x_dev, R.x64[cur], nb8, hipMemcpyDeviceToDevice, R.stream));
    HIP_TRY(hipStreamSynchronize(R.stream));
    if (outer) *outer = o;
    if (inner_total) *inner_total = total;
    if (hist_len) *hist_len = o + 1;
    if (true_relres) *true_relres = rel;
    return result;
}

}  // namespace

extern "C" {

int pcga_pcg_solve_mixed_ex(pcga_solver_t *S, const double *b_dev, double *x_dev, double tol,
                            double inner_tol, int32_t max_outer, int32_t inner_maxit,
                            int32_t refine, int32_t *outer, int32_t *inner_total,
                            double *hist_host, int32_t hist_cap, int32_t *hist_len,
                            double *true_relres) {
    if (!S || !b_dev || !x_dev) return fail(PCGA_EINVAL, "NULL argument");
    if (S->precision != PCGA_MIXED && S->precision != PCGA_MIXED_A32)
        return fail(PCGA_EINVAL, "pcga_pcg_solve_mixed needs a PCGA_MIXED or PCGA_MIXED_A32 solver");
    if (!(tol >= 0.0) || !(inner_tol > 0.0) || max_outer < 0)
        return fail(PCGA_EINVAL, "bad tolerances or max_outer");
    if (refine != PCGA_REFINE_RESTART && refine != PCGA_REFINE_KEEP)
        return fail(PCGA_EINVAL, "refine must be PCGA_REFINE_RESTART or PCGA_REFINE_KEEP");
    if (refine == PCGA_REFINE_KEEP && !(inner_tol < 1.0))
        return fail(PCGA_EINVAL, "PCGA_REFINE_KEEP needs inner_tol < 1");
    if (inner_maxit < 0) inner_maxit = (int32_t)std::min<int64_t>(S->n, INT32_MAX);
    if (hist_cap < 0 || (hist_cap > 0 && !hist_host)) return fail(PCGA_EINVAL, "bad history buffer");
    HIP_TRY(hipSetDevice(S->device));
    if (refine == PCGA_REFINE_KEEP)
        return mixed_keep(*S, b_dev, x_dev, tol, inner_tol, max_outer, inner_maxit, outer, inner_total,
                          hist_host, hist_cap, hist_len, true_relres);
    return mixed_restart(*S, b_dev, x_dev, tol, inner_tol, max_outer, inner_maxit, outer, inner_total,
                         hist_host, hist_cap, hist_len, true_relres);
}

int pcga_pcg_solve_mixed(pcga_solver_t *S, const double *b_dev, double *x_dev, double tol,
                         double inner_tol, int32_t max_outer, int32_t inner_maxit, int32_t *outer,
                         int32_t *inner_total, double *hist_host, int32_t hist_cap,
                         int32_t *hist_len, double *true_relres) {
    return pcga_pcg_solve_mixed_ex(S, b_dev, x_dev, tol, inner_tol, max_outer, inner_maxit,
                                   PCGA_REFINE_RESTART, outer, inner_total, hist_host, hist_cap,
                                   hist_len, true_relres);
}

int pcga_apply_a(pcga_solver_t *S, const double *x_dev, double *y_dev) {
    if (!S || !x_dev || !y_dev) return fail(PCGA_EINVAL, "NULL argument");
    HIP_TRY(hipSetDevice(S->device));
    const int g = (int)std::min<int64_t>(4096, (S->n + kBS - 1) / kBS);
    if (S->csr)
        k_residual_sell<false, true><<<S->g_a, kBS, 0, S->stream>>>(S->a64, x_dev, nullptr, y_dev, S->P);
    else
        k_apply_a<<<g, kBS, 0, S->stream>>>(S->A64, x_dev, y_dev);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(S->stream));
    return PCGA_OK;
}

int pcga_apply_prec(pcga_solver_t *S, const double *r_dev, double *t_dev, double *s_dev) {
    if (!S || !r_dev || !t_dev || !s_dev) return fail(PCGA_EINVAL, "NULL argument");
    HIP_TRY(hipSetDevice(S->device));
    const int gc = (int)std::min<int64_t>(4096, (S->n + kBS - 1) / kBS);
    if (S->band_q > 0 && S->precision == PCGA_FP64) {
        k_zt_band<double, false><<<S->g_st, kBS, 0, S->stream>>>(
            S->zb64, S->band_q, S->dinv64, r_dev, nullptr, nullptr, nullptr, nullptr, t_dev,
            (int)S->n, S->cb, S->P, 0, 0);
        k_z_band<double, false, false><<<S->g_st, kBS, 0, S->stream>>>(
            S->zb64, S->band_q, t_dev, nullptr, s_dev, (int)S->n, S->cb, S->P, 0, 0);
    } else if (S->band_q > 0) {
        k_convert<double, float><<<gc, kBS, 0, S->stream>>>((int)S->n, r_dev, S->r32[0]);
        k_zt_band<float, false><<<S->g_st, kBS, 0, S->stream>>>(
            S->zb32, S->band_q, S->dinv32, S->r32[0], nullptr, nullptr, nullptr, nullptr, S->t32,
            (int)S->n, S->cb, S->P, 0, 0);
        k_z_band<float, false, false><<<S->g_st, kBS, 0, S->stream>>>(
            S->zb32, S->band_q, S->t32, nullptr, S->tmp32, (int)S->n, S->cb, S->P, 0, 0);
        k_convert<float, double><<<gc, kBS, 0, S->stream>>>((int)S->n, S->t32, t_dev);
        k_convert<float, double><<<gc, kBS, 0, S->stream>>>((int)S->n, S->tmp32, s_dev);
    } else if (S->precision == PCGA_FP64) {
        launch_zt<double, false>(S->zt64, S->fmt_zt, false, S->g_zt, S->stream, (const double *)S->dinv64, r_dev,
                                 (const double *)nullptr, (const double *)nullptr, (double *)nullptr,
                                 (double *)nullptr, t_dev, S->cb, S->P, 0, 0);
        launch_z<double, false, false>(S->z64, S->fmt_z, S->g_z, S->stream, (const double *)t_dev,
                                       (const double *)nullptr, s_dev, S->cb, S->P, 0, 0);
    } else {
        k_convert<double, float><<<gc, kBS, 0, S->stream>>>((int)S->n, r_dev, S->r32[0]);
        launch_zt<float, false>(S->zt32, S->fmt_zt, false, S->g_zt, S->stream, (const float *)S->dinv32,
                                (const float *)S->r32[0], (const float *)nullptr,
                                (const float *)nullptr, (float *)nullptr, (float *)nullptr, S->t32,
                                S->cb, S->P, 0, 0);
        launch_z<float, false, false>(S->z32, S->fmt_z, S->g_z, S->stream, (const float *)S->t32,
                                      (const float *)nullptr, S->tmp32, S->cb, S->P, 0, 0);
        k_convert<float, double><<<gc, kBS, 0, S->stream>>>((int)S->n, S->t32, t_dev);
        k_convert<float, double><<<gc, kBS, 0, S->stream>>>((int)S->n, S->tmp32, s_dev);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(S->stream));
    return PCGA_OK;
}

int pcga_step_stencil(pcga_solver_t *S, const double *s_dev, const double *d_dev, double beta,
                      double *dnew_dev, double *q_dev, double *dq) {
    if (!S || !s_dev || !d_dev || !dnew_dev || !q_dev || !dq)
        return fail(PCGA_EINVAL, "NULL argument");
    if (!(beta >= 0.0) || std::isinf(beta)) return fail(PCGA_EINVAL, "beta must be finite and >= 0");
    if (S->csr) return fail(PCGA_EINVAL, "pcga_step_stencil needs a five-point solver");
    HIP_TRY(hipSetDevice(S->device));
    pcga_solver &R = *S;
    const int gc = (int)std::min<int64_t>(4096, (R.n + kBS - 1) / kBS);
    k_step_state<<<1, 1, 0, R.stream>>>(R.cb, R.P, beta);
    if (R.precision == PCGA_FP64) {
        k_stencil<double, false><<<R.g_tile, kBS, 0, R.stream>>>(R.A64, s_dev, d_dev, dnew_dev,
                                                                     q_dev, nullptr, R.cb, R.P, 1, 0);
    } else {
        k_convert<double, float><<<gc, kBS, 0, R.stream>>>((int)R.n, s_dev, R.s32);
        k_convert<double, float><<<gc, kBS, 0, R.stream>>>((int)R.n, d_dev, R.d32[0]);
        if (R.precision == PCGA_MIXED_A32)
            k_stencil<float, false, float><<<R.g_tile, kBS, 0, R.stream>>>(
                R.A32, R.s32, R.d32[0], R.d32[1], R.q32, nullptr, R.cb, R.P, 1, 0);
        else
            k_stencil<float, false><<<R.g_tile, kBS, 0, R.stream>>>(
                R.A64, R.s32, R.d32[0], R.d32[1], R.q32, nullptr, R.cb, R.P, 1, 0);
        k_convert<float, double><<<gc, kBS, 0, R.stream>>>((int)R.n, R.d32[1], dnew_dev);
        k_convert<float, double><<<gc, kBS, 0, R.stream>>>((int)R.n, R.q32, q_dev);
    }
    k_step_dq<<<1, kBS, 0, R.stream>>>(R.P, R.g_dq());
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(dq, R.P.res, sizeof(double), hipMemcpyDeviceToHost, R.stream));
    HIP_TRY(hipStreamSynchronize(R.stream));
    return PCGA_OK;
}

int pcga_profile_iteration(pcga_solver_t *S, const double *b_dev, int32_t reps, int32_t mode,
                           double *ms_out) {
    if (!S || !b_dev || !ms_out || reps < 1 || reps > 100000 || (mode != 0 && mode != 1))
        return fail(PCGA_EINVAL, "bad profile arguments");
    HIP_TRY(hipSetDevice(S->device));
    pcga_solver &R = *S;
    const int big = INT32_MAX;
    int st;
    // start state: x0 = 0, tolerance 0 so that no kernel stops early
    auto prologue = [&]() -> int {
        if (R.precision == PCGA_FP64) {
            HIP_TRY(hipMemsetAsync(R.x, 0, R.n * sizeof(double), R.stream));
            launch_residual_prologue(R, R.cb, R.P, R.x, b_dev, R.r[0], 0.0, big);
            return prologue_prec<double>(R, bufs64(R));
        }
        HIP_TRY(hipMemsetAsync(R.x64[0], 0, R.n * sizeof(double), R.stream));
        launch_refine(R, false, R.x64[0], nullptr, b_dev, 0.0, big);
        HIP_TRY(hipMemsetAsync(R.e32, 0, R.n * sizeof(float), R.stream));
        return prologue_prec<float>(R, bufs32(R));
    };
    if ((st = prologue())) return st;
    const int nk = R.kernels_per_iter();   // 2 with the diagonal preconditioner
    const int nev = mode == 0 ? 2 : nk * reps + 1;
    ms_out[2] = 0.0;
    std::vector<hipEvent_t> ev(nev, nullptr);
    for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
    hipGraphExec_t gx = nullptr;
    auto cleanup = [&]() {
        if (gx) (void)hipGraphExecDestroy(gx);
        gx = nullptr;
        for (auto &e : ev) (void)hipEventDestroy(e);
    };
    // Run `body` once to warm up and once between events ev[first], ev[last];
    // from a captured graph when the solver replays its chunks that way.
    // With `inner`, body records its own events (direct launches only).
    auto timed = [&](auto body, bool inner) -> hipError_t {
        hipError_t e = hipSuccess;
        if (R.use_graph && !inner) {
            hipGraph_t g = nullptr;
            if ((e = hipStreamBeginCapture(R.stream, hipStreamCaptureModeThreadLocal))) return e;
            body(false);
            if ((e = hipStreamEndCapture(R.stream, &g))) return e;
            e = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e) return e;
            if ((e = hipGraphLaunch(gx, R.stream))) return e;   // warm
            if ((e = hipEventRecord(ev.front(), R.stream))) return e;
            if ((e = hipGraphLaunch(gx, R.stream))) return e;
            if ((e = hipEventRecord(ev.back(), R.stream))) return e;
        } else {
            body(false);   // warm
            if (!inner && (e = hipEventRecord(ev.front(), R.stream))) return e;
            body(inner);
            if (!inner && (e = hipEventRecord(ev.back(), R.stream))) return e;
        }
        if ((e = hipGetLastError())) return e;
        if ((e = hipStreamSynchronize(R.stream))) return e;
        if (gx) {
            (void)hipGraphExecDestroy(gx);
            gx = nullptr;
        }
        return hipSuccess;
    };
    auto elapsed = [&](int a, int b, double &ms) -> hipError_t {
        float f = 0.f;
        const hipError_t e = hipEventElapsedTime(&f, ev[a], ev[b]);
        ms = f;
        return e;
    };
    auto run = [&](auto B) -> hipError_t {
        using T = std::remove_pointer_t<decltype(B.x)>;
        hipError_t e;
        double ms = 0.0;
        if (mode == 0) {
            // each kernel alone, `reps` launches back to back (inputs stay
            // valid for every repetition: the stencil reads the prologue's
            // (s,r) partials, the residual update the last stencil's (d,q)
            // partials, and no stopping test can fire at tol 0)
            for (int w = 0; w < nk; w++) {
                e = timed([&](bool) { for (int i = 0; i < reps; i++) launch_kernel<T>(R, B, i & 1, w); },
                          false);
                if (e || (e = elapsed(0, 1, ms))) return e;
                ms_out[w] = ms / reps;
            }
        } else {
            // `reps` whole iterations with an event between every two kernels
            // (direct launches): each kernel sees the cache state of a solve
            e = timed([&](bool rec) {
                for (int i = 0; i < reps; i++)
                    for (int w = 0; w < nk; w++) {
                        if (rec) (void)hipEventRecord(ev[nk * i + w], R.stream);
                        launch_kernel<T>(R, B, i & 1, w);
                    }
                if (rec) (void)hipEventRecord(ev[nk * reps], R.stream);
            }, true);
            if (e) return e;
            double acc[3] = {0, 0, 0};
            for (int i = 0; i < reps; i++)
                for (int w = 0; w < nk; w++) {
                    if ((e = elapsed(nk * i + w, nk * i + w + 1, ms))) return e;
                    acc[w] += ms;
                }
            for (int w = 0; w < nk; w++) ms_out[w] = acc[w] / reps;
        }
        // whole iterations without events, launched as in a solve
        if (prologue()) return hipErrorUnknown;
        e = timed([&](bool) { launch_iters<T>(R, B, reps); }, false);
        if (e || (e = elapsed(0, nev - 1, ms))) return e;
        ms_out[3] = ms / reps;
        return hipSuccess;
    };
    const hipError_t e = (R.precision == PCGA_FP64) ? run(bufs64(R)) : run(bufs32(R));
    cleanup();
    if (e != hipSuccess) return fail(PCGA_EHIP, std::string("profile: ") + hipGetErrorString(e));
    return PCGA_OK;
}

}  // extern "C"
