// pcga_dev.h -- device-visible layouts shared by the kernels and the host
// driver of the PCG-AINV solver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pcga {

constexpr int kBS = 256;           // threads per workgroup (4 wavefronts, one per SIMD)
constexpr int kWave = 64;          // CDNA wavefront
constexpr int kWavesPerBlock = kBS / kWave;
#ifndef PCGA_CPT
#define PCGA_CPT 1
#endif
constexpr int kCPT = PCGA_CPT;     // cells per thread per step (elementwise kernels)
constexpr int kStep = kBS * kCPT;  // cells per workgroup step
constexpr int kHistRing = 4096;    // residual-history ring (entries)
constexpr int kMaxBlocks = 2048;   // workgroups per kernel = partial sums per reduction
// k_stencil: grid rows per tile (tiles are TR x kBS cells), by vector type:
// FP64 8 rows (1442 x 1021: 94.0 us per iteration, 4 rows 95.4, 2 rows
// 98.5), FP32 4 rows (48.8 us per inner iteration, 8 rows 49.1)
#ifndef PCGA_TILE_ROWS_F64
#define PCGA_TILE_ROWS_F64 8
#endif
#ifndef PCGA_TILE_ROWS_F32
#define PCGA_TILE_ROWS_F32 4
#endif
template <typename T>
constexpr int tile_rows() { return sizeof(T) == 8 ? PCGA_TILE_ROWS_F64 : PCGA_TILE_ROWS_F32; }
__host__ __device__ inline int tile_count(int nx, int ny, int tr) {
    return ((nx + kBS - 1) / kBS) * ((ny + tr - 1) / tr);
}
// Default workgroups per kernel (256 CUs), as the autotuner picks them at
// 1442 x 1021 with the default slice widths: FP64 5 per CU (86.6-87.4 us
// per iteration against 89.0-89.7 with 4), mixed 6 per CU.
constexpr int kDefaultBlocks = 1280;
constexpr int kTailChunk = 4;        // iterations of the short chunk launched near a stop
constexpr int kDefaultBlocksMixed = 1536;
constexpr int kMaxBand = 8;          // widest band stored by diagonals
// Memory-side cache (Infinity Cache) of one MI355X: 256 MiB.  The streams an
// iteration reads are kept resident up to 95% of it (see cache_plan).
constexpr double kMallBytes = 268435456.0;
constexpr double kResidentBudget = 0.95 * kMallBytes;
// Above this share of the cache the resident set sheds the solution vector.
constexpr double kSpillFraction = 0.90;
constexpr int kSlotCells = 2048;   // cells per workgroup of a batch slot (target; ensemble 170 ms, 177 at 4096, 179 at 1024)

// Workgroups of a batch slot: a function of the grid alone, so that a slot's
// reductions do not depend on the rest of the batch.
inline int slot_blocks(int64_t n) {
    const int64_t g = (n + kSlotCells - 1) / kSlotCells;
    return (int)(g < 1 ? 1 : (g > kMaxBlocks ? kMaxBlocks : g));
}

// Workgroups are dispatched round-robin over the 8 XCDs; logical_block maps
// the hardware index so that the logical blocks of one XCD are consecutive
// (then contiguous cell or slice ranges of one XCD share its L2: grid
// neighbours and gathered rows are read from the same L2).
__device__ __forceinline__ int logical_block(int b, int G) {
    const int q = G >> 3, rem = G & 7, x = b & 7, i = b >> 3;
    return x * q + (x < rem ? x : rem) + i;
}

// Range [a, b) of `total` items of logical block L out of G.
__device__ __forceinline__ void range_of(int L, int G, int total, int &a, int &b) {
    a = (int)(((int64_t)L * total) / G);
    b = (int)(((int64_t)(L + 1) * total) / G);
}

// Five-point operator in A5 form, device copy.  inv_nx = 1/nx (row index by
// multiplication, corrected to the exact quotient).
template <typename T>
struct DevOp {
    const T *diag, *ae, *an;
    int32_t nx, ny, periodic, n;
    double inv_nx;
};

// Sliced ELL with per-slice lanes per row (layout described in pcga_host.h).
template <typename T>
struct DevSell {
    const int32_t *row0, *meta;
    const int64_t *off;
    const int32_t *idx;      // columns, or null in the narrow form
    const uint16_t *dist;    // narrow form: |column - row| (direction fixed per matrix)
    const T *val;
    const int32_t *toff;     // per slice: start of its offset table in tab, -1: per-lane indices
    const int32_t *tab;      // offset tables (col - row, ascending)
    const int32_t *bounds;   // slice range of wave v = L * kWavesPerBlock + w: [bounds[v], bounds[v+1])
    const int32_t *bounds_b; // the same for the block count of a batch slot
    int32_t nslices, nrows;
    // Z only (format bit kFmtZtVal): its table steps' values read from Z^T's
    // value array `alt` (runs parallel to tab: lanes l < alt_k read
    // alt[alt_a + l], the others alt[alt_b + l]; alt_k < 0: own values)
    const T *alt;
    const int32_t *alt_a, *alt_b, *alt_k;
};

// Per-workgroup partial sums of the three reductions of an iteration and of
// the residual passes (each kMaxBlocks doubles, one slot per workgroup).
struct Partials {
    double *dq, *rr, *sr, *res;   // res: 3 x kMaxBlocks
};

// Scalars and flags of one solve; lives in device memory, copied to pinned
// host memory between chunks.  Fields that a kernel both reads (all
// workgroups) and updates (workgroup 0) are double-buffered by iteration
// parity so that no workgroup can observe the update of the same launch.
struct Ctl {
    double rho[2];               // rho_k = (s_k, r_k), slot k & 1
    double nb, tol, relres;
    double bb, rr_true;          // ||b||^2 and ||b - A x||^2 of the last residual pass
    double inner_nb2;            // ||fl32(r)||^2 (mixed: inner right-hand side)
    double alpha;                // last alpha (diagnostics)
    int32_t kk[2];               // iteration count k, slot k & 1 (read by kernels)
    int32_t maxit, done, status;
    int32_t k;                   // iteration count for the host (never read by kernels)
    // x += alpha_k d_k deferred to the next iteration's stencil: the last
    // iteration whose alpha was formed, and the last whose update was applied
    int32_t ax, xa;
    // 1: this inner run continues the previous one (mixed solve with the
    // direction kept): its first iteration forms beta = rho_0 / rho[1]
    // instead of taking d = s
    int32_t cont;
    int32_t pad[2];
};

struct CtlBlock {
    Ctl c;
    double hist[kHistRing];
};

}  // namespace pcga
