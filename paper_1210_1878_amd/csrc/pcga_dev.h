// pcga_dev.h -- device-visible layouts shared by the kernels and the host
// driver of the PCG-AINV solver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pcga {

constexpr int kBlock = 256;        // threads per workgroup (4 wavefronts)
constexpr int kWave = 64;          // CDNA wavefront
constexpr int kHistRing = 4096;    // residual-history ring (entries)
constexpr int kMaxBlocks = 4096;   // upper bound on partial sums per kernel

// Five-point operator in A5 form, device copy.
template <typename T>
struct DevOp {
    const T *diag, *ae, *an;
    int32_t nx, ny, periodic, n;
};

// Sliced ELL with per-slice lanes per row (layout described in pcga_host.h).
template <typename T>
struct DevSell {
    const int32_t *row0, *meta;
    const int64_t *off;
    const int32_t *idx;
    const T *val;
    int32_t nslices, nrows;
};

// Scalars and flags of one solve; lives in device memory, copied to pinned
// host memory between chunks.
struct Ctl {
    double rho, alpha, beta, nb, tol, relres;
    double bb, rr_true;          // ||b||^2 and ||b - A x||^2 of the last residual pass
    double inner_nb2;            // ||fl32(r)||^2 (mixed: inner right-hand side)
    int32_t k, maxit, done, status;
    uint32_t cnt[8];             // last-workgroup counters, one per kernel kind
    int32_t pad[4];
};

struct CtlBlock {
    Ctl c;
    double hist[kHistRing];
};

// Counter slots
enum : int { kCntStencil = 0, kCntZt = 1, kCntZ = 2, kCntResid = 3, kCntRefine = 4 };

}  // namespace pcga
