// solver_internal.h -- the device solver object shared by the single-grid
// driver (solver.hip) and the batched driver (batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "pcga_dev.h"
#include "pcgainv.h"

struct pcga_solver {
    // (all device pointers point into the caller-provided workspace)
    int precision = PCGA_FP64;
    int64_t n = 0, nnz_off = 0;
    int nx = 0, ny = 0, periodic = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;

    pcga::DevOp<double> A64{};
    pcga::DevOp<float> A32{};   // PCGA_MIXED_A32: the operator rounded to FP32 (inner solve)
    // General sparse A (pcga_solver_create_csr): stored in sliced ELL, applied
    // by k_spmv_sell / k_residual_sell with g_a workgroups; A64 is unused
    bool csr = false;
    int64_t nnz_a = 0;
    pcga::DevSell<double> a64{};
    int32_t *bnd_a = nullptr;
    std::vector<int32_t> cost_a;
    int g_a = 1;
    pcga::DevSell<double> zt64{}, z64{};
    pcga::DevSell<float> zt32{}, z32{};
    double *dinv64 = nullptr;
    float *dinv32 = nullptr;

    // FP64 iteration vectors (PCGA_FP64)
    double *x = nullptr, *r[2] = {nullptr, nullptr}, *s = nullptr, *d[2] = {nullptr, nullptr},
           *q = nullptr, *t = nullptr;
    // FP32 inner vectors and FP64 outer solution (PCGA_MIXED)
    float *e32 = nullptr, *r32[2] = {nullptr, nullptr}, *s32 = nullptr,
          *d32[2] = {nullptr, nullptr}, *q32 = nullptr, *t32 = nullptr;
    double *x64[2] = {nullptr, nullptr};
    float *tmp32 = nullptr;   // apply_prec staging (mixed)

    pcga::Partials P{};
    pcga::CtlBlock *cb = nullptr;
    pcga::CtlBlock *snap[2] = {nullptr, nullptr};   // pinned host
    pcga::CtlBlock *snap_dev[2] = {nullptr, nullptr};   // the same, as device addresses
    hipEvent_t ev[2] = {nullptr, nullptr};

    int g_st = 1, g_zt = 1, g_z = 1;
    int g_tile = 1;   // k_stencil workgroups (five-point operator)
    int max_blocks = pcga::kDefaultBlocks;
    int chunk = 32;
    bool use_graph = true;
    // Chunk graphs, one per snapshot slot: `chunk` iterations, then a
    // one-workgroup kernel that writes the control block to that slot's
    // pinned host copy.  The tail graphs hold kTailChunk iterations: they
    // are launched instead of a full chunk when the run is predicted to
    // stop within the next chunk (fewer iterations left to run as no-ops
    // after the stop).
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t graph_tail[2] = {nullptr, nullptr};
    int graph_chunk = 0;
    void drop_graphs() {
        for (int i = 0; i < 2; i++) {
            if (graph[i]) (void)hipGraphExecDestroy(graph[i]);
            if (graph_tail[i]) (void)hipGraphExecDestroy(graph_tail[i]);
            graph[i] = graph_tail[i] = nullptr;
        }
        graph_chunk = 0;
    }
    int64_t sell_entries = 0;
    int index_bytes = 4;   // 2 when Z^T and Z use 16-bit distances
    int fmt_zt = 0, fmt_z = 0;   // storage/read format of Z^T and Z (kFmt* bits)
    // Z = I (no stored off-diagonal entries: the diagonal preconditioner):
    // two launches per iteration (k_stencil<STOP>, k_jacobi) instead of three
    bool jacobi = false;
    int kernels_per_iter() const { return jacobi ? 2 : 3; }
    // the five-point three-kernel iteration leaves x += alpha d to the next
    // iteration's stencil; the band, diagonal and CSR paths keep it in
    // their second kernel
    bool x_deferred() const { return !csr && !jacobi && band_q == 0; }
    // Banded Z (every entry within band_q <= kMaxBand rows above the
    // diagonal, e.g. the banded factor of T): stored by diagonals, applied by
    // k_zt_band / k_z_band (elementwise launches of g_st workgroups)
    int band_q = 0;
    double *zb64 = nullptr;
    float *zb32 = nullptr;
    int g_prec() const { return band_q > 0 ? g_st : g_z; }   // workgroups writing (s,r) partials
    std::vector<int32_t> cost_zt, cost_z;    // per-slice work estimates (host)
    int32_t *bnd_zt = nullptr, *bnd_z = nullptr;   // device: wavefront slice ranges
    int32_t *bnd_zt_b = nullptr, *bnd_z_b = nullptr;   // device: ranges for a batch slot
    double bytes_per_iter = 0.0;

    // per-kernel workgroup caps (five-point kernels, Z^T sweep, Z sweep); 0:
    // max_blocks
    int g_cap[3] = {0, 0, 0};
    void grids() {
        auto cap = [&](int i) {
            const int c = g_cap[i] > 0 ? g_cap[i] : max_blocks;
            return std::max(1, std::min(c, pcga::kMaxBlocks));
        };
        const int nsteps = (int)((n + pcga::kStep - 1) / pcga::kStep);
        g_st = std::max(1, std::min(nsteps, cap(0)));
        // one tile per workgroup up to kMaxBlocks (its loads all in flight at
        // once), unless capped explicitly
        // (the stencil's vector type: FP64 for a PCGA_FP64 solver, FP32 for
        // the inner iteration of the mixed forms)
        const int tr = precision == PCGA_FP64 ? pcga::tile_rows<double>() : pcga::tile_rows<float>();
        g_tile = std::max(1, std::min(pcga::tile_count(nx, ny, tr),
                                      g_cap[0] > 0 ? g_cap[0] : pcga::kMaxBlocks));
        const int nsz = precision == PCGA_FP64 ? zt64.nslices : zt32.nslices;
        const int nsr = precision == PCGA_FP64 ? z64.nslices : z32.nslices;
        g_zt = std::max(1, std::min((nsz + pcga::kWavesPerBlock - 1) / pcga::kWavesPerBlock, cap(1)));
        g_z = std::max(1, std::min((nsr + pcga::kWavesPerBlock - 1) / pcga::kWavesPerBlock, cap(2)));
        g_a = std::max(1, std::min((a64.nslices + pcga::kWavesPerBlock - 1) / pcga::kWavesPerBlock,
                                   cap(0)));
    }
    // workgroups of the operator kernels (their partial sums are read by the
    // next kernel): the five-point kernels, or the sliced-ELL sweep of a CSR A
    int g_op() const { return csr ? g_a : g_st; }
    // workgroups writing the (d, q) partials of an iteration: the tiled
    // five-point step, or the sliced-ELL sweep of a CSR A
    int g_dq() const { return csr ? g_a : g_tile; }
};
