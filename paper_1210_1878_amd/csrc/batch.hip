// batch.hip -- batched mixed-precision PCG-AINV over many independent grids.
//
// A batch is a table of slots.  A slot is one grid (the resident operator,
// D^-1 and sliced-ELL Z^T / Z of a PCGA_MIXED solver) with R right-hand
// sides (R = 1, 2 or 4) stored interleaved, [n][R], so that one read of A or
// Z serves all R.  Each right-hand side is solved by FP64 iterative
// refinement around an FP32 inner PCG (Algorithm 1 with P = Z D^-1 Z^T), the
// method of pcga_pcg_solve_mixed.
//
// One launch of each of three kernels advances every slot by one step; the
// launches do not depend on which slots exist, so a chunk of iterations is
// captured once as a HIP graph and replayed while slots come and go (the
// block table and slot descriptors live in device memory).  Each slot runs
// its own state machine; what a kernel does for a slot is given by that
// slot's state word for that kernel:
//
//   kernel      CG step (inner PCG)            refinement steps
//   kb_stencil  d = s + beta d, q = A d        RESID: r = b - A x (FP64),
//                                              r32 = fl32(r), norms
//   kb_zt       alpha, e += alpha d,           DECIDE: outer stop test; else
//               r -= alpha q, ||r||^2,         e = 0, t = D^-1 Z^T r32
//               t = D^-1 Z^T r
//   kb_z        inner stop test; s = Z t,      FIRST: s = Z t, (s,r); the next
//               (s,r); or, once the inner      CG step is inner iteration 0
//               solve ended, x += e -> RESID   (beta = 0, d = s; with the
//                                              direction kept, after the
//                                              first run: beta = rho / the
//                                              last run's rho, d = s + beta d)
//
// A slot's right-hand sides share its state; one whose inner solve converged
// is frozen (alpha = 0) until the slot's refinement step, and one that met the
// outer tolerance stays frozen (with the direction kept, a frozen right-hand
// side carries its direction and last rho to the next run).  The stop of an
// inner run is inner_tol relative to its start (restarted refinement) or
// max(inner_tol, tol / the outer residual) (direction kept).  A kernel reads only its own state word and
// writes the next kernel's, and values read by all workgroups of a launch and
// updated by workgroup 0 (rho, iteration count, active set) are
// double-buffered by the parity of the graph iteration.
//
// Workgroups reach slots through a table of logical blocks.  A slot's block
// count depends only on its grid, so each of its reductions is summed in the
// same order whatever else is in the batch: a solve gives bitwise the same
// result alone or in any mix.  The host places all blocks of a small slot on
// one XCD and splits a large one into eight contiguous ranges, one per XCD
// (table index congruent to the XCD mod 8; the launch has a multiple of 8
// workgroups and workgroup b serves table entries b, b + grid, ...).  Slice
// ranges of a slot's workgroups are balanced by Z entries (host-computed).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels.h"
#include "pcga_host.h"
#include "solver_internal.h"

namespace pcga {

constexpr int kMaxR = 4;
constexpr int kBatchGrid = 2048;     // workgroups per batched launch (multiple of 8)
constexpr int kSpreadBlocks = 128;   // slots with at least this many blocks use all XCDs

enum : int { kActSkip = 0, kActCG = 1, kActResid = 2, kActDecide = 3, kActFirst = 4 };

struct SlotCtl {
    double rho[2][kMaxR];      // rho_k, by graph parity
    double rho_keep[kMaxR];    // rho of each right-hand side's last active CG step (keep)
    double nb[kMaxR];          // ||r32|| at the start of the inner solve
    double rel[kMaxR];         // last outer relative true residual
    double bb[kMaxR];          // ||b||^2
    int32_t kk[2];             // inner iteration count, by graph parity
    int32_t act[2];            // active right-hand sides (bit mask), by graph parity
    int32_t st[3];             // next action of kb_stencil, kb_zt, kb_z
    int32_t conv;              // right-hand sides that met the outer tolerance
    int32_t outer;             // inner solves started (written by kb_z only)
    int32_t inner_total;       // inner iterations summed over inner solves
    int32_t done, status;
    int32_t pad[1];
};

struct SlotDesc {
    DevOp<double> A64;   // FP64 coefficients, also for the FP32 inner steps
    DevSell<float> zt, z;
    const float *dinv;
    float *e, *r[2], *s, *d[2], *q, *t;   // [n][R]
    double *x;                            // [n][R] FP64 solution
    const double *b;                      // [n][R] FP64 right-hand sides
    double *part;                         // partials [6][kMaxR][G]
    SlotCtl *ctl;
    double tol, inner_tol;
    int32_t max_outer, inner_maxit;
    int32_t R, G;
    int32_t keep;   // refinement keeps the inner direction across corrections
    int32_t pad;
};

struct BlkEnt {
    int32_t slot, L;
};

// One of a slot's two buffers by parity.  A select, not an index: an array
// member indexed at run time would make the compiler keep the whole
// descriptor in per-lane scratch memory instead of scalar registers.
template <typename T>
__device__ __forceinline__ T *pick(T *const (&a)[2], int i) {
    return i ? a[1] : a[0];
}

__device__ __forceinline__ double *part_at(const SlotDesc &D, int kind, int r) {
    return D.part + ((size_t)kind * kMaxR + r) * D.G;
}

// Sum, in a fixed order, NK consecutive partial kinds for R right-hand sides.
template <int NK, int R>
__device__ __forceinline__ void slot_sum(const SlotDesc &D, int kind0, double (&out)[NK][R]) {
    double v[NK * R];
#pragma unroll
    for (int i = 0; i < NK * R; i++) v[i] = 0.0;
    for (int b0 = 0; b0 < D.G; b0 += kBS) {
        const int b = b0 + threadIdx.x;
        const int bb = b < D.G ? b : 0;
        double w[NK * R];
#pragma unroll
        for (int k = 0; k < NK; k++)
#pragma unroll
            for (int r = 0; r < R; r++) w[k * R + r] = part_at(D, kind0 + k, r)[bb];
#pragma unroll
        for (int i = 0; i < NK * R; i++)
            if (b < D.G) v[i] += w[i];
    }
    block_sum_all<NK * R>(v);
#pragma unroll
    for (int k = 0; k < NK; k++)
#pragma unroll
        for (int r = 0; r < R; r++) out[k][r] = v[k * R + r];
}

template <int NK, int R>
__device__ __forceinline__ void slot_put(const SlotDesc &D, int kind0, int L, const double (&in)[NK][R]) {
    double v[NK * R];
#pragma unroll
    for (int k = 0; k < NK; k++)
#pragma unroll
        for (int r = 0; r < R; r++) v[k * R + r] = in[k][r];
    block_sum_all<NK * R>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NK; k++)
#pragma unroll
            for (int r = 0; r < R; r++) part_at(D, kind0 + k, r)[L] = v[k * R + r];
    }
}

// R consecutive values of an interleaved vector.  The slot's vectors live in
// global memory; the pointers come from the descriptor (read from memory, so
// generic to the compiler, which would emit flat loads whose completion is
// counted with LDS operations): the access goes through a global pointer.
template <typename T>
using gmem_t = __attribute__((address_space(1))) T;
template <int R, typename T>
__device__ __forceinline__ void ldv(const T *p, int k, T (&o)[R]) {
    const gmem_t<T> *g = (const gmem_t<T> *)p;
#pragma unroll
    for (int r = 0; r < R; r++) o[r] = g[(size_t)k * R + r];
}
template <int R, typename T>
__device__ __forceinline__ void stv(T *p, int k, const T (&o)[R]) {
    gmem_t<T> *g = (gmem_t<T> *)p;
#pragma unroll
    for (int r = 0; r < R; r++) g[(size_t)k * R + r] = o[r];
}

// ---------------------------------------------------------------------------
// kb_stencil
// ---------------------------------------------------------------------------
template <int R>
__device__ void stencil_cg(const SlotDesc &D, int L, int par) {
    SlotCtl *c = D.ctl;
    double rs[1][R];
    slot_sum<1, R>(D, 2, rs);
    const int k = c->kk[par];
    const int act = c->act[par];
    // keep: the first step of a later inner run continues the last direction
    const bool fresh = k == 0 && !(D.keep && c->outer > 1);
    float bt[R];
    bool bad = false, nan = false;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const bool on = (act >> r) & 1;
        if (on && !finite_pos(rs[0][r])) {
            bad = true;
            nan = nan || is_bad(rs[0][r]);
        }
        bt[r] = (fresh || !on) ? 0.f : (float)(rs[0][r] / c->rho[par ^ 1][r]);
    }
    if (bad) {
        if (L == 0 && threadIdx.x == 0) {
            c->status = nan ? kStNan : kStBreak;
            c->done = 1;
            c->st[1] = kActSkip;
        }
        return;
    }
    if (L == 0 && threadIdx.x == 0) {
#pragma unroll
        for (int r = 0; r < R; r++) {
            c->rho[par][r] = rs[0][r];
            if ((act >> r) & 1) c->rho_keep[r] = rs[0][r];
        }
        c->st[1] = kActCG;
    }
    const DevOp<double> &A = D.A64;
    const float *s = D.s, *dold = pick(D.d, par);
    float *dnew = pick(D.d, par ^ 1), *q = D.q;
    double acc[1][R];
#pragma unroll
    for (int r = 0; r < R; r++) acc[0][r] = 0.0;
    int c0, c1;
    range_of(L, D.G, A.n, c0, c1);
    // U cells per thread and pass, all their loads issued before any
    // arithmetic (more loads in flight: a slot has few workgroups)
    constexpr int U = R == 4 ? 2 : 4;
    for (int base = c0 + threadIdx.x; base < c1; base += U * kBS) {
        Nbr<double> m[U];
        float sv[U][5][R], dv[U][5][R];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int kc = base + u * kBS < c1 ? base + u * kBS : base;
            m[u] = neighbours(A, kc);
            const int idx[5] = {m[u].kS, m[u].kW, kc, m[u].kE, m[u].kN};
#pragma unroll
            for (int e = 0; e < 5; e++) {
                ldv<R>(s, idx[e], sv[u][e]);
                ldv<R>(dold, idx[e], dv[u][e]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int kc = base + u * kBS;
            if (kc >= c1) break;
            float dn[R], qn[R];
#pragma unroll
            for (int r = 0; r < R; r++) {
                float v[5];
#pragma unroll
                for (int e = 0; e < 5; e++)
                    v[e] = fresh ? sv[u][e][r] : fmaf(bt[r], dv[u][e][r], sv[u][e][r]);
                // keep: a right-hand side at rest carries its direction forward
                dn[r] = (D.keep && !fresh && !((act >> r) & 1)) ? dv[u][2][r] : v[2];
                qn[r] = (float)apply_row(m[u], (double)v[0], (double)v[1], (double)v[2],
                                         (double)v[3], (double)v[4]);
                acc[0][r] += (double)dn[r] * (double)qn[r];
            }
            stv<R>(dnew, kc, dn);
            stv<R>(q, kc, qn);
        }
    }
    slot_put<1, R>(D, 0, L, acc);
}

// r = b - A x (FP64), r32 = fl32(r) into the residual buffer of the next
// graph iteration, with ||b||^2, ||r||^2, ||r32||^2.
template <int R>
__device__ void stencil_resid(const SlotDesc &D, int L, int par) {
    SlotCtl *c = D.ctl;
    if (L == 0 && threadIdx.x == 0) c->st[1] = kActDecide;
    const DevOp<double> &A = D.A64;
    const double *x = D.x, *b = D.b;
    float *r32 = pick(D.r, par ^ 1);
    // keep: the last CG step wrote its direction to d[par]; the next run's
    // first step, one graph iteration later, reads d[par ^ 1]
    const float *dlast = pick(D.d, par);
    float *dnext = pick(D.d, par ^ 1);
    double acc[3][R];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int r = 0; r < R; r++) acc[i][r] = 0.0;
    int c0, c1;
    range_of(L, D.G, A.n, c0, c1);
    for (int kc = c0 + threadIdx.x; kc < c1; kc += kBS) {
        const Nbr<double> m = neighbours(A, kc);
        const int idx[5] = {m.kS, m.kW, kc, m.kE, m.kN};
        double xv[5][R], bv[R];
#pragma unroll
        for (int e = 0; e < 5; e++) ldv<R>(x, idx[e], xv[e]);
        ldv<R>(b, kc, bv);
        float rf[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            const double y = apply_row(m, xv[0][r], xv[1][r], xv[2][r], xv[3][r], xv[4][r]);
            const double rk = bv[r] - y;
            rf[r] = (float)rk;
            acc[0][r] += bv[r] * bv[r];
            acc[1][r] += rk * rk;
            acc[2][r] += (double)rf[r] * (double)rf[r];
        }
        stv<R>(r32, kc, rf);
        if (D.keep) {
            float dv[R];
            ldv<R>(dlast, kc, dv);
            stv<R>(dnext, kc, dv);
        }
    }
    slot_put<3, R>(D, 3, L, acc);
}

template <int R>
__device__ void stencil_body(const SlotDesc &D, int L, int par) {
    const int st = D.ctl->st[0];
    if (st == kActCG) stencil_cg<R>(D, L, par);
    else if (st == kActResid) stencil_resid<R>(D, L, par);
    else if (L == 0 && threadIdx.x == 0) D.ctl->st[1] = kActSkip;
}

__global__ __launch_bounds__(kBS) void kb_stencil(const BlkEnt *tab, int ntab, const SlotDesc *descs,
                                                  int par) {
    for (int e = blockIdx.x; e < ntab; e += gridDim.x) {
        const BlkEnt be = tab[e];
        if (be.slot < 0) continue;
        const SlotDesc D = descs[be.slot];
        switch (D.R) {
            case 1: stencil_body<1>(D, be.L, par); break;
            case 2: stencil_body<2>(D, be.L, par); break;
            default: stencil_body<4>(D, be.L, par); break;
        }
    }
}

// ---------------------------------------------------------------------------
// kb_zt
// ---------------------------------------------------------------------------
// t = D^-1 Z^T r' with r' = r - alpha q per right-hand side (FUSED) or r' = r.
// FUSED also writes r', updates e += alpha d and returns ||r'||^2.
template <int R, bool FUSED, bool NARROW>
__device__ void zt_apply_f(const SlotDesc &D, int L, const float (&al)[R], const float *rcur,
                           float *rnext, const float *dcur, double (&rr)[1][R]) {
    const DevSell<float> &M = D.zt;
    const float *q = D.q;
    float *e = D.e, *t = D.t;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    int s0, s1;
    s0 = M.bounds_b[L];
    s1 = M.bounds_b[L + 1];
    const int nsw = (s1 - s0 - w + kWavesPerBlock - 1) / kWavesPerBlock;
    for (int i0 = 0; i0 < nsw; i0 += kWave) {
        const int cnt = nsw - i0 < kWave ? nsw - i0 : kWave;
        const SliceHeaders hd = load_headers(M, s0 + w + i0 * kWavesPerBlock, kWavesPerBlock, cnt, lane);
        for (int i = 0; i < cnt; i++) {
            const SliceMeta m = header_of(hd, i);
            const int row = m.row0 + (lane >> m.lg);
            const bool lead = (lane & ((1 << m.lg) - 1)) == 0 && row < M.nrows;
            const int rw = row < M.nrows ? row : M.nrows - 1;
            float rj[R];
            {
                float rv[R], qv[R];
                ldv<R>(rcur, rw, rv);
                if (FUSED) ldv<R>(q, rw, qv);
#pragma unroll
                for (int r = 0; r < R; r++) rj[r] = FUSED ? fmaf(-al[r], qv[r], rv[r]) : rv[r];
            }
            float acc[R];
#pragma unroll
            for (int r = 0; r < R; r++) acc[r] = 0.f;
            const gmem_t<float> *vp = (const gmem_t<float> *)(M.val + m.off + lane);
            const int last = m.width - 1;
            constexpr int U = 4;
            for (int cc = 0; cc < m.width; cc += U) {
                int kk[U];
                float zv[U];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const int ci = cc + u <= last ? cc + u : last;
                    kk[u] = entry_col<NARROW ? kFmtNarrow : 0, true>(
                        load_idx<float, NARROW ? kFmtNarrow : 0>(M, m.off + (int64_t)ci * kWave + lane), rw);
                    zv[u] = vp[(int64_t)ci * kWave];
                }
                float gr[U][R], gq[U][R];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    ldv<R>(rcur, kk[u], gr[u]);
                    if (FUSED) ldv<R>(q, kk[u], gq[u]);
                }
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const float z = cc + u <= last ? zv[u] : 0.f;
#pragma unroll
                    for (int r = 0; r < R; r++) {
                        const float rk = FUSED ? fmaf(-al[r], gq[u][r], gr[u][r]) : gr[u][r];
                        acc[r] = fmaf(z, rk, acc[r]);
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < R; r++)
                for (int o = (1 << m.lg) >> 1; o > 0; o >>= 1) acc[r] += __shfl_xor(acc[r], o, kWave);
            if (lead) {
                const float di = D.dinv[row];
                float tv[R];
#pragma unroll
                for (int r = 0; r < R; r++) tv[r] = (acc[r] + rj[r]) * di;
                stv<R>(t, row, tv);
                if (FUSED) {
                    float ev[R], dv[R];
                    ldv<R>(e, row, ev);
                    ldv<R>(dcur, row, dv);
#pragma unroll
                    for (int r = 0; r < R; r++) {
                        ev[r] = fmaf(al[r], dv[r], ev[r]);
                        rr[0][r] += (double)rj[r] * (double)rj[r];
                    }
                    stv<R>(e, row, ev);
                    stv<R>(rnext, row, rj);
                }
            }
        }
    }
}

// the slot's index format (uniform over the workgroup)
template <int R, bool FUSED>
__device__ __forceinline__ void zt_apply(const SlotDesc &D, int L, const float (&al)[R],
                                         const float *rcur, float *rnext, const float *dcur,
                                         double (&rr)[1][R]) {
    if (D.zt.dist)
        zt_apply_f<R, FUSED, true>(D, L, al, rcur, rnext, dcur, rr);
    else
        zt_apply_f<R, FUSED, false>(D, L, al, rcur, rnext, dcur, rr);
}

template <int R>
__device__ void zt_cg(const SlotDesc &D, int L, int par) {
    SlotCtl *c = D.ctl;
    double dq[1][R];
    slot_sum<1, R>(D, 0, dq);
    const int act = c->act[par];
    float al[R];
    bool bad = false, nan = false;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const bool on = (act >> r) & 1;
        if (on && !finite_pos(dq[0][r])) {
            bad = true;
            nan = nan || is_bad(dq[0][r]);
        }
        al[r] = on ? (float)(c->rho[par][r] / dq[0][r]) : 0.f;
    }
    if (bad) {
        if (L == 0 && threadIdx.x == 0) {
            c->status = nan ? kStNan : kStBreak;
            c->done = 1;
            c->st[2] = kActSkip;
        }
        return;
    }
    if (L == 0 && threadIdx.x == 0) c->st[2] = kActCG;
    double rr[1][R];
#pragma unroll
    for (int r = 0; r < R; r++) rr[0][r] = 0.0;
    zt_apply<R, true>(D, L, al, pick(D.r, par), pick(D.r, par ^ 1), pick(D.d, par ^ 1), rr);
    slot_put<1, R>(D, 1, L, rr);
}

// Outer step decision after RESID (which wrote r32 into r[par ^ 1], the
// residual buffer of the inner solve's first iteration).
template <int R>
__device__ void zt_decide(const SlotDesc &D, int L, int par) {
    SlotCtl *c = D.ctl;
    double v[3][R];
    slot_sum<3, R>(D, 3, v);
    int conv = c->conv;
    bool nan = false;
    double rel[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        nan = nan || is_bad(v[0][r]) || is_bad(v[1][r]);
        // relative residual; absolute when b = 0 (then x is driven to 0)
        rel[r] = v[0][r] > 0.0 ? sqrt(v[1][r] / v[0][r]) : sqrt(v[1][r]);
        if (rel[r] <= D.tol) conv |= 1 << r;
    }
    const int all = (1 << R) - 1;
    const bool finished = nan || conv == all || c->outer >= D.max_outer;
    if (L == 0 && threadIdx.x == 0) {
#pragma unroll
        for (int r = 0; r < R; r++) {
            c->rel[r] = rel[r];
            c->bb[r] = v[0][r];
            c->nb[r] = sqrt(v[2][r]);
        }
        c->conv = conv;
        int live = 0;
#pragma unroll
        for (int r = 0; r < R; r++)
            if (v[2][r] > 0.0) live |= 1 << r;
        c->act[par] = all & ~conv & live;   // nothing to do where fl32(r) = 0
        if (finished) {
            c->status = nan ? kStNan : (conv == all ? kStOk : kStNoconv);
            c->done = 1;
            c->st[2] = kActSkip;
        } else {
            c->st[2] = kActFirst;
        }
    }
    if (finished) return;
    // e = 0 on this block's cells, then t = D^-1 Z^T r32
    int c0, c1;
    range_of(L, D.G, D.A64.n, c0, c1);
    for (int kc = c0 + threadIdx.x; kc < c1; kc += kBS) {
        float z[R];
#pragma unroll
        for (int r = 0; r < R; r++) z[r] = 0.f;
        stv<R>(D.e, kc, z);
    }
    float al[R];
#pragma unroll
    for (int r = 0; r < R; r++) al[r] = 0.f;
    double rr[1][R];
    zt_apply<R, false>(D, L, al, pick(D.r, par ^ 1), nullptr, nullptr, rr);
}

template <int R>
__device__ void zt_body(const SlotDesc &D, int L, int par) {
    const int st = D.ctl->st[1];
    if (st == kActCG) zt_cg<R>(D, L, par);
    else if (st == kActDecide) zt_decide<R>(D, L, par);
    else if (L == 0 && threadIdx.x == 0) D.ctl->st[2] = kActSkip;
}

__global__ __launch_bounds__(kBS) void kb_zt(const BlkEnt *tab, int ntab, const SlotDesc *descs,
                                             int par) {
    for (int e = blockIdx.x; e < ntab; e += gridDim.x) {
        const BlkEnt be = tab[e];
        if (be.slot < 0) continue;
        const SlotDesc D = descs[be.slot];
        switch (D.R) {
            case 1: zt_body<1>(D, be.L, par); break;
            case 2: zt_body<2>(D, be.L, par); break;
            default: zt_body<4>(D, be.L, par); break;
        }
    }
}

// ---------------------------------------------------------------------------
// kb_z
// ---------------------------------------------------------------------------
// s = Z t and (s, r) partials for R right-hand sides.
template <int R, bool NARROW>
__device__ void z_apply_f(const SlotDesc &D, int L, const float *r, double (&sr)[1][R]) {
    const DevSell<float> &M = D.z;
    const float *t = D.t;
    float *s = D.s;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    int s0, s1;
    s0 = M.bounds_b[L];
    s1 = M.bounds_b[L + 1];
    const int nsw = (s1 - s0 - w + kWavesPerBlock - 1) / kWavesPerBlock;
    for (int i0 = 0; i0 < nsw; i0 += kWave) {
        const int cnt = nsw - i0 < kWave ? nsw - i0 : kWave;
        const SliceHeaders hd = load_headers(M, s0 + w + i0 * kWavesPerBlock, kWavesPerBlock, cnt, lane);
        for (int i = 0; i < cnt; i++) {
            const SliceMeta m = header_of(hd, i);
            const int row = m.row0 + (lane >> m.lg);
            const bool lead = (lane & ((1 << m.lg) - 1)) == 0 && row < M.nrows;
            const int rw = row < M.nrows ? row : M.nrows - 1;
            float tk[R], rk[R];
            ldv<R>(t, rw, tk);
            ldv<R>(r, rw, rk);
            float acc[R];
#pragma unroll
            for (int q = 0; q < R; q++) acc[q] = 0.f;
            const gmem_t<float> *vp = (const gmem_t<float> *)(M.val + m.off + lane);
            const int last = m.width - 1;
            constexpr int U = 8;
            for (int cc = 0; cc < m.width; cc += U) {
                int jj[U];
                float zv[U];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const int ci = cc + u <= last ? cc + u : last;
                    jj[u] = entry_col<NARROW ? kFmtNarrow : 0, false>(
                        load_idx<float, NARROW ? kFmtNarrow : 0>(M, m.off + (int64_t)ci * kWave + lane), rw);
                    zv[u] = vp[(int64_t)ci * kWave];
                }
                float tv[U][R];
#pragma unroll
                for (int u = 0; u < U; u++) ldv<R>(t, jj[u], tv[u]);
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const float z = cc + u <= last ? zv[u] : 0.f;
#pragma unroll
                    for (int q = 0; q < R; q++) acc[q] = fmaf(z, tv[u][q], acc[q]);
                }
            }
#pragma unroll
            for (int q = 0; q < R; q++)
                for (int o = (1 << m.lg) >> 1; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, kWave);
            if (lead) {
                float sv[R];
#pragma unroll
                for (int q = 0; q < R; q++) {
                    sv[q] = tk[q] + acc[q];
                    sr[0][q] += (double)sv[q] * (double)rk[q];
                }
                stv<R>(s, row, sv);
            }
        }
    }
}

template <int R>
__device__ __forceinline__ void z_apply(const SlotDesc &D, int L, const float *r, double (&sr)[1][R]) {
    if (D.z.dist)
        z_apply_f<R, true>(D, L, r, sr);
    else
        z_apply_f<R, false>(D, L, r, sr);
}

template <int R>
__device__ void z_cg(const SlotDesc &D, int L, int par) {
    SlotCtl *c = D.ctl;
    double rr[1][R];
    slot_sum<1, R>(D, 1, rr);
    const int act = c->act[par];
    const int k = c->kk[par] + 1;
    int nact = act;
    bool nan = false;
#pragma unroll
    for (int r = 0; r < R; r++) {
        if (!((act >> r) & 1)) continue;
        const double rel = sqrt(rr[0][r]) / D.ctl->nb[r];
        nan = nan || is_bad(rel);
        // keep: a run stops at max(inner_tol, tol / outer residual)
        double itol = D.inner_tol;
        if (D.keep && c->rel[r] > 0.0 && D.tol / c->rel[r] > itol) itol = D.tol / c->rel[r];
        if (rel <= itol) nact &= ~(1 << r);
    }
    const bool inner_done = nact == 0 || k >= D.inner_maxit;
    if (L == 0 && threadIdx.x == 0) {
        c->kk[par ^ 1] = k;
        c->act[par ^ 1] = nact;
        if (nan) {
            c->status = kStNan;
            c->done = 1;
            c->st[0] = kActSkip;
        } else if (inner_done) {
            c->inner_total += k;
            c->st[0] = kActResid;
        } else {
            c->st[0] = kActCG;
        }
    }
    if (nan) return;
    if (inner_done) {
        // x += e (FP64) on this block's cells; the next step recomputes r
        int c0, c1;
        range_of(L, D.G, D.A64.n, c0, c1);
        for (int kc = c0 + threadIdx.x; kc < c1; kc += kBS) {
            float ev[R];
            double xv[R];
            ldv<R>(D.e, kc, ev);
            ldv<R>(D.x, kc, xv);
#pragma unroll
            for (int r = 0; r < R; r++) xv[r] += (double)ev[r];
            stv<R>(D.x, kc, xv);
        }
        return;
    }
    double sr[1][R];
#pragma unroll
    for (int r = 0; r < R; r++) sr[0][r] = 0.0;
    z_apply<R>(D, L, pick(D.r, par ^ 1), sr);
    slot_put<1, R>(D, 2, L, sr);
}

template <int R>
__device__ void z_first(const SlotDesc &D, int L, int par) {
    SlotCtl *c = D.ctl;
    if (L == 0 && threadIdx.x == 0) {
        c->kk[par ^ 1] = 0;
        c->act[par ^ 1] = c->act[par];
        c->outer += 1;
        c->st[0] = kActCG;
        // keep: the next step's beta divides by the last active rho, read
        // from the slot of this parity
        if (D.keep)
#pragma unroll
            for (int r = 0; r < R; r++) c->rho[par][r] = c->rho_keep[r];
    }
    double sr[1][R];
#pragma unroll
    for (int r = 0; r < R; r++) sr[0][r] = 0.0;
    z_apply<R>(D, L, pick(D.r, par ^ 1), sr);
    slot_put<1, R>(D, 2, L, sr);
}

template <int R>
__device__ void z_body(const SlotDesc &D, int L, int par) {
    const int st = D.ctl->st[2];
    if (st == kActCG) z_cg<R>(D, L, par);
    else if (st == kActFirst) z_first<R>(D, L, par);
    else if (L == 0 && threadIdx.x == 0) D.ctl->st[0] = kActSkip;
}

__global__ __launch_bounds__(kBS) void kb_z(const BlkEnt *tab, int ntab, const SlotDesc *descs,
                                            int par) {
    for (int e = blockIdx.x; e < ntab; e += gridDim.x) {
        const BlkEnt be = tab[e];
        if (be.slot < 0) continue;
        const SlotDesc D = descs[be.slot];
        switch (D.R) {
            case 1: z_body<1>(D, be.L, par); break;
            case 2: z_body<2>(D, be.L, par); break;
            default: z_body<4>(D, be.L, par); break;
        }
    }
}

// Copy every occupied slot's control block into one array (one host copy).
__global__ void kb_gather_ctl(const SlotDesc *descs, int nslots, SlotCtl *out) {
    const int words = (int)(sizeof(SlotCtl) / sizeof(int32_t));
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nslots * words; i += gridDim.x * blockDim.x) {
        const int s = i / words, w = i - s * words;
        const SlotCtl *c = descs[s].ctl;
        reinterpret_cast<int32_t *>(out + s)[w] = c ? reinterpret_cast<const int32_t *>(c)[w] : 0;
    }
}

// Interleave R separate FP64 vectors into [n][R] (load) or back (store).
__global__ __launch_bounds__(kBS) void kb_interleave(int n, int R, const double *const *src,
                                                     double *dst) {
    for (int k = blockIdx.x * kBS + threadIdx.x; k < n; k += gridDim.x * kBS)
        for (int r = 0; r < R; r++) dst[(size_t)k * R + r] = src[r][k];
}
__global__ __launch_bounds__(kBS) void kb_deinterleave(int n, int R, const double *src,
                                                       double *const *dst) {
    for (int k = blockIdx.x * kBS + threadIdx.x; k < n; k += gridDim.x * kBS)
        for (int r = 0; r < R; r++) dst[r][k] = src[(size_t)k * R + r];
}

}  // namespace pcga

using namespace pcga;

// ===========================================================================
// host side
// ===========================================================================
namespace {

// Per-item device workspace: [n][R] FP32 e, r[2], s, d[2], q, t; FP64 x, b;
// partials; control; pointer tables for (de)interleaving.
struct ItemLayout {
    size_t off_e, off_r0, off_r1, off_s, off_d0, off_d1, off_q, off_t, off_x, off_b, off_part,
        off_ctl, off_ptrs, total;
};

ItemLayout item_layout(int64_t n, int R, int G) {
    ItemLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        o = (o + 255) & ~size_t(255);
        const size_t at = o;
        o += bytes;
        return at;
    };
    const size_t f = (size_t)n * R * sizeof(float), dd = (size_t)n * R * sizeof(double);
    L.off_e = take(f);
    L.off_r0 = take(f);
    L.off_r1 = take(f);
    L.off_s = take(f);
    L.off_d0 = take(f);
    L.off_d1 = take(f);
    L.off_q = take(f);
    L.off_t = take(f);
    L.off_x = take(dd);
    L.off_b = take(dd);
    L.off_part = take(6 * (size_t)kMaxR * G * sizeof(double));
    L.off_ctl = take(sizeof(SlotCtl));
    L.off_ptrs = take(2 * kMaxR * sizeof(double *));
    L.total = o + 256;
    return L;
}


}  // namespace

struct pcga_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    int max_slots = 0;
    char *scratch = nullptr;          // device: descs, ctl snapshot source, table
    SlotDesc *d_desc = nullptr;
    BlkEnt *d_tab = nullptr;
    SlotCtl *d_ctl = nullptr;         // gathered control blocks
    int tab_cap = 0;
    int ntab = 0;
    bool table_dirty = true;
    std::vector<SlotDesc> desc;       // host mirror
    std::vector<int> used;            // 1 if slot occupied
    std::vector<int> xcd_of;          // XCD a slot's blocks run on
    std::vector<double *const *> x_out;
    std::vector<std::vector<double *>> x_out_ptrs;
    SlotCtl *snap = nullptr;          // pinned host, max_slots entries
    hipEvent_t ev = nullptr;
    int chunk = 16;
    int grid = kBatchGrid;            // workgroups per launch (multiple of 8)
    hipGraphExec_t graph = nullptr;
    int graph_chunk = 0, graph_grid = 0;
    int64_t iterations = 0;
    bool in_flight = false;           // chunks launched, snapshot not yet consumed
};

namespace {

size_t batch_scratch_layout(int max_slots, size_t *off_desc, size_t *off_tab, int *tab_cap,
                            size_t *off_ctl = nullptr) {
    size_t o = 0;
    auto take = [&](size_t bytes) {
        o = (o + 255) & ~size_t(255);
        const size_t at = o;
        o += bytes;
        return at;
    };
    const int cap = kBatchGrid * 8;   // up to 8 table entries per workgroup
    *off_desc = take((size_t)max_slots * sizeof(SlotDesc));
    *off_tab = take((size_t)cap * sizeof(BlkEnt));
    const size_t oc = take((size_t)max_slots * sizeof(SlotCtl));
    if (off_ctl) *off_ctl = oc;
    *tab_cap = cap;
    return o + 256;
}

// Rebuild the block table: slots are assigned to XCDs (least loaded first,
// largest slots first), and each slot's logical blocks take table indices
// congruent to its XCD mod 8.
int rebuild_table(pcga_batch &B) {
    std::vector<int> order;
    for (int i = 0; i < B.max_slots; i++)
        if (B.used[i]) order.push_back(i);
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        if (B.desc[a].G != B.desc[b].G) return B.desc[a].G > B.desc[b].G;
        return a < b;
    });
    int load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    std::vector<std::vector<BlkEnt>> per(8);
    for (int s : order) {
        const int G = B.desc[s].G;
        if (G >= kSpreadBlocks) {
            // large grid: eight contiguous block ranges, one per XCD
            for (int x = 0; x < 8; x++) {
                const int a = (int)((int64_t)G * x / 8), e = (int)((int64_t)G * (x + 1) / 8);
                for (int L = a; L < e; L++) per[x].push_back({s, L});
                load[x] += e - a;
            }
            B.xcd_of[s] = -1;
            continue;
        }
        int x = 0;
        for (int i = 1; i < 8; i++)
            if (load[i] < load[x]) x = i;
        B.xcd_of[s] = x;
        for (int L = 0; L < G; L++) per[x].push_back({s, L});
        load[x] += G;
    }
    int depth = 0;
    for (int x = 0; x < 8; x++) depth = std::max<int>(depth, (int)per[x].size());
    const int ntab = depth * 8;
    if (ntab > B.tab_cap) return fail(PCGA_ENOMEM, "batch too large for the block table");
    std::vector<BlkEnt> tab(B.tab_cap, BlkEnt{-1, 0});   // whole table: clears stale entries
    for (int x = 0; x < 8; x++)
        for (size_t i = 0; i < per[x].size(); i++) tab[i * 8 + x] = per[x][i];
    B.ntab = ntab;
    hipError_t e = hipMemcpyAsync(B.d_tab, tab.data(), tab.size() * sizeof(BlkEnt),
                                  hipMemcpyHostToDevice, B.stream);
    if (e != hipSuccess) return fail(PCGA_EHIP, std::string("table upload: ") + hipGetErrorString(e));
    e = hipMemcpyAsync(B.d_desc, B.desc.data(), B.desc.size() * sizeof(SlotDesc),
                       hipMemcpyHostToDevice, B.stream);
    if (e != hipSuccess) return fail(PCGA_EHIP, std::string("desc upload: ") + hipGetErrorString(e));
    B.table_dirty = false;
    return PCGA_OK;
}

void launch_batch_iters(pcga_batch &B, int count) {
    // ntab is read by the kernels from their argument: capture with the
    // table capacity and let empty entries be skipped.
    for (int it = 0; it < count; it++) {
        const int p = it & 1;
        kb_stencil<<<B.grid, kBS, 0, B.stream>>>(B.d_tab, B.tab_cap, B.d_desc, p);
        kb_zt<<<B.grid, kBS, 0, B.stream>>>(B.d_tab, B.tab_cap, B.d_desc, p);
        kb_z<<<B.grid, kBS, 0, B.stream>>>(B.d_tab, B.tab_cap, B.d_desc, p);
    }
}

}  // namespace

extern "C" {

int pcga_batch_scratch_bytes(int32_t max_slots, size_t *bytes) {
    if (max_slots < 1 || max_slots > 4096 || !bytes) return fail(PCGA_EINVAL, "bad max_slots");
    size_t a, b;
    int cap;
    *bytes = batch_scratch_layout(max_slots, &a, &b, &cap);
    return PCGA_OK;
}

int pcga_batch_item_bytes(const pcga_solver_t *S, int32_t nrhs, size_t *bytes) {
    if (!S || !bytes || !(nrhs == 1 || nrhs == 2 || nrhs == 4))
        return fail(PCGA_EINVAL, "bad solver or nrhs (1, 2 or 4)");
    *bytes = item_layout(S->n, nrhs, slot_blocks(S->n)).total;
    return PCGA_OK;
}

int pcga_batch_create(int32_t max_slots, void *scratch, size_t bytes, void *stream,
                      pcga_batch_t **out) {
    if (!out) return fail(PCGA_EINVAL, "out is NULL");
    *out = nullptr;
    size_t od, ot, oc;
    int cap;
    if (max_slots < 1 || max_slots > 4096) return fail(PCGA_EINVAL, "bad max_slots");
    const size_t need = batch_scratch_layout(max_slots, &od, &ot, &cap, &oc);
    if (!scratch || bytes < need) return fail(PCGA_ENOMEM, "batch scratch too small");
    if (((uintptr_t)scratch & 255u) != 0) return fail(PCGA_EINVAL, "scratch must be 256-byte aligned");
    pcga_batch *B = new (std::nothrow) pcga_batch;
    if (!B) return fail(PCGA_ENOMEM, "host allocation failed");
    B->stream = (hipStream_t)stream;
    B->max_slots = max_slots;
    B->scratch = (char *)scratch;
    B->d_desc = (SlotDesc *)(B->scratch + od);
    B->d_tab = (BlkEnt *)(B->scratch + ot);
    B->d_ctl = (SlotCtl *)(B->scratch + oc);
    B->tab_cap = cap;
    B->desc.assign(max_slots, SlotDesc{});
    B->used.assign(max_slots, 0);
    B->xcd_of.assign(max_slots, 0);
    B->x_out_ptrs.assign(max_slots, {});
    hipError_t e = hipGetDevice(&B->device);
    if (e == hipSuccess) e = hipHostMalloc((void **)&B->snap, max_slots * sizeof(SlotCtl), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&B->ev, hipEventDisableTiming);
    if (e == hipSuccess) {
        std::vector<BlkEnt> empty(cap, BlkEnt{-1, 0});
        e = hipMemcpyAsync(B->d_tab, empty.data(), cap * sizeof(BlkEnt), hipMemcpyHostToDevice, B->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    }
    if (e != hipSuccess) {
        if (B->snap) (void)hipHostFree(B->snap);
        if (B->ev) (void)hipEventDestroy(B->ev);
        delete B;
        return fail(PCGA_EHIP, std::string("batch create: ") + hipGetErrorString(e));
    }
    *out = B;
    return PCGA_OK;
}

int pcga_batch_destroy(pcga_batch_t *B) {
    if (!B) return PCGA_OK;
    if (B->graph) (void)hipGraphExecDestroy(B->graph);
    if (B->snap) (void)hipHostFree(B->snap);
    if (B->ev) (void)hipEventDestroy(B->ev);
    delete B;
    return PCGA_OK;
}

int pcga_batch_add(pcga_batch_t *B, pcga_solver_t *S, int32_t nrhs, const double *const *b_dev,
                   const double *const *x0_dev, double *const *x_out_dev, void *item_ws,
                   size_t item_bytes, double tol, double inner_tol, int32_t max_outer,
                   int32_t inner_maxit, int32_t *slot) {
    return pcga_batch_add_ex(B, S, nrhs, b_dev, x0_dev, x_out_dev, item_ws, item_bytes, tol,
                             inner_tol, max_outer, inner_maxit, PCGA_REFINE_RESTART, slot);
}

int pcga_batch_add_ex(pcga_batch_t *B, pcga_solver_t *S, int32_t nrhs, const double *const *b_dev,
                      const double *const *x0_dev, double *const *x_out_dev, void *item_ws,
                      size_t item_bytes, double tol, double inner_tol, int32_t max_outer,
                      int32_t inner_maxit, int32_t refine, int32_t *slot) {
    if (B && B->in_flight) return fail(PCGA_EINVAL, "a launch of this batch is still in flight");
    if (!B || !S || !b_dev || !x0_dev || !x_out_dev || !item_ws || !slot)
        return fail(PCGA_EINVAL, "NULL argument");
    if (S->precision != PCGA_MIXED) return fail(PCGA_EINVAL, "batch items need PCGA_MIXED solvers");
    if (!(nrhs == 1 || nrhs == 2 || nrhs == 4)) return fail(PCGA_EINVAL, "nrhs must be 1, 2 or 4");
    if (!(tol >= 0.0) || !(inner_tol > 0.0) || max_outer < 0)
        return fail(PCGA_EINVAL, "bad tolerances or max_outer");
    if (refine != PCGA_REFINE_RESTART && refine != PCGA_REFINE_KEEP)
        return fail(PCGA_EINVAL, "refine must be PCGA_REFINE_RESTART or PCGA_REFINE_KEEP");
    if (refine == PCGA_REFINE_KEEP && !(inner_tol < 1.0))
        return fail(PCGA_EINVAL, "PCGA_REFINE_KEEP needs inner_tol < 1");
    if (((uintptr_t)item_ws & 255u) != 0) return fail(PCGA_EINVAL, "item workspace must be 256-byte aligned");
    const int G = slot_blocks(S->n);
    const ItemLayout IL = item_layout(S->n, nrhs, G);
    if (item_bytes < IL.total) return fail(PCGA_ENOMEM, "item workspace too small");
    int s = -1;
    for (int i = 0; i < B->max_slots; i++)
        if (!B->used[i]) {
            s = i;
            break;
        }
    if (s < 0) return fail(PCGA_ENOMEM, "no free batch slot");
    char *w = (char *)item_ws;
    SlotDesc D{};
    D.A64 = S->A64;
    D.zt = S->zt32;
    D.z = S->z32;
    D.dinv = S->dinv32;
    D.e = (float *)(w + IL.off_e);
    D.r[0] = (float *)(w + IL.off_r0);
    D.r[1] = (float *)(w + IL.off_r1);
    D.s = (float *)(w + IL.off_s);
    D.d[0] = (float *)(w + IL.off_d0);
    D.d[1] = (float *)(w + IL.off_d1);
    D.q = (float *)(w + IL.off_q);
    D.t = (float *)(w + IL.off_t);
    D.x = (double *)(w + IL.off_x);
    D.b = (const double *)(w + IL.off_b);
    D.part = (double *)(w + IL.off_part);
    D.ctl = (SlotCtl *)(w + IL.off_ctl);
    D.tol = tol;
    D.inner_tol = inner_tol;
    D.max_outer = max_outer;
    D.inner_maxit = inner_maxit < 0 ? (int32_t)std::min<int64_t>(S->n, INT32_MAX) : inner_maxit;
    D.R = nrhs;
    D.G = G;
    D.keep = refine == PCGA_REFINE_KEEP ? 1 : 0;
    // interleave b and x0 into the item workspace; initial state: RESID
    const double **ptrs = (const double **)(w + IL.off_ptrs);
    std::vector<const double *> hp(2 * kMaxR, nullptr);
    for (int r = 0; r < nrhs; r++) {
        if (!b_dev[r] || !x0_dev[r] || !x_out_dev[r]) return fail(PCGA_EINVAL, "NULL vector pointer");
        hp[r] = b_dev[r];
        hp[kMaxR + r] = x0_dev[r];
    }
    SlotCtl c0{};
    c0.st[0] = kActResid;
    c0.st[1] = kActSkip;
    c0.st[2] = kActSkip;
    hipStream_t sm = B->stream;
    hipError_t e = hipMemcpyAsync((void *)ptrs, hp.data(), hp.size() * sizeof(double *),
                                  hipMemcpyHostToDevice, sm);
    if (e == hipSuccess) e = hipMemcpyAsync(D.ctl, &c0, sizeof(SlotCtl), hipMemcpyHostToDevice, sm);
    const int gi = (int)std::min<int64_t>(1024, (S->n + kBS - 1) / kBS);
    if (e == hipSuccess) {
        kb_interleave<<<gi, kBS, 0, sm>>>((int)S->n, nrhs, ptrs, (double *)D.b);
        kb_interleave<<<gi, kBS, 0, sm>>>((int)S->n, nrhs, ptrs + kMaxR, D.x);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(sm);
    if (e != hipSuccess) return fail(PCGA_EHIP, std::string("batch add: ") + hipGetErrorString(e));
    B->desc[s] = D;
    B->used[s] = 1;
    B->x_out_ptrs[s].assign(x_out_dev, x_out_dev + nrhs);
    B->table_dirty = true;
    *slot = s;
    return PCGA_OK;
}

// Run `chunks` chunks of `chunk` graph iterations (or until every slot is
// done), then snapshot every slot's control block.  *active receives the
// number of slots still running.
int pcga_batch_launch(pcga_batch_t *B, int32_t chunks) {
    if (!B || chunks < 1) return fail(PCGA_EINVAL, "bad arguments");
    if (B->in_flight) return fail(PCGA_EINVAL, "a launch of this batch is still in flight");
    int st;
    if (B->table_dirty && (st = rebuild_table(*B))) return st;
    if (!B->graph || B->graph_chunk != B->chunk || B->graph_grid != B->grid) {
        if (B->graph) (void)hipGraphExecDestroy(B->graph);
        B->graph = nullptr;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return fail(PCGA_EHIP, std::string("capture: ") + hipGetErrorString(e));
        launch_batch_iters(*B, B->chunk);
        e = hipStreamEndCapture(B->stream, &g);
        if (e != hipSuccess) return fail(PCGA_EHIP, std::string("capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&B->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            B->graph = nullptr;
            return fail(PCGA_EHIP, std::string("instantiate: ") + hipGetErrorString(e));
        }
        B->graph_chunk = B->chunk;
        B->graph_grid = B->grid;
    }
    for (int c = 0; c < chunks; c++) {
        const hipError_t e = hipGraphLaunch(B->graph, B->stream);
        if (e != hipSuccess) return fail(PCGA_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
        B->iterations += B->chunk;
    }
    kb_gather_ctl<<<16, 256, 0, B->stream>>>(B->d_desc, B->max_slots, B->d_ctl);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(B->snap, B->d_ctl, B->max_slots * sizeof(SlotCtl), hipMemcpyDeviceToHost,
                           B->stream);
    if (e == hipSuccess) e = hipEventRecord(B->ev, B->stream);
    if (e != hipSuccess) return fail(PCGA_EHIP, std::string("snapshot: ") + hipGetErrorString(e));
    B->in_flight = true;
    return PCGA_OK;
}

int pcga_batch_wait(pcga_batch_t *B, int32_t block, int32_t *ready, int32_t *active) {
    if (!B) return fail(PCGA_EINVAL, "B is NULL");
    if (B->in_flight) {
        const hipError_t e = block ? hipEventSynchronize(B->ev) : hipEventQuery(B->ev);
        if (!block && e == hipErrorNotReady) {
            if (ready) *ready = 0;
            return PCGA_OK;
        }
        if (e != hipSuccess) return fail(PCGA_EHIP, std::string("batch wait: ") + hipGetErrorString(e));
        B->in_flight = false;
    }
    int n_active = 0;
    for (int s = 0; s < B->max_slots; s++)
        if (B->used[s] && !B->snap[s].done) n_active++;
    if (ready) *ready = 1;
    if (active) *active = n_active;
    return PCGA_OK;
}

int pcga_batch_run(pcga_batch_t *B, int32_t chunks, int32_t *active) {
    if (!B || chunks < 1) return fail(PCGA_EINVAL, "bad arguments");
    int n_active = 0, st;
    for (int c = 0; c < chunks; c++) {
        if ((st = pcga_batch_launch(B, 1))) return st;
        if ((st = pcga_batch_wait(B, 1, nullptr, &n_active))) return st;
        if (n_active == 0) break;
    }
    if (active) *active = n_active;
    return PCGA_OK;
}

// Results of a slot (valid once done): status, outer steps, inner iterations
// and the per-right-hand-side relative true residuals.  done = 0 if running.
int pcga_batch_query(pcga_batch_t *B, int32_t slot, int32_t *done, int32_t *status, int32_t *outer,
                     int32_t *inner_total, double *true_relres) {
    if (B && B->in_flight) return fail(PCGA_EINVAL, "a launch of this batch is still in flight");
    if (!B || slot < 0 || slot >= B->max_slots || !B->used[slot]) return fail(PCGA_EINVAL, "bad slot");
    const SlotCtl &c = B->snap[slot];
    if (done) *done = c.done;
    if (status) {
        switch (c.status) {
            case kStOk: *status = PCGA_OK; break;
            case kStNoconv: *status = PCGA_NOCONV; break;
            case kStBreak: *status = PCGA_EBREAKDOWN; break;
            default: *status = PCGA_ENAN; break;
        }
    }
    if (outer) *outer = std::max(0, c.outer);
    if (inner_total) *inner_total = c.inner_total;
    if (true_relres)
        for (int r = 0; r < B->desc[slot].R; r++) true_relres[r] = c.rel[r];
    return PCGA_OK;
}

// Copy a slot's solution to its output vectors and free the slot.
int pcga_batch_remove(pcga_batch_t *B, int32_t slot) {
    if (B && B->in_flight) return fail(PCGA_EINVAL, "a launch of this batch is still in flight");
    if (!B || slot < 0 || slot >= B->max_slots || !B->used[slot]) return fail(PCGA_EINVAL, "bad slot");
    const SlotDesc &D = B->desc[slot];
    const int64_t n = D.A64.n;
    const ItemLayout IL = item_layout(n, D.R, D.G);
    double **ptrs = (double **)((char *)D.e - IL.off_e + IL.off_ptrs);
    std::vector<double *> hp(B->x_out_ptrs[slot]);
    hipError_t e = hipMemcpyAsync(ptrs, hp.data(), hp.size() * sizeof(double *), hipMemcpyHostToDevice,
                                  B->stream);
    const int gi = (int)std::min<int64_t>(1024, (n + kBS - 1) / kBS);
    if (e == hipSuccess) {
        kb_deinterleave<<<gi, kBS, 0, B->stream>>>((int)n, D.R, D.x, ptrs);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    if (e != hipSuccess) return fail(PCGA_EHIP, std::string("batch remove: ") + hipGetErrorString(e));
    B->used[slot] = 0;
    B->desc[slot] = SlotDesc{};
    B->table_dirty = true;
    return PCGA_OK;
}

int pcga_batch_set_chunk(pcga_batch_t *B, int32_t chunk) {
    if (B && B->in_flight) return fail(PCGA_EINVAL, "a launch of this batch is still in flight");
    if (!B || chunk < 2 || chunk > 512 || (chunk & 1)) return fail(PCGA_EINVAL, "chunk must be even, 2..512");
    B->chunk = chunk;
    return PCGA_OK;
}

int pcga_batch_set_grid(pcga_batch_t *B, int32_t grid) {
    if (B && B->in_flight) return fail(PCGA_EINVAL, "a launch of this batch is still in flight");
    if (!B || grid < 8 || grid > kBatchGrid || (grid & 7))
        return fail(PCGA_EINVAL, "grid must be a multiple of 8, 8.." + std::to_string(kBatchGrid));
    B->grid = grid;
    return PCGA_OK;
}

}  // extern "C"
