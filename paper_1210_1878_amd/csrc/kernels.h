// kernels.h -- gfx950 kernels of one PCG-AINV iteration and its prologue.
//
// One iteration k of Algorithm 1 (with the preconditioned direction update
// d = s + beta d) is three launches, each streaming its arrays once:
//
//   k_stencil  rho_k = sum of (s,r) partials; beta = rho_k / rho_{k-1};
//              d_new = s + beta d_old;  q = A d_new;  (d_new, q) partials
//   k_zt       alpha = rho_k / sum of (d,q) partials;
//              r' = r - alpha q;  x += alpha d_new;  ||r'||^2 partials;
//              t = D^-1 Z^T r'   (r' is recomputed at the gathered rows)
//   k_z        stop test on sqrt(sum ||r'||^2 partials) / ||b||;
//              s = Z t;  (s, r') partials
//
// The three global dependencies of the method (alpha needs all of (d,q); the
// Z^T gather needs r' at other rows; beta needs all of (s,r)) are the kernel
// boundaries.  No workgroup ever waits for another inside a launch: each
// launch writes one partial sum per workgroup, and every workgroup of the
// next launch adds all of them up in the same fixed order, so all workgroups
// hold bitwise-identical scalars.  Coherence across the 8 XCDs is then only
// needed at kernel boundaries, where the runtime provides it.
//
// d and r are double-buffered because neighbouring workgroups read old values
// while others write new ones.
//
// Work split: a launch of G workgroups gives each workgroup one contiguous
// range of cells, and each wavefront of the sliced-ELL kernels one contiguous
// range of slices, balanced by a per-slice cost estimate (the polar slices
// are much heavier than ocean-interior ones).  Workgroups are dispatched
// round-robin over the 8 XCDs, so the hardware index is remapped to make the
// ranges of one XCD contiguous: grid neighbours (rows above and below, rows a
// Z column reaches) are then read from the same L2.
//
// Memory-level parallelism: every kernel issues its first loads before it
// reduces the previous launch's partial sums, so that round trip overlaps
// them.  The stencil issues every load of a step before any arithmetic
// (branch-free neighbour indices).  The sliced-ELL kernels are software
// pipelined: while one chunk of a slice is accumulated, the value and gather
// loads of the next chunk (and the next slice's own-row operands) are in
// flight; the headers of all of a wavefront's slices come with one load.
#pragma once

#include <hip/hip_runtime.h>

#include "pcga_dev.h"

namespace pcga {

enum : int { kStOk = 0, kStNoconv = 1, kStBreak = -2, kStNan = -3 };


__device__ __forceinline__ bool finite_pos(double v) { return v > 0.0 && v < INFINITY; }
__device__ __forceinline__ bool is_bad(double v) { return !(v == v) || v == INFINITY || v == -INFINITY; }

#ifndef PCGA_DPP_SUM
#define PCGA_DPP_SUM 1
#endif

// v from another lane by a DPP pattern (both 32-bit halves); lanes whose row
// is masked off, or whose source lies outside the row, read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wavefront, the same value returned to every lane.
// Fixed order: scans within rows of 16 lanes (row_shr 1, 2, 4, 8), then rows
// combined by row broadcasts; lane 63 ends with the total.
__device__ __forceinline__ double wave_sum(double v) {
#if PCGA_DPP_SUM
    v += dpp_d<0x111, 0xf>(v);   // row_shr:1
    v += dpp_d<0x112, 0xf>(v);   // row_shr:2
    v += dpp_d<0x114, 0xf>(v);   // row_shr:4
    v += dpp_d<0x118, 0xf>(v);   // row_shr:8
    v += dpp_d<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_d<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
#else
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
#endif
}

// Sum NV values over the workgroup in a fixed order; result in every thread.
template <int NV>
__device__ __forceinline__ void block_sum_all(double (&v)[NV]) {
    __shared__ double red[NV][kWavesPerBlock];
    __shared__ double tot[NV];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < NV; q++) {
        const double s = wave_sum(v[q]);
        if (lane == 0) red[q][w] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < kWavesPerBlock; i++) s += red[threadIdx.x][i];
        tot[threadIdx.x] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; q++) v[q] = tot[q];
    __syncthreads();
}

// Total of G per-workgroup partials (stride kMaxBlocks between the NV
// quantities), identical in every workgroup and thread.  Split in two so that
// a kernel can issue its own first loads between them: load_partials issues
// every load (fixed trip count, predicated), reduce_partials consumes them,
// so the read costs one memory round trip, overlapped with the caller's.
template <int NV>
struct PartialsLoad {
    static constexpr int R = kMaxBlocks / kBS;
    double v[NV][R];
};

template <int NV>
__device__ __forceinline__ PartialsLoad<NV> load_partials(const double *part, int G) {
    PartialsLoad<NV> pl;
#pragma unroll
    for (int i = 0; i < PartialsLoad<NV>::R; i++) {
        const int b = threadIdx.x + i * kBS;
        const int bb = b < G ? b : 0;
#pragma unroll
        for (int q = 0; q < NV; q++) pl.v[q][i] = part[q * kMaxBlocks + bb];
    }
    return pl;
}

template <int NV>
__device__ __forceinline__ void reduce_partials(const PartialsLoad<NV> &pl, int G, double (&out)[NV]) {
#pragma unroll
    for (int q = 0; q < NV; q++) {
        out[q] = 0.0;
#pragma unroll
        for (int i = 0; i < PartialsLoad<NV>::R; i++)
            if (threadIdx.x + i * kBS < G) out[q] += pl.v[q][i];
    }
    block_sum_all<NV>(out);
}

template <int NV>
__device__ __forceinline__ void sum_partials(const double *part, int G, double (&out)[NV]) {
    const PartialsLoad<NV> pl = load_partials<NV>(part, G);
    reduce_partials<NV>(pl, G, out);
}

// Publish this workgroup's NV partial sums.
template <int NV>
__device__ __forceinline__ void put_partials(double (&v)[NV], double *part, int L) {
    block_sum_all<NV>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; q++) part[q * kMaxBlocks + L] = v[q];
    }
}


// Neighbour indices and couplings of cell k, branch-free: an absent
// neighbour points at k itself with a zero coupling.
// Loads through a global-memory pointer.  The operator and factor arrays are
// in global memory; a kernel that takes them as arguments has its loads
// known to be global, but one that reads its descriptors from memory (the
// batch kernels) would otherwise get flat loads, whose completion is
// counted with LDS and scalar operations.
template <typename P>
using gmem = __attribute__((address_space(1))) P;
template <typename P>
__device__ __forceinline__ P gload(const P *p) {
    return *(const gmem<P> *)p;
}

template <typename T>
struct Nbr {
    int kS, kW, kE, kN;
    T cS, cW, cC, cE, cN;
};

template <typename T>
__device__ __forceinline__ Nbr<T> neighbours(const DevOp<T> &A, int k) {
    const int nx = A.nx;
    int j = (int)((double)k * A.inv_nx);
    if (j * nx > k) j--;
    if ((j + 1) * nx <= k) j++;
    const int i = k - j * nx;
    Nbr<T> m;
    const bool hasS = j > 0;
    const bool hasW = i > 0 || A.periodic;
    m.kS = hasS ? k - nx : k;
    m.kN = (j < A.ny - 1) ? k + nx : k;
    m.kW = (i > 0) ? k - 1 : (A.periodic ? k + nx - 1 : k);
    m.kE = (i < nx - 1) ? k + 1 : (A.periodic ? k - nx + 1 : k);
    const T aS = gload(A.an + m.kS);
    const T aW = gload(A.ae + m.kW);
    m.cS = hasS ? aS : T(0);
    m.cW = hasW ? aW : T(0);
    m.cC = gload(A.diag + k);
    m.cE = gload(A.ae + k);     // zero across a non-periodic east edge (input rule)
    m.cN = gload(A.an + k);     // zero on the last row (input rule)
    return m;
}

// y_k = (A v)_k with the terms in increasing column order for interior cells.
template <typename T>
__device__ __forceinline__ T apply_row(const Nbr<T> &m, T vS, T vW, T vC, T vE, T vN) {
    T acc = m.cS * vS;
    acc = fma(m.cW, vW, acc);
    acc = fma(m.cC, vC, acc);
    acc = fma(m.cE, vE, acc);
    return fma(m.cN, vN, acc);
}

// Slice header of the sliced-ELL layout (wave-uniform, scalar loads).
struct SliceMeta {
    int row0, lg, width, toff;
    int64_t off;
};

// Headers of up to 64 slices of one wavefront, one per lane (a single
// coalesced load), handed out with readlane: the wave pays one memory round
// trip for all its headers.
struct SliceHeaders {
    int row0, meta, off_lo, off_hi, toff;
};

template <typename T>
__device__ __forceinline__ SliceHeaders load_headers(const DevSell<T> &M, int first, int stride,
                                                     int count, int lane) {
    SliceHeaders h{0, 0, 0, 0, -1};
    if (lane < count) {
        const int sl = first + lane * stride;
        h.row0 = gload(M.row0 + sl);
        h.meta = gload(M.meta + sl);
        const int64_t o = gload(M.off + sl);
        h.off_lo = (int)(o & 0xffffffff);
        h.off_hi = (int)(o >> 32);
        h.toff = gload(M.toff + sl);
    }
    return h;
}

__device__ __forceinline__ SliceMeta header_of(const SliceHeaders &h, int i) {
    SliceMeta m;
    m.row0 = __builtin_amdgcn_readlane(h.row0, i);
    const int mt = __builtin_amdgcn_readlane(h.meta, i);
    m.lg = mt & 255;
    m.width = mt >> 8;
    m.off = ((int64_t)__builtin_amdgcn_readlane(h.off_hi, i) << 32) |
            (uint32_t)__builtin_amdgcn_readlane(h.off_lo, i);
    m.toff = __builtin_amdgcn_readlane(h.toff, i);
    return m;
}

// Storage and read format of a sliced-ELL matrix, a kernel template argument:
//   bit 0: 16-bit distances instead of 32-bit columns;
//   bit 1: indices read with non-temporal loads;
//   bit 2: values read with non-temporal loads.
//   bit 3 (Z^T kernel only): the solution x read and written non-temporally.
// Non-temporal reads keep a stream out of the caches, so that the data the
// host chose to keep resident in the 256 MB memory-side cache (the vectors,
// then as much of Z as fits) is not evicted by a stream that cannot fit.
//   bit 4 (Z^T kernel only): x += alpha d left to the next iteration's
//   stencil (k_zt neither reads d and x nor writes x).
//   bit 5 (Z kernel only): the values of mapped table steps read from Z^T's
//   value array (DevSell::alt), which stays resident, instead of Z's own.
constexpr int kFmtNarrow = 1, kFmtNtIdx = 2, kFmtNtVal = 4, kFmtNtX = 8, kFmtXDef = 16,
              kFmtZtVal = 32;

template <bool NT, typename P>
__device__ __forceinline__ P stream_load(const P *p) {
    if (NT) return __builtin_nontemporal_load((const gmem<P> *)p);
    return *(const gmem<P> *)p;
}

// One per-lane index (32-bit column or 16-bit distance), undecoded.
template <typename T, int FMT>
__device__ __forceinline__ int load_idx(const DevSell<T> &M, int64_t pos) {
    constexpr bool nt = (FMT & kFmtNtIdx) != 0;
    if (FMT & kFmtNarrow) return stream_load<nt>(M.dist + pos);
    return stream_load<nt>(M.idx + pos);
}

// Column of a per-lane index for a lane whose row (clamped to the matrix) is
// rowc: Z^T (LOWER) stores row - col, Z stores col - row.
template <int FMT, bool LOWER>
__device__ __forceinline__ int entry_col(int kr, int rowc) {
    if (FMT & kFmtNarrow) return LOWER ? rowc - kr : rowc + kr;
    return kr;
}

// Pass over a wavefront's slices first .. first + nsw - 1, slice by slice.
//   Table slices (one lane per row, column offsets from the slice's table):
//   the gathered column of step c is row + table[c], known as soon as the
//   table (one load per slice, fetched while the previous slice runs) is in,
//   so values and gathers of a chunk of U steps are issued together, the
//   next chunk's loads in flight while the current one is accumulated.
//   Other slices (several lanes per row, or rows too unlike each other): a
//   per-lane column index is loaded first, then gathered, one chunk ahead.
// g(k) loads the operands gathered at column k, raw; g.fin(v) makes the
// vector value from them when the chunk is summed.
// ownf(m) loads a slice's own-row operands (issued one slice ahead); pre()
// runs once, after the first slice's loads are issued and before any gather
// (the kernels reduce the previous launch's partial sums there); it is called
// by every wave, also one without slices, and the pass ends early when it
// returns false.  epi(m, acc, own) finishes a slice (called by all lanes; acc
// is this lane's partial row sum, entries in increasing column order).
template <typename T, int U, int FMT, bool LOWER, typename Gth, typename OwnF, typename EpiF,
          typename PreF>
__device__ __forceinline__ bool sell_stream(const DevSell<T> &M, int first, int nsw, int lane,
                                            const Gth &g, const OwnF &ownf, const EpiF &epi,
                                            const PreF &pre) {
    using Own = decltype(ownf(SliceMeta{}));
    using GR = decltype(g(0));   // raw gathered operands; g.fin() makes the vector value
    constexpr bool ntv = (FMT & kFmtNtVal) != 0;
    const int nlast = M.nrows - 1;
    SliceHeaders hd{0, 0, 0, 0, -1};
    int cnt = nsw < kWave ? nsw : kWave;
    auto rowc_of = [&](const SliceMeta &m) {
        const int row = m.row0 + (lane >> m.lg);
        return row < M.nrows ? row : nlast;
    };
    // offset table of a table slice: lane c holds table[min(c, width - 1)]
    // (and, for Z with kFmtZtVal, the step's map into Z^T's values)
    constexpr bool ztv = (FMT & kFmtZtVal) != 0;
    struct Tab {
        int o, a, b, k;
    };
    auto load_tab = [&](const SliceMeta &m) {
        Tab v{0, 0, 0, -1};
        if (m.toff >= 0 && m.width > 0) {
            const int i = m.toff + (lane < m.width ? lane : m.width - 1);
            v.o = M.tab[i];
            if (ztv) {
                v.a = M.alt_a[i];
                v.b = M.alt_b[i];
                v.k = M.alt_k[i];
            }
        }
        return v;
    };
    // values of steps c0..c0+U-1 (clamped to the last step; masked when summed)
    auto load_vals = [&](const SliceMeta &m, int c0, T (&zv)[U]) {
        const int last = m.width > 0 ? m.width - 1 : 0;
        const int64_t base = m.width > 0 ? m.off + lane : 0;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int c = c0 + u <= last ? c0 + u : last;
            zv[u] = stream_load<ntv>(M.val + base + (m.width > 0 ? (int64_t)c * kWave : 0));
        }
    };
    // gathers of a table slice's steps c0..c0+U-1 for a lane whose row is rowc
    auto gather_tab = [&](const SliceMeta &m, const Tab &tv, int rowc, int c0, GR (&gv)[U]) {
        const int last = m.width > 0 ? m.width - 1 : 0;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int c = c0 + u <= last ? c0 + u : last;
            const int o = __builtin_amdgcn_readlane(tv.o, c);
            int k = rowc + o;
            k = k < 0 ? 0 : (k > nlast ? nlast : k);
            gv[u] = g(k);
        }
    };
    // values of a table slice's steps c0..c0+U-1: Z's own, or through the map
    auto load_vals_tab = [&](const SliceMeta &m, const Tab &tv, int c0, T (&zv)[U]) {
        if constexpr (!ztv) {
            load_vals(m, c0, zv);
        } else {
            const int last = m.width > 0 ? m.width - 1 : 0;
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int c = c0 + u <= last ? c0 + u : last;
                const int kk = __builtin_amdgcn_readlane(tv.k, c);
                const int ka = __builtin_amdgcn_readlane(tv.a, c);
                const int kb = __builtin_amdgcn_readlane(tv.b, c);
                // Z^T's values are resident: read them with ordinary loads (a
                // non-temporal load of a resident line would mark it for early
                // eviction, before the next Z^T sweep reads it); Z's own values
                // of an unmapped step keep the stream's policy
                if (kk < 0)
                    zv[u] = stream_load<ntv>(M.val + (m.width > 0 ? m.off + lane + (int64_t)c * kWave : 0));
                else
                    zv[u] = M.alt[(lane < kk ? ka : kb) + lane];
            }
        }
    };
    T acc = T(0);
    auto accumulate = [&](const SliceMeta &m, int c0, const T (&zv)[U], const GR (&gv)[U]) {
#pragma unroll
        for (int u = 0; u < U; u++) acc = fma(c0 + u < m.width ? zv[u] : T(0), g.fin(gv[u]), acc);
    };
    // a chunk known to lie inside the slice (no step to mask)
    auto accumulate_full = [&](const T (&zv)[U], const GR (&gv)[U]) {
#pragma unroll
        for (int u = 0; u < U; u++) acc = fma(zv[u], g.fin(gv[u]), acc);
    };
    // next slice's header, table and own-row operands (prefetched)
    SliceMeta mn{0, 0, 0, -1, 0};
    Tab tabn{0, 0, 0, -1};
    Own ownn{};
    auto prefetch = [&](int i) {
        mn = header_of(hd, i);
        tabn = load_tab(mn);
        ownn = ownf(mn);
    };
    if (nsw > 0) {
        hd = load_headers(M, first, 1, cnt, lane);
        prefetch(0);
    }
    __builtin_amdgcn_sched_barrier(0);   // the loads above stay ahead of pre()
    if (!pre()) return false;
    for (int i0 = 0; i0 < nsw;) {
        for (int i = 0; i < cnt; i++) {
            // Issue priority by progress: a wave that has done less of its
            // slices gets priority (3 in its first quarter, 0 in its last).
            // Without it the oldest waves of a CU win issue arbitration and
            // finish first, and the kernel ends on a tail of the youngest
            // ones (per-wave timestamps at 1442x1021: ends spread over
            // 23-39 us; with it 32-38 us, about 2% off an iteration).
            {
                const int lvl = 3 - (4 * (i0 + i)) / nsw;
                if (lvl >= 3) __builtin_amdgcn_s_setprio(3);
                else if (lvl == 2) __builtin_amdgcn_s_setprio(2);
                else if (lvl == 1) __builtin_amdgcn_s_setprio(1);
                else __builtin_amdgcn_s_setprio(0);
            }
            const SliceMeta m = mn;
            const Tab tabv = tabn;
            const Own own = ownn;
            if (i + 1 < cnt) prefetch(i + 1);
            const int rowc = rowc_of(m);
            if (m.toff >= 0) {
                T za[U], zb[U];
                GR ga[U], gb[U];
                load_vals_tab(m, tabv, 0, za);
                gather_tab(m, tabv, rowc, 0, ga);
                // Chunks alternate between the buffers a and b; every chunk is
                // summed with the next chunk's loads already issued.  The loop
                // has a fixed trip count and no exit in its body, so that its
                // head is reached with the same loads in flight (chunk a) on
                // every path, and the waits before each sum are exact.
                // (the scheduling barriers keep each chunk's loads ahead of the
                // previous chunk's sum)
                const int nch = (m.width + U - 1) / U;
                int c0 = 0;
                for (int k = 2; k < nch; k += 2) {
                    load_vals_tab(m, tabv, c0 + U, zb);
                    gather_tab(m, tabv, rowc, c0 + U, gb);
                    __builtin_amdgcn_sched_barrier(0);
                    accumulate_full(za, ga);
                    load_vals_tab(m, tabv, c0 + 2 * U, za);
                    gather_tab(m, tabv, rowc, c0 + 2 * U, ga);
                    __builtin_amdgcn_sched_barrier(0);
                    accumulate_full(zb, gb);
                    c0 += 2 * U;
                }
                if (c0 + U < m.width) {
                    load_vals_tab(m, tabv, c0 + U, zb);
                    gather_tab(m, tabv, rowc, c0 + U, gb);
                    __builtin_amdgcn_sched_barrier(0);
                    accumulate_full(za, ga);
                    accumulate(m, c0 + U, zb, gb);
                } else {
                    accumulate(m, c0, za, ga);
                }
            } else {
                for (int c0 = 0; c0 < m.width; c0 += U) {
                    int kr[U];
                    T zv[U];
                    GR gv[U];
                    const int last = m.width - 1;
#pragma unroll
                    for (int u = 0; u < U; u++) {
                        const int c = c0 + u <= last ? c0 + u : last;
                        kr[u] = load_idx<T, FMT>(M, m.off + (int64_t)c * kWave + lane);
                    }
                    load_vals(m, c0, zv);
#pragma unroll
                    for (int u = 0; u < U; u++) gv[u] = g(entry_col<FMT, LOWER>(kr[u], rowc));
                    accumulate(m, c0, zv, gv);
                }
            }
            epi(m, acc, own);
            acc = T(0);
        }
        i0 += kWave;
        if (i0 < nsw) {
            cnt = nsw - i0 < kWave ? nsw - i0 : kWave;
            hd = load_headers(M, first + i0, 1, cnt, lane);
            prefetch(0);
        }
    }
    return true;
}

// Entry steps per chunk: FP64 for the Z^T sweep / the Z sweep, FP32 for both
// (measured at 1442 x 1021 over 2..4).
#ifndef PCGA_PIPE_UD_ZT
#define PCGA_PIPE_UD_ZT 3
#endif
#ifndef PCGA_PIPE_UD_Z
#define PCGA_PIPE_UD_Z 3
#endif
#ifndef PCGA_PIPE_UF
#define PCGA_PIPE_UF 4
#endif
template <typename T, bool LOWER>
struct PipeUnroll {
    static constexpr int U = sizeof(T) == 8 ? (LOWER ? PCGA_PIPE_UD_ZT : PCGA_PIPE_UD_Z) : PCGA_PIPE_UF;
};

// Stopping test of Algorithm 1 on ||r_k||^2 = rr (every workgroup computes
// the same): history entry k, and the solve ends when ||r_k|| / ||b|| <= tol,
// k reaches maxit, or the norm is not finite.  Returns whether it stopped.
__device__ __forceinline__ bool stop_test(CtlBlock *cb, double rr, int k) {
    Ctl *c = &cb->c;
    const double rel = sqrt(rr) / c->nb;
    const bool bad = is_bad(rel);
    const bool conv = !bad && rel <= c->tol;
    const bool stop = bad || conv || k >= c->maxit;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->k = k;
        c->relres = rel;
        cb->hist[k & (kHistRing - 1)] = rel;
        if (stop) {
            c->status = bad ? kStNan : (conv ? kStOk : kStNoconv);
            c->done = 1;
        }
    }
    return stop;
}

// ---------------------------------------------------------------------------
// k_stencil: rho_k, beta; d_new = s + beta d_old; q = A d_new; (d_new,q) partials
// par = k & 1 (fixed per position in a captured chunk; chunks are even).
// ---------------------------------------------------------------------------
// The grid is cut into tiles of TR rows by kBS columns, one column per
// thread and one tile per workgroup (a workgroup takes a contiguous range of
// tiles when there are more tiles than workgroups).  Each thread reads s and
// d_old of its column once, over the tile's rows and one halo row either
// side, and keeps d_new of those rows in registers: they are its south and
// north neighbours.  Rows of d_new and of the east couplings go through LDS
// to the west and east neighbours; a few threads load the two halo columns
// (periodic wrap included).  That is about 8 vector loads per cell where
// gathering the five neighbours' s and d_old takes 15.  An absent neighbour
// takes the cell's own d_new with a zero coupling, and the terms of
// q = A d_new are added in increasing column order (apply_row).
// STOP (diagonal preconditioner path, two launches per iteration): the stop
// test on ||r_k|| from the previous k_jacobi's partials runs here first.
// C: type of the coefficients and of the product's arithmetic (double also
// for FP32 vectors; float for the mixed form with an FP32 operator).
// XD (x update deferred from the previous iteration's k_zt, whose alpha is
// in the control block): 0 none; 1 x += alpha_{k-1} d_old on the tile's
// cells for k > 0 (the same fma on the same values as k_zt would do, so x
// is bitwise the same); 2 the same with x streamed non-temporally.  The
// update of the iteration that ends a solve is left pending and applied by
// k_x_pending.
// Column held at a tile's LDS position for grid column i in [-1, nx]: the
// periodic wrap, else clamped (a clamped column's value is never used).
__device__ __forceinline__ int tile_col(int i, int nx, bool periodic) {
    if (i < 0) return periodic ? nx - 1 : 0;
    if (i >= nx) return (periodic && i == nx) ? 0 : nx - 1;
    return i;
}

template <typename T, bool STOP, typename C = double, int XD = 0>
__global__ __launch_bounds__(kBS) void k_stencil(DevOp<C> A, const T *__restrict__ s,
                                                 const T *__restrict__ dold,
                                                 T *__restrict__ dnew, T *__restrict__ q,
                                                 T *__restrict__ x, CtlBlock *cb, Partials P,
                                                 int g_sr, int par) {
    Ctl *c = &cb->c;
    if (c->done) return;
    const PartialsLoad<1> pr = load_partials<1>(P.rr, STOP ? g_sr : 0);
    constexpr int TR = tile_rows<T>(), TH = TR + 2, TW = kBS + 2;
    __shared__ T vt[TH][TW];          // d_new of the tile, halo included
    __shared__ C at[TR][kBS + 1];     // east couplings, column 0: the west halo
    const int nx = A.nx, ny = A.ny;
    const bool per = A.periodic != 0;
    const int ntc = (nx + kBS - 1) / kBS;
    const int ntiles = ntc * ((ny + TR - 1) / TR);
    const int G = gridDim.x, L = logical_block(blockIdx.x, G);
    int t0, t1;
    range_of(L, G, ntiles, t0, t1);
    const int tx = threadIdx.x;
    // halo thread h < 2 TH: row h >> 1, west (even h) or east (odd h) column
    const bool halo = tx < 2 * TH;
    struct Tile {
        T sv[TH], dv[TH], hs, hd;
        C an[TR + 1], ae[TR], dg[TR], hae;
        T xv[XD ? TR : 1];
    };
    auto load_tile = [&](int tile, Tile &w) {
        const int tr = tile / ntc, i0 = (tile - tr * ntc) * kBS, j0 = tr * TR;
        const int i = tile_col(i0 + tx, nx, per);
#pragma unroll
        for (int r = 0; r < TH; r++) {
            const int j = min(max(j0 - 1 + r, 0), ny - 1);
            w.sv[r] = s[j * nx + i];
            w.dv[r] = dold[j * nx + i];
        }
#pragma unroll
        for (int r = 0; r < TR + 1; r++) {
            const int j = min(max(j0 - 1 + r, 0), ny - 1);
            w.an[r] = A.an[j * nx + i];
        }
#pragma unroll
        for (int r = 0; r < TR; r++) {
            const int k = min(j0 + r, ny - 1) * nx + i;
            w.ae[r] = A.ae[k];
            w.dg[r] = A.diag[k];
            if (XD) w.xv[r] = stream_load<XD == 2>(x + k);
        }
        if (halo) {
            const int hr = tx >> 1;
            const int j = min(max(j0 - 1 + hr, 0), ny - 1);
            const int hi = tile_col((tx & 1) ? i0 + kBS : i0 - 1, nx, per);
            w.hs = s[j * nx + hi];
            w.hd = dold[j * nx + hi];
            // threads of the tile's rows also bring the west column's coupling
            const int jr = min(j0 + min(hr, TR - 1), ny - 1);
            w.hae = A.ae[jr * nx + tile_col(i0 - 1, nx, per)];
        }
    };
    const PartialsLoad<1> pl = load_partials<1>(P.sr, g_sr);
    Tile w;
    if (t0 < t1) load_tile(t0, w);   // in flight during the reduction
    __builtin_amdgcn_sched_barrier(0);
    const int k = c->kk[par];
    if (STOP && k > 0) {
        double rr[1];
        reduce_partials<1>(pr, g_sr, rr);
        if (stop_test(cb, rr[0], k)) return;
    }
    double rs[1];
    reduce_partials<1>(pl, g_sr, rs);
    const double rho = rs[0];
    if (!finite_pos(rho)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            c->status = is_bad(rho) ? kStNan : kStBreak;
            c->done = 1;
        }
        return;
    }
    const double beta = (k == 0 && !c->cont) ? 0.0 : rho / c->rho[par ^ 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->rho[par] = rho;
        if (XD && k > 0) c->xa = k - 1;
    }
    const T bt = (T)beta;
    const bool xup = XD && k > 0;
    const T axp = xup ? (T)c->alpha : T(0);   // alpha_{k-1}
    double acc = 0.0;
    for (int tile = t0; tile < t1; tile++) {
        if (tile > t0) {
            __syncthreads();   // the previous tile's LDS reads are done
            load_tile(tile, w);
        }
        const int tr = tile / ntc, i0 = (tile - tr * ntc) * kBS, j0 = tr * TR;
        T v[TH];
#pragma unroll
        for (int r = 0; r < TH; r++) {
            v[r] = fma(bt, w.dv[r], w.sv[r]);
            vt[r][tx + 1] = v[r];
        }
#pragma unroll
        for (int r = 0; r < TR; r++) at[r][tx + 1] = w.ae[r];
        if (halo) {
            vt[tx >> 1][(tx & 1) ? TW - 1 : 0] = fma(bt, w.hd, w.hs);
            if ((tx & 1) == 0 && (tx >> 1) < TR) at[tx >> 1][0] = w.hae;
        }
        __syncthreads();
        const int i = i0 + tx;
        if (i < nx) {
            const bool hasW = i > 0 || per;
            const bool hasE = i < nx - 1 || per;
#pragma unroll
            for (int r = 0; r < TR; r++) {
                const int j = j0 + r;
                if (j < ny) {
                    const T vC = v[r + 1];
                    const T vS = j > 0 ? v[r] : vC;
                    const T vN = j < ny - 1 ? v[r + 2] : vC;
                    const T vW = hasW ? vt[r + 1][tx] : vC;
                    const T vE = hasE ? vt[r + 1][tx + 2] : vC;
                    Nbr<C> m;
                    m.cS = j > 0 ? w.an[r] : C(0);
                    m.cW = hasW ? at[r][tx] : C(0);
                    m.cC = w.dg[r];
                    m.cE = w.ae[r];
                    m.cN = w.an[r + 1];
                    const T y = (T)apply_row(m, (C)vS, (C)vW, (C)vC, (C)vE, (C)vN);
                    const int kc = j * nx + i;
                    dnew[kc] = vC;
                    q[kc] = y;
                    acc += (double)vC * (double)y;
                    if (XD && xup) {
                        const T xn = fma(axp, w.dv[r + 1], w.xv[XD ? r : 0]);
                        if (XD == 2) __builtin_nontemporal_store(xn, x + kc);
                        else x[kc] = xn;
                    }
                }
            }
        }
    }
    double pv[1] = {acc};
    put_partials<1>(pv, P.dq, L);
}

// ---------------------------------------------------------------------------
// k_zt: t = D^-1 Z^T r'.  FUSED: alpha = rho_k / (d,q); r' = r - alpha q
// (written to rnext), x += alpha d (unless FMT has kFmtXDef: then the next
// iteration's stencil applies it), ||r'||^2 partials.  Not fused: r' = r.
// Rows of Z^T are the columns of Z; the unit diagonal is added last.
// ---------------------------------------------------------------------------
template <typename T, bool FUSED, int FMT>
__global__ __launch_bounds__(kBS) void k_zt(DevSell<T> Zt, const T *__restrict__ dinv,
                                            const T *__restrict__ rcur, const T *__restrict__ q,
                                            const T *__restrict__ dcur, T *__restrict__ rnext,
                                            T *__restrict__ x, T *__restrict__ t, CtlBlock *cb,
                                            Partials P, int g_dq, int par) {
    Ctl *c = &cb->c;
    if (FUSED && c->done) return;
    const PartialsLoad<1> pl = load_partials<1>(P.dq, FUSED ? g_dq : 0);
    const int G = gridDim.x, L = logical_block(blockIdx.x, G);
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform
    const int v = L * kWavesPerBlock + w;   // this wave's contiguous slice range
    const int s0 = Zt.bounds[v], s1 = Zt.bounds[v + 1];
    double rr = 0.0;
    T at = T(0);
    // gathered r' = r - alpha q: loaded raw, combined only when summed (an
    // operation on a load right after it is issued would wait for it)
    struct GZt {
        T r, q;
    };
    struct {
        const T *rc, *qq;
        const T *pat;
        __device__ GZt operator()(int kk) const { return GZt{rc[kk], FUSED ? qq[kk] : T(0)}; }
        __device__ T fin(const GZt &v) const { return FUSED ? fma(-*pat, v.q, v.r) : v.r; }
    } g{rcur, q, &at};
    // own-row operands of a slice, raw (alpha is not known when the first is loaded)
    struct OwnZt {
        T rj, qj, dj, xj, ij;
    };
    constexpr bool XUPD = FUSED && !(FMT & kFmtXDef);   // x += alpha d here
    auto ownf = [&](const SliceMeta &m) {
        const int row = m.row0 + (lane >> m.lg);
        const int rw = row < Zt.nrows ? row : Zt.nrows - 1;
        OwnZt o;
        o.rj = rcur[rw];
        o.qj = FUSED ? q[rw] : T(0);
        o.dj = XUPD ? dcur[rw] : T(0);
        o.xj = XUPD ? stream_load<(FMT & kFmtNtX) != 0>(x + rw) : T(0);
        o.ij = dinv[rw];
        return o;
    };
    auto epi = [&](const SliceMeta &m, T acc, const OwnZt &o) {
        for (int sh = (1 << m.lg) >> 1; sh > 0; sh >>= 1) acc += __shfl_xor(acc, sh, kWave);
        const int row = m.row0 + (lane >> m.lg);
        if ((lane & ((1 << m.lg) - 1)) == 0 && row < Zt.nrows) {
            const T rj = FUSED ? fma(-at, o.qj, o.rj) : o.rj;
            if (FUSED) {
                rnext[row] = rj;
                if (XUPD) {
                    if (FMT & kFmtNtX)
                        __builtin_nontemporal_store(fma(at, o.dj, o.xj), x + row);
                    else
                        x[row] = fma(at, o.dj, o.xj);
                }
                rr += (double)rj * (double)rj;
            }
            t[row] = (acc + rj) * o.ij;
        }
    };
    auto pre = [&]() {
        if (!FUSED) return true;
        double dq[1];
        reduce_partials<1>(pl, g_dq, dq);
        if (!finite_pos(dq[0])) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                c->status = is_bad(dq[0]) ? kStNan : kStBreak;
                c->done = 1;
            }
            return false;
        }
        const double alpha = c->rho[par] / dq[0];
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            c->alpha = alpha;
            c->ax = c->kk[par];
        }
        at = (T)alpha;
        return true;
    };
    if (!sell_stream<T, PipeUnroll<T, true>::U, FMT, true>(Zt, s0, s1 - s0, lane, g, ownf, epi, pre))
        return;
    if (FUSED) {
        double pv[1] = {rr};
        put_partials<1>(pv, P.rr, L);
    }
}

// ---------------------------------------------------------------------------
// k_z: (DOT, not FIRST) stop test from the ||r'||^2 partials, then s = Z t and
// (s, r') partials.  FIRST: prologue (no stop test).  Neither: s = Z t only.
// ---------------------------------------------------------------------------
template <typename T, bool DOT, bool FIRST, int FMT>
__global__ __launch_bounds__(kBS) void k_z(DevSell<T> Z, const T *__restrict__ t,
                                           const T *__restrict__ r, T *__restrict__ s,
                                           CtlBlock *cb, Partials P, int g_rr, int par) {
    Ctl *c = &cb->c;
    if (DOT && c->done) return;
    constexpr bool TEST = DOT && !FIRST;
    const PartialsLoad<1> pl = load_partials<1>(P.rr, TEST ? g_rr : 0);
    const int G = gridDim.x, L = logical_block(blockIdx.x, G);
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform
    const int v = L * kWavesPerBlock + w;   // this wave's contiguous slice range
    const int s0 = Z.bounds[v], s1 = Z.bounds[v + 1];
    double sr = 0.0;
    struct {
        const T *tt;
        __device__ T operator()(int jj) const { return tt[jj]; }
        __device__ T fin(T v) const { return v; }
    } g{t};
    struct OwnZ {
        T tk, rk;
    };
    auto ownf = [&](const SliceMeta &m) {
        const int row = m.row0 + (lane >> m.lg);
        const int rw = row < Z.nrows ? row : Z.nrows - 1;
        OwnZ o;
        o.tk = t[rw];
        o.rk = DOT ? r[rw] : T(0);
        return o;
    };
    auto epi = [&](const SliceMeta &m, T acc, const OwnZ &o) {
        for (int sh = (1 << m.lg) >> 1; sh > 0; sh >>= 1) acc += __shfl_xor(acc, sh, kWave);
        const int row = m.row0 + (lane >> m.lg);
        if ((lane & ((1 << m.lg) - 1)) == 0 && row < Z.nrows) {
            const T sk = o.tk + acc;
            s[row] = sk;
            if (DOT) sr += (double)sk * (double)o.rk;
        }
    };
    // stop test on the recursive residual of the iteration that just ended
    auto pre = [&]() {
        if (!TEST) return true;
        double rr[1];
        reduce_partials<1>(pl, g_rr, rr);
        const int k = c->kk[par] + 1;
        if (blockIdx.x == 0 && threadIdx.x == 0) c->kk[par ^ 1] = k;
        return !stop_test(cb, rr[0], k);
    };
    if (!sell_stream<T, PipeUnroll<T, false>::U, FMT, false>(Z, s0, s1 - s0, lane, g, ownf, epi, pre))
        return;
    if (DOT) {
        double pv[1] = {sr};
        put_partials<1>(pv, P.sr, L);
    }
}

// ---------------------------------------------------------------------------
// General sparse A (a CSR matrix from outside the grid, as in the comparison
// of Sec. 5), stored in the sliced-ELL layout with its diagonal among the
// entries (32-bit columns, or per-slice offset tables).
//
// k_spmv_sell: the five-point kernel's step on such an operator:
// rho_k = sum of (s,r) partials, beta = rho_k / rho_{k-1};
// d_new = s + beta d_old on the wave's rows and, recomputed, at every gathered
// column; q = A d_new; (d_new, q) partials.
// ---------------------------------------------------------------------------
template <int FMT>
__global__ __launch_bounds__(kBS) void k_spmv_sell(DevSell<double> A, const double *__restrict__ s,
                                                   const double *__restrict__ dold,
                                                   double *__restrict__ dnew, double *__restrict__ q,
                                                   CtlBlock *cb, Partials P, int g_sr, int par) {
    Ctl *c = &cb->c;
    if (c->done) return;
    const PartialsLoad<1> pl = load_partials<1>(P.sr, g_sr);
    const int G = gridDim.x, L = logical_block(blockIdx.x, G);
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform
    const int v = L * kWavesPerBlock + w;
    const int s0 = A.bounds[v], s1 = A.bounds[v + 1];
    double bt = 0.0, dq = 0.0;
    // gathered d_new = s + beta d_old: loaded raw, combined when summed
    struct GS {
        double s, d;
    };
    struct {
        const double *ss, *dd;
        const double *pb;
        __device__ GS operator()(int kk) const { return GS{ss[kk], dd[kk]}; }
        __device__ double fin(const GS &g) const { return fma(*pb, g.d, g.s); }
    } g{s, dold, &bt};
    struct OwnA {
        double sk, dk;
    };
    auto ownf = [&](const SliceMeta &m) {
        const int row = m.row0 + (lane >> m.lg);
        const int rw = row < A.nrows ? row : A.nrows - 1;
        return OwnA{s[rw], dold[rw]};
    };
    auto epi = [&](const SliceMeta &m, double acc, const OwnA &o) {
        for (int sh = (1 << m.lg) >> 1; sh > 0; sh >>= 1) acc += __shfl_xor(acc, sh, kWave);
        const int row = m.row0 + (lane >> m.lg);
        if ((lane & ((1 << m.lg) - 1)) == 0 && row < A.nrows) {
            const double dn = fma(bt, o.dk, o.sk);
            dnew[row] = dn;
            q[row] = acc;
            dq += dn * acc;
        }
    };
    auto pre = [&]() {
        double rs[1];
        reduce_partials<1>(pl, g_sr, rs);
        const double rho = rs[0];
        if (!finite_pos(rho)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                c->status = is_bad(rho) ? kStNan : kStBreak;
                c->done = 1;
            }
            return false;
        }
        const int k = c->kk[par];
        bt = (k == 0) ? 0.0 : rho / c->rho[par ^ 1];
        if (blockIdx.x == 0 && threadIdx.x == 0) c->rho[par] = rho;
        return true;
    };
    if (!sell_stream<double, PipeUnroll<double, false>::U, FMT, false>(A, s0, s1 - s0, lane, g, ownf,
                                                                        epi, pre))
        return;
    double pv[1] = {dq};
    put_partials<1>(pv, P.dq, L);
}

// r = b - A x over a sliced-ELL operator (WRITE: store r), with ||b||^2 and
// ||r||^2 partials in P.res, as k_residual for the five-point operator.
// APPLY: y = A x into r instead (b not read, no partials).
template <bool WRITE, bool APPLY>
__global__ __launch_bounds__(kBS) void k_residual_sell(DevSell<double> A,
                                                       const double *__restrict__ x,
                                                       const double *__restrict__ b,
                                                       double *__restrict__ r, Partials P) {
    const int G = gridDim.x, L = logical_block(blockIdx.x, G);
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int v = L * kWavesPerBlock + w;
    const int s0 = A.bounds[v], s1 = A.bounds[v + 1];
    double bb = 0.0, rr = 0.0;
    struct {
        const double *xx;
        __device__ double operator()(int kk) const { return xx[kk]; }
        __device__ double fin(double t) const { return t; }
    } g{x};
    struct OwnR {
        double bk;
    };
    auto ownf = [&](const SliceMeta &m) {
        const int row = m.row0 + (lane >> m.lg);
        const int rw = row < A.nrows ? row : A.nrows - 1;
        return OwnR{APPLY ? 0.0 : b[rw]};
    };
    auto epi = [&](const SliceMeta &m, double acc, const OwnR &o) {
        for (int sh = (1 << m.lg) >> 1; sh > 0; sh >>= 1) acc += __shfl_xor(acc, sh, kWave);
        const int row = m.row0 + (lane >> m.lg);
        if ((lane & ((1 << m.lg) - 1)) == 0 && row < A.nrows) {
            if (APPLY) {
                r[row] = acc;
            } else {
                const double rk = o.bk - acc;
                if (WRITE) r[row] = rk;
                bb += o.bk * o.bk;
                rr += rk * rk;
            }
        }
    };
    sell_stream<double, PipeUnroll<double, false>::U, 0, false>(A, s0, s1 - s0, lane, g, ownf, epi,
                                                                 []() { return true; });
    if (!APPLY) {
        double pv[2] = {bb, rr};
        put_partials<2>(pv, P.res, L);
    }
}

// ---------------------------------------------------------------------------
// Banded factor (the paper's factor of T with band q, Sec. 3): Z has entries
// only at Z[j-m, j], m = 1..q, stored by diagonals, zb[(m-1) n + j] (0 where
// absent).  Z^T row j then reads r at j-q..j-1 and Z row i reads t at
// i+1..i+q: shifted, coalesced reads of the vectors instead of index-driven
// gathers, and no index arrays.  Entries are summed in increasing column
// order, the unit diagonal last, as in the sliced-ELL kernels.
// ---------------------------------------------------------------------------
template <typename T, bool FUSED>
__global__ __launch_bounds__(kBS) void k_zt_band(const T *__restrict__ zb, int qb,
                                                 const T *__restrict__ dinv,
                                                 const T *__restrict__ rcur,
                                                 const T *__restrict__ q,
                                                 const T *__restrict__ dcur, T *__restrict__ rnext,
                                                 T *__restrict__ x, T *__restrict__ t, int n,
                                                 CtlBlock *cb, Partials P, int g_dq, int par) {
    Ctl *c = &cb->c;
    if (FUSED && c->done) return;
    const PartialsLoad<1> pl = load_partials<1>(P.dq, FUSED ? g_dq : 0);
    const int G = gridDim.x, L = logical_block(blockIdx.x, G);
    int c0, c1;
    range_of(L, G, n, c0, c1);
    __builtin_amdgcn_sched_barrier(0);
    T at = T(0);
    if (FUSED) {
        double dq[1];
        reduce_partials<1>(pl, g_dq, dq);
        if (!finite_pos(dq[0])) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                c->status = is_bad(dq[0]) ? kStNan : kStBreak;
                c->done = 1;
            }
            return;
        }
        const double alpha = c->rho[par] / dq[0];
        if (blockIdx.x == 0 && threadIdx.x == 0) c->alpha = alpha;
        at = (T)alpha;
    }
    auto rp = [&](int k) { return FUSED ? fma(-at, q[k], rcur[k]) : rcur[k]; };
    double rr = 0.0;
    for (int j = c0 + threadIdx.x; j < c1; j += kBS) {
        T acc = T(0);
        for (int m = qb; m >= 1; m--) {
            if (j - m >= 0) acc = fma(zb[(int64_t)(m - 1) * n + j], rp(j - m), acc);
        }
        const T rj = rp(j);
        t[j] = (acc + rj) * dinv[j];
        if (FUSED) {
            rnext[j] = rj;
            x[j] = fma(at, dcur[j], x[j]);
            rr += (double)rj * (double)rj;
        }
    }
    if (FUSED) {
        double pv[1] = {rr};
        put_partials<1>(pv, P.rr, L);
    }
}

template <typename T, bool DOT, bool FIRST>
__global__ __launch_bounds__(kBS) void k_z_band(const T *__restrict__ zb, int qb,
                                                const T *__restrict__ t,
                                                const T *__restrict__ r, T *__restrict__ s, int n,
                                                CtlBlock *cb, Partials P, int g_rr, int par) {
    Ctl *c = &cb->c;
    if (DOT && c->done) return;
    constexpr bool TEST = DOT && !FIRST;
    const PartialsLoad<1> pl = load_partials<1>(P.rr, TEST ? g_rr : 0);
    const int G = gridDim.x, L = logical_block(blockIdx.x, G);
    int c0, c1;
    range_of(L, G, n, c0, c1);
    __builtin_amdgcn_sched_barrier(0);
    if (TEST) {
        double rr[1];
        reduce_partials<1>(pl, g_rr, rr);
        const int k = c->kk[par] + 1;
        if (blockIdx.x == 0 && threadIdx.x == 0) c->kk[par ^ 1] = k;
        if (stop_test(cb, rr[0], k)) return;
    }
    double sr = 0.0;
    for (int i = c0 + threadIdx.x; i < c1; i += kBS) {
        T acc = T(0);
        for (int m = 1; m <= qb; m++) {
            if (i + m < n) acc = fma(zb[(int64_t)(m - 1) * n + i + m], t[i + m], acc);
        }
        const T si = t[i] + acc;
        s[i] = si;
        if (DOT) sr += (double)si * (double)r[i];
    }
    if (DOT) {
        double pv[1] = {sr};
        put_partials<1>(pv, P.sr, L);
    }
}

// ---------------------------------------------------------------------------
// k_jacobi (diagonal preconditioner, Z = I): alpha = rho_k / (d,q);
// r' = r - alpha q; x += alpha d; s = D^-1 r'; ||r'||^2 and (s, r') partials;
// iteration count k + 1.  With k_stencil<STOP> it makes a two-launch
// iteration of the same Algorithm 1 (t = s needs no separate pass).
// FIRST (prologue): s0 = D^-1 r0 and the (s0, r0) partials only.
// ---------------------------------------------------------------------------
template <typename T, bool FIRST>
__global__ __launch_bounds__(kBS) void k_jacobi(const T *__restrict__ dinv,
                                                const T *__restrict__ rcur,
                                                const T *__restrict__ q,
                                                const T *__restrict__ dcur, T *__restrict__ rnext,
                                                T *__restrict__ x, T *__restrict__ s, int n,
                                                CtlBlock *cb, Partials P, int g_dq, int par) {
    Ctl *c = &cb->c;
    if (!FIRST && c->done) return;
    const PartialsLoad<1> pl = load_partials<1>(P.dq, FIRST ? 0 : g_dq);
    const int G = gridDim.x, L = logical_block(blockIdx.x, G);
    int c0, c1;
    range_of(L, G, n, c0, c1);
    int k0 = c0 + threadIdx.x;
    const int kc = k0 < c1 ? k0 : (c1 > 0 ? c1 - 1 : 0);
    T rv = rcur[kc], iv = dinv[kc];
    T qv = FIRST ? T(0) : q[kc], dv = FIRST ? T(0) : dcur[kc], xv = FIRST ? T(0) : x[kc];
    __builtin_amdgcn_sched_barrier(0);   // the loads above stay ahead of the reduction
    T at = T(0);
    if (!FIRST) {
        double dq[1];
        reduce_partials<1>(pl, g_dq, dq);
        if (!finite_pos(dq[0])) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                c->status = is_bad(dq[0]) ? kStNan : kStBreak;
                c->done = 1;
            }
            return;
        }
        const double alpha = c->rho[par] / dq[0];
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            c->alpha = alpha;
            c->kk[par ^ 1] = c->kk[par] + 1;
        }
        at = (T)alpha;
    }
    double rr = 0.0, sr = 0.0;
    for (; k0 < c1; k0 += kBS) {
        const T rj = FIRST ? rv : fma(-at, qv, rv);
        const T sj = rj * iv;
        if (!FIRST) {
            rnext[k0] = rj;
            x[k0] = fma(at, dv, xv);
        }
        s[k0] = sj;
        rr += (double)rj * (double)rj;
        sr += (double)sj * (double)rj;
        const int kn = k0 + kBS;
        if (kn < c1) {
            rv = rcur[kn];
            iv = dinv[kn];
            if (!FIRST) {
                qv = q[kn];
                dv = dcur[kn];
                xv = x[kn];
            }
        }
    }
    double pv[2] = {rr, sr};
    block_sum_all<2>(pv);
    if (threadIdx.x == 0) {
        P.rr[L] = pv[0];
        P.sr[L] = pv[1];
    }
}

// ---------------------------------------------------------------------------
// Residual passes (FP64): r = b - A x with ||b||^2, ||r||^2 partials in P.res.
// WRITE: store r.  Finalised by k_fin_residual (one workgroup).
// ---------------------------------------------------------------------------
template <bool WRITE>
__global__ __launch_bounds__(kBS) void k_residual(DevOp<double> A, const double *__restrict__ x,
                                                  const double *__restrict__ b,
                                                  double *__restrict__ r, Partials P) {
    const int G = gridDim.x, L = logical_block(blockIdx.x, G);
    double bb = 0.0, rr = 0.0;
    int c0, c1;
    range_of(L, G, A.n, c0, c1);
    for (int base = c0 + threadIdx.x; base < c1 + (int)threadIdx.x; base += kStep) {
#pragma unroll
        for (int u = 0; u < kCPT; u++) {
            const int k = base + u * kBS;
            if (k < c1) {
                const Nbr<double> m = neighbours(A, k);
                const double y = apply_row(m, x[m.kS], x[m.kW], x[k], x[m.kE], x[m.kN]);
                const double bk = b[k];
                const double rk = bk - y;
                if (WRITE) r[k] = rk;
                bb += bk * bk;
                rr += rk * rk;
            }
        }
    }
    double pv[2] = {bb, rr};
    put_partials<2>(pv, P.res, L);
}

// MODE 0 (solve prologue): nb, tol, maxit, k = 0, hist[0], done when ||b|| = 0,
// the start is converged or maxit = 0.  MODE 1 (true residual): bb, rr_true.
template <int MODE>
__global__ __launch_bounds__(kBS) void k_fin_residual(CtlBlock *cb, Partials P, int g,
                                                      double tol, int maxit) {
    double v[2];
    sum_partials<2>(P.res, g, v);
    if (threadIdx.x != 0) return;
    Ctl *c = &cb->c;
    c->bb = v[0];
    if (MODE == 1) {
        c->rr_true = v[1];
        return;
    }
    const double nb = sqrt(v[0]);
    c->nb = nb;
    c->tol = tol;
    c->maxit = maxit;
    c->kk[0] = 0;
    c->kk[1] = 0;
    c->k = 0;
    c->ax = -1;
    c->xa = -1;
    c->cont = 0;
    c->status = kStOk;
    c->done = 0;
    const double rel = (nb > 0.0) ? sqrt(v[1]) / nb : 0.0;
    c->relres = rel;
    cb->hist[0] = rel;
    if (is_bad(v[0]) || is_bad(v[1]) || is_bad(rel)) {
        c->status = kStNan;
        c->done = 1;
    } else if (nb == 0.0 || rel <= tol) {
        c->done = 1;
    } else if (maxit <= 0) {
        c->status = kStNoconv;
        c->done = 1;
    }
}

// ---------------------------------------------------------------------------
// k_refine (mixed outer step): x' = x + e (FP64; e is the FP32 correction, or
// absent on the first step), r = b - A x' in FP64, r32 = fl32(r), with
// ||b||^2, ||r||^2, ||r32||^2 partials.  Finalised by k_fin_refine, which
// records the outer residual and initialises the inner solve.
// ---------------------------------------------------------------------------
template <bool ADD_E>
__global__ __launch_bounds__(kBS) void k_refine(DevOp<double> A, const double *__restrict__ x,
                                                const float *__restrict__ e,
                                                double *__restrict__ xnew,
                                                const double *__restrict__ b,
                                                float *__restrict__ r32, Partials P) {
    const int G = gridDim.x, L = logical_block(blockIdx.x, G);
    auto xv = [&](int k) { return ADD_E ? x[k] + (double)e[k] : x[k]; };
    double bb = 0.0, rr = 0.0, r2 = 0.0;
    int c0, c1;
    range_of(L, G, A.n, c0, c1);
    for (int base = c0 + threadIdx.x; base < c1 + (int)threadIdx.x; base += kStep) {
#pragma unroll
        for (int u = 0; u < kCPT; u++) {
            const int k = base + u * kBS;
            if (k < c1) {
                const Nbr<double> m = neighbours(A, k);
                const double own = xv(k);
                const double y = apply_row(m, xv(m.kS), xv(m.kW), own, xv(m.kE), xv(m.kN));
                const double bk = b[k];
                const double rk = bk - y;
                const float rf = (float)rk;
                if (ADD_E) xnew[k] = own;
                r32[k] = rf;
                bb += bk * bk;
                rr += rk * rk;
                r2 += (double)rf * (double)rf;
            }
        }
    }
    double pv[3] = {bb, rr, r2};
    put_partials<3>(pv, P.res, L);
}

// keep (mixed solve with the direction kept across corrections): the inner
// run stops at max(inner_tol, outer_tol / rel) relative to ||fl32(r)||, rel
// = ||r|| / ||b||, and nothing runs (done) once rel <= outer_tol.  cont: the
// run continues the last one; its first beta divides by that run's last
// rho, formed at its iteration K-1 (K = c->k iterations) and stored in
// rho[(K-1) & 1], which is moved to rho[1], the slot read at iteration 0.
static __global__ __launch_bounds__(kBS) void k_fin_refine(CtlBlock *cb, Partials P, int g,
                                                           double inner_tol, int inner_maxit,
                                                           int keep, int cont, double outer_tol) {
    double v[3];
    sum_partials<3>(P.res, g, v);
    if (threadIdx.x != 0) return;
    Ctl *c = &cb->c;
    c->bb = v[0];
    c->rr_true = v[1];
    c->inner_nb2 = v[2];
    c->nb = sqrt(v[2]);
    double itol = inner_tol;
    bool outer_done = false;
    if (keep) {
        const double rel = sqrt(v[1]) / sqrt(v[0]);
        outer_done = rel <= outer_tol;
        if (rel > 0.0 && outer_tol / rel > itol) itol = outer_tol / rel;
    }
    if (cont && c->k > 0 && (c->k & 1)) c->rho[1] = c->rho[0];
    c->cont = cont ? 1 : 0;
    c->tol = itol;
    c->maxit = inner_maxit;
    c->kk[0] = 0;
    c->kk[1] = 0;
    c->k = 0;
    c->ax = -1;
    c->xa = -1;
    c->status = kStOk;
    c->relres = 1.0;
    cb->hist[0] = 1.0;
    c->done = (v[2] > 0.0 && !outer_done) ? 0 : 1;
    if (is_bad(v[0]) || is_bad(v[1]) || is_bad(v[2])) {
        c->status = kStNan;
        c->done = 1;
    }
}

// y = A x in FP64 (single step, for tests).
static __global__ __launch_bounds__(kBS) void k_apply_a(DevOp<double> A, const double *__restrict__ x,
                                                 double *__restrict__ y) {
    for (int k = blockIdx.x * kBS + threadIdx.x; k < A.n; k += gridDim.x * kBS) {
        const Nbr<double> m = neighbours(A, k);
        y[k] = apply_row(m, x[m.kS], x[m.kW], x[k], x[m.kE], x[m.kN]);
    }
}

// v = 0 (a fill kernel rather than a memset, so that it is an ordinary node
// when the caller captures the stream).
// The x += alpha d of a solve's last iteration when the stencil that would
// have applied it did not run (the solve stopped): pending when the last
// alpha formed (iteration ax) is newer than the last update applied (xa).
// d_new of iteration k is in d[(k & 1) ^ 1].
template <typename T>
__global__ __launch_bounds__(kBS) void k_x_pending(int n, T *__restrict__ x, const T *__restrict__ d0,
                                                   const T *__restrict__ d1, const CtlBlock *cb) {
    const Ctl *c = &cb->c;
    const int ax = c->ax;
    if (ax < 0 || ax <= c->xa) return;
    const T a = (T)c->alpha;
    const T *d = (ax & 1) ? d0 : d1;
    for (int i = blockIdx.x * kBS + threadIdx.x; i < n; i += gridDim.x * kBS) x[i] = fma(a, d[i], x[i]);
}

template <typename T>
__global__ __launch_bounds__(kBS) void k_zero(int n, T *__restrict__ v) {
    for (int k = blockIdx.x * kBS + threadIdx.x; k < n; k += gridDim.x * kBS) v[k] = T(0);
}

inline int zero_grid(int64_t n) {
    const int64_t g = (n + kBS - 1) / kBS;
    return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

template <typename S, typename D>
__global__ __launch_bounds__(kBS) void k_convert(int n, const S *__restrict__ in,
                                                 D *__restrict__ out) {
    for (int k = blockIdx.x * kBS + threadIdx.x; k < n; k += gridDim.x * kBS) out[k] = (D)in[k];
}

}  // namespace pcga
