// kernels.h -- gfx950 kernels of one PCG-AINV iteration and its prologue.
//
// One iteration of Algorithm 1 (with the preconditioned direction update
// d = s + beta d) is three launches, each streaming its arrays once and
// ending in a deterministic grid reduction finished by the last workgroup:
//
//   k_stencil  d_new = s + beta d_old;  q = A d_new;  (d_new, q)  -> alpha
//   k_zt       r' = r - alpha q;  x += alpha d_new;  ||r'||^2;
//              t = D^-1 Z^T r'    (r' is recomputed at the gathered rows)
//                                                         -> stop test, history
//   k_z        s = Z t;  (s, r')                               -> rho, beta
//
// The three global dependencies of the method (alpha needs all of (d,q); the
// Z^T gather needs r' at other rows; beta needs all of (s,r)) are exactly the
// kernel boundaries.  d and r are double-buffered because neighbouring
// workgroups read the old values while others write the new ones.
//
// Work split: a launch of G workgroups assigns each workgroup one contiguous
// range of tiles (stencil) or slices (sliced ELL).  Workgroups are dispatched
// round-robin over the 8 XCDs, so the hardware index is remapped to make the
// ranges of one XCD contiguous: grid neighbours (the rows above and below,
// and the rows a Z column reaches) then live in the same L2.
//
// Reductions: FP64 per-lane sums, a fixed butterfly per wavefront, a fixed
// order over the 4 wavefronts, per-workgroup partials, and a fixed strided
// order in the last workgroup.  Results are bitwise reproducible for a given
// launch shape.
#pragma once

#include <hip/hip_runtime.h>

#include "pcga_dev.h"

namespace pcga {

enum : int { kStOk = 0, kStNoconv = 1, kStBreak = -2, kStNan = -3 };

__device__ __forceinline__ int logical_block(int b, int G) {
    const int q = G >> 3, rem = G & 7, x = b & 7, i = b >> 3;
    return x * q + (x < rem ? x : rem) + i;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum NV values over the workgroup; the totals are valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
    __shared__ double red[NV][kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < NV; q++) {
        const double s = wave_sum(v[q]);
        if (lane == 0) red[q][w] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; q++) v[q] = ((red[q][0] + red[q][1]) + red[q][2]) + red[q][3];
    }
    __syncthreads();
}

// Publish this workgroup's sums; the last workgroup to arrive reduces all
// partials (fixed order) and returns true with the totals in v (thread 0).
template <int NV>
__device__ bool grid_finish(double (&v)[NV], double *partials, int G, int L, uint32_t *cnt) {
    __shared__ int is_last;
    block_sum<NV>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; q++) partials[q * kMaxBlocks + L] = v[q];
        __threadfence();
        const uint32_t prev = atomicAdd(cnt, 1u);
        is_last = (prev == (uint32_t)(G - 1));
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) acc[q] = 0.0;
    for (int b = threadIdx.x; b < G; b += kBlock) {
#pragma unroll
        for (int q = 0; q < NV; q++) acc[q] += partials[q * kMaxBlocks + b];
    }
    block_sum<NV>(acc);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; q++) v[q] = acc[q];
        *cnt = 0u;
    }
    return true;
}

// One 256-cell tile of the five-point product y = A v, where v(k) is a value
// provider (it may combine several arrays on the fly).  East/west neighbours
// come from LDS (row interior) or from v (periodic wrap); north/south from v.
// Terms are added in increasing column order (south, west, self, east, north).
template <typename T, typename V>
__device__ __forceinline__ void stencil_tile(const DevOp<T> &A, int k0, const V &v, T *sh,
                                             T &own, T &y, bool &valid) {
    const int tid = threadIdx.x;
    const int k = k0 + tid;
    const int n = A.n, nx = A.nx;
    valid = k < n;
    own = valid ? v(k) : T(0);
    sh[tid + 1] = own;
    if (tid == 0) sh[0] = (k0 > 0) ? v(k0 - 1) : T(0);
    if (tid == kBlock - 1) sh[kBlock + 1] = (k0 + kBlock < n) ? v(k0 + kBlock) : T(0);
    __syncthreads();
    T acc = T(0);
    if (valid) {
        const int j = k / nx;
        const int i = k - j * nx;
        if (j > 0) acc = A.an[k - nx] * v(k - nx);
        if (i > 0) acc = fma(A.ae[k - 1], sh[tid], acc);
        else if (A.periodic) acc = fma(A.ae[k + nx - 1], v(k + nx - 1), acc);
        acc = fma(A.diag[k], own, acc);
        if (i < nx - 1) acc = fma(A.ae[k], sh[tid + 2], acc);
        else if (A.periodic) acc = fma(A.ae[k], v(k - nx + 1), acc);
        if (j < A.ny - 1) acc = fma(A.an[k], v(k + nx), acc);
    }
    y = acc;
    __syncthreads();
}

__device__ __forceinline__ void tile_range(int L, int G, int ntiles, int &t0, int &t1) {
    t0 = (int)(((int64_t)L * ntiles) / G);
    t1 = (int)(((int64_t)(L + 1) * ntiles) / G);
}

// ---------------------------------------------------------------------------
// k_stencil: d_new = s + beta*d_old; q = A d_new; (d_new, q) -> alpha = rho/(d,q)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_stencil(DevOp<T> A, const T *__restrict__ s,
                                                    const T *__restrict__ dold,
                                                    T *__restrict__ dnew, T *__restrict__ q,
                                                    CtlBlock *cb, double *partials, int ntiles) {
    Ctl *c = &cb->c;
    if (c->done) return;
    const int G = gridDim.x, L = logical_block(blockIdx.x, G);
    const T beta = (T)c->beta;
    __shared__ T sh[kBlock + 2];
    auto val = [&](int k) { return fma(beta, dold[k], s[k]); };
    double acc = 0.0;
    int t0, t1;
    tile_range(L, G, ntiles, t0, t1);
    for (int t = t0; t < t1; t++) {
        T own, y;
        bool valid;
        stencil_tile(A, t * kBlock, val, sh, own, y, valid);
        if (valid) {
            const int k = t * kBlock + threadIdx.x;
            dnew[k] = own;
            q[k] = y;
            acc += (double)own * (double)y;
        }
    }
    double v[1] = {acc};
    if (grid_finish<1>(v, partials, G, L, &c->cnt[kCntStencil]) && threadIdx.x == 0) {
        const double dq = v[0];
        if (dq > 0.0 && dq < INFINITY) {
            c->alpha = c->rho / dq;
        } else {
            c->status = (dq == dq && dq != INFINITY) ? kStBreak : kStNan;
            c->done = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// k_zt: t = D^-1 Z^T r'.  FUSED: r' = r - alpha q (written to rnext),
// x += alpha d, ||r'||^2 -> stop test and history.  Not fused: r' = r.
// Each wavefront handles slices of the sliced-ELL layout of Z^T (rows of Z^T
// are the columns of Z; the unit diagonal is added last).
// ---------------------------------------------------------------------------
template <typename T, bool FUSED>
__global__ __launch_bounds__(kBlock) void k_zt(DevSell<T> Zt, const T *__restrict__ dinv,
                                               const T *__restrict__ rcur,
                                               const T *__restrict__ q,
                                               const T *__restrict__ dcur,
                                               T *__restrict__ rnext, T *__restrict__ x,
                                               T *__restrict__ t, CtlBlock *cb,
                                               double *partials) {
    Ctl *c = &cb->c;
    if (FUSED && c->done) return;
    const int G = gridDim.x, L = logical_block(blockIdx.x, G);
    const T at = FUSED ? (T)c->alpha : T(0);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int s0, s1;
    tile_range(L, G, Zt.nslices, s0, s1);
    double rr = 0.0;
    for (int sl = s0 + w; sl < s1; sl += kBlock / kWave) {
        const int row0 = Zt.row0[sl];
        const int meta = Zt.meta[sl];
        const int64_t off = Zt.off[sl];
        const int lg = meta & 255, width = meta >> 8;
        const int row = row0 + (lane >> lg);
        const int32_t *ip = Zt.idx + off + lane;
        const T *vp = Zt.val + off + lane;
        T acc = T(0);
        for (int cc = 0; cc < width; cc++) {
            const int kk = ip[(int64_t)cc * kWave];
            const T zv = vp[(int64_t)cc * kWave];
            const T rk = FUSED ? fma(-at, q[kk], rcur[kk]) : rcur[kk];
            acc = fma(zv, rk, acc);
        }
        for (int o = (1 << lg) >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
        if ((lane & ((1 << lg) - 1)) == 0 && row < Zt.nrows) {
            const T rj = FUSED ? fma(-at, q[row], rcur[row]) : rcur[row];
            if (FUSED) {
                rnext[row] = rj;
                x[row] = fma(at, dcur[row], x[row]);
                rr += (double)rj * (double)rj;
            }
            t[row] = (acc + rj) * dinv[row];
        }
    }
    if (!FUSED) return;
    double v[1] = {rr};
    if (grid_finish<1>(v, partials, G, L, &c->cnt[kCntZt]) && threadIdx.x == 0) {
        const double rel = sqrt(v[0]) / c->nb;
        const int k = c->k + 1;
        c->k = k;
        c->relres = rel;
        cb->hist[k & (kHistRing - 1)] = rel;
        if (!(rel == rel) || rel == INFINITY) {
            c->status = kStNan;
            c->done = 1;
        } else if (rel <= c->tol) {
            c->status = kStOk;
            c->done = 1;
        } else if (k >= c->maxit) {
            c->status = kStNoconv;
            c->done = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// k_z: s = Z t (unit diagonal implicit); DOT: (s, r) -> rho, beta.
// FIRST (prologue): rho = (s0, r0), beta = 0 so that d0 = s0.
// ---------------------------------------------------------------------------
template <typename T, bool DOT, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_z(DevSell<T> Z, const T *__restrict__ t,
                                              const T *__restrict__ r, T *__restrict__ s,
                                              CtlBlock *cb, double *partials) {
    Ctl *c = &cb->c;
    if (DOT && c->done) return;
    const int G = gridDim.x, L = logical_block(blockIdx.x, G);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int s0, s1;
    tile_range(L, G, Z.nslices, s0, s1);
    double sr = 0.0;
    for (int sl = s0 + w; sl < s1; sl += kBlock / kWave) {
        const int row0 = Z.row0[sl];
        const int meta = Z.meta[sl];
        const int64_t off = Z.off[sl];
        const int lg = meta & 255, width = meta >> 8;
        const int row = row0 + (lane >> lg);
        const int32_t *ip = Z.idx + off + lane;
        const T *vp = Z.val + off + lane;
        T acc = T(0);
        for (int cc = 0; cc < width; cc++) {
            const int jj = ip[(int64_t)cc * kWave];
            acc = fma(vp[(int64_t)cc * kWave], t[jj], acc);
        }
        for (int o = (1 << lg) >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
        if ((lane & ((1 << lg) - 1)) == 0 && row < Z.nrows) {
            const T sk = t[row] + acc;
            s[row] = sk;
            if (DOT) sr += (double)sk * (double)r[row];
        }
    }
    if (!DOT) return;
    double v[1] = {sr};
    if (grid_finish<1>(v, partials, G, L, &c->cnt[kCntZ]) && threadIdx.x == 0) {
        const double rn = v[0];
        if (rn > 0.0 && rn < INFINITY) {
            c->beta = FIRST ? 0.0 : rn / c->rho;
            c->rho = rn;
        } else {
            c->status = (rn == rn && rn != INFINITY) ? kStBreak : kStNan;
            c->done = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// k_residual (FP64): r = b - A x with ||b||^2 and ||r||^2.
// MODE 0 (solve prologue): writes r, sets nb, tol, maxit, k = 0, hist[0],
//   and done when ||b|| = 0, the start is converged, or maxit = 0.
// MODE 1 (true residual): only the norms (bb, rr_true).
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_residual(DevOp<double> A, const double *__restrict__ x,
                                                     const double *__restrict__ b,
                                                     double *__restrict__ r, CtlBlock *cb,
                                                     double *partials, int ntiles, double tol,
                                                     int maxit) {
    Ctl *c = &cb->c;
    const int G = gridDim.x, L = logical_block(blockIdx.x, G);
    __shared__ double sh[kBlock + 2];
    auto val = [&](int k) { return x[k]; };
    double bb = 0.0, rr = 0.0;
    int t0, t1;
    tile_range(L, G, ntiles, t0, t1);
    for (int t = t0; t < t1; t++) {
        double own, y;
        bool valid;
        stencil_tile(A, t * kBlock, val, sh, own, y, valid);
        if (valid) {
            const int k = t * kBlock + threadIdx.x;
            const double bk = b[k];
            const double rk = bk - y;
            if (MODE == 0) r[k] = rk;
            bb += bk * bk;
            rr += rk * rk;
        }
    }
    double v[2] = {bb, rr};
    if (grid_finish<2>(v, partials, G, L, &c->cnt[kCntResid]) && threadIdx.x == 0) {
        c->bb = v[0];
        if (MODE == 0) {
            const double nb = sqrt(v[0]);
            c->nb = nb;
            c->tol = tol;
            c->maxit = maxit;
            c->k = 0;
            c->status = kStOk;
            c->done = 0;
            c->beta = 0.0;
            const double rel = (nb > 0.0) ? sqrt(v[1]) / nb : 0.0;
            c->relres = rel;
            cb->hist[0] = rel;
            if (!(rel == rel) || rel == INFINITY) {
                c->status = kStNan;
                c->done = 1;
            } else if (nb == 0.0 || rel <= tol) {
                c->done = 1;
            } else if (maxit <= 0) {
                c->status = kStNoconv;
                c->done = 1;
            }
        } else {
            c->rr_true = v[1];
        }
    }
}

// ---------------------------------------------------------------------------
// k_refine (mixed outer step): x' = x + e (FP64; e is the FP32 correction, or
// absent on the first step), r = b - A x' in FP64, r32 = fl32(r).
// Norms: ||b||^2, ||r||^2, ||r32||^2.  The last workgroup records the outer
// residual and initialises the inner solve (nb = ||r32||, k = 0, hist[0] = 1).
// ---------------------------------------------------------------------------
template <bool ADD_E>
__global__ __launch_bounds__(kBlock) void k_refine(DevOp<double> A, const double *__restrict__ x,
                                                   const float *__restrict__ e,
                                                   double *__restrict__ xnew,
                                                   const double *__restrict__ b,
                                                   float *__restrict__ r32, CtlBlock *cb,
                                                   double *partials, int ntiles,
                                                   double inner_tol, int inner_maxit) {
    Ctl *c = &cb->c;
    const int G = gridDim.x, L = logical_block(blockIdx.x, G);
    __shared__ double sh[kBlock + 2];
    auto val = [&](int k) { return ADD_E ? x[k] + (double)e[k] : x[k]; };
    double bb = 0.0, rr = 0.0, r2 = 0.0;
    int t0, t1;
    tile_range(L, G, ntiles, t0, t1);
    for (int t = t0; t < t1; t++) {
        double own, y;
        bool valid;
        stencil_tile(A, t * kBlock, val, sh, own, y, valid);
        if (valid) {
            const int k = t * kBlock + threadIdx.x;
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
    double v[3] = {bb, rr, r2};
    if (grid_finish<3>(v, partials, G, L, &c->cnt[kCntRefine]) && threadIdx.x == 0) {
        c->bb = v[0];
        c->rr_true = v[1];
        c->inner_nb2 = v[2];
        c->nb = sqrt(v[2]);
        c->tol = inner_tol;
        c->maxit = inner_maxit;
        c->k = 0;
        c->status = kStOk;
        c->beta = 0.0;
        c->relres = 1.0;
        cb->hist[0] = 1.0;
        c->done = (v[2] > 0.0) ? 0 : 1;
        if (!(v[1] == v[1]) || v[1] == INFINITY) {
            c->status = kStNan;
            c->done = 1;
        }
    }
}

// y = A x in FP64 (single step, for tests).
__global__ __launch_bounds__(kBlock) void k_apply_a(DevOp<double> A, const double *__restrict__ x,
                                                    double *__restrict__ y, int ntiles) {
    __shared__ double sh[kBlock + 2];
    auto val = [&](int k) { return x[k]; };
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        double own, yy;
        bool valid;
        stencil_tile(A, t * kBlock, val, sh, own, yy, valid);
        if (valid) y[t * kBlock + threadIdx.x] = yy;
    }
}

template <typename S, typename D>
__global__ __launch_bounds__(kBlock) void k_convert(int n, const S *__restrict__ in,
                                                    D *__restrict__ out) {
    for (int k = blockIdx.x * kBlock + threadIdx.x; k < n; k += gridDim.x * kBlock)
        out[k] = (D)in[k];
}

}  // namespace pcga
