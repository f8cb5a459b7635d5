// timestep.hip -- the time step around the elliptic solve, on the device.
//
// The solve of eq. (10) sits inside the model's sea-surface time step
// (Sec. 2, eq. (1)-(2); Sec. 3, eq. (8)).  Three cell-wise passes on the
// solver's grid and stream:
//
//   pcga_ts_rhs    b = -(delta_i(e2 Mu) - delta_j(e1 Mv))   (eq. (8), negated
//                  like the operator: the system solved is -(eq. (10)))
//   pcga_ts_eta    eta^{n+1} = eta^{n-1} - 2 dt D^n          (eq. (1))
//   pcga_ts_guess  x0 = a D^{t-1} + c D^{t-2}                 (first guess of
//                  Algorithm 1 from earlier solutions)
//
// Each is one HBM-bound pass (the face values a cell needs from its west and
// south neighbours are neighbouring addresses, read through L2).  The
// arithmetic is written out operation by operation with contraction off, so
// that results are bitwise reproducible against a plain FP64 reference.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "pcga_host.h"
#include "solver_internal.h"

namespace pcga {

constexpr int kTsBlock = 256;

static int ts_grid(int64_t n) { return (int)std::min<int64_t>(4096, (n + kTsBlock - 1) / kTsBlock); }

// Face values are stored at the cell west (east faces) or south (north faces)
// of the face.  Closed faces: the west face of i = 0 without periodicity (with
// it, the east face of i = nx-1), the east face of i = nx-1 without
// periodicity, the south face of j = 0 and the north face of j = ny-1.
static __global__ __launch_bounds__(kTsBlock) void k_ts_rhs(int nx, int ny, int periodic,
                                                    const double *__restrict__ e2u,
                                                    const double *__restrict__ mu,
                                                    const double *__restrict__ e1v,
                                                    const double *__restrict__ mv,
                                                    double *__restrict__ b) {
#pragma clang fp contract(off)
    // contiguous cell ranges, consecutive on each XCD: the west and south
    // face values a cell reads were, mostly, fetched by a workgroup of the
    // same XCD (its L2)
    const int n = nx * ny;
    int c0, c1;
    range_of(logical_block(blockIdx.x, gridDim.x), gridDim.x, n, c0, c1);
    for (int k = c0 + threadIdx.x; k < c1; k += kTsBlock) {
        const int j = k / nx, i = k - j * nx;
        double fe = 0.0, fw = 0.0, fn = 0.0, fs = 0.0;
        if (i < nx - 1 || periodic) fe = e2u[k] * mu[k];
        if (i > 0)
            fw = e2u[k - 1] * mu[k - 1];
        else if (periodic)
            fw = e2u[k + nx - 1] * mu[k + nx - 1];
        if (j < ny - 1) fn = e1v[k] * mv[k];
        if (j > 0) fs = e1v[k - nx] * mv[k - nx];
        const double bp = (fe - fw) - (fn - fs);
        b[k] = -bp;
    }
}

// eta_next may alias eta_prev (each cell reads, then writes, its own entry)
static __global__ __launch_bounds__(kTsBlock) void k_ts_eta(int64_t n, const double *eta_prev,
                                                    const double *__restrict__ D, double s,
                                                    double *eta_next) {
#pragma clang fp contract(off)
    for (int64_t k = blockIdx.x * (int64_t)kTsBlock + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * kTsBlock)
        eta_next[k] = eta_prev[k] - s * D[k];
}

// x0 may alias D1 or D2 (each cell reads, then writes, its own entry)
template <bool TWO>
static __global__ __launch_bounds__(kTsBlock) void k_ts_guess(int64_t n, const double *D1,
                                                      const double *D2, double a, double c,
                                                      double *x0) {
#pragma clang fp contract(off)
    for (int64_t k = blockIdx.x * (int64_t)kTsBlock + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * kTsBlock) {
        if (TWO)
            x0[k] = a * D1[k] + c * D2[k];
        else
            x0[k] = a * D1[k];
    }
}

static int launched(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PCGA_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return PCGA_OK;
}

}  // namespace pcga

using namespace pcga;

extern "C" {

int pcga_ts_rhs(pcga_solver_t *S, const double *e2u, const double *mu, const double *e1v,
                const double *mv, double *b) {
    if (!S || !e2u || !mu || !e1v || !mv || !b) return fail(PCGA_EINVAL, "NULL argument");
    if (S->csr) return fail(PCGA_EINVAL, "pcga_ts_rhs needs a five-point (grid) solver");
    if (hipSetDevice(S->device) != hipSuccess) return fail(PCGA_EHIP, "hipSetDevice failed");
    k_ts_rhs<<<ts_grid(S->n), kTsBlock, 0, S->stream>>>(S->nx, S->ny, S->periodic, e2u, mu, e1v,
                                                         mv, b);
    return launched("k_ts_rhs");
}

int pcga_ts_eta(pcga_solver_t *S, const double *eta_prev, const double *D, double dt,
                double *eta_next) {
    if (!S || !eta_prev || !D || !eta_next) return fail(PCGA_EINVAL, "NULL argument");
    if (!(dt >= 0.0) || dt == INFINITY) return fail(PCGA_EINVAL, "dt must be finite and >= 0");
    if (hipSetDevice(S->device) != hipSuccess) return fail(PCGA_EHIP, "hipSetDevice failed");
    const double s = 2.0 * dt;
    k_ts_eta<<<ts_grid(S->n), kTsBlock, 0, S->stream>>>(S->n, eta_prev, D, s, eta_next);
    return launched("k_ts_eta");
}

int pcga_ts_guess(pcga_solver_t *S, const double *D1, const double *D2, double a, double c,
                  double *x0) {
    if (!S || !D1 || !x0 || (c != 0.0 && !D2)) return fail(PCGA_EINVAL, "NULL argument");
    if (hipSetDevice(S->device) != hipSuccess) return fail(PCGA_EHIP, "hipSetDevice failed");
    if (c != 0.0)
        k_ts_guess<true><<<ts_grid(S->n), kTsBlock, 0, S->stream>>>(S->n, D1, D2, a, c, x0);
    else
        k_ts_guess<false><<<ts_grid(S->n), kTsBlock, 0, S->stream>>>(S->n, D1, nullptr, a, c, x0);
    return launched("k_ts_guess");
}

}  // extern "C"
