"""Oracle: plain FP64 CPU reference of the PCG-AINV method (test infrastructure).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The device library never calls into it and it never
calls into the device library; the two share only the seeded inputs of `gen`.

The arithmetic lives in `oracle.c` (plain C, one thread, sequential sums,
-ffp-contract=off); this module only marshals numpy arrays into it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# A different build of the same source may be named here (mutation checks).
_LIB = os.environ.get("PCGA_ORACLE_LIB", os.path.join(_HERE, "liboracle.so"))

OK, NOCONV, EINVAL, EBREAKDOWN, ENOMEM = 0, 1, -1, -2, -3


# Evaluation-order builds of the same source (see oracle.c): the method is the
# same, only the order of the inner products' additions or the fusing of
# multiply-adds differs.  Used to measure rounding sensitivity.
VARIANTS = {
    "reverse": ["-ffp-contract=off", "-DORA_DOT_ORDER=1"],
    "blocked": ["-ffp-contract=off", "-DORA_DOT_ORDER=2"],
    "fused": ["-ffp-contract=fast", "-mfma"],
    "fused_blocked": ["-ffp-contract=fast", "-mfma", "-DORA_DOT_ORDER=2"],
}


def _variant_path(name):
    return os.path.join(_HERE, f"liboracle_{name}.so")


def _compile(out, flags):
    tmp = out + ".tmp"
    subprocess.run(["gcc", "-O2"] + flags + ["-fno-fast-math", "-fPIC", "-shared", "-std=c99",
                                             "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile liboracle.so from oracle.c with gcc (unfused FP64), and the
    evaluation-order builds liboracle_<variant>.so."""
    def stale(path):
        return force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC)
    if stale(_LIB):
        _compile(_LIB, ["-ffp-contract=off"])
    for name, flags in VARIANTS.items():
        if stale(_variant_path(name)):
            _compile(_variant_path(name), flags)
    return _LIB


_lib = None

_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_int = ctypes.c_int


_variant_libs = {}


def lib(variant=None):
    """The default build, or the evaluation-order build `variant`."""
    global _lib
    if variant is not None:
        if variant not in VARIANTS:
            raise ValueError(f"unknown oracle build {variant!r}")
        if variant not in _variant_libs:
            path = _variant_path(variant)
            if not os.path.exists(path):
                build(force=False)
            _variant_libs[variant] = _declare(ctypes.CDLL(path))
        return _variant_libs[variant]
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _declare(ctypes.CDLL(_LIB))
    return _lib


def _declare(L):
    """Argument and result types of the entry points."""
    L.ora_spmv.argtypes = [_i64, _i64, _int, _p, _p, _p, _p, _p]
    L.ora_spmv.restype = None
    L.ora_ainv_setup.argtypes = [_i64, _i64, _int, _p, _p, _p, _dbl,
                                 ctypes.POINTER(_p), ctypes.POINTER(_i64),
                                 ctypes.POINTER(_i64)]
    L.ora_ainv_setup.restype = _int
    L.ora_ainv_setup_fill.argtypes = [_i64, _i64, _int, _p, _p, _p, _dbl, _i64,
                                      ctypes.POINTER(_p), ctypes.POINTER(_i64),
                                      ctypes.POINTER(_i64)]
    L.ora_ainv_setup_fill.restype = _int
    L.ora_ainv_export.argtypes = [_p, _p, _p, _p, _p]
    L.ora_ainv_export.restype = None
    L.ora_ainv_free.argtypes = [_p]
    L.ora_ainv_free.restype = None
    L.ora_zt_apply.argtypes = [_i64, _p, _p, _p, _p, _p, _p]
    L.ora_zt_apply.restype = None
    L.ora_z_apply.argtypes = [_i64, _p, _p, _p, _p, _p]
    L.ora_z_apply.restype = None
    L.ora_prec_apply.argtypes = [_i64, _p, _p, _p, _p, _p, _p, _p]
    L.ora_prec_apply.restype = None
    L.ora_pcg.argtypes = [_i64, _i64, _int, _p, _p, _p, _p, _p, _p, _p, _p, _p,
                          _dbl, _i64, ctypes.POINTER(_i64), _p, _p, _p]
    L.ora_pcg.restype = _int
    L.ora_csr_spmv.argtypes = [_i64, _p, _p, _p, _p, _p]
    L.ora_csr_spmv.restype = None
    L.ora_ainv_setup_csr.argtypes = [_i64, _p, _p, _p, _dbl, _i64, ctypes.POINTER(_p),
                                     ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
    L.ora_ainv_setup_csr.restype = _int
    L.ora_pcg_csr.argtypes = [_i64, _p, _p, _p, _p, _p, _p, _p, _p, _p, _dbl, _i64,
                              ctypes.POINTER(_i64), _p, _p, _p]
    L.ora_pcg_csr.restype = _int
    L.ora_pcg_mixed.argtypes = [_i64, _i64, _int, _p, _p, _p, _p, _p, _p, _p, _p,
                                _p, _dbl, _dbl, _i64, _i64, ctypes.POINTER(_i64),
                                ctypes.POINTER(_i64), _p]
    L.ora_pcg_mixed.restype = _int
    L.ora_pcg_mixed_ex.argtypes = L.ora_pcg_mixed.argtypes + [_int]
    L.ora_pcg_mixed_ex.restype = _int
    L.ora_pcg_mixed_opt.argtypes = L.ora_pcg_mixed.argtypes + [_int, _int]
    L.ora_pcg_mixed_opt.restype = _int
    L.ora_spmv32.argtypes = [_i64, _i64, _int, _p, _p, _p, _p, _p, _int]
    L.ora_spmv32.restype = None
    L.ora_fsai_band.argtypes = [_i64, _i64, _int, _p, _p, _p, _i64, _p, _p]
    L.ora_fsai_band.restype = _int
    L.ora_ts_rhs.argtypes = [_i64, _i64, _int, _p, _p, _p, _p, _p]
    L.ora_ts_rhs.restype = None
    L.ora_ts_eta.argtypes = [_i64, _p, _p, _dbl, _p]
    L.ora_ts_eta.restype = None
    L.ora_ts_guess.argtypes = [_i64, _p, _p, _dbl, _dbl, _p]
    L.ora_ts_guess.restype = None
    return L


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"oracle status {status} {msg}")
        self.status = status


class AInv:
    """Z (strict upper part, CSC: colptr/rowidx/val, rows ascending) and D."""

    def __init__(self, n, colptr, rowidx, val, D):
        self.n = n
        self.colptr = colptr
        self.rowidx = rowidx
        self.val = val
        self.D = D

    @property
    def nnz_off(self) -> int:
        return int(self.colptr[-1])

    def dense_z(self) -> np.ndarray:
        Z = np.eye(self.n)
        for j in range(self.n):
            for a in range(self.colptr[j], self.colptr[j + 1]):
                Z[self.rowidx[a], j] = self.val[a]
        return Z


def _is_csr(p):
    return hasattr(p, "rowptr")


def _i64a(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def spmv(p, x):
    """y = A x, rows summed in increasing column order (five-point or CSR)."""
    x = _f64(x)
    y = np.empty_like(x)
    if _is_csr(p):
        lib().ora_csr_spmv(p.n, _ptr(_i64a(p.rowptr)), _ptr(_i64a(p.col)), _ptr(_f64(p.val)),
                           _ptr(x), _ptr(y))
        return y
    lib().ora_spmv(p.nx, p.ny, int(p.periodic), _ptr(_f64(p.diag)), _ptr(_f64(p.ae)),
                   _ptr(_f64(p.an)), _ptr(x), _ptr(y))
    return y


def ainv_setup(p, tau, fill=None) -> AInv:
    """AINV by A-orthogonalisation with drop tolerance tau (tau=inf: Jacobi).

    fill: at most this many off-diagonal entries per column of Z, the ones of
    largest magnitude (the fixed-fill Bridson class of Sec. 5); None: no cap."""
    L = lib()
    h = ctypes.c_void_p()
    nnz = ctypes.c_int64()
    brow = ctypes.c_int64()
    if _is_csr(p):
        rp, cl, vl = _i64a(p.rowptr), _i64a(p.col), _f64(p.val)
        st = L.ora_ainv_setup_csr(p.n, _ptr(rp), _ptr(cl), _ptr(vl), float(tau),
                                  -1 if fill is None else int(fill), ctypes.byref(h),
                                  ctypes.byref(nnz), ctypes.byref(brow))
        if st != OK:
            raise OracleError(st, f"(breakdown row {brow.value})")
        return _export(L, h, p.n, nnz.value)
    diag, ae, an = _f64(p.diag), _f64(p.ae), _f64(p.an)
    if fill is None:
        st = L.ora_ainv_setup(p.nx, p.ny, int(p.periodic), _ptr(diag), _ptr(ae), _ptr(an),
                              float(tau), ctypes.byref(h), ctypes.byref(nnz), ctypes.byref(brow))
    else:
        if int(fill) < 0:
            raise ValueError("fill must be >= 0")
        st = L.ora_ainv_setup_fill(p.nx, p.ny, int(p.periodic), _ptr(diag), _ptr(ae),
                                   _ptr(an), float(tau), int(fill), ctypes.byref(h),
                                   ctypes.byref(nnz), ctypes.byref(brow))
    if st != OK:
        raise OracleError(st, f"(breakdown row {brow.value})")
    return _export(L, h, p.nx * p.ny, nnz.value)


def _export(L, h, n, nnz):
    colptr = np.empty(n + 1, dtype=np.int64)
    rowidx = np.empty(max(nnz, 1), dtype=np.int64)
    val = np.empty(max(nnz, 1), dtype=np.float64)
    D = np.empty(n, dtype=np.float64)
    L.ora_ainv_export(h, _ptr(colptr), _ptr(rowidx), _ptr(val), _ptr(D))
    L.ora_ainv_free(h)
    return AInv(n, colptr, rowidx[:nnz], val[:nnz], D)


def zt_apply(F: AInv, r):
    r = _f64(r)
    t = np.empty_like(r)
    lib().ora_zt_apply(F.n, _ptr(F.colptr), _ptr(F.rowidx), _ptr(F.val), _ptr(F.D),
                       _ptr(r), _ptr(t))
    return t


def z_apply(F: AInv, t):
    t = _f64(t)
    s = np.empty_like(t)
    lib().ora_z_apply(F.n, _ptr(F.colptr), _ptr(F.rowidx), _ptr(F.val), _ptr(t), _ptr(s))
    return s


def prec_apply(F: AInv, r):
    r = _f64(r)
    s = np.empty_like(r)
    tmp = np.empty_like(r)
    lib().ora_prec_apply(F.n, _ptr(F.colptr), _ptr(F.rowidx), _ptr(F.val), _ptr(F.D),
                         _ptr(r), _ptr(s), _ptr(tmp))
    return s


class PCGResult:
    def __init__(self, x, iters, hist, status, alphas=None, betas=None):
        self.x = x
        self.iters = iters
        self.hist = hist
        self.status = status
        self.alphas = alphas
        self.betas = betas


def pcg(p, F: AInv, b=None, x0=None, tol=1e-10, maxit=None, scalars=False,
        variant=None) -> PCGResult:
    """Algorithm 1 in FP64.  Returns x, iteration count and residual history.
    variant: run an evaluation-order build (VARIANTS) instead of the default."""
    n = p.n
    b = _f64(p.b if b is None else b)
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    maxit = n if maxit is None else int(maxit)
    hist = np.zeros(maxit + 1)
    it = ctypes.c_int64()
    al = np.zeros(max(maxit, 1)) if scalars else None
    be = np.zeros(max(maxit, 1)) if scalars else None
    tail = (_ptr(F.colptr), _ptr(F.rowidx), _ptr(F.val), _ptr(F.D), _ptr(b), _ptr(x),
            float(tol), maxit, ctypes.byref(it), _ptr(hist), _ptr(al) if scalars else None,
            _ptr(be) if scalars else None)
    if _is_csr(p):
        rp, cl, vl = _i64a(p.rowptr), _i64a(p.col), _f64(p.val)
        st = lib(variant).ora_pcg_csr(p.n, _ptr(rp), _ptr(cl), _ptr(vl), *tail)
    else:
        st = lib(variant).ora_pcg(p.nx, p.ny, int(p.periodic), _ptr(_f64(p.diag)),
                                  _ptr(_f64(p.ae)), _ptr(_f64(p.an)), *tail)
    if st < 0:
        raise OracleError(st)
    k = it.value
    return PCGResult(x, k, hist[: k + 1].copy(), st,
                     al[:k].copy() if scalars else None,
                     be[: max(k - 1, 0)].copy() if scalars else None)


def stop_window(p, F: AInv, b=None, x0=None, tol=1e-10):
    """Stopping iterations of Algorithm 1 under the default build and every
    evaluation-order build: {build: iterations}, with None for the default.
    Their spread is what rounding order alone does to the stopping test."""
    out = {None: pcg(p, F, b=b, x0=x0, tol=tol).iters}
    for v in VARIANTS:
        out[v] = pcg(p, F, b=b, x0=x0, tol=tol, variant=v).iters
    return out


class MixedResult:
    def __init__(self, x, outer, inner_total, outer_hist, status):
        self.x = x
        self.outer = outer
        self.inner_total = inner_total
        self.outer_hist = outer_hist
        self.status = status


def spmv32(p, x, a32=False):
    """q = A d of the mixed form's inner solve on float32 x: FP64 coefficients
    summed in FP64 and rounded (a32 False), or coefficients and sums in FP32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty_like(x)
    lib().ora_spmv32(p.nx, p.ny, int(p.periodic), _ptr(_f64(p.diag)), _ptr(_f64(p.ae)),
                     _ptr(_f64(p.an)), _ptr(x), _ptr(y), int(bool(a32)))
    return y


def pcg_mixed(p, F: AInv, b=None, x0=None, tol=1e-10, inner_tol=1e-5, max_outer=30,
              inner_maxit=None, a32=False, keep=False) -> MixedResult:
    """FP64 refinement around an FP32 inner PCG (FP64 scalars).  a32: the
    inner operator in FP32 as well (coefficients rounded, sums in FP32).
    keep: the inner direction is kept across corrections (reliable updates);
    inner_tol is then the residual reduction of one segment."""
    n = p.nx * p.ny
    b = _f64(p.b if b is None else b)
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    inner_maxit = n if inner_maxit is None else int(inner_maxit)
    hist = np.zeros(max_outer + 1)
    o = ctypes.c_int64()
    tot = ctypes.c_int64()
    st = lib().ora_pcg_mixed_opt(p.nx, p.ny, int(p.periodic), _ptr(_f64(p.diag)),
                              _ptr(_f64(p.ae)), _ptr(_f64(p.an)), _ptr(F.colptr),
                              _ptr(F.rowidx), _ptr(F.val), _ptr(F.D), _ptr(b), _ptr(x),
                              float(tol), float(inner_tol), int(max_outer), inner_maxit,
                              ctypes.byref(o), ctypes.byref(tot), _ptr(hist), int(bool(a32)),
                              int(bool(keep)))
    if st < 0:
        raise OracleError(st)
    return MixedResult(x, o.value, tot.value, hist[: o.value + 1].copy(), st)


def fsai_band(p, q):
    """The paper's banded factor of T (|col-row|<=1 part of A), band q."""
    n = p.nx * p.ny
    zb = np.zeros(n * max(q, 1))
    D = np.zeros(n)
    st = lib().ora_fsai_band(p.nx, p.ny, int(p.periodic), _ptr(_f64(p.diag)),
                             _ptr(_f64(p.ae)), _ptr(_f64(p.an)), int(q), _ptr(zb), _ptr(D))
    if st != OK:
        raise OracleError(st)
    # convert to CSC AInv (drop structural zeros outside the matrix)
    colptr = np.zeros(n + 1, dtype=np.int64)
    rows, vals = [], []
    for j in range(n):
        for m in range(q - 1, -1, -1):         # rows ascending: j-q .. j-1
            r = j - 1 - m
            if r >= 0:
                v = zb[j * q + (q - 1 - m)]
                if v != 0.0:
                    rows.append(r)
                    vals.append(v)
        colptr[j + 1] = len(rows)
    return AInv(n, colptr, np.array(rows, dtype=np.int64), np.array(vals), D), zb


# --- the time step around the solve (eq. (1), eq. (8), Algorithm 1's first guess)

def ts_rhs(nx, ny, periodic, e2u, mu, e1v, mv):
    """b = -(delta_i(e2 Mu) - delta_j(e1 Mv)) (eq. (8); the solved system is the
    negation of eq. (10)).  Face arrays are indexed by the cell west / south of
    the face; see oracle.c for the closed faces."""
    n = nx * ny
    arrs = [_f64(a) for a in (e2u, mu, e1v, mv)]
    for a in arrs:
        if a.shape != (n,):
            raise ValueError("face arrays must have shape (nx*ny,)")
    b = np.empty(n)
    lib().ora_ts_rhs(nx, ny, int(bool(periodic)), *[_ptr(a) for a in arrs], _ptr(b))
    return b


def ts_eta(eta_prev, D, dt):
    """eta^{n+1} = eta^{n-1} - 2 dt D^n (eq. (1))."""
    e, d = _f64(eta_prev), _f64(D)
    out = np.empty_like(e)
    lib().ora_ts_eta(e.shape[0], _ptr(e), _ptr(d), float(dt), _ptr(out))
    return out


def ts_guess(D1, D2, a, c):
    """x0 = a D^{t-1} + c D^{t-2} (the second term left out when c = 0)."""
    d1 = _f64(D1)
    d2 = _f64(D2) if D2 is not None else np.zeros_like(d1)
    out = np.empty_like(d1)
    lib().ora_ts_guess(d1.shape[0], _ptr(d1), _ptr(d2), float(a), float(c), _ptr(out))
    return out
