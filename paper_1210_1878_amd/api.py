"""Python face of the C ABI: the paper's problem statement as calls.

    F = ainv_setup(A, drop_tol)                      # (Z, D), host FP64
    x, iters, hist = pcg_solve(A, F, b, x0, tol, maxit)
    res = pcg_solve_mixed(A, F, b, x0, tol, inner_tol=1e-5, max_outer=...)

`A` is a Stencil5 (host numpy FP64 arrays in A5 form), `b` and `x0` are torch
tensors on a ROCm device.  Torch provides the device memory (the solver's
workspace is one uint8 tensor) and the stream; every step of the solve runs
in the HIP kernels of libpcgainv.so.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np

from . import _lib
from ._lib import FP64, MIXED, MIXED_A32, PERIODIC_X, check

_PRECISIONS = {"fp64": FP64, "mixed": MIXED, "mixed_a32": MIXED_A32}


@dataclasses.dataclass
class Stencil5:
    """Five-point operator in A5 form (see include/pcgainv.h)."""
    nx: int
    ny: int
    periodic: bool
    diag: np.ndarray
    ae: np.ndarray
    an: np.ndarray

    def __post_init__(self):
        n = self.nx * self.ny
        for f in ("diag", "ae", "an"):
            a = np.ascontiguousarray(getattr(self, f), dtype=np.float64)
            if a.shape != (n,):
                raise ValueError(f"{f} must have shape ({n},)")
            setattr(self, f, a)

    @property
    def n(self) -> int:
        return self.nx * self.ny

    @classmethod
    def from_problem(cls, p) -> "Stencil5":
        return cls(p.nx, p.ny, bool(p.periodic), p.diag, p.ae, p.an)

    def c_struct(self) -> _lib.A5:
        return _lib.A5(self.nx, self.ny, PERIODIC_X if self.periodic else 0,
                       self.diag.ctypes.data, self.ae.ctypes.data, self.an.ctypes.data)


@dataclasses.dataclass
class CsrMatrix:
    """General sparse SPD operator in CSR (see pcga_csr_t in include/pcgainv.h):
    rowptr int64[n+1], col int32[nnz] ascending per row, val float64[nnz]."""
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    def __post_init__(self):
        self.rowptr = np.ascontiguousarray(self.rowptr, dtype=np.int64)
        self.col = np.ascontiguousarray(self.col, dtype=np.int32)
        self.val = np.ascontiguousarray(self.val, dtype=np.float64)
        if self.rowptr.shape != (self.n + 1,) or self.col.shape != self.val.shape:
            raise ValueError("CSR arrays do not match n")

    @classmethod
    def from_problem(cls, p) -> "CsrMatrix":
        return cls(int(p.n), p.rowptr, p.col, p.val)

    def c_struct(self) -> _lib.Csr:
        return _lib.Csr(self.n, self.rowptr.ctypes.data, self.col.ctypes.data,
                        self.val.ctypes.data)


class AInv:
    """Handle to (Z, D) computed on the host."""

    def __init__(self, handle, keep=None):
        self._h = handle
        self._keep = keep
        L = _lib.load()
        n = ctypes.c_int64()
        nnz = ctypes.c_int64()
        check(L.pcga_ainv_info(self._h, ctypes.byref(n), ctypes.byref(nnz)), "pcga_ainv_info")
        self.n = n.value
        self.nnz_off = nnz.value

    @property
    def handle(self):
        return self._h

    def export(self):
        """(colptr int64[n+1], rowidx int32[nnz], val float64[nnz], D float64[n])."""
        L = _lib.load()
        colptr = np.empty(self.n + 1, dtype=np.int64)
        rowidx = np.empty(max(self.nnz_off, 1), dtype=np.int32)
        val = np.empty(max(self.nnz_off, 1), dtype=np.float64)
        D = np.empty(self.n, dtype=np.float64)
        check(L.pcga_ainv_export(self._h, colptr.ctypes.data, rowidx.ctypes.data,
                                 val.ctypes.data, D.ctypes.data), "pcga_ainv_export")
        return colptr, rowidx[: self.nnz_off], val[: self.nnz_off], D

    def layout_info(self, slice_width: int = 0) -> dict:
        """Shape of the sliced-ELL layouts a solver would build at this target
        width (host only): per matrix ("zt", "z") the slice count, table
        slices, widest table slice, widest slice, stored entries and index
        bytes."""
        L = _lib.load()
        out = np.zeros(12, dtype=np.int64)
        check(L.pcga_layout_info(self._h, int(slice_width), out.ctypes.data), "pcga_layout_info")
        keys = ("slices", "table_slices", "table_width_max", "width_max", "entries", "index_bytes")
        return {m: {k: int(out[6 * i + j]) for j, k in enumerate(keys)}
                for i, m in enumerate(("zt", "z"))}

    @classmethod
    def from_csc(cls, n, colptr, rowidx, val, D) -> "AInv":
        L = _lib.load()
        colptr = np.ascontiguousarray(colptr, dtype=np.int64)
        rowidx = np.ascontiguousarray(rowidx, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        D = np.ascontiguousarray(D, dtype=np.float64)
        h = ctypes.c_void_p()
        check(L.pcga_ainv_import(int(n), colptr.ctypes.data, rowidx.ctypes.data if len(rowidx) else None,
                                 val.ctypes.data if len(val) else None, D.ctypes.data,
                                 ctypes.byref(h)), "pcga_ainv_import")
        return cls(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                _lib.load().pcga_ainv_free(h)
            except Exception:
                pass
            self._h = None


def ainv_setup(A: Stencil5, drop_tol: float, fill=None) -> AInv:
    """Approximate inverse factor by A-orthogonalisation with a drop tolerance.

    fill: keep at most this many off-diagonal entries in each column of Z, the
    largest in magnitude (the fixed-fill Bridson class of Sec. 5); None: no
    cap."""
    L = _lib.load()
    h = ctypes.c_void_p()
    if isinstance(A, CsrMatrix):
        cs = A.c_struct()
        check(L.pcga_ainv_setup_csr(ctypes.byref(cs), float(drop_tol),
                                    -1 if fill is None else int(fill), ctypes.byref(h)),
              "pcga_ainv_setup_csr")
        return AInv(h)
    a5 = A.c_struct()
    if fill is None:
        check(L.pcga_ainv_setup(ctypes.byref(a5), float(drop_tol), ctypes.byref(h)),
              "pcga_ainv_setup")
    else:
        check(L.pcga_ainv_setup_fill(ctypes.byref(a5), float(drop_tol), int(fill),
                                     ctypes.byref(h)), "pcga_ainv_setup_fill")
    return AInv(h)


def fsai_band_setup(A: Stencil5, q: int) -> AInv:
    """The paper's banded factor of T (Sec. 3 scheme), band q."""
    L = _lib.load()
    h = ctypes.c_void_p()
    a5 = A.c_struct()
    check(L.pcga_fsai_band_setup(ctypes.byref(a5), int(q), ctypes.byref(h)), "pcga_fsai_band_setup")
    return AInv(h)


def _dev_ptr(t, dtype, n):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()
            and t.numel() == n):
        raise ValueError(f"expected a contiguous {dtype} device tensor with {n} elements")
    return ctypes.c_void_p(t.data_ptr())


@dataclasses.dataclass
class SolveResult:
    x: object
    iters: int
    hist: np.ndarray
    status: int
    true_relres: float
    outer: int = 0
    inner_total: int = 0

    def __iter__(self):          # x, iters, hist = pcg_solve(...)
        return iter((self.x, self.iters, self.hist))


WS_ALIGN = 16 << 20     # alignment of a solver's workspace base (bytes)
PROBE_STEP = 4 << 20    # distance between the bases a placement probe tries


def workspace_size(A: Stencil5, F: AInv, precision: str = "fp64", slice_width: int = 0) -> int:
    """Device bytes a Solver of these settings allocates (workspace plus the
    alignment slack)."""
    return _workspace_bytes(A, F, _PRECISIONS[precision],
                            int(slice_width)) + WS_ALIGN


def _workspace_bytes(A, F, precision, slice_width):
    L = _lib.load()
    nbytes = ctypes.c_size_t()
    cs = A.c_struct()
    if isinstance(A, CsrMatrix):
        check(L.pcga_workspace_bytes_csr(ctypes.byref(cs), F.handle, precision, slice_width,
                                         ctypes.byref(nbytes)), "pcga_workspace_bytes_csr")
    else:
        check(L.pcga_workspace_bytes_ex(ctypes.byref(cs), F.handle, precision, slice_width,
                                        ctypes.byref(nbytes)), "pcga_workspace_bytes_ex")
    return nbytes.value


def _create(A, F, precision, slice_width, ws_ptr, ws_bytes, stream_ptr):
    L = _lib.load()
    h = ctypes.c_void_p()
    cs = A.c_struct()
    if isinstance(A, CsrMatrix):
        check(L.pcga_solver_create_csr(ctypes.byref(cs), F.handle, precision, slice_width,
                                       ctypes.c_void_p(ws_ptr), ws_bytes,
                                       ctypes.c_void_p(stream_ptr), ctypes.byref(h)),
              "pcga_solver_create_csr")
    else:
        check(L.pcga_solver_create_ex(ctypes.byref(cs), F.handle, precision, slice_width,
                                      ctypes.c_void_p(ws_ptr), ws_bytes,
                                      ctypes.c_void_p(stream_ptr), ctypes.byref(h)),
              "pcga_solver_create_ex")
    return h


class Solver:
    """Device solver for one grid: A, Z^T/Z (sliced ELL) and D^-1 resident in
    a torch-allocated workspace; FP64 or mixed precision."""

    def __init__(self, A: Stencil5, F: AInv, precision: str = "fp64", device=None, stream=None,
                 slice_width: int = 0, buffer=None, probe_placements: int = 1):
        """buffer: optional uint8 device tensor to carve the workspace from
        (at least workspace_size(...) bytes); solvers built one after another
        on the same buffer sit at the same address, which lets timings of
        different settings be compared.  No other work may be using the
        buffer (an earlier solver on it must be closed and its work finished).

        probe_placements: with k > 1 (and no buffer), the workspace is
        allocated with room for k bases PROBE_STEP apart; the solver is built
        at each, one whole iteration is timed, and the fastest base is kept
        (`placement_ms` lists them).  Setup then costs k + 1 layout uploads."""
        import torch
        L = _lib.load()
        self.A = A
        self.slice_width = int(slice_width)
        self.precision = _PRECISIONS[precision]
        self.device = torch.device("cuda" if device is None else device)
        self.workspace_bytes = _workspace_bytes(A, F, self.precision, self.slice_width)
        with torch.cuda.device(self.device):
            # a stream of its own (default priority): chunks are captured into
            # HIP graphs, which the legacy default stream does not allow
            self.stream = torch.cuda.Stream(self.device) if stream is None else stream
            # the workspace starts on a 16 MiB boundary: at 1442x1021 an FP64
            # iteration took 96-98 us from such a base and 102-106 us from
            # some others (the resident part of the workspace fills most of
            # the 256 MiB memory-side cache, so where it starts matters)
            probes = max(1, int(probe_placements)) if buffer is None else 1
            if buffer is None:
                self._ws_buf = torch.empty(self.workspace_bytes + WS_ALIGN
                                           + (probes - 1) * PROBE_STEP,
                                           dtype=torch.uint8, device=self.device)
            else:
                want = (self.device.index if self.device.index is not None
                        else torch.cuda.current_device())
                if (buffer.dtype != torch.uint8 or buffer.device.type != "cuda"
                        or buffer.device.index != want or not buffer.is_contiguous()):
                    raise ValueError("buffer must be a contiguous uint8 tensor on the solver's device")
                self._ws_buf = buffer
            lead = (-self._ws_buf.data_ptr()) % WS_ALIGN
            if lead + self.workspace_bytes > self._ws_buf.numel():
                raise ValueError(f"buffer holds {self._ws_buf.numel()} bytes; this solver needs "
                                 f"{self.workspace_bytes} from a 16 MiB boundary")
            self.placement_ms = None
            if probes > 1:
                lead = self._probe(L, F, [lead + k * PROBE_STEP for k in range(probes)])
            self.ws = self._ws_buf[lead:lead + self.workspace_bytes]
            self.footprint_bytes = (self._ws_buf.numel() if buffer is None
                                    else self.workspace_bytes + WS_ALIGN)
            h = _create(A, F, self.precision, self.slice_width, self.ws.data_ptr(),
                        self.workspace_bytes, self.stream.cuda_stream)
        self._h = h
        n = ctypes.c_int64()
        nnz = ctypes.c_int64()
        prec = ctypes.c_int32()
        bpi = ctypes.c_double()
        ib = ctypes.c_int32()
        fm = (ctypes.c_int32 * 3)()
        check(L.pcga_solver_info(self._h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(prec),
                                 ctypes.byref(bpi), ctypes.byref(ib), fm), "pcga_solver_info")
        self.formats = (fm[0], fm[1])     # Z^T, Z: bit 0 16-bit index, bit 1/2 streamed idx/val
        self.band_q = fm[2]               # > 0: Z applied from its diagonals
        self.n = n.value
        self.nnz_off = nnz.value
        self.bytes_per_iter = bpi.value
        self.index_bytes = ib.value

    @property
    def handle(self):
        return self._h

    def tune(self, chunk=32, use_graph=True, max_blocks=0):
        check(_lib.load().pcga_solver_tune(self._h, int(chunk), int(bool(use_graph)),
                                           int(max_blocks)), "pcga_solver_tune")

    def set_grids(self, g_stencil=0, g_zt=0, g_z=0):
        """Workgroups per launch of the five-point, Z^T and Z kernels (0: the
        tune() cap)."""
        check(_lib.load().pcga_solver_set_grids(self._h, int(g_stencil), int(g_zt), int(g_z)),
              "pcga_solver_set_grids")

    def _xb(self, b, x0):
        import torch
        if x0 is None:
            x = torch.zeros(self.n, dtype=torch.float64, device=self.device)
        else:
            x = x0.clone()
        # order the solver's stream after the caller's work on b and x0 and
        # after the fill or copy of x just enqueued on the caller's stream
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        return _dev_ptr(b, torch.float64, self.n), x, _dev_ptr(x, torch.float64, self.n)

    def solve(self, b, x0=None, tol=1e-10, maxit=None, hist_cap=None) -> SolveResult:
        L = _lib.load()
        bp, x, xp = self._xb(b, x0)
        maxit = -1 if maxit is None else int(maxit)
        cap = (self.n if maxit < 0 else maxit) + 1 if hist_cap is None else int(hist_cap)
        hist = np.zeros(max(cap, 1))
        iters = ctypes.c_int32()
        hl = ctypes.c_int32()
        tr = ctypes.c_double()
        st = L.pcga_pcg_solve(self._h, bp, xp, float(tol), maxit, ctypes.byref(iters),
                              hist.ctypes.data, cap, ctypes.byref(hl), ctypes.byref(tr))
        check(st, "pcga_pcg_solve", allow=(_lib.OK, _lib.NOCONV))
        return SolveResult(x, iters.value, hist[: min(hl.value, cap)].copy(), st, tr.value)

    def solve_noalloc(self, b, x, tol=1e-10, maxit=None, hist=None) -> SolveResult:
        """pcga_pcg_solve_noalloc: the FP64 solve with the library's static
        scratch in place of the solver's vectors.  x holds x0 and receives
        the solution in place; hist (a float64 numpy array, optional)
        receives the history.  Allocates no device memory."""
        import torch
        L = _lib.load()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        bp = _dev_ptr(b, torch.float64, self.n)
        xp = _dev_ptr(x, torch.float64, self.n)
        maxit = -1 if maxit is None else int(maxit)
        cap = 0 if hist is None else int(hist.shape[0])
        iters = ctypes.c_int32()
        hl = ctypes.c_int32()
        tr = ctypes.c_double()
        st = L.pcga_pcg_solve_noalloc(self._h, bp, xp, float(tol), maxit, ctypes.byref(iters),
                                      None if hist is None else hist.ctypes.data, cap,
                                      ctypes.byref(hl), ctypes.byref(tr))
        check(st, "pcga_pcg_solve_noalloc", allow=(_lib.OK, _lib.NOCONV))
        h = hist[: min(hl.value, cap)].copy() if hist is not None else np.zeros(0)
        return SolveResult(x, iters.value, h, st, tr.value)

    def solve_mixed(self, b, x0=None, tol=1e-10, inner_tol=None, max_outer=None,
                    inner_maxit=None, refine="restart") -> SolveResult:
        """FP64 refinement around the FP32 inner PCG.  refine="restart": every
        inner run starts from d = s and stops at inner_tol (default 1e-5)
        relative to its own start; refine="keep": the direction is kept across
        corrections and inner_tol (default 0.1) is the reduction of one run."""
        L = _lib.load()
        mode = {"restart": _lib.REFINE_RESTART, "keep": _lib.REFINE_KEEP}[refine]
        if inner_tol is None:
            inner_tol = 0.1 if mode == _lib.REFINE_KEEP else 1e-5
        if max_outer is None:
            max_outer = 200 if mode == _lib.REFINE_KEEP else 20
        bp, x, xp = self._xb(b, x0)
        cap = max_outer + 1
        hist = np.zeros(cap)
        outer = ctypes.c_int32()
        tot = ctypes.c_int32()
        hl = ctypes.c_int32()
        tr = ctypes.c_double()
        st = L.pcga_pcg_solve_mixed_ex(self._h, bp, xp, float(tol), float(inner_tol),
                                       int(max_outer),
                                       -1 if inner_maxit is None else int(inner_maxit), mode,
                                       ctypes.byref(outer), ctypes.byref(tot), hist.ctypes.data,
                                       cap, ctypes.byref(hl), ctypes.byref(tr))
        check(st, "pcga_pcg_solve_mixed_ex", allow=(_lib.OK, _lib.NOCONV))
        return SolveResult(x, tot.value, hist[: hl.value].copy(), st, tr.value,
                           outer=outer.value, inner_total=tot.value)

    def apply_a(self, x):
        import torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        y = torch.empty_like(x)
        check(_lib.load().pcga_apply_a(self._h, _dev_ptr(x, torch.float64, self.n),
                                       _dev_ptr(y, torch.float64, self.n)), "pcga_apply_a")
        return y

    def apply_prec(self, r):
        import torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        t = torch.empty_like(r)
        s = torch.empty_like(r)
        check(_lib.load().pcga_apply_prec(self._h, _dev_ptr(r, torch.float64, self.n),
                                          _dev_ptr(t, torch.float64, self.n),
                                          _dev_ptr(s, torch.float64, self.n)), "pcga_apply_prec")
        return t, s

    def step_stencil(self, s, d, beta):
        """One launch of the fused direction update and operator product:
        (d_new = s + beta d, q = A d_new, (d_new, q)) in the solver's inner
        precision (see pcga_step_stencil)."""
        import torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        dn = torch.empty_like(s)
        q = torch.empty_like(s)
        dq = ctypes.c_double()
        check(_lib.load().pcga_step_stencil(self._h, _dev_ptr(s, torch.float64, self.n),
                                            _dev_ptr(d, torch.float64, self.n), float(beta),
                                            _dev_ptr(dn, torch.float64, self.n),
                                            _dev_ptr(q, torch.float64, self.n), ctypes.byref(dq)),
              "pcga_step_stencil")
        return dn, q, dq.value

    # --- the time step around the solve (eq. (1), eq. (8), the first guess) ---
    def _on_stream(self, fn):
        import torch
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)       # inputs written by the caller's stream
        fn()
        cur.wait_stream(self.stream)       # outputs visible to the caller's stream

    def ts_rhs(self, e2u, mu, e1v, mv):
        """Right-hand side of eq. (8) from face transports (see pcga_ts_rhs):
        b = -(delta_i(e2 Mu) - delta_j(e1 Mv))."""
        import torch
        ptrs = [_dev_ptr(t, torch.float64, self.n) for t in (e2u, mu, e1v, mv)]
        b = torch.empty(self.n, dtype=torch.float64, device=self.device)
        self._on_stream(lambda: check(_lib.load().pcga_ts_rhs(
            self._h, *ptrs, _dev_ptr(b, torch.float64, self.n)), "pcga_ts_rhs"))
        return b

    def ts_eta(self, eta_prev, D, dt):
        """eta^{n+1} = eta^{n-1} - 2 dt D^n (eq. (1))."""
        import torch
        out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        ep, dp = _dev_ptr(eta_prev, torch.float64, self.n), _dev_ptr(D, torch.float64, self.n)
        self._on_stream(lambda: check(_lib.load().pcga_ts_eta(
            self._h, ep, dp, float(dt), _dev_ptr(out, torch.float64, self.n)), "pcga_ts_eta"))
        return out

    def ts_guess(self, D1, D2=None, a=2.0, c=0.0):
        """First guess x0 = a D^{t-1} + c D^{t-2} (D2 unused when c = 0)."""
        import torch
        if c != 0.0 and D2 is None:
            raise ValueError("D2 is needed when c != 0")
        out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        p1 = _dev_ptr(D1, torch.float64, self.n)
        p2 = _dev_ptr(D2, torch.float64, self.n) if D2 is not None else None
        self._on_stream(lambda: check(_lib.load().pcga_ts_guess(
            self._h, p1, p2, float(a), float(c), _dev_ptr(out, torch.float64, self.n)),
            "pcga_ts_guess"))
        return out

    def _probe(self, L, F, offsets):
        """Build the solver at each offset of the buffer in turn, time one
        whole iteration there, and return the fastest offset."""
        import torch
        self.n = self.A.n
        probe_b = torch.ones(self.n, dtype=torch.float64, device=self.device)
        times = []
        for off in offsets:
            h = _create(self.A, F, self.precision, self.slice_width,
                        self._ws_buf.data_ptr() + off, self.workspace_bytes,
                        self.stream.cuda_stream)
            self._h = h
            try:
                self.profile_iteration(probe_b, reps=3, mode=1)
                times.append(min(self.profile_iteration(probe_b, reps=20, mode=1)[3]
                                 for _ in range(2)))
            finally:
                torch.cuda.synchronize()
                L.pcga_solver_destroy(h)
                self._h = None
        self.placement_ms = times
        return offsets[min(range(len(times)), key=times.__getitem__)]

    def profile_iteration(self, b, reps=50, mode=1):
        """Average ms of the three iteration kernels and of a whole iteration
        (HIP events on the solver stream).  mode 1: kernels timed inside whole
        iterations (the cache state of a solve); mode 0: each kernel repeated
        alone."""
        import torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        ms = (ctypes.c_double * 4)()
        check(_lib.load().pcga_profile_iteration(self._h, _dev_ptr(b, torch.float64, self.n),
                                                 int(reps), int(mode), ms),
              "pcga_profile_iteration")
        return list(ms)

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.load().pcga_solver_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HwStream:
    """A stream made by the library (pcga_stream_create) on `device`, for
    work that must overlap with work on other streams: streams made together
    are bound to distinct hardware queues (up to GPU_MAX_HW_QUEUES), which
    torch's pooled streams need not be.  `.torch` is the torch view of it
    (pass that as a Solver's or Batch's stream); close() waits for its work
    and destroys it, after every solver and batch on it has been closed."""

    def __init__(self, device=None):
        import torch
        L = _lib.load()
        self.device = torch.device("cuda" if device is None else device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(L.pcga_stream_create(ctypes.byref(h)), "pcga_stream_create")
        self._h = h.value
        self.torch = torch.cuda.ExternalStream(self._h, device=self.device)

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            import torch
            with torch.cuda.device(self.device):
                check(_lib.load().pcga_stream_destroy(ctypes.c_void_p(h)), "pcga_stream_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pcg_solve(A: Stencil5, F: AInv, b, x0=None, tol=1e-10, maxit=None, solver=None) -> SolveResult:
    """Algorithm 1 in FP64 on the device: returns (x, iters, hist) (plus status
    and the FP64 true residual as attributes)."""
    S = solver if solver is not None else Solver(A, F, "fp64", device=b.device)
    return S.solve(b, x0, tol=tol, maxit=maxit)


def pcg_solve_mixed(A: Stencil5, F: AInv, b, x0=None, tol=1e-10, inner_tol=None, max_outer=None,
                    inner_maxit=None, solver=None, refine="restart") -> SolveResult:
    """FP32 inner PCG with FP64 iterative refinement (restarted, or with the
    direction kept across corrections: refine="keep")."""
    S = solver if solver is not None else Solver(A, F, "mixed", device=b.device)
    return S.solve_mixed(b, x0, tol=tol, inner_tol=inner_tol, max_outer=max_outer,
                         inner_maxit=inner_maxit, refine=refine)


class Batch:
    """Many mixed-precision solves advanced together (one launch per kernel per
    iteration for all items); items can be added and removed between runs."""

    def __init__(self, max_slots=64, device=None, stream=None, chunk=16, grid=None):
        import torch
        L = _lib.load()
        self.device = torch.device("cuda" if device is None else device)
        nb = ctypes.c_size_t()
        check(L.pcga_batch_scratch_bytes(int(max_slots), ctypes.byref(nb)), "pcga_batch_scratch_bytes")
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.Stream(self.device) if stream is None else stream
            self.scratch = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
            h = ctypes.c_void_p()
            check(L.pcga_batch_create(int(max_slots), ctypes.c_void_p(self.scratch.data_ptr()),
                                      nb.value, ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(h)), "pcga_batch_create")
        self._h = h
        self.items = {}
        check(L.pcga_batch_set_chunk(self._h, int(chunk)), "pcga_batch_set_chunk")
        if grid is not None:
            self.set_grid(grid)

    def set_grid(self, grid):
        """Workgroups per launch (multiple of 8, 8..2048; results do not depend on it)."""
        check(_lib.load().pcga_batch_set_grid(self._h, int(grid)), "pcga_batch_set_grid")

    @staticmethod
    def item_bytes(solver, nrhs):
        nb = ctypes.c_size_t()
        check(_lib.load().pcga_batch_item_bytes(solver.handle, int(nrhs), ctypes.byref(nb)),
              "pcga_batch_item_bytes")
        return nb.value

    def add(self, solver, B, X0=None, tol=1e-10, inner_tol=None, max_outer=None, inner_maxit=None,
            tag=None, refine="restart"):
        """B: [nrhs, n] float64 device tensor (nrhs in 1, 2, 4).  Returns the slot.
        refine as in Solver.solve_mixed ("restart": inner_tol default 1e-5;
        "keep": the inner direction kept across corrections, inner_tol
        default 0.1)."""
        import torch
        L = _lib.load()
        mode = {"restart": _lib.REFINE_RESTART, "keep": _lib.REFINE_KEEP}[refine]
        if inner_tol is None:
            inner_tol = 0.1 if mode == _lib.REFINE_KEEP else 1e-5
        if max_outer is None:
            max_outer = 200 if mode == _lib.REFINE_KEEP else 20
        if B.dim() == 1:
            B = B.unsqueeze(0)
        nrhs, n = B.shape
        B = B.contiguous()
        X0 = torch.zeros_like(B) if X0 is None else X0.reshape(nrhs, n).contiguous()
        X = torch.empty_like(B)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        nbytes = self.item_bytes(solver, nrhs)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        arr = ctypes.c_void_p * nrhs
        bp = arr(*[B[r].data_ptr() for r in range(nrhs)])
        xp = arr(*[X0[r].data_ptr() for r in range(nrhs)])
        op = arr(*[X[r].data_ptr() for r in range(nrhs)])
        slot = ctypes.c_int32()
        check(L.pcga_batch_add_ex(self._h, solver.handle, int(nrhs), bp, xp, op,
                                  ctypes.c_void_p(ws.data_ptr()), nbytes, float(tol),
                                  float(inner_tol), int(max_outer),
                                  -1 if inner_maxit is None else int(inner_maxit), mode,
                                  ctypes.byref(slot)), "pcga_batch_add_ex")
        self.items[slot.value] = dict(solver=solver, B=B, X=X, ws=ws, nrhs=nrhs, tag=tag)
        return slot.value

    def run(self, chunks=1):
        active = ctypes.c_int32()
        check(_lib.load().pcga_batch_run(self._h, int(chunks), ctypes.byref(active)), "pcga_batch_run")
        return active.value

    def launch(self, chunks=1):
        """Enqueue `chunks` chunks on the batch's stream without waiting."""
        check(_lib.load().pcga_batch_launch(self._h, int(chunks)), "pcga_batch_launch")

    def wait(self, block=True):
        """Wait for (block) or check on the last launch: (ready, active items)."""
        ready = ctypes.c_int32()
        active = ctypes.c_int32()
        check(_lib.load().pcga_batch_wait(self._h, int(bool(block)), ctypes.byref(ready),
                                          ctypes.byref(active)), "pcga_batch_wait")
        return bool(ready.value), active.value

    def query(self, slot):
        it = self.items[slot]
        done, st, outer, inner = (ctypes.c_int32() for _ in range(4))
        rel = (ctypes.c_double * 4)()
        check(_lib.load().pcga_batch_query(self._h, int(slot), ctypes.byref(done), ctypes.byref(st),
                                           ctypes.byref(outer), ctypes.byref(inner), rel),
              "pcga_batch_query")
        return dict(done=bool(done.value), status=st.value, outer=outer.value,
                    inner_total=inner.value, true_relres=list(rel[: it["nrhs"]]))

    def remove(self, slot):
        """Write the solutions and free the slot; returns (X [nrhs, n], query dict)."""
        q = self.query(slot)
        check(_lib.load().pcga_batch_remove(self._h, int(slot)), "pcga_batch_remove")
        it = self.items.pop(slot)
        return it["X"], q

    def solve(self, max_chunks=100000):
        """Run until every item is done; returns {slot: (X, query)} and removes all."""
        left = self.run(1)
        guard = 0
        while left > 0 and guard < max_chunks:
            left = self.run(4)
            guard += 1
        return {s: self.remove(s) for s in list(self.items)}

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.load().pcga_batch_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
