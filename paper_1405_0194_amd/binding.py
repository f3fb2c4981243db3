"""Thin ctypes binding of libpexsi_hip.so (include/pexsi_hip.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  PyTorch provides device memory (the caller-owned buffers of the
C ABI) and the current HIP stream.  There is no fallback: if the compiled
library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpexsi_hip.so")

PXS_OK, PXS_EINVAL, PXS_ENOMEM, PXS_EHIP, PXS_ESTATE, PXS_TINY_PIVOT = 0, -1, -2, -3, -4, 1
SETS = ("rho", "E", "F", "d")


class PxsError(RuntimeError):
    def __init__(self, fn, code, detail=""):
        self.code = code
        super().__init__(f"{fn} failed with status {code}: {detail}")


class c64(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class Options(C.Structure):
    _fields_ = [("ordering", C.c_int32), ("leaf_cols", C.c_int32), ("panel_width", C.c_int32),
                ("selinv_chunk", C.c_int32), ("pivot_tol", C.c_double), ("tile_rows", C.c_int32),
                ("selinv_streams", C.c_int32), ("sep_cols", C.c_int32), ("fused_lanes", C.c_int32),
                ("reserved1", C.c_double * 2)]


class SymInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz_lower", C.c_int64), ("nnz_L", C.c_int64),
                ("nnz_L_exact", C.c_int64), ("nsuper", C.c_int64), ("npanel", C.c_int64),
                ("bytes_per_shift", C.c_int64), ("work_bytes", C.c_int64),
                ("work_fixed", C.c_int64), ("work_per_shift", C.c_int64),
                ("gather_per_shift", C.c_int64), ("selinv_chunk", C.c_int64),
                ("map_bytes", C.c_int64), ("max_front", C.c_int64),
                ("flops_factor", C.c_double), ("flops_selinv", C.c_double),
                ("macs_exact", C.c_double * 8), ("fused_lanes", C.c_int64), ("sel_lanes", C.c_int64)]


_P = C.c_void_p
_lib = None


def load():
    """Loads the compiled library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # PyTorch brings its own HIP runtime; load it first so that the library
    # resolves libamdhip64 to that same runtime (one runtime per process).
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    sig = {
        "pxs_poles": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_int32, C.c_int32, _P, _P]),
        "pxs_analyze": (C.c_int, [C.c_int32, _P, _P, C.c_int32, _P, _P, _P, _P]),
        "pxs_symbolic_info": (C.c_int, [_P, _P]),
        "pxs_workspace_size": (C.c_int, [_P, C.c_int32, C.c_int32, _P]),
        "pxs_symbolic_export": (C.c_int, [_P, _P, _P, _P, _P, _P]),
        "pxs_symbolic_bind": (C.c_int, [_P, _P, _P]),
        "pxs_factor": (C.c_int, [_P, _P, _P, C.c_int32, _P, _P, _P, _P, _P, _P]),
        "pxs_selinv": (C.c_int, [_P, _P]),
        "pxs_pole_sum": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P]),
        "pxs_get_selected": (C.c_int, [_P, C.c_int32, _P, _P]),
        "pxs_get_selected_upper": (C.c_int, [_P, C.c_int32, _P, _P]),
        "pxs_hermitian_sizes": (C.c_int, [_P, C.c_int32, _P, _P]),
        "pxs_factor_hermitian": (C.c_int, [_P, _P, _P, C.c_int32, _P, _P, _P, _P, _P, _P]),
        "pxs_get_diag": (C.c_int, [_P, C.c_int32, _P, _P]),
        "pxs_inertia": (C.c_int, [_P, _P, _P, C.c_int32, _P, _P, _P, _P, _P, _P]),
        "pxs_inertia_hermitian": (C.c_int, [_P, _P, _P, C.c_int32, _P, _P, _P, _P, _P, _P]),
        "pxs_inertia_async": (C.c_int, [_P, _P, _P, C.c_int32, _P, _P, _P, _P, _P, _P]),
        "pxs_plan_run_device": (C.c_int, [_P, _P, _P, _P]),
        "pxs_plan_copy_results": (C.c_int, [_P, _P, _P, _P]),
        "pxs_batch_create": (C.c_int, [C.c_int32, _P, _P, _P, _P, C.c_int32, _P, _P, _P, _P]),
        "pxs_batch_info": (C.c_int, [_P, _P, _P]),
        "pxs_batch_bind": (C.c_int, [_P, _P, _P]),
        "pxs_batch_run": (C.c_int, [_P, _P, _P, _P]),
        "pxs_batch_results": (C.c_int, [_P, _P, _P, _P]),
        "pxs_batch_free": (None, [_P]),
        "pxs_density_matrix": (C.c_int, [_P, _P, _P, C.c_double, C.c_double, C.c_double, C.c_int32,
                                         C.c_int32, _P, _P, _P, _P, _P, _P, _P, _P]),
        "pxs_density_matrix_noalloc": (C.c_int, [_P, _P, _P, C.c_double, C.c_double, C.c_double, C.c_int32,
                                                 C.c_int32, _P, _P, _P, _P, _P, _P, _P]),
        "pxs_plan_create": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, _P, _P, _P, C.c_int32, _P]),
        "pxs_plan_create_hermitian": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, _P, _P, _P, C.c_int32, _P]),
        "pxs_plan_run": (C.c_int, [_P, _P, _P, _P, _P, _P]),
        "pxs_plan_results": (C.c_int, [_P, _P, _P, _P]),
        "pxs_plan_free": (None, [_P]),
        "pxs_profile_begin": (C.c_int, [C.c_int32]),
        "pxs_profile_end": (C.c_int, [_P, _P, _P, _P, _P]),
        "pxs_free_symbolic": (None, [_P]),
        "pxs_free_numeric": (None, [_P]),
        "pxs_status_string": (C.c_char_p, [C.c_int]),
        "pxs_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(fn, code, allow=(PXS_OK,)):
    if code not in allow:
        lib = load()
        detail = lib.pxs_status_string(code).decode()
        extra = lib.pxs_last_error().decode()
        raise PxsError(fn, code, detail + (f" ({extra})" if extra else ""))
    return code


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_P)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return _P(s.cuda_stream)


def _dptr(t):
    return _P(t.data_ptr())


def _nbytes(t):
    return t.numel() * t.element_size()


def _require(t, nbytes, what):
    """Caller buffers go to the kernels as raw pointers: check them here."""
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what}: needs a contiguous device tensor")
    if _nbytes(t) < nbytes:
        raise ValueError(f"{what}: {_nbytes(t)} bytes, needs {nbytes}")
    if t.data_ptr() % 256:
        raise ValueError(f"{what}: must be 256-byte aligned")


def _require_vec(t, dtype, n, what):
    """A small device array passed as a raw pointer: contiguous, right type
    and at least n elements."""
    if not t.is_cuda or not t.is_contiguous() or t.dtype != dtype or t.numel() < n:
        raise ValueError(f"{what}: needs a contiguous {dtype} device tensor of {n} elements")


def _require_values(analysis, H, S):
    import torch
    nnz = analysis.info["nnz_lower"]
    for t, name in ((H, "H values"), (S, "S values")):
        if t.dtype != torch.float64 or t.numel() != nnz or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name}: need a contiguous float64 device tensor of {nnz} entries")


# --------------------------------------------------------------------------
def poles(beta: float, dE: float, mu: float, P: int, nsets: int = 2):
    """Pole table from the library: shifts (P,) complex, weights (nsets, P)."""
    lib = load()
    sh = np.zeros(P, dtype=np.complex128)
    wt = np.zeros(nsets * P, dtype=np.complex128)
    _check("pxs_poles", lib.pxs_poles(beta, dE, mu, P, nsets, _ptr(sh), _ptr(wt)))
    return sh, wt.reshape(nsets, P)


class Analysis:
    """Symbolic analysis handle (host), optionally bound to device maps."""

    def __init__(self, n, colptr, rowind, blkptr=None, coords=None, ordering=0, leaf_cols=0,
                 panel_width=0, pivot_tol=0.0, selinv_chunk=0, tile_rows=0, selinv_streams=0, sep_cols=0,
                 fused_lanes=0):
        lib = load()
        self._lib = lib
        self.n = int(n)
        colptr = np.ascontiguousarray(colptr, dtype=np.int64)
        rowind = np.ascontiguousarray(rowind, dtype=np.int32)
        self.options = dict(ordering=ordering, leaf_cols=leaf_cols, panel_width=panel_width,
                            pivot_tol=pivot_tol, selinv_chunk=selinv_chunk, tile_rows=tile_rows,
                            selinv_streams=selinv_streams, sep_cols=sep_cols, fused_lanes=fused_lanes)
        opt = Options(ordering, leaf_cols, panel_width, selinv_chunk, pivot_tol, tile_rows, selinv_streams,
                      sep_cols, fused_lanes)
        h = _P()
        nblk = 0
        bp = None
        cp = None
        if blkptr is not None:
            blkptr = np.ascontiguousarray(blkptr, dtype=np.int32)
            nblk = blkptr.shape[0] - 1
            bp = _ptr(blkptr)
        if coords is not None:
            coords = np.ascontiguousarray(coords, dtype=np.float64)
            if blkptr is None:
                nblk = coords.shape[0]
            cp = _ptr(coords)
        _check("pxs_analyze", lib.pxs_analyze(self.n, _ptr(colptr), _ptr(rowind), nblk, bp, cp,
                                               C.byref(opt), C.byref(h)))
        self._h = h
        info = SymInfo()
        _check("pxs_symbolic_info", lib.pxs_symbolic_info(h, C.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in SymInfo._fields_}
        self.info["macs_exact"] = list(info.macs_exact)
        self.maps = None

    @classmethod
    def from_system(cls, system, **kw):
        return cls(system.n, system.colptr, system.rowind, blkptr=system.blkptr,
                   coords=system.coords, **kw)

    def export(self):
        i = self.info
        ns = i["nsuper"]
        perm = np.zeros(self.n, dtype=np.int32)
        sp = np.zeros(ns + 1, dtype=np.int32)
        par = np.zeros(ns, dtype=np.int32)
        rp = np.zeros(ns + 1, dtype=np.int64)
        _check("pxs_symbolic_export", self._lib.pxs_symbolic_export(self._h, _ptr(perm), _ptr(sp), _ptr(par),
                                                                     _ptr(rp), None))
        rows = np.zeros(int(rp[-1]), dtype=np.int32)
        _check("pxs_symbolic_export", self._lib.pxs_symbolic_export(self._h, None, None, None, None,
                                                                     _ptr(rows)))
        return dict(perm=perm, super_ptr=sp, parent=par, row_ptr=rp, rows=rows)

    def bind(self, device="cuda"):
        import torch
        if self.maps is None:
            self.maps = torch.empty(self.info["map_bytes"], dtype=torch.uint8, device=device)
            _check("pxs_symbolic_bind", self._lib.pxs_symbolic_bind(self._h, _dptr(self.maps), _stream()))
        return self

    def buffers(self, nshift, real=False, device="cuda"):
        """Allocates (Lbuf, work) device buffers for a batch of nshift shifts."""
        import torch
        per = self.info["bytes_per_shift"] // (2 if real else 1)
        L = torch.empty(per * nshift, dtype=torch.uint8, device=device)
        W = torch.empty(self.workspace_size(nshift, real), dtype=torch.uint8, device=device)
        return L, W

    def workspace_size(self, nshift, real=False):
        b = C.c_int64()
        _check("pxs_workspace_size", self._lib.pxs_workspace_size(self._h, nshift, int(real), C.byref(b)))
        return b.value

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                self._lib.pxs_free_symbolic(self._h)
                self._h = None
        except Exception:
            pass


class Factorization:
    """A batch of shifts factored (and optionally inverted) in caller buffers."""

    def __init__(self, analysis: Analysis, H, S, shifts, L=None, work=None, stream=None):
        lib = load()
        self._lib = lib
        self.analysis = analysis
        analysis.bind()
        self.shifts = np.ascontiguousarray(shifts, dtype=np.complex128)
        nshift = self.shifts.shape[0]
        self.nshift = nshift
        if L is None or work is None:
            L, work = analysis.buffers(nshift)
        _require_values(analysis, H, S)
        _require(L, nshift * analysis.info["bytes_per_shift"], "factor storage")
        _require(work, analysis.workspace_size(nshift), "workspace")
        self.L, self.work = L, work
        self.H, self.S = H, S   # keep the device value arrays alive
        self.info = np.zeros(nshift, dtype=np.int64)
        h = _P()
        code = lib.pxs_factor(analysis._h, _dptr(H), _dptr(S), nshift, _ptr(self.shifts),
                              _dptr(L), _dptr(work), _ptr(self.info), _stream(stream), C.byref(h))
        _check("pxs_factor", code, allow=(PXS_OK, PXS_TINY_PIVOT))
        self._h = h
        self.inverted = False

    def diag(self, l, stream=None):
        import torch
        out = torch.empty(self.analysis.n, dtype=torch.complex128, device=self.L.device)
        _check("pxs_get_diag", self._lib.pxs_get_diag(self._h, l, _dptr(out), _stream(stream)))
        return out

    def selinv(self, stream=None):
        _check("pxs_selinv", self._lib.pxs_selinv(self._h, _stream(stream)))
        self.inverted = True
        return self

    def selected(self, l, stream=None):
        """Z_l on the input pattern (complex128 tensor, input ordering)."""
        import torch
        out = torch.empty(self.analysis.info["nnz_lower"], dtype=torch.complex128, device=self.L.device)
        _check("pxs_get_selected", self._lib.pxs_get_selected(self._h, l, _dptr(out), _stream(stream)))
        return out

    def pole_sum(self, weights, stream=None, out=None, traces=True):
        """weights: (nsets, nshift) complex.  Returns (out (nsets, nnz), traces
        array (nsets, 2) = [Tr(G S), Tr(G H)], or None without traces)."""
        import torch
        weights = np.ascontiguousarray(weights, dtype=np.complex128)
        nsets = weights.shape[0]
        nnz = self.analysis.info["nnz_lower"]
        if out is None:
            out = torch.empty(nsets * nnz, dtype=torch.float64, device=self.L.device)
        _require(out, 8 * nsets * nnz, "pole-sum output")
        if weights.shape != (nsets, self.nshift):
            raise ValueError("weights must be (nsets, nshift)")
        tr = np.zeros(2 * nsets)
        _check("pxs_pole_sum", self._lib.pxs_pole_sum(self._h, nsets, _ptr(weights), _dptr(out),
                                                       _ptr(tr) if traces else None, _stream(stream)))
        return out.view(nsets, nnz), (tr.reshape(nsets, 2) if traces else None)

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                self._lib.pxs_free_numeric(self._h)
                self._h = None
        except Exception:
            pass


class HermitianFactorization:
    """A batch of shifts of a complex Hermitian pencil factored as L D U
    (and optionally inverted) in caller buffers.  H and S: complex128 device
    tensors with the lower triangle on the input pattern."""

    def __init__(self, analysis: Analysis, H, S, shifts, L=None, work=None, stream=None):
        import torch
        lib = load()
        self._lib = lib
        self.analysis = analysis
        analysis.bind()
        self.shifts = np.ascontiguousarray(shifts, dtype=np.complex128)
        nshift = self.shifts.shape[0]
        self.nshift = nshift
        lb, wb = hermitian_sizes(analysis, nshift)
        if L is None or work is None:
            L = torch.empty(lb, dtype=torch.uint8, device=H.device)
            work = torch.empty(wb, dtype=torch.uint8, device=H.device)
        nnz = analysis.info["nnz_lower"]
        for t, name in ((H, "H values"), (S, "S values")):
            if t.dtype != torch.complex128 or t.numel() != nnz or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name}: need a contiguous complex128 device tensor of {nnz} entries")
        _require(L, lb, "factor storage")
        _require(work, wb, "workspace")
        self.L, self.work = L, work
        self.H, self.S = H, S
        self.info = np.zeros(nshift, dtype=np.int64)
        h = _P()
        code = lib.pxs_factor_hermitian(analysis._h, _dptr(H), _dptr(S), nshift, _ptr(self.shifts), _dptr(L),
                                        _dptr(work), _ptr(self.info), _stream(stream), C.byref(h))
        _check("pxs_factor_hermitian", code, allow=(PXS_OK, PXS_TINY_PIVOT))
        self._h = h

    def diag(self, l, stream=None):
        import torch
        out = torch.empty(self.analysis.n, dtype=torch.complex128, device=self.L.device)
        _check("pxs_get_diag", self._lib.pxs_get_diag(self._h, l, _dptr(out), _stream(stream)))
        return out

    def selinv(self, stream=None):
        _check("pxs_selinv", self._lib.pxs_selinv(self._h, _stream(stream)))
        return self

    def selected(self, l, upper=False, stream=None):
        """Z_l[i][j] (or Z_l[j][i] with upper) at the input entries i >= j."""
        import torch
        out = torch.empty(self.analysis.info["nnz_lower"], dtype=torch.complex128, device=self.L.device)
        f = self._lib.pxs_get_selected_upper if upper else self._lib.pxs_get_selected
        _check("pxs_get_selected", f(self._h, l, _dptr(out), _stream(stream)))
        return out

    def pole_sum(self, weights, stream=None):
        """Gamma^g = (M - M^H) / 2i, M = sum_l omega_{g,l} Z_l: returns
        ((nsets, nnz) complex tensor of Gamma_ij at the input entries,
        traces (nsets, 2) = [Re Tr(G S), Re Tr(G H)])."""
        import torch
        weights = np.ascontiguousarray(weights, dtype=np.complex128)
        nsets = weights.shape[0]
        if weights.shape != (nsets, self.nshift):
            raise ValueError("weights must be (nsets, nshift)")
        nnz = self.analysis.info["nnz_lower"]
        out = torch.empty(nsets * nnz, dtype=torch.complex128, device=self.L.device)
        tr = np.zeros(2 * nsets)
        _check("pxs_pole_sum", self._lib.pxs_pole_sum(self._h, nsets, _ptr(weights), _dptr(out), _ptr(tr),
                                                       _stream(stream)))
        return out.view(nsets, nnz), tr.reshape(nsets, 2)

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                self._lib.pxs_free_numeric(self._h)
                self._h = None
        except Exception:
            pass


def hermitian_sizes(analysis: Analysis, nshift: int):
    """(factor storage bytes, workspace bytes) of a Hermitian batch."""
    lb, wb = C.c_int64(), C.c_int64()
    _check("pxs_hermitian_sizes", load().pxs_hermitian_sizes(analysis._h, nshift, C.byref(lb), C.byref(wb)))
    return lb.value, wb.value


class Plan:
    """A graph-captured density matrix for a fixed batch size on fixed
    buffers: run() uploads a pole table and replays the graph."""

    def __init__(self, analysis: Analysis, H, S, nshift, nsets=2, L=None, work=None, device="cuda",
                 out=None, accumulate=False):
        """Complex H and S (complex128) capture the Hermitian path; out is
        then complex."""
        import torch
        lib = load()
        self._lib = lib
        self.analysis = analysis.bind()
        self.nshift, self.nsets = int(nshift), int(nsets)
        self.hermitian = H.is_complex()
        nnz = analysis.info["nnz_lower"]
        if self.hermitian:
            lb, wb = hermitian_sizes(analysis, self.nshift)
            if L is None or work is None:
                L = torch.empty(lb, dtype=torch.uint8, device=H.device)
                work = torch.empty(wb, dtype=torch.uint8, device=H.device)
            for t, name in ((H, "H values"), (S, "S values")):
                if t.dtype != torch.complex128 or t.numel() != nnz or not t.is_cuda or not t.is_contiguous():
                    raise ValueError(f"{name}: need a contiguous complex128 device tensor of {nnz} entries")
            _require(L, lb, "factor storage")
            _require(work, wb, "workspace")
        else:
            if L is None or work is None:
                L, work = analysis.buffers(nshift)
            _require_values(analysis, H, S)
            _require(L, self.nshift * analysis.info["bytes_per_shift"], "factor storage")
            _require(work, analysis.workspace_size(self.nshift), "workspace")
        self.L, self.work, self.H, self.S = L, work, H, S
        dt = torch.complex128 if self.hermitian else torch.float64
        if out is None:
            out = torch.empty(nsets * nnz, dtype=dt, device=L.device)
        _require(out, (16 if self.hermitian else 8) * nsets * nnz, "pole-sum output")
        self.out = out
        h = _P()
        if self.hermitian:
            if accumulate:
                raise ValueError("accumulate is not available for Hermitian plans")
            _check("pxs_plan_create_hermitian",
                   lib.pxs_plan_create_hermitian(analysis._h, _dptr(H), _dptr(S), self.nshift, self.nsets,
                                                 _dptr(L), _dptr(work), _dptr(self.out), 0, C.byref(h)))
        else:
            _check("pxs_plan_create", lib.pxs_plan_create(analysis._h, _dptr(H), _dptr(S), self.nshift,
                                                           self.nsets, _dptr(L), _dptr(work), _dptr(self.out),
                                                           1 if accumulate else 0, C.byref(h)))
        self._h = h

    def run(self, shifts, weights, stream=None, sync=True):
        """Returns (out view (nsets, nnz), traces (nsets, 2) or None, info)."""
        shifts = np.ascontiguousarray(shifts, dtype=np.complex128)
        weights = np.ascontiguousarray(weights, dtype=np.complex128).reshape(self.nsets, self.nshift)
        tr = np.zeros(2 * self.nsets) if sync else None
        info = np.zeros(self.nshift, dtype=np.int64) if sync else None
        code = self._lib.pxs_plan_run(self._h, _ptr(shifts), _ptr(weights), _ptr(tr) if sync else None,
                                      _ptr(info) if sync else None, _stream(stream))
        _check("pxs_plan_run", code, allow=(PXS_OK, PXS_TINY_PIVOT))
        nnz = self.analysis.info["nnz_lower"]
        return self.out.view(self.nsets, nnz), (tr.reshape(self.nsets, 2) if sync else None), info

    def run_device(self, shifts, weights, stream=None):
        """Replays the graph with a pole table already on the device
        (complex128 tensors: shifts (nshift,), weights (nsets * nshift,)
        set-major); waits for nothing."""
        import torch
        _require_vec(shifts, torch.complex128, self.nshift, "shifts")
        _require_vec(weights, torch.complex128, self.nsets * self.nshift, "weights")
        _check("pxs_plan_run_device", self._lib.pxs_plan_run_device(self._h, _dptr(shifts), _dptr(weights),
                                                                     _stream(stream)))

    def copy_results(self, traces, info, stream=None):
        """Enqueues copies of the last run's traces (float64 device tensor of
        2 * nsets) and pivot info (int64 device tensor of nshift)."""
        import torch
        _require_vec(traces, torch.float64, 2 * self.nsets, "traces")
        _require_vec(info, torch.int64, self.nshift, "info")
        _check("pxs_plan_copy_results", self._lib.pxs_plan_copy_results(self._h, _dptr(traces), _dptr(info),
                                                                         _stream(stream)))

    def results(self, stream=None):
        """(traces (nsets, 2), info) of the last run (synchronises stream)."""
        tr = np.zeros(2 * self.nsets)
        info = np.zeros(self.nshift, dtype=np.int64)
        _check("pxs_plan_results", self._lib.pxs_plan_results(self._h, _ptr(tr), _ptr(info), _stream(stream)),
               allow=(PXS_OK, PXS_TINY_PIVOT))
        return tr.reshape(self.nsets, 2), info

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                self._lib.pxs_plan_free(self._h)
                self._h = None
        except Exception:
            pass


def inertia(analysis: Analysis, H, S, eps, L=None, work=None, stream=None):
    """Counts #{k : d_k < 0} of H - eps_q S for each q (host int64 array) and
    the per-shift tiny-pivot info."""
    lib = load()
    analysis.bind()
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    q = eps.shape[0]
    if L is None or work is None:
        L, work = analysis.buffers(q, real=True)
    _require_values(analysis, H, S)
    _require(L, q * analysis.info["bytes_per_shift"] // 2, "factor storage")
    _require(work, analysis.workspace_size(q, real=True), "workspace")
    neg = np.zeros(q, dtype=np.int64)
    info = np.zeros(q, dtype=np.int64)
    code = lib.pxs_inertia(analysis._h, _dptr(H), _dptr(S), q, _ptr(eps), _dptr(L), _dptr(work),
                           _ptr(neg), _ptr(info), _stream(stream))
    _check("pxs_inertia", code, allow=(PXS_OK, PXS_TINY_PIVOT))
    return neg, info


def inertia_async(analysis: Analysis, H, S, eps, neg, info, L, work, stream=None):
    """Enqueues the inertia counts of H - eps_q S (eps: float64 device
    tensor) into the int64 device tensors neg and info on `stream`, without
    waiting for the device."""
    import torch
    lib = load()
    q = eps.numel()
    _require_vec(eps, torch.float64, q, "eps")
    _require_vec(neg, torch.int64, q, "neg")
    _require_vec(info, torch.int64, q, "info")
    _require_values(analysis, H, S)
    _require(L, q * analysis.info["bytes_per_shift"] // 2, "factor storage")
    _require(work, analysis.workspace_size(q, real=True), "workspace")
    _check("pxs_inertia_async", lib.pxs_inertia_async(analysis._h, _dptr(H), _dptr(S), q, _dptr(eps), _dptr(L),
                                                       _dptr(work), _dptr(neg), _dptr(info), _stream(stream)))


def inertia_hermitian(analysis: Analysis, H, S, eps, L=None, work=None, stream=None):
    """Counts #{k : Re d_k < 0} of the L D U of the Hermitian H - eps_q S for
    each q (host int64 array) and the per-shift tiny-pivot info.  H, S:
    complex128 device tensors on the input pattern."""
    import torch
    lib = load()
    analysis.bind()
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    q = eps.shape[0]
    lb, wb = hermitian_sizes(analysis, q)
    if L is None or work is None:
        L = torch.empty(lb, dtype=torch.uint8, device=H.device)
        work = torch.empty(wb, dtype=torch.uint8, device=H.device)
    nnz = analysis.info["nnz_lower"]
    for t, name in ((H, "H values"), (S, "S values")):
        if t.dtype != torch.complex128 or t.numel() != nnz or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name}: need a contiguous complex128 device tensor of {nnz} entries")
    _require(L, lb, "factor storage")
    _require(work, wb, "workspace")
    neg = np.zeros(q, dtype=np.int64)
    info = np.zeros(q, dtype=np.int64)
    code = lib.pxs_inertia_hermitian(analysis._h, _dptr(H), _dptr(S), q, _ptr(eps), _dptr(L), _dptr(work),
                                     _ptr(neg), _ptr(info), _stream(stream))
    _check("pxs_inertia_hermitian", code, allow=(PXS_OK, PXS_TINY_PIVOT))
    return neg, info


def density_matrix(analysis: Analysis, H, S, beta, dE, mu, P, nsets=2, L=None, work=None,
                   stream=None):
    """Fused poles + factor + selinv + pole sums.  Returns (out (nsets, nnz)
    tensor, traces (nsets, 2), info, shifts, weights)."""
    import torch
    lib = load()
    analysis.bind()
    if L is None or work is None:
        L, work = analysis.buffers(P)
    _require_values(analysis, H, S)
    _require(L, P * analysis.info["bytes_per_shift"], "factor storage")
    _require(work, analysis.workspace_size(P), "workspace")
    nnz = analysis.info["nnz_lower"]
    out = torch.empty(nsets * nnz, dtype=torch.float64, device=L.device)
    tr = np.zeros(2 * nsets)
    info = np.zeros(P, dtype=np.int64)
    sh = np.zeros(P, dtype=np.complex128)
    wt = np.zeros(nsets * P, dtype=np.complex128)
    code = lib.pxs_density_matrix(analysis._h, _dptr(H), _dptr(S), beta, dE, mu, P, nsets, _dptr(L),
                                  _dptr(work), _dptr(out), _ptr(tr), _ptr(info), _ptr(sh), _ptr(wt),
                                  _stream(stream))
    _check("pxs_density_matrix", code, allow=(PXS_OK, PXS_TINY_PIVOT))
    return out.view(nsets, nnz), tr.reshape(nsets, 2), info, sh, wt.reshape(nsets, P)


class FusedBatch:
    """The density matrices of several real systems as one sequence of
    fused launches captured in one HIP graph (pxs_batch_*).  systems: list
    of (analysis, H, S, nshift); buffers: optional list of (L, work) device
    tensors per system (views into a shared arena, say), else allocated
    here; the outputs and the launch table are allocated here."""

    def __init__(self, systems, nsets=2, device="cuda", buffers=None):
        import torch
        lib = load()
        self._lib = lib
        self.nsets = int(nsets)
        self.systems = []
        for i, (a, H, S, P) in enumerate(systems):
            a.bind(device)
            _require_values(a, H, S)
            L, W = buffers[i] if buffers is not None else a.buffers(P, device=device)
            _require(L, int(P) * a.info["bytes_per_shift"], "factor storage")
            _require(W, a.workspace_size(int(P)), "workspace")
            out = torch.empty(self.nsets * a.info["nnz_lower"], dtype=torch.float64, device=device)
            self.systems.append((a, H, S, int(P), L, W, out))
        n = len(self.systems)
        arr = lambda vals: (_P * n)(*vals)
        self.nshift = np.array([y[3] for y in self.systems], dtype=np.int32)
        h = _P()
        _check("pxs_batch_create", lib.pxs_batch_create(
            n, arr([y[0]._h for y in self.systems]), arr([_dptr(y[1]) for y in self.systems]),
            arr([_dptr(y[2]) for y in self.systems]), _ptr(self.nshift), self.nsets,
            arr([_dptr(y[4]) for y in self.systems]), arr([_dptr(y[5]) for y in self.systems]),
            arr([_dptr(y[6]) for y in self.systems]), C.byref(h)))
        self._h = h
        tb, nl = C.c_int64(), C.c_int64()
        _check("pxs_batch_info", lib.pxs_batch_info(h, C.byref(tb), C.byref(nl)))
        self.launches = nl.value
        self.table = torch.empty(max(256, tb.value), dtype=torch.uint8, device=device)
        _check("pxs_batch_bind", lib.pxs_batch_bind(h, _dptr(self.table), _stream()))

    def footprint(self):
        """Device bytes of the buffers this batch allocated itself."""
        return sum(_nbytes(y[6]) for y in self.systems) + _nbytes(self.table)

    def run(self, tables, stream=None):
        """tables: per system (shifts (nshift,), weights (nsets, nshift)).
        Uploads them and replays the graph on `stream` (no wait)."""
        sh = np.concatenate([np.ascontiguousarray(t[0], dtype=np.complex128) for t in tables])
        wt = np.concatenate([np.ascontiguousarray(t[1], dtype=np.complex128).reshape(-1) for t in tables])
        _check("pxs_batch_run", self._lib.pxs_batch_run(self._h, _ptr(sh), _ptr(wt), _stream(stream)))

    def results(self, stream=None):
        """(list of traces (nsets, 2) per system, list of info per system)
        after synchronising `stream`."""
        n = len(self.systems)
        tr = np.zeros(2 * self.nsets * n)
        info = np.zeros(int(self.nshift.sum()), dtype=np.int64)
        _check("pxs_batch_results", self._lib.pxs_batch_results(self._h, _ptr(tr), _ptr(info), _stream(stream)),
               allow=(PXS_OK, PXS_TINY_PIVOT))
        tr = tr.reshape(n, self.nsets, 2)
        offs = np.concatenate([[0], np.cumsum(self.nshift)])
        return [tr[i] for i in range(n)], [info[offs[i]:offs[i + 1]] for i in range(n)]

    def outputs(self):
        """Per system the (nsets, nnz) pole-sum output tensor."""
        return [y[6].view(self.nsets, -1) for y in self.systems]

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                self._lib.pxs_batch_free(self._h)
                self._h = None
        except Exception:
            pass


def density_matrix_noalloc(analysis: Analysis, H, S, beta, dE, mu, P, nsets=2, L=None, out=None,
                           stream=None):
    """pxs_density_matrix_noalloc: the fused density matrix with the
    workspace in the library's device scratch array (no workspace
    argument).  L and out are caller buffers as for density_matrix.
    Returns (out (nsets, nnz), traces (nsets, 2), info, shifts, weights)."""
    import torch
    lib = load()
    analysis.bind()
    nnz = analysis.info["nnz_lower"]
    if L is None:
        L = torch.empty(P * analysis.info["bytes_per_shift"], dtype=torch.uint8, device=H.device)
    if out is None:
        out = torch.empty(nsets * nnz, dtype=torch.float64, device=H.device)
    _require_values(analysis, H, S)
    _require(L, P * analysis.info["bytes_per_shift"], "factor storage")
    _require(out, 8 * nsets * nnz, "pole-sum output")
    tr = np.zeros(2 * nsets)
    info = np.zeros(P, dtype=np.int64)
    sh = np.zeros(P, dtype=np.complex128)
    wt = np.zeros(nsets * P, dtype=np.complex128)
    code = lib.pxs_density_matrix_noalloc(analysis._h, _dptr(H), _dptr(S), beta, dE, mu, P, nsets, _dptr(L),
                                          _dptr(out), _ptr(tr), _ptr(info), _ptr(sh), _ptr(wt), _stream(stream))
    _check("pxs_density_matrix_noalloc", code, allow=(PXS_OK, PXS_TINY_PIVOT))
    return out.view(nsets, nnz), tr.reshape(nsets, 2), info, sh, wt.reshape(nsets, P)


KERNELS = {"update": 1, "selinv_off": 2, "trsm": 3, "selinv_diag": 4, "lhat": 5, "diag": 6,
           "assemble": 7, "pole_sum": 8, "gather": 9}


def profile_begin(kernel: str):
    """Starts HIP-event timing of one kernel class inside the library."""
    _check("pxs_profile_begin", load().pxs_profile_begin(KERNELS[kernel]))


def profile_end(with_bytes=False, with_stored=False):
    """Returns (total kernel ms, launches, algorithmic flops on the exact
    structure of L or bytes), plus the algorithmic HBM bytes when with_bytes
    is set and the flops on the stored structure when with_stored is set."""
    ms = C.c_double()
    n = C.c_int64()
    w = C.c_double()
    b = C.c_double()
    st = C.c_double()
    _check("pxs_profile_end", load().pxs_profile_end(C.byref(ms), C.byref(n), C.byref(w), C.byref(b),
                                                     C.byref(st)))
    out = (ms.value, n.value, w.value)
    if with_bytes:
        out += (b.value,)
    if with_stored:
        out += (st.value,)
    return out
