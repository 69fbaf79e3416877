"""Accuracy-controlled H^2 direct solver for AMD MI355X.

Thin ctypes binding of ``libh2mi.so`` (the C ABI declared in ``include/h2.h``):
argument marshalling only.  Every step of construction, factorization and the
sweeps runs in the library's gfx950 kernels; PyTorch provides device memory and
the stream.  The library is built in-tree by ``__graft_entry__.build()``; when
it is missing the binding raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libh2mi.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "h2.h")

H2_OK, H2_ERR_ARG, H2_ERR_OOM, H2_ERR_SINGULAR, H2_ERR_STATE, H2_ERR_DEVICE, H2_ERR_NOCONV, H2_ERR_INTERNAL = range(8)
STATUS_NAMES = ["H2_OK", "H2_ERR_ARG", "H2_ERR_OOM", "H2_ERR_SINGULAR", "H2_ERR_STATE", "H2_ERR_DEVICE",
                "H2_ERR_NOCONV", "H2_ERR_INTERNAL"]
H2_FP64, H2_MIXED = 0, 1
H2_BATCH_FUSED, H2_BATCH_STREAMS = 0, 1


class H2Error(RuntimeError):
    def __init__(self, status: int, message: str, call: str):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{call}: {name}: {message}")


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("precision", ctypes.c_int32), ("order", ctypes.c_int32),
                ("eps_fill", ctypes.c_double), ("forced_ranks", ctypes.POINTER(ctypes.c_int32)),
                ("forced_ranks_len", ctypes.c_int64), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_ctx", ctypes.c_void_p), ("stop_level", ctypes.c_int32)]


def _torch_alloc(nbytes, stream, ctx):
    """h2_options.alloc backed by PyTorch's caching allocator (NULL on failure)."""
    torch = _torch()
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:  # out of memory, or no device: the library reports H2_ERR_OOM
        return None


def _torch_free(ptr, stream, ctx):
    try:
        _torch().cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


# the C function pointers must outlive every handle that uses them
TORCH_ALLOCATOR = (ALLOC_FN(_torch_alloc), FREE_FN(_torch_free))


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("rel_residual_first", ctypes.c_double)]


TUNING_MAX_LEVELS = 64


class Tuning(ctypes.Structure):
    _fields_ = [("stop_level", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("split_below", ctypes.c_int64 * TUNING_MAX_LEVELS),
                ("mixed_flush", ctypes.c_int32 * TUNING_MAX_LEVELS),
                ("schur_chunk", ctypes.c_int32 * TUNING_MAX_LEVELS), ("factor_ms", ctypes.c_double)]


_lib = None
_P = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
_I64P = ctypes.POINTER(ctypes.c_int64)
_I32P = ctypes.POINTER(ctypes.c_int32)


def lib():
    """The loaded libh2mi; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.h2_build.argtypes = [_DP, ctypes.c_int64, ctypes.c_double, ctypes.c_double, _DP, ctypes.c_int32,
                               ctypes.c_double, ctypes.c_double, ctypes.POINTER(Options), _P, ctypes.POINTER(_P)]
        L.h2_factor.argtypes = [_P, _P]
        L.h2_solve.argtypes = [_P, _P, _P, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, _P,
                               ctypes.POINTER(SolveInfo)]
        L.h2_solve_noalloc.argtypes = [_P, _P, _P, ctypes.c_int32, ctypes.c_int64, _P]
        L.h2_solve_adjoint.argtypes = [_P, _P, _P, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, _P,
                                       ctypes.POINTER(SolveInfo)]
        L.h2_contrast_gradient.argtypes = [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int64, _P, _P]
        L.h2_set_contrast.argtypes = [_P, _DP, _P]
        L.h2_set_precision.argtypes = [_P, ctypes.c_int32]
        L.h2_set_sweep_graph.argtypes = [_P, ctypes.c_int32]
        L.h2_factor_batch.argtypes = [ctypes.POINTER(_P), ctypes.c_int32, _P]
        L.h2_factor_batch_mode.argtypes = [ctypes.POINTER(_P), ctypes.c_int32, _P, ctypes.c_int32]
        L.h2_solve_batch.argtypes = [ctypes.POINTER(_P), ctypes.c_int32, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                     ctypes.c_int32, _I64P, ctypes.c_double, ctypes.c_int32, _P,
                                     ctypes.POINTER(SolveInfo)]
        L.h2_solve_batch_mode.argtypes = [ctypes.POINTER(_P), ctypes.c_int32, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                          ctypes.c_int32, _I64P, ctypes.c_double, ctypes.c_int32, _P,
                                          ctypes.POINTER(SolveInfo), ctypes.c_int32]
        L.h2_matvec.argtypes = [_P, _P, _P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _P]
        L.h2_destroy.argtypes = [_P]
        L.h2_destroy.restype = None
        L.h2_last_error.argtypes = []
        L.h2_last_error.restype = ctypes.c_char_p
        L.h2_structure.argtypes = [_DP, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, ctypes.c_double, _I64P,
                                   _I64P, _I32P]
        L.h2_schur_schedule.argtypes = [_DP, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_int32, _I32P, _I64P, ctypes.c_int64, _I64P]
        L.h2_merge_schedule.argtypes = [_DP, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_int32, _I64P, ctypes.c_int64, _I64P]
        L.h2_stats.argtypes = [_P, _I64P, ctypes.c_int32, _I32P]
        L.h2_forced_ranks_layout.argtypes = [_P, _I32P, ctypes.c_int64, _I64P]
        L.h2_factor_timing.argtypes = [_P, _DP, ctypes.c_int32]
        L.h2_set_kernel_timing.argtypes = [_P, ctypes.c_int32]
        L.h2_kernel_ledger.argtypes = [_P, _DP, ctypes.c_int32]
        L.h2_level_timing.argtypes = [_P, _DP, ctypes.c_int32, _I32P]
        L.h2_set_stop_level.argtypes = [_P, ctypes.c_int32]
        L.h2_stop_level.argtypes = [_P, _I32P]
        L.h2_tune_stop_level.argtypes = [_P, ctypes.c_int64, _P, _I32P, _DP, ctypes.c_int32]
        L.h2_set_schur_split.argtypes = [_P, ctypes.c_int32, ctypes.c_int64]
        L.h2_set_mixed_flush.argtypes = [_P, ctypes.c_int32, ctypes.c_int32]
        L.h2_set_schur_chunk.argtypes = [_P, ctypes.c_int32, ctypes.c_int32]
        L.h2_tune.argtypes = [_P, ctypes.c_int64, _P, ctypes.POINTER(Tuning)]
        L.h2_tune_cache_clear.argtypes = []
        for name in ("h2_build", "h2_factor", "h2_solve", "h2_solve_adjoint", "h2_matvec", "h2_structure",
                     "h2_schur_schedule", "h2_merge_schedule",
                     "h2_stats", "h2_forced_ranks_layout", "h2_factor_timing", "h2_contrast_gradient",
                     "h2_set_contrast", "h2_set_precision", "h2_set_sweep_graph", "h2_factor_batch",
                     "h2_factor_batch_mode", "h2_solve_batch_mode",
                     "h2_solve_batch", "h2_set_kernel_timing", "h2_kernel_ledger", "h2_level_timing",
                     "h2_solve_noalloc", "h2_set_stop_level", "h2_stop_level", "h2_tune_stop_level",
                     "h2_set_schur_split", "h2_set_mixed_flush", "h2_set_schur_chunk", "h2_tune",
                     "h2_tune_cache_clear"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def declared_functions() -> list:
    """Function names declared by include/h2.h."""
    with open(HEADER) as f:
        src = f.read()
    return sorted(set(re.findall(r"^\s*(?:h2_status|void|const char\*)\s+(h2_\w+)\s*\(", src, re.M)))


def _check(status: int, call: str):
    if status != H2_OK:
        raise H2Error(status, lib().h2_last_error().decode(errors="replace"), call)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_DP)


def structure(points, h: float, leaf: int, eta: float) -> dict:
    """Host-only tree / partition / colouring summary (no device touched)."""
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    n = pts.shape[0]
    counts = np.zeros(8, np.int64)
    perm = np.zeros(n, np.int64)
    _check(lib().h2_structure(_dptr(pts), n, float(h), int(leaf), float(eta), counts.ctypes.data_as(_I64P),
                              perm.ctypes.data_as(_I64P), None), "h2_structure")
    cols = np.zeros(int(counts[3]), np.int32)
    _check(lib().h2_structure(_dptr(pts), n, float(h), int(leaf), float(eta), counts.ctypes.data_as(_I64P), None,
                              cols.ctypes.data_as(_I32P)), "h2_structure")
    keys = ["N", "L", "l0", "leaves", "leaf_min", "leaf_max", "adm_leaf", "near_leaf"]
    out = {k: int(v) for k, v in zip(keys, counts)}
    out["perm"] = perm
    out["colours"] = cols
    return out


def schur_schedule(points, h: float, leaf: int, eta: float, level: int) -> tuple:
    """Host-only deferred Schur updates of one level (no device touched): (number of
    colours, int64 array of (event, a, b, i) rows in flush order)."""
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    n = pts.shape[0]
    ncol = ctypes.c_int32(0)
    cnt = ctypes.c_int64(0)
    _check(lib().h2_schur_schedule(_dptr(pts), n, float(h), int(leaf), float(eta), int(level), ctypes.byref(ncol),
                                   None, 0, ctypes.byref(cnt)), "h2_schur_schedule")
    out = np.zeros((int(cnt.value), 4), np.int64)
    _check(lib().h2_schur_schedule(_dptr(pts), n, float(h), int(leaf), float(eta), int(level), ctypes.byref(ncol),
                                   out.ctypes.data_as(_I64P), out.size, ctypes.byref(cnt)), "h2_schur_schedule")
    return int(ncol.value), out


def merge_schedule(points, h: float, leaf: int, eta: float, level: int) -> np.ndarray:
    """Host-only merge of one level's blocks into its parent level (no device touched):
    int64 rows (parent row, parent column, ci, dj, kind, a, b)."""
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    n = pts.shape[0]
    cnt = ctypes.c_int64(0)
    _check(lib().h2_merge_schedule(_dptr(pts), n, float(h), int(leaf), float(eta), int(level), None, 0,
                                   ctypes.byref(cnt)), "h2_merge_schedule")
    out = np.zeros((int(cnt.value), 7), np.int64)
    _check(lib().h2_merge_schedule(_dptr(pts), n, float(h), int(leaf), float(eta), int(level),
                                   out.ctypes.data_as(_I64P), out.size, ctypes.byref(cnt)), "h2_merge_schedule")
    return out


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _as_cols(x, n: int):
    """complex128 device tensor -> (column-major buffer (nrhs, n) contiguous, nrhs, was_vector)."""
    torch = _torch()
    if not isinstance(x, torch.Tensor):
        x = torch.as_tensor(np.asarray(x))
    x = x.to(device="cuda", dtype=torch.complex128)
    vec = x.dim() == 1
    if vec:
        x = x.reshape(n, 1)
    if x.shape[0] != n:
        raise ValueError(f"expected {n} rows, got {tuple(x.shape)}")
    return x.t().contiguous(), x.shape[1], vec


def _from_cols(buf, vec: bool):
    return buf[0] if vec else buf.t()


class H2:
    """An H^2 representation of the VIE matrix A = Z D on the device, and its factorization.

    Parameters follow h2_build: cell centres ``points`` (N x 3), wavenumber ``k``,
    cell size ``h``, per-cell contrast ``chi`` (> 0), leaf size, admissibility
    ``eta`` and construction accuracy ``eps``; ``eps_fill`` (default eps) controls
    the basis updates of the factorization; ``forced_ranks`` pins rank decisions
    (the format of :meth:`forced_ranks`).
    """

    def __init__(self, points, k, h, chi, leaf, eta, eps, eps_fill=None, precision="fp64", forced_ranks=None,
                 stream=None, allocator="torch", stop_level=0):
        pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
        chi = np.ascontiguousarray(chi, dtype=np.float64).reshape(-1)
        self._points = pts
        self.n = pts.shape[0]
        self.k, self.h, self.leaf, self.eta, self.eps = float(k), float(h), int(leaf), float(eta), float(eps)
        self.chi = chi.copy()
        self._forced = None
        opt = Options()
        opt.struct_size = ctypes.sizeof(Options)
        opt.precision = H2_MIXED if precision == "mixed" else H2_FP64
        opt.order = 0
        opt.eps_fill = float(eps_fill) if eps_fill else 0.0
        opt.stop_level = int(stop_level or 0)
        if forced_ranks is not None:
            self._forced = np.ascontiguousarray(forced_ranks, dtype=np.int32).reshape(-1)
            opt.forced_ranks = self._forced.ctypes.data_as(_I32P)
            opt.forced_ranks_len = self._forced.size
        # device memory: PyTorch's caching allocator ("torch"), the library's own hipMalloc
        # (None), or a pair of ctypes callbacks (ALLOC_FN, FREE_FN)
        if allocator == "torch":
            allocator = TORCH_ALLOCATOR
        self._allocator = allocator
        if allocator is not None:
            opt.alloc, opt.free = allocator
        self._h = ctypes.c_void_p()
        st = _stream_ptr(stream)
        _check(lib().h2_build(_dptr(pts), self.n, self.k, self.h, _dptr(chi), self.leaf, self.eta, self.eps,
                              ctypes.byref(opt), st, ctypes.byref(self._h)), "h2_build")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().h2_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_precision(self, precision: str):
        """"fp64" or "mixed" for the next factorization (the handle becomes unfactored)."""
        if precision not in ("fp64", "mixed"):
            raise ValueError(precision)
        _check(lib().h2_set_precision(self._h, H2_MIXED if precision == "mixed" else H2_FP64), "h2_set_precision")
        return self

    def set_stop_level(self, level: int = 0):
        """Last factored level of later factorizations (0: l0); the handle becomes unfactored."""
        _check(lib().h2_set_stop_level(self._h, int(level)), "h2_set_stop_level")
        return self

    def stop_level(self) -> int:
        out = ctypes.c_int32()
        _check(lib().h2_stop_level(self._h, ctypes.byref(out)), "h2_stop_level")
        return out.value

    def tune_stop_level(self, max_final: int = 12288, stream=None):
        """Pick the fastest stop level by factoring with each candidate (h2_tune_stop_level);
        returns (chosen level, {level: factor ms}) and leaves the handle factored."""
        ms = np.full(64, -1.0)
        chosen = ctypes.c_int32()
        _check(lib().h2_tune_stop_level(self._h, int(max_final), _stream_ptr(stream), ctypes.byref(chosen),
                                        _dptr(ms), ms.size), "h2_tune_stop_level")
        base = self.stop_level_range()[0]
        return chosen.value, {base + e: float(t) for e, t in enumerate(ms) if t >= 0}

    def set_schur_split(self, below_wgs: int, level: int = -1):
        """Schur flush split threshold in workgroups at `level` (-1: every level; below_wgs -1:
        the default, 0: never split) (h2_set_schur_split)."""
        _check(lib().h2_set_schur_split(self._h, int(level), int(below_wgs)), "h2_set_schur_split")
        return self

    def tune(self, max_final: int = 12288, stream=None) -> dict:
        """Autotune the stop level and the per-level Schur split threshold (h2_tune, cached per
        problem structure); leaves the handle factored with the chosen settings."""
        t = Tuning()
        _check(lib().h2_tune(self._h, int(max_final), _stream_ptr(stream), ctypes.byref(t)), "h2_tune")
        split = {l: int(v) for l, v in enumerate(t.split_below) if v >= 0}
        out = {"stop_level": t.stop_level, "from_cache": bool(t.from_cache), "split_below": split,
               "factor_ms": t.factor_ms}
        mflush = {l: int(v) for l, v in enumerate(t.mixed_flush) if v >= 0}
        if mflush:
            out["mixed_flush"] = mflush
        out["schur_chunk"] = {l: int(v) for l, v in enumerate(t.schur_chunk) if v > 0}
        return out

    def set_schur_chunk(self, terms: int, level: int = -1):
        """Terms per chunk of split Schur tasks at `level` (-1: every level; terms -1: the
        default) (h2_set_schur_chunk)."""
        _check(lib().h2_set_schur_chunk(self._h, int(level), int(terms)), "h2_set_schur_chunk")
        return self

    def set_mixed_flush(self, mode: int, level: int = -1):
        """Mixed form: the Schur flush kernel at `level` (-1: every level): 1 FP32 routing,
        0 every term in FP64, -1 the default rule (h2_set_mixed_flush)."""
        _check(lib().h2_set_mixed_flush(self._h, int(level), int(mode)), "h2_set_mixed_flush")
        return self

    def stop_level_range(self):
        """(l0, L) of the handle's block tree."""
        st = structure(self._points, self.h, self.leaf, self.eta)
        return st["l0"], st["L"]

    def set_sweep_graph(self, enable: bool = True):
        """Replay the solve sweeps from captured HIP graphs."""
        _check(lib().h2_set_sweep_graph(self._h, 1 if enable else 0), "h2_set_sweep_graph")
        return self

    def factor(self, stream=None):
        _check(lib().h2_factor(self._h, _stream_ptr(stream)), "h2_factor")
        return self

    def solve(self, b, tol=0.0, max_iter=20, stream=None, info=False):
        buf, nrhs, vec = _as_cols(b, self.n)
        out = _torch().empty_like(buf)
        si = SolveInfo()
        _check(lib().h2_solve(self._h, ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(out.data_ptr()), nrhs,
                              self.n, float(tol), int(max_iter), _stream_ptr(stream), ctypes.byref(si)), "h2_solve")
        x = _from_cols(out, vec)
        if info:
            return x, {"iterations": si.iterations, "rel_residual": si.rel_residual,
                       "rel_residual_first": si.rel_residual_first}
        return x

    def solve_noalloc(self, b, stream=None):
        """x = M^-1 b through h2_solve_noalloc (the library allocates no device memory;
        its work space is a fixed 64 MiB array per device)."""
        buf, nrhs, vec = _as_cols(b, self.n)
        out = _torch().empty_like(buf)
        _check(lib().h2_solve_noalloc(self._h, ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                      nrhs, self.n, _stream_ptr(stream)), "h2_solve_noalloc")
        return _from_cols(out, vec)

    def solve_adjoint(self, g, tol=0.0, max_iter=20, stream=None, info=False):
        buf, nrhs, vec = _as_cols(g, self.n)
        out = _torch().empty_like(buf)
        si = SolveInfo()
        _check(lib().h2_solve_adjoint(self._h, ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                      nrhs, self.n, float(tol), int(max_iter), _stream_ptr(stream), ctypes.byref(si)),
               "h2_solve_adjoint")
        lam = _from_cols(out, vec)
        if info:
            return lam, {"iterations": si.iterations, "rel_residual": si.rel_residual,
                         "rel_residual_first": si.rel_residual_first}
        return lam

    def contrast_gradient(self, x, g, lam, stream=None):
        """dL/dchi (float64 device tensor, caller order) from x, g = dL/d conj(x) and lam = A^-H g."""
        xb, nrhs, _ = _as_cols(x, self.n)
        gb, nrhs_g, _ = _as_cols(g, self.n)
        lb, nrhs_l, _ = _as_cols(lam, self.n)
        if not (nrhs == nrhs_g == nrhs_l):
            raise ValueError("x, g and lam need the same number of columns")
        out = _torch().empty(self.n, dtype=_torch().float64, device="cuda")
        _check(lib().h2_contrast_gradient(self._h, ctypes.c_void_p(xb.data_ptr()), ctypes.c_void_p(gb.data_ptr()),
                                          ctypes.c_void_p(lb.data_ptr()), nrhs, self.n,
                                          ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
               "h2_contrast_gradient")
        return out

    def set_contrast(self, chi, stream=None):
        """New per-cell contrast (host values); the handle must be factored again."""
        chi = np.ascontiguousarray(chi, dtype=np.float64).reshape(-1)
        if chi.size != self.n:
            raise ValueError(f"expected {self.n} contrast values, got {chi.size}")
        _check(lib().h2_set_contrast(self._h, _dptr(chi), _stream_ptr(stream)), "h2_set_contrast")
        self.chi = chi.copy()
        return self

    def matvec(self, x, adjoint=False, stream=None):
        buf, nrhs, vec = _as_cols(x, self.n)
        out = _torch().empty_like(buf)
        _check(lib().h2_matvec(self._h, ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(out.data_ptr()), nrhs,
                               self.n, 1 if adjoint else 0, _stream_ptr(stream)), "h2_matvec")
        return _from_cols(out, vec)

    def stats(self) -> np.ndarray:
        rows = ctypes.c_int32()
        buf = np.zeros(64 * 10, np.int64)
        _check(lib().h2_stats(self._h, buf.ctypes.data_as(_I64P), 64, ctypes.byref(rows)), "h2_stats")
        return buf[:rows.value * 10].reshape(-1, 10)

    def forced_ranks(self) -> np.ndarray:
        cnt = ctypes.c_int64()
        _check(lib().h2_forced_ranks_layout(self._h, None, 0, ctypes.byref(cnt)), "h2_forced_ranks_layout")
        out = np.zeros(4 * cnt.value, np.int32)
        _check(lib().h2_forced_ranks_layout(self._h, out.ctypes.data_as(_I32P), cnt.value, ctypes.byref(cnt)),
               "h2_forced_ranks_layout")
        return out.reshape(-1, 4)

    def timing(self, ledger: bool = True) -> np.ndarray:
        """[total, steps 0-2, LU + panels, Schur, merges, final LU] ms of the last
        factorization, then (ledger=True) its algorithmic ledger: Schur flops,
        Schur launches, factor flops, Schur bytes (computed on the host on first request)."""
        out = np.zeros(10 if ledger else 6)
        _check(lib().h2_factor_timing(self._h, _dptr(out), out.size), "h2_factor_timing")
        return out

    def level_timing(self) -> np.ndarray:
        """Milliseconds of each factored level of the last factorization (rows of
        :meth:`stats`, the final dense LU last)."""
        cnt = ctypes.c_int32()
        _check(lib().h2_level_timing(self._h, None, 0, ctypes.byref(cnt)), "h2_level_timing")
        out = np.zeros(max(cnt.value, 1))
        _check(lib().h2_level_timing(self._h, _dptr(out), out.size, ctypes.byref(cnt)), "h2_level_timing")
        return out[:cnt.value]

    def set_kernel_timing(self, enable: bool = True):
        """Time every kernel family of later factorizations with HIP events (diagnostics)."""
        _check(lib().h2_set_kernel_timing(self._h, 1 if enable else 0), "h2_set_kernel_timing")
        return self

    def kernel_ledger(self) -> dict:
        """{family: (ms, flops, bytes)} of the last factorization (h2_kernel_ledger; ms is -1
        when kernel timing was off), plus the bytes one right-hand side's sweeps and one
        matvec must read."""
        out = np.zeros(27)
        _check(lib().h2_kernel_ledger(self._h, _dptr(out), out.size), "h2_kernel_ledger")
        d = {f: (out[3 * i], out[3 * i + 1], out[3 * i + 2]) for i, f in enumerate(KERNEL_FAMILIES)}
        d["sweep_bytes_per_rhs"] = out[24]
        d["matvec_bytes"] = out[25]
        d["schur_fp32_flop_frac"] = out[26]
        return d


KERNEL_FAMILIES = ("gram_fill", "step0_basis", "projection", "partial_lu", "panels", "schur", "merge", "final_lu")


def forced_ranks_from_oracle(construct_ranks: dict, factor_ranks: dict) -> np.ndarray:
    """(level, cluster, k, k~) rows from {(l, t): k} and {(l, i): k~} dictionaries, in the
    library's order (finest level first, clusters ascending)."""
    keys = sorted(construct_ranks, key=lambda lt: (-lt[0], lt[1]))
    rows = [(l, t, construct_ranks[(l, t)], factor_ranks.get((l, t), -1)) for (l, t) in keys]
    return np.asarray(rows, dtype=np.int32).reshape(-1, 4)


def tune_cache_clear():
    """Empty the autotuner's process-wide cache (h2_tune_cache_clear)."""
    _check(lib().h2_tune_cache_clear(), "h2_tune_cache_clear")


def factor_batch(solvers, stream=None, mode="fused"):
    """Factor several independent :class:`H2` handles together (h2_factor_batch_mode):
    mode "fused" launches each colour stage once for all problems, "streams" gives each
    handle a stream of its own."""
    modes = {"fused": H2_BATCH_FUSED, "streams": H2_BATCH_STREAMS}
    if mode not in modes:
        raise ValueError(f"mode must be one of {sorted(modes)}")
    arr = (_P * len(solvers))(*[sv._h.value for sv in solvers])
    _check(lib().h2_factor_batch_mode(arr, len(solvers), _stream_ptr(stream), modes[mode]), "h2_factor_batch_mode")
    return solvers


def solve_batch(solvers, rhs, tol=0.0, max_iter=20, stream=None, info=False, mode="fused"):
    """x_k = M_k^-1 b_k for every handle (h2_solve_batch_mode); every b_k has the same number of
    columns.  mode "fused" runs the sweeps of all problems in shared launches, "streams" gives
    each handle a stream of its own."""
    modes = {"fused": H2_BATCH_FUSED, "streams": H2_BATCH_STREAMS}
    if mode not in modes:
        raise ValueError(f"mode must be one of {sorted(modes)}")
    torch = _torch()
    bufs, outs, nrhs = [], [], None
    for sv, b in zip(solvers, rhs):
        buf, nr, vec = _as_cols(b, sv.n)
        if nrhs is None:
            nrhs = nr
        elif nr != nrhs:
            raise ValueError("every right-hand side needs the same number of columns")
        bufs.append((buf, vec))
        outs.append(torch.empty_like(buf))
    cnt = len(solvers)
    hs = (_P * cnt)(*[sv._h.value for sv in solvers])
    bp = (_P * cnt)(*[b.data_ptr() for b, _ in bufs])
    xp = (_P * cnt)(*[o.data_ptr() for o in outs])
    ld = np.ascontiguousarray([sv.n for sv in solvers], dtype=np.int64)
    infos = (SolveInfo * cnt)()
    _check(lib().h2_solve_batch_mode(hs, cnt, bp, xp, nrhs, ld.ctypes.data_as(_I64P), float(tol), int(max_iter),
                                     _stream_ptr(stream), infos, modes[mode]), "h2_solve_batch_mode")
    xs = [_from_cols(o, vec) for o, (_, vec) in zip(outs, bufs)]
    if info:
        return xs, [{"iterations": i.iterations, "rel_residual": i.rel_residual,
                     "rel_residual_first": i.rel_residual_first} for i in infos]
    return xs
