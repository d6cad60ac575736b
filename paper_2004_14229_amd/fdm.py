"""Thin Python binding of the C ABI in ``include/fdm.h`` (argument marshalling
only; every step of the method runs in the gfx950 library ``libfdm.so``).

Torch is used for device memory and streams: points and vectors are CUDA
(HIP) tensors, and calls are enqueued on ``torch.cuda.current_stream()``
unless a stream is given.  If the library is missing this module raises; it
never falls back to another implementation.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfdm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "fdm.h")

FDM_OK = 0
STATUS = {0: "FDM_OK", -1: "FDM_ERR_INVALID_ARG", -2: "FDM_ERR_POINT_OUTSIDE_BOX",
          -3: "FDM_ERR_UNSUPPORTED", -4: "FDM_ERR_OUT_OF_MEMORY", -5: "FDM_ERR_HIP",
          -6: "FDM_ERR_STATE"}
PRECISION = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}

_lib = None


class FdmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Tune(ctypes.Structure):
    """fdm_tune: nb, persistent, lpt, p2p_in_queue, compact (0 never, 1
    items that save a fifth of their columns, 2 every item)."""
    _fields_ = [("nb", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("lpt", ctypes.c_int32), ("p2p_in_queue", ctypes.c_int32),
                ("compact", ctypes.c_int32)]
    DEFAULTS = {"nb": 64, "persistent": 1, "lpt": 1, "p2p_in_queue": 0, "compact": 1}

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}

    @classmethod
    def from_dict(cls, d: dict, precision: str = "fp64") -> "Tune":
        """Fields missing from d take the library's defaults (32 targets per
        item for the six-product BF16 split, 64 otherwise)."""
        defaults = dict(cls.DEFAULTS, nb=32 if precision == "bf16x6" else 64)
        return cls(*(int(d.get(name, defaults[name])) for name, _ in cls._fields_))


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("l_hf", ctypes.c_int32),
                ("bank_budget_bytes", ctypes.c_int64), ("tune", Tune),
                ("full_bank", ctypes.c_int32), ("aca_rank", ctypes.c_int32),
                ("aca_eps", ctypes.c_double), ("aca_chunk_bytes", ctypes.c_int64),
                ("n_max", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("n_T", ctypes.c_int64), ("n_S", ctypes.c_int64),
                ("levels", ctypes.c_int32), ("m", ctypes.c_int32),
                ("K", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("l_hf", ctypes.c_int32), ("l_min", ctypes.c_int32),
                ("n_couplings", ctypes.c_int64), ("n_stored_couplings", ctypes.c_int64),
                ("n_bank_matrices", ctypes.c_int64), ("near_pairs", ctypes.c_int64),
                ("near_entries", ctypes.c_int64), ("m2l_columns", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("setup_ms", ctypes.c_double),
                ("aca_rank_cap", ctypes.c_int32), ("aca_rank_max", ctypes.c_int32),
                ("aca_rank_mean", ctypes.c_double), ("aca_flops", ctypes.c_double),
                ("aca_issued_flops", ctypes.c_double)]


def header_functions() -> list[str]:
    """Names of the functions declared in include/fdm.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(fdm_\w+)\s*\(", text, re.M)))


def lib() -> ctypes.CDLL:
    """Load ``libfdm.so`` (built by ``paper_2004_14229_amd/build.py``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python paper_2004_14229_amd/build.py`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    L.fdm_build_tree.argtypes = [vp, i64, vp, i64, dbl, ctypes.POINTER(dbl), ci, ci, ci,
                                 vp, ctypes.POINTER(vp)]
    L.fdm_build_tree_ex.argtypes = [vp, i64, vp, i64, dbl, ctypes.POINTER(dbl), ci, ci, ci,
                                    ci, vp, ctypes.POINTER(vp)]
    L.fdm_plan_matvec.argtypes = [vp, vp, vp, vp]
    L.fdm_plan_matvec_c64.argtypes = [vp, vp, vp, vp]
    L.fdm_plan_matvec_noalloc.argtypes = [vp, vp, vp, ci, vp]
    L.fdm_plan_matvec_multi.argtypes = [vp, vp, vp, ci, ci, vp]
    L.fdm_plan_destroy.argtypes = [vp]
    L.fdm_plan_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.fdm_plan_export.argtypes = [vp, ctypes.c_char_p, vp, i64, ctypes.POINTER(i64)]
    L.fdm_dense_matvec.argtypes = [vp, i64, vp, i64, dbl, vp, vp, vp]
    L.fdm_plan_set_timing.argtypes = [vp, ci]
    L.fdm_plan_phase_ms.argtypes = [vp, ctypes.POINTER(dbl)]
    L.fdm_plan_prepare.argtypes = [vp, vp]
    L.fdm_plan_coupling_launches.argtypes = [vp, ctypes.POINTER(ci)]
    L.fdm_plan_wait_launch.argtypes = [vp, ci, ctypes.POINTER(dbl)]
    L.fdm_build_tree_opts.argtypes = [vp, i64, vp, i64, dbl, ctypes.POINTER(dbl), ci, ci,
                                      ctypes.POINTER(Options), vp, ctypes.POINTER(vp)]
    L.fdm_plan_get_tune.argtypes = [vp, ctypes.POINTER(Tune)]
    L.fdm_plan_set_tune.argtypes = [vp, ctypes.POINTER(Tune), vp]
    L.fdm_plan_autotune.argtypes = [vp, vp, vp, ci, ci, vp, ctypes.POINTER(Tune),
                                    ctypes.POINTER(dbl)]
    L.fdm_batch_create.argtypes = [ctypes.POINTER(vp), ci, i64, vp, ctypes.POINTER(vp)]
    L.fdm_batch_matvec.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ci, vp]
    L.fdm_batch_set_graph.argtypes = [vp, ci]
    L.fdm_batch_get_tune.argtypes = [vp, ctypes.POINTER(Tune)]
    L.fdm_batch_set_tune.argtypes = [vp, ctypes.POINTER(Tune), vp]
    L.fdm_batch_autotune.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ci, ci, vp,
                                     ctypes.POINTER(Tune), ctypes.POINTER(dbl)]
    L.fdm_batch_destroy.argtypes = [vp]
    L.fdm_aca.argtypes = [vp, ci, ci, dbl, ci, vp, vp, ctypes.POINTER(ci)]
    L.fdm_last_error.restype = ctypes.c_char_p
    L.fdm_version.restype = ctypes.c_char_p
    for f in ("fdm_build_tree", "fdm_build_tree_ex", "fdm_build_tree_opts", "fdm_plan_matvec",
              "fdm_plan_matvec_c64", "fdm_plan_matvec_noalloc", "fdm_plan_matvec_multi",
              "fdm_plan_destroy",
              "fdm_plan_stats",
              "fdm_plan_export", "fdm_dense_matvec", "fdm_plan_set_timing",
              "fdm_plan_phase_ms", "fdm_plan_get_tune", "fdm_plan_set_tune",
              "fdm_plan_prepare", "fdm_plan_coupling_launches", "fdm_plan_wait_launch",
              "fdm_plan_autotune", "fdm_batch_create", "fdm_batch_matvec",
              "fdm_batch_set_graph", "fdm_batch_get_tune", "fdm_batch_set_tune",
              "fdm_batch_autotune", "fdm_batch_destroy", "fdm_aca"):
        getattr(L, f).restype = ci
    _lib = L
    return L


def _check(status: int) -> None:
    if status != FDM_OK:
        raise FdmError(status, lib().fdm_last_error().decode())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class _OnStream:
    """Runs a library call on ``stream`` (None: the current stream).

    With a stream other than the current one: the stream first waits for
    the work already queued on the current stream (so inputs written there
    are complete), tensors made inside the block are allocated on the given
    stream, and every tensor passed to ``keep`` is marked as used by that
    stream, so that torch's caching allocator does not hand its memory to
    other work before the library's kernels are done with it."""

    def __init__(self, stream):
        self.stream, self._ctx = None, None
        if stream is not None:
            import torch
            cur = torch.cuda.current_stream()
            if stream != cur:
                self.stream = stream
                stream.wait_stream(cur)
                self._ctx = torch.cuda.stream(stream)

    def __enter__(self):
        if self._ctx is not None:
            self._ctx.__enter__()
        return self

    def __exit__(self, *exc):
        if self._ctx is not None:
            self._ctx.__exit__(*exc)

    def handle(self):
        return _stream_handle(self.stream)

    def keep(self, *tensors):
        if self.stream is not None:
            for t in tensors:
                if t is not None and t.numel():
                    t.record_stream(self.stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() else 0)


def _points(p):
    import torch
    if not isinstance(p, torch.Tensor) or not p.is_cuda:
        raise TypeError("points must be a CUDA tensor")
    if p.dtype != torch.float64 or p.dim() != 2 or p.shape[1] != 3:
        raise TypeError("points must be an (n, 3) float64 tensor")
    return p.contiguous()


class Plan:
    """A built plan of the fast directional matvec (wraps ``fdm_plan*``)."""

    def __init__(self, points_T, points_S, kappa: float, box, levels: int, m: int,
                 precision: str = "fp64", l_hf: int | None = None, stream=None,
                 bank_budget: int = 0, tune: dict | None = None, full_bank: bool = False,
                 aca_eps: float = 0.0, aca_rank: int = 0, aca_chunk_bytes: int = 0,
                 n_max: int = 0):
        box_arr = (ctypes.c_double * 6)(*[float(b) for b in box])
        opts = Options(PRECISION[precision], -2 if l_hf is None else int(l_hf),
                       int(bank_budget), Tune.from_dict(tune, precision) if tune else Tune(),
                       int(bool(full_bank)), int(aca_rank), float(aca_eps),
                       int(aca_chunk_bytes), int(n_max))
        h = ctypes.c_void_p()
        # the library synchronises the stream before returning
        with _OnStream(stream) as on:
            pt, ps = _points(points_T), _points(points_S)
            st = lib().fdm_build_tree_opts(
                _ptr(pt), pt.shape[0], _ptr(ps), ps.shape[0], float(kappa), box_arr,
                int(levels), int(m), ctypes.byref(opts), on.handle(), ctypes.byref(h))
        _check(st)
        self._h = h
        self.n_T, self.n_S = pt.shape[0], ps.shape[0]
        self.precision = precision

    def _vectors(self, v, out):
        """Checks v (n_S) and out (n_T) before any pointer reaches the
        library, which cannot see sizes."""
        import torch
        if not isinstance(v, torch.Tensor) or not v.is_cuda:
            raise TypeError("v must be a CUDA tensor")
        if v.dtype not in (torch.complex128, torch.complex64) or v.shape != (self.n_S,):
            raise TypeError("v must be a complex128/complex64 vector of length n_S")
        v = v.contiguous()
        if out is None:
            out = torch.empty(self.n_T, dtype=v.dtype, device=v.device)
        elif (not isinstance(out, torch.Tensor) or not out.is_cuda or out.dtype != v.dtype
              or out.shape != (self.n_T,) or not out.is_contiguous()):
            raise TypeError("out must be a contiguous CUDA vector of length n_T, same dtype as v")
        return v, out

    def matvec(self, v, out=None, stream=None):
        """``y = A~ v`` (complex128, or complex64 in and out)."""
        import torch
        with _OnStream(stream) as on:
            v, out = self._vectors(v, out)
            fn = lib().fdm_plan_matvec if v.dtype == torch.complex128 else lib().fdm_plan_matvec_c64
            _check(fn(self._h, _ptr(v), _ptr(out), on.handle()))
            on.keep(v, out)
        return out

    def matvec_multi(self, V, out=None, stream=None):
        """``Y = A~ V`` for the rows of V (nrhs x n_S, complex128 or complex64,
        one right-hand side per row); returns Y (nrhs x n_T)."""
        import torch
        if not isinstance(V, torch.Tensor) or not V.is_cuda or V.dim() != 2:
            raise TypeError("V must be a 2-D CUDA tensor (nrhs x n_S)")
        if V.dtype not in (torch.complex128, torch.complex64) or V.shape[1] != self.n_S:
            raise TypeError("V must be complex128/complex64 with n_S columns")
        V = V.contiguous()
        nrhs = V.shape[0]
        if out is None:
            out = torch.empty(nrhs, self.n_T, dtype=V.dtype, device=V.device)
        elif (not isinstance(out, torch.Tensor) or not out.is_cuda or out.dtype != V.dtype
              or out.shape != (nrhs, self.n_T) or not out.is_contiguous()):
            raise TypeError("out must be a contiguous CUDA tensor nrhs x n_T, same dtype as V")
        with _OnStream(stream) as on:
            _check(lib().fdm_plan_matvec_multi(self._h, _ptr(V), _ptr(out), int(nrhs),
                                               int(V.dtype == torch.complex64), on.handle()))
            on.keep(V, out)
        return out

    def matvec_noalloc(self, v, out, stream=None):
        """``out = A~ v`` with the streamed coupling bank in the library's
        static workspace (``fdm_plan_matvec_noalloc``): the library allocates
        nothing; ``out`` must be given.  The plan must have been prepared."""
        import torch
        if out is None:
            raise TypeError("out must be given (nothing is allocated)")
        with _OnStream(stream) as on:
            v, out = self._vectors(v, out)
            _check(lib().fdm_plan_matvec_noalloc(self._h, _ptr(v), _ptr(out),
                                                 int(v.dtype == torch.complex64), on.handle()))
            on.keep(v, out)
        return out

    def stats(self) -> dict:
        s = Stats()
        _check(lib().fdm_plan_stats(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in Stats._fields_}

    def export(self, name: str) -> np.ndarray:
        size = ctypes.c_int64()
        _check(lib().fdm_plan_export(self._h, name.encode(), None, 0, ctypes.byref(size)))
        is_f64 = name.startswith(("dirs_", "mom_", "loc_"))
        buf = np.zeros(size.value // 8, dtype=np.float64 if is_f64 else np.int64)
        if size.value:
            _check(lib().fdm_plan_export(self._h, name.encode(), buf.ctypes.data_as(ctypes.c_void_p),
                                         size.value, ctypes.byref(size)))
        if name.startswith(("mom_", "loc_")):
            return buf.view(np.complex128)
        if name.startswith("dirs_"):
            return buf.reshape(-1, 3)
        if name.startswith("off_"):
            return buf.reshape(-1, 3)
        return buf

    def get_tune(self) -> dict:
        t = Tune()
        _check(lib().fdm_plan_get_tune(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tune(self, tune: dict, stream=None) -> None:
        t = Tune.from_dict({**self.get_tune(), **tune})
        _check(lib().fdm_plan_set_tune(self._h, ctypes.byref(t), _stream_handle(stream)))

    def autotune(self, v, out=None, max_candidates: int = 8, stream=None):
        """Time the coupling step under each launch shape and keep the
        fastest; also computes ``out = A~ v``.  Returns (best, times_ms, out)."""
        import torch
        if max_candidates < 1:
            raise ValueError("max_candidates must be at least 1")
        with _OnStream(stream) as on:
            v, out = self._vectors(v, out)
            best = Tune()
            ms = (ctypes.c_double * max_candidates)()
            _check(lib().fdm_plan_autotune(self._h, _ptr(v), _ptr(out),
                                           int(v.dtype == torch.complex64), int(max_candidates),
                                           on.handle(), ctypes.byref(best), ms))
            on.keep(v, out)
        return best.as_dict(), list(ms), out

    def prepare(self, stream=None) -> None:
        """Build the launch schedule (and streamed-bank workspace) now."""
        _check(lib().fdm_plan_prepare(self._h, _stream_handle(stream)))

    def coupling_launches(self) -> int:
        n = ctypes.c_int()
        _check(lib().fdm_plan_coupling_launches(self._h, ctypes.byref(n)))
        return n.value

    def wait_launch(self, i: int) -> float:
        """Wait for coupling launch i of the last timed matvec; ms since its start."""
        ms = ctypes.c_double()
        _check(lib().fdm_plan_wait_launch(self._h, int(i), ctypes.byref(ms)))
        return ms.value

    PHASES = ("s2m", "m2m", "m2l", "l2l", "l2t", "near", "total")

    def set_timing(self, enable: bool = True) -> None:
        """Record HIP events around each phase of later matvecs."""
        _check(lib().fdm_plan_set_timing(self._h, int(enable)))

    def phase_ms(self) -> dict:
        """Milliseconds per phase of the last timed matvec (waits for it)."""
        out = (ctypes.c_double * 7)()
        _check(lib().fdm_plan_phase_ms(self._h, out))
        return dict(zip(self.PHASES, list(out)))

    def close(self) -> None:
        """Free the plan (FdmError while it belongs to a live batch)."""
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().fdm_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def dense_matvec(points_T, points_S, kappa: float, v, out=None, stream=None):
    """Dense ``y = A v`` by direct FP64 summation on the GPU."""
    import torch
    if not isinstance(v, torch.Tensor) or not v.is_cuda or v.dtype != torch.complex128:
        raise TypeError("v must be a complex128 CUDA vector of length n_S")
    with _OnStream(stream) as on:
        pt, ps = _points(points_T), _points(points_S)
        if v.shape != (ps.shape[0],):
            raise TypeError("v must be a complex128 CUDA vector of length n_S")
        v = v.contiguous()
        if out is None:
            out = torch.empty(pt.shape[0], dtype=torch.complex128, device=v.device)
        elif (not isinstance(out, torch.Tensor) or not out.is_cuda
              or out.dtype != torch.complex128 or out.shape != (pt.shape[0],)
              or not out.is_contiguous()):
            raise TypeError("out must be a contiguous complex128 CUDA vector of length n_T")
        _check(lib().fdm_dense_matvec(_ptr(pt), pt.shape[0], _ptr(ps), ps.shape[0],
                                      float(kappa), _ptr(v), _ptr(out), on.handle()))
        on.keep(pt, ps, v, out)
    return out


def aca(A, eps: float, max_rank: int | None = None):
    """Low-rank ``A ~ U @ W.conj().T`` of a host complex matrix by partially
    pivoted ACA (wraps ``fdm_aca``; host code, no device).  Returns numpy
    arrays U (n_rows, k) and W (n_cols, k)."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    if A.ndim != 2:
        raise TypeError("A must be a 2-d array")
    n, m = A.shape
    R = min(n, m) if max_rank is None else int(max_rank)
    U = np.zeros((n, max(R, 1)), np.complex128)
    W = np.zeros((m, max(R, 1)), np.complex128)
    k = ctypes.c_int()
    _check(lib().fdm_aca(A.ctypes.data, n, m, float(eps), R, U.ctypes.data, W.ctypes.data,
                         ctypes.byref(k)))
    return U[:, :k.value].copy(), W[:, :k.value].copy()


class Batch:
    """Many plans (same m and precision) whose matvecs run together: one
    device queue for all coupling work and near fields, the whole batched
    matvec captured in a HIP graph (wraps ``fdm_batch*``).  The plans must
    outlive the batch."""

    def __init__(self, plans, workspace_bytes: int = 0, stream=None):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib().fdm_batch_create(arr, len(self.plans), int(workspace_bytes),
                                      _stream_handle(stream), ctypes.byref(h)))
        self._h = h

    def _vectors(self, vs, outs):
        import torch
        if len(vs) != len(self.plans):
            raise ValueError("one v per plan")
        dtype = vs[0].dtype
        if dtype not in (torch.complex128, torch.complex64):
            raise TypeError("v must be complex128 or complex64")
        vs = [v.contiguous() for v in vs]
        for v, p in zip(vs, self.plans):
            if v.dtype != dtype or v.shape != (p.n_S,) or not v.is_cuda:
                raise TypeError("each v must be a CUDA vector of its plan's n_S, one dtype")
        if outs is None:
            outs = [torch.empty(p.n_T, dtype=dtype, device=vs[0].device) for p in self.plans]
        if len(outs) != len(self.plans):
            raise ValueError("one out per plan")
        for y, p in zip(outs, self.plans):
            if (not isinstance(y, torch.Tensor) or not y.is_cuda or y.dtype != dtype
                    or y.shape != (p.n_T,) or not y.is_contiguous()):
                raise TypeError("each out must be a contiguous CUDA vector of its plan's n_T")
        n = len(self.plans)
        va = (ctypes.c_void_p * n)(*[v.data_ptr() if v.numel() else None for v in vs])
        ya = (ctypes.c_void_p * n)(*[y.data_ptr() if y.numel() else None for y in outs])
        return vs, outs, va, ya, int(dtype == torch.complex64)

    def matvec(self, vs, outs=None, stream=None):
        """``outs[i] = A~_i vs[i]`` for every plan; returns outs."""
        with _OnStream(stream) as on:
            vs, outs, va, ya, c64 = self._vectors(vs, outs)
            _check(lib().fdm_batch_matvec(self._h, va, ya, c64, on.handle()))
            on.keep(*vs, *outs)
        return outs

    def set_graph(self, enable: bool) -> None:
        _check(lib().fdm_batch_set_graph(self._h, int(enable)))

    def get_tune(self) -> dict:
        t = Tune()
        _check(lib().fdm_batch_get_tune(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tune(self, tune: dict, stream=None) -> None:
        t = Tune.from_dict({**self.get_tune(), **tune})
        _check(lib().fdm_batch_set_tune(self._h, ctypes.byref(t), _stream_handle(stream)))

    def autotune(self, vs, outs=None, max_candidates: int = 4, stream=None):
        """Time the batch's coupling launches under each candidate launch
        shape and keep the fastest; also computes outs.  Returns
        (best, times_ms, outs)."""
        if max_candidates < 1:
            raise ValueError("max_candidates must be at least 1")
        with _OnStream(stream) as on:
            vs, outs, va, ya, c64 = self._vectors(vs, outs)
            best = Tune()
            ms = (ctypes.c_double * max_candidates)()
            _check(lib().fdm_batch_autotune(self._h, va, ya, c64, int(max_candidates),
                                            on.handle(), ctypes.byref(best), ms))
            on.keep(*vs, *outs)
        return best.as_dict(), list(ms), outs

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().fdm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
