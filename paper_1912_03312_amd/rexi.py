"""Thin ctypes binding of ``librexi.so`` (the C ABI of ``include/rexi.h``).

Argument marshalling only: tensors are passed by ``data_ptr()`` and the
current torch stream by handle; every step of the computation runs in the
HIP kernels of the library. Importing this module fails loudly when the
library has not been built (``python -m paper_1912_03312_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librexi.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1912_03312_amd.build`")

_lib = C.CDLL(LIB_PATH)

REXI_OK, REXI_E_INVALID_ARG, REXI_E_NO_MEMORY, REXI_E_HIP, REXI_E_NOT_CONVERGED, REXI_E_NOT_BUILT = range(6)
PREC_C128, PREC_C64_REFINE = 0, 1
TOL_RELRES, TOL_CERTIFIED = 0, 1
SOLVER_PER_POLE, SOLVER_SHIFTED = 0, 1

#: every entry point the header declares
EXPORTS = ("rexi_default_options", "rexi_setup", "rexi_setup_batch", "rexi_apply_H", "rexi_step",
           "rexi_step_adjoint", "rexi_get_profile", "rexi_profile_reset", "rexi_workspace_info",
           "rexi_tiling_info", "rexi_estimate_spectrum", "rexi_estimate_spectrum_noalloc", "rexi_get_solution",
           "rexi_destroy", "rexi_status_string", "rexi_last_error")


class c128(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class Grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("reserved", C.c_int32), ("n", C.c_int64 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("solver", C.c_int32), ("m", C.c_int32),
                ("max_cycles", C.c_int32), ("tol", C.c_double), ("tol_policy", C.c_int32),
                ("reorth", C.c_int32), ("reorth_eta", C.c_double), ("inner_rtol", C.c_double),
                ("check_every", C.c_int32), ("lanczos", C.c_int32), ("capture_safe", C.c_int32),
                ("capture_cycles", C.c_int32), ("graph_chunks", C.c_int32),
                ("profile", C.c_int32), ("tile", C.c_int32), ("grid_blocks", C.c_int32), ("autotune", C.c_int32),
                ("max_workspace_bytes", C.c_int64), ("march_planes", C.c_int32), ("march_slots", C.c_int32),
                ("fallback", C.c_int32), ("fallback_m", C.c_int32), ("fallback_bytes", C.c_int64),
                ("stab_eps", C.c_double), ("center", C.c_int32), ("discretization", C.c_int32),
                ("adjoint_shared", C.c_int32), ("keep_solutions", C.c_int32), ("capture_pauses", C.c_int32),
                ("reserved_opt2_", C.c_int32)]


class StepInfo(C.Structure):
    _fields_ = [("K", C.c_int32), ("steps", C.c_int32), ("total_iterations", C.c_int64),
                ("max_cycles_used", C.c_int32), ("not_converged", C.c_int32),
                ("max_rel_residual", C.c_double), ("certified_bound", C.c_double),
                ("reorth_passes", C.c_int32), ("explicit_residuals", C.c_int32),
                ("norm_in", C.c_double), ("norm_out", C.c_double),
                ("iterations", C.POINTER(C.c_int32)), ("cycles", C.POINTER(C.c_int32)),
                ("rel_residual", C.POINTER(C.c_double)), ("implicit_residual", C.POINTER(C.c_double))]


class Tiling(C.Structure):
    _fields_ = [("tile", C.c_int32), ("grid_blocks", C.c_int32), ("march_slots", C.c_int32),
                ("march_planes", C.c_int32), ("march_items", C.c_int32), ("reserved_", C.c_int32)]


class Profile(C.Structure):
    _fields_ = [("nclasses", C.c_int32), ("names", C.c_char_p * 12), ("launches", C.c_int64 * 12),
                ("ms", C.c_double * 12), ("bytes", C.c_double * 12)]


_H = C.c_void_p
_P = C.c_void_p
_lib.rexi_default_options.argtypes = [C.POINTER(Options)]
_lib.rexi_default_options.restype = None
_lib.rexi_setup.argtypes = [C.POINTER(_H), C.POINTER(Grid), _P, C.c_double, C.c_double, C.c_double, C.c_int32,
                            C.POINTER(c128), C.POINTER(c128), C.POINTER(Options), _P]
_lib.rexi_setup_batch.argtypes = [C.POINTER(_H), C.c_int32, C.POINTER(Grid), _P, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                  C.POINTER(c128), C.POINTER(c128), C.POINTER(Options), _P]
_lib.rexi_apply_H.argtypes = [_H, _P, _P, c128, _P]
_lib.rexi_step.argtypes = [_H, _P, _P, C.c_int32, C.POINTER(StepInfo), _P]
_lib.rexi_step_adjoint.argtypes = [_H, _P, _P, _P, _P, _P]
_lib.rexi_get_profile.argtypes = [_H, C.POINTER(Profile)]
_lib.rexi_profile_reset.argtypes = [_H]
_lib.rexi_workspace_info.argtypes = [_H, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
_lib.rexi_tiling_info.argtypes = [_H, C.POINTER(Tiling)]
_lib.rexi_get_solution.argtypes = [_H, C.c_int32, _P, _P]
_lib.rexi_destroy.argtypes = [_H]
_lib.rexi_status_string.argtypes = [C.c_int]
_lib.rexi_status_string.restype = C.c_char_p
_lib.rexi_last_error.argtypes = [_H, C.c_char_p, C.c_size_t]
for _f in ("rexi_setup", "rexi_setup_batch", "rexi_apply_H", "rexi_step", "rexi_step_adjoint", "rexi_get_profile",
           "rexi_profile_reset", "rexi_workspace_info", "rexi_destroy", "rexi_last_error", "rexi_estimate_spectrum",
           "rexi_estimate_spectrum_noalloc", "rexi_get_solution"):
    getattr(_lib, _f).restype = C.c_int


class RexiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_lib.rexi_status_string(status).decode()}: {msg}")
        self.status = status


def _last_error(h) -> str:
    buf = C.create_string_buffer(512)
    _lib.rexi_last_error(h, buf, 512)
    return buf.value.decode()


def _check(status: int, h=None):
    if status != REXI_OK:
        raise RexiError(status, _last_error(h))


def default_options(**kw) -> Options:
    o = Options()
    _lib.rexi_default_options(C.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"c128": PREC_C128, "c64": PREC_C64_REFINE}[v]
        if k == "solver" and isinstance(v, str):
            v = {"per_pole": SOLVER_PER_POLE, "shifted": SOLVER_SHIFTED}[v]
        if k == "tol_policy" and isinstance(v, str):
            v = {"relres": TOL_RELRES, "certified": TOL_CERTIFIED}[v]
        if k == "discretization" and isinstance(v, str):
            v = {"fd": 0, "fem": 1}[v]
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def make_grid(n: Sequence[int], lo: Sequence[float], hi: Sequence[float]) -> Grid:
    g = Grid()
    g.ndim = len(n)
    for a in range(len(n)):
        g.n[a], g.lo[a], g.hi[a] = int(n[a]), float(lo[a]), float(hi[a])
    return g


def _c128_array(z) -> C.Array:
    z = np.asarray(z, dtype=np.complex128).ravel()
    arr = (c128 * max(1, z.size))()
    for i, v in enumerate(z):
        arr[i].re, arr[i].im = float(v.real), float(v.imag)
    return arr


def _stream(stream) -> int:
    if stream is not None:
        return int(stream)
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype_name: str, numel: int):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"expected a CUDA (HIP) tensor of {dtype_name}")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise TypeError(f"expected dtype {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return t.data_ptr()


class Handle:
    """A configured REXI propagator (one instance or an uneven batch)."""

    def __init__(self, raw, npts: int, K: int, count: int = 1):
        self._h = raw
        self._destroy = _lib.rexi_destroy  # kept: the module may be torn down first at exit
        self.npts = npts
        self.K = K
        self.count = count

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None

    def apply_H(self, x, y, shift: complex = 0.0, stream=None):
        """y = (H - shift I) x in FP64."""
        px = _ptr(x, "complex128", self.npts)
        py = _ptr(y, "complex128", self.npts)
        s = c128(float(np.real(shift)), float(np.imag(shift)))
        _check(_lib.rexi_apply_H(self._h, px, py, s, _stream(stream)), self._h)

    def estimate_spectrum(self, iters: int = 30, stream=None):
        """``rexi_estimate_spectrum``: (lo, hi) float64 arrays per instance,
        the extreme Ritz values of H after ``iters`` Lanczos iterations."""
        lo = (C.c_double * self.count)()
        hi = (C.c_double * self.count)()
        _check(_lib.rexi_estimate_spectrum(self._h, int(iters), lo, hi, _stream(stream)), self._h)
        return np.array(lo[:]), np.array(hi[:])

    def estimate_spectrum_noalloc(self, iters: int = 30, stream=None):
        """``rexi_estimate_spectrum_noalloc``: the same estimate in the library's
        fixed device workspace (no device allocation)."""
        lo = (C.c_double * self.count)()
        hi = (C.c_double * self.count)()
        _check(_lib.rexi_estimate_spectrum_noalloc(self._h, int(iters), lo, hi, _stream(stream)), self._h)
        return np.array(lo[:]), np.array(hi[:])

    def step(self, psi_in, psi_out, nsteps: int = 1, info: bool = True, stream=None, raise_on_nc: bool = True):
        """``nsteps`` REXI steps; returns a dict of solve diagnostics (or None)."""
        pi = _ptr(psi_in, "complex128", self.npts)
        po = _ptr(psi_out, "complex128", self.npts)
        if not info:
            _check(_lib.rexi_step(self._h, pi, po, int(nsteps), None, _stream(stream)), self._h)
            return None
        it = (C.c_int32 * self.K)()
        cy = (C.c_int32 * self.K)()
        rr = (C.c_double * self.K)()
        ri = (C.c_double * self.K)()
        inf = StepInfo()
        inf.iterations = C.cast(it, C.POINTER(C.c_int32))
        inf.cycles = C.cast(cy, C.POINTER(C.c_int32))
        inf.rel_residual = C.cast(rr, C.POINTER(C.c_double))
        inf.implicit_residual = C.cast(ri, C.POINTER(C.c_double))
        st = _lib.rexi_step(self._h, pi, po, int(nsteps), C.byref(inf), _stream(stream))
        out = dict(K=inf.K, steps=inf.steps, total_iterations=inf.total_iterations,
                   max_cycles_used=inf.max_cycles_used, not_converged=inf.not_converged,
                   max_rel_residual=inf.max_rel_residual, certified_bound=inf.certified_bound,
                   norm_in=inf.norm_in, norm_out=inf.norm_out, reorth_passes=inf.reorth_passes,
                   iterations=list(it), cycles=list(cy), explicit_residuals=bool(inf.explicit_residuals),
                   rel_residual=list(rr), implicit_residual=list(ri), status=st)
        if st != REXI_OK and (st != REXI_E_NOT_CONVERGED or raise_on_nc):
            _check(st, self._h)
        return out

    def solution(self, pole: int, x, stream=None):
        """``rexi_get_solution``: x_j of pole ``pole`` of the last step into the
        complex128 CUDA tensor ``x`` (the pole's instance size)."""
        px = x.data_ptr() if x.is_contiguous() and str(x.dtype) == "torch.complex128" else None
        if px is None or x.device.type != "cuda":
            raise TypeError("expected a contiguous complex128 CUDA tensor")
        _check(_lib.rexi_get_solution(self._h, int(pole), px, _stream(stream)), self._h)

    def step_adjoint(self, psi_n, gbar_next, gbar_n, dV_accum=None, stream=None):
        """One backward step: gbar_n = R^H gbar_next, dV_accum += dL/dV."""
        pp = _ptr(psi_n, "complex128", self.npts)
        pg = _ptr(gbar_next, "complex128", self.npts)
        po = _ptr(gbar_n, "complex128", self.npts)
        pd = _ptr(dV_accum, "float64", self.npts) if dV_accum is not None else None
        _check(_lib.rexi_step_adjoint(self._h, pp, pg, po, pd, _stream(stream)), self._h)

    def profile(self) -> dict:
        p = Profile()
        _check(_lib.rexi_get_profile(self._h, C.byref(p)), self._h)
        return {p.names[c].decode(): dict(launches=p.launches[c], ms=p.ms[c], bytes=p.bytes[c])
                for c in range(p.nclasses)}

    def profile_reset(self):
        _check(_lib.rexi_profile_reset(self._h), self._h)

    def tiling(self) -> dict:
        """``rexi_tiling_info``: the tiling and fused Lanczos pass in use."""
        t = Tiling()
        _check(_lib.rexi_tiling_info(self._h, C.byref(t)), self._h)
        return {k: int(getattr(t, k)) for k, _ in Tiling._fields_ if k != "reserved_"}

    def workspace(self):
        b = C.c_int64()
        m = C.c_int32()
        _check(_lib.rexi_workspace_info(self._h, C.byref(b), C.byref(m)), self._h)
        return int(b.value), int(m.value)


def setup(grid_n, lo, hi, V, hbar: float, mass: float, dt: float, sigma, beta,
          options: Optional[Options] = None, stream=None, **opt) -> Handle:
    """``rexi_setup``: V is a contiguous float64 CUDA tensor of prod(grid_n) values."""
    n = int(np.prod(grid_n))
    g = make_grid(grid_n, lo, hi)
    pv = _ptr(V, "float64", n)
    sig = np.asarray(sigma, dtype=np.complex128).ravel()
    bet = np.asarray(beta, dtype=np.complex128).ravel()
    if sig.size != bet.size:
        raise ValueError("sigma and beta must have the same length")
    o = options if options is not None else default_options(**opt)
    raw = _H()
    st = _lib.rexi_setup(C.byref(raw), C.byref(g), pv, float(hbar), float(mass), float(dt), int(sig.size),
                         _c128_array(sig), _c128_array(bet), C.byref(o), _stream(stream))
    _check(st, None)
    return Handle(raw, n, int(sig.size))


def setup_batch(grids, V, hbar, mass, dt, K, sigma, beta, options: Optional[Options] = None,
                stream=None, **opt) -> Handle:
    """``rexi_setup_batch``: ``grids`` is a list of (n, lo, hi); V, sigma, beta packed."""
    cnt = len(grids)
    G = (Grid * cnt)()
    npts = 0
    for i, (n, lo, hi) in enumerate(grids):
        G[i] = make_grid(n, lo, hi)
        npts += int(np.prod(n))
    pv = _ptr(V, "float64", npts)
    dbl = lambda a: (C.c_double * cnt)(*[float(x) for x in a])
    Ks = (C.c_int32 * cnt)(*[int(k) for k in K])
    sig = np.asarray(sigma, dtype=np.complex128).ravel()
    bet = np.asarray(beta, dtype=np.complex128).ravel()
    if sig.size != sum(int(k) for k in K) or bet.size != sig.size:
        raise ValueError("sigma/beta must hold sum(K) values")
    o = options if options is not None else default_options(**opt)
    raw = _H()
    st = _lib.rexi_setup_batch(C.byref(raw), cnt, G, pv, dbl(hbar), dbl(mass), dbl(dt), Ks,
                               _c128_array(sig), _c128_array(bet), C.byref(o), _stream(stream))
    _check(st, None)
    return Handle(raw, npts, int(sig.size), cnt)


def status_string(s: int) -> str:
    return _lib.rexi_status_string(s).decode()
