"""Thin Python binding of libgrmhd.so (include/grmhd.h).

Argument marshalling only: every step of the method runs in the HIP library.  Host arrays are
numpy float64 arrays; device arrays are torch tensors on the GPU (passed by pointer).  Loading
fails with an ImportError when the library has not been built -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrmhd.so")

OK, EINVAL, ENOMEM, EDEVICE, ENUMERIC, EAGAIN, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
MKS, MINKOWSKI_CART = 0, 1
LLF, HLL = 0, 1
PLM, PPM = 0, 1

# exported symbols of include/grmhd.h
SYMBOLS = [
    "grmhd_params_default", "grmhd_init", "grmhd_step", "grmhd_steps", "grmhd_cons2prim",
    "grmhd_prim2cons", "grmhd_diag", "grmhd_diag_full", "grmhd_diag_full_noalloc", "grmhd_get_prims", "grmhd_get_time", "grmhd_set_time", "grmhd_get_codes",
    "grmhd_debug_fluxes", "grmhd_debug_fixup", "grmhd_kernel_timing", "grmhd_kernel_times", "grmhd_autotune", "grmhd_destroy", "grmhd_last_error", "grmhd_footprint_bytes",
    "grmhd_batch_create", "grmhd_batch_admit", "grmhd_batch_advance", "grmhd_batch_autotune", "grmhd_batch_poll",
    "grmhd_batch_kernel_timing", "grmhd_batch_kernel_times",
    "grmhd_batch_fetch", "grmhd_batch_get_time", "grmhd_batch_diag_full", "grmhd_batch_release", "grmhd_batch_usage", "grmhd_batch_destroy",
]


class Grid(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("n3", ctypes.c_int32),
                ("coords", ctypes.c_int32), ("r_in", ctypes.c_double), ("r_out", ctypes.c_double),
                ("h", ctypes.c_double), ("xmin", ctypes.c_double * 3), ("xmax", ctypes.c_double * 3),
                ("r_br", ctypes.c_double), ("n_x", ctypes.c_int32), ("pole_fix", ctypes.c_int32)]


class Horizon(ctypes.Structure):
    _fields_ = [("mdot", ctypes.c_double), ("phi_b", ctypes.c_double), ("ldot", ctypes.c_double),
                ("edot", ctypes.c_double), ("phi_b_norm", ctypes.c_double), ("i_h", ctypes.c_int32),
                ("reserved_", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("spin", ctypes.c_double), ("gam", ctypes.c_double), ("cfl", ctypes.c_double),
                ("riemann", ctypes.c_int32), ("recon", ctypes.c_int32),
                ("rho_fl_coef", ctypes.c_double), ("rho_fl_pow", ctypes.c_double),
                ("u_fl_coef", ctypes.c_double), ("u_fl_pow", ctypes.c_double), ("fl_abs", ctypes.c_double),
                ("bsq_rho_max", ctypes.c_double), ("bsq_u_max", ctypes.c_double),
                ("gamma_max", ctypes.c_double), ("beta_entropy", ctypes.c_double),
                ("c2p_tol", ctypes.c_double), ("c2p_maxit", ctypes.c_int32),
                ("fixup_max_rounds", ctypes.c_int32)]


class GrmhdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libgrmhd.so and declare its signatures (raises ImportError if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(path)
    vp, dp, i32, i64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_int64
    pp = ctypes.POINTER(ctypes.c_void_p)
    gp, ppar = ctypes.POINTER(Grid), ctypes.POINTER(Params)
    L.grmhd_params_default.argtypes = [ppar]
    L.grmhd_params_default.restype = None
    L.grmhd_init.argtypes = [pp, gp, ppar, vp, i32, vp]
    L.grmhd_step.argtypes = [vp, ctypes.c_double, dp]
    L.grmhd_steps.argtypes = [vp, i32, ctypes.c_double]
    L.grmhd_cons2prim.argtypes = [vp, vp, vp, vp, i32]
    L.grmhd_prim2cons.argtypes = [vp, vp, vp, i32]
    L.grmhd_diag.argtypes = [vp, dp, dp]
    L.grmhd_diag_full.argtypes = [vp, ctypes.POINTER(Horizon), vp]
    L.grmhd_diag_full_noalloc.argtypes = [vp, ctypes.POINTER(Horizon), vp]
    L.grmhd_diag_full_noalloc.restype = ctypes.c_int
    L.grmhd_get_prims.argtypes = [vp, vp, i32]
    L.grmhd_get_time.argtypes = [vp, dp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.grmhd_set_time.argtypes = [vp, ctypes.c_double, i64]
    L.grmhd_get_codes.argtypes = [vp, vp]
    L.grmhd_debug_fluxes.argtypes = [vp, i32, vp, dp]
    L.grmhd_debug_fixup.argtypes = [vp, vp, vp, vp, ctypes.POINTER(i64)]
    L.grmhd_kernel_timing.argtypes = [vp, i32]
    L.grmhd_kernel_times.argtypes = [vp, dp, ctypes.POINTER(i64), i32]
    L.grmhd_autotune.argtypes = [vp, i32, ctypes.c_char_p, i32]
    L.grmhd_batch_autotune.argtypes = [vp, i32, ctypes.c_char_p, i32]
    L.grmhd_batch_kernel_timing.argtypes = [vp, i32]
    L.grmhd_batch_kernel_times.argtypes = [vp, dp, ctypes.POINTER(i64), i32]
    L.grmhd_destroy.argtypes = [vp]
    L.grmhd_destroy.restype = None
    L.grmhd_last_error.argtypes = []
    L.grmhd_last_error.restype = ctypes.c_char_p
    L.grmhd_footprint_bytes.argtypes = [gp]
    L.grmhd_footprint_bytes.restype = i64
    L.grmhd_batch_create.argtypes = [pp, i64, i32, vp]
    L.grmhd_batch_admit.argtypes = [vp, gp, ppar, vp, i32, i64, ctypes.POINTER(i64)]
    L.grmhd_batch_advance.argtypes = [vp, i32]
    L.grmhd_batch_poll.argtypes = [vp, ctypes.POINTER(i64), i32, ctypes.POINTER(i32)]
    L.grmhd_batch_fetch.argtypes = [vp, i64, vp, dp, ctypes.POINTER(i64)]
    L.grmhd_batch_get_time.argtypes = [vp, i64, dp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.grmhd_batch_diag_full.argtypes = [vp, i64, ctypes.POINTER(Horizon), vp]
    L.grmhd_batch_release.argtypes = [vp, i64]
    L.grmhd_batch_usage.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32)]
    L.grmhd_batch_destroy.argtypes = [vp]
    L.grmhd_batch_destroy.restype = None
    _lib = L
    return L


def _check(rc: int, allow=(OK,)):
    if rc not in allow:
        raise GrmhdError(rc, load().grmhd_last_error().decode())
    return rc


def make_grid(cfg, **over) -> Grid:
    """Grid struct from a config-like object (TorusConfig or anything with n1, n2, n3, ...)."""
    def get(name, default):
        return over[name] if name in over else getattr(cfg, name, default)
    g = Grid()
    g.n1, g.n2, g.n3 = int(get("n1", 1)), int(get("n2", 1)), int(get("n3", 1))
    coords = get("coords", "mks")
    g.coords = MKS if coords in ("mks", MKS) else MINKOWSKI_CART
    spin = float(get("spin", 0.0))
    rin = get("r_in_grid", None)
    g.r_in = float(rin) if rin is not None else 0.98 * (1.0 + math.sqrt(1.0 - spin * spin))
    g.r_out = float(get("r_out", 40.0))
    g.h = float(get("h", 0.3))
    xmin, xmax = get("xmin", (0.0, 0.0, 0.0)), get("xmax", (1.0, 1.0, 1.0))
    for d in range(3):
        g.xmin[d], g.xmax[d] = float(xmin[d]), float(xmax[d])
    g.r_br = float(get("r_br", 0.0) or 0.0)
    g.n_x = int(get("n_x", 4))
    g.pole_fix = int(get("pole_fix", 0))
    return g


def make_params(cfg, **over) -> Params:
    def get(name, default):
        return over[name] if name in over else getattr(cfg, name, default)
    p = Params()
    load().grmhd_params_default(ctypes.byref(p))
    p.spin = float(get("spin", p.spin))
    p.gam = float(get("gam", p.gam))
    p.cfl = float(get("cfl", p.cfl))
    r = get("riemann", "llf")
    p.riemann = HLL if r in ("hll", HLL) else LLF
    rec = get("recon", "plm")
    p.recon = PPM if rec in ("ppm", PPM) else PLM
    for name in ("rho_fl_coef", "rho_fl_pow", "u_fl_coef", "u_fl_pow", "fl_abs", "bsq_rho_max",
                 "bsq_u_max", "gamma_max", "beta_entropy", "c2p_tol"):
        setattr(p, name, float(get(name, getattr(p, name))))
    p.c2p_maxit = int(get("c2p_maxit", p.c2p_maxit))
    p.fixup_max_rounds = int(get("fixup_max_rounds", p.fixup_max_rounds))
    return p


def _host(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def _is_device(a) -> bool:
    return hasattr(a, "is_cuda") and a.is_cuda


def _ptr(a):
    if _is_device(a):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        return ctypes.c_void_p(0)
    return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))


class Context:
    """One resident run (grmhd_init ... grmhd_destroy)."""

    def __init__(self, cfg, prims, stream=None, **over):
        L = load()
        self.grid = make_grid(cfg, **over)
        self.params = make_params(cfg, **over)
        self.shape = (self.grid.n1, self.grid.n2, self.grid.n3)
        self._h = ctypes.c_void_p()
        on_dev = _is_device(prims)
        if on_dev:
            import torch
            torch.cuda.synchronize()
            src = prims.contiguous()
        else:
            src = _host(prims)
        if tuple(src.shape) != (8,) + self.shape:
            raise ValueError(f"prims shape {tuple(src.shape)} != {(8,) + self.shape}")
        _check(L.grmhd_init(ctypes.byref(self._h), ctypes.byref(self.grid), ctypes.byref(self.params),
                            _ptr(src), int(on_dev), _stream_handle(stream)))

    def close(self):
        if self._h:
            load().grmhd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, dt: float = -1.0) -> float:
        out = ctypes.c_double(0.0)
        _check(load().grmhd_step(self._h, float(dt), ctypes.byref(out)), allow=(OK, ENUMERIC))
        return out.value

    def steps(self, n: int, dt: float = -1.0):
        _check(load().grmhd_steps(self._h, int(n), float(dt)))

    def get_prims(self, out=None):
        if out is None:
            out = np.empty((8,) + self.shape)
        _check(load().grmhd_get_prims(self._h, _ptr(out), int(_is_device(out))))
        return out

    def get_time(self):
        t = ctypes.c_double()
        n = ctypes.c_int64()
        f = ctypes.c_int64()
        _check(load().grmhd_get_time(self._h, ctypes.byref(t), ctypes.byref(n), ctypes.byref(f)))
        return t.value, n.value, f.value

    def set_time(self, t: float, nstep: int):
        _check(load().grmhd_set_time(self._h, float(t), int(nstep)))

    def get_codes(self):
        out = np.empty(self.shape, dtype=np.int8)
        _check(load().grmhd_get_codes(self._h, _ptr(out)))
        return out

    def cons2prim(self, U, Pguess):
        U = _host(U)
        P = _host(Pguess).copy()
        code = np.empty(self.shape, dtype=np.int8)
        _check(load().grmhd_cons2prim(self._h, _ptr(U), _ptr(P), _ptr(code), 0))
        return P, code

    def prim2cons(self, P):
        P = _host(P)
        U = np.empty((9,) + self.shape)
        _check(load().grmhd_prim2cons(self._h, _ptr(P), _ptr(U), 0))
        return U

    def diag(self):
        m = ctypes.c_double()
        f = ctypes.c_double()
        _check(load().grmhd_diag(self._h, ctypes.byref(m), ctypes.byref(f)))
        return m.value, f.value

    def diag_full(self):
        """Horizon diagnostics (dict) and the radial profiles [6][n1]: Mdot, phi_B, Ldot, Edot,
        ldot_in, ldot_out per radial cell."""
        hz = Horizon()
        rad = np.empty((6, self.grid.n1))
        _check(load().grmhd_diag_full(self._h, ctypes.byref(hz), _ptr(rad)))
        return ({k: getattr(hz, k) for k in ("mdot", "phi_b", "ldot", "edot", "phi_b_norm", "i_h")}, rad)

    def autotune(self, steps_per_candidate: int = 2) -> str:
        buf = ctypes.create_string_buffer(1 << 16)
        _check(load().grmhd_autotune(self._h, int(steps_per_candidate), buf, len(buf)))
        return buf.value.decode()

    KERNELS = ("bound", "flux1", "flux2", "flux3", "dt", "update", "fixup", "update_slow", "emf")

    def kernel_timing(self, on: bool):
        _check(load().grmhd_kernel_timing(self._h, int(bool(on))))

    def kernel_times(self):
        n = len(self.KERNELS)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(load().grmhd_kernel_times(self._h, ms, cnt, n))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.KERNELS)}

    def debug_fixup(self, pout, pin, code):
        """Device fixup rounds on (pout, pin, code); returns (fixed P, codes, cells left)."""
        shape = (8, self.grid.n1, self.grid.n2, self.grid.n3)
        P = np.ascontiguousarray(pout, dtype=np.float64).reshape(shape).copy()
        Pi = np.ascontiguousarray(pin, dtype=np.float64).reshape(shape)
        cd = np.ascontiguousarray(code, dtype=np.int8).reshape(shape[1:]).copy()
        left = ctypes.c_int64()
        _check(load().grmhd_debug_fixup(self._h, _ptr(P), _ptr(Pi), cd.ctypes.data, ctypes.byref(left)))
        return P, cd, left.value

    def debug_fluxes(self, d: int):
        m = [self.grid.n1, self.grid.n2, self.grid.n3]
        m[d - 1] += 1
        F = np.empty((9,) + tuple(m))
        cmax = ctypes.c_double()
        _check(load().grmhd_debug_fluxes(self._h, int(d), _ptr(F), ctypes.byref(cmax)))
        return F, cmax.value


def footprint_bytes(cfg, **over) -> int:
    g = make_grid(cfg, **over)
    return int(load().grmhd_footprint_bytes(ctypes.byref(g)))


class Batch:
    """Ensemble of resident runs advanced together (grmhd_batch_*)."""

    def __init__(self, budget_bytes: int = 0, max_jobs: int = 1024, stream=None):
        self._h = ctypes.c_void_p()
        _check(load().grmhd_batch_create(ctypes.byref(self._h), int(budget_bytes), int(max_jobs),
                                         _stream_handle(stream)))
        self.shapes = {}

    def admit(self, cfg, prims, nsteps: int, **over) -> Optional[int]:
        """Job id, or None when the job does not fit the memory budget now."""
        g = make_grid(cfg, **over)
        p = make_params(cfg, **over)
        src = _host(prims)
        jid = ctypes.c_int64()
        rc = load().grmhd_batch_admit(self._h, ctypes.byref(g), ctypes.byref(p), _ptr(src), 0, int(nsteps),
                                      ctypes.byref(jid))
        if rc == EAGAIN:
            return None
        _check(rc)
        self.shapes[jid.value] = (g.n1, g.n2, g.n3)
        return jid.value

    def advance(self, steps: int):
        _check(load().grmhd_batch_advance(self._h, int(steps)))

    def autotune(self, steps_per_candidate: int = 2) -> str:
        buf = ctypes.create_string_buffer(1 << 16)
        _check(load().grmhd_batch_autotune(self._h, int(steps_per_candidate), buf, len(buf)))
        return buf.value.decode()

    def kernel_timing(self, on: bool):
        _check(load().grmhd_batch_kernel_timing(self._h, int(bool(on))))

    def kernel_times(self):
        """{kernel kind: (average ms per launch over all active jobs, launches)}, as Context."""
        n = len(Context.KERNELS)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(load().grmhd_batch_kernel_times(self._h, ms, cnt, n))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(Context.KERNELS)}

    def poll(self, cap: int = 1024):
        ids = (ctypes.c_int64 * cap)()
        n = ctypes.c_int32()
        _check(load().grmhd_batch_poll(self._h, ids, int(cap), ctypes.byref(n)))
        return [ids[i] for i in range(n.value)]

    def fetch(self, jid: int):
        out = np.empty((8,) + self.shapes[jid])
        t = ctypes.c_double()
        n = ctypes.c_int64()
        _check(load().grmhd_batch_fetch(self._h, int(jid), _ptr(out), ctypes.byref(t), ctypes.byref(n)))
        return out, t.value, n.value

    def get_time(self, jid: int):
        """(t, step count, cells left unfixed since admission) of a job."""
        t = ctypes.c_double()
        n = ctypes.c_int64()
        f = ctypes.c_int64()
        _check(load().grmhd_batch_get_time(self._h, int(jid), ctypes.byref(t), ctypes.byref(n), ctypes.byref(f)))
        return t.value, n.value, f.value

    def diag_full(self, jid: int):
        """Horizon diagnostics (dict) and radial profiles [6][n1] of a job's current state, as
        Context.diag_full."""
        hz = Horizon()
        shape = self.shapes.get(jid)             # unknown job: no profile buffer, the library reports it
        rad = np.empty((6, shape[0])) if shape else None
        _check(load().grmhd_batch_diag_full(self._h, int(jid), ctypes.byref(hz),
                                            _ptr(rad) if rad is not None else None))
        return ({k: getattr(hz, k) for k in ("mdot", "phi_b", "ldot", "edot", "phi_b_norm", "i_h")}, rad)

    def release(self, jid: int):
        _check(load().grmhd_batch_release(self._h, int(jid)))
        self.shapes.pop(jid, None)

    def usage(self):
        b = ctypes.c_int64()
        j = ctypes.c_int32()
        _check(load().grmhd_batch_usage(self._h, ctypes.byref(b), ctypes.byref(j)))
        return b.value, j.value

    def close(self):
        if self._h:
            load().grmhd_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
