"""ctypes binding of the FP64 CPU oracle (grmhd_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the CPU-baseline leg of
bench.py.  It imports nothing from the HIP package; run configurations are read duck-typed from
any object with the usual attribute names (n1, n2, n3, spin, gam, ...).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "grmhd_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

MKS, CART = 0, 1
LLF, HLL = 0, 1


class OrcCfg(ctypes.Structure):
    _fields_ = [
        ("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("n3", ctypes.c_int32),
        ("coords", ctypes.c_int32),
        ("r_in", ctypes.c_double), ("r_out", ctypes.c_double), ("h", ctypes.c_double),
        ("xmin", ctypes.c_double * 3), ("xmax", ctypes.c_double * 3),
        ("a", ctypes.c_double), ("gam", ctypes.c_double), ("cfl", ctypes.c_double),
        ("riemann", ctypes.c_int32), ("pole_fix", ctypes.c_int32),
        ("rho_fl_coef", ctypes.c_double), ("rho_fl_pow", ctypes.c_double),
        ("u_fl_coef", ctypes.c_double), ("u_fl_pow", ctypes.c_double), ("fl_abs", ctypes.c_double),
        ("bsq_rho_max", ctypes.c_double), ("bsq_u_max", ctypes.c_double),
        ("gamma_max", ctypes.c_double), ("beta_entropy", ctypes.c_double),
        ("c2p_tol", ctypes.c_double),
        ("c2p_maxit", ctypes.c_int32), ("fixup_max_rounds", ctypes.c_int32),
        ("r_br", ctypes.c_double), ("n_x", ctypes.c_int32), ("recon", ctypes.c_int32),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no FP contraction, OpenMP over cells)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-o", LIB, SRC, "-lm"]
        subprocess.check_call(cmd)
    return LIB


_lib = None


def _load(path):
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    cp = ctypes.POINTER(OrcCfg)
    bp = ctypes.POINTER(ctypes.c_int8)
    L.orc_step.argtypes = [cp, dp, ctypes.c_int, ctypes.c_double, dp, ctypes.POINTER(ctypes.c_int64), bp]
    L.orc_fluxes.argtypes = [cp, dp, ctypes.c_int, dp, dp]
    L.orc_prim2cons.argtypes = [cp, dp, dp]
    L.orc_cons2prim.argtypes = [cp, dp, dp, bp]
    L.orc_diag.argtypes = [cp, dp, dp, dp]
    L.orc_diag_full.argtypes = [cp, dp, dp, dp, dp]
    L.orc_grid_x1.argtypes = [cp, dp, dp]
    L.orc_ppm_face.argtypes = [dp, dp, dp]
    L.orc_geom.argtypes = [cp, ctypes.c_double, ctypes.c_double, dp, dp, dp, dp]
    L.orc_point_state.argtypes = [cp, ctypes.c_double, ctypes.c_double, dp] + [dp] * 10
    L.orc_point_c2p.argtypes = [cp, ctypes.c_double, ctypes.c_double, dp, dp, dp, ctypes.c_int]
    L.orc_point_floors.argtypes = [cp, ctypes.c_double, ctypes.c_double, dp]
    L.orc_mc_slope.argtypes = [ctypes.c_double] * 3
    L.orc_mc_slope.restype = ctypes.c_double
    L.orc_ghosts.argtypes = [cp, dp, dp]
    L.orc_fixups.restype = ctypes.c_int64
    L.orc_fixups.argtypes = [cp, dp, dp, bp]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        _lib = _load(LIB)
    return _lib


def build_variant(source_text: str, out_dir: str, tag: str) -> str:
    """Compile a modified copy of the oracle source (tests plant mistakes this way, to show that a
    pin fails for them) with the oracle's own flags; returns the library path."""
    src = os.path.join(out_dir, f"oracle_{tag}.c")
    out = os.path.join(out_dir, f"liboracle_{tag}.so")
    with open(src, "w") as fh:
        fh.write(source_text)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                           "-o", out, src, "-lm"])
    return out


class using_library:
    """Context manager: the module's functions call the oracle library at `path` inside the block."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = _load(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _g(obj, name, default):
    return getattr(obj, name, default) if obj is not None else default


def make_cfg(obj=None, **over) -> OrcCfg:
    """Build the oracle's run description from a config-like object plus overrides."""
    def get(name, default):
        if name in over:
            return over[name]
        return _g(obj, name, default)

    c = OrcCfg()
    c.n1, c.n2, c.n3 = int(get("n1", 1)), int(get("n2", 1)), int(get("n3", 1))
    coords = get("coords", "mks")
    c.coords = MKS if coords in ("mks", MKS) else CART
    spin = float(get("spin", 0.0))
    r_hor = 1.0 + (1.0 - spin * spin) ** 0.5
    rin = get("r_in_grid", None)
    c.r_in = float(rin) if rin is not None else 0.98 * r_hor
    c.r_out = float(get("r_out", 40.0))
    c.h = float(get("h", 0.3))
    xmin = get("xmin", (0.0, 0.0, 0.0))
    xmax = get("xmax", (1.0, 1.0, 1.0))
    for d in range(3):
        c.xmin[d] = float(xmin[d])
        c.xmax[d] = float(xmax[d])
    c.a = spin
    c.gam = float(get("gam", 4.0 / 3.0))
    c.cfl = float(get("cfl", 0.45))
    riem = get("riemann", "llf")
    c.riemann = HLL if riem in ("hll", HLL) else LLF
    c.rho_fl_coef = float(get("rho_fl_coef", 1e-5))
    c.rho_fl_pow = float(get("rho_fl_pow", -0.5))
    c.u_fl_coef = float(get("u_fl_coef", 1e-5 / 3.0))
    c.u_fl_pow = float(get("u_fl_pow", -2.5))
    c.fl_abs = float(get("fl_abs", 1e-20))
    c.bsq_rho_max = float(get("bsq_rho_max", 50.0))
    c.bsq_u_max = float(get("bsq_u_max", 2500.0))
    c.gamma_max = float(get("gamma_max", 50.0))
    c.beta_entropy = float(get("beta_entropy", 1e-2))
    c.c2p_tol = float(get("c2p_tol", 1e-10))
    c.c2p_maxit = int(get("c2p_maxit", 50))
    c.fixup_max_rounds = int(get("fixup_max_rounds", 8))
    c.r_br = float(get("r_br", 0.0) or 0.0)
    c.n_x = int(get("n_x", 4))
    rec = get("recon", "plm")
    c.recon = 1 if rec in ("ppm", 1) else 0
    c.pole_fix = int(get("pole_fix", 0))
    return c


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _bp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))


def _arr(P, shape=None):
    a = np.ascontiguousarray(P, dtype=np.float64).copy()
    if shape is not None and a.shape != shape:
        raise ValueError(f"shape {a.shape} != {shape}")
    return a


def step(cfg: OrcCfg, P, nsteps: int = 1, dt: float = -1.0):
    """Advance P[8][n1][n2][n3] by nsteps RK2 steps; dt <= 0 takes the CFL step each time.
    Returns (P_new, dts, nfail, codes of the last stage)."""
    P = _arr(P, (8, cfg.n1, cfg.n2, cfg.n3))
    dts = np.zeros(max(nsteps, 1))
    nfail = ctypes.c_int64(0)
    codes = np.zeros((cfg.n1, cfg.n2, cfg.n3), dtype=np.int8)
    rc = lib().orc_step(ctypes.byref(cfg), _dp(P), int(nsteps), float(dt), _dp(dts), ctypes.byref(nfail), _bp(codes))
    if rc != 0:
        raise RuntimeError(f"orc_step failed ({rc})")
    return P, dts[:nsteps], int(nfail.value), codes


def fluxes(cfg: OrcCfg, P, d: int):
    """Raw Riemann fluxes of direction d on the faces of interior cells and the largest c_w."""
    P = _arr(P, (8, cfg.n1, cfg.n2, cfg.n3))
    m = [cfg.n1, cfg.n2, cfg.n3]
    m[d - 1] += 1
    F = np.zeros((9,) + tuple(m))
    cmax = ctypes.c_double(0.0)
    rc = lib().orc_fluxes(ctypes.byref(cfg), _dp(P), int(d), _dp(F), ctypes.byref(cmax))
    if rc != 0:
        raise RuntimeError(f"orc_fluxes failed ({rc})")
    return F, cmax.value


def prim2cons(cfg: OrcCfg, P):
    P = _arr(P, (8, cfg.n1, cfg.n2, cfg.n3))
    U = np.zeros((9, cfg.n1, cfg.n2, cfg.n3))
    rc = lib().orc_prim2cons(ctypes.byref(cfg), _dp(P), _dp(U))
    if rc != 0:
        raise RuntimeError(f"orc_prim2cons failed ({rc})")
    return U


def cons2prim(cfg: OrcCfg, U, Pguess):
    U = _arr(U, (9, cfg.n1, cfg.n2, cfg.n3))
    P = _arr(Pguess, (8, cfg.n1, cfg.n2, cfg.n3))
    code = np.zeros((cfg.n1, cfg.n2, cfg.n3), dtype=np.int8)
    rc = lib().orc_cons2prim(ctypes.byref(cfg), _dp(U), _dp(P), _bp(code))
    if rc != 0:
        raise RuntimeError(f"orc_cons2prim failed ({rc})")
    return P, code


def diag(cfg: OrcCfg, P):
    P = _arr(P, (8, cfg.n1, cfg.n2, cfg.n3))
    m = ctypes.c_double(0.0)
    f = ctypes.c_double(0.0)
    ih = lib().orc_diag(ctypes.byref(cfg), _dp(P), ctypes.byref(m), ctypes.byref(f))
    return m.value, f.value, ih


def diag_full(cfg: OrcCfg, P, with_absum: bool = False):
    """Horizon (Mdot, phi_B, Ldot, Edot, Phi_B), the radial profiles [6][n1] (Mdot, phi_B, Ldot,
    Edot, ldot_in, ldot_out per radial cell) and the horizon index; with_absum also returns the
    per-shell sums of the magnitudes of the terms (the rounding scale of each signed sum)."""
    P = _arr(P, (8, cfg.n1, cfg.n2, cfg.n3))
    hz = np.full(5, np.nan)
    rad = np.empty((6, cfg.n1))
    ab = np.empty((6, cfg.n1))
    ih = lib().orc_diag_full(ctypes.byref(cfg), _dp(P), _dp(hz), _dp(rad), _dp(ab))
    if with_absum:
        return hz, rad, ih, ab
    return hz, rad, ih


def ppm_face(q6):
    """PPM (left, right) states on the face between cells 2 and 3 of six cell values."""
    q = np.ascontiguousarray(q6, dtype=np.float64)
    l, r = ctypes.c_double(), ctypes.c_double()
    lib().orc_ppm_face(_dp(q), ctypes.byref(l), ctypes.byref(r))
    return l.value, r.value


def grid_x1(cfg: OrcCfg):
    """(lower X1 face, X1 cell width) of the grid."""
    lo, dx = ctypes.c_double(), ctypes.c_double()
    lib().orc_grid_x1(ctypes.byref(cfg), ctypes.byref(lo), ctypes.byref(dx))
    return lo.value, dx.value


def geom(cfg: OrcCfg, X1: float, X2: float):
    gcov = np.zeros((4, 4))
    gcon = np.zeros((4, 4))
    conn = np.zeros((4, 4, 4))
    gdet = ctypes.c_double(0.0)
    lib().orc_geom(ctypes.byref(cfg), X1, X2, _dp(gcov), _dp(gcon), ctypes.byref(gdet), _dp(conn))
    return gcov, gcon, gdet.value, conn


def point_state(cfg: OrcCfg, X1: float, X2: float, P):
    P = _arr(P, (8,))
    out = {k: np.zeros(4) for k in ("ucon", "ucov", "bcon", "bcov")}
    U, F1, F2, F3 = (np.zeros(9) for _ in range(4))
    speeds = np.zeros(6)
    src = np.zeros(4)
    lib().orc_point_state(ctypes.byref(cfg), X1, X2, _dp(P), _dp(out["ucon"]), _dp(out["ucov"]),
                          _dp(out["bcon"]), _dp(out["bcov"]), _dp(U), _dp(F1), _dp(F2), _dp(F3),
                          _dp(speeds), _dp(src))
    out.update(U=U, F=[U, F1, F2, F3], speeds=speeds.reshape(3, 2), src=src)
    return out


def point_c2p(cfg: OrcCfg, X1: float, X2: float, U, Pguess, mode: int = 0):
    U = _arr(U, (9,))
    Pg = _arr(Pguess, (8,))
    P = np.zeros(8)
    m = lib().orc_point_c2p(ctypes.byref(cfg), X1, X2, _dp(U), _dp(Pg), _dp(P), int(mode))
    return P, m


def point_floors(cfg: OrcCfg, X1: float, X2: float, P):
    P = _arr(P, (8,))
    lib().orc_point_floors(ctypes.byref(cfg), X1, X2, _dp(P))
    return P


def mc_slope(qm: float, q0: float, qp: float) -> float:
    return lib().orc_mc_slope(float(qm), float(q0), float(qp))


def fixups(cfg: OrcCfg, Pout, Pin, code):
    """Run the neighbour-averaging fixup rounds; returns (P, code, cells left unfixed)."""
    Pout = _arr(Pout, (8, cfg.n1, cfg.n2, cfg.n3))
    Pin = _arr(Pin, (8, cfg.n1, cfg.n2, cfg.n3))
    code = np.ascontiguousarray(code, dtype=np.int8).copy()
    left = lib().orc_fixups(ctypes.byref(cfg), _dp(Pout), _dp(Pin), _bp(code))
    return Pout, code, int(left)


def ghosts(cfg: OrcCfg, P):
    """The interior state P[8][n1][n2][n3] with the boundary ghosts of Sec. 4.1 filled as a stage
    fills them (polar interpolation first when the run sets it), returned with its ghost layers:
    [8][n1 + 2 g1][n2 + 2 g2][n3 + 2 g3], g = 2 (PLM) or 3 (PPM) in every active direction."""
    P = _arr(P, (8, cfg.n1, cfg.n2, cfg.n3))
    g = 3 if cfg.recon == 1 else 2
    shp = [n + (2 * g if n > 1 else 0) for n in (cfg.n1, cfg.n2, cfg.n3)]
    out = np.zeros((8,) + tuple(shp))
    rc = lib().orc_ghosts(ctypes.byref(cfg), _dp(P), _dp(out))
    if rc != 0:
        raise RuntimeError(f"orc_ghosts failed ({rc})")
    return out
