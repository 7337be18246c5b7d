"""ctypes wrapper of the FP64 CPU oracle (oracle/orc.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke()`` and
by the ``cpu_baseline`` leg of ``bench.py``.  The product package never imports
it.  Problem descriptions are plain dicts (see
``paper_2505_24504_amd.workloads``); this module maps them onto the oracle's
own C struct and parses the multigrid key ``mg a b c d e f G`` itself.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_SRC = os.path.join(_HERE, "orc.c")
# ORC_LIB names another build of orc.c to load (the sanitizer test's)
_LOAD_PATH = os.environ.get("ORC_LIB") or _LIB_PATH

GCC_CMD = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-o", _LIB_PATH, _SRC, "-lm"]


def build() -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction, OpenMP over the
    element and cell loops)."""
    subprocess.check_call(GCC_CMD)
    return _LIB_PATH


class OrcCfg(C.Structure):
    _fields_ = [(n, C.c_int) for n in (
        "nx", "nz", "k", "physics", "background", "bc", "mass_fix", "transfer", "mg_levels",
        "nu_pre_fine", "nu_post_fine", "nu_pre", "nu_post", "cycle", "rk_stages",
        "fd_eps_mode", "gmres_m", "gmres_max_restarts", "newton_maxit", "scheme",
        "precond")] + [(n, C.c_double) for n in (
        "x0", "x1", "z0", "z1", "g", "gamma", "R", "p0", "theta0", "N", "u_mean",
        "mu", "c_ip")] + [("rk_alpha", C.c_double * 4)] + [(n, C.c_double) for n in (
        "pseudo_cfl", "newton_rtol", "ew_gamma", "ew_alpha", "ew_eta0", "ew_eta_max",
        "dt", "newton_stall")] + [("nu_pre_dg", C.c_int), ("nu_post_dg", C.c_int),
                                  ("pseudo_cfl_dg", C.c_double)]


class OrcPert(C.Structure):
    _fields_ = [("shape", C.c_int), ("pad", C.c_int)] + [
        (n, C.c_double) for n in ("amp", "xc", "zc", "xr", "zr", "a", "Z")]


class OrcStats(C.Structure):
    _fields_ = [("newton_its", C.c_int), ("gmres_its", C.c_int), ("lh_evals", C.c_int),
                ("jvps", C.c_int), ("fv_matvecs", C.c_int * 8), ("status", C.c_int),
                ("stalls", C.c_int), ("g0_norm", C.c_double), ("g_norm", C.c_double)]

    def as_dict(self):
        return {"newton_its": self.newton_its, "gmres_its": self.gmres_its,
                "lh_evals": self.lh_evals, "jvps": self.jvps,
                "fv_matvecs": list(self.fv_matvecs), "status": self.status,
                "stalls": self.stalls, "g0_norm": self.g0_norm, "g_norm": self.g_norm}


_OP = C.CFUNCTYPE(None, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double))
_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LOAD_PATH == _LIB_PATH and (not os.path.exists(_LIB_PATH)
                                        or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build()
        L = C.CDLL(_LOAD_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(OrcCfg)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_num_dofs.restype = C.c_long
        L.orc_num_dofs.argtypes = [C.c_void_p]
        L.orc_fv_dims.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_ref_tables.argtypes = [C.c_int] + [dp] * 10
        L.orc_proj_tables.argtypes = [C.c_int, dp, dp]
        L.orc_background.argtypes = [C.c_void_p, C.c_double, dp, dp]
        L.orc_flux.argtypes = [C.c_void_p, dp, C.c_double, C.c_double, dp]
        L.orc_hllc.argtypes = [C.c_void_p, dp, dp, C.c_double, C.c_double, dp]
        L.orc_initial_state.argtypes = [C.c_void_p, C.POINTER(OrcPert), dp]
        L.orc_residual.argtypes = [C.c_void_p, dp, dp, C.c_int]
        L.orc_stage_residual.argtypes = [C.c_void_p, dp, dp, C.c_double, dp]
        L.orc_transfer_T.argtypes = [C.c_void_p, dp, dp]
        L.orc_transfer_Tinv.argtypes = [C.c_void_p, dp, dp]
        L.orc_restrict.argtypes = [C.c_void_p, C.c_int, dp, dp]
        L.orc_prolong.argtypes = [C.c_void_p, C.c_int, dp, dp]
        L.orc_fv_residual.argtypes = [C.c_void_p, C.c_int, dp, dp]
        L.orc_subgrid_map.argtypes = [C.c_void_p, C.POINTER(C.c_int)]
        L.orc_linearize.argtypes = [C.c_void_p, dp, C.c_double]
        L.orc_fv_level_state.argtypes = [C.c_void_p, C.c_int, dp]
        L.orc_fv_dtau.restype = C.c_double
        L.orc_fv_dtau.argtypes = [C.c_void_p, C.c_int]
        L.orc_dg_dtau.restype = C.c_double
        L.orc_dg_dtau.argtypes = [C.c_void_p]
        L.orc_fv_matvec.argtypes = [C.c_void_p, C.c_int, dp, dp]
        L.orc_counters.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                   C.c_int]
        L.orc_jvp.argtypes = [C.c_void_p, dp, dp]
        L.orc_mg_fv.argtypes = [C.c_void_p, dp, dp]
        L.orc_mg_apply.argtypes = [C.c_void_p, dp, dp]
        L.orc_fgmres.argtypes = [C.c_long, _OP, C.c_void_p, _OP, C.c_void_p, dp, C.c_double,
                                 C.c_int, C.c_int, dp, C.POINTER(C.c_int)]
        L.orc_newton_stage.argtypes = [C.c_void_p, dp, C.c_double, dp, C.POINTER(OrcStats)]
        L.orc_implicit_step.argtypes = [C.c_void_p, dp, C.POINTER(OrcStats)]
        L.orc_explicit_steps.argtypes = [C.c_void_p, dp, C.c_double, C.c_int]
        _lib = L
    return _lib


def _p(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def parse_mg_key(key: str):
    """Parse the preconditioner key 'mg a b c d e f G' (one digit per count)."""
    if len(key) != 9 or not key.startswith("mg") or key[8] not in "VW" or not key[2:8].isdigit():
        raise ValueError(f"bad multigrid key {key!r}")
    a, b, c, d, e, f = (int(ch) for ch in key[2:8])
    return {"a": a, "b": b, "c": c, "d": d, "e": e, "f": f, "cycle": 1 if key[8] == "V" else 2}


def ref_tables(k: int):
    n = k + 1
    out = {name: np.zeros(shape) for name, shape in (
        ("xi", n), ("w", n), ("D", (n, n)), ("em", n), ("ep", n), ("dm", n), ("dp", n),
        ("V", (n, n)), ("Vinv", (n, n)), ("wnc", n))}
    rc = lib().orc_ref_tables(k, *[_p(out[nm]) for nm in (
        "xi", "w", "D", "em", "ep", "dm", "dp", "V", "Vinv", "wnc")])
    if rc:
        raise ValueError("k out of range")
    return out


def proj_tables(k: int):
    """L2 projection onto the k+1 subintervals: P[i][a] = mean of l_a over subinterval i, and P^-1."""
    n = k + 1
    P, Pinv = np.zeros((n, n)), np.zeros((n, n))
    if lib().orc_proj_tables(k, _p(P), _p(Pinv)):
        raise ValueError("k out of range")
    return P, Pinv


def make_cfg(d: dict) -> OrcCfg:
    c = OrcCfg()
    key = parse_mg_key(d.get("mg_key", "mg002222V"))
    for name in ("nx", "nz", "k"):
        setattr(c, name, int(d[name]))
    c.physics = int(d.get("physics", 0))
    c.background = int(d.get("background", 0))
    c.bc = int(d.get("bc", 0))
    c.mass_fix = int(d.get("mass_fix", 1))
    c.transfer = int(d.get("transfer", 0))
    c.mg_levels = int(d.get("mg_levels", 3))
    c.nu_pre_fine, c.nu_post_fine, c.nu_pre, c.nu_post = key["c"], key["d"], key["e"], key["f"]
    c.cycle = key["cycle"]
    c.nu_pre_dg, c.nu_post_dg = key["a"], key["b"]
    c.pseudo_cfl_dg = float(d.get("pseudo_cfl_dg", 1.0))
    c.rk_stages = int(d.get("rk_stages", 3))
    c.fd_eps_mode = int(d.get("fd_eps_mode", 1))
    c.gmres_m = int(d.get("gmres_m", 30))
    c.gmres_max_restarts = int(d.get("gmres_max_restarts", 10))
    c.newton_maxit = int(d.get("newton_maxit", 20))
    c.scheme = int(d.get("scheme", 1))
    c.precond = int(d.get("precond", 1))
    for name, default in (("x0", 0.0), ("x1", 1000.0), ("z0", 0.0), ("z1", 1000.0),
                          ("g", 9.81), ("gamma", 1.4), ("R", 287.0), ("p0", 1e5),
                          ("theta0", 300.0), ("N", 0.0), ("u_mean", 0.0), ("mu", 0.0),
                          ("c_ip", 2.0), ("pseudo_cfl", 1.0), ("newton_rtol", 1e-8),
                          ("ew_gamma", 0.1), ("ew_alpha", 1.0), ("ew_eta0", 0.1),
                          ("ew_eta_max", 0.9), ("dt", 1.0), ("newton_stall", 0.0)):
        setattr(c, name, float(d.get(name, default)))
    s = c.rk_stages
    alpha = d.get("rk_alpha") or [1.0 / (s - j) for j in range(s)]
    for j in range(4):
        c.rk_alpha[j] = float(alpha[j]) if j < len(alpha) else 0.0
    return c


def make_pert(p: dict) -> OrcPert:
    P = OrcPert()
    P.shape = int(p.get("shape", 0))
    for name in ("amp", "xc", "zc", "xr", "zr", "a", "Z"):
        setattr(P, name, float(p.get(name, 1.0)))
    return P


class Oracle:
    """One problem of the oracle: DG space, FV levels and linearization state."""

    def __init__(self, d: dict):
        self.d = dict(d)
        self.cfg = make_cfg(d)
        self.L = lib()
        self.h = self.L.orc_create(C.byref(self.cfg))
        if not self.h:
            raise ValueError("oracle rejected the configuration")
        self.ndof = self.L.orc_num_dofs(self.h)
        self.k = self.cfg.k
        self.np = (self.k + 1) ** 2

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_destroy(self.h)
            self.h = None

    def fv_dims(self, level):
        a, b = C.c_int(), C.c_int()
        if self.L.orc_fv_dims(self.h, level, C.byref(a), C.byref(b)):
            raise ValueError("level out of range")
        return a.value, b.value

    def fv_size(self, level):
        nx, nz = self.fv_dims(level)
        return 4 * nx * nz

    def background(self, z):
        Ub, dUb = np.zeros(4), np.zeros(4)
        self.L.orc_background(self.h, float(z), _p(Ub), _p(dUb))
        return Ub, dUb

    def flux(self, U, nx, nz):
        U = np.ascontiguousarray(U, dtype=np.float64)
        F = np.zeros(4)
        self.L.orc_flux(self.h, _p(U), float(nx), float(nz), _p(F))
        return F

    def hllc(self, UL, UR, nx, nz):
        UL = np.ascontiguousarray(UL, dtype=np.float64)
        UR = np.ascontiguousarray(UR, dtype=np.float64)
        F = np.zeros(4)
        self.L.orc_hllc(self.h, _p(UL), _p(UR), float(nx), float(nz), _p(F))
        return F

    def initial_state(self, pert: dict):
        U = np.zeros(self.ndof)
        P = make_pert(pert)
        self.L.orc_initial_state(self.h, C.byref(P), _p(U))
        return U

    def residual(self, U, mode=0):
        U = np.ascontiguousarray(U, dtype=np.float64)
        out = np.zeros(self.ndof)
        self.L.orc_residual(self.h, _p(U), _p(out), int(mode))
        return out

    def stage_residual(self, U, Ubar, alpha_dt):
        U = np.ascontiguousarray(U, dtype=np.float64)
        Ubar = np.ascontiguousarray(Ubar, dtype=np.float64)
        G = np.zeros(self.ndof)
        self.L.orc_stage_residual(self.h, _p(U), _p(Ubar), float(alpha_dt), _p(G))
        return G

    def transfer_T(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        u = np.zeros(self.fv_size(0))
        self.L.orc_transfer_T(self.h, _p(U), _p(u))
        return u

    def transfer_Tinv(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        U = np.zeros(self.ndof)
        self.L.orc_transfer_Tinv(self.h, _p(u), _p(U))
        return U

    def restrict(self, fine_level, uf):
        uf = np.ascontiguousarray(uf, dtype=np.float64)
        uc = np.zeros(self.fv_size(fine_level + 1))
        self.L.orc_restrict(self.h, fine_level, _p(uf), _p(uc))
        return uc

    def prolong(self, coarse_level, uc):
        uc = np.ascontiguousarray(uc, dtype=np.float64)
        uf = np.zeros(self.fv_size(coarse_level - 1))
        self.L.orc_prolong(self.h, coarse_level, _p(uc), _p(uf))
        return uf

    def fv_residual(self, level, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        f = np.zeros(self.fv_size(level))
        self.L.orc_fv_residual(self.h, level, _p(u), _p(f))
        return f

    def subgrid_map(self):
        n = self.fv_size(0) // 4
        out = np.zeros(n, dtype=np.int32)
        self.L.orc_subgrid_map(self.h, out.ctypes.data_as(C.POINTER(C.c_int)))
        return out

    def linearize(self, U, alpha_dt):
        U = np.ascontiguousarray(U, dtype=np.float64)
        return self.L.orc_linearize(self.h, _p(U), float(alpha_dt))

    def fv_level_state(self, level):
        u = np.zeros(self.fv_size(level))
        self.L.orc_fv_level_state(self.h, level, _p(u))
        return u

    def fv_dtau(self, level):
        return self.L.orc_fv_dtau(self.h, level)

    def dg_dtau(self):
        """Pseudo time step of the DG-level smoother (key counts a, b)."""
        return self.L.orc_dg_dtau(self.h)

    def counters(self, reset=False):
        """Operation counts since creation or the last reset: FV matvecs per level,
        DG JVPs and L_h calls (instrumentation; no arithmetic)."""
        mv = (C.c_int * 8)()
        j, lh = C.c_int(), C.c_int()
        self.L.orc_counters(self.h, mv, C.byref(j), C.byref(lh), int(bool(reset)))
        return {"fv_matvecs": list(mv), "jvps": j.value, "lh_evals": lh.value}

    def fv_matvec(self, level, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.zeros_like(x)
        self.L.orc_fv_matvec(self.h, level, _p(x), _p(out))
        return out

    def jvp(self, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        out = np.zeros(self.ndof)
        self.L.orc_jvp(self.h, _p(y), _p(out))
        return out

    def mg_fv(self, b):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b)
        self.L.orc_mg_fv(self.h, _p(b), _p(x))
        return x

    def mg_apply(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.zeros(self.ndof)
        self.L.orc_mg_apply(self.h, _p(r), _p(z))
        return z

    def newton_stage(self, Ubar, alpha_dt):
        Ubar = np.ascontiguousarray(Ubar, dtype=np.float64)
        U = np.zeros(self.ndof)
        st = OrcStats()
        rc = self.L.orc_newton_stage(self.h, _p(Ubar), float(alpha_dt), _p(U), C.byref(st))
        return rc, U, st.as_dict()

    def explicit_steps(self, U, dt, nsteps):
        """nsteps explicit SSP RK(4,3) steps of size dt; returns the new state."""
        U = np.array(U, dtype=np.float64, copy=True)
        self.L.orc_explicit_steps(self.h, _p(U), float(dt), int(nsteps))
        return U

    def implicit_step(self, U):
        U = np.array(U, dtype=np.float64, copy=True)
        st = OrcStats()
        rc = self.L.orc_implicit_step(self.h, _p(U), C.byref(st))
        d = st.as_dict()
        d["status"] = rc
        return rc, U, d


def fgmres(n, matvec, precond, rhs, tol_abs, m, max_restarts):
    """Oracle FGMRES on Python callables (used with assembled operators)."""
    def wrap(fn):
        def cb(_ctx, pin, pout):
            a = np.ctypeslib.as_array(pin, shape=(n,))
            b = np.ctypeslib.as_array(pout, shape=(n,))
            b[:] = fn(a.copy())
        return _OP(cb)
    A, P = wrap(matvec), wrap(precond)
    rhs = np.ascontiguousarray(rhs, dtype=np.float64)
    x = np.zeros(n)
    its = C.c_int()
    rc = lib().orc_fgmres(n, A, None, P, None, _p(rhs), float(tol_abs), m, max_restarts,
                          _p(x), C.byref(its))
    return rc, x, its.value
