"""Thin ctypes binding of the jfmg C-ABI (include/jfmg.h).

Argument marshalling only: every numerical step runs in the HIP kernels of
libjfmg.so.  PyTorch provides device memory (the workspace and the vectors)
and the HIP stream.  There is no CPU fallback: the library must be built
(``python -m paper_2505_24504_amd.build``) and a GPU must be present.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjfmg.so")

OK, EINVAL, ENOMEM, ENOCONV, ENONFINITE, ESTATE, EDEVICE = range(7)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "ENOCONV", 4: "ENONFINITE", 5: "ESTATE", 6: "EDEVICE"}


class JfmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"jfmg {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Config(C.Structure):
    _fields_ = [(n, C.c_int) for n in (
        "nx", "nz", "k", "physics", "background", "bc", "scheme", "newton_maxit", "gmres_m",
        "gmres_max_restarts", "fd_eps_mode", "mg_levels", "rk_stages", "mass_fix", "mg_precision",
        "precond")] + [("mg_key", C.c_char * 16)] + [(n, C.c_double) for n in (
        "x0", "x1", "z0", "z1", "g", "gamma", "R", "p0", "theta0", "N", "u_mean", "mu", "c_ip", "dt",
        "newton_rtol", "ew_gamma", "ew_alpha", "ew_eta0", "ew_eta_max")] + [
        ("rk_alpha", C.c_double * 4), ("pseudo_cfl", C.c_double), ("newton_stall", C.c_double),
        ("batch", C.c_int), ("transfer", C.c_int), ("pseudo_cfl_dg", C.c_double)]


class Perturbation(C.Structure):
    _fields_ = [("shape", C.c_int), ("pad", C.c_int)] + [
        (n, C.c_double) for n in ("amp", "xc", "zc", "xr", "zr", "a", "Z")]


class Stats(C.Structure):
    _fields_ = [("newton_its", C.c_int), ("gmres_its", C.c_int), ("lh_evals", C.c_int), ("jvps", C.c_int),
                ("fv_matvecs", C.c_int * 8), ("host_syncs", C.c_int), ("status", C.c_int),
                ("stall_stops", C.c_int), ("reorth_its", C.c_int),
                ("g0_norm", C.c_double), ("g_norm", C.c_double), ("seconds", C.c_double),
                ("reached_rtol", C.c_double)]

    def as_dict(self):
        return {"newton_its": self.newton_its, "gmres_its": self.gmres_its, "lh_evals": self.lh_evals,
                "jvps": self.jvps, "fv_matvecs": list(self.fv_matvecs), "host_syncs": self.host_syncs,
                "status": self.status, "stall_stops": self.stall_stops, "reorth_its": self.reorth_its, "g0_norm": self.g0_norm,
                "g_norm": self.g_norm,
                "seconds": self.seconds, "reached_rtol": self.reached_rtol}


_lib = None

EXPORTS = [
    "jfmg_config_default", "jfmg_workspace_bytes", "jfmg_create_problem", "jfmg_destroy_problem",
    "jfmg_num_dofs", "jfmg_fv_size", "jfmg_initial_state", "jfmg_residual", "jfmg_stage_residual",
    "jfmg_linearize", "jfmg_jvp", "jfmg_mg_apply", "jfmg_implicit_step", "jfmg_explicit_steps", "jfmg_transfer",
    "jfmg_restrict", "jfmg_prolong", "jfmg_fv_level_state", "jfmg_fv_dtau", "jfmg_dg_dtau", "jfmg_fv_matvec",
    "jfmg_mg_fv", "jfmg_subgrid_map", "jfmg_profile_enable", "jfmg_profile_read", "jfmg_last_error",
    "jfmg_batch_create", "jfmg_batch_destroy", "jfmg_batch_admit", "jfmg_batch_member", "jfmg_batch_run",
    "jfmg_batch_start", "jfmg_batch_stop", "jfmg_batch_wait_any", "jfmg_batch_poll", "jfmg_batch_retire",
    "jfmg_batch_arena_free", "jfmg_batch_last_error", "jfmg_get_tiles", "jfmg_set_tiles", "jfmg_autotune",
    "jfmg_stage_residual_noalloc", "jfmg_newton_stage", "jfmg_ensemble_workspace_bytes", "jfmg_create_ensemble",
    "jfmg_member_dofs",
]

# FV operator tile shapes (jfmg_tile), by index
TILES = ["64x4", "64x8", "16x4", "8x4", "32x4", "64x4_512"]

KERNEL_CLASSES = ["dg_residual", "dg_jvp", "fv_stage", "fv_stage_zero", "fv_defect_restrict",
                  "fv_prolong_correct", "fv_linearize", "transfer_T", "transfer_Tinv", "multidot",
                  "update", "fv_stage_small", "dg_smooth", "dg_linearize"]


def load_library(path: str = LIB_PATH):
    """Load libjfmg.so and declare the C signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libjfmg.so is not built ({path}); run __graft_entry__.build()")
    L = C.CDLL(path)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)
    sig = {
        "jfmg_config_default": (C.c_int, [C.POINTER(Config)]),
        "jfmg_workspace_bytes": (C.c_int, [C.POINTER(Config), C.POINTER(C.c_size_t)]),
        "jfmg_create_problem": (C.c_int, [C.POINTER(Config), vp, C.c_size_t, vp, C.POINTER(vp)]),
        "jfmg_destroy_problem": (C.c_int, [vp]),
        "jfmg_num_dofs": (C.c_size_t, [vp]),
        "jfmg_fv_size": (C.c_size_t, [vp, C.c_int]),
        "jfmg_initial_state": (C.c_int, [vp, C.POINTER(Perturbation), vp]),
        "jfmg_residual": (C.c_int, [vp, vp, vp, C.c_int]),
        "jfmg_stage_residual": (C.c_int, [vp, vp, vp, C.c_double, vp, dp]),
        "jfmg_linearize": (C.c_int, [vp, vp, C.c_double]),
        "jfmg_jvp": (C.c_int, [vp, vp, vp]),
        "jfmg_mg_apply": (C.c_int, [vp, vp, vp]),
        "jfmg_implicit_step": (C.c_int, [vp, vp, C.POINTER(Stats)]),
        "jfmg_explicit_steps": (C.c_int, [vp, vp, C.c_double, C.c_int]),
        "jfmg_transfer": (C.c_int, [vp, C.c_int, vp, vp]),
        "jfmg_restrict": (C.c_int, [vp, C.c_int, vp, vp]),
        "jfmg_prolong": (C.c_int, [vp, C.c_int, vp, vp]),
        "jfmg_fv_level_state": (C.c_int, [vp, C.c_int, vp]),
        "jfmg_fv_dtau": (C.c_int, [vp, C.c_int, dp]),
        "jfmg_dg_dtau": (C.c_int, [vp, dp]),
        "jfmg_fv_matvec": (C.c_int, [vp, C.c_int, vp, vp]),
        "jfmg_mg_fv": (C.c_int, [vp, vp, vp]),
        "jfmg_subgrid_map": (C.c_int, [vp, vp]),
        "jfmg_profile_enable": (C.c_int, [vp, C.c_uint]),
        "jfmg_profile_read": (C.c_int, [vp, dp, C.POINTER(C.c_longlong), dp]),
        "jfmg_last_error": (C.c_char_p, [vp]),
        "jfmg_batch_create": (C.c_int, [C.c_size_t, vp, C.c_int, C.c_int, vp, C.POINTER(vp)]),
        "jfmg_batch_destroy": (C.c_int, [vp]),
        "jfmg_batch_admit": (C.c_int, [vp, C.POINTER(Config), C.POINTER(Perturbation), vp, C.c_int, ip]),
        "jfmg_batch_member": (vp, [vp, C.c_int]),
        "jfmg_batch_run": (C.c_int, [vp, C.c_int]),
        "jfmg_batch_start": (C.c_int, [vp]),
        "jfmg_batch_stop": (C.c_int, [vp]),
        "jfmg_batch_wait_any": (C.c_int, [vp, C.c_double, ip]),
        "jfmg_batch_poll": (C.c_int, [vp, C.c_int, ip, ip, C.POINTER(Stats)]),
        "jfmg_batch_retire": (C.c_int, [vp, C.c_int]),
        "jfmg_batch_arena_free": (C.c_size_t, [vp]),
        "jfmg_batch_last_error": (C.c_char_p, [vp]),
        "jfmg_get_tiles": (C.c_int, [vp, ip]),
        "jfmg_set_tiles": (C.c_int, [vp, ip]),
        "jfmg_autotune": (C.c_int, [vp, C.c_int, ip, dp]),
        "jfmg_stage_residual_noalloc": (C.c_int, [C.POINTER(Config), vp, vp, C.c_double, vp, vp, vp]),
        "jfmg_newton_stage": (C.c_int, [vp, vp, C.c_double, vp, C.POINTER(Stats)]),
        "jfmg_ensemble_workspace_bytes": (C.c_int, [C.POINTER(Config), C.c_int, C.POINTER(C.c_size_t)]),
        "jfmg_create_ensemble": (C.c_int, [C.POINTER(Config), C.c_int, vp, C.c_size_t, vp, C.POINTER(vp)]),
        "jfmg_member_dofs": (C.c_size_t, [vp, C.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def make_config(d: dict) -> Config:
    """Map a problem description dict (paper_2505_24504_amd.workloads) onto jfmg_config."""
    L = load_library()
    c = Config()
    L.jfmg_config_default(C.byref(c))
    ints = ("nx", "nz", "k", "physics", "background", "bc", "scheme", "newton_maxit", "gmres_m",
            "gmres_max_restarts", "fd_eps_mode", "mg_levels", "rk_stages", "mass_fix", "mg_precision",
            "precond", "batch", "transfer")
    dbls = ("x0", "x1", "z0", "z1", "g", "gamma", "R", "p0", "theta0", "N", "u_mean", "mu", "c_ip", "dt",
            "newton_rtol", "ew_gamma", "ew_alpha", "ew_eta0", "ew_eta_max", "pseudo_cfl", "newton_stall",
            "pseudo_cfl_dg")
    for n in ints:
        if n in d:
            setattr(c, n, int(d[n]))
    for n in dbls:
        if n in d:
            setattr(c, n, float(d[n]))
    c.mg_key = d.get("mg_key", "mg002222V").encode()
    alpha = d.get("rk_alpha") or []
    for j in range(4):
        c.rk_alpha[j] = float(alpha[j]) if j < len(alpha) else 0.0
    return c


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return C.c_void_p(t.data_ptr())


def workspace_bytes(d: dict) -> int:
    L = load_library()
    cfg = make_config(d)
    n = C.c_size_t()
    rc = L.jfmg_workspace_bytes(C.byref(cfg), C.byref(n))
    if rc:
        raise JfmgError(rc, L.jfmg_last_error(None).decode())
    return n.value


def _configs(ds):
    arr = (Config * len(ds))()
    for i, d in enumerate(ds):
        arr[i] = make_config(d)
    return arr


def ensemble_workspace_bytes(ds) -> int:
    """Workspace bytes of a ragged batch of the member descriptions ds."""
    L = load_library()
    n = C.c_size_t()
    rc = L.jfmg_ensemble_workspace_bytes(_configs(ds), len(ds), C.byref(n))
    if rc:
        raise JfmgError(rc, L.jfmg_last_error(None).decode())
    return n.value


class Problem:
    """One problem in a device workspace owned by this object (a torch tensor)."""

    def __init__(self, d, device="cuda", stream=None, workspace=None):
        """d: a problem description, or a list of them for a ragged batch (ensemble members
        of different grid sizes in one problem)."""
        self.L = load_library()
        ragged = isinstance(d, (list, tuple))
        self.d = [dict(x) for x in d] if ragged else dict(d)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if ragged:
            self.cfgs = _configs(d)
            self.cfg = self.cfgs[0]
            nbytes = ensemble_workspace_bytes(d)
        else:
            self.cfg = make_config(d)
            nbytes = workspace_bytes(d)
        self.ws_bytes = nbytes
        if workspace is None:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self.ws = workspace
        base = workspace.data_ptr()
        off = (-base) % 256
        h = C.c_void_p()
        if ragged:
            rc = self.L.jfmg_create_ensemble(self.cfgs, len(d), C.c_void_p(base + off), nbytes,
                                             C.c_void_p(self.stream.cuda_stream), C.byref(h))
        else:
            rc = self.L.jfmg_create_problem(C.byref(self.cfg), C.c_void_p(base + off), nbytes,
                                            C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc:
            raise JfmgError(rc, self.L.jfmg_last_error(None).decode())
        self.h = h
        self.ragged = ragged
        self.members = len(d) if ragged else max(1, int(self.cfg.batch))   # batch size
        # DG entries of each member; state vectors hold the members back to back
        self.member_ndof = [self.L.jfmg_member_dofs(h, m) for m in range(self.members)]
        self.ndof = self.L.jfmg_num_dofs(h)            # per member (the envelope's in a ragged batch)
        self.fv_dtype = torch.float32 if self.cfg.mg_precision == 32 else torch.float64

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.L.jfmg_destroy_problem(h)
            self.h = None

    def _check(self, rc):
        if rc:
            raise JfmgError(rc, self.L.jfmg_last_error(self.h).decode())

    # ---- vectors ----
    def dg_zeros(self):
        return torch.zeros(self.ndof, dtype=torch.float64, device=self.device)

    def state_zeros(self):
        """A state of every member, members back to back."""
        return torch.zeros(sum(self.member_ndof), dtype=torch.float64, device=self.device)

    def member_slices(self):
        """The slice of each member in a state vector."""
        out, o = [], 0
        for n in self.member_ndof:
            out.append(slice(o, o + n))
            o += n
        return out

    def fv_size(self, level=0):
        return self.L.jfmg_fv_size(self.h, level)

    def fv_zeros(self, level=0):
        return torch.zeros(self.fv_size(level), dtype=self.fv_dtype, device=self.device)

    # ---- entry points ----
    def initial_state(self, pert: dict):
        P = _perturbation(pert)
        U = self.state_zeros()
        self._check(self.L.jfmg_initial_state(self.h, C.byref(P), _ptr(U)))
        return U

    def residual(self, U, apply_minv=False):
        out = self.dg_zeros()
        self._check(self.L.jfmg_residual(self.h, _ptr(U), _ptr(out), int(apply_minv)))
        return out

    def stage_residual(self, U, Ubar, alpha_dt):
        G = self.dg_zeros()
        nrm = C.c_double()
        self._check(self.L.jfmg_stage_residual(self.h, _ptr(U), _ptr(Ubar), float(alpha_dt), _ptr(G),
                                               C.byref(nrm)))
        return G, nrm.value

    def linearize(self, U, alpha_dt):
        self._check(self.L.jfmg_linearize(self.h, _ptr(U), float(alpha_dt)))

    def jvp(self, y):
        out = self.dg_zeros()
        self._check(self.L.jfmg_jvp(self.h, _ptr(y), _ptr(out)))
        return out

    def mg_apply(self, r):
        z = self.dg_zeros()
        self._check(self.L.jfmg_mg_apply(self.h, _ptr(r), _ptr(z)))
        return z

    def implicit_step(self, U, raise_on_error=True):
        """Advance U (device tensor) in place by one implicit step; returns the stats dict."""
        st = Stats()
        rc = self.L.jfmg_implicit_step(self.h, _ptr(U), C.byref(st))
        d = st.as_dict()
        d["status"] = rc
        if rc and raise_on_error:
            self._check(rc)
        return d

    def newton_stage(self, Ubar, alpha_dt, raise_on_error=True):
        """Solve the stage equation U - alpha_dt f(U) - Ubar = 0; returns (U, stats)."""
        U = self.dg_zeros()
        st = Stats()
        rc = self.L.jfmg_newton_stage(self.h, _ptr(Ubar), float(alpha_dt), _ptr(U), C.byref(st))
        d = st.as_dict()
        d["status"] = rc
        if rc and raise_on_error:
            self._check(rc)
        return U, d

    def explicit_steps(self, U, dt, nsteps):
        """Advance U (device tensor) in place by nsteps explicit SSP RK(4,3) steps of size dt."""
        self._check(self.L.jfmg_explicit_steps(self.h, _ptr(U), float(dt), int(nsteps)))

    def transfer(self, direction, x):
        if direction == 0:
            out = self.fv_zeros(0)
        else:
            out = self.dg_zeros()
        self._check(self.L.jfmg_transfer(self.h, int(direction), _ptr(x), _ptr(out)))
        return out

    def restrict(self, fine_level, x):
        out = self.fv_zeros(fine_level + 1)
        self._check(self.L.jfmg_restrict(self.h, fine_level, _ptr(x), _ptr(out)))
        return out

    def prolong(self, coarse_level, x):
        out = self.fv_zeros(coarse_level - 1)
        self._check(self.L.jfmg_prolong(self.h, coarse_level, _ptr(x), _ptr(out)))
        return out

    def fv_level_state(self, level):
        out = self.fv_zeros(level)
        self._check(self.L.jfmg_fv_level_state(self.h, level, _ptr(out)))
        return out

    def fv_dtau(self, level):
        v = C.c_double()
        self._check(self.L.jfmg_fv_dtau(self.h, level, C.byref(v)))
        return v.value

    def dg_dtau(self):
        v = C.c_double()
        self._check(self.L.jfmg_dg_dtau(self.h, C.byref(v)))
        return v.value

    def fv_matvec(self, level, x):
        out = self.fv_zeros(level)
        self._check(self.L.jfmg_fv_matvec(self.h, level, _ptr(x), _ptr(out)))
        return out

    def mg_fv(self, b):
        x = self.fv_zeros(0)
        self._check(self.L.jfmg_mg_fv(self.h, _ptr(b), _ptr(x)))
        return x

    def profile_enable(self, classes=()):
        mask = 0
        for c in classes:
            mask |= 1 << KERNEL_CLASSES.index(c)
        self._check(self.L.jfmg_profile_enable(self.h, mask))

    def profile_read(self):
        n = len(KERNEL_CLASSES)
        ms = (C.c_double * n)()
        cnt = (C.c_longlong * n)()
        by = (C.c_double * n)()
        self._check(self.L.jfmg_profile_read(self.h, ms, cnt, by))
        return {KERNEL_CLASSES[i]: {"ms": ms[i], "launches": cnt[i], "bytes": by[i]} for i in range(n)}

    def subgrid_map(self):
        out = torch.zeros(self.fv_size(0) // 4, dtype=torch.int32, device=self.device)
        self._check(self.L.jfmg_subgrid_map(self.h, _ptr(out)))
        return out

    def get_tiles(self):
        """Tile shape names of the FV operator kernels, finest level first."""
        n = int(self.cfg.mg_levels)
        a = (C.c_int * n)()
        self._check(self.L.jfmg_get_tiles(self.h, a))
        return [TILES[a[i]] for i in range(n)]

    def set_tiles(self, shapes):
        n = int(self.cfg.mg_levels)
        if len(shapes) != n:
            raise ValueError(f"{n} shapes expected")
        a = (C.c_int * n)(*[TILES.index(s) if isinstance(s, str) else int(s) for s in shapes])
        self._check(self.L.jfmg_set_tiles(self.h, a))

    def autotune(self, reps: int = 10):
        """Time every tile shape on every level (needs linearize) and keep the
        fastest; returns (shapes, {level: {shape: mean us per launch}})."""
        n = int(self.cfg.mg_levels)
        a = (C.c_int * n)()
        t = (C.c_double * (n * len(TILES)))()
        self._check(self.L.jfmg_autotune(self.h, int(reps), a, t))
        times = {l: {TILES[s]: t[l * len(TILES) + s] for s in range(len(TILES))} for l in range(n)}
        return [TILES[a[i]] for i in range(n)], times


def stage_residual_noalloc(d: dict, U, Ubar, alpha_dt, G=None, norm2=None, stream=None):
    """jfmg_stage_residual_noalloc: G = U - alpha_dt f(U) - Ubar and ||G||^2 into the
    device tensors G and norm2 (one FP64 entry), without a problem or a workspace;
    returns (G, norm2).  Stream ordered on `stream` (default: torch's current one)."""
    L = load_library()
    cfg = make_config(d)
    if G is None:
        G = torch.empty_like(U)
    if norm2 is None:
        norm2 = torch.empty(1, dtype=torch.float64, device=U.device)
    st = stream if stream is not None else torch.cuda.current_stream(U.device)
    rc = L.jfmg_stage_residual_noalloc(C.byref(cfg), _ptr(U), _ptr(Ubar), float(alpha_dt), _ptr(G), _ptr(norm2),
                                       C.c_void_p(st.cuda_stream))
    if rc:
        raise JfmgError(rc, L.jfmg_last_error(None).decode())
    return G, norm2


def num_dofs(d: dict) -> int:
    """N = 4 nx nz (k+1)^2 of a problem description."""
    return 4 * int(d["nx"]) * int(d["nz"]) * (int(d["k"]) + 1) ** 2


def _perturbation(pert: dict) -> Perturbation:
    P = Perturbation()
    P.shape = int(pert.get("shape", 0))
    for n in ("amp", "xc", "zc", "xr", "zr", "a", "Z"):
        setattr(P, n, float(pert.get(n, 1.0)))
    return P


class Batch:
    """Independent members advanced concurrently from one device arena
    (jfmg_batch_*).  The arena (a torch uint8 tensor of arena_bytes) is the HBM
    budget of the batch; each member's state is a torch FP64 tensor."""

    def __init__(self, arena_bytes: int, max_members: int, workers: int = 0, device="cuda", stream=None):
        self.L = load_library()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=self.device)
        base = self.arena.data_ptr()
        off = (-base) % 256
        h = C.c_void_p()
        rc = self.L.jfmg_batch_create(int(arena_bytes), C.c_void_p(base + off), int(max_members), int(workers),
                                      C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc:
            raise JfmgError(rc, "jfmg_batch_create failed")
        self.h = h
        self.U = {}
        self.cfgs = {}

    def _check(self, rc):
        if rc:
            raise JfmgError(rc, self.L.jfmg_batch_last_error(self.h).decode())

    def admit(self, d: dict, n_steps: int, pert: dict = None, U=None):
        """Admit a member; returns its slot, or None when the arena or the slots are full.
        With pert, U is set to that initial state (on the batch stream)."""
        if U is None:
            U = torch.zeros(num_dofs(d), dtype=torch.float64, device=self.device)
        cfg = make_config(d)
        slot = C.c_int(-1)
        P = C.byref(_perturbation(pert)) if pert is not None else None
        rc = self.L.jfmg_batch_admit(self.h, C.byref(cfg), P, _ptr(U), int(n_steps), C.byref(slot))
        if rc == ENOMEM:
            return None
        self._check(rc)
        self.U[slot.value] = U
        self.cfgs[slot.value] = cfg
        return slot.value

    def autotune(self, slot: int, reps: int = 5):
        """Tune the FV tile shapes of a member that has not started (jfmg_autotune on
        the member's problem, linearized at its current state with its stage alpha dt);
        returns the shapes, finest level first."""
        h = self.L.jfmg_batch_member(self.h, int(slot))
        if not h:
            raise JfmgError(EINVAL, f"no member in slot {slot}")
        torch.cuda.synchronize(self.device)   # the member state may come from another stream
        cfg = self.cfgs[slot]
        alpha = 1.0 if cfg.scheme == 0 else 1.0 - 2.0 ** -0.5
        rc = self.L.jfmg_linearize(C.c_void_p(h), _ptr(self.U[slot]), alpha * cfg.dt)
        if rc:
            raise JfmgError(rc, self.L.jfmg_last_error(C.c_void_p(h)).decode())
        n = int(cfg.mg_levels)
        a = (C.c_int * n)()
        rc = self.L.jfmg_autotune(C.c_void_p(h), int(reps), a, None)
        if rc:
            raise JfmgError(rc, self.L.jfmg_last_error(C.c_void_p(h)).decode())
        return [TILES[a[i]] for i in range(n)]

    def run(self, max_steps: int = 0):
        self._check(self.L.jfmg_batch_run(self.h, int(max_steps)))

    def start(self):
        self._check(self.L.jfmg_batch_start(self.h))

    def stop(self):
        self._check(self.L.jfmg_batch_stop(self.h))

    def wait_any(self, timeout_s: float = -1.0):
        """Slot of a member that finished (each reported once), or None."""
        s = C.c_int(-1)
        self._check(self.L.jfmg_batch_wait_any(self.h, float(timeout_s), C.byref(s)))
        return s.value if s.value >= 0 else None

    def poll(self, slot: int):
        fin, steps, st = C.c_int(), C.c_int(), Stats()
        rc = self.L.jfmg_batch_poll(self.h, int(slot), C.byref(fin), C.byref(steps), C.byref(st))
        d = st.as_dict()
        d["status"] = rc
        return bool(fin.value), steps.value, d

    def retire(self, slot: int):
        """Destroy the member and return its state tensor."""
        self._check(self.L.jfmg_batch_retire(self.h, int(slot)))
        return self.U.pop(slot)

    def arena_free(self) -> int:
        return self.L.jfmg_batch_arena_free(self.h)

    def close(self):
        h = getattr(self, "h", None)
        if h:
            self.L.jfmg_batch_destroy(h)
            self.h = None

    def __del__(self):
        self.close()
