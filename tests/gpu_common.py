"""Helpers shared by the GPU parity tests: build the same problem on both sides
(HIP library through the C-ABI, and the CPU oracle) from one description."""
import numpy as np
import torch

import oracle
from paper_2505_24504_amd import jfmg, workloads as W

DEV = "cuda:0"
EPS = 2.0 ** -52

# Parity bounds: a constant times a scale the arithmetic fixes, the constant about 8x
# (never above 10x) the largest normalized error measured on MI355X.
C_LH = 4.0            # L_h: x eps ||sigma (/ m)||, sigma the rounding scale    (measured 0.41-0.50)
C_JVP = 5.0           # JVP: x (alpha dt / eps) eps ||sigma / m||               (measured 0.56-0.70)
C_FV = 1.65           # FV matvec: x (alpha dt / eps) eps (4 p0 / h) sqrt(n)    (measured 0.17-0.21)
REL_MG_FV = 1.1e-7    # one FV cycle, relative                                 (measured <= 1.34e-8)
REL_MG_APPLY = 2.25e-7  # Q^-1, relative                                       (measured <= 2.81e-8)
REL_STEP_BUBBLE = 1e-10   # relative L2 of U', 16x16 bubble steps              (measured <= 4.1e-11)
REL_STEP_SDIRK2 = 5e-11   # relative L2 of U', 8x8 SDIRK2 steps                (measured <= 6.2e-12)


def pair(d):
    return jfmg.Problem(d, device=DEV), oracle.Oracle(d)


def to_dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype=dtype)


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rand_state(o, seed, rel=1e-2):
    """Seeded perturbation with component scales of the background state."""
    return W.random_state(o.ndof, seed, [rel * 1.0, rel * 30.0, rel * 30.0, rel * 300.0])


def node_total_norm(o, d, U):
    """||U' + Ubar||_2 over all DG nodes, background from the oracle."""
    t = oracle.ref_tables(d["k"])
    n1 = d["k"] + 1
    dz = (d["z1"] - d["z0"]) / d["nz"]
    n = o.ndof // 4
    Ut = U.reshape(4, d["nz"], d["nx"], n1, n1).copy()
    for ez in range(d["nz"]):
        for b in range(n1):
            Ub, _ = o.background(d["z0"] + (ez + 0.5 * (1 + t["xi"][b])) * dz)
            for c in range(4):
                Ut[c, ez, :, b, :] += Ub[c]
    return float(np.sqrt((Ut ** 2).sum())), n


def dg_mass(d):
    t = oracle.ref_tables(d["k"])
    ww = np.kron(t["w"], t["w"])
    J = (d["x1"] - d["x0"]) / d["nx"] * (d["z1"] - d["z0"]) / d["nz"] / 4
    return np.tile(ww, d["nx"] * d["nz"]) * J


def fv_total_norm(o, d, lev, u):
    """||u + Ubar(cell centres)||_2 on FV level lev."""
    nx, nz = o.fv_dims(lev)
    hz = (d["z1"] - d["z0"]) / nz
    Ut = u.reshape(4, nz, nx).copy()
    for J in range(nz):
        Ub, _ = o.background(d["z0"] + (J + 0.5) * hz)
        for c in range(4):
            Ut[c, J, :] += Ub[c]
    return float(np.sqrt((Ut ** 2).sum()))


def fv_scale(o, d, lev, u, x, adt):
    """Rounding scale of the FD FV matvec: (alpha dt / eps) eps_mach (4 p0 / h) sqrt(n),
    f_low summing four face fluxes of size p / h per cell."""
    nx, nz = o.fv_dims(lev)
    h = min((d["x1"] - d["x0"]) / nx, (d["z1"] - d["z0"]) / nz)
    eps = np.sqrt(EPS) * fv_total_norm(o, d, lev, u) / np.linalg.norm(x)
    return (adt / eps) * EPS * (4 * 1.1e5 / h) * np.sqrt(x.size)


def lh_scale(o, d, U, minv):
    """Rounding scale of L_h (or M^-1 L_h): the 2-norm of the oracle's per-node sums of
    absolute values of the terms, before the background subtraction."""
    sig = o.residual(U, 3)
    if minv:
        sig = sig / np.tile(dg_mass(d), 4)
    return float(np.linalg.norm(sig))
