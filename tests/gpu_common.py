"""Helpers shared by the GPU parity tests: build the same problem on both sides
(HIP library through the C-ABI, and the CPU oracle) from one description."""
import numpy as np
import torch

import oracle
from paper_2505_24504_amd import jfmg, workloads as W

DEV = "cuda:0"
EPS = 2.0 ** -52


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
