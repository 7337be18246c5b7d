"""Seeded synthetic workloads.

Problem descriptions are plain dicts of parameters; this module holds none of
the method's arithmetic (no fluxes, no transfers, no solver).  Both the GPU
binding and the CPU oracle take these dicts, so it is the one module the two
sides share.  The test cases are analytic (paper Sec. "Numerical
Experiments"): the workloads below take the shapes and value ranges of the
rising-bubble, density-current and inertia-gravity setups.
"""
from __future__ import annotations

import numpy as np

# Common physical constants: g = 9.81, gamma = 1.4, R = 287 for every workload.
PHYS = {"g": 9.81, "gamma": 1.4, "R": 287.0, "p0": 1.0e5}

# Weak perturbations (0.01 - 0.1 K) on fine grids put the rounding floor of the
# stage residual G near 1e-8 ||G^0|| (measured 1.25e-8), so the workloads with
# such perturbations let a stage end at that floor (newton_stall) instead of
# failing at the cap; the stall threshold sits a factor 8 above the floor.
STALL = 1e-7


def bubble_small():
    """16x16 quads, k = 1, warm cosine bubble, one implicit-Euler step."""
    d = dict(PHYS)
    d.update(nx=16, nz=16, k=1, x0=0.0, x1=1000.0, z0=0.0, z1=1000.0,
             physics=0, background=0, bc=0, theta0=300.0, N=0.0, u_mean=0.0, mu=0.0,
             scheme=0, dt=1.0, newton_rtol=1e-6, gmres_m=20, mg_levels=3,
             mg_key="mg002222V", rk_stages=3, mass_fix=1, fd_eps_mode=1, mg_precision=64)
    pert = dict(shape=0, amp=0.5, xc=500.0, zc=350.0, xr=250.0, zr=250.0)
    return d, pert, 1


def density_current():
    """256x64 quads on 25.6 km x 6.4 km, k = 3, viscous, cold bubble, 10 SDIRK2 steps.

    The smoother is the one-stage explicit Euler pseudo-time iteration, the one the
    paper's experiments use (Sec. "Smoother / Pseudo time iteration")."""
    d = dict(PHYS)
    d.update(nx=256, nz=64, k=3, x0=0.0, x1=25600.0, z0=0.0, z1=6400.0,
             physics=1, background=0, bc=0, theta0=300.0, N=0.0, u_mean=0.0, mu=75.0,
             scheme=1, dt=2.0, newton_rtol=1e-8, gmres_m=30, mg_levels=4,
             mg_key="mg002222V", rk_stages=1, mass_fix=1, fd_eps_mode=1, mg_precision=64)
    pert = dict(shape=0, amp=-15.0, xc=0.0, zc=3000.0, xr=4000.0, zr=2000.0)
    return d, pert, 10


def inertia_gravity(mg_precision=32):
    """600x20 quads on 300 km x 10 km, k = 3, stratified N = 0.01, mean wind 20 m/s.

    The smoother of this and the ensemble and serving workloads is the one-stage explicit
    Euler iteration of the paper's experiments, as for the density current."""
    d = dict(PHYS)
    d.update(nx=600, nz=20, k=3, x0=0.0, x1=300000.0, z0=0.0, z1=10000.0,
             physics=0, background=1, bc=1, theta0=300.0, N=0.01, u_mean=20.0, mu=0.0,
             scheme=1, dt=12.0, newton_rtol=1e-8, gmres_m=30, mg_levels=4,
             mg_key="mg002222V", rk_stages=1, mass_fix=1, fd_eps_mode=1,
             mg_precision=mg_precision, newton_stall=STALL)
    pert = dict(shape=1, amp=0.01, xc=100000.0, a=5000.0, Z=10000.0)
    return d, pert, 20


ENSEMBLE_GRIDS = [(32, 16), (64, 32), (96, 48)]


def ensemble(seed=4, members=64):
    """Batched ensemble: k = 2 warm bubbles on uneven grids, 5 SDIRK2 steps each.

    Draw order per member: grid index, amplitude, x centre, z centre."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(members):
        gi = int(rng.integers(3))
        amp = float(rng.uniform(0.1, 1.0))
        xc = float(rng.uniform(300.0, 700.0))
        zc = float(rng.uniform(250.0, 450.0))
        nx, nz = ENSEMBLE_GRIDS[gi]
        d = dict(PHYS)
        d.update(nx=nx, nz=nz, k=2, x0=0.0, x1=1000.0, z0=0.0, z1=1000.0,
                 physics=0, background=0, bc=0, theta0=300.0, N=0.0, u_mean=0.0, mu=0.0,
                 scheme=1, dt=1.0, newton_rtol=1e-8, gmres_m=30, mg_levels=3,
                 mg_key="mg002222V", rk_stages=1, mass_fix=1, fd_eps_mode=1, mg_precision=32,
                 newton_stall=STALL)
        pert = dict(shape=0, amp=amp, xc=xc, zc=zc, xr=250.0, zr=250.0)
        out.append((d, pert, 5))
    return out


SERVE_GRIDS = [(16, 8), (32, 16), (64, 32), (128, 64), (256, 128)]


def serving_requests(seed=5, n_requests=2000, rate=200.0):
    """Poisson arrivals; per request: steps, physics, grid, k, then bubble draws."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += float(rng.exponential(1.0 / rate))
        steps = int(rng.integers(1, 11))
        physics = int(rng.integers(2))
        gi = int(rng.integers(5))
        k = int(rng.integers(1, 4))
        amp = float(rng.uniform(0.1, 1.0))
        xc = float(rng.uniform(300.0, 700.0))
        zc = float(rng.uniform(250.0, 450.0))
        nx, nz = SERVE_GRIDS[gi]
        d = dict(PHYS)
        d.update(nx=nx, nz=nz, k=k, x0=0.0, x1=1000.0, z0=0.0, z1=1000.0,
                 physics=physics, background=0, bc=0, theta0=300.0, N=0.0, u_mean=0.0,
                 mu=75.0 if physics else 0.0, scheme=1, dt=1.0, newton_rtol=1e-8,
                 gmres_m=30, mg_levels=4, mg_key="mg002222V", rk_stages=1, mass_fix=1,
                 fd_eps_mode=1, mg_precision=32, newton_stall=STALL)
        pert = dict(shape=0, amp=amp, xc=xc, zc=zc, xr=250.0, zr=250.0)
        out.append({"id": i, "arrival": t, "cfg": d, "pert": pert, "steps": steps})
    return out


def random_state(ndof, seed, scale):
    """Seeded random perturbation vector; scale is per component (rho, rho u, rho w, rho theta)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(ndof)
    n = ndof // 4
    for c in range(4):
        v[c * n:(c + 1) * n] *= scale[c]
    return v


def small(nx=4, nz=3, k=2, **kw):
    """Tiny problem description for parity tests (several tiles plus ragged tails)."""
    d = dict(PHYS)
    d.update(nx=nx, nz=nz, k=k, x0=0.0, x1=1000.0, z0=0.0, z1=1000.0 * nz / nx,
             physics=0, background=0, bc=0, theta0=300.0, N=0.0, u_mean=0.0, mu=0.0,
             scheme=1, dt=1.0, newton_rtol=1e-8, gmres_m=20, mg_levels=1,
             mg_key="mg002222V", rk_stages=3, mass_fix=1, fd_eps_mode=1, mg_precision=64)
    d.update(kw)
    return d
