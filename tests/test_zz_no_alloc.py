"""The allocation-free stage residual (jfmg_stage_residual_noalloc) against the
problem entry point jfmg_stage_residual on the same inputs: two calls in a row
through the static scratch, the second on a smaller problem, and the rest state.

Tolerance: the allocation-free call evaluates the background tables on the
device, the problem on the host, so the two differ by the rounding of L_h (the
rounding scale of the residual, the sums of absolute values of the unsubtracted
terms, times alpha dt / m per node: measured 0.22 eps of that scale, bound 2 eps)."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2505_24504_amd import jfmg, workloads as W  # noqa: E402

from gpu_common import DEV, EPS, dg_mass, pair, rand_state, to_dev, to_np  # noqa: E402


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    jfmg.load_library()


def _case(k, nx, nz, physics):
    return W.small(nx=nx, nz=nz, k=k, physics=physics, mu=75.0 if physics else 0.0, x1=11000.0, z1=5000.0,
                   mg_levels=1)


def _check(d, seed, adt):
    p, o = pair(d)
    U = rand_state(o, seed)
    Ub = rand_state(o, seed + 1)
    Gp, np_ = p.stage_residual(to_dev(U), to_dev(Ub), adt)
    Gs, n2 = jfmg.stage_residual_noalloc(d, to_dev(U), to_dev(Ub), adt)
    gp, gs = to_np(Gp), to_np(Gs)
    sig = adt * o.residual(U, 3) / np.tile(dg_mass(d), 4)
    tol = 2 * EPS * np.linalg.norm(sig)
    err = np.linalg.norm(gs - gp)
    nrm = float(np.sqrt(to_np(n2)[0]))
    print(f"noalloc k={d['k']} {d['nx']}x{d['nz']} physics={d['physics']}: err {err:.3e} tol {tol:.3e} "
          f"bitwise {np.array_equal(gs, gp)} norm {nrm:.15e} vs {np_:.15e}", flush=True)
    assert err <= tol
    assert abs(nrm - np_) <= 1e-13 * np_ + tol


def test_noalloc_two_calls_second_smaller():
    _check(_case(3, 40, 12, 1), 201, 0.7)
    _check(_case(2, 11, 5, 0), 203, 1.3)


def test_noalloc_rest_state_and_norm_pointer():
    """The rest state of the Euler system is well balanced through the device-built
    tables (G = 0 bitwise); without a norm pointer only G is written."""
    d = _case(1, 16, 8, 0)
    n = jfmg.num_dofs(d)
    z = torch.zeros(n, dtype=torch.float64, device=DEV)
    G = torch.full((n,), 7.0, dtype=torch.float64, device=DEV)
    nrm = torch.full((1,), 7.0, dtype=torch.float64, device=DEV)
    jfmg.stage_residual_noalloc(d, z, z, 0.5, G=G, norm2=nrm)
    torch.cuda.synchronize()
    assert torch.count_nonzero(G).item() == 0 and nrm.item() == 0.0
    L = jfmg.load_library()
    cfg = jfmg.make_config(d)
    G.fill_(7.0)
    rc = L.jfmg_stage_residual_noalloc(ctypes.byref(cfg), jfmg._ptr(z), jfmg._ptr(z), 0.5, jfmg._ptr(G), None,
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert rc == 0 and torch.count_nonzero(G).item() == 0
