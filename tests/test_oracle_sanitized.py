"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host code,
gcc) runs its residual, transfer, linearization, FV and FD products, multigrid
cycle and an implicit step on small viscous and Euler problems of every degree
without a report (any report aborts the child process)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import numpy as np
import oracle
from paper_2505_24504_amd import workloads as W
d0, pert, _ = W.bubble_small()
cases = [dict(d0, nx=8, nz=8, k=1), dict(d0, nx=6, nz=4, k=2, physics=1, mu=75.0, mg_levels=2),
         dict(d0, nx=4, nz=4, k=3, bc=1, scheme=1, mg_key="mg002222W", mg_levels=3)]
for d in cases:
    o = oracle.Oracle(d)
    U = o.initial_state(pert)
    rng = np.random.default_rng(1)
    y = rng.standard_normal(U.size)
    o.residual(U, 1)
    o.stage_residual(U, U, d["dt"])
    u = o.transfer_T(U)
    o.transfer_Tinv(u)
    o.linearize(U, d["dt"])
    o.fv_matvec(0, rng.standard_normal(u.size))
    o.jvp(y)
    o.mg_apply(y)
    rc, U1, st = o.implicit_step(U)
    assert rc == 0, rc
print("sanitized oracle ok")
"""


def _asan_runtime():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True, check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    asan = _asan_runtime()
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    lib = str(tmp_path / "liborc_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           "-ffp-contract=off", "-o", lib, os.path.join(ROOT, "oracle", "orc.c"), "-lm"])
    env = dict(os.environ, ORC_LIB=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "sanitized oracle ok" in r.stdout, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
