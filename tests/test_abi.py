"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/jfmg.h declares, its struct layouts match the binding, and it rejects
bad configurations (no GPU call is made)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2505_24504_amd import jfmg, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jfmg.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(jfmg.LIB_PATH):
        from paper_2505_24504_amd import build
        build.build()
    return jfmg.load_library()


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(jfmg_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert len(syms) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", jfmg.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (jfmg_\w+)", out))
    missing = [s for s in syms if s not in exported]
    assert not missing, missing
    for s in syms:
        getattr(lib, s)
    assert set(jfmg.EXPORTS) == set(syms)


def test_tile_enum_matches_binding():
    text = open(HEADER).read()
    vals = dict((n, int(v)) for n, v in re.findall(r"JFMG_TILE_(\w+)\s*=\s*(\d+)", text))
    assert vals.pop("NSHAPE") == len(jfmg.TILES)
    assert sorted(vals, key=vals.get) == jfmg.TILES


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "lay.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "jfmg.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(jfmg_config), offsetof(jfmg_config, mg_key),
         offsetof(jfmg_config, x0), offsetof(jfmg_config, rk_alpha), offsetof(jfmg_config, newton_stall),
         offsetof(jfmg_config, pseudo_cfl_dg), sizeof(jfmg_perturbation), sizeof(jfmg_stats),
         offsetof(jfmg_stats, g0_norm), offsetof(jfmg_stats, reached_rtol));
  printf("%zu %zu\n", offsetof(jfmg_stats, stall_stops), offsetof(jfmg_stats, reorth_its));
  return 0; }
''')
    exe = tmp_path / "lay"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    vals = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert vals == [C.sizeof(jfmg.Config), jfmg.Config.mg_key.offset, jfmg.Config.x0.offset,
                    jfmg.Config.rk_alpha.offset, jfmg.Config.newton_stall.offset, jfmg.Config.pseudo_cfl_dg.offset,
                    C.sizeof(jfmg.Perturbation),
                    C.sizeof(jfmg.Stats), jfmg.Stats.g0_norm.offset, jfmg.Stats.reached_rtol.offset,
                    jfmg.Stats.stall_stops.offset, jfmg.Stats.reorth_its.offset]


def test_workspace_sizes(lib):
    for d, _, _ in (W.bubble_small(), W.density_current(), W.inertia_gravity()):
        n = jfmg.workspace_bytes(d)
        N = 4 * d["nx"] * d["nz"] * (d["k"] + 1) ** 2
        assert n > 8 * N * (2 * d["gmres_m"] + 1)


@pytest.mark.parametrize("bad,what", [
    ({"k": 0}, "k must"), ({"k": 4}, "k must"), ({"gmres_m": 65}, "gmres_m"),
    ({"mg_levels": 9}, "mg_levels"), ({"mg_key": "mg102222V", "pseudo_cfl_dg": 0.0}, "pseudo_cfl_dg"), ({"mg_key": "mgxx"}, "key"),
    ({"nx": 3, "mg_levels": 3}, "odd"), ({"mg_precision": 16}, "precision"), ({"rk_stages": 5}, "rk_stages"),
    ({"background": 1, "N": 0.0}, "N > 0"), ({"dt": 0.0}, "constants"), ({"transfer": 2}, "transfer"),
])
def test_invalid_configs_rejected(lib, bad, what):
    d, _, _ = W.bubble_small()
    d = dict(d, **bad)
    with pytest.raises(jfmg.JfmgError) as ei:
        jfmg.workspace_bytes(d)
    assert ei.value.status == jfmg.EINVAL
    assert what in str(ei.value)


def test_ensemble_workspace_and_member_checks(lib):
    """A ragged batch is laid out for the envelope grid (each member a region of the
    largest nx and nz, plus the member table); members that differ in anything but
    the grid and the domain, or a key with DG-level smoothing, are EINVAL."""
    ens = W.ensemble(seed=4, members=64)
    ds = [ens[0][0], dict(ens[0][0], nx=96, nz=16), dict(ens[0][0], nx=32, nz=48, x1=800.0)]
    b = jfmg.ensemble_workspace_bytes(ds)
    env = jfmg.workspace_bytes(dict(ds[0], nx=96, nz=48))
    assert 3 * env < b <= 3 * env + 3 * 8192 + 256
    assert jfmg.ensemble_workspace_bytes(ds[:1]) > jfmg.workspace_bytes(ds[0])
    for bad, what in [({"k": 3}, "differ only"), ({"dt": 2.0}, "differ only"), ({"batch": 2}, "single problems"),
                      ({"nx": 3}, "member 1")]:
        with pytest.raises(jfmg.JfmgError) as ei:
            jfmg.ensemble_workspace_bytes([ds[0], dict(ds[1], **bad)])
        assert ei.value.status == jfmg.EINVAL and what in str(ei.value), (bad, str(ei.value))
    with pytest.raises(jfmg.JfmgError) as ei:
        jfmg.ensemble_workspace_bytes([dict(d, mg_key="mg102222V", pseudo_cfl_dg=0.3) for d in ds])
    assert "DG-level smoothing" in str(ei.value)
    with pytest.raises(jfmg.JfmgError):
        jfmg.ensemble_workspace_bytes([])
    cfgs = (jfmg.Config * 2)(jfmg.make_config(ds[0]), jfmg.make_config(ds[1]))
    h = C.c_void_p()
    assert lib.jfmg_create_ensemble(cfgs, 2, C.c_void_p(256), 16, None, C.byref(h)) == jfmg.ENOMEM


def test_create_rejects_small_workspace(lib):
    d, _, _ = W.bubble_small()
    cfg = jfmg.make_config(d)
    h = C.c_void_p()
    rc = lib.jfmg_create_problem(C.byref(cfg), C.c_void_p(256), 16, None, C.byref(h))
    assert rc == jfmg.ENOMEM
    assert b"workspace" in lib.jfmg_last_error(None)


def test_noalloc_residual_rejects_bad_arguments_before_device_work(lib):
    """The allocation-free residual checks its arguments and the size of the static
    scratch before it touches the device: null vectors and invalid configurations are
    EINVAL, a problem whose tables and partials exceed the array is ENOMEM."""
    d, _, _ = W.bubble_small()
    fake = C.c_void_p(256)   # never dereferenced: every case fails its host checks first
    cfg = jfmg.make_config(d)
    assert lib.jfmg_stage_residual_noalloc(C.byref(cfg), None, fake, 1.0, fake, None, None) == jfmg.EINVAL
    bad = jfmg.make_config(dict(d, k=5))
    assert lib.jfmg_stage_residual_noalloc(C.byref(bad), fake, fake, 1.0, fake, None, None) == jfmg.EINVAL
    assert b"k must" in lib.jfmg_last_error(None)
    batched = jfmg.make_config(dict(d, batch=2))
    assert lib.jfmg_stage_residual_noalloc(C.byref(batched), fake, fake, 1.0, fake, None, None) == jfmg.EINVAL
    assert lib.jfmg_stage_residual_noalloc(C.byref(cfg), fake, fake, float("nan"), fake, None, None) == jfmg.EINVAL
    big = jfmg.make_config(dict(d, nx=1024, nz=1024, k=3, mg_levels=1))   # 131072 partials: 1 MiB alone
    assert lib.jfmg_stage_residual_noalloc(C.byref(big), fake, fake, 1.0, fake, None, None) == jfmg.ENOMEM
    assert b"static scratch" in lib.jfmg_last_error(None)
