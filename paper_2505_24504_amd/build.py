"""Build the gfx950 HIP library libjfmg.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libjfmg.so")
SOURCES = ["dg.hip", "transfer.hip", "fv.hip", "la.hip", "driver.hip", "batch.hip", "noalloc.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=on",                        # contract a*b+c only inside one expression
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose: bool = False, jobs: int = 5, out: str = LIB, defines: tuple = ()) -> str:
    """Compile every HIP source to an object, then link the shared library.

    `defines` (e.g. ("FV_COARSE_NTH=192",)) override the tile constants of the
    kernels; `out` names the library file (objects go to a folder beside it)."""
    objdir = os.path.join(HERE, "_build") if out == LIB else out + ".objs"
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [hipcc(), "-c", "-x", "hip", os.path.join(CSRC, src), "-o", obj] + FLAGS + ["-D" + d for d in defines]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    while procs:
        _wait(procs.pop(0))
    tmp = out + ".tmp"
    cmd = [hipcc(), "-shared", "--offload-arch=gfx950", "-fPIC", "-o", tmp] + objs
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if res.returncode:
        raise RuntimeError("link failed:\n" + res.stdout.decode())
    os.replace(tmp, out)
    return out


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    if p.returncode:
        raise RuntimeError(f"hipcc failed on {src}:\n{out.decode()}")
    text = out.decode()
    if "warning" in text and "packed-fp32-ops" not in text:
        sys.stderr.write(text)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
