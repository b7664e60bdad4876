"""Build libcutamp.so (the C ABI of include/cutamp.h) for gfx950 with hipcc.

The fused particle kernels are instantiated per lane split, plain and
extended (self-collision pass and per-particle term weights), each in its own
object (pk_instances.hip with -DCT_SPLIT=s -DCT_EXT=0|1) so the objects
compile in parallel;
the host side (cutamp.hip) holds the C ABI and the small elementwise kernels,
mlp.hip the seed proposer's matrix-core kernels and their C ABI.

Usage: python -m paper_2411_11833_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libcutamp.so")
SPLITS = (1, 2, 4)

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay disabled: hipcc must not emit v_pk_* f32 ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-Wno-unused-result", "-Wno-unused-value",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}): {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return res


def build(verbose: bool = False, extra: list[str] | None = None, jobs: int | None = None,
          out: str | None = None, objdir: str | None = None) -> str:
    """Compile every HIP source and link the in-tree shared library (always
    recompiles).  `extra` adds hipcc flags; `out` / `objdir`
    redirect the library and objects.  Returns the library path."""
    lib = out or LIB
    obj_dir = objdir or OBJ
    os.makedirs(obj_dir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    units = [(os.path.join(CSRC, "cutamp.hip"), os.path.join(obj_dir, "cutamp.o"), []),
             (os.path.join(CSRC, "mlp.hip"), os.path.join(obj_dir, "mlp.o"), [])]
    for split in SPLITS:
        for ext in (0, 1):
            units.append((os.path.join(CSRC, "pk_instances.hip"),
                          os.path.join(obj_dir, f"pk_s{split}{'_ext' if ext else ''}.o"),
                          [f"-DCT_SPLIT={split}", f"-DCT_EXT={ext}"]))
    cmds = [[hipcc(), *HIPCC_FLAGS, *(extra or []), *inc, *defs, "-c", src, "-o", obj]
            for src, obj, defs in units]
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = lib + ".tmp"
    _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *[u[1] for u in units]], verbose)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
