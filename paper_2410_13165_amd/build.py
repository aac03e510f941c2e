"""Build the gfx950 shared library liblbm.so in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbm.so")
SOURCES = ["kernels.hip", "walls_d1.hip", "walls_d2.hip", "walls_d3.hip", "walls_d3t.hip",
           "walls_d4.hip", "walls_d4t.hip",
           "adjoint.hip", "stability.hip", "probe.hip", "capi.hip"]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed fp32 instructions stay off: only scalar/float2 code is emitted
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


# The wall kernels of d = 3 and 4 unroll over the populations (19 of D3Q19, 33
# of D4Q33) and index the field table of their by-value parameter block by mode
# at run time. The front end first copies that block (3184 B) to private
# memory, and LLVM's InstCombine turns the copy back into reads of the
# kernel-argument segment only while the copy has at most 300 users (its
# default); past that, every thread copied the block to scratch at launch (4.5
# KB of scratch per lane). The limit is raised for those translation units only.
SOURCE_FLAGS = {
    "walls_d3.hip": ["-mllvm", "-instcombine-max-copied-from-constant-users=4000"],
    "walls_d3t.hip": ["-mllvm", "-instcombine-max-copied-from-constant-users=4000"],
    "walls_d4.hip": ["-mllvm", "-instcombine-max-copied-from-constant-users=4000"],
    "walls_d4t.hip": ["-mllvm", "-instcombine-max-copied-from-constant-users=4000"],
}


def compile_command(src: str, obj: str) -> list[str]:
    return ([hipcc()] + FLAGS + SOURCE_FLAGS.get(src, [])
            + ["-c", "-o", obj, os.path.join(CSRC, src)])


def link_command(objs: list[str], out: str = LIB) -> list[str]:
    return [hipcc(), f"--offload-arch={ARCH}", "-fPIC", "-shared", "-o", out] + objs


def build(verbose: bool = False) -> str:
    """Compile every source to an object in parallel (each translation unit
    carries its own gfx950 code object), then link liblbm.so."""
    tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory(prefix="lbm_build_") as work:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(work, os.path.splitext(src)[0] + ".o")
            cmd = compile_command(src, obj)
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        failed = []
        for src, proc in procs:
            out, _ = proc.communicate()
            if proc.returncode != 0:
                sys.stderr.write(out)
                failed.append(src)
        if failed:
            raise RuntimeError(f"hipcc failed on {', '.join(failed)}")
        cmd = link_command(objs, tmp)
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking liblbm.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
