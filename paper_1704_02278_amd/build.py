"""Build ``libglop.so`` (gfx950) in-tree with hipcc.

    python paper_1704_02278_amd/build.py

(Run it by path: importing the package would load the library being rebuilt.)
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
sys.path.insert(0, str(PKG))
import isa_check  # noqa: E402  (a sibling module; the package itself is not imported)

ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "libglop.so"
SOURCES = ["glop_capi.cpp", "glop_trie.cpp", "glop_serve.cpp", "glop_kernels.hip"] + [
    f"glop_kernels_{tag}.hip" for tag in "abcdef"
]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are kept out of every device build.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", f"-I{ROOT / 'include'}", f"-I{CSRC}"]


def build(verbose: bool = False) -> Path:
    """Compile every source and link the shared library (always rebuilds)."""
    objdir = PKG / "_build"
    objdir.mkdir(exist_ok=True)
    def compile_one(src):
        obj = objdir / (src + ".o")
        device = src.endswith(".hip")
        # Device sources keep their assembly (-save-temps, same compile) so
        # that every kernel can be checked for barriers in divergent loops.
        temps = objdir / (src + ".temps")
        if device:
            shutil.rmtree(temps, ignore_errors=True)
            temps.mkdir()
        lang = ["-x", "hip", "-save-temps"] if device else []
        cmd = [HIPCC, *DEVICE_FLAGS, *COMMON_FLAGS, *lang, "-c", str(CSRC / src), "-o", str(obj)]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True, cwd=str(temps) if device else None)
        errs = "\n".join(l for l in (res.stderr or "").splitlines() if "packed-fp32-ops" not in l)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{errs}")
        if errs.strip() and verbose:
            print(errs, file=sys.stderr)
        if device:
            problems = []
            for asm in sorted(temps.glob("*-hip-amdgcn-amd-amdhsa-gfx950.s")):
                for kernel, probs in isa_check.check_file(asm).items():
                    problems += [f"{src}: {kernel}: {p}" for p in probs]
            if not any(temps.glob("*-hip-amdgcn-amd-amdhsa-gfx950.s")):
                raise RuntimeError(f"no device assembly kept for {src}")
            shutil.rmtree(temps, ignore_errors=True)
            if problems:
                raise RuntimeError("kernel check failed:\n" + "\n".join(problems))
        return str(obj)

    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as pool:
        objs = list(pool.map(compile_one, SOURCES))
    tmp = LIB.with_name(LIB.name + ".tmp")
    cmd = [HIPCC, *DEVICE_FLAGS, "-shared", "-fPIC", *objs, "-o", str(tmp)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
