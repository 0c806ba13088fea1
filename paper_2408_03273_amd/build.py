"""Build the HIP library libmpewald.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmpewald.so")
SOURCES = ["kernels.hip", "region.hip", "recip32.hip", "peak.hip", "api.hip", "noalloc.hip"]
ARCH = os.environ.get("MPEWALD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int = 2, out: str = LIB, objdir: str | None = None,
          extra_flags: tuple = ()) -> str:
    """Compile every source to an object, then link the shared library (out).
    extra_flags are added to every compile (e.g. host-pass-only options given
    as "-Xarch_host", option pairs)."""
    objdir = objdir or os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    # MFMA accumulators in ordinary VGPRs (gfx950 allows either file): keeps
    # loop-carried accumulators from being copied between AGPRs and VGPRs
    flags = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-mllvm", "-amdgpu-mfma-vgpr-form=1", "-Wall", "-Wno-unused-function",
             "-Wno-unknown-pragmas", *extra_flags]
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [hipcc(), *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    errs = []
    for src, p in procs:
        log, _ = p.communicate()
        text = log.decode(errors="replace")
        # the host pass does not know the gfx feature flag; that warning is harmless
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            errs.append(f"{src}:\n" + "\n".join(lines))
        elif verbose and lines:
            print("\n".join(lines))
    if errs:
        raise RuntimeError("HIP build failed:\n" + "\n".join(errs))
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
