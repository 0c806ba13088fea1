"""Compile the plain-C consumer of the library (tests/c/abi_roundtrip.c) with
gcc against include/mpewald.h, the in-tree libmpewald.so, the HIP runtime and
the CPU oracle (test infrastructure)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
EXE = os.path.join(HERE, "abi_roundtrip")


def build() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    pkg = os.path.join(ROOT, "paper_2408_03273_amd")
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include",
           os.path.join(HERE, "abi_roundtrip.c"), os.path.join(ROOT, "oracle", "ewald_oracle.c"),
           f"-L{pkg}", "-lmpewald", f"-L{rocm}/lib", "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_2408_03273_amd", f"-Wl,-rpath,{rocm}/lib", "-lm", "-o", EXE + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(EXE + ".tmp", EXE)
    return EXE


if __name__ == "__main__":
    print(build())
