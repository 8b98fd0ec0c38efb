"""Compile the plain C-ABI caller (sbr_c_example.cpp) against the built
libsbr.so, in place.  Run after the library build."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_2311_13182_amd")
EXE = os.path.join(HERE, "sbr_c_example")


def build() -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = EXE + ".tmp"
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "-o", tmp, os.path.join(HERE, "sbr_c_example.cpp"),
                           "-I", os.path.join(ROOT, "include"), "-L", PKG, "-lsbr",
                           "-Wl,-rpath," + PKG, "-Wl,-rpath,$ORIGIN/../../paper_2311_13182_amd"])
    os.replace(tmp, EXE)
    return EXE


if __name__ == "__main__":
    print(build())
