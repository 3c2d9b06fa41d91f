"""Builds tests/capi/capi_check: a C program that uses the library only
through include/sgm.h (linked against libsgm.so and the CPU oracle)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
EXE = os.path.join(HERE, "capi_check")


def build() -> str:
    pkg = os.path.join(ROOT, "paper_1610_04121_amd")
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
           "-o", EXE + ".tmp", os.path.join(HERE, "capi_check.c"), os.path.join(ROOT, "oracle", "sgm_oracle.c"),
           "-L", pkg, "-lsgm", "-Wl,-rpath," + pkg, "-Wl,-rpath,$ORIGIN/../../paper_1610_04121_amd",
           "-L", "/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    subprocess.run(cmd, check=True)
    os.replace(EXE + ".tmp", EXE)
    return EXE


if __name__ == "__main__":
    print(build())
