"""Builds tests/c_api/halo_world, a C program that uses libhx.so through its
C ABI alone (gcc, the HIP runtime API for device memory)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
EXE = os.path.join(HERE, "halo_world")


def build_c_api() -> str:
    tmp = EXE + ".tmp"
    cmd = ["gcc", "-std=c11", "-O1", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "halo_world.c"),
           "-L", os.path.join(ROOT, "paper_2309_07337_amd"), "-lhx", "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_2309_07337_amd", "-Wl,-rpath,/opt/rocm/lib", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"gcc failed for halo_world.c:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, EXE)
    return EXE


if __name__ == "__main__":
    build_c_api()
