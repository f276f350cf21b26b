"""Builds tests/c_abi/embed_file (a plain C caller of liblne.so) with gcc:
C11, include/lne.h and the HIP runtime API only.  Test infrastructure."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "embed_file.c")
EXE = os.path.join(HERE, "embed_file")
ROCM = "/opt/rocm"


def build() -> str:
    libdir = os.path.join(ROOT, "paper_2302_07084_amd")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           f"-I{ROCM}/include", f"-I{os.path.join(ROOT, 'include')}", SRC, "-o", EXE,
           f"-L{libdir}", "-llne", f"-L{ROCM}/lib", "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_2302_07084_amd", f"-Wl,-rpath,{ROCM}/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"gcc failed for embed_file.c:\n{r.stderr}")
    return EXE


if __name__ == "__main__":
    print(build())
