"""Builds tests/probe/mfma_ceiling (the register-only matrix-core rate probe
that `bench.py --report mfma` runs beside the dense kernels) with hipcc for
gfx950.  Measurement infrastructure."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mfma_ceiling.hip")
EXE = os.path.join(HERE, "mfma_ceiling")


def build() -> str:
    arch = os.environ.get("LNE_OFFLOAD_ARCH", "gfx950")
    cmd = ["hipcc", "-O3", "-std=c++17", f"--offload-arch={arch}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", SRC, "-o", EXE]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for mfma_ceiling.hip:\n{r.stderr}")
    return EXE


if __name__ == "__main__":
    print(build())
