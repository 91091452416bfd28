"""Builds the plain-C ABI smoke program (pcg_c_smoke.c) against the built
libpcg.so: gcc, C99, the HIP runtime API only (no device code).  The
binary finds libpcg.so next to the package through an $ORIGIN-relative
rpath, so it runs from any copy of the repository."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "pcg_c_smoke.c")
BIN = os.path.join(HERE, "pcg_c_smoke")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(force: bool = False, verbose: bool = False) -> str:
    if not force and os.path.exists(BIN) and os.path.getmtime(BIN) >= os.path.getmtime(SRC):
        return BIN
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           SRC, "-o", BIN + ".tmp",
           "-L", os.path.join(ROOT, "paper_1706_05988_amd"), "-lpcg",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN/../../paper_1706_05988_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(BIN + ".tmp", BIN)
    return BIN


if __name__ == "__main__":
    print(build(force=True, verbose="-v" in sys.argv))
