"""Build the plain C client of libspx (spx_client.c) with gcc, next to its
source.  It links the in-tree libspx.so and the HIP runtime by rpath."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "spx_client.c")
BIN = os.path.join(HERE, "spx_client")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(force: bool = False) -> str:
    if not force and os.path.exists(BIN) and os.path.getmtime(BIN) >= os.path.getmtime(SRC):
        return BIN
    pkg = os.path.join(ROOT, "paper_1302_1078_amd")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), SRC, "-o", BIN,
           "-L", pkg, "-lspx", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_1302_1078_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    subprocess.run(cmd, check=True)
    return BIN


if __name__ == "__main__":
    print(build(force=True))
