"""Builds the plain C client of the C ABI (eigupd_client.c) with gcc, next to
this file, linked against the HIP runtime and ../../paper_1706_00773_amd/libeigupd.so
(found at run time through an $ORIGIN-relative rpath)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(out: str | None = None) -> str:
    out = out or os.path.join(HERE, "eigupd_client")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROCM, "include"), "-I" + os.path.join(ROOT, "include"),
           os.path.join(HERE, "eigupd_client.c"), "-o", out,
           "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
           "-L" + os.path.join(ROOT, "paper_1706_00773_amd"), "-l:libeigupd.so",
           "-Wl,-rpath," + os.path.join(ROCM, "lib"),
           "-Wl,-rpath,$ORIGIN/../../paper_1706_00773_amd", "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("C client build failed:\n" + r.stderr)
    return out


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else None))
