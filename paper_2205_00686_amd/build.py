"""Compile the HIP library liblbm.so for gfx950 (in-tree, next to this file)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", n) for n in ("lbm.hip", "lbm3d.hip", "hbm_copy.hip")]
HEADERS = [os.path.join(HERE, "csrc", n) for n in ("lbm_device.hpp", "lbm_step.hpp", "lbm_persist.hpp", "lbm_aux.hpp", "host_range.hpp")] + \
          [os.path.join(ROOT, "include", n) for n in ("lbm.h", "lbm3d.h")]
OUT = os.path.join(HERE, "liblbm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
         # fuse a multiply and an add only inside one expression: the arithmetic of a node is then
         # fixed by the source, whatever the tile shape or code layout of the kernel instance
         "-ffp-contract=on",
         # no packed FP32 instructions (v_pk_*_f32) anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"),
         # host ranges in the profiler's marker trace (csrc/host_range.hpp)
         "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def build(verbose: bool = False) -> str:
    tmp = OUT + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for liblbm.so")
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
