"""Build step of the HIP library (gfx950) behind include/lb.h.

``python -m paper_2101_03055_amd.build`` compiles ``csrc/*.hip`` with hipcc
into ``liblbcdf.so`` next to this file.  Packed-FP32 instructions are disabled
for all device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBS = {
    "liblbcdf.so": ["lb_kernels.hip", "lb_batch.hip", "lb_cde.hip", "lb_api.hip", "sg_kernels.hip", "lb3.hip"],
}
ARCH = os.environ.get("LBCDF_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


# host-side AddressSanitizer / UndefinedBehaviorSanitizer (device code is never
# instrumented): each flag reaches only the host compilation
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def build(verbose: bool = False, jobs: int = 4, sanitize: bool = False, out_dir: str | None = None) -> list[str]:
    """Compile every library.  sanitize=True builds a host-sanitized copy into
    out_dir (for the CPU-only sanitizer test) and leaves the product build alone."""
    out = []
    for lib, srcs in LIBS.items():
        objs = []
        procs = []
        for src in srcs:
            obj = os.path.join(CSRC, "_build_san" if sanitize else "_build", src.replace(".hip", ".o"))
            os.makedirs(os.path.dirname(obj), exist_ok=True)
            cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++20", "-fPIC", "-c",
                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                   "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
                   f"-I{os.path.join(ROOT, 'include')}", os.path.join(CSRC, src), "-o", obj]
            if sanitize:
                cmd[1:1] = SANITIZE_HOST
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append(subprocess.Popen(cmd))
            objs.append(obj)
        for p in procs:
            if p.wait() != 0:
                raise RuntimeError(f"hipcc failed building {lib}")
        target = os.path.join(out_dir if sanitize else HERE, lib)
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", target + ".tmp"]
        if sanitize:
            cmd[1:1] = SANITIZE_HOST
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(target + ".tmp", target)
        out.append(target)
    return out


if __name__ == "__main__":
    for p in build(verbose="-v" in sys.argv):
        print("built", p)
