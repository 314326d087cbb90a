"""Build libsdint.so (HIP for gfx950) in-tree with hipcc.

Every HIP translation unit is compiled to an object in ``_build/`` in parallel,
then linked into ``paper_1511_03614_amd/libsdint.so``.  Always recompiles.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libsdint.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-mcode-object-version=5",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(HERE, "..", "include"), "-Wall", "-Wno-unused-result"]
SOURCES = ["tiles_real_e7.hip", "cubature_real.hip", "cubature_cplx.hip", "suave_real.hip", "suave_cplx.hip", "divonne_real.hip", "divonne_cplx.hip", "tiles_real_dd.hip", "tiles_real_nv16.hip", "tiles_real_nv10.hip", "tiles_real_nv10_s2.hip", "tiles_real_nv10_g.hip", "tiles_real_nv8.hip", "tiles_real_nv6.hip", "tiles_real_nv4.hip",
           "tiles_real_nv16_s2.hip", "tiles_real_nv8_s2.hip", "tiles_real_nv6_s2.hip", "tiles_real_nv4_s2.hip", "tiles_real_nv16_g.hip", "tiles_real_nv8_g.hip", "tiles_real_nv6_g.hip", "tiles_real_nv4_g.hip", "eval_points_real.hip", "tiles_cplx.hip", "tiles_cplx_nv4.hip", "tiles_cplx_nv6.hip", "tiles_cplx_nv8.hip", "tiles_cplx_dd.hip",
           "kernels_misc.hip", "mc_points.hip", "flow.hip", "tiles_expr.hip", "expr_host.cpp", "api.cpp", "driver.cpp", "flow_host.cpp", "deform_host.cpp", "lattice_cbc.cpp", "prefactor.cpp", "cubature.cpp", "feynman_host.cpp", "poles_host.cpp"]


def kernel_hash() -> str:
    """FNV-1a 64 over every source of the library, in name order (keys saved autotuner decisions)."""
    h = 0xCBF29CE484222325
    for name in sorted(os.listdir(CSRC)):
        if not name.endswith((".hip", ".hpp", ".h", ".cpp")):
            continue
        with open(os.path.join(CSRC, name), "rb") as f:
            for b in name.encode() + b"\0" + f.read():
                h = ((h ^ b) * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return f"{h:016x}"


def _compile(src: str) -> tuple:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC] + COMMON + lang + [f'-DSDI_KERNEL_HASH="{_HASH}"', "-c", os.path.join(CSRC, src), "-o", obj]
    t = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    return src, r.returncode, msg, time.time() - t, obj


_HASH = ""


def build(verbose: bool = True, jobs: int = 0) -> str:
    global _HASH
    _HASH = kernel_hash()
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))
    objs = []
    with cf.ThreadPoolExecutor(jobs) as ex:
        for src, rc, msg, dt, obj in ex.map(_compile, SOURCES):
            if verbose:
                print(f"[build] {src}: rc={rc} {dt:.1f}s", flush=True)
            if msg.strip() and (rc != 0 or verbose):
                print(msg, flush=True)
            if rc != 0:
                raise RuntimeError(f"hipcc failed on {src}")
            objs.append(obj)
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        print(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, OUT)
    if verbose:
        print(f"[build] wrote {OUT}", flush=True)
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
