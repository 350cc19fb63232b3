"""Build the hfv shared library for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhfv.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# (source, extra flags, object): hfv_hot.cpp is compiled once per group of
# (dim, order) instantiations and once for its dispatch, in parallel; the
# longest compilations are listed first
SOURCES = [(src, [], src.replace(".cpp", ".o")) for src in ("hfv_char.cpp", "hfv_vjp.cpp")] + \
          [("hfv_hot.cpp", [f"-DHFV_HOT_PART={k}"], f"hfv_hot_p{k}.o") for k in (5, 8, 4, 7, 3, 2, 6, 1, 0)] + \
          [(src, [], src.replace(".cpp", ".o")) for src in ("hfv_visc.cpp", "hfv_setup.cpp", "hfv_api.cpp",
                                                            "hfv_tune.cpp", "hfv_time.cpp")]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-x", "hip",
         # no packed FP32 instructions anywhere in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-Wno-pass-failed"]


def build(verbose: bool = False, jobs: int = 8) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(item):
        src, extra, objname = item
        obj = os.path.join(objdir, objname)
        cmd = [HIPCC] + FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-6000:]}")
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-4000:])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
