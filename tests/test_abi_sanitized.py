"""The C ABI's host-side argument validation under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; no GPU): hfv_api.cpp is rebuilt
with the sanitizers on its host pass, linked with the library's other objects,
and every rejection path below runs in a child Python with the ASan runtime
preloaded.  Any out-of-bounds read, use-after-free or undefined operation in
the validation aborts the child, which fails the test."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2510_25906_amd")
ASAN_RT = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
HIPCC = "/opt/rocm/bin/hipcc"

CHILD = r'''
import sys
sys.path.insert(0, ROOT); sys.path.insert(0, ROOT + "/tests")
from dataclasses import replace
import numpy as np
from paper_2510_25906_amd import hfv
hfv.LIB_PATH = LIB
from paper_2510_25906_amd.inputs import configs
import test_abi

lib = hfv.load()
import ctypes as C
out = C.c_void_p()
assert lib.hfv_create(None, None, None, None, C.byref(out)) == -1

def rejects(mesh, st, params, code):
    try:
        test_abi.hfv_ctx_no_gpu(hfv, mesh, st, params)
    except hfv.HfvError as e:
        assert code in str(e), (code, str(e))
        return
    raise AssertionError("accepted")

for w in (configs.c1_density_jump(8, 2), configs.c4_mixed("small")):
    m, st, p = w.mesh, w.stencils, w.params
    for bad in (dict(lambda1_prime=0.5), dict(kappa=-1.0), dict(gamma=1.0), dict(alpha_m=-1e-3),
                dict(order_r=9), dict(b_w=-1.0), dict(eps_w=0.0)):
        rejects(m, st, p.with_(**bad), "HFV_ERR_PARAM")
    N = m.n_cells
    ct = m.cell_type.copy(); ct[N // 2] = 7
    rejects(replace(m, cell_type=ct), st, p, "HFV_ERR_MESH")
    cv = m.cell_vtx.copy(); cv[-1] = m.vertices.shape[0]
    rejects(replace(m, cell_vtx=cv), st, p, "HFV_ERR_MESH")
    fc = m.face_cells.copy(); fc[3, 0] = N
    rejects(replace(m, face_cells=fc), st, p, "HFV_ERR_MESH")
    fc = m.face_cells.copy(); fc[3, 1] = fc[3, 0]
    rejects(replace(m, face_cells=fc), st, p, "HFV_ERR_MESH")
    fv = m.face_vtx.copy(); fv[0] = -2
    rejects(replace(m, face_vtx=fv), st, p, "HFV_ERR_MESH")
    cs = st.central.copy(); cs.flat[-1] = N
    rejects(m, replace(st, central=cs), p, "HFV_ERR_MESH")
    nd = st.n_dir.copy(); nd[0] = st.dir.shape[1] + 1
    rejects(m, replace(st, n_dir=nd), p, "HFV_ERR_MESH")
    dr = st.dir.copy(); dr[N - 1, 0, 0] = -1
    rejects(m, replace(st, dir=dr), p, "HFV_ERR_MESH")
    nm = st.n_muscl.copy(); nm[1] = 0
    rejects(m, replace(st, n_muscl=nm), p, "HFV_ERR_MESH")
    ms = st.muscl.copy(); ms[N - 1, 0] = N + 5
    rejects(m, replace(st, muscl=ms), p, "HFV_ERR_MESH")
print("sanitized validation ok", flush=True)
'''


def _objects():
    return [o for o in glob.glob(os.path.join(PKG, "_build", "*.o")) if not o.endswith("hfv_api.o")]


@pytest.mark.skipif(not ASAN_RT or not os.path.exists(HIPCC), reason="no ASan runtime or hipcc")
@pytest.mark.skipif(not os.path.exists(os.path.join(PKG, "_build", "hfv_api.o")), reason="library not built")
def test_host_validation_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, PKG)
    import build as B
    obj = str(tmp_path / "hfv_api_asan.o")
    lib = str(tmp_path / "libhfv_asan.so")
    flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1"]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    r = subprocess.run([HIPCC] + flags + san + ["-c", os.path.join(PKG, "csrc", "hfv_api.cpp"), "-o", obj],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib, obj] + _objects(),
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, LD_PRELOAD=ASAN_RT[-1], ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    code = f"ROOT = {ROOT!r}\nLIB = {lib!r}\n" + CHILD
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "sanitized validation ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
