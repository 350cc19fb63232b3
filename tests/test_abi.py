"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2510_25906_amd", "libhfv.so")


def declared():
    src = open(os.path.join(ROOT, "include", "hfv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hfv_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("hfv_create", "hfv_reconstruct", "hfv_residual", "hfv_residual_vjp", "hfv_query",
              "hfv_destroy", "hfv_last_error", "hfv_set_params", "hfv_copy_table", "hfv_set_launch"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_create_rejects_null_arguments_without_touching_the_gpu():
    lib = ctypes.CDLL(LIB)
    lib.hfv_create.restype = ctypes.c_int
    lib.hfv_last_error.restype = ctypes.c_char_p
    out = ctypes.c_void_p()
    rc = lib.hfv_create(None, None, None, None, ctypes.byref(out))
    assert rc == -1
    assert b"NULL" in lib.hfv_last_error(None)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_validation_errors_on_cpu():
    """Invalid parameters and inconsistent stencils fail in host validation."""
    import numpy as np
    from paper_2510_25906_amd import hfv
    from paper_2510_25906_amd.inputs import configs
    w = configs.c1_density_jump(8, 2)
    for bad in (dict(lambda1_prime=0.5), dict(kappa=-1.0), dict(gamma=1.0), dict(alpha_m=-1e-3)):
        with pytest.raises(hfv.HfvError) as ei:
            hfv_ctx_no_gpu(hfv, w.mesh, w.stencils, w.params.with_(**bad))
        assert "HFV_ERR_PARAM" in str(ei.value)
    st = w.stencils
    from dataclasses import replace
    bad_st = replace(st, central=np.where(st.central == 3, 10 ** 6, st.central).astype(np.int32))
    with pytest.raises(hfv.HfvError) as ei:
        hfv_ctx_no_gpu(hfv, w.mesh, bad_st, w.params)
    assert "HFV_ERR_MESH" in str(ei.value)


def hfv_ctx_no_gpu(hfv, mesh, st, params):
    """Drive hfv_create up to validation only: invalid inputs return before any HIP call."""
    lib = hfv.load()
    import ctypes as C
    import numpy as np
    keep = []

    def arr(x, dt):
        a = np.ascontiguousarray(x, dtype=dt)
        keep.append(a)
        return a
    m = hfv.HfvMesh(dim=mesh.dim, n_vertices=mesh.vertices.shape[0], n_cells=mesh.n_cells,
                    n_faces=mesh.n_faces,
                    vertices=hfv._ptr(arr(mesh.vertices, np.float64), C.c_double),
                    cell_type=hfv._ptr(arr(mesh.cell_type, np.int8), C.c_int8),
                    cell_vtx_off=hfv._ptr(arr(mesh.cell_vtx_off, np.int32), C.c_int32),
                    cell_vtx=hfv._ptr(arr(mesh.cell_vtx, np.int32), C.c_int32),
                    face_cells=hfv._ptr(arr(mesh.face_cells, np.int32), C.c_int32),
                    face_vtx_off=hfv._ptr(arr(mesh.face_vtx_off, np.int32), C.c_int32),
                    face_vtx=hfv._ptr(arr(mesh.face_vtx, np.int32), C.c_int32),
                    face_shift=hfv._ptr(arr(mesh.face_shift, np.int8), C.c_int8),
                    period=hfv._ptr(arr(mesh.period, np.float64), C.c_double))
    s = hfv.HfvStencils(M=st.M, nf_max=st.dir.shape[1], Md=st.Md,
                        central=hfv._ptr(arr(st.central, np.int32), C.c_int32),
                        central_shift=hfv._ptr(arr(st.central_shift, np.int8), C.c_int8),
                        dir=hfv._ptr(arr(st.dir, np.int32), C.c_int32),
                        dir_shift=hfv._ptr(arr(st.dir_shift, np.int8), C.c_int8),
                        n_dir=hfv._ptr(arr(st.n_dir, np.int32), C.c_int32),
                        muscl=hfv._ptr(arr(st.muscl, np.int32), C.c_int32),
                        muscl_shift=hfv._ptr(arr(st.muscl_shift, np.int8), C.c_int8),
                        n_muscl=hfv._ptr(arr(st.n_muscl, np.int32), C.c_int32))
    p = hfv.params_struct(params, 64)
    h = C.c_void_p()
    rc = lib.hfv_create(C.byref(m), C.byref(s), C.byref(p), None, C.byref(h))
    if rc != 0:
        raise hfv.HfvError(rc, lib.hfv_last_error(None).decode())
    raise AssertionError("validation unexpectedly passed")


def _shell_context():
    """A Context with the sizes of a small mesh but no device tables: the
    buffer checks run before any library call, so they can be exercised on
    the CPU."""
    import torch
    from paper_2510_25906_amd import hfv
    ctx = hfv.Context.__new__(hfv.Context)
    ctx.h = None
    ctx.lib = None
    ctx.precision, ctx.dtype = 64, torch.float64
    ctx.n_cells, ctx.nvar, ctx.ngp_cell, ctx.n_faces = 10, 4, 6, 15
    return ctx


def test_every_buffer_argument_is_checked_before_the_abi():
    """Wrong dtype, shape, layout or device on any buffer argument raises
    HfvError before its address reaches the library (the calls would
    otherwise hand a CPU pointer or an undersized buffer to the kernels)."""
    import torch
    from paper_2510_25906_amd import hfv
    ctx = _shell_context()
    N, nv, ng = ctx.n_cells, ctx.nvar, ctx.ngp_cell
    f64 = lambda *s: torch.zeros(s, dtype=torch.float64)
    u8 = lambda *s: torch.zeros(s, dtype=torch.uint8)
    good_u, good_cls, good_fs = f64(nv, N), u8(N), f64(ng, nv, N)
    bad = {
        "dtype": (f64(nv, N).float(), u8(N).int(), f64(ng, nv, N).float(), f64(N).float()),
        "shape": (f64(nv, N + 1), u8(N - 1), f64(ng - 1, nv, N), f64(N + 1)),
        "contiguous": (f64(N, nv).t(), u8(2 * N)[::2], f64(ng, N, nv).transpose(1, 2), f64(2 * N)[::2]),
        "CUDA": (good_u, good_cls, good_fs, f64(N)),   # right layout, host memory
    }

    def calls(u, cls, fs, mg):
        """(name, thunk) for each buffer argument of every entry point, the
        buffer under test in that argument and well-formed CPU tensors
        elsewhere (U is checked first, so it is the bad one or good)."""
        yield "U", lambda: ctx.reconstruct(u)
        yield "reconstruct face_states", lambda: ctx.reconstruct(good_u, face_states=fs)
        yield "reconstruct cell_class", lambda: ctx.reconstruct(good_u, cell_class=cls)
        yield "reconstruct near_margin", lambda: ctx.reconstruct(good_u, near_margin=mg)
        yield "residual R", lambda: ctx.residual(good_u, R=u)
        yield "residual face_states", lambda: ctx.residual(good_u, face_states=fs)
        yield "residual cell_class", lambda: ctx.residual(good_u, cell_class=cls)
        yield "frozen cell_class", lambda: ctx.residual_frozen(good_u, cls)
        yield "frozen R", lambda: ctx.residual_frozen(good_u, good_cls, R=u)
        yield "vjp cell_class", lambda: ctx.residual_vjp(good_u, cls, good_u)
        yield "vjp gR", lambda: ctx.residual_vjp(good_u, good_cls, u)
        yield "vjp gU", lambda: ctx.residual_vjp(good_u, good_cls, good_u, gU=u)
        yield "vjp face_states", lambda: ctx.residual_vjp(good_u, good_cls, good_u, face_states=fs)
        yield "rk_stage out", lambda: ctx.rk_stage(u, 1.0, good_u)
        yield "rk_stage U1", lambda: ctx.rk_stage(good_u, 1.0, good_u, 1.0, u)

    for what, (u, cls, fs, mg) in bad.items():
        for name, thunk in calls(u, cls, fs, mg):
            with pytest.raises(hfv.HfvError) as ei:
                thunk()
            msg = str(ei.value)
            # layouts are checked before devices, so the message names the
            # bad buffer's fault, not the host placement of the good ones
            assert what in msg, (what, name, msg)
            if what != "CUDA":
                assert name.split()[-1] in msg, (what, name, msg)
