"""Python binding of the hfv C ABI (argument marshalling only).

Every step of the reconstruction runs in the HIP library ``libhfv.so``; this
module converts meshes, stencils and parameters to the ABI structs and hands
torch device tensors to it.  There is no fallback: a missing or unloadable
library raises at import of ``load()``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .inputs.params import Params

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhfv.so")
_lib = None

HFV_OK = 0
HFV_ERR_STATE = -7
ERRORS = {-1: "HFV_ERR_PARAM", -2: "HFV_ERR_MESH", -3: "HFV_ERR_RANK", -4: "HFV_ERR_DTYPE",
          -5: "HFV_ERR_HIP", -6: "HFV_ERR_OOM", -7: "HFV_ERR_STATE"}
Q = dict(N_CELLS=0, N_FACES=1, N_GP=2, NVAR=3, K=4, M=5, PRECISION=6, DIM=7, TABLE_BYTES=8,
         COUNT_CWENOZ=9, COUNT_MUSCL=10, COUNT_FIRST=11, NGP_CELL_MAX=12, NOALLOC_BYTES=13)
NOALLOC_SCRATCH_BYTES = 64 << 20   # HFV_NOALLOC_SCRATCH_BYTES
SLOTS = dict(linear=0, classify=1, cwenoz=2, muscl=3, flux=5, gather=6, vjp=7)
TABLES = dict(PINV=0, OI=1, PSIBAR=2, GEOM=3, PDIR=4, PMUS=5, FACE_SLOTS=6, GP_XI=7)

_p = C.c_void_p
_i32p = C.POINTER(C.c_int32)
_i8p = C.POINTER(C.c_int8)
_f64p = C.POINTER(C.c_double)


class HfvMesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_vertices", C.c_int32), ("n_cells", C.c_int32), ("n_faces", C.c_int32),
                ("vertices", _f64p), ("cell_type", _i8p), ("cell_vtx_off", _i32p), ("cell_vtx", _i32p),
                ("face_cells", _i32p), ("face_vtx_off", _i32p), ("face_vtx", _i32p), ("face_shift", _i8p),
                ("period", _f64p)]


class HfvStencils(C.Structure):
    _fields_ = [("M", C.c_int32), ("nf_max", C.c_int32), ("Md", C.c_int32), ("central", _i32p),
                ("central_shift", _i8p), ("dir", _i32p), ("dir_shift", _i8p), ("n_dir", _i32p),
                ("muscl", _i32p), ("muscl_shift", _i8p), ("n_muscl", _i32p)]


class HfvParams(C.Structure):
    _fields_ = [("order_r", C.c_int32), ("scheme_mode", C.c_int32), ("precision", C.c_int32),
                ("riemann", C.c_int32), ("cweno_form", C.c_int32), ("limiter", C.c_int32),
                ("cweno_vars", C.c_int32), ("viscous", C.c_int32),
                ("gamma", C.c_double), ("alpha_m", C.c_double), ("beta_m", C.c_double), ("alpha_w", C.c_double),
                ("beta_w", C.c_double), ("kappa", C.c_double), ("n_exp", C.c_double),
                ("lambda1_prime", C.c_double), ("eps_w", C.c_double), ("b_w", C.c_double),
                ("tvd_theta", C.c_double), ("tvd_eps", C.c_double),
                ("mu0", C.c_double), ("T0", C.c_double), ("sutherland_S", C.c_double), ("prandtl", C.c_double),
                ("visc_alpha", C.c_double)]


def load():
    """Load libhfv.so and declare the ABI; raises if the library is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"hfv HIP library not built: {LIB_PATH} missing (run __graft_entry__.build())")
    # torch first: the library then binds to the HIP runtime torch has loaded,
    # so that device memory and streams from torch are valid in its calls
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    lib.hfv_create.argtypes = [C.POINTER(HfvMesh), C.POINTER(HfvStencils), C.POINTER(HfvParams), _p,
                               C.POINTER(_p)]
    lib.hfv_set_params.argtypes = [_p, C.POINTER(HfvParams)]
    lib.hfv_reconstruct.argtypes = [_p, _p, _p, _p, _p, _p]
    lib.hfv_residual.argtypes = [_p, _p, _p, _p, _p, _p]
    lib.hfv_residual_noalloc.argtypes = [_p, _p, _p, _p, _p, _p]
    lib.hfv_residual_vjp.argtypes = [_p, _p, _p, _p, _p, _p]
    lib.hfv_residual_vjp_states.argtypes = [_p, _p, _p, _p, _p, _p, _p]
    lib.hfv_residual_frozen.argtypes = [_p, _p, _p, _p, _p]
    lib.hfv_rk_stage.argtypes = [_p, C.c_double, _p, C.c_double, _p, C.c_double, _p, _p, _p]
    lib.hfv_cfl_rate.argtypes = [_p, _p, _p, _p]
    lib.hfv_query.argtypes = [_p, C.c_int32, C.POINTER(C.c_int64)]
    lib.hfv_copy_table.argtypes = [_p, C.c_int32, _p, C.c_int64]
    lib.hfv_set_launch.argtypes = [_p, C.POINTER(HfvLaunch)]
    lib.hfv_get_launch.argtypes = [_p, C.POINTER(HfvLaunch)]
    lib.hfv_autotune.argtypes = [_p, _p, C.c_int32, C.POINTER(HfvLaunch), C.POINTER(HfvTuneRecord), C.c_int32,
                                 C.POINTER(C.c_int32), _p]
    lib.hfv_profile_enable.argtypes = [_p, C.c_int32, C.c_int32]
    lib.hfv_profile_read.argtypes = [_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.hfv_last_error.argtypes = [_p]
    lib.hfv_last_error.restype = C.c_char_p
    lib.hfv_destroy.argtypes = [_p]
    lib.hfv_destroy.restype = None
    for name in ("hfv_create", "hfv_set_params", "hfv_reconstruct", "hfv_residual", "hfv_residual_noalloc",
                 "hfv_residual_vjp",
                 "hfv_residual_vjp_states",
                 "hfv_residual_frozen", "hfv_rk_stage", "hfv_cfl_rate",
                 "hfv_query", "hfv_copy_table", "hfv_set_launch", "hfv_get_launch", "hfv_autotune",
                 "hfv_profile_enable",
                 "hfv_profile_read"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


class HfvLaunch(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("lanes_per_cell", "block", "list_blocks", "linear_split",
                                         "linear_lanes", "cwenoz_reuse", "fused_residual", "xcd_remap",
                                         "muscl_lanes", "merged_lists", "lists_cell_major")]


class HfvTuneRecord(C.Structure):
    _fields_ = [("cfg", HfvLaunch), ("ms", C.c_double)]


class HfvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def params_struct(p: Params, precision: int) -> HfvParams:
    return HfvParams(order_r=p.order_r, scheme_mode=p.scheme_mode, precision=precision, riemann=p.riemann,
                     cweno_form=p.cweno_form, limiter=p.limiter, cweno_vars=p.cweno_vars, gamma=p.gamma, alpha_m=p.alpha_m, beta_m=p.beta_m,
                     alpha_w=p.alpha_w, beta_w=p.beta_w, kappa=p.kappa, n_exp=p.n_exp,
                     lambda1_prime=p.lambda1_prime, eps_w=p.eps_w, b_w=p.b_w, tvd_theta=p.tvd_theta,
                     tvd_eps=p.tvd_eps, viscous=p.viscous, mu0=p.mu0, T0=p.T0, sutherland_S=p.sutherland_S,
                     prandtl=p.prandtl, visc_alpha=p.visc_alpha)


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Context:
    """A reconstruction context: device tables for one mesh, stencil set, order and precision."""

    def __init__(self, mesh, stencils, params: Params, precision: int = 64, stream=None):
        import torch
        self.lib = load()
        self.precision = precision
        self.dtype = torch.float64 if precision == 64 else torch.float32
        self.params = params
        d = mesh.dim
        keep = []

        def arr(x, dt):
            a = np.ascontiguousarray(x, dtype=dt)
            keep.append(a)
            return a

        per = arr(mesh.period, np.float64) if mesh.period is not None else None
        self._mesh = HfvMesh(
            dim=d, n_vertices=mesh.vertices.shape[0], n_cells=mesh.n_cells, n_faces=mesh.n_faces,
            vertices=_ptr(arr(mesh.vertices, np.float64), C.c_double),
            cell_type=_ptr(arr(mesh.cell_type, np.int8), C.c_int8),
            cell_vtx_off=_ptr(arr(mesh.cell_vtx_off, np.int32), C.c_int32),
            cell_vtx=_ptr(arr(mesh.cell_vtx, np.int32), C.c_int32),
            face_cells=_ptr(arr(mesh.face_cells, np.int32), C.c_int32),
            face_vtx_off=_ptr(arr(mesh.face_vtx_off, np.int32), C.c_int32),
            face_vtx=_ptr(arr(mesh.face_vtx, np.int32), C.c_int32),
            face_shift=_ptr(arr(mesh.face_shift, np.int8), C.c_int8) if per is not None else None,
            period=_ptr(per, C.c_double) if per is not None else None)
        st = stencils
        self._st = HfvStencils(
            M=st.M, nf_max=st.dir.shape[1], Md=st.Md,
            central=_ptr(arr(st.central, np.int32), C.c_int32),
            central_shift=_ptr(arr(st.central_shift, np.int8), C.c_int8) if per is not None else None,
            dir=_ptr(arr(st.dir, np.int32), C.c_int32),
            dir_shift=_ptr(arr(st.dir_shift, np.int8), C.c_int8) if per is not None else None,
            n_dir=_ptr(arr(st.n_dir, np.int32), C.c_int32),
            muscl=_ptr(arr(st.muscl, np.int32), C.c_int32),
            muscl_shift=_ptr(arr(st.muscl_shift, np.int8), C.c_int8) if per is not None else None,
            n_muscl=_ptr(arr(st.n_muscl, np.int32), C.c_int32))
        self._p = params_struct(params, precision)
        h = C.c_void_p()
        torch.cuda.init()
        rc = self.lib.hfv_create(C.byref(self._mesh), C.byref(self._st), C.byref(self._p),
                                 _stream_handle(stream), C.byref(h))
        if rc != HFV_OK:
            raise HfvError(rc, self.lib.hfv_last_error(None).decode())
        self.h = h
        self.n_cells = self.query("N_CELLS")
        self.n_faces = self.query("N_FACES")
        self.n_gp = self.query("N_GP")
        self.ngp_cell = self.query("NGP_CELL_MAX")
        self.nvar = self.query("NVAR")
        self.K = self.query("K")
        self.M = self.query("M")
        self.dim = d

    def _check(self, rc):
        if rc != HFV_OK:
            raise HfvError(rc, self.lib.hfv_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.hfv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self, what: str) -> int:
        out = C.c_int64()
        self._check(self.lib.hfv_query(self.h, Q[what], C.byref(out)))
        return out.value

    def set_params(self, params: Params):
        self.params = params
        self._p = params_struct(params, self.precision)
        self._check(self.lib.hfv_set_params(self.h, C.byref(self._p)))

    def get_launch(self) -> dict:
        cfg = HfvLaunch()
        self._check(self.lib.hfv_get_launch(self.h, C.byref(cfg)))
        return {n: getattr(cfg, n) for n, _ in HfvLaunch._fields_}

    def set_launch(self, lanes=None, block=None, list_blocks=None, linear_split=None, linear_lanes=None,
                   cwenoz_reuse=None, fused_residual=None, xcd_remap=None, muscl_lanes=None,
                   merged_lists=None, lists_cell_major=None):
        """Change the launch configuration; fields left None keep their current value."""
        cur = self.get_launch()
        new = dict(lanes_per_cell=lanes, block=block, list_blocks=list_blocks, linear_split=linear_split,
                   linear_lanes=linear_lanes, cwenoz_reuse=cwenoz_reuse, fused_residual=fused_residual,
                   xcd_remap=xcd_remap, muscl_lanes=muscl_lanes,
                   merged_lists=merged_lists, lists_cell_major=lists_cell_major)
        cur.update({k: int(v) for k, v in new.items() if v is not None})
        self._check(self.lib.hfv_set_launch(self.h, C.byref(HfvLaunch(**cur))))

    def autotune(self, U, reps: int = 5, max_records: int = 256):
        """Pick the fastest launch configuration for this state and the current
        parameters (applied); returns (chosen configuration, [(configuration, ms)])."""
        self._chk_u(U)
        best = HfvLaunch()
        recs = (HfvTuneRecord * max_records)()
        n = C.c_int32()
        self._check(self.lib.hfv_autotune(self.h, C.c_void_p(U.data_ptr()), reps, C.byref(best), recs, max_records,
                                          C.byref(n), None))
        as_dict = lambda cfg: {k: getattr(cfg, k) for k, _ in HfvLaunch._fields_}
        return as_dict(best), [(as_dict(r.cfg), r.ms) for r in recs[:min(n.value, max_records)]]

    def profile_enable(self, capacity: int, slots=None):
        mask = 0xff if slots is None else sum(1 << SLOTS[k] for k in slots)
        self._check(self.lib.hfv_profile_enable(self.h, capacity, mask))
        self._prof_on = capacity > 0

    def prof_enabled(self) -> bool:
        return getattr(self, "_prof_on", False)

    def profile_read(self):
        """{slot: (total ms, launches)} of the timed launches since the last read."""
        ms = (C.c_double * 8)()
        n = (C.c_int64 * 8)()
        self._check(self.lib.hfv_profile_read(self.h, ms, n))
        return {k: (ms[i], n[i]) for k, i in SLOTS.items() if n[i]}

    def table(self, name: str) -> np.ndarray:
        N, K, M, d = self.n_cells, self.K, self.M, self.dim
        nfm = 4 if d == 2 else 6
        shapes = dict(PINV=(K, M, N), OI=(K * (K + 1) // 2, N), PSIBAR=(K, N), GEOM=(d + 2, N),
                      PDIR=(nfm, d, 2 * d, N), PMUS=(d, nfm, N), FACE_SLOTS=(self.n_faces,),
                      GP_XI=(self.ngp_cell, d, N))
        if name == "FACE_SLOTS":
            dt = np.int32
        else:
            dt = np.float64 if (name == "GEOM" or self.precision == 64) else np.float32
        out = np.empty(shapes[name], dt)
        self._check(self.lib.hfv_copy_table(self.h, TABLES[name], out.ctypes.data_as(C.c_void_p), out.nbytes))
        return out

    def _chk(self, *bufs):
        """Check every device buffer argument of a call before any address
        crosses the ABI (the library trusts the pointers it is given).

        bufs: (tensor or None, name, kind) with kind "u" ([nvar, n_cells] in
        the context's dtype), "cls" (uint8 [n_cells]), "fs" (the shape of
        new_face_states()) or "rate" (float64 [1]); None entries are skipped.
        Dtype, shape and layout of all buffers are checked first, then that
        each is a CUDA tensor; HfvError on the first failure."""
        import torch
        kinds = dict(u=(self.dtype, (self.nvar, self.n_cells)),
                     cls=(torch.uint8, (self.n_cells,)),
                     fs=(self.dtype, (self.ngp_cell, self.nvar, self.n_cells)),
                     margin=(self.dtype, (self.n_cells,)),
                     rate=(torch.float64, (1,)))
        given = [(x, name, kind) for x, name, kind in bufs if x is not None]
        for x, name, kind in given:
            dtype, shape = kinds[kind]
            if not isinstance(x, torch.Tensor):
                raise HfvError(-1, f"{name} must be a torch tensor, got {type(x).__name__}")
            if x.dtype != dtype:
                raise HfvError(-4, f"{name} must have dtype {dtype}, got {x.dtype}")
            if tuple(x.shape) != tuple(shape):
                raise HfvError(-1, f"{name} must have shape {tuple(shape)}, got {tuple(x.shape)}")
            if not x.is_contiguous():
                raise HfvError(-1, f"{name} must be contiguous")
        for x, name, kind in given:
            if not x.is_cuda:
                raise HfvError(-1, f"{name} must be a CUDA (device) tensor")

    def _chk_u(self, U, name="U"):
        self._chk((U, name, "u"))
        return U

    def new_face_states(self):
        import torch
        return torch.empty((self.ngp_cell, self.nvar, self.n_cells), dtype=self.dtype, device="cuda")

    def reconstruct(self, U, face_states=None, cell_class=None, stream=None, near_margin=None):
        """Face states and classes of U; near_margin, when given (a [n_cells]
        tensor of the context's dtype), receives each cell's relative distance
        to its nearest class threshold."""
        import torch
        self._chk((U, "U", "u"), (face_states, "face_states", "fs"), (cell_class, "cell_class", "cls"),
                  (near_margin, "near_margin", "margin"))
        fs = face_states if face_states is not None else self.new_face_states()
        cls = cell_class if cell_class is not None else torch.empty(self.n_cells, dtype=torch.uint8,
                                                                     device="cuda")
        mgp = C.c_void_p(near_margin.data_ptr()) if near_margin is not None else None
        self._check(self.lib.hfv_reconstruct(self.h, C.c_void_p(U.data_ptr()), C.c_void_p(fs.data_ptr()),
                                             C.c_void_p(cls.data_ptr()), mgp, _stream_handle(stream)))
        return fs, cls

    def residual(self, U, R=None, face_states=None, cell_class=None, stream=None):
        import torch
        self._chk((U, "U", "u"), (R, "R", "u"), (face_states, "face_states", "fs"),
                  (cell_class, "cell_class", "cls"))
        R = R if R is not None else torch.empty_like(U)
        fsp = C.c_void_p(face_states.data_ptr()) if face_states is not None else None
        clp = C.c_void_p(cell_class.data_ptr()) if cell_class is not None else None
        self._check(self.lib.hfv_residual(self.h, C.c_void_p(U.data_ptr()), C.c_void_p(R.data_ptr()), fsp, clp,
                                          _stream_handle(stream)))
        return R

    def residual_noalloc(self, U, R, face_states, cell_class, stream=None):
        """hfv_residual_noalloc: the residual with the kernels' scratch in the
        library's fixed per-device array (no device allocation anywhere in
        the call); every output buffer is the caller's."""
        if R is None or face_states is None or cell_class is None:
            raise HfvError(-1, "R, face_states and cell_class must be given")
        self._chk((U, "U", "u"), (R, "R", "u"), (face_states, "face_states", "fs"),
                  (cell_class, "cell_class", "cls"))
        self._check(self.lib.hfv_residual_noalloc(self.h, C.c_void_p(U.data_ptr()), C.c_void_p(R.data_ptr()),
                                                  C.c_void_p(face_states.data_ptr()),
                                                  C.c_void_p(cell_class.data_ptr()), _stream_handle(stream)))
        return R

    def graph_residual(self, U, R, face_states=None, cell_class=None):
        """Capture one residual evaluation on these buffers into a HIP graph
        (torch.cuda.CUDAGraph); `graph.replay()` then re-runs the whole hot path
        with one launch.  The graph keeps the buffers' addresses: refill U in
        place between replays.  The launch configuration and parameters in
        force at capture are baked in.  The library's per-kernel timing must be
        off while capturing."""
        import torch
        if self.prof_enabled():
            raise HfvError(HFV_ERR_STATE, "disable hfv kernel timing before capturing a graph")
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):                    # warm-up outside the capture
            self.residual(U, R, face_states, cell_class)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.residual(U, R, face_states, cell_class)
        return g

    def residual_vjp(self, U, cell_class, gR, gU=None, stream=None, face_states=None):
        """gU = (dR/dU)^T gR with cell_class frozen; face_states, when given, are
        the states of U from residual / reconstruct (the recompute is skipped)."""
        import torch
        if cell_class is None or gR is None:
            raise HfvError(-1, "cell_class and gR must be given")
        self._chk((U, "U", "u"), (cell_class, "cell_class", "cls"), (gR, "gR", "u"), (gU, "gU", "u"),
                  (face_states, "face_states", "fs"))
        gU = gU if gU is not None else torch.empty_like(U)
        if face_states is None:
            self._check(self.lib.hfv_residual_vjp(self.h, C.c_void_p(U.data_ptr()),
                                                  C.c_void_p(cell_class.data_ptr()), C.c_void_p(gR.data_ptr()),
                                                  C.c_void_p(gU.data_ptr()), _stream_handle(stream)))
        else:
            self._check(self.lib.hfv_residual_vjp_states(
                self.h, C.c_void_p(U.data_ptr()), C.c_void_p(cell_class.data_ptr()),
                C.c_void_p(face_states.data_ptr()), C.c_void_p(gR.data_ptr()), C.c_void_p(gU.data_ptr()),
                _stream_handle(stream)))
        return gU

    def rk_stage(self, out, a, U0, b=0.0, U1=None, c=0.0, R=None, stream=None):
        """out = a U0 + b U1 + c R (one Shu-Osher Runge-Kutta stage); None terms are left out."""
        if out is None:
            raise HfvError(-1, "out must be given")
        self._chk((out, "out", "u"), (U0, "U0", "u"), (U1, "U1", "u"), (R, "R", "u"))
        ptr = lambda x: C.c_void_p(x.data_ptr()) if x is not None else None
        self._check(self.lib.hfv_rk_stage(self.h, a, ptr(U0), b, ptr(U1), c, ptr(R), ptr(out),
                                          _stream_handle(stream)))
        return out

    def cfl_rate(self, U, out=None, stream=None):
        """Device tensor [1] (float64): max over cells of (|u| + c) / h_c."""
        import torch
        self._chk((U, "U", "u"), (out, "out", "rate"))
        out = out if out is not None else torch.empty(1, dtype=torch.float64, device="cuda")
        self._check(self.lib.hfv_cfl_rate(self.h, C.c_void_p(U.data_ptr()), C.c_void_p(out.data_ptr()),
                                          _stream_handle(stream)))
        return out

    def residual_frozen(self, U, cell_class, R=None, stream=None):
        """Residual with the given classes held fixed (what the VJP linearises)."""
        import torch
        if cell_class is None:
            raise HfvError(-1, "cell_class must be given")
        self._chk((U, "U", "u"), (cell_class, "cell_class", "cls"), (R, "R", "u"))
        R = R if R is not None else torch.empty_like(U)
        self._check(self.lib.hfv_residual_frozen(self.h, C.c_void_p(U.data_ptr()),
                                                 C.c_void_p(cell_class.data_ptr()), C.c_void_p(R.data_ptr()),
                                                 _stream_handle(stream)))
        return R

    def residual_autograd(self, U, keep_states: bool = True):
        """R(U) as a differentiable torch op; backward is the library's VJP with
        the classes of this forward evaluation frozen.

        keep_states=True saves the forward's face states for the backward pass
        (no frozen recompute there), at the cost of one [ngp_cell, nvar,
        n_cells] array held per evaluation until backward: ngp_cell * nvar *
        n_cells * 8 bytes in FP64, e.g. 24 * 5 * 1e6 * 4 B = 480 MB in FP32 on
        a million mixed 3D cells at r = 3, once per Runge-Kutta stage of an
        unrolled time loop.  keep_states=False saves only U and the classes
        (n_cells bytes) and the backward pass recomputes the states."""
        return _residual_function().apply(U, self, bool(keep_states))


_RF = None


def _residual_function():
    global _RF
    if _RF is not None:
        return _RF
    import torch

    class Residual(torch.autograd.Function):
        @staticmethod
        def forward(fctx, U, hctx, keep_states):
            U = U.contiguous()
            cls = torch.empty(hctx.n_cells, dtype=torch.uint8, device=U.device)
            fs = hctx.new_face_states() if keep_states else None
            R = hctx.residual(U, face_states=fs, cell_class=cls)
            if keep_states:
                fctx.save_for_backward(U, cls, fs)
            else:
                fctx.save_for_backward(U, cls)
            fctx.hctx = hctx
            fctx.keep_states = keep_states
            return R

        @staticmethod
        def backward(fctx, gR):
            saved = fctx.saved_tensors
            U, cls = saved[0], saved[1]
            fs = saved[2] if fctx.keep_states else None
            gU = fctx.hctx.residual_vjp(U, cls, gR.contiguous(), face_states=fs)
            return gU, None, None

    _RF = Residual
    return _RF
