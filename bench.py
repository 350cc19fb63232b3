"""Benchmark of the hybrid reconstruction + residual on one MI355X.

Default workload: the 2D mixed mesh of 256 x 256 quads with a seeded 30%
split into triangles (85,197 cells), degree r = 3 (4th order), four-quadrant
Riemann data with 1% seeded noise, HLL fluxes.  A step is one residual
evaluation through the whole hot path: linear candidate + NAD, tagging and
compaction, CWENOZ / MUSCL / first-order on the class lists, Harten check,
face fluxes and residual.  Inputs are resident in HBM before the timed region.

Before timing, each (precision, scheme mode) pair is autotuned on the same
state (the library's hfv_autotune), and the chosen launch configuration is
reported.  Prints one JSON line: `value` is the hybrid residual throughput
in cells/s at the workload's headline precision (FP64 for the 2D mixed mesh
and the r = 2 hexahedral case, FP32 for the r = 4 hexahedral case and the
mixed tetrahedron / prism / hexahedron box, as their configurations state);
`modes` holds cells reconstructed/s, residual evaluations/s, the fraction of
the HBM roofline of the reconstruction and of the residual, and per-kernel
times, for hybrid, all-CWENOZ and all-linear in FP64 and FP32.

Bytes: `roofline.bytes_per_launch` and every `*_hbm_frac` count the
algorithmic bytes of the scope definition (ByteModel.s_*: per-cell tables and
states the method must move, neighbours' averages as cache hits, the linear
fit kept on chip for CWENOZ); the `*_model` keys count what each kernel as
built must read and write (it re-reads the fit's tables or the kept fit).
`roofline` is the live measurement of the kernel that takes the most time in
the headline hybrid residual, against the 8 TB/s peak and against the
bandwidth a plain 1 GiB device copy reaches in the same process;
`roofline.traffic` is the counted HBM traffic of that kernel (rocprofv3
FETCH_SIZE + WRITE_SIZE, calibrated) while its sources are unchanged.

Each mode also reports the median of single residuals started after a 1 GiB
write that flushes the last-level cache (`ms_residual_cold`), the step
captured once into a HIP graph and replayed (`ms_residual_graph`), the
adjoint (vector-Jacobian product of the residual with the step's classes
frozen: `ms_vjp`, `vjp_evals_per_s`; `ms_vjp_given_states` when the step's
face states are passed in and not recomputed) and, on workloads whose field
is smooth and known in closed form (the hexahedral Taylor-Green cases), the
RMS error of its face states against the exact point values
(`face_err_rms_rel`), the accuracy at which the modes are compared.  FP32
modes report their face states' largest error against the FP64 path's on
cells of equal class (`fp32_state_err_vs_fp64`) and the number of class
flips (`fp32_class_flips`).  `workloads` repeats the FP32 hybrid /
all-CWENOZ / all-linear measurement, warm and cache-flushed, on the ~1M-cell
mixed 3D box (`--extra`), whose working set exceeds the last-level cache.
Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNELS = {"linear": "k_linear", "classify": "k_classify", "cwenoz": "k_cwenoz", "muscl": "k_muscl",
           "flux": "k_flux", "gather": "k_gather"}
FUSED_NAME = "k_residual"
CSRC = os.path.join(ROOT, "paper_2510_25906_amd", "csrc")


# ---------------------------------------------------------------------------
# Algorithmic bytes.  Each kernel's count is the data it must move once: its
# per-cell (or per-face) tables and inputs, and its outputs.  Values of
# neighbouring cells are taken as cache hits (every cell's averages are
# counted once, as the cell's own).  s is the element size.

class ByteModel:
    def __init__(self, mesh, st, ctx, prec, r):
        self.s = 8 if prec == 64 else 4
        self.K, self.M, self.nv, self.d = ctx.K, ctx.M, ctx.nvar, mesh.dim
        self.Md = 2 * self.d
        nvf = np.diff(mesh.face_vtx_off)
        n = (r + 2) // 2
        if mesh.dim == 2:
            fgp = np.full(mesh.n_faces, n)
        else:
            fgp = np.where(nvf == 3, 3 if r <= 2 else 6, n * n)
        self.fgp = fgp
        owner = np.repeat(np.arange(mesh.n_cells), np.diff(mesh.cell_face_off))
        self.ngp = np.bincount(owner, weights=fgp[mesh.cell_face], minlength=mesh.n_cells)
        self.nfc = np.diff(mesh.cell_face_off)
        self.nvtx = np.diff(mesh.cell_vtx_off)
        self.ndir = st.n_dir.astype(np.float64)
        self.nmus = st.n_muscl.astype(np.float64)
        self.N, self.NF = mesh.n_cells, mesh.n_faces

    def linear(self, keep_fit=False):
        s, K, M, nv, d = self.s, self.K, self.M, self.nv, self.d
        per_cell = s * K * M + 4 * M + s * nv + s * K + 2 + s + 1 + (s * K * nv if keep_fit else 0)
        return self.N * per_cell + self.ngp.sum() * (s * d + s * nv) + 4 * self.nfc.sum()

    def classify(self, n_listed):
        return 3 * self.N + 4 * self.nfc.sum() + 4 * n_listed

    def cwenoz(self, m, reuse=False, listed=True):
        s, K, M, nv, d, Md = self.s, self.K, self.M, self.nv, self.d, self.Md
        fit = s * K * nv if reuse else s * K * M + 4 * M
        per = fit + s * nv + 2 + s * K * (K + 1) // 2 + s * K + (4 if listed else 0) + 1
        return (m.sum() * per + (self.ndir[m] * (4 * Md + s * d * Md)).sum()
                + self.ngp[m].sum() * (s * d + s * nv))

    def muscl(self, m):
        s, nv, d = self.s, self.nv, self.d
        per = s * nv + 2 + s * d + 4 + 1
        return (m.sum() * per + (self.nmus[m] * (4 + s * d)).sum() + 4 * self.nfc[m].sum()
                + self.ngp[m].sum() * (s * d + s * nv))

    def first(self, m):
        return m.sum() * (4 + self.s * self.nv + 1) + self.ngp[m].sum() * self.s * self.nv

    def flux(self):
        s, nv, d = self.s, self.nv, self.d
        return self.NF * (s * d + 16 + s * nv) + self.fgp.sum() * (2 * s * nv + s)

    def gather(self):
        s, nv = self.s, self.nv
        return self.N * (8 + s + s * nv) + self.nfc.sum() * (4 + s * nv)

    def residual_fused(self):
        # flux and gather without the face-flux array between them
        s, nv = self.s, self.nv
        return self.flux() - self.NF * s * nv + self.gather() - self.nfc.sum() * s * nv

    # --- the scope definition's algorithmic bytes --------------------------
    # What the method must move per unit, the neighbours' averages taken as
    # cache hits and the linear pass's fit as kept on chip:
    #   linear (every cell): s K M (pseudo-inverse) + 4 M (stencil ids)
    #     + s nvar (U) + s K (basis means) + s d n_vtx (geometry for the Gauss
    #     points) + s nvar n_gp (face states) + 1 (class);
    #   CWENOZ extra (listed cell): s K (K+1)/2 (OI) + N_f (s d M_d + 4 M_d)
    #     (directional fits and ids) + s nvar n_gp (states re-written);
    #   MUSCL extra: s d N_f + s nvar n_gp;  first-order extra: s nvar n_gp;
    #   residual: both sides' face states, face geometry (normal, weight x
    #     area), F written (nvar per face), F gathered (twice per face), R.
    def s_linear(self):
        s, K, M, nv, d = self.s, self.K, self.M, self.nv, self.d
        return (self.N * (s * K * M + 4 * M + s * nv + s * K + 1) + s * d * self.nvtx.sum()
                + self.ngp.sum() * s * nv)

    def s_cwenoz_extra(self, m):
        s, K, nv, d, Md = self.s, self.K, self.nv, self.d, self.Md
        return (m.sum() * s * K * (K + 1) // 2 + (self.ndir[m] * (s * d * Md + 4 * Md)).sum()
                + self.ngp[m].sum() * s * nv)

    def s_muscl_extra(self, m):
        return (self.s * self.d * self.nfc[m].sum() + self.ngp[m].sum() * self.s * self.nv)

    def s_first_extra(self, m):
        return self.ngp[m].sum() * self.s * self.nv

    def s_flux(self):
        s, nv, d = self.s, self.nv, self.d
        return self.fgp.sum() * (2 * s * nv + s) + self.NF * (s * d + s * nv)

    def s_gather(self):
        s, nv = self.s, self.nv
        return 2 * self.NF * s * nv + self.N * s * nv

    def s_per_kernel(self, mode, cls, fused, merged=False):
        """{kernel: bytes} of one reconstruction + residual in `mode` by the
        scope definition (all-CWENOZ cells count the linear bytes too, with
        one write of the states: the direct CWENOZ pass does the fit itself;
        merged: the MUSCL and first-order lists' bytes are the CWENOZ
        launch's)."""
        cw, mu, fo = cls == 1, cls == 2, cls == 3
        if mode == "cwenoz":   # the direct pass writes each cell's states once
            out = {"cwenoz": self.s_linear() + self.s_cwenoz_extra(np.ones(self.N, bool))
                   - self.ngp.sum() * self.s * self.nv}
        else:
            out = {"linear": self.s_linear()}
            if mode == "hybrid":
                out["cwenoz"] = self.s_cwenoz_extra(cw)
            out["muscl"] = self.s_muscl_extra(mu) + self.s_first_extra(fo)
            if merged and mode == "hybrid":
                out["cwenoz"] += out.pop("muscl")
        if fused:
            out["flux"] = self.s_flux() + self.s_gather() - 3 * self.NF * self.s * self.nv
        else:
            out["flux"] = self.s_flux()
            out["gather"] = self.s_gather()
        return {k: int(v) for k, v in out.items()}

    def per_kernel(self, mode, cls, reuse, fused, merged=False):
        """{kernel: bytes} of one reconstruction + residual in `mode`."""
        cw, mu, fo = cls == 1, cls == 2, cls == 3
        if mode == "cwenoz":
            out = {"cwenoz": self.cwenoz(np.ones(self.N, bool), listed=False)}
        else:
            out = {"linear": self.linear(keep_fit=(mode == "hybrid" and reuse)),
                   "classify": self.classify(int((cls > 0).sum()))}
            if mode == "hybrid":
                out["cwenoz"] = self.cwenoz(cw, reuse=reuse)
            out["muscl"] = self.muscl(mu) + self.first(fo)
            if merged and mode == "hybrid":
                out["cwenoz"] += out.pop("muscl")
        if fused:
            out["flux"] = self.residual_fused()
        else:
            out["flux"] = self.flux()
            out["gather"] = self.gather()
        return {k: int(v) for k, v in out.items()}


def kernel_name(slot, launch):
    """The kernel a timing slot runs under this launch configuration."""
    if slot == "flux" and launch.get("fused_residual"):
        return FUSED_NAME
    if slot == "linear":
        return ("k_linear", "k_linear_ms", "k_linear_ks")[launch.get("linear_split", 0)]
    return KERNELS[slot]


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def time_cold(fn, reps, flush, torch):
    """Median time of single steps, each started after a write over `flush`
    (>= 1 GiB), so that none of its inputs is left in the 256 MB last-level
    cache (MALL)."""
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    ts = []
    for i in range(reps):
        flush.fill_(float(i))
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def probe_bandwidth(torch, mib=1024, reps=20):
    """HBM bandwidth a plain device-to-device copy achieves: (read + written
    bytes) / time, median over `reps` copies of `mib` MiB."""
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        a.record()
        y.copy_(x)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    del x, y
    return 2.0 * n * 4 / (float(np.median(ts)) * 1e-3) / 1e9


class FaceAccuracy:
    """Face Gauss-point states against the exact point values of a smooth
    workload: RMS error over every (Gauss point, cell) relative to the
    variable's largest exact value, the largest over the variables."""

    def __init__(self, ctx, w, ngp):
        d, N = w.mesh.dim, w.mesh.n_cells
        xi = ctx.table("GP_XI").astype(np.float64)        # [NGPC][d][N]
        geom = ctx.table("GEOM")                          # centroid, volume, h_c
        self.valid = np.arange(xi.shape[0])[:, None] < ngp[None, :].astype(np.int64)  # [NGPC][N]
        ex = np.zeros((xi.shape[0], N, w.U.shape[1]))
        for g in range(xi.shape[0]):
            x = (geom[:d] + geom[d + 1][None, :] * xi[g]).T    # [N, d]
            ex[g] = w.exact(x)
        self.ex = ex.transpose(0, 2, 1)                   # [NGPC][nvar][N], like the states
        self.scale = np.abs(self.ex).max(axis=(0, 2))

    def error(self, fs):
        f = fs.cpu().numpy().astype(np.float64)
        m = self.valid[:, None, :]
        e2 = np.where(m, (f - self.ex) ** 2, 0.0).sum(axis=(0, 2)) / m.sum()
        return float((np.sqrt(e2) / self.scale).max())


def fp32_error(ref, fs32, cls32, ngp, U, face_cells=None):
    """FP32 face states against the FP64 path's (which the parity tests hold to
    1e-12 of the FP64 oracle): largest error over the Gauss points of cells of
    equal class, relative to the variable's largest cell average, and the number
    of cells whose class differs (FP32 flips near an NAD threshold).  With the
    FP64 path's near_margin in `ref` and the mesh's face_cells, also the flips
    in cells neither within 1e-6 of a threshold nor next to such a cell, and
    the flag level every flip does meet: the largest over the flipped cells of
    the smallest margin of the cell and its face neighbours."""
    fs64, cls64 = ref[0], ref[1]
    margin = ref[2] if len(ref) > 2 else None
    same = cls64 == cls32
    valid = (np.arange(fs64.shape[0])[:, None] < ngp[None, :]) & same[None, :]     # [NGPC][N]
    scale = np.abs(U).max(0)                                                        # [nvar]
    err = 0.0
    for v in range(fs64.shape[1]):
        d = np.abs(fs32[:, v, :].astype(np.float64) - fs64[:, v, :])
        err = max(err, float(np.where(valid, d, 0.0).max()) / scale[v])
    out = {"fp32_state_err_vs_fp64": float(f"{err:.4g}"), "fp32_class_flips": int((~same).sum())}
    if margin is not None and face_cells is not None:
        small = margin <= 1e-6
        flagged = small.copy()
        inner = face_cells[:, 1] >= 0
        a, b = face_cells[inner, 0], face_cells[inner, 1]
        np.logical_or.at(flagged, a, small[b])
        np.logical_or.at(flagged, b, small[a])
        out["fp32_flips_unflagged"] = int((~same & ~flagged).sum())
        out["cells_margin_le_1e-6"] = int(small.sum())
        near = margin.astype(np.float64).copy()
        np.minimum.at(near, a, margin[b])
        np.minimum.at(near, b, margin[a])
        out["fp32_flip_margin_max"] = float(f"{near[~same].max():.3g}") if (~same).any() else None
    return out


# the sources the forward hot-path kernels are compiled from: a change to any of
# them invalidates counter records taken before it
HOT_SOURCES = ("hfv_hot.cpp", "hfv_device.hpp", "hfv_internal.hpp")


def source_hash():
    h = hashlib.sha256()
    for f in HOT_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def launch_string(launch):
    """A launch configuration as the profile records write it: k=v,... in field order."""
    return ",".join(f"{k}={v}" for k, v in launch.items())


def kernel_instance(slot, launch, dim, r, prec):
    """The compiled kernel (template instance, as rocprofv3 names it) that a
    hybrid-mode timing slot runs under this launch configuration; None for
    slots whose instance is not modelled here."""
    T = "double" if prec == 64 else "float"
    tf = lambda b: "true" if b else "false"
    if slot == "linear":
        return f"{kernel_name(slot, launch)}<{dim}, {r}, {T}, {launch['linear_lanes']}, false>"
    if slot == "cwenoz":
        g = launch["lanes_per_cell"]
        cm = launch.get("lists_cell_major", 0) and g != 1      # one lane per cell keeps the [entry][cell] reads
        return (f"k_cwenoz<{dim}, {r}, {T}, {g}, {tf(launch['cwenoz_reuse'])}, "
                f"{tf(launch.get('merged_lists', 0))}, {tf(cm)}>")
    return None


def measured_traffic(kernel, workload, instance=None):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel and workload (a file holds one record, or a list under
    "records", one per kernel instance), or None when there is none for this
    instance, or it was taken on other sources.  The launch's grid shape is
    not matched: it changes how the kernel is spread over the chip, not the
    kernel."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    for r in rec.get("records", [rec]):
        if r.get("source_hash") == source_hash() and (instance is None or r.get("kernel") == instance):
            return r.get("bytes_per_launch")
    return None


def cpu_baseline(w, cells_target=None, min_seconds=10.0):
    """The FP64 oracle's residual on the host: tables precomputed (untimed), one
    BLAS thread, the whole mesh (or ``cells_target`` cells), repeated until at
    least ``min_seconds`` of work have been timed."""
    from oracle import OracleModel
    om = OracleModel(w.mesh, w.stencils, w.params)
    N = w.mesh.n_cells
    n = N if cells_target is None else min(N, cells_target)
    sample = np.arange(n)
    fc = w.mesh.face_cells
    fmask = np.isin(fc[:, 0], sample) | np.isin(fc[:, 1], sample)
    faces = np.nonzero(fmask)[0]
    closure = np.unique(fc[faces].ravel())
    closure = closure[closure >= 0]
    nb = om.nbr[closure].ravel()
    om.tables(np.unique(np.concatenate([closure, nb[nb >= 0]])))
    geo = om.geo
    passes, dt = 0, 0.0
    while dt < min_seconds:
        dt += _oracle_pass(om, w, closure, fc, fmask, geo, n, N)
        passes += 1
    return dict(value=round(passes * n / dt, 1), unit="cells/s", cores=1, kind="oracle",
                sample=f"FP64 NumPy oracle, hybrid residual of {n} of {N} cells (with their face-neighbour "
                       f"closure), one BLAS thread, tables precomputed outside the timing, {passes} passes "
                       f"in {dt:.1f} s")


_CPU_SHARED = None


def _oracle_chunk(cells):
    om, U = _CPU_SHARED
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        return om.reconstruct_cells(cells, U)[0]


def cpu_baseline_all_cores(w, workers, min_seconds=10.0):
    """The same FP64 oracle residual over the whole mesh on `workers` host
    cores: the per-cell reconstruction (the bulk of the work) split by cell
    range over forked processes with one BLAS thread each, the face fluxes
    and the residual in the parent; tables precomputed and the pool started
    outside the timing.  Must run before the process touches the GPU."""
    import multiprocessing as mp
    from oracle import OracleModel
    from oracle import flux as oflux
    global _CPU_SHARED
    om = OracleModel(w.mesh, w.stencils, w.params)
    N = w.mesh.n_cells
    cells = np.arange(N)
    om.tables(cells)
    chunks = np.array_split(cells, 8 * workers)
    _CPU_SHARED = (om, w.U)
    passes, dt = 0, 0.0
    with mp.get_context("fork").Pool(workers) as pool:
        while dt < min_seconds:
            t0 = time.perf_counter()
            fv = np.concatenate(pool.map(_oracle_chunk, chunks))
            fs = om.scatter_face_states(cells, fv)
            oflux.residual_from_face_fluxes(om, oflux.face_fluxes(om, fs, w.params.riemann))
            dt += time.perf_counter() - t0
            passes += 1
    _CPU_SHARED = None
    return dict(value=round(passes * N / dt, 1), unit="cells/s", cores=workers, kind="oracle",
                sample=f"FP64 NumPy oracle, hybrid residual of all {N} cells; per-cell reconstruction over {workers} "
                       f"forked processes (one BLAS thread each), face fluxes and residual in the parent; tables "
                       f"precomputed outside the timing, {passes} passes in {dt:.1f} s")


def _oracle_pass(om, w, closure, fc, fmask, geo, n, N):
    from threadpoolctl import threadpool_limits
    from oracle import flux as oflux
    with threadpool_limits(1):
        t0 = time.perf_counter()
        fv, cls = om.reconstruct_cells(closure, w.U)
        fs = om.scatter_face_states(closure, fv) if n == N else None
        if fs is None:
            fs = np.zeros((2, om.nvar, geo.n_gp))
            for i, c in enumerate(closure):
                k = geo.c_ngp[c]
                fs[geo.c_side[c, :k], :, geo.c_gidx[c, :k]] = fv[i, :k]
            bnd = fc[:, 1] < 0
            for f in np.nonzero(bnd & fmask)[0]:
                a, b = geo.gp_off[f], geo.gp_off[f + 1]
                fs[1, :, a:b] = fs[0, :, a:b]
        Ff = oflux.face_fluxes(om, fs, w.params.riemann)
        oflux.residual_from_face_fluxes(om, Ff)
        return time.perf_counter() - t0


WORKLOADS = {
    "c2": ("2D Euler, 256x256 quads with seeded 30% split into triangles (85,197 cells), r=3 (4th order), "
           "four-quadrant Riemann data + 1% noise, HLL; hybrid residual", "mixed2d_85k_r3", 64),
    "c3": ("3D Euler, periodic 64^3 hexahedra (262,144 cells), r=4 (5th order), Taylor-Green vortex at "
           "Mach 1.25 with seeded perturbation, HLLC; hybrid residual", "hex64_r4", 32),
    "c4": ("3D Euler, mixed box of 569,024 tetrahedra, 5,792 pyramids, 28,672 prisms (wall layer) and "
           "396,032 hexahedra (999,520 cells), r=3 (4th order), Mach-3 normal shock with Rankine-Hugoniot "
           "states and three Gaussian vortices, HLLC; hybrid residual", "mixed3d_1m_r3", 32),
    "c5": ("3D Euler, periodic 64^3 hexahedra (262,144 cells), r=2, Taylor-Green vortex at Mach 1.25 with "
           "seeded perturbation, HLLC; hybrid residual", "hex64_r2", 64),
}


def make_workload(name, workers, cell_order="lattice"):
    from paper_2510_25906_amd.inputs import configs
    return {"c2": lambda: configs.c2_riemann(256, 3), "c3": lambda: configs.tgv_hex(64, 4),
            "c4": lambda: configs.c4_mixed("full", workers=workers, cell_order=cell_order),
            "c5": lambda: configs.tgv_hex(64, 2)}[name]()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse_args(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c2")
    ap.add_argument("--extra", default="c4",
                    help="comma-separated workloads also measured (FP32 hybrid / all-CWENOZ / all-linear, "
                         "warm and cache-flushed) under `workloads` in the JSON line; empty for none")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the library's default launch configuration")
    ap.add_argument("--launch", default="",
                    help="fixed launch configuration instead of tuning, e.g. lanes_per_cell=2,linear_split=1")
    ap.add_argument("--quick", action="store_true", help="headline hybrid variant only (for profiling runs)")
    ap.add_argument("--spinup", type=float, default=1.0,
                    help="seconds of untimed residual evaluations before each variant (steady clocks)")
    ap.add_argument("--workers", type=int, default=max(1, min(16, os.cpu_count() or 1)),
                    help="processes for input generation (1 when a profiler has initialised the GPU "
                         "before the program starts: the generator forks)")
    ap.add_argument("--cell-order", choices=("lattice", "morton"), default="lattice",
                    help="cell numbering of the mixed box: cubes in lattice order or along a Morton curve")
    ap.add_argument("--cold", type=int, default=10,
                    help="also time this many single residuals, each after a 1 GiB cache-flushing write "
                         "(0: skip)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    return ap.parse_args(argv)


def measure(w, wl_tag, head_prec, variants, args, torch, hfv, probe, flush, extra_leg=False):
    """Autotune and time each (precision, mode) variant of workload `w`.
    Returns (modes, headline ms per residual, roofline of the headline's
    dominant kernel, headline class counts)."""
    from paper_2510_25906_amd.inputs.params import HYBRID, ALL_CWENOZ, ALL_LINEAR
    acc = None
    ref64 = {}    # FP64 face states and classes per mode, for the FP32 error
    mesh = w.mesh
    N = mesh.n_cells
    names = {HYBRID: "hybrid", ALL_CWENOZ: "cwenoz", ALL_LINEAR: "linear"}
    modes, headline, roof, classes = {}, None, None, None
    for prec in sorted(set(p for p, _ in variants), reverse=True):
        t0 = time.perf_counter()
        ctx = hfv.Context(mesh, w.stencils, w.params, prec)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        bm = ByteModel(mesh, w.stencils, ctx, prec, w.params.order_r)
        dtype = torch.float64 if prec == 64 else torch.float32
        U = torch.tensor(np.ascontiguousarray(w.U.T), dtype=dtype, device="cuda")
        fs = ctx.new_face_states()
        cls = torch.empty(N, dtype=torch.uint8, device="cuda")
        R = torch.empty_like(U)
        default_launch = ctx.get_launch()
        for p_, mode in variants:
            if p_ != prec:
                continue
            name = names[mode]
            ctx.set_params(w.params.with_(scheme_mode=mode))
            dl = dict(default_launch)
            ctx.set_launch(lanes=dl.pop("lanes_per_cell"), **dl)
            t_tune = 0.0
            if args.launch and not extra_leg:
                fixed = dict(kv.split("=") for kv in args.launch.split(","))
                fixed = {k: int(v) for k, v in fixed.items()}
                if "lanes_per_cell" in fixed:
                    fixed["lanes"] = fixed.pop("lanes_per_cell")
                ctx.set_launch(**fixed)
            elif not args.no_tune:
                t0 = time.perf_counter()
                ctx.autotune(U, reps=5)
                t_tune = time.perf_counter() - t0
            launch = ctx.get_launch()
            log(f"{wl_tag} FP{prec} {name}: setup {t_setup:.1f} s, tuned in {t_tune:.1f} s")
            # spin-up: first launches load code objects, and the clocks settle
            # under sustained load
            t_end = time.perf_counter() + args.spinup
            while True:
                for _ in range(20):
                    ctx.residual(U, R, fs, cls)
                torch.cuda.synchronize()
                if time.perf_counter() >= t_end:
                    break
            # per-kernel times of this configuration (untimed pass, all slots)
            ctx.profile_enable(16 * 8)
            for _ in range(8):
                ctx.residual(U, R, fs, cls)
            torch.cuda.synchronize()
            kern = {k: v[0] / 8 for k, v in ctx.profile_read().items()}  # ms per step
            ctx.profile_enable(0)
            dominant = max(kern, key=kern.get)
            ms_rec = time_steps(lambda: ctx.reconstruct(U, fs, cls), args.steps, args.warmup, torch)
            live = prec == head_prec and mode == HYBRID
            if live:  # the dominant kernel timed with HIP events on its stream, inside the timed region
                ctx.profile_enable(args.steps * 2, slots=[dominant])
            ms_res = time_steps(lambda: ctx.residual(U, R, fs, cls), args.steps, 0 if live else args.warmup, torch)
            cl_dev = cls.cpu().numpy()
            reuse, fused = bool(launch["cwenoz_reuse"]), bool(launch["fused_residual"])
            merged = bool(launch.get("merged_lists", 0))
            mbyts = bm.per_kernel(name, cl_dev, reuse, fused, merged)    # the kernels' own byte counts
            sbyts = bm.s_per_kernel(name, cl_dev, fused, merged)         # the scope definition's bytes
            if live:
                prof = ctx.profile_read()
                ctx.profile_enable(0)
                k_ms, k_n = prof[dominant]
                avg = k_ms / k_n
                ach = sbyts[dominant] / (avg * 1e-3) / 1e9
                ach_m = mbyts[dominant] / (avg * 1e-3) / 1e9
                kname = kernel_name(dominant, launch)
                traffic = measured_traffic(kname, wl_tag,
                                           kernel_instance(dominant, launch, mesh.dim, w.params.order_r, prec))
                roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                        "traffic_over_bytes": round(traffic / sbyts[dominant], 3) if traffic else None,
                        "probe_copy_GBps": round(probe, 1), "frac_of_probe": round(ach / probe, 4),
                        "kernel": f"{kname} ({name}, FP{prec})",
                        "bytes_per_launch": sbyts[dominant], "avg_launch_ms": round(avg, 5),
                        "model_bytes_per_launch": mbyts[dominant], "achieved_model": round(ach_m, 1),
                        "frac_model": round(ach_m / HBM_PEAK_GBS, 4),
                        "step_bytes": int(sum(sbyts.values())),
                        "step_frac": round(sum(sbyts.values()) / (ms_res * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
                headline = ms_res
                classes = np.bincount(cl_dev, minlength=4)
            ms_cold = time_cold(lambda: ctx.residual(U, R, fs, cls), args.cold, flush, torch) if args.cold else None
            rec = {}
            if not extra_leg:
                # the adjoint with these classes frozen (vector-Jacobian product of the residual)
                gR = torch.ones_like(U)
                gU = torch.empty_like(U)
                ctx.residual(U, R, fs, cls)
                ms_vjp = time_steps(lambda: ctx.residual_vjp(U, cls, gR, gU), args.steps, args.warmup, torch)
                ms_vjp_states = time_steps(lambda: ctx.residual_vjp(U, cls, gR, gU, face_states=fs), args.steps,
                                           args.warmup, torch)
                del gR, gU
                # the same step captured once into a HIP graph and replayed (one launch per step)
                graph = ctx.graph_residual(U, R, fs, cls)
                ms_graph = time_steps(graph.replay, args.steps, args.warmup, torch)
                del graph
                rec.update(ms_residual_graph=round(ms_graph, 4), ms_vjp=round(ms_vjp, 4),
                           vjp_evals_per_s=round(1.0 / (ms_vjp * 1e-3), 2),
                           vjp_over_residual=round(ms_vjp / ms_res, 3),
                           ms_vjp_given_states=round(ms_vjp_states, 4))
            face_err = None
            if w.exact is not None:
                if acc is None:
                    acc = FaceAccuracy(ctx, w, bm.ngp)
                face_err = acc.error(fs)
            fp32_err = None
            if prec == 64 and any(p_ == 32 for p_, m_ in variants if m_ == mode):
                mg = torch.empty(N, dtype=torch.float64, device="cuda")
                ctx.reconstruct(U, fs, cls, near_margin=mg)
                ref64[mode] = (fs.cpu().numpy(), cls.cpu().numpy(), mg.cpu().numpy())
                del mg
            elif prec == 32 and mode in ref64:
                fp32_err = fp32_error(ref64.pop(mode), fs.cpu().numpy(), cl_dev, bm.ngp, w.U, mesh.face_cells)
            cl = np.bincount(cl_dev, minlength=4)
            rec_s = sum(v for k, v in sbyts.items() if k not in ("flux", "gather"))
            rec_m = sum(v for k, v in mbyts.items() if k not in ("flux", "gather"))
            frac = lambda b, ms: round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            modes[f"{name}_fp{prec}"] = {
                "recon_cells_per_s": round(N / (ms_rec * 1e-3), 1),
                "residual_evals_per_s": round(1.0 / (ms_res * 1e-3), 2),
                "residual_cells_per_s": round(N / (ms_res * 1e-3), 1),
                "ms_recon": round(ms_rec, 4), "ms_residual": round(ms_res, 4),
                "recon_hbm_frac": frac(rec_s, ms_rec),
                "residual_hbm_frac": frac(sum(sbyts.values()), ms_res),
                "recon_hbm_frac_model": frac(rec_m, ms_rec),
                "residual_hbm_frac_model": frac(sum(mbyts.values()), ms_res),
                "class_fractions": [round(x / N, 4) for x in cl],
                "kernel_us": {k: round(v * 1e3, 1) for k, v in kern.items()},
                "kernel_hbm_frac": {k: frac(sbyts[k], kern[k]) for k in kern if k in sbyts},
                "kernel_hbm_frac_model": {k: frac(mbyts[k], kern[k]) for k in kern if k in mbyts},
                "launch": launch, "tune_s": round(t_tune, 2), "setup_s": round(t_setup, 3),
                **rec,
            }
            if ms_cold is not None:
                modes[f"{name}_fp{prec}"]["ms_residual_cold"] = round(ms_cold, 4)
                modes[f"{name}_fp{prec}"]["residual_hbm_frac_cold"] = frac(sum(sbyts.values()), ms_cold)
            if face_err is not None:
                modes[f"{name}_fp{prec}"]["face_err_rms_rel"] = float(f"{face_err:.6g}")
            if fp32_err is not None:
                modes[f"{name}_fp{prec}"].update(fp32_err)
        ctx.close()
        del U, fs, cls, R
        torch.cuda.empty_cache()
    for prec in (64, 32):
        h, c = modes.get(f"hybrid_fp{prec}"), modes.get(f"cwenoz_fp{prec}")
        if h and c:
            h["speedup_vs_cwenoz_residual"] = round(c["ms_residual"] / h["ms_residual"], 3)
            h["speedup_vs_cwenoz_recon"] = round(c["ms_recon"] / h["ms_recon"], 3)
            if "ms_residual_cold" in h and "ms_residual_cold" in c:
                h["speedup_vs_cwenoz_residual_cold"] = round(c["ms_residual_cold"] / h["ms_residual_cold"], 3)
    return modes, headline, roof, classes


def main():
    args = parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding of the mesh "
                                   "is described in the design notes but not built", "n_gpus": args.gpus}))
        sys.exit(2)

    # inputs first: the mixed-mesh generator forks worker processes, which must
    # happen before this process touches the GPU
    t0 = time.perf_counter()
    w = make_workload(args.workload, workers=args.workers, cell_order=args.cell_order)
    wl_text, wl_tag, head_prec = WORKLOADS[args.workload]
    log(f"workload {args.workload}: {w.mesh.n_cells} cells, built in {time.perf_counter() - t0:.1f} s")
    extras = [x for x in args.extra.split(",") if x and x != args.workload] if not args.quick else []
    extra_w = {}
    for x in extras:
        t0 = time.perf_counter()
        extra_w[x] = make_workload(x, workers=args.workers, cell_order=args.cell_order)
        log(f"extra workload {x}: {extra_w[x].mesh.n_cells} cells, built in {time.perf_counter() - t0:.1f} s")
    # the oracle on the host cores, before the GPU is touched (the all-core leg forks)
    cpu1 = cpuN = None
    if not args.no_cpu_baseline and args.workload == "c2":
        cpu1 = cpu_baseline(w)
        cpuN = cpu_baseline_all_cores(w, args.workers) if args.workers > 1 else None
        log(f"oracle: {cpu1['value']:.3g} cells/s on 1 core"
            + (f", {cpuN['value']:.3g} on {cpuN['cores']}" if cpuN else ""))
        for rec in (cpu1, cpuN):
            if rec is not None:
                rec["host_cpu"] = host_cpu_model()

    import torch
    from paper_2510_25906_amd import hfv
    from paper_2510_25906_amd.inputs.params import HYBRID, ALL_CWENOZ, ALL_LINEAR

    hfv.load()
    if args.copy_mib:
        n = args.copy_mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    probe = probe_bandwidth(torch)
    log(f"copy probe {probe:.0f} GB/s")
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda") if args.cold else None
    variants = [(head_prec, HYBRID)] if args.quick else \
        [(p, m) for p in (64, 32) for m in (HYBRID, ALL_CWENOZ, ALL_LINEAR)]
    modes, headline, roof, classes = measure(w, wl_tag, head_prec, variants, args, torch, hfv, probe, flush)
    N = w.mesh.n_cells
    others = {}
    for x, wx in extra_w.items():
        text_x, tag_x, prec_x = WORKLOADS[x]
        m_x, h_x, roof_x, cls_x = measure(wx, tag_x, prec_x,
                                          [(prec_x, HYBRID), (prec_x, ALL_CWENOZ), (prec_x, ALL_LINEAR)],
                                          args, torch, hfv, probe, flush, extra_leg=True)
        Nx = wx.mesh.n_cells
        others[x] = {"workload": text_x, "n_cells": Nx, "precision": f"fp{prec_x}",
                     "residual_cells_per_s": round(Nx / (h_x * 1e-3), 1), "ms_per_step": round(h_x, 5),
                     "class_fractions": [round(v / Nx, 4) for v in cls_x], "roofline": roof_x, "modes": m_x}
        del wx
    out = {
        "metric": "cells reconstructed/s & residual evals/s: hybrid vs all-CWENOZ, FP32 vs FP64",
        "value": round(N / (headline * 1e-3), 1),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(headline, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"f{head_prec}",
        "data": "synthetic",
        "config": {"workload": wl_text, "n_cells": N, "order_r": w.params.order_r, "precision": f"fp{head_prec}",
                   "class_fractions": [round(x / N, 4) for x in classes] if classes is not None else None},
        "roofline": roof,
        "modes": modes,
        "paper_context": "paper: up to 2.5x hybrid over CWENOZ, whole viscous solver on ARCHER2 CPUs "
                         "(10 nodes x 128 cores), 128^3 hex TGV",
    }
    if others:
        out["workloads"] = others
    if cpu1 is not None:
        out["cpu_baseline"] = cpu1
    if cpuN is not None:
        out["cpu_baseline_all_cores"] = cpuN
    print(json.dumps(out), flush=True)


def host_cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
