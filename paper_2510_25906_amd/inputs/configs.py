"""The workloads: meshes, stencils and seeded initial fields.

Seeds: 0 for the mesh, 1 for field noise or perturbation, 2 for random
directions.  The workloads mirror the paper's test cases (Section 3) at the
sizes listed in ``CONFIGS``.

When the environment variable HFV_INPUT_CACHE names a directory, meshes with
their stencils (and the mixed box's field) are stored there on first use and
loaded from there afterwards; the cache is keyed by workload and size only, so
clear it after changing a generator.
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np

from .mesh import Mesh, quad_tri_2d, hex_3d, mixed_box
from .stencil import Stencils, build_stencils, build_stencils_periodic_hex
from . import fields
from .params import Params


@dataclass
class Workload:
    name: str
    mesh: Mesh
    stencils: Stencils
    U: np.ndarray      # float64 [N, nvar] cell averages of conserved variables
    params: Params
    # point values of the conserved variables, f(points [..., d]) -> [..., nvar],
    # where the field is smooth everywhere (None otherwise)
    exact: object = None


def _cache_path(key):
    root = os.environ.get("HFV_INPUT_CACHE")
    if not root:
        return None
    os.makedirs(root, exist_ok=True)
    return os.path.join(root, key + ".npz")


def _save(path, mesh, st):
    arrs = {}
    for k, v in mesh.__dict__.items():
        if isinstance(v, np.ndarray):
            arrs["m_" + k] = v
    arrs["m_dim"] = np.array(mesh.dim)
    for k, v in st.__dict__.items():
        arrs["s_" + k] = np.asarray(v)
    np.savez(path, **arrs)


def _load(path):
    z = np.load(path)
    mk = {k[2:]: z[k] for k in z.files if k.startswith("m_")}
    sk = {k[2:]: z[k] for k in z.files if k.startswith("s_")}
    dim = int(mk.pop("dim"))
    period = mk.pop("period", None)
    mesh = Mesh(dim=dim, period=period, **{k: v for k, v in mk.items()
                                           if k not in ("cell_face_off", "cell_face", "cell_face_side")})
    mesh.finalize()
    st = Stencils(**{k: (int(v) if v.ndim == 0 else v) for k, v in sk.items()})
    return mesh, st


def mesh_and_stencils(key, make_mesh, r, workers=1):
    path = _cache_path(key)
    if path and os.path.exists(path):
        return _load(path)
    mesh = make_mesh()
    st = build_stencils(mesh, r, workers=workers)
    if path:
        _save(path, mesh, st)
    return mesh, st


# ---------------------------------------------------------------------------

def c1_density_jump(n=32, r=2, jump=True) -> Workload:
    """Periodic unit square, n x n quads each split into two triangles."""
    mk = lambda: quad_tri_2d(n, n, split=np.ones((n, n), bool), periodic=True, name=f"tri{n}")
    mesh, st = mesh_and_stencils(f"tri{n}_r{r}", mk, r)
    U = fields.cell_average(mesh, lambda p: fields.density_jump_2d(p, jump=jump), nq=r + 4)
    return Workload(f"c1_tri{n}_r{r}", mesh, st, U, Params(order_r=r))


def c2_riemann(n=256, r=3, frac=0.3, noise=0.01) -> Workload:
    """[-1/2, 1/2]^2, n x n quads with a seeded 30% split into triangles."""
    def mk():
        rng = np.random.default_rng(0)
        nsplit = int(round(frac * n * n))
        split = np.zeros(n * n, bool)
        split[rng.choice(n * n, nsplit, replace=False)] = True
        return quad_tri_2d(n, n, lo=(-0.5, -0.5), hi=(0.5, 0.5), split=split.reshape(n, n),
                           periodic=False, name=f"mixed{n}")
    mesh, st = mesh_and_stencils(f"mixed{n}_r{r}", mk, r)
    prim = fields.cell_average(mesh, fields.riemann_2d_prim, nq=2)
    rng = np.random.default_rng(1)
    xi = rng.uniform(-1, 1, size=prim.shape)
    prim[:, 0] *= 1 + noise * xi[:, 0]
    prim[:, 3] *= 1 + noise * xi[:, 3]
    prim[:, 1] += noise * xi[:, 1]
    prim[:, 2] += noise * xi[:, 2]
    U = fields.prim_to_cons(prim)
    return Workload(f"c2_mixed{n}_r{r}", mesh, st, U, Params(order_r=r, riemann=1))


def tgv_hex(n=64, r=4, perturb=True) -> Workload:
    """Periodic [0, 2 pi)^3, n^3 hexahedra, Taylor-Green vortex at Mach 1.25."""
    L = 2 * np.pi
    mesh = hex_3d(n, n, n, hi=(L, L, L), periodic=True, name=f"hex{n}")
    st = build_stencils_periodic_hex(mesh, (n, n, n), r) if n > 16 else build_stencils(mesh, r)
    pert = fields.tgv_perturbation(seed=1) if perturb else None
    exact = lambda p: fields.prim_to_cons(fields.tgv_prim(p, perturb=pert))
    U = fields.cell_average(mesh, exact, nq=max(3, (r + 3) // 2 + 1))
    return Workload(f"tgv_hex{n}_r{r}", mesh, st, U, Params(order_r=r, riemann=0), exact)


def vortex_2d(n=16, r=2) -> Workload:
    """The isentropic vortex of Section 3.1 on a periodic 10 x 10 square, triangles."""
    mk = lambda: quad_tri_2d(n, n, hi=(10.0, 10.0), split=np.ones((n, n), bool), periodic=True,
                             name=f"vortex{n}")
    mesh, st = mesh_and_stencils(f"vortex{n}_r{r}", mk, r)
    U = fields.cell_average(mesh, fields.isentropic_vortex_2d, nq=r + 4)
    return Workload(f"vortex{n}_r{r}", mesh, st, U, Params(order_r=r, lambda1_prime=1e4))


CONFIGS = {
    "c1": lambda: c1_density_jump(32, 2),
    "c2": lambda: c2_riemann(256, 3),
    "c3": lambda: tgv_hex(64, 4),
    "c5": lambda: tgv_hex(64, 2),
}


# Mixed-mesh sizes: (nx, ny, nz, core x-range, prism layers).  "full" is the
# ~1M-cell shock-vortex workload; the smaller ones have the same layout.
C4_SIZES = {"small": (24, 8, 8, (8, 16), 2), "medium": (60, 20, 20, (24, 36), 3),
            "full": (160, 56, 56, (64, 96), 8)}


def c4_mixed(size="small", r=3, workers=1, cell_order="lattice") -> Workload:
    """3D Euler on the mixed tetrahedron / prism / pyramid / hexahedron box of
    ``mixed_box`` (tetrahedral core with a prism layer on the wall z = 0,
    pyramid-and-tetrahedron transition columns, hexahedral far field): a
    Mach-3 normal shock in the middle of the core and three Gaussian vortices,
    HLLC, r = 3."""
    nx, ny, nz, core, kb = C4_SIZES[size]
    h = 1.0 / ny
    length = nx * h
    x_shock = 0.5 * (core[0] + core[1]) * h + 0.37 * h   # inside a cube layer, not on a lattice plane
    tag = "" if cell_order == "lattice" else f"_{cell_order}"
    mesh, st = mesh_and_stencils(f"c4_{size}{tag}_r{r}",
                                 lambda: mixed_box(nx, ny, nz, core=core, prism_layers=kb, jitter=0.2, seed=0,
                                                   cell_order=cell_order),
                                 r, workers=workers)
    upath = _cache_path(f"c4_{size}{tag}_field")
    if upath and os.path.exists(upath):
        U = np.load(upath)["U"]
    else:
        U = fields.cell_average(mesh, lambda p: fields.prim_to_cons(fields.shock_vortices_prim(p, length, x_shock)),
                                nq=4, workers=workers)
        if upath:
            np.savez(upath, U=U)
    return Workload(f"c4_mixed_{size}_r{r}", mesh, st, U, Params(order_r=r, riemann=0))
