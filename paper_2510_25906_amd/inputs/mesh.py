"""Seeded synthetic mixed-element meshes.

The paper's solver works on unstructured meshes built from triangles and
quadrilaterals in 2D and tetrahedra, pyramids, prisms and hexahedra in 3D
(Section 2, the paragraph before Eq. EulerEquationsDetails).  No mesh from the
paper is available, so this module generates meshes of the same element
families and sizes.  It holds no arithmetic of the reconstruction method:
it only lays out vertices, cells and faces.

Conventions (shared by every consumer of a ``Mesh``):

* local vertex order per type: TRI (0,1,2) counter-clockwise; QUAD (0,1,2,3)
  counter-clockwise; TET positively oriented; PYR base quad (0..3) seen
  counter-clockwise from the apex side, apex 4; PRISM bottom (0,1,2), top
  (3,4,5); HEX bottom (0..3), top (4..7) above them.
* ``face_cells[f] = (left, right)``; ``right == -1`` marks a boundary face.
  ``face_vtx`` lists the face's vertices oriented so that the normal given by
  the right-hand rule points out of the left cell.
* ``face_shift[f]`` is the periodic image of the right cell: adding
  ``face_shift[f] * period`` to the right cell's coordinates places it
  next to the left cell.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

TRI, QUAD, TET, PYR, PRISM, HEX = 0, 1, 2, 3, 4, 5
TYPE_NAMES = {TRI: "tri", QUAD: "quad", TET: "tet", PYR: "pyr", PRISM: "prism", HEX: "hex"}
TYPE_DIM = {TRI: 2, QUAD: 2, TET: 3, PYR: 3, PRISM: 3, HEX: 3}
TYPE_NVTX = {TRI: 3, QUAD: 4, TET: 4, PYR: 5, PRISM: 6, HEX: 8}

# Outward-oriented local faces of each element type.
CELL_FACES = {
    TRI: [(0, 1), (1, 2), (2, 0)],
    QUAD: [(0, 1), (1, 2), (2, 3), (3, 0)],
    TET: [(0, 2, 1), (0, 1, 3), (1, 2, 3), (0, 3, 2)],
    PYR: [(0, 3, 2, 1), (0, 1, 4), (1, 2, 4), (2, 3, 4), (3, 0, 4)],
    PRISM: [(0, 2, 1), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (2, 0, 3, 5)],
    HEX: [(0, 3, 2, 1), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)],
}


@dataclass
class Mesh:
    dim: int
    vertices: np.ndarray          # float64 [nv, dim]
    cell_type: np.ndarray         # int8 [N]
    cell_vtx_off: np.ndarray      # int32 [N+1]
    cell_vtx: np.ndarray          # int32 [...]
    face_cells: np.ndarray        # int32 [nf, 2]
    face_vtx_off: np.ndarray      # int32 [nf+1]
    face_vtx: np.ndarray          # int32 [...]
    face_shift: np.ndarray        # int8 [nf, dim]
    period: Optional[np.ndarray]  # float64 [dim] or None
    name: str = ""
    # derived cell->face incidence, CSR, ordered by face id
    cell_face_off: np.ndarray = field(default=None, repr=False)
    cell_face: np.ndarray = field(default=None, repr=False)
    cell_face_side: np.ndarray = field(default=None, repr=False)

    @property
    def n_cells(self) -> int:
        return int(self.cell_type.shape[0])

    @property
    def n_faces(self) -> int:
        return int(self.face_cells.shape[0])

    def cell_vertices(self, c: int) -> np.ndarray:
        return self.cell_vtx[self.cell_vtx_off[c]:self.cell_vtx_off[c + 1]]

    def face_vertices(self, f: int) -> np.ndarray:
        return self.face_vtx[self.face_vtx_off[f]:self.face_vtx_off[f + 1]]

    def finalize(self) -> "Mesh":
        """Build the cell->face incidence lists (ordered by face id)."""
        nf = self.n_faces
        left = self.face_cells[:, 0].astype(np.int64)
        right = self.face_cells[:, 1].astype(np.int64)
        fid = np.arange(nf, dtype=np.int64)
        inner = right >= 0
        cells = np.concatenate([left, right[inner]])
        faces = np.concatenate([fid, fid[inner]])
        sides = np.concatenate([np.zeros(nf, np.int8), np.ones(int(inner.sum()), np.int8)])
        order = np.lexsort((faces, cells))
        cells, faces, sides = cells[order], faces[order], sides[order]
        off = np.zeros(self.n_cells + 1, np.int64)
        np.add.at(off, cells + 1, 1)
        self.cell_face_off = np.cumsum(off).astype(np.int32)
        self.cell_face = faces.astype(np.int32)
        self.cell_face_side = sides
        return self

    def face_neighbours(self):
        """Per cell: list of (neighbour cell, image shift of the neighbour) over faces."""
        out_c = []
        out_s = []
        for c in range(self.n_cells):
            a, b = self.cell_face_off[c], self.cell_face_off[c + 1]
            cs, ss = [], []
            for f, side in zip(self.cell_face[a:b], self.cell_face_side[a:b]):
                l, r = self.face_cells[f]
                if r < 0:
                    continue
                if side == 0:
                    cs.append(r)
                    ss.append(self.face_shift[f].astype(np.int64))
                else:
                    cs.append(l)
                    ss.append(-self.face_shift[f].astype(np.int64))
            out_c.append(cs)
            out_s.append(ss)
        return out_c, out_s


def _build_faces(dim, vertices, cell_type, cell_vtx_off, cell_vtx, canon, period):
    """Match the local faces of all cells into global faces.

    ``canon`` maps every vertex to a canonical id; two local faces whose sorted
    canonical ids agree are the same face (periodic identification happens by
    giving periodic copies of a vertex the same canonical id).
    """
    n = cell_type.shape[0]
    loc_cell, loc_idx, loc_vtx = [], [], []
    for t, faces in CELL_FACES.items():
        cells_t = np.nonzero(cell_type == t)[0]
        if cells_t.size == 0:
            continue
        nv = TYPE_NVTX[t]
        cv = np.stack([cell_vtx[cell_vtx_off[cells_t] + k] for k in range(nv)], axis=1)
        for li, fv in enumerate(faces):
            vv = cv[:, list(fv)]
            pad = np.full((cells_t.size, 4), -1, np.int64)
            pad[:, :len(fv)] = vv
            loc_cell.append(cells_t)
            loc_idx.append(np.full(cells_t.size, li))
            loc_vtx.append(pad)
    loc_cell = np.concatenate(loc_cell)
    loc_idx = np.concatenate(loc_idx)
    loc_vtx = np.concatenate(loc_vtx)
    # canonical sort of the vertex keys
    key = np.where(loc_vtx >= 0, canon[np.maximum(loc_vtx, 0)], np.iinfo(np.int64).max)
    key = np.sort(key, axis=1)
    # order local faces by (cell, local index) so that face ids follow the owner
    base = np.lexsort((loc_idx, loc_cell))
    loc_cell, loc_idx, loc_vtx, key = loc_cell[base], loc_idx[base], loc_vtx[base], key[base]
    order = np.lexsort((np.arange(key.shape[0]),) + tuple(key[:, k] for k in range(3, -1, -1)))
    ks = key[order]
    same = np.all(ks[1:] == ks[:-1], axis=1)
    # every key occurs once (boundary) or twice (interior)
    first = np.ones(ks.shape[0], bool)
    first[1:] = ~same
    grp = np.cumsum(first) - 1
    counts = np.bincount(grp)
    if counts.max() > 2:
        raise ValueError("non-manifold mesh: a face is shared by more than two cells")
    n_face = counts.size
    left_loc = np.full(n_face, -1, np.int64)
    right_loc = np.full(n_face, -1, np.int64)
    starts = np.nonzero(first)[0]
    left_loc[:] = order[starts]
    two = counts == 2
    right_loc[two] = order[starts[two] + 1]
    # face ids ordered by the owner's (cell, local face)
    fo = np.argsort(left_loc, kind="stable")
    left_loc, right_loc = left_loc[fo], right_loc[fo]
    face_cells = np.stack([loc_cell[left_loc],
                           np.where(right_loc >= 0, loc_cell[np.maximum(right_loc, 0)], -1)], 1)
    fvl = loc_vtx[left_loc]
    nfv = (fvl >= 0).sum(1)
    face_vtx_off = np.zeros(n_face + 1, np.int64)
    face_vtx_off[1:] = np.cumsum(nfv)
    face_vtx = fvl[fvl >= 0]
    shift = np.zeros((n_face, dim), np.int8)
    if period is not None:
        inner = right_loc >= 0
        fr = loc_vtx[right_loc[inner]]
        # centroid of the face vertices seen from each side
        def vmean(vv):
            m = vv >= 0
            s = np.zeros((vv.shape[0], dim))
            for k in range(4):
                s += np.where(m[:, k:k + 1], vertices[np.maximum(vv[:, k], 0)], 0.0)
            return s / m.sum(1, keepdims=True)
        cl = vmean(fvl[inner])
        cr = vmean(fr)
        sh = np.rint((cl - cr) / period).astype(np.int8)
        shift[inner] = sh
    return (face_cells.astype(np.int32), face_vtx_off.astype(np.int32),
            face_vtx.astype(np.int32), shift)


def _assemble(dim, vertices, cell_type, cells_vtx_list, canon, period, name):
    cell_type = np.asarray(cell_type, np.int8)
    counts = np.array([len(c) for c in cells_vtx_list], np.int64) if isinstance(cells_vtx_list, list) \
        else np.full(cell_type.shape[0], cells_vtx_list.shape[1])
    off = np.zeros(cell_type.shape[0] + 1, np.int64)
    off[1:] = np.cumsum(counts)
    flat = np.concatenate([np.asarray(c) for c in cells_vtx_list]) if isinstance(cells_vtx_list, list) \
        else np.asarray(cells_vtx_list).reshape(-1)
    fc, fo, fv, fs = _build_faces(dim, vertices, cell_type, off, flat.astype(np.int64), canon, period)
    m = Mesh(dim=dim, vertices=np.ascontiguousarray(vertices, np.float64), cell_type=cell_type,
             cell_vtx_off=off.astype(np.int32), cell_vtx=flat.astype(np.int32), face_cells=fc,
             face_vtx_off=fo, face_vtx=fv, face_shift=fs,
             period=None if period is None else np.asarray(period, np.float64), name=name)
    return m.finalize()


def quad_tri_2d(nx, ny, lo=(0.0, 0.0), hi=(1.0, 1.0), split=None, periodic=False, name=""):
    """Structured 2D mesh of quads, each optionally split into two triangles.

    ``split`` is a boolean array [ny, nx] (row j, column i); a split quad
    becomes the triangles (v00, v10, v11) and (v00, v11, v01), i.e. it is cut
    along the diagonal from (x_i, y_j) to (x_{i+1}, y_{j+1}).  Cells are
    numbered row-major over the quads, a split quad contributing two
    consecutive cells.
    """
    if split is None:
        split = np.zeros((ny, nx), bool)
    xs = np.linspace(lo[0], hi[0], nx + 1)
    ys = np.linspace(lo[1], hi[1], ny + 1)
    X, Y = np.meshgrid(xs, ys)  # [ny+1, nx+1]
    vertices = np.stack([X.ravel(), Y.ravel()], 1)
    vid = lambda i, j: j * (nx + 1) + i
    if periodic:
        I, J = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1))
        canon = ((J % ny) * nx + (I % nx)).ravel().astype(np.int64)
        period = np.array([hi[0] - lo[0], hi[1] - lo[1]])
    else:
        canon = np.arange(vertices.shape[0], dtype=np.int64)
        period = None
    types, cells = [], []
    for j in range(ny):
        for i in range(nx):
            v00, v10, v11, v01 = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            if split[j, i]:
                types += [TRI, TRI]
                cells += [(v00, v10, v11), (v00, v11, v01)]
            else:
                types.append(QUAD)
                cells.append((v00, v10, v11, v01))
    return _assemble(2, vertices, types, cells, canon, period, name)


def hex_3d(nx, ny, nz, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), periodic=False, name=""):
    """Structured hexahedral mesh, cells numbered x-fastest."""
    xs = np.linspace(lo[0], hi[0], nx + 1)
    ys = np.linspace(lo[1], hi[1], ny + 1)
    zs = np.linspace(lo[2], hi[2], nz + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    vertices = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    vid = lambda i, j, k: (k * (ny + 1) + j) * (nx + 1) + i
    cells = np.stack([vid(I, J, K), vid(I + 1, J, K), vid(I + 1, J + 1, K), vid(I, J + 1, K),
                      vid(I, J, K + 1), vid(I + 1, J, K + 1), vid(I + 1, J + 1, K + 1),
                      vid(I, J + 1, K + 1)], 1)
    if periodic:
        Kv, Jv, Iv = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
        canon = (((Kv % nz) * ny + (Jv % ny)) * nx + (Iv % nx)).ravel().astype(np.int64)
        period = np.array([hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]])
    else:
        canon = np.arange(vertices.shape[0], dtype=np.int64)
        period = None
    types = np.full(cells.shape[0], HEX, np.int8)
    return _assemble(3, vertices, types, cells, canon, period, name)


def jitter_vertices(mesh: Mesh, amplitude: float, seed: int) -> Mesh:
    """Displace interior vertices of a simplex mesh by a seeded random offset.

    Only meaningful for meshes whose faces stay planar under arbitrary vertex
    motion (triangles / edges in 2D, tetrahedra in 3D).
    """
    rng = np.random.default_rng(seed)
    v = mesh.vertices.copy()
    lo, hi = v.min(0), v.max(0)
    interior = np.all((v > lo + 1e-12) & (v < hi - 1e-12), axis=1)
    v[interior] += amplitude * rng.uniform(-1, 1, size=(int(interior.sum()), mesh.dim))
    mesh.vertices = v
    return mesh


def simplex_decomposition(cell_type: int):
    """Local simplices that tile each element type (used to build geometry)."""
    return {
        TRI: [(0, 1, 2)],
        QUAD: [(0, 1, 2), (0, 2, 3)],
        TET: [(0, 1, 2, 3)],
        PYR: [(0, 1, 2, 4), (0, 2, 3, 4)],
        PRISM: [(0, 1, 2, 3), (1, 2, 3, 4), (2, 3, 4, 5)],
        HEX: [(0, 1, 2, 6), (0, 3, 2, 6), (0, 3, 7, 6), (0, 4, 7, 6), (0, 4, 5, 6), (0, 1, 5, 6)],
    }[cell_type]


# The six tetrahedra of a cube along its main diagonal (local cube vertex
# numbering as for HEX): every tetrahedron is a monotone path 0 -> a -> b -> 6.
_KUHN = [(0, 1, 2, 6), (0, 3, 2, 6), (0, 3, 7, 6), (0, 4, 7, 6), (0, 4, 5, 6), (0, 1, 5, 6)]


def tet_box(nx, ny, nz, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), jitter=0.0, seed=0, name=""):
    """Conforming tetrahedral mesh of a box: every cube cut into six tetrahedra
    along its main diagonal; interior vertices optionally jittered (seeded)."""
    xs = np.linspace(lo[0], hi[0], nx + 1)
    ys = np.linspace(lo[1], hi[1], ny + 1)
    zs = np.linspace(lo[2], hi[2], nz + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    vertices = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    if jitter > 0:
        rng = np.random.default_rng(seed)
        h = np.array([(hi[0] - lo[0]) / nx, (hi[1] - lo[1]) / ny, (hi[2] - lo[2]) / nz])
        Kv, Jv, Iv = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
        inner = ((Iv > 0) & (Iv < nx) & (Jv > 0) & (Jv < ny) & (Kv > 0) & (Kv < nz)).ravel()
        vertices[inner] += jitter * h * rng.uniform(-1, 1, size=(int(inner.sum()), 3))
    K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    vid = lambda i, j, k: (k * (ny + 1) + j) * (nx + 1) + i
    cube = np.stack([vid(I, J, K), vid(I + 1, J, K), vid(I + 1, J + 1, K), vid(I, J + 1, K),
                     vid(I, J, K + 1), vid(I + 1, J, K + 1), vid(I + 1, J + 1, K + 1),
                     vid(I, J + 1, K + 1)], 1)
    tets = np.concatenate([cube[:, list(t)] for t in _KUHN], 0)
    order = np.argsort(np.tile(np.arange(cube.shape[0]), len(_KUHN)), kind="stable")
    tets = tets[order]
    P = vertices[tets]
    det = np.linalg.det(P[:, 1:] - P[:, :1])
    neg = det < 0
    tets[neg, 1], tets[neg, 2] = tets[neg, 2].copy(), tets[neg, 1].copy()
    canon = np.arange(vertices.shape[0], dtype=np.int64)
    return _assemble(3, vertices, np.full(tets.shape[0], TET, np.int8), tets, canon, None, name)


# Hex faces in CELL_FACES[HEX] order and the lattice offset of the cube across each.
_HEX_FACE_NB = [(0, 0, -1), (0, 0, 1), (0, -1, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0)]
_HEX_CORNER = np.array([(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)])
CUBE_HEX, CUBE_PRISM, CUBE_TET, CUBE_TRANSITION = 0, 1, 2, 3


def _morton3(i, j, k):
    """Morton (Z-order) key of integer lattice coordinates below 2^10."""
    key = np.zeros(np.shape(i), np.int64)
    for b in range(10):
        key |= (((i >> b) & 1) << (3 * b)) | (((j >> b) & 1) << (3 * b + 1)) | (((k >> b) & 1) << (3 * b + 2))
    return key


def mixed_box(nx, ny, nz, core=None, prism_layers=2, jitter=0.2, seed=0, h=None, name="", cell_order="lattice"):
    """Conforming mixed tetrahedron / prism / pyramid / hexahedron mesh of a box.

    A lattice of nx x ny x nz cubes of edge h (default 1/ny) is split by
    region: in the core x-range ``core = (i1, i2)`` the bottom
    ``prism_layers`` cube layers become two prisms each (a boundary layer on
    the wall z = 0) and the cubes above them six Kuhn tetrahedra each, with the
    interior core vertices jittered (seeded); the cube columns just outside
    the core (i1 - 1 and i2), above the prism layers, are transition cubes:
    split around an added centre vertex into a pyramid on every face shared
    with a hexahedron (or on the boundary) and two tetrahedra on every other
    face; every other cube is a hexahedron.  Every split quad face is cut along
    the diagonal from its lowest to its highest lattice corner, which is the
    cut the Kuhn tetrahedra and the prism caps make, so all faces match.
    Cells are numbered cube by cube, the cubes in lattice order (x fastest)
    or, with ``cell_order="morton"``, along a Morton (Z-order) curve, which
    keeps cells that are close in space close in memory in every direction.
    """
    if cell_order not in ("lattice", "morton"):
        raise ValueError("cell_order must be 'lattice' or 'morton'")
    h = 1.0 / ny if h is None else h
    i1, i2 = core if core is not None else (nx // 3, nx - nx // 3)
    kb = prism_layers
    if not (1 <= i1 < i2 <= nx - 1 and 0 <= kb < nz):
        raise ValueError("core must leave a transition column on both sides")
    nvl = (nx + 1) * (ny + 1) * (nz + 1)
    vid = lambda i, j, k: (k * (ny + 1) + j) * (nx + 1) + i
    Kv, Jv, Iv = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    verts = np.stack([Iv.ravel(), Jv.ravel(), Kv.ravel()], 1).astype(np.float64) * h
    if jitter > 0:
        inner = ((Iv > i1) & (Iv < i2) & (Jv > 0) & (Jv < ny) & (Kv > kb) & (Kv < nz)).ravel()
        rng = np.random.default_rng(seed)
        verts[inner] += jitter * h * rng.uniform(-1, 1, size=(int(inner.sum()), 3))
    K3, J3, I3 = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    kind = np.full((nz, ny, nx), CUBE_HEX, np.int8)
    in_core = (I3 >= i1) & (I3 < i2)
    kind[in_core & (K3 < kb)] = CUBE_PRISM
    kind[in_core & (K3 >= kb)] = CUBE_TET
    kind[((I3 == i1 - 1) | (I3 == i2)) & (K3 >= kb)] = CUBE_TRANSITION
    flat_kind = kind.ravel()
    I, J, Kk = I3.ravel(), J3.ravel(), K3.ravel()
    cube = np.stack([vid(I + a, J + b, Kk + c) for a, b, c in _HEX_CORNER], 1)
    cells, ctype, owner = [], [], []

    def add(kind_mask, local, t):
        idx = np.nonzero(kind_mask)[0]
        for loc in local:
            cells.append(cube[idx][:, list(loc)])
            ctype.append(np.full(idx.size, t, np.int8))
            owner.append(idx)

    add(flat_kind == CUBE_HEX, [tuple(range(8))], HEX)
    add(flat_kind == CUBE_PRISM, [(0, 1, 2, 4, 5, 6), (0, 2, 3, 4, 6, 7)], PRISM)
    add(flat_kind == CUBE_TET, _KUHN, TET)
    # transition cubes: centre vertex, pyramids toward hexahedra, tetrahedra elsewhere
    tr = np.nonzero(flat_kind == CUBE_TRANSITION)[0]
    centre = nvl + np.arange(tr.size)
    verts = np.concatenate([verts, verts[cube[tr]].mean(1)], 0)
    pyr, tet, pyr_own, tet_own = [], [], [], []
    for n_, q in enumerate(tr):
        i, j, k = int(I[q]), int(J[q]), int(Kk[q])
        for fl, (di, dj, dk) in zip(CELL_FACES[HEX], _HEX_FACE_NB):
            a, b, c = i + di, j + dj, k + dk
            outside = not (0 <= a < nx and 0 <= b < ny and 0 <= c < nz)
            quad = outside or kind[c, b, a] in (CUBE_HEX, CUBE_PRISM)
            loop = [int(cube[q, v]) for v in fl]
            if quad:
                pyr.append(loop[::-1] + [int(centre[n_])])
                pyr_own.append(q)
            else:
                corner = [tuple(_HEX_CORNER[v]) for v in fl]
                lo_ = min(range(4), key=lambda t: sum(corner[t]))
                la, lb, lc, ld = (loop[(lo_ + t) % 4] for t in range(4))
                for tri in ((la, lb, lc), (la, lc, ld)):
                    tet.append(list(tri) + [int(centre[n_])])
                    tet_own.append(q)
    if pyr:
        cells.append(np.array(pyr, np.int64))
        ctype.append(np.full(len(pyr), PYR, np.int8))
        owner.append(np.array(pyr_own))
    if tet:
        cells.append(np.array(tet, np.int64))
        ctype.append(np.full(len(tet), TET, np.int8))
        owner.append(np.array(tet_own))
    # positive orientation of every tetrahedron
    for c_, t_ in zip(cells, ctype):
        if t_.size and t_[0] == TET:
            P = verts[c_]
            neg = np.linalg.det(P[:, 1:] - P[:, :1]) < 0
            c_[neg, 1], c_[neg, 2] = c_[neg, 2].copy(), c_[neg, 1].copy()
    # cube-major order, cells padded to 8 vertices (-1) and then flattened
    own = np.concatenate(owner)
    if cell_order == "morton":
        own = _morton3(I[own], J[own], Kk[own])
    order = np.argsort(own, kind="stable")
    types = np.concatenate(ctype)[order]
    padded = np.concatenate([np.pad(c_, ((0, 0), (0, 8 - c_.shape[1])), constant_values=-1) for c_ in cells])[order]
    counts = (padded >= 0).sum(1)
    off = np.zeros(types.size + 1, np.int64)
    off[1:] = np.cumsum(counts)
    flat = padded[padded >= 0].astype(np.int64)
    canon = np.arange(verts.shape[0], dtype=np.int64)
    fc, fo, fv, fs = _build_faces(3, verts, types, off, flat, canon, None)
    m = Mesh(dim=3, vertices=np.ascontiguousarray(verts, np.float64), cell_type=types,
             cell_vtx_off=off.astype(np.int32), cell_vtx=flat.astype(np.int32), face_cells=fc,
             face_vtx_off=fo, face_vtx=fv, face_shift=fs, period=None,
             name=name or f"mixed{nx}x{ny}x{nz}").finalize()
    # every unmatched face must lie on the box boundary (conformity check)
    bnd = np.nonzero(m.face_cells[:, 1] < 0)[0]
    first = m.vertices[m.face_vtx[m.face_vtx_off[bnd]]]
    third = m.vertices[m.face_vtx[m.face_vtx_off[bnd] + 2]]
    ext = np.array([nx, ny, nz]) * h
    tol = 1e-9 * h
    # a boundary face has all its vertices on one box plane; testing two of them suffices here
    on = np.any(((np.abs(first) < tol) & (np.abs(third) < tol)) |
                ((np.abs(first - ext) < tol) & (np.abs(third - ext) < tol)), axis=1)
    if not np.all(on):
        raise AssertionError("non-conforming mixed mesh: interior faces left unmatched")
    return m
