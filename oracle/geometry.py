"""Oracle mesh geometry (test infrastructure only).

Volumes and centroids come from a simplex tiling of every element, the
tiling the paper uses for reconstruction (Section 2.1, the paragraph before
Eq. AVGVariables2).  This module uses its own tiling tables (quads cut along
the (1,3) diagonal, hexahedra into five tetrahedra), which give exact results
for the planar-faced elements generated here.  Face quadrature follows
Section 2 (paragraph after Eq. EulerEquationsDetails); see ``quadrature``.
"""
from __future__ import annotations

from dataclasses import dataclass
from math import factorial

import numpy as np

from .quadrature import gauss_legendre_01, n_line_points, triangle_rule

TRI, QUAD, TET, PYR, PRISM, HEX = 0, 1, 2, 3, 4, 5
NVTX = {TRI: 3, QUAD: 4, TET: 4, PYR: 5, PRISM: 6, HEX: 8}
TILING = {
    TRI: [(0, 1, 2)],
    QUAD: [(0, 1, 3), (1, 2, 3)],
    TET: [(0, 1, 2, 3)],
    PYR: [(0, 1, 3, 4), (1, 2, 3, 4)],
    PRISM: [(0, 1, 2, 5), (0, 1, 5, 4), (0, 4, 5, 3)],
    HEX: [(0, 1, 3, 4), (2, 1, 3, 6), (5, 1, 4, 6), (7, 3, 4, 6), (1, 3, 4, 6)],
}


def cell_simplices(mesh, cells):
    """Simplex vertex coordinates of the given cells.

    Returns (S [n_simplices, d+1, d], owner [n_simplices]) where owner indexes
    into ``cells``.
    """
    cells = np.asarray(cells)
    S_all, own_all = [], []
    types = mesh.cell_type[cells]
    for t in np.unique(types):
        sel = np.nonzero(types == t)[0]
        cc = cells[sel]
        cv = np.stack([mesh.cell_vtx[mesh.cell_vtx_off[cc] + k] for k in range(NVTX[int(t)])], 1)
        X = mesh.vertices[cv]
        for simp in TILING[int(t)]:
            S_all.append(X[:, list(simp)])
            own_all.append(sel)
    S = np.concatenate(S_all, 0)
    own = np.concatenate(own_all, 0)
    order = np.argsort(own, kind="stable")
    return S[order], own[order]


@dataclass
class Geometry:
    vol: np.ndarray        # [N]
    cen: np.ndarray        # [N, d]
    h: np.ndarray          # [N] characteristic size |V|^(1/d)
    normal: np.ndarray     # [nf, d] unit normal, outward from the left cell
    area: np.ndarray       # [nf]
    gp_off: np.ndarray     # [nf+1]
    gp_x: np.ndarray       # [NGPT, d] Gauss points (left cell's coordinates)
    gp_wS: np.ndarray      # [NGPT] weight x surface Jacobian (sums to the face area)
    # per-cell Gauss point lists, padded to the largest count
    c_ngp: np.ndarray      # [N]
    c_gidx: np.ndarray     # [N, NGPC] global Gauss point index
    c_side: np.ndarray     # [N, NGPC] 0 owner / 1 neighbour
    c_x: np.ndarray        # [N, NGPC, d] Gauss point in the cell's own image
    c_face: np.ndarray     # [N, NGPC] face of each Gauss point

    @property
    def n_gp(self) -> int:
        return int(self.gp_off[-1])


def compute_geometry(mesh, r: int) -> Geometry:
    d = mesh.dim
    N = mesh.n_cells
    S, own = cell_simplices(mesh, np.arange(N))
    v = np.abs(np.linalg.det(S[:, 1:] - S[:, :1])) / factorial(d)
    vol = np.bincount(own, weights=v, minlength=N)
    cen = np.stack([np.bincount(own, weights=v * S[:, :, j].mean(1), minlength=N) for j in range(d)], 1)
    cen /= vol[:, None]
    h = vol ** (1.0 / d)

    nf = mesh.n_faces
    nfv = np.diff(mesh.face_vtx_off)
    normal = np.zeros((nf, d))
    area = np.zeros(nf)
    counts = np.zeros(nf, np.int64)
    pts_by_face = [None] * 0
    gp_list_x, gp_list_w, gp_face = [], [], []
    line_x, line_w = gauss_legendre_01(n_line_points(r))
    for k in np.unique(nfv):
        fs = np.nonzero(nfv == k)[0]
        V = np.stack([mesh.vertices[mesh.face_vtx[mesh.face_vtx_off[fs] + j]] for j in range(k)], 1)
        if d == 2:
            t = V[:, 1] - V[:, 0]
            L = np.linalg.norm(t, axis=1)
            normal[fs] = np.stack([t[:, 1], -t[:, 0]], 1) / L[:, None]
            area[fs] = L
            X = V[:, None, 0] + line_x[None, :, None] * t[:, None, :]
            W = line_w[None, :] * L[:, None]
        elif k == 3:
            av = 0.5 * np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0])
            A = np.linalg.norm(av, axis=1)
            normal[fs] = av / A[:, None]
            area[fs] = A
            bc, w = triangle_rule(r)
            X = np.einsum("ql,fld->fqd", bc, V)
            W = w[None, :] * A[:, None]
        elif k == 4:
            av = 0.5 * (np.cross(V[:, 0], V[:, 1]) + np.cross(V[:, 1], V[:, 2]) +
                        np.cross(V[:, 2], V[:, 3]) + np.cross(V[:, 3], V[:, 0]))
            A = np.linalg.norm(av, axis=1)
            normal[fs] = av / A[:, None]
            area[fs] = A
            s, t = [a.ravel() for a in np.meshgrid(line_x, line_x, indexing="ij")]
            ws = np.outer(line_w, line_w).ravel()
            Nsh = np.stack([(1 - s) * (1 - t), s * (1 - t), s * t, (1 - s) * t], 1)
            dNs = np.stack([-(1 - t), (1 - t), t, -t], 1)
            dNt = np.stack([-(1 - s), -s, s, (1 - s)], 1)
            X = np.einsum("ql,fld->fqd", Nsh, V)
            xs = np.einsum("ql,fld->fqd", dNs, V)
            xt = np.einsum("ql,fld->fqd", dNt, V)
            W = ws[None, :] * np.linalg.norm(np.cross(xs, xt), axis=2)
        else:
            raise ValueError("unsupported face")
        counts[fs] = X.shape[1]
        gp_list_x.append((fs, X))
        gp_list_w.append((fs, W))
    gp_off = np.zeros(nf + 1, np.int64)
    gp_off[1:] = np.cumsum(counts)
    gp_x = np.zeros((gp_off[-1], d))
    gp_wS = np.zeros(gp_off[-1])
    for (fs, X), (_, W) in zip(gp_list_x, gp_list_w):
        idx = gp_off[fs][:, None] + np.arange(X.shape[1])[None, :]
        gp_x[idx] = X
        gp_wS[idx] = W

    # per-cell Gauss point lists in cell-face order
    per_cell = np.zeros(N, np.int64)
    cf_cell = np.repeat(np.arange(N), np.diff(mesh.cell_face_off))
    np.add.at(per_cell, cf_cell, counts[mesh.cell_face])
    NGPC = int(per_cell.max())
    c_gidx = np.full((N, NGPC), -1, np.int64)
    c_side = np.zeros((N, NGPC), np.int64)
    c_face = np.full((N, NGPC), -1, np.int64)
    c_x = np.zeros((N, NGPC, d))
    period = mesh.period if mesh.period is not None else np.zeros(d)
    fill = np.zeros(N, np.int64)
    for j in range(int(np.diff(mesh.cell_face_off).max())):
        cells = np.nonzero(np.diff(mesh.cell_face_off) > j)[0]
        f = mesh.cell_face[mesh.cell_face_off[cells] + j]
        side = mesh.cell_face_side[mesh.cell_face_off[cells] + j].astype(np.int64)
        for a in range(int(counts[f].max())):
            ok = counts[f] > a
            cc, ff, ss = cells[ok], f[ok], side[ok]
            g = gp_off[ff] + a
            slot = fill[cc]
            c_gidx[cc, slot] = g
            c_side[cc, slot] = ss
            c_face[cc, slot] = ff
            c_x[cc, slot] = gp_x[g] - (ss[:, None] == 1) * mesh.face_shift[ff].astype(np.float64) * period
            fill[cc] += 1
    return Geometry(vol=vol, cen=cen, h=h, normal=normal, area=area, gp_off=gp_off, gp_x=gp_x,
                    gp_wS=gp_wS, c_ngp=per_cell, c_gidx=c_gidx, c_side=c_side, c_x=c_x, c_face=c_face)
