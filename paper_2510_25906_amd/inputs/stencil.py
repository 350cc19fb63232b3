"""Seeded stencil construction: central, directional and MUSCL stencils.

The paper builds its central stencil with the stencil-based compact (SBC)
algorithm, which it only cites (Section 2.1, after the definition of the
central stencil); its directional stencils are lower-order stencils contained
in the central one (Section 2.3), and neither construction is given.  These
builders follow fixed rules instead (listed in the design notes):

* central: grow face-neighbour layers over periodic images until at least
  ``2M`` candidates are known, force-include every face neighbour, then take
  the ``M`` nearest by centroid distance; ties break on the quantised relative
  offset, then on the cell id, so uniform meshes get translation-invariant
  stencils.  ``M = 2K`` where K is the number of non-constant unknowns of a
  degree-r polynomial in d dimensions (Section 2.1, definition of K(r, d)).
* directional: one per face; members are central-stencil cells whose centroid
  lies in the cone (sector in 2D) spanned from the cell centroid by the face,
  the face neighbour first, nearest first, filled from the half-space beyond
  the face and then from the rest of the central stencil up to ``2d``.
* MUSCL: the face neighbours, padded with the nearest central members up to
  ``d + 1`` cells.

Every stencil entry is a pair (cell id, periodic image shift); the image
shift multiplies the mesh period.
"""
from __future__ import annotations

from dataclasses import dataclass
from math import comb

import numpy as np

from . import pool
from .mesh import Mesh, simplex_decomposition, TYPE_NVTX, CELL_FACES


def n_unknowns(r: int, d: int) -> int:
    """Number of non-constant coefficients of a degree-r polynomial in d dims."""
    return comb(r + d, d) - 1


def nf_max(d: int) -> int:
    return 4 if d == 2 else 6


@dataclass
class Stencils:
    r: int
    M: int
    Md: int
    central: np.ndarray        # int32 [N, M]
    central_shift: np.ndarray  # int8 [N, M, d]
    dir: np.ndarray            # int32 [N, NFMAX, Md]
    dir_shift: np.ndarray      # int8 [N, NFMAX, Md, d]
    n_dir: np.ndarray          # int32 [N] number of directional stencils (= faces)
    muscl: np.ndarray          # int32 [N, NFMAX]
    muscl_shift: np.ndarray    # int8 [N, NFMAX, d]
    n_muscl: np.ndarray        # int32 [N]


def cell_centroids(mesh: Mesh):
    """Volume-weighted centroids and volumes from the simplex tiling."""
    d = mesh.dim
    N = mesh.n_cells
    cen = np.zeros((N, d))
    vol = np.zeros(N)
    for t in np.unique(mesh.cell_type):
        cells = np.nonzero(mesh.cell_type == t)[0]
        nv = TYPE_NVTX[int(t)]
        cv = np.stack([mesh.cell_vtx[mesh.cell_vtx_off[cells] + k] for k in range(nv)], 1)
        X = mesh.vertices[cv]  # [n, nv, d]
        acc_v = np.zeros(cells.size)
        acc_c = np.zeros((cells.size, d))
        for simp in simplex_decomposition(int(t)):
            P = X[:, list(simp)]
            J = P[:, 1:] - P[:, :1]
            v = np.abs(np.linalg.det(J)) / (2.0 if d == 2 else 6.0)
            acc_v += v
            acc_c += v[:, None] * P.mean(1)
        vol[cells] = acc_v
        cen[cells] = acc_c / acc_v[:, None]
    return cen, vol


def _adjacency(mesh: Mesh):
    fc = mesh.face_cells.astype(np.int64)
    inner = fc[:, 1] >= 0
    l, r = fc[inner, 0], fc[inner, 1]
    sh = mesh.face_shift[inner].astype(np.int64)
    src = np.concatenate([l, r])
    dst = np.concatenate([r, l])
    ssh = np.concatenate([sh, -sh])
    order = np.lexsort((dst, src))
    src, dst, ssh = src[order], dst[order], ssh[order]
    off = np.zeros(mesh.n_cells + 1, np.int64)
    np.add.at(off, src + 1, 1)
    return np.cumsum(off), dst, ssh


_SB = 5  # bits per shift component


def _encode(s, c, sh, d):
    k = (s.astype(np.int64) << 22) | c.astype(np.int64)
    for j in range(d):
        k = (k << _SB) | ((sh[:, j] + (1 << (_SB - 1))) & ((1 << _SB) - 1))
    return k


def _decode(k, d):
    sh = np.zeros((k.shape[0], d), np.int64)
    for j in range(d - 1, -1, -1):
        sh[:, j] = (k & ((1 << _SB) - 1)) - (1 << (_SB - 1))
        k = k >> _SB
    c = k & ((1 << 22) - 1)
    s = k >> 22
    return s, c, sh


def _moment_block(item):
    from .fields import cell_quadrature
    mesh, r, cen = pool.SHARED
    cc = item
    d = mesh.dim
    pts, w = cell_quadrature(mesh, cc, r + 1)
    y = pts - cen[cc][:, None, :]
    vol = w.sum(1)
    ypow = [[np.ones_like(y[..., j])] for j in range(d)]
    for j in range(d):
        for _ in range(r):
            ypow[j].append(ypow[j][-1] * y[..., j])
    out = np.zeros((cc.size, len(_moment_exps(d, r))))
    for i, b in enumerate(_moment_exps(d, r)):
        term = w * ypow[0][b[0]]
        for j in range(1, d):
            term = term * ypow[j][b[j]]
        out[:, i] = term.sum(1) / vol
    return out


def _central_moments(mesh, r, cen, workers=1):
    """Per cell, the means of (x - x_c)^beta over the cell for |beta| <= r
    (quadrature exact for these degrees), in the order of ``_moment_exps``."""
    blocks = []
    for t in np.unique(mesh.cell_type):
        cells = np.nonzero(mesh.cell_type == t)[0]
        blocks += [cells[a:a + 32768] for a in range(0, cells.size, 32768)]
    parts = pool.pool_map(_moment_block, blocks, workers, (mesh, r, cen))
    mom = np.zeros((mesh.n_cells, len(_moment_exps(mesh.dim, r))))
    for cc, m in zip(blocks, parts):
        mom[cc] = m
    return mom


def _moment_exps(d, r):
    return [e for e in np.ndindex(*([r + 1] * d)) if sum(e) <= r]


def _member_rows(mom, src, mem, off, h, d, r):
    """Rows of the least-squares system in the source cell's frame: the mean of
    xi^alpha over each member minus its mean over the source cell, xi = (x -
    x_src) / h_src, |alpha| = 1..r, from the members' central moments."""
    bexps = _moment_exps(d, r)
    bidx = {b: i for i, b in enumerate(bexps)}
    exps = [e for e in bexps if sum(e) >= 1]
    hs = h[src]
    rows = np.zeros(src.shape + (len(exps),))
    for k, a in enumerate(exps):
        acc = np.zeros(src.shape)
        for b in np.ndindex(*[x + 1 for x in a]):
            coef = np.prod([comb(a[j], b[j]) for j in range(d)])
            term = coef * mom[mem, bidx[b]]
            for j in range(d):
                if a[j] - b[j]:
                    term = term * off[..., j] ** (a[j] - b[j])
            acc += term
        rows[..., k] = (acc - mom[src, bidx[a]]) / hs ** sum(a)
    return rows


# condition number of the least-squares rows above which a stencil is rebuilt
COND_MAX = 1e3


def _row_cond(V):
    sv = np.linalg.svd(V, compute_uv=False)
    return sv[..., 0] / np.maximum(sv[..., -1], 1e-300)


def _degenerate(take, s_all, c_all, off, h, d, r, N, M, mom):
    """Cells whose selected members separate the degree-r polynomials badly:
    the least-squares rows (member means of the monomials, from quadrature
    moments) are rank deficient or have a condition number above COND_MAX
    (one-sided stencils at walls, thin cell layers)."""
    order = np.argsort(s_all[take], kind="stable")
    t = take[order]
    V = _member_rows(mom, s_all[t].reshape(N, M), c_all[t].reshape(N, M), off[t].reshape(N, M, d), h, d, r)
    cond = np.zeros(N)
    for a in range(0, N, 65536):
        cond[a:a + 65536] = _row_cond(V[a:a + 65536])
    return cond > COND_MAX, cond


def _central_stencils(mesh, r, lo, hi, cen, h, period, adj_off, adj_dst, adj_sh, mom):
    """Central stencils (ids, periodic images) of the source cells lo..hi-1."""
    d = mesh.dim
    N = mesh.n_cells
    K = n_unknowns(r, d)
    M = 2 * K
    deg = np.diff(adj_off)
    n = hi - lo
    # ---- breadth-first growth over (cell, image) pairs ----------------------
    ids = np.arange(lo, hi, dtype=np.int64)
    visited = _encode(ids, ids, np.zeros((n, d), np.int64), d)
    layer_keys = [visited]
    layer_ids = [np.zeros(n, np.int64)]
    front_s, front_c, front_sh = ids, ids, np.zeros((n, d), np.int64)
    count = np.ones(n, np.int64)
    target = 2 * M + 1
    for layer in range(1, 64):
        need = count[front_s - lo] < target
        fs, fcc, fsh = front_s[need], front_c[need], front_sh[need]
        if fs.size == 0:
            break
        rep = deg[fcc]
        es = np.repeat(fs, rep)
        esh = np.repeat(fsh, rep, axis=0)
        starts = np.repeat(adj_off[fcc], rep)
        within = np.arange(es.size) - np.repeat(np.cumsum(rep) - rep, rep)
        eidx = starts + within
        ec = adj_dst[eidx]
        esh = esh + adj_sh[eidx]
        keys = np.unique(_encode(es, ec, esh, d))
        keys = keys[~np.isin(keys, visited, assume_unique=True)]
        if keys.size == 0:
            break
        visited = np.union1d(visited, keys)
        layer_keys.append(keys)
        layer_ids.append(np.full(keys.size, layer, np.int64))
        front_s, front_c, front_sh = _decode(keys, d)
        count = np.bincount(_decode(visited, d)[0] - lo, minlength=n)
    all_keys = np.concatenate(layer_keys)
    all_layer = np.concatenate(layer_ids)
    s_all, c_all, sh_all = _decode(all_keys, d)
    self_mask = (s_all == c_all) & np.all(sh_all == 0, axis=1)
    s_all, c_all, sh_all, hop = s_all[~self_mask], c_all[~self_mask], sh_all[~self_mask], all_layer[~self_mask]
    if np.any(np.bincount(s_all - lo, minlength=n) < M):
        raise ValueError("mesh too small for a central stencil of %d cells" % M)

    off = cen[c_all] + sh_all * period - cen[s_all]
    hs = h[s_all][:, None]
    qoff = np.rint(off / hs * 1e6).astype(np.int64)
    qd = np.rint((off ** 2).sum(1) / hs[:, 0] ** 2 * 1e8).astype(np.int64)
    # forced face neighbours
    src = np.repeat(np.arange(N), deg)
    fsel = (src >= lo) & (src < hi)
    fn_key = _encode(src[fsel], adj_dst[fsel], adj_sh[fsel], d)
    forced = np.isin(_encode(s_all, c_all, sh_all, d), fn_key)

    def select(primary):
        sort_keys = [c_all] + [qoff[:, j] for j in range(d - 1, -1, -1)] + [qd, primary, ~forced, s_all]
        order = np.lexsort(tuple(sort_keys))
        s_o = s_all[order]
        first = np.searchsorted(s_o, ids)
        rank = np.arange(s_o.size) - first[s_o - lo]
        return order[rank < M]

    take = select(np.zeros_like(hop))
    if mesh.period is None or np.any(mesh.face_cells[:, 1] < 0):
        # one-sided stencils at boundaries can be degenerate (e.g. too few cell
        # layers normal to a wall): rebuild those greedily, nearest first,
        # accepting a candidate only while it adds a new direction in the space
        # of degree-r monomials of the centroid offsets, then fill by distance
        flag, cond0 = _degenerate(take, s_all, c_all, off, h, d, r, n, M, mom)
        bad = lo + np.nonzero(flag)[0]
        if bad.size:
            order = np.lexsort(tuple([c_all] + [qoff[:, j] for j in range(d - 1, -1, -1)]
                                     + [qd, ~forced, s_all]))
            s_o = s_all[order]
            starts = np.searchsorted(s_o, bad)
            ncand = np.searchsorted(s_o, bad, side="right") - starts
            # candidates of every flagged cell side by side, nearest first,
            # padded with the cell's first candidate (masked out)
            L = int(ncand.max())
            slot = np.arange(L)
            valid = slot[None, :] < ncand[:, None]
            cand = order[starts[:, None] + np.where(valid, slot[None, :], 0)]
            fc = forced[cand] & valid
            V = _member_rows(mom, s_all[cand], c_all[cand], off[cand], h, d, r)
            V[~valid] = 0.0
            nrm = np.linalg.norm(V, axis=2)
            nb = bad.size
            KK = V.shape[2]
            # take is grouped by source cell, M members each
            best = take.reshape(n, M)[bad - lo].copy()
            best_cond = cond0[bad - lo].copy()
            rows = np.arange(nb)
            # nearest first, a candidate joins while it adds a direction of at
            # least tau of its own norm (face neighbours always join); larger
            # tau spreads the members; then fill by distance
            for tau in (0.3, 0.1, 0.03, 1e-6):
                Q = np.zeros((nb, KK, KK))
                qn = np.zeros(nb, np.int64)
                chosen = np.zeros((nb, L), bool)
                for t in range(L):
                    vt = V[:, t]
                    v = vt - np.einsum("nki,nk->ni", Q, np.einsum("nki,ni->nk", Q, vt))
                    nv = np.linalg.norm(v, axis=1)
                    room = qn < KK
                    new_dir = valid[:, t] & (nv > tau * nrm[:, t])
                    chosen[:, t] = fc[:, t] | (room & new_dir)
                    add = room & new_dir
                    ia = rows[add]
                    Q[ia, qn[ia]] = v[ia] / nv[ia, None]
                    qn[ia] += 1
                ok = qn == KK
                n_ch = chosen.sum(1)
                crank = np.cumsum(chosen, 1) - 1
                urank = np.cumsum(valid & ~chosen, 1) - 1
                sel = (chosen & (crank < M)) | (valid & ~chosen & (urank < (M - n_ch)[:, None]))
                ok &= sel.sum(1) == M
                if not ok.any():
                    continue
                io = rows[ok]
                pick = np.nonzero(sel[io])[1].reshape(io.size, M)
                cnd = _row_cond(V[io[:, None], pick])
                better = cnd < best_cond[io]
                ib = io[better]
                best[ib] = cand[ib[:, None], pick[better]]
                best_cond[ib] = cnd[better]
            repl = {int(c): best[i] for i, c in enumerate(bad)}
            keep = ~np.isin(s_all[take], bad)
            take = np.concatenate([take[keep]] + [repl[int(c)] for c in bad])
            take = take[np.argsort(s_all[take], kind="stable")]
    sel_s, sel_c, sel_sh = s_all[take], c_all[take], sh_all[take]
    sel_qd, sel_qoff = qd[take], qoff[take]
    # final nearest-first order
    sort_keys = [sel_c] + [sel_qoff[:, j] for j in range(d - 1, -1, -1)] + [sel_qd, sel_s]
    o2 = np.lexsort(tuple(sort_keys))
    central = sel_c[o2].reshape(n, M).astype(np.int32)
    central_shift = sel_sh[o2].reshape(n, M, d).astype(np.int8)
    return central, central_shift


def _cell_stencils(lo_hi):
    """Central, directional and MUSCL stencils of the source cells lo..hi-1."""
    lo, hi = lo_hi
    mesh, r, cen, h, period, adj_off, adj_dst, adj_sh, mom = pool.SHARED
    central, central_shift = _central_stencils(mesh, r, lo, hi, cen, h, period, adj_off, adj_dst, adj_sh, mom)
    return (central, central_shift) + _face_stencils(mesh, r, lo, hi, central, central_shift, cen, h, period)


def _face_stencils(mesh, r, lo, hi, central, central_shift, cen, h, period):
    """Directional and MUSCL stencils of the cells lo..hi-1, whose central
    stencils (rows 0..hi-lo-1) are given."""
    d = mesh.dim
    n = hi - lo
    M = central.shape[1]
    Md = 2 * d
    NF = nf_max(d)
    gid = np.arange(lo, hi)
    coff = (cen[central] + central_shift * period - cen[gid][:, None, :])  # [n, M, d]
    hl = h[lo:hi]

    # ---- face data per cell (in cell_face order) -----------------------------
    nfc = np.diff(mesh.cell_face_off)[lo:hi]
    fverts_rel = np.zeros((n, NF, 4, d))   # face vertices relative to cell centroid
    f_nverts = np.zeros((n, NF), np.int64)
    f_valid = np.zeros((n, NF), bool)
    f_nbr = np.full((n, NF), -1, np.int64)
    f_nbr_sh = np.zeros((n, NF, d), np.int64)
    for k in range(NF):
        cells = np.nonzero(nfc > k)[0]      # local rows
        gc = cells + lo
        f = mesh.cell_face[mesh.cell_face_off[gc] + k]
        side = mesh.cell_face_side[mesh.cell_face_off[gc] + k]
        f_valid[cells, k] = True
        nv = np.diff(mesh.face_vtx_off)[f]
        f_nverts[cells, k] = nv
        for j in range(4):
            ok = nv > j
            vv = mesh.face_vtx[mesh.face_vtx_off[f] + np.minimum(j, nv - 1)]
            pos = mesh.vertices[vv]
            # the right cell sees the face shifted back by its image
            pos = pos - (side[:, None] == 1) * mesh.face_shift[f].astype(np.float64) * period
            fverts_rel[cells, k, j] = np.where(ok[:, None], pos - cen[gc], 0.0)
        l, rr = mesh.face_cells[f, 0], mesh.face_cells[f, 1]
        nb = np.where(side == 0, rr, l)
        nsh = np.where((side == 0)[:, None], mesh.face_shift[f], -mesh.face_shift[f].astype(np.int64))
        f_nbr[cells, k] = nb
        f_nbr_sh[cells, k] = np.where((nb >= 0)[:, None], nsh, 0)
        # a right-side cell sees the face with reversed orientation
        for n_ in (2, 3, 4):
            sel = (side == 1) & (nv == n_)
            if np.any(sel):
                rc = cells[sel]
                fverts_rel[rc, k, :n_] = fverts_rel[rc, k, :n_][:, ::-1]

    # position of each face neighbour inside the central stencil
    def member_pos(rows_, nb, nbsh):
        eq = (central[rows_] == nb[:, None]) & np.all(central_shift[rows_] == nbsh[:, None, :], 2)
        pos = np.argmax(eq, 1)
        pos[~eq.any(1)] = -1
        return pos

    # ---- directional stencils ------------------------------------------------
    dir_pos = np.zeros((n, NF, Md), np.int64)
    tol = 1e-9
    dist2 = (coff ** 2).sum(2)  # [n, M]
    for k in range(NF):
        cells = np.nonzero(f_valid[:, k])[0]
        if cells.size == 0:
            continue
        V = fverts_rel[cells, k]  # [nc, 4, d]
        nv = f_nverts[cells, k]
        P = coff[cells]           # [nc, M, d]
        inside = np.ones((cells.size, M), bool)
        if d == 2:
            a, b = V[:, 0], V[:, 1]
            cr_a = a[:, None, 0] * P[:, :, 1] - a[:, None, 1] * P[:, :, 0]
            cr_b = P[:, :, 0] * b[:, None, 1] - P[:, :, 1] * b[:, None, 0]
            scale = (np.linalg.norm(a, axis=1) * np.linalg.norm(P, axis=2).T).T * tol
            inside &= (cr_a >= -scale) & (cr_b >= -scale)
            normal = np.stack([b[:, 1] - a[:, 1], a[:, 0] - b[:, 0]], 1)
        else:
            normal = np.zeros((cells.size, 3))
            for j in range(4):
                jn = (j + 1) % 4
                vj = V[:, j]
                vn = np.where((jn < nv)[:, None], V[:, jn % 4], V[:, 0])
                use = j < nv
                nk = np.cross(vj, vn)
                normal += np.where(use[:, None], nk, 0.0)
                dots = np.einsum("nd,nmd->nm", nk, P)
                scale = np.linalg.norm(nk, axis=1)[:, None] * np.linalg.norm(P, axis=2) * tol
                inside &= np.where(use[:, None], dots >= -scale, True)
        half = np.einsum("nd,nmd->nm", normal, P) > \
            tol * np.linalg.norm(normal, axis=1)[:, None] * np.linalg.norm(P, axis=2)
        fpos = member_pos(cells, f_nbr[cells, k], f_nbr_sh[cells, k])
        is_fn = np.zeros((cells.size, M), bool)
        okf = fpos >= 0
        is_fn[np.nonzero(okf)[0], fpos[okf]] = True
        # priority: face neighbour, sector/cone, half-space, rest; then distance
        pri = np.where(is_fn, 0, np.where(inside, 1, np.where(half, 2, 3)))
        key = pri * 10 ** 12 + np.rint(dist2[cells] / (hl[cells, None] ** 2) * 1e8).astype(np.int64)
        # stable tie-break by stencil position (which is already nearest-first and deterministic)
        full = np.argsort(key, axis=1, kind="stable")
        o = full[:, :Md]
        # a degree-1 fit needs members spanning d directions; where the first Md
        # do not (e.g. the wall face of a prism layer, whose nearest cells share
        # one plane), take members in the same order, accepting one only while it
        # adds a direction, then fill in that order
        Po = np.take_along_axis(P, o[:, :, None], axis=1)
        sv = np.linalg.svd(Po, compute_uv=False)
        for i in np.nonzero(sv[:, -1] <= 1e-6 * sv[:, 0])[0]:
            basis, chosen = [], []
            for t in full[i]:
                v = P[i, t].copy()
                for b in basis:
                    v -= (v @ b) * b
                nv_ = np.linalg.norm(v)
                if len(basis) < d and nv_ > 1e-6 * np.linalg.norm(P[i, t]):
                    basis.append(v / nv_)
                    chosen.append(t)
            for t in full[i]:
                if len(chosen) >= Md:
                    break
                if t not in chosen:
                    chosen.append(t)
            o[i] = np.array(sorted(chosen[:Md], key=lambda t: list(full[i]).index(t)))
        dir_pos[cells, k] = o
    rows = np.arange(n)[:, None, None]
    dir_ids = central[rows, dir_pos].astype(np.int32)
    dir_sh = central_shift[rows, dir_pos].astype(np.int8)
    n_dir = nfc.astype(np.int32)
    for k in range(NF):
        dir_ids[~f_valid[:, k], k] = -1
        dir_sh[~f_valid[:, k], k] = 0

    # ---- MUSCL stencils --------------------------------------------------------
    muscl = np.full((n, NF), -1, np.int32)
    muscl_sh = np.zeros((n, NF, d), np.int8)
    n_muscl = np.zeros(n, np.int32)
    has_nb = (f_nbr >= 0) & f_valid
    # face neighbours first, in cell-face order
    rank = np.cumsum(has_nb, axis=1) - 1
    rr, kk = np.nonzero(has_nb)
    muscl[rr, rank[rr, kk]] = f_nbr[rr, kk]
    muscl_sh[rr, rank[rr, kk]] = f_nbr_sh[rr, kk]
    n_muscl[:] = has_nb.sum(1)
    for c in np.nonzero(n_muscl < d + 1)[0]:
        lst = [(int(muscl[c, j]), tuple(int(x) for x in muscl_sh[c, j])) for j in range(n_muscl[c])]
        for m in range(M):
            cand = (int(central[c, m]), tuple(int(x) for x in central_shift[c, m]))
            if cand not in lst:
                lst.append(cand)
            if len(lst) >= d + 1:
                break
        n_muscl[c] = len(lst)
        for j, (cc, ss) in enumerate(lst):
            muscl[c, j] = cc
            muscl_sh[c, j] = ss
    return dir_ids, dir_sh, n_dir, muscl, muscl_sh, n_muscl


def build_stencils(mesh: Mesh, r: int, chunk: int = 65536, workers: int = 1) -> Stencils:
    """Stencils of every cell, built in chunks of source cells (each cell's
    stencils depend only on its own neighbourhood).  ``workers`` > 1 builds
    the chunks in a pool of forked processes (use only in a process that has
    not initialised a GPU)."""
    d = mesh.dim
    N = mesh.n_cells
    if N >= (1 << 21):
        raise ValueError("stencil builder supports fewer than 2^21 cells")
    cen, vol = cell_centroids(mesh)
    h = vol ** (1.0 / d)
    period = mesh.period if mesh.period is not None else np.zeros(d)
    adj_off, adj_dst, adj_sh = _adjacency(mesh)
    ranges = [(lo, min(N, lo + chunk)) for lo in range(0, N, chunk)]
    bounded = mesh.period is None or np.any(mesh.face_cells[:, 1] < 0)
    mom = _central_moments(mesh, r, cen, workers) if bounded else None
    parts = pool.pool_map(_cell_stencils, ranges, workers,
                          (mesh, r, cen, h, period, adj_off, adj_dst, adj_sh, mom))
    cat = [np.concatenate([p_[i] for p_ in parts]) for i in range(8)]
    return Stencils(r=r, M=cat[0].shape[1], Md=2 * d, central=cat[0], central_shift=cat[1],
                    dir=cat[2], dir_shift=cat[3], n_dir=cat[4], muscl=cat[5],
                    muscl_shift=cat[6], n_muscl=cat[7])


def build_stencils_periodic_hex(mesh: Mesh, dims, r: int, n_small: int = 12) -> Stencils:
    """Stencils of a uniform periodic hexahedral mesh (cells numbered x-fastest).

    Such a mesh is translation invariant, so every cell's stencils are the
    translates of one template.  The template comes from ``build_stencils`` on a
    small periodic mesh of the same spacing (checked against several of its
    cells), and is replicated here by index arithmetic.
    """
    from .mesh import hex_3d
    nx, ny, nz = dims
    d = 3
    L = mesh.period
    hx, hy, hz = L[0] / nx, L[1] / ny, L[2] / nz
    ns = n_small
    ms = hex_3d(ns, ns, ns, hi=(ns * hx, ns * hy, ns * hz), periodic=True)
    ss = build_stencils(ms, r)

    def pos(c, n3):
        a, b, _ = n3
        return np.stack([c % a, (c // a) % b, c // (a * b)], -1)

    n_s = (ns, ns, ns)
    ref = 0
    toff = pos(ss.central[ref], n_s) + ss.central_shift[ref] * ns - pos(np.array(ref), n_s)

    def face_dirs(m, c_arr, n3):
        """Neighbour offsets of every face of each cell, in cell-face order: [n, 6, 3]."""
        out = np.zeros((c_arr.size, 6, 3), np.int64)
        for k in range(6):
            f = m.cell_face[m.cell_face_off[c_arr] + k]
            side = m.cell_face_side[m.cell_face_off[c_arr] + k]
            l, rr = m.face_cells[f, 0], m.face_cells[f, 1]
            nb = np.where(side == 0, rr, l)
            sh = np.where((side == 0)[:, None], m.face_shift[f], -m.face_shift[f].astype(np.int64))
            out[:, k] = pos(nb, n3) + sh * np.array(n3) - pos(c_arr, n3)
        return out

    tdir = {}
    fd0 = face_dirs(ms, np.array([ref]), n_s)[0]
    for k in range(6):
        tdir[tuple(fd0[k])] = pos(ss.dir[ref, k], n_s) + ss.dir_shift[ref, k] * ns - pos(np.array(ref), n_s)
    # the template must describe every cell of the small mesh
    for c in (1, ns + 2, ns * ns * 3 + ns + 5, ms.n_cells - 1):
        off_c = pos(ss.central[c], n_s) + ss.central_shift[c] * ns - pos(np.array(c), n_s)
        if not np.array_equal(off_c, toff):
            raise RuntimeError("central stencil template is not translation invariant")
        fdc = face_dirs(ms, np.array([c]), n_s)[0]
        for k in range(6):
            o = pos(ss.dir[c, k], n_s) + ss.dir_shift[c, k] * ns - pos(np.array(c), n_s)
            if not np.array_equal(o, tdir[tuple(fdc[k])]):
                raise RuntimeError("directional stencil template is not translation invariant")

    N = mesh.n_cells
    n3 = np.array([nx, ny, nz])
    cells = np.arange(N)
    P = pos(cells, (nx, ny, nz))

    def place(offsets):  # offsets [..., 3] relative to each cell -> ids, shifts
        q = P.reshape((N,) + (1,) * (offsets.ndim - 2) + (3,)) + offsets
        sh = np.floor_divide(q, n3)
        w = q - sh * n3
        ids = w[..., 0] + nx * (w[..., 1] + ny * w[..., 2])
        return ids.astype(np.int32), sh.astype(np.int8)

    central, central_shift = place(toff[None])
    fd = face_dirs(mesh, cells, (nx, ny, nz))
    dir_off = np.zeros((N, 6, ss.Md, 3), np.int64)
    for key, val in tdir.items():
        msk = np.all(fd == np.array(key), axis=2)
        dir_off[msk] = val
    dir_ids, dir_sh = place(dir_off)
    mus_ids, mus_sh = place(fd)
    return Stencils(r=r, M=ss.M, Md=ss.Md, central=central, central_shift=central_shift, dir=dir_ids,
                    dir_shift=dir_sh, n_dir=np.full(N, 6, np.int32), muscl=mus_ids, muscl_shift=mus_sh,
                    n_muscl=np.full(N, 6, np.int32))
