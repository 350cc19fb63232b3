"""Shared test helpers: tolerance checks and near-threshold accounting."""
from __future__ import annotations

import numpy as np


def state_scale(U):
    """S_v = max over cells of |U_v|  (floor for zero-mean components)."""
    return np.abs(U).max(0)


def rel_err(x, ref, scale_b):
    """max |x - ref| / max(|ref|, S_v); ``scale_b`` is S_v broadcast against ``ref``."""
    den = np.maximum(np.maximum(np.abs(ref), scale_b), 1e-300)
    return float(np.nanmax(np.abs(x - ref) / den))


def _mask(out, geo, cells):
    valid = np.arange(out.shape[1])[None, :] < geo.c_ngp[cells][:, None]
    return np.where(valid[..., None], out, np.nan)


def oracle_cell_values(fs, geo, cells):
    """Per-cell Gauss-point values [n, NGPC, nvar] (NaN past a cell's count)
    gathered from the oracle's face states [2, nvar, NGPT]."""
    cells = np.asarray(cells)
    out = fs[geo.c_side[cells], :, np.maximum(geo.c_gidx[cells], 0)]
    return _mask(out, geo, cells)


def gpu_cell_values(fs, geo, cells):
    """Per-cell Gauss-point values [n, NGPC, nvar] (NaN past a cell's count)
    from the library's cell-major states [NGPC, nvar, N]."""
    cells = np.asarray(cells)
    assert fs.shape[0] == geo.c_gidx.shape[1]
    out = np.moveaxis(fs[:, :, cells], 2, 0)
    valid = np.arange(out.shape[1])[None, :] < geo.c_ngp[cells][:, None]
    # slots past a cell's count are never written: drop them before widening
    return np.where(valid[..., None], np.where(valid[..., None], out, 0).astype(np.float64), np.nan)


def states_err(fs_gpu, fs_o, geo, S, cells=None):
    """rel_err of the library's Gauss-point states against the oracle's, all
    (or the given) cells, scaled per variable by S."""
    fs_gpu = fs_gpu.cpu().numpy() if hasattr(fs_gpu, "cpu") else fs_gpu
    cells = np.arange(fs_gpu.shape[2]) if cells is None else cells
    return rel_err(gpu_cell_values(fs_gpu, geo, cells), oracle_cell_values(fs_o, geo, cells), S[None, None, :])


def near_riemann_branch(om, fs_o, stencils, tol):
    """Cells whose gradient can see a Riemann-solver branch point: the two cells
    of every face with a Gauss point where |S_L|, |S_R| or (HLLC) |S*| is
    within tol * max sound speed of zero, and every cell in their central
    stencils.  The flux Jacobian jumps there, so a state rounding can switch
    the branch the adjoint differentiates."""
    g = om.p.gamma
    geo = om.geo
    nrm = np.repeat(geo.normal, np.diff(geo.gp_off), axis=0)

    def prim(q):
        r = q[:, 0]
        v = q[:, 1:-1] / r[:, None]
        return r, v, (g - 1) * (q[:, -1] - 0.5 * r * (v ** 2).sum(1))
    rL, vL, pL = prim(fs_o[0].T)
    rR, vR, pR = prim(fs_o[1].T)
    unL, unR = (vL * nrm).sum(1), (vR * nrm).sum(1)
    cL, cR = np.sqrt(g * pL / rL), np.sqrt(g * pR / rR)
    SL, SR = np.minimum(unL - cL, unR - cR), np.maximum(unL + cL, unR + cR)
    near = np.minimum(np.abs(SL), np.abs(SR))
    if om.p.riemann == 0:  # HLLC contact speed
        Ss = (pR - pL + rL * unL * (SL - unL) - rR * unR * (SR - unR)) / (rL * (SL - unL) - rR * (SR - unR))
        near = np.minimum(near, np.abs(Ss))
    thr = tol * max(cL.max(), cR.max())
    faces = np.nonzero(np.minimum.reduceat(near, geo.gp_off[:-1]) <= thr)[0]
    cells = np.unique(om.mesh.face_cells[faces].ravel())
    cells = cells[cells >= 0]
    out = np.zeros(om.mesh.n_cells, bool)
    out[cells] = True
    out[stencils.central[cells].ravel()] = True
    return out


def near_threshold(om, U, cells, tol):
    """Cells whose class decision lies within ``tol`` (relative) of a threshold.

    NAD: |d - delta_w| or |d - delta_m| within tol * S with S = max(|m|, |M|, R)
    for a variable whose stencil range is non-zero, when the higher of the two
    classes at that tie exceeds the class the other variables give (the cell
    takes the maximum over variables), in a cell that is not deactivated (a
    deactivated cell is linear whatever the NAD says);
    deactivation: |dU - (kappa h)^n| within tol * max(dU, (kappa h)^n); Harten:
    any point of the linear candidate within tol of its bound.
    """
    own, info = om.own_class(cells, U)
    S = np.maximum(np.maximum(np.abs(info["m"]), np.abs(info["M"])), info["R"])
    live = info["R"] > 0
    dv = info["dv"]
    wm, dm = info["wmarg"], info["dmarg"]
    cv = np.where(~live | (dv <= wm), 0, np.where(dv >= dm, 2, 1))      # per-variable class
    tie_w = live & (np.abs(dv - wm) <= tol * S)
    tie_m = live & (np.abs(dv - dm) <= tol * S)
    hi = np.where(tie_m, 2, np.where(dv >= dm, 2, 1))                    # higher class at the tie
    nv = cv.shape[1]
    others = np.stack([np.delete(cv, v, axis=1).max(1) if nv > 1 else np.zeros(len(cv), int)
                       for v in range(nv)], 1)
    nad = (tie_w | tie_m) & (others < hi)
    deact_near = np.abs(info["dU"] - info["thr"]) <= tol * np.maximum(info["dU"], info["thr"])
    deactivated = (info["dU"] < info["thr"]) & ~deact_near
    flag = nad.any(1) & ~deactivated
    flag |= deact_near
    _, fv, _ = om.linear(cells, U)
    g = om.p.gamma
    ngp = om.geo.c_ngp[cells]
    valid = np.arange(fv.shape[1])[None, :] < ngp[:, None]
    Ub = U[cells]
    rb = Ub[:, 0][:, None]
    pb = ((g - 1) * (Ub[:, -1] - 0.5 * (Ub[:, 1:-1] ** 2).sum(1) / Ub[:, 0]))[:, None]
    with np.errstate(all="ignore"):
        pr = (g - 1) * (fv[..., -1] - 0.5 * (fv[..., 1:-1] ** 2).sum(-1) / fv[..., 0])
        hr = np.abs(np.abs(fv[..., 0] - rb) - om.p.tvd_theta * np.abs(rb)) <= tol * np.abs(rb)
        hp = np.abs(np.abs(pr - pb) - om.p.tvd_theta * np.abs(pb)) <= tol * np.abs(pb)
    flag |= np.any(valid & (hr | hp), axis=1)
    return flag


def margin_tolerance(om, U, cells, tol):
    """Per-cell bound on the error of near_margin when the states carry an
    error of tol * S_v (S_v = max over cells of |U_v|, the state bar): the
    margin divides an excursion by the cell's own scale max(|m|, |M|, R), so
    the bound is tol * max over the cell's live variables of max(1, S_v /
    that scale)."""
    _, info = om.own_class(cells, U)
    Sc = np.maximum(np.maximum(np.abs(info["m"]), np.abs(info["M"])), info["R"])
    Sv = state_scale(U)[None, :]
    with np.errstate(divide="ignore"):
        ratio = np.where(info["R"] > 0, np.maximum(1.0, Sv / Sc), 1.0)
    return tol * ratio.max(1)
