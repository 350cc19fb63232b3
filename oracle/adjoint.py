"""Oracle of the residual's vector-Jacobian product (test infrastructure only).

The residual with the cell classes held fixed is written here in plain
PyTorch CPU float64 operations, step by step as in ``reconstruction`` and
``flux`` (Sections 2.1-2.4), with the oracle's precomputed tables as
constants; torch autograd then gives the exact vector-Jacobian product.
Switch conventions match the library: the class of every cell, the Harten
fallback and the CWENOZ |SI_s - SI_1| sign (0 at a tie) are frozen; the
Barth-Jespersen and Venkatakrishnan limiters differentiate through their
minimising Gauss point and bound cell; the Riemann solver through its active
branch.

Pinned in tests against central finite differences of the NumPy oracle.
"""
from __future__ import annotations

import numpy as np
import torch

from .reconstruction import OracleModel, LIN, CW, MU, VENKAT


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x))


def frozen_face_values(model: OracleModel, U: torch.Tensor, cls: np.ndarray) -> torch.Tensor:
    """Per-cell Gauss-point values [N, NGPC, nvar] for the given classes."""
    p = model.p
    st = model.st
    d, K = model.d, model.K
    N = model.mesh.n_cells
    cells = np.arange(N)
    tab = model.tables(cells)
    phi = _t(model.phi_at_gp(tab))
    U0 = U[:, None, :]
    # linear least squares (Section 2.1)
    dU = U[_t(st.central.astype(np.int64))] - U0
    a = torch.einsum("nkm,nmv->nkv", _t(tab["P"]), dU)
    fv_lin = U0 + torch.einsum("ngk,nkv->ngv", phi, a)
    # CWENOZ (Section 2.3)
    nd = _t(st.n_dir.astype(np.float64))
    NF = st.dir.shape[1]
    ids = np.where(st.dir >= 0, st.dir, cells[:, None, None]).astype(np.int64)
    dUd = U[_t(ids)] - U[:, None, None, :]
    a_dir = torch.einsum("nfjm,nfmv->nfjv", _t(tab["Pdir"]), dUd)
    svalid = _t((np.arange(NF)[None, :] < st.n_dir[:, None]).astype(np.float64))
    a_hat = torch.cat([a_dir, torch.zeros(N, NF, K - d, model.nvar, dtype=U.dtype)], 2) * svalid[..., None, None]
    lam1 = 1.0 - 1.0 / p.lambda1_prime
    lams = (1.0 - lam1) / nd
    a1 = (a - lams[:, None, None] * a_hat.sum(1)) / lam1
    OI = _t(tab["OI"])
    SI1 = torch.einsum("nkv,nkq,nqv->nv", a1, OI, a1)
    SIs = torch.einsum("nfkv,nkq,nfqv->nfv", a_hat, OI, a_hat)
    tau = (torch.abs(SIs - SI1[:, None, :]) * svalid[..., None]).sum(1) / nd[:, None]
    if p.cweno_form == 0:
        w1 = lam1 * (1.0 + (tau / (p.eps_w + SI1)) ** p.b_w)
        ws = lams[:, None, None] * (1.0 + (tau[:, None, :] / (p.eps_w + SIs)) ** p.b_w)
    else:
        w1 = lam1 * (1.0 + tau ** p.b_w / (p.eps_w + SI1))
        ws = lams[:, None, None] * (1.0 + tau[:, None, :] ** p.b_w / (p.eps_w + SIs))
    ws = ws * svalid[..., None]
    tot = w1 + ws.sum(1)
    a_cw = (w1 / tot)[:, None, :] * a1 + torch.einsum("nfv,nfkv->nkv", ws / tot[:, None, :], a_hat)
    fv_cw = U0 + torch.einsum("ngk,nkv->ngv", phi, a_cw)
    # MUSCL + Barth-Jespersen or Venkatakrishnan (Sections 2.2, 3.2)
    mid = np.where(st.muscl >= 0, st.muscl, cells[:, None]).astype(np.int64)
    g = torch.einsum("njm,nmv->njv", _t(tab["Pmus"]), U[_t(mid)] - U0)
    delta = torch.einsum("ngj,njv->ngv", phi[..., :d], g)
    nb = model.nbr
    nbv = U[_t(np.where(nb >= 0, nb, cells[:, None]).astype(np.int64))]
    allv = torch.cat([U0, nbv], 1)
    mn = allv.min(1).values
    mx = allv.max(1).values
    up = (mx - U)[:, None, :]
    dn = (mn - U)[:, None, :]
    safe = torch.where(delta == 0, torch.ones_like(delta), delta)
    one = torch.ones_like(delta)
    if p.limiter == VENKAT:
        room = torch.where(delta > 0, up, dn)
        eps2 = _t((p.kappa * model.geo.h) ** 3)[:, None, None]
        num = room * room + 2.0 * delta * room + eps2
        den = room * room + 2.0 * delta * delta + delta * room + eps2
        ratio = torch.where(delta != 0, num / den, one)
    else:
        ratio = torch.where(delta > 0, torch.minimum(one, up / safe),
                            torch.where(delta < 0, torch.minimum(one, dn / safe), one))
    valid = _t(np.arange(phi.shape[1])[None, :] < model.geo.c_ngp[:, None])[..., None]
    ratio = torch.where(valid, ratio, one)
    theta = ratio.min(1).values
    if p.limiter == VENKAT:          # its function exceeds 1 past twice the room; theta stays <= 1
        theta = torch.clamp(theta, max=1.0)
    fv_mu = U0 + theta[:, None, :] * delta
    c = _t(cls.astype(np.int64))[:, None, None]
    return torch.where(c == LIN, fv_lin, torch.where(c == CW, fv_cw, torch.where(c == MU, fv_mu, U0.expand_as(fv_lin))))


def _primitives(U, gamma):
    rho = U[..., 0]
    vel = U[..., 1:-1] / rho[..., None]
    pr = (gamma - 1.0) * (U[..., -1] - 0.5 * rho * (vel ** 2).sum(-1))
    return rho, vel, pr


def _flux(U, n, gamma):
    rho, vel, pr = _primitives(U, gamma)
    un = (vel * n).sum(-1)
    return torch.cat([(rho * un)[..., None], rho[..., None] * vel * un[..., None] + pr[..., None] * n,
                      (un * (U[..., -1] + pr))[..., None]], -1), (rho, vel, pr, un)


def riemann(UL, UR, n, gamma, hllc):
    FL, (rL, vL, pL, unL) = _flux(UL, n, gamma)
    FR, (rR, vR, pR, unR) = _flux(UR, n, gamma)
    cL = torch.sqrt(gamma * pL / rL)
    cR = torch.sqrt(gamma * pR / rR)
    SL = torch.minimum(unL - cL, unR - cR)
    SR = torch.maximum(unL + cL, unR + cR)
    if not hllc:
        mid = (SR[..., None] * FL - SL[..., None] * FR + (SL * SR)[..., None] * (UR - UL)) / (SR - SL)[..., None]
        return torch.where((SL >= 0)[..., None], FL, torch.where((SR <= 0)[..., None], FR, mid))
    Ss = (pR - pL + rL * unL * (SL - unL) - rR * unR * (SR - unR)) / (rL * (SL - unL) - rR * (SR - unR))

    def star(U, r, v, pr, un, S):
        fac = r * (S - un) / (S - Ss)
        return torch.cat([fac[..., None], fac[..., None] * (v + (Ss - un)[..., None] * n),
                          (fac * (U[..., -1] / r + (Ss - un) * (Ss + pr / (r * (S - un)))))[..., None]], -1)

    FsL = FL + SL[..., None] * (star(UL, rL, vL, pL, unL, SL) - UL)
    FsR = FR + SR[..., None] * (star(UR, rR, vR, pR, unR, SR) - UR)
    return torch.where((SL >= 0)[..., None], FL,
                       torch.where((Ss >= 0)[..., None], FsL, torch.where((SR > 0)[..., None], FsR, FR)))


def frozen_residual(model: OracleModel, U: torch.Tensor, cls: np.ndarray) -> torch.Tensor:
    """R(U) [N, nvar] with the classes held at ``cls`` (Eq. EulerEquationsDetails)."""
    geo = model.geo
    mesh = model.mesh
    N, nvar = U.shape
    fv = frozen_face_values(model, U, cls)
    NGPC = fv.shape[1]
    cc, ss = np.nonzero(np.arange(NGPC)[None, :] < geo.c_ngp[:, None])
    src = cc * NGPC + ss
    dst = geo.c_side[cc, ss] * geo.n_gp + geo.c_gidx[cc, ss]
    fs = torch.zeros(2 * geo.n_gp, nvar, dtype=U.dtype).index_copy(0, _t(dst.astype(np.int64)),
                                                                     fv.reshape(-1, nvar)[_t(src.astype(np.int64))])
    face_of_gp = np.repeat(np.arange(mesh.n_faces), np.diff(geo.gp_off))
    bnd = mesh.face_cells[face_of_gp, 1] < 0
    gidx = np.arange(geo.n_gp)
    UL = fs[_t(gidx)]
    UR = fs[_t(np.where(bnd, gidx, geo.n_gp + gidx))]
    F = riemann(UL, UR, _t(geo.normal[face_of_gp]), model.p.gamma, model.p.riemann == 0)
    Fw = F * _t(geo.gp_wS)[:, None]
    Ff = torch.zeros(mesh.n_faces, nvar, dtype=U.dtype).index_add(0, _t(face_of_gp), Fw)
    l = mesh.face_cells[:, 0].astype(np.int64)
    r = mesh.face_cells[:, 1].astype(np.int64)
    inner = r >= 0
    R = torch.zeros(N, nvar, dtype=U.dtype).index_add(0, _t(l), -Ff)
    R = R.index_add(0, _t(r[inner]), Ff[_t(np.nonzero(inner)[0])])
    return R / _t(geo.vol)[:, None]


def residual_vjp(model: OracleModel, U: np.ndarray, cls: np.ndarray, gR: np.ndarray) -> np.ndarray:
    """(dR/dU)^T gR with frozen classes; U, gR [N, nvar] float64."""
    Ut = torch.tensor(U, dtype=torch.float64, requires_grad=True)
    R = frozen_residual(model, Ut, cls)
    (gU,) = torch.autograd.grad(R, Ut, torch.tensor(gR, dtype=torch.float64))
    return gU.numpy()
