"""Oracle Riemann fluxes and finite-volume residual (test infrastructure only).

* Euler flux F_c . n (Section 2, Eq. Terms1), perfect gas
  E = p/(gamma-1) + rho |u|^2 / 2.
* HLLC (Toro) and HLL approximate Riemann solvers (Section 2.4); the wave
  speeds are not given in the paper, Davis estimates are used:
  S_L = min(u_nL - c_L, u_nR - c_R), S_R = max(u_nL + c_L, u_nR + c_R), and
  the contact speed S* of the HLLC solver.
* Residual of Eq. EulerEquationsDetails:
  R_i = -(1/|V_i|) sum_faces sum_alpha (F_c(U_L, U_R) - F_v) w_alpha |S_l|,
  the flux taken along the normal pointing out of the face's left cell;
  F_v = 0 (Euler) unless the parameters turn the viscous fluxes on.
"""
from __future__ import annotations

import numpy as np


def primitives(U, gamma):
    rho = U[..., 0]
    vel = U[..., 1:-1] / rho[..., None]
    p = (gamma - 1.0) * (U[..., -1] - 0.5 * rho * (vel ** 2).sum(-1))
    return rho, vel, p


def euler_flux(U, n, gamma):
    rho, vel, p = primitives(U, gamma)
    un = (vel * n).sum(-1)
    F = np.empty_like(U)
    F[..., 0] = rho * un
    F[..., 1:-1] = rho[..., None] * vel * un[..., None] + p[..., None] * n
    F[..., -1] = un * (U[..., -1] + p)
    return F


def _speeds(UL, UR, n, gamma):
    rL, vL, pL = primitives(UL, gamma)
    rR, vR, pR = primitives(UR, gamma)
    unL = (vL * n).sum(-1)
    unR = (vR * n).sum(-1)
    cL = np.sqrt(gamma * pL / rL)
    cR = np.sqrt(gamma * pR / rR)
    SL = np.minimum(unL - cL, unR - cR)
    SR = np.maximum(unL + cL, unR + cR)
    return (rL, vL, pL, unL), (rR, vR, pR, unR), SL, SR


def hll(UL, UR, n, gamma):
    _, _, SL, SR = _speeds(UL, UR, n, gamma)
    FL = euler_flux(UL, n, gamma)
    FR = euler_flux(UR, n, gamma)
    mid = (SR[..., None] * FL - SL[..., None] * FR + (SL * SR)[..., None] * (UR - UL)) / (SR - SL)[..., None]
    return np.where((SL >= 0)[..., None], FL, np.where((SR <= 0)[..., None], FR, mid))


def hllc_star_states(UL, UR, n, gamma):
    """Toro's HLLC intermediate states: (S_L, S_R, S*, U*_L, U*_R, F_L, F_R).

    S* is the contact speed that makes the two star states carry equal
    pressure; each star state keeps its side's tangential velocity and moves
    with normal velocity S*."""
    (rL, vL, pL, unL), (rR, vR, pR, unR), SL, SR = _speeds(UL, UR, n, gamma)
    FL = euler_flux(UL, n, gamma)
    FR = euler_flux(UR, n, gamma)
    Ss = (pR - pL + rL * unL * (SL - unL) - rR * unR * (SR - unR)) / (rL * (SL - unL) - rR * (SR - unR))

    def star(U, r, v, p, un, S):
        fac = r * (S - un) / (S - Ss)
        Us = np.empty_like(U)
        Us[..., 0] = fac
        Us[..., 1:-1] = fac[..., None] * (v + (Ss - un)[..., None] * n)
        Us[..., -1] = fac * (U[..., -1] / r + (Ss - un) * (Ss + p / (r * (S - un))))
        return Us

    return SL, SR, Ss, star(UL, rL, vL, pL, unL, SL), star(UR, rR, vR, pR, unR, SR), FL, FR


def hllc(UL, UR, n, gamma):
    SL, SR, Ss, UsL, UsR, FL, FR = hllc_star_states(UL, UR, n, gamma)
    FsL = FL + SL[..., None] * (UsL - UL)
    FsR = FR + SR[..., None] * (UsR - UR)
    return np.where((SL >= 0)[..., None], FL,
                    np.where((Ss >= 0)[..., None], FsL,
                             np.where((SR > 0)[..., None], FsR, FR)))


def face_fluxes(model, fs, riemann):
    """Integrated face fluxes F_f [nvar, nf] from face states [2, nvar, NGPT]."""
    geo = model.geo
    g = model.p.gamma
    UL = fs[0].T
    UR = fs[1].T
    face_of_gp = np.repeat(np.arange(model.mesh.n_faces), np.diff(geo.gp_off))
    n = geo.normal[face_of_gp]
    F = hllc(UL, UR, n, g) if riemann == 0 else hll(UL, UR, n, g)
    Fw = F * geo.gp_wS[:, None]
    out = np.zeros((model.mesh.n_faces, model.nvar))
    np.add.at(out, face_of_gp, Fw)
    return out.T


def residual_from_face_fluxes(model, Ff):
    mesh = model.mesh
    R = np.zeros((model.nvar, mesh.n_cells))
    l = mesh.face_cells[:, 0]
    r = mesh.face_cells[:, 1]
    np.add.at(R.T, l, -Ff.T)
    inner = r >= 0
    np.add.at(R.T, r[inner], Ff.T[inner])
    return R / model.geo.vol[None, :]


def residual(model, U):
    """R(U) [nvar, N], face states and classes (Eq. EulerEquationsDetails);
    with viscous fluxes when the parameters ask for them (oracle/viscous.py)."""
    fs, cls = model.reconstruct(U)
    Ff = face_fluxes(model, fs, model.p.riemann)
    if getattr(model.p, "viscous", 0):
        from .viscous import face_viscous_fluxes
        Ff = Ff - face_viscous_fluxes(model, fs, U)
    return residual_from_face_fluxes(model, Ff), fs, cls
