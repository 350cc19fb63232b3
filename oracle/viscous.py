"""Viscous fluxes of the Navier-Stokes equations (test infrastructure only).

Section 2, Eqs. NAVIERCOMPLETE, Terms1, sutherlandlaw, HeatConduct, Stresses
and Section 2.4, Eq. viscous_jump.  Readings taken where the paper is silent:

* Temperature T = p / rho (the gas constant folded into the nondimensional
  pressure), so the conduction term (mu / Pr) gamma / (gamma - 1) dT/dx_j of
  Eq. HeatConduct is the flux of c_p T with c_p = gamma / (gamma - 1).
* Viscosity by Sutherland's law, mu = mu_0 (T / T_0)^(3/2) (T_0 + S) / (T + S),
  with mu_0, T_0, S and Pr given.
* Gradients at the face Gauss points come from each side's central
  least-squares polynomial of Section 2.1 (the unlimited high-order fit,
  whatever the cell's class): grad U(x) = sum_k a_k grad phi_k(xi) / h_c.
* The face gradient is Eq. viscous_jump: the mean of the two sides' gradients
  plus (alpha / L_int) (U_R - U_L) n, alpha = 4/3, L_int the distance between
  the two cell centres (the right cell's periodic image next to the left
  cell); at a boundary face (transmissive ghost, U_R = U_L) the right side
  is the left side.
* The flux is taken at the mean state (U_L + U_R) / 2: viscosity,
  velocity in the work term, and the chain rule from conserved to velocity
  and temperature gradients,
      grad u_i = (grad m_i - u_i grad rho) / rho,
      grad p = (gamma - 1) (grad E - sum_i u_i grad m_i + |u|^2 grad rho / 2),
      grad T = (grad p - T grad rho) / rho.
* F_v . n = (0, tau n, (tau u + (mu / Pr) gamma / (gamma - 1) grad T) . n),
  tau_ij = mu (du_i/dx_j + du_j/dx_i - (2/3) div u delta_ij), and the
  residual gains +(1/|V_i|) sum_faces sum_alpha F_v w_alpha |S| along the
  normal out of cell i (Eq. EulerEquationsDetails).
"""
from __future__ import annotations

import numpy as np


def monomial_gradients(xi, exps):
    """xi [..., d] -> [..., K, d]: d(xi^alpha_k)/d xi_j."""
    d = xi.shape[-1]
    K = exps.shape[0]
    out = np.zeros(xi.shape[:-1] + (K, d))
    for j in range(d):
        g = np.ones(xi.shape[:-1] + (K,))
        for i in range(d):
            e = exps[:, i] - (1 if i == j else 0)
            g = g * np.where(e >= 0, xi[..., i:i + 1] ** np.maximum(e, 0), 0.0)
        out[..., j] = g * exps[:, j]
    return out


def cell_gradients(model, U):
    """Gradients of the conserved variables at every cell's face Gauss
    points from its central least-squares polynomial: [N, NGPC, d, nvar]."""
    cells = np.arange(model.mesh.n_cells)
    a, _, tab = model.linear(cells, U)                       # a [N, K, nvar]
    dm = monomial_gradients(tab["xi"], model.exps)           # [N, NGPC, K, d]
    g = np.einsum("nskj,nkv->nsjv", dm, a)
    return g / model.geo.h[:, None, None, None]


def sutherland(T, p):
    return p.mu0 * (T / p.T0) ** 1.5 * (p.T0 + p.sutherland_S) / (T + p.sutherland_S)


def viscous_flux(UL, UR, gL, gR, n, inv_l, p):
    """F_v . n at face points: states [..., nv], gradients [..., d, nv],
    unit normal [..., d], 1 / L_int [...]."""
    g = p.gamma
    Um = 0.5 * (UL + UR)
    G = 0.5 * (gL + gR) + (p.visc_alpha * inv_l)[..., None, None] * n[..., :, None] * (UR - UL)[..., None, :]
    rho = Um[..., 0]
    u = Um[..., 1:-1] / rho[..., None]
    pr = (g - 1.0) * (Um[..., -1] - 0.5 * rho * (u ** 2).sum(-1))
    T = pr / rho
    grho = G[..., 0]                                         # [..., d]
    gm = G[..., 1:-1]                                        # [..., d, i]: d m_i / d x_j at [j, i]
    gu = (gm - grho[..., :, None] * u[..., None, :]) / rho[..., None, None]   # [..., j, i] = du_i/dx_j
    gp = (g - 1.0) * (G[..., -1] - (gm * u[..., None, :]).sum(-1) + 0.5 * (u ** 2).sum(-1)[..., None] * grho)
    gT = (gp - T[..., None] * grho) / rho[..., None]
    mu = sutherland(T, p)
    du = np.swapaxes(gu, -1, -2)                             # [..., i, j] = du_i/dx_j
    div = np.trace(du, axis1=-2, axis2=-1)
    d = n.shape[-1]
    tau = mu[..., None, None] * (du + np.swapaxes(du, -1, -2) - (2.0 / 3.0) * div[..., None, None] * np.eye(d))
    k = mu / p.prandtl * g / (g - 1.0)
    F = np.zeros(UL.shape)
    F[..., 1:-1] = np.einsum("...ij,...j->...i", tau, n)
    F[..., -1] = np.einsum("...i,...ij,...j->...", u, tau, n) + k * (gT * n).sum(-1)
    return F


def face_inverse_distances(model):
    """1 / L_int per face: the distance between the two cell centres, the
    right cell's periodic image placed next to the left cell (boundary
    faces: 0, no jump term)."""
    mesh, geo = model.mesh, model.geo
    fc = mesh.face_cells
    out = np.zeros(mesh.n_faces)
    inner = fc[:, 1] >= 0
    xr = geo.cen[fc[inner, 1]]
    if mesh.period is not None and mesh.face_shift is not None:
        xr = xr + mesh.face_shift[inner] * np.asarray(mesh.period)[None, :]
    out[inner] = 1.0 / np.linalg.norm(xr - geo.cen[fc[inner, 0]], axis=1)
    return out


def face_viscous_fluxes(model, fs, U):
    """Integrated viscous face fluxes [nvar, nf] from the face states
    [2, nvar, NGPT] and the cells' polynomial gradients."""
    geo, mesh = model.geo, model.mesh
    grads = cell_gradients(model, U)                        # [N, NGPC, d, nvar]
    nv, d = model.nvar, model.d
    gf = np.zeros((2, geo.n_gp, d, nv))
    for c in range(mesh.n_cells):
        k = geo.c_ngp[c]
        gf[geo.c_side[c, :k], geo.c_gidx[c, :k]] = grads[c, :k]
    bnd = mesh.face_cells[:, 1] < 0
    face_of_gp = np.repeat(np.arange(mesh.n_faces), np.diff(geo.gp_off))
    gb = bnd[face_of_gp]
    gf[1, gb] = gf[0, gb]                                   # transmissive ghost: the left side again
    UL, UR = fs[0].T, fs[1].T
    n = geo.normal[face_of_gp]
    inv_l = face_inverse_distances(model)[face_of_gp]
    F = viscous_flux(UL, UR, gf[0], gf[1], n, inv_l, model.p)
    out = np.zeros((mesh.n_faces, nv))
    np.add.at(out, face_of_gp, F * geo.gp_wS[:, None])
    return out.T
