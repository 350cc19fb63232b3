"""Characteristic variables of the Euler equations for CWENOZ (test
infrastructure only: the oracle of the library's characteristic-variable
CWENOZ).

Section 2.3 lets the CWENOZ reconstruction act on characteristic, primitive
or conserved variables without fixing the details.  Reading taken here (the
usual one for unstructured WENO schemes): each face f of cell i has its own
projection, built from the eigenvectors of the flux Jacobian
A(U~, n) = d(F(U) . n)/dU in the face's unit normal n (outward from i), at
the Roe average U~ of the averages of i and of the cell across f (i itself
at a boundary face).  The stencil data are projected with the left
eigenvectors, W = L U; CWENOZ runs per characteristic field on W; the values
at the face's Gauss points are projected back with the right eigenvectors,
U(x) = U_i + R (W(x) - W_i).

Eigenvectors, for velocity u, sound speed c, total enthalpy H, u_n = u . n,
q2 = |u|^2, b1 = (gamma - 1) / c^2, b2 = b1 q2 / 2, and unit tangents t_1
(t_2) completing n to an orthonormal basis:

  right (columns)                    left (rows)
  (1, u - c n, H - c u_n)            ((b2 + u_n / c) / 2, -(b1 u + n / c) / 2, b1 / 2)
  (1, u, q2 / 2)                     (1 - b2, b1 u, -b1)
  (0, t_k, u . t_k)                  (-u . t_k, t_k, 0)
  (1, u + c n, H + c u_n)            ((b2 - u_n / c) / 2, -(b1 u - n / c) / 2, b1 / 2)

in the order acoustic (u_n - c), entropy, shear (t_1[, t_2]), acoustic
(u_n + c).  Tangents: t_1 = (-n_y, n_x) in 2D; in 3D t_1 = e x n / |e x n|
with e the coordinate axis of the smallest |n_k| (the first on a tie) and
t_2 = n x t_1.
"""
from __future__ import annotations

import numpy as np


def tangents(n):
    """Unit tangents [..., d-1, d] completing unit normals n [..., d]."""
    n = np.asarray(n, np.float64)
    d = n.shape[-1]
    if d == 2:
        return np.stack([-n[..., 1], n[..., 0]], -1)[..., None, :]
    k = np.argmin(np.abs(n), axis=-1)
    e = np.zeros_like(n)
    np.put_along_axis(e, k[..., None], 1.0, axis=-1)
    t1 = np.cross(e, n)
    t1 /= np.linalg.norm(t1, axis=-1, keepdims=True)
    t2 = np.cross(n, t1)
    return np.stack([t1, t2], -2)


def roe_average(UL, UR, gamma):
    """Roe-averaged velocity [..., d], total enthalpy and sound speed of
    conserved states UL, UR [..., d+2]."""
    def prim(U):
        r = U[..., 0]
        v = U[..., 1:-1] / r[..., None]
        p = (gamma - 1.0) * (U[..., -1] - 0.5 * r * (v ** 2).sum(-1))
        return r, v, (U[..., -1] + p) / r
    rL, vL, HL = prim(UL)
    rR, vR, HR = prim(UR)
    sL, sR = np.sqrt(rL), np.sqrt(rR)
    wL, wR = sL / (sL + sR), sR / (sL + sR)
    v = wL[..., None] * vL + wR[..., None] * vR
    H = wL * HL + wR * HR
    c = np.sqrt((gamma - 1.0) * (H - 0.5 * (v ** 2).sum(-1)))
    return v, H, c


def eigenvectors(v, H, c, n, gamma):
    """Right eigenvectors R [..., nv, nv] (columns) and left eigenvectors L
    [..., nv, nv] (rows) of A(n) at velocity v, enthalpy H, sound speed c,
    and the eigenvalues [..., nv], in the order of the module docstring."""
    v, n = np.asarray(v, np.float64), np.asarray(n, np.float64)
    d = n.shape[-1]
    nv = d + 2
    shape = n.shape[:-1]
    t = tangents(n)                                          # [..., d-1, d]
    un = (v * n).sum(-1)
    q2 = (v ** 2).sum(-1)
    b1 = (gamma - 1.0) / c ** 2
    b2 = 0.5 * b1 * q2
    R = np.zeros(shape + (nv, nv))
    L = np.zeros(shape + (nv, nv))
    lam = np.zeros(shape + (nv,))
    # acoustic u_n - c
    R[..., 0, 0] = 1.0
    R[..., 1:-1, 0] = v - c[..., None] * n
    R[..., -1, 0] = H - c * un
    L[..., 0, 0] = 0.5 * (b2 + un / c)
    L[..., 0, 1:-1] = -0.5 * (b1[..., None] * v + n / c[..., None])
    L[..., 0, -1] = 0.5 * b1
    lam[..., 0] = un - c
    # entropy
    R[..., 0, 1] = 1.0
    R[..., 1:-1, 1] = v
    R[..., -1, 1] = 0.5 * q2
    L[..., 1, 0] = 1.0 - b2
    L[..., 1, 1:-1] = b1[..., None] * v
    L[..., 1, -1] = -b1
    lam[..., 1] = un
    # shear waves
    for k in range(d - 1):
        tk = t[..., k, :]
        R[..., 1:-1, 2 + k] = tk
        R[..., -1, 2 + k] = (v * tk).sum(-1)
        L[..., 2 + k, 0] = -(v * tk).sum(-1)
        L[..., 2 + k, 1:-1] = tk
        lam[..., 2 + k] = un
    # acoustic u_n + c
    R[..., 0, -1] = 1.0
    R[..., 1:-1, -1] = v + c[..., None] * n
    R[..., -1, -1] = H + c * un
    L[..., -1, 0] = 0.5 * (b2 - un / c)
    L[..., -1, 1:-1] = -0.5 * (b1[..., None] * v - n / c[..., None])
    L[..., -1, -1] = 0.5 * b1
    lam[..., -1] = un + c
    return R, L, lam
