"""Pins of the oracle's viscous fluxes (Section 2: Eqs. Terms1,
sutherlandlaw, HeatConduct, Stresses; Section 2.4: Eq. viscous_jump)."""
import numpy as np
import pytest

from oracle import OracleModel, flux
from oracle.viscous import (viscous_flux, cell_gradients, face_viscous_fluxes, sutherland,
                            face_inverse_distances)
from paper_2510_25906_amd.inputs import configs, fields
from paper_2510_25906_amd.inputs.mesh import quad_tri_2d
from paper_2510_25906_amd.inputs.stencil import build_stencils
from paper_2510_25906_amd.inputs.params import Params, ALL_LINEAR

GAMMA = 1.4
VISC = dict(viscous=1, mu0=0.05, T0=0.8, sutherland_S=0.4, prandtl=0.72, visc_alpha=4.0 / 3.0)


def test_sutherland_law_closed_form():
    """mu(T0) = mu0, and the ratio of the viscosities at two temperatures
    written out from Eq. sutherlandlaw."""
    p = Params(**VISC)
    assert sutherland(np.array(p.T0), p) == pytest.approx(p.mu0, rel=1e-15)
    T1, T2 = 0.5, 2.0
    ratio = (T2 / T1) ** 1.5 * (T1 + p.sutherland_S) / (T2 + p.sutherland_S)
    assert sutherland(np.array(T2), p) / sutherland(np.array(T1), p) == pytest.approx(ratio, rel=1e-14)


def test_linear_velocity_field_gives_the_exact_stress():
    """Uniform density and pressure, velocity u = A x + b: the degree-2
    reconstruction is exact (E is quadratic), the two sides agree (no
    penalty), T is uniform, so at every face point F_v . n = (0, tau n,
    u . tau n) with tau = mu(T) (A + A^T - (2/3) tr A I), no heat flux."""
    mesh = quad_tri_2d(10, 10, lo=(-0.5, -0.5), hi=(0.5, 0.5), split=np.ones((10, 10), bool))
    st = build_stencils(mesh, 2)
    A = np.array([[0.3, -0.7], [0.4, 0.2]])
    b = np.array([0.5, -0.1])
    rho0, p0 = 1.3, 0.9

    def ev(x):
        u = x @ A.T + b
        return fields.prim_to_cons(np.concatenate([np.full(x.shape[:-1] + (1,), rho0), u,
                                                   np.full(x.shape[:-1] + (1,), p0)], -1))
    U = fields.cell_average(mesh, ev, nq=4)
    p = Params(order_r=2, scheme_mode=ALL_LINEAR, **VISC)
    om = OracleModel(mesh, st, p)
    fs, _ = om.reconstruct(U)
    geo = om.geo
    face_of_gp = np.repeat(np.arange(mesh.n_faces), np.diff(geo.gp_off))
    inner = mesh.face_cells[face_of_gp, 1] >= 0
    grads = cell_gradients(om, U)
    gf = np.zeros((2, geo.n_gp, 2, 4))
    for c in range(mesh.n_cells):
        k = geo.c_ngp[c]
        gf[geo.c_side[c, :k], geo.c_gidx[c, :k]] = grads[c, :k]
    n = geo.normal[face_of_gp]
    F = viscous_flux(fs[0].T[inner], fs[1].T[inner], gf[0][inner], gf[1][inner], n[inner],
                     face_inverse_distances(om)[face_of_gp][inner], p)
    x = geo.gp_x[inner]
    mu = sutherland(np.array(p0 / rho0), p)
    tau = mu * (A + A.T - (2.0 / 3.0) * np.trace(A) * np.eye(2))
    want_m = n[inner] @ tau.T
    u = x @ A.T + b
    want_E = (u * want_m).sum(1)
    assert np.abs(F[:, 0]).max() == 0.0
    assert np.abs(F[:, 1:3] - want_m).max() <= 1e-11
    assert np.abs(F[:, 3] - want_E).max() <= 1e-11


@pytest.mark.parametrize("alpha", [4.0 / 3.0, 0.5])
def test_penalty_term_on_a_velocity_jump(alpha):
    """Zero gradients on both sides and a momentum jump dm at equal density
    and pressure: the face gradient is alpha / L (U_R - U_L) n, so
    tau n = mu alpha / (L rho) (dm + (n . dm) n / 3), the pressure gradient
    vanishes (no heat flux) and the work term is u_mean . tau n."""
    rng = np.random.default_rng(0)
    p = Params(**dict(VISC, visc_alpha=alpha))
    for d in (2, 3):
        n = rng.normal(size=(20, d))
        n /= np.linalg.norm(n, axis=1, keepdims=True)
        rho, pr = 1.1, 0.7
        uL = rng.normal(size=(20, d))
        uR = rng.normal(size=(20, d))
        mk = lambda u: np.stack([fields.prim_to_cons(np.concatenate([[rho], ui, [pr]])) for ui in u])
        UL, UR = mk(uL), mk(uR)
        inv_l = rng.uniform(5, 50, 20)
        zero = np.zeros((20, d, d + 2))
        F = viscous_flux(UL, UR, zero, zero, n, inv_l, p)
        dm = (UR - UL)[:, 1:-1]
        um = 0.5 * (UL + UR)[:, 1:-1] / rho
        Tm = (GAMMA - 1) * (0.5 * (UL + UR)[:, -1] - 0.5 * rho * (um ** 2).sum(1)) / rho
        mu = sutherland(Tm, p)
        want = (mu * alpha * inv_l / rho)[:, None] * (dm + ((n * dm).sum(1) / 3.0)[:, None] * n)
        assert np.abs(F[:, 1:-1] - want).max() <= 1e-12 * np.abs(want).max()
        # equal pressures: no conduction; the energy flux is the work of the stress
        assert np.abs(F[:, -1] - (um * want).sum(1)).max() <= 1e-12 * np.abs(want).max()


def test_constant_state_has_no_viscous_flux_and_residual_telescopes():
    w = configs.c1_density_jump(8, 2)
    p = w.params.with_(**VISC)
    om = OracleModel(w.mesh, w.stencils, p)
    Uc = np.tile(fields.prim_to_cons(np.array([1.3, 0.4, -0.2, 2.0])), (w.mesh.n_cells, 1))
    fs, _ = om.reconstruct(Uc)
    assert np.abs(face_viscous_fluxes(om, fs, Uc)).max() <= 1e-15
    fs, _ = om.reconstruct(w.U)
    Rv = flux.residual_from_face_fluxes(om, -face_viscous_fluxes(om, fs, w.U))
    vol = om.geo.vol
    assert np.abs((Rv * vol).sum(1)).max() <= 1e-13 * np.abs(Rv * vol).sum()
    assert np.abs(Rv).max() > 0


@pytest.mark.parametrize("r", [2, 3])
def test_viscous_residual_converges_to_the_exact_divergence(r):
    """Periodic shear layer u = (U0 sin(2 pi y), 0), rho and p uniform: the
    inviscid flux divergence vanishes and the viscous one is exactly
    (0, mu u'', 0, mu (u'^2 + u u'')) with constant mu.  The viscous part of
    the residual matches its cell averages, the error falling at order >= r - 1
    (second derivatives of a degree-r reconstruction) under refinement."""
    U0, rho0, p0 = 0.4, 1.0, 1.0
    k = 2 * np.pi
    p = Params(order_r=r, **dict(VISC, T0=p0 / rho0))
    mu = p.mu0

    def ev(x):
        y = x[..., 1]
        u = np.stack([U0 * np.sin(k * y), np.zeros_like(y)], -1)
        return fields.prim_to_cons(np.concatenate([np.full(y.shape + (1,), rho0), u,
                                                   np.full(y.shape + (1,), p0)], -1))

    def exact(x):
        y = x[..., 1]
        u, du, d2u = U0 * np.sin(k * y), U0 * k * np.cos(k * y), -U0 * k * k * np.sin(k * y)
        return np.stack([np.zeros_like(y), mu * d2u, np.zeros_like(y), mu * (du * du + u * d2u)], -1)

    errs = []
    for n in (16, 32, 64):
        w = configs.c1_density_jump(n, r, jump=False)
        U = fields.cell_average(w.mesh, ev, nq=r + 3)
        om = OracleModel(w.mesh, w.stencils, p.with_(order_r=r))
        fs, _ = om.reconstruct(U)
        Rv = flux.residual_from_face_fluxes(om, -face_viscous_fluxes(om, fs, U))
        want = fields.cell_average(w.mesh, exact, nq=r + 3).T
        errs.append(np.abs(Rv - want).max() / np.abs(want).max())
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print(f"r={r}: errors {errs}, orders {order}")
    assert np.all(np.diff(errs) < 0)
    assert order[-1] >= r - 1 - 0.3      # measured: 1.0 at r = 2, 3.0 at r = 3
