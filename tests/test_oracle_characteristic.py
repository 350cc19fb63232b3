"""Pins of the oracle's characteristic-variable CWENOZ (Section 2.3: CWENOZ
on characteristic variables; eigenvectors of the Euler flux Jacobian)."""
import numpy as np
import pytest

from oracle import OracleModel
from oracle.characteristic import tangents, roe_average, eigenvectors
from paper_2510_25906_amd.inputs import configs, fields
from paper_2510_25906_amd.inputs.params import CHARACTERISTIC, ALL_CWENOZ, ALL_LINEAR

GAMMA = 1.4


def normal_flux(U, n):
    """F(U) . n of the Euler equations, written out from their definition."""
    r = U[..., 0]
    m = U[..., 1:-1]
    E = U[..., -1]
    v = m / r[..., None]
    p = (GAMMA - 1.0) * (E - 0.5 * (m * v).sum(-1))
    un = (v * n).sum(-1)
    return np.concatenate([(r * un)[..., None], m * un[..., None] + p[..., None] * n,
                           ((E + p) * un)[..., None]], -1)


def random_states(rng, d, k):
    prim = np.column_stack([rng.uniform(0.3, 3.0, k)] + [rng.uniform(-2, 2, k) for _ in range(d)]
                           + [rng.uniform(0.2, 5.0, k)])
    U = np.stack([fields.prim_to_cons(q) for q in prim])
    n = rng.normal(size=(k, d))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    return U, n


def state_eigen(U, n):
    r = U[:, 0]
    v = U[:, 1:-1] / r[:, None]
    p = (GAMMA - 1.0) * (U[:, -1] - 0.5 * r * (v ** 2).sum(1))
    H = (U[:, -1] + p) / r
    c = np.sqrt(GAMMA * p / r)
    return v, H, c


@pytest.mark.parametrize("d", [2, 3])
def test_left_and_right_eigenvectors_are_inverse_and_diagonalise_the_jacobian(d):
    """L R = I, and R diagonalises the Jacobian of F . n taken by central
    differences of the flux itself: A R = R diag(lambda)."""
    rng = np.random.default_rng(0)
    U, n = random_states(rng, d, 50)
    v, H, c = state_eigen(U, n)
    R, L, lam = eigenvectors(v, H, c, n, GAMMA)
    eye = np.eye(d + 2)
    assert np.abs(L @ R - eye).max() <= 1e-12
    for i in range(U.shape[0]):
        A = np.zeros((d + 2, d + 2))
        for j in range(d + 2):
            h = 1e-6 * max(1.0, abs(U[i, j]))
            e = np.zeros(d + 2)
            e[j] = h
            A[:, j] = (normal_flux(U[i] + e, n[i]) - normal_flux(U[i] - e, n[i])) / (2 * h)
        scale = np.abs(A).max()
        assert np.abs(A @ R[i] - R[i] * lam[i][None, :]).max() <= 1e-7 * scale
    # eigenvalues: u_n - c, u_n (d times), u_n + c
    un = (v * n).sum(1)
    assert np.allclose(lam[:, 0], un - c) and np.allclose(lam[:, -1], un + c)
    assert np.allclose(lam[:, 1:-1], un[:, None])


@pytest.mark.parametrize("d", [2, 3])
def test_tangents_complete_an_orthonormal_basis(d):
    rng = np.random.default_rng(1)
    n = rng.normal(size=(40, d))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    n[0] = np.eye(d)[0]                       # axis-aligned normals too
    n[1] = -np.eye(d)[d - 1]
    B = np.concatenate([n[:, None, :], tangents(n)], 1)          # [k, d, d]
    assert np.abs(np.einsum("kij,klj->kil", B, B) - np.eye(d)).max() <= 1e-14


@pytest.mark.parametrize("d", [2, 3])
def test_roe_average_satisfies_the_roe_property(d):
    """The Jacobian R diag(lambda) L at the Roe average maps the jump in the
    states onto the jump in the normal fluxes, exactly:
    F(U_R) . n - F(U_L) . n = A~ (U_R - U_L)."""
    rng = np.random.default_rng(2)
    UL, n = random_states(rng, d, 60)
    UR, _ = random_states(rng, d, 60)
    v, H, c = roe_average(UL, UR, GAMMA)
    R, L, lam = eigenvectors(v, H, c, n, GAMMA)
    A = R @ (lam[..., None] * L)
    jump = normal_flux(UR, n) - normal_flux(UL, n)
    got = np.einsum("kij,kj->ki", A, UR - UL)
    assert np.abs(got - jump).max() <= 1e-11 * np.abs(jump).max()
    # the Roe average of a state with itself is the state
    v2, H2, c2 = roe_average(UL, UL, GAMMA)
    v0, H0, c0 = state_eigen(UL, n)
    assert np.allclose(v2, v0, rtol=0, atol=1e-13) and np.allclose(c2, c0, rtol=1e-13)


def _smooth_2d(n=16, r=2):
    w = configs.c1_density_jump(n, r, jump=False)
    return w


def test_identity_projection_reduces_to_conserved_cwenoz():
    """With L = R = I the face-by-face characteristic path is the conserved
    one, at every Gauss point (checks the per-face plumbing: slots, faces,
    projection and back-projection)."""
    w = configs.c1_density_jump(16, 3)
    p = w.params.with_(scheme_mode=ALL_CWENOZ)
    om = OracleModel(w.mesh, w.stencils, p)
    cells = np.arange(w.mesh.n_cells)
    fv_c, _ = om.cwenoz(cells, w.U)
    ident = lambda UL, UR, n: (np.broadcast_to(np.eye(4), UL.shape[:-1] + (4, 4)),) * 2
    fv_i, _ = om.cwenoz_characteristic(cells, w.U, eig=ident)
    valid = np.arange(fv_c.shape[1])[None, :] < om.geo.c_ngp[:, None]
    assert np.abs(np.where(valid[..., None], fv_i - fv_c, 0)).max() <= 1e-13


def test_single_entropy_wave_projects_onto_one_field():
    """An entropy wave (density varying, velocity and pressure uniform):
    every stencil difference lies along the entropy eigenvector, so its
    characteristic differences vanish in every other field, and the
    characteristic reconstruction moves only the entropy field (the face
    values then keep velocity and pressure uniform)."""
    mesh = configs.c1_density_jump(16, 2).mesh
    u, v, pr = 0.7, -0.3, 2.0
    ev = lambda x: fields.prim_to_cons(np.stack([1.0 + 0.3 * np.sin(2 * np.pi * x[..., 0])
                                                 * np.cos(2 * np.pi * x[..., 1]),
                                                 np.full(x.shape[:-1], u), np.full(x.shape[:-1], v),
                                                 np.full(x.shape[:-1], pr)], -1))
    U = fields.cell_average(mesh, ev, nq=5)
    w = configs.c1_density_jump(16, 2)
    om = OracleModel(mesh, w.stencils, w.params.with_(scheme_mode=ALL_CWENOZ, cweno_vars=CHARACTERISTIC))
    # the velocity of the averages is uniform only to quadrature accuracy: take
    # a field whose averages are exactly of the wave's form
    prim = np.column_stack([U[:, 0], np.full(len(U), u), np.full(len(U), v), np.full(len(U), pr)])
    U = np.stack([fields.prim_to_cons(q) for q in prim])
    vr, H, c = roe_average(U[:5], U[5:10], GAMMA)
    nrm = np.tile([[0.6, 0.8]], (5, 1))
    R, L, _ = eigenvectors(vr, H, c, nrm, GAMMA)
    dW = np.einsum("kij,kj->ki", L, U[5:10] - U[:5])
    assert np.abs(dW[:, [0, 2, 3]]).max() <= 1e-14 * np.abs(dW[:, 1]).max()
    cells = np.arange(mesh.n_cells)
    fv, info = om.cwenoz_characteristic(cells, U)
    valid = np.arange(fv.shape[1])[None, :] < om.geo.c_ngp[:, None]
    vel = fv[..., 1:3] / fv[..., :1]
    pres = (GAMMA - 1) * (fv[..., 3] - 0.5 * (fv[..., 1:3] ** 2).sum(-1) / fv[..., 0])
    assert np.abs(np.where(valid[..., None], vel - np.array([u, v]), 0)).max() <= 1e-12
    assert np.abs(np.where(valid, pres - pr, 0)).max() <= 1e-12
    # the non-entropy fields carry no data: their smoothness indicators vanish
    assert np.abs(info["SI1"][..., [0, 2, 3]]).max() <= 1e-20


@pytest.mark.parametrize("r", [2, 3])
def test_characteristic_cwenoz_is_linear_on_affine_data(r):
    """On affine conserved data every candidate polynomial of every face's
    characteristic fields is the same affine function, so SI_s are equal,
    tau = 0, the weights are the linear weights and the face values are the
    linear reconstruction's (both exact)."""
    w = configs.c1_density_jump(12, r)
    rng = np.random.default_rng(4)
    A = rng.normal(size=(2, 4)) * 0.05
    b = np.array([1.2, 0.3, -0.2, 2.5])
    ev = lambda x: b + x @ A
    U = fields.cell_average(w.mesh, ev, nq=r + 2)
    # a non-periodic affine field on the periodic mesh: use interior cells only
    om = OracleModel(w.mesh, w.stencils, w.params.with_(scheme_mode=ALL_CWENOZ, cweno_vars=CHARACTERISTIC))
    c = om.geo.cen
    stc = w.stencils.central
    span = np.abs(c[stc] - c[:, None, :]).max(axis=(1, 2))
    cells = np.nonzero(span < 0.3)[0]
    assert cells.size > 20
    fv, info = om.cwenoz_characteristic(cells, U)
    _, fl, _ = om.linear(cells, U)
    valid = np.arange(fv.shape[1])[None, :] < om.geo.c_ngp[cells][:, None]
    assert np.abs(np.where(valid[..., None], fv - fl, 0)).max() <= 1e-12
    for s in range(fv.shape[1]):
        ok = valid[:, s]
        assert np.abs(info["om1"][ok, s] - (1 - 1 / w.params.lambda1_prime)).max() <= 1e-12


def test_characteristic_cwenoz_preserves_a_constant_state():
    w = configs.c1_density_jump(8, 2)
    U = np.tile(fields.prim_to_cons(np.array([1.3, 0.4, -0.2, 2.0])), (w.mesh.n_cells, 1))
    om = OracleModel(w.mesh, w.stencils, w.params.with_(scheme_mode=ALL_CWENOZ, cweno_vars=CHARACTERISTIC))
    cells = np.arange(w.mesh.n_cells)
    fv, _ = om.cwenoz_characteristic(cells, U)
    valid = np.arange(fv.shape[1])[None, :] < om.geo.c_ngp[:, None]
    assert np.abs(np.where(valid[..., None], fv - U[:, None, :], 0)).max() <= 1e-14
