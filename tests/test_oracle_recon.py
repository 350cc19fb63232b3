"""Pins of the oracle's reconstruction steps (Sections 2.1-2.5)."""
import numpy as np
import pytest

from oracle import OracleModel, flux
from oracle.reconstruction import monomials, LIN, CW, MU, FO
from paper_2510_25906_amd.inputs import configs, fields
from paper_2510_25906_amd.inputs.mesh import quad_tri_2d, hex_3d, mixed_box, TET, PYR, PRISM, HEX
from paper_2510_25906_amd.inputs.stencil import build_stencils
from paper_2510_25906_amd.inputs.params import Params, preset, ALL_CWENOZ, ALL_MUSCL, ALL_LINEAR


def mixed_2d(n=12, frac=0.4, seed=0):
    rng = np.random.default_rng(seed)
    return quad_tri_2d(n, n, lo=(-0.5, -0.5), hi=(0.5, 0.5), split=rng.random((n, n)) < frac)


def interior_cells(model, margin):
    """Cells whose whole central stencil is at least ``margin`` cells away from the boundary."""
    c = model.geo.cen
    lo, hi = c.min(0), c.max(0)
    span = (hi - lo).max()
    return np.nonzero(np.all((c > lo + margin * span) & (c < hi - margin * span), axis=1))[0]


@pytest.mark.parametrize("case", [("mixed2d", 2), ("mixed2d", 3), ("hex3d", 2), ("hex3d", 3), ("mixed3d", 2),
                                  ("mixed3d", 3)])
def test_polynomial_exactness(case):
    """Cell averages of a degree-r polynomial reproduce it exactly at the face points
    (the mixed 3D box has tetrahedra, pyramids, prisms and hexahedra)."""
    kind, r = case
    if kind == "mixed2d":
        mesh = mixed_2d(12)
    elif kind == "mixed3d":
        mesh = mixed_box(10, 5, 5, core=(3, 7), prism_layers=2, jitter=0.2, seed=0)
        assert set(np.unique(mesh.cell_type)) == {TET, PYR, PRISM, HEX}
    else:
        mesh = hex_3d(7, 7, 7, lo=(-1, -1, -1), hi=(1, 1, 1))
    st = build_stencils(mesh, r)
    d = mesh.dim
    _, _, ev = fields.random_polynomial(d, r, d + 2, seed=3)
    U = fields.cell_average(mesh, ev, nq=r + 2)
    om = OracleModel(mesh, st, Params(order_r=r))
    cells = np.arange(mesh.n_cells)
    _, fv, _ = om.linear(cells, U)
    for i, c in enumerate(cells):
        k = om.geo.c_ngp[c]
        exact = ev(om.geo.c_x[c, :k])
        assert np.allclose(fv[i, :k], exact, rtol=1e-9, atol=1e-9 * np.abs(exact).max())


def test_basis_means_vanish_by_independent_quadrature():
    """int over V_0' of phi_k = 0 (Section 2.1), checked with a Gauss rule."""
    mesh = mixed_2d(6)
    st = build_stencils(mesh, 3)
    om = OracleModel(mesh, st, Params(order_r=3))
    for t in (0, 1):
        cells = np.nonzero(mesh.cell_type == t)[0][:5]
        pts, w = fields.cell_quadrature(mesh, cells, 5)
        tab = om.tables(cells)
        xi = (pts - om.geo.cen[cells][:, None, :]) / om.geo.h[cells][:, None, None]
        phi = monomials(xi, om.exps) - tab["psibar"][:, None, :]
        integ = np.einsum("cqk,cq->ck", phi, w)
        assert np.abs(integ).max() < 1e-13


def test_smoothness_indicator_by_hand():
    """SI of p = xi1^2 + 3 xi1 xi2 (Eq. SI1, reference-frame derivatives)."""
    mesh = mixed_2d(6)
    st = build_stencils(mesh, 2)
    om = OracleModel(mesh, st, Params(order_r=2))
    cells = np.array([0, 7, 20])
    tab = om.tables(cells)
    # coefficients in the hierarchical basis (xi1, xi2, xi1^2, xi1 xi2, xi2^2)
    a = np.array([0.0, 0.0, 1.0, 3.0, 0.0])
    si_oracle = np.einsum("k,nkq,q->n", a, tab["OI"], a)
    for i, c in enumerate(cells):
        pts, w = fields.cell_quadrature(mesh, np.array([c]), 6)
        xi = (pts[0] - om.geo.cen[c]) / om.geo.h[c]
        wx = w[0] / om.geo.h[c] ** 2
        x1, x2 = xi[:, 0], xi[:, 1]
        integrand = (2 * x1 + 3 * x2) ** 2 + (3 * x1) ** 2 + 2.0 ** 2 + 3.0 ** 2 + 0.0
        assert si_oracle[i] == pytest.approx((integrand * wx).sum(), rel=1e-12)


def test_cwenoz_reduces_to_linear_on_affine_data():
    """Affine data: every candidate polynomial is the same plane, so SI_s are equal,
    tau = 0 and the nonlinear weights are the linear weights (Section 2.3)."""
    mesh = mixed_2d(10)
    st = build_stencils(mesh, 3)
    g = np.array([[0.3, -1.2, 0.7, 2.0], [1.1, 0.4, -0.5, 0.2]])
    U = fields.cell_average(mesh, lambda p: np.array([2.0, 0.5, -0.3, 7.0]) + p @ g, nq=3)
    om = OracleModel(mesh, st, Params(order_r=3, scheme_mode=ALL_CWENOZ))
    cells = interior_cells(om, 0.25)
    fv_cw, info = om.cwenoz(cells, U)
    _, fv_lin, _ = om.linear(cells, U)
    assert np.allclose(info["om1"], info["lam1"], rtol=0, atol=1e-12)
    nd = st.n_dir[cells]
    assert np.allclose(info["oms"][:, :3], (info["lams"])[:, None, None], atol=1e-12)
    assert np.allclose(fv_cw, fv_lin, atol=1e-11)


def test_cwenoz_weights_convex_and_mean_preserving():
    """Sum of the weights is one, each weight is non-negative, the combined
    polynomial keeps the cell average (Section 2.3: every basis function has
    zero mean over the cell), and across the jump the central weight drops."""
    w = configs.c1_density_jump(16, 2)
    om = OracleModel(w.mesh, w.stencils, w.params.with_(scheme_mode=ALL_CWENOZ))
    cells = np.arange(w.mesh.n_cells)
    fv, info = om.cwenoz(cells, w.U)
    tot = info["om1"] + info["oms"].sum(1)
    assert np.allclose(tot, 1.0, atol=1e-14)
    assert info["om1"].min() >= 0 and info["oms"].min() >= 0
    # mean over the cell of U_i + sum_k a_k phi_k by a Gauss rule of its own
    sel = cells[::7]
    pts, wq = fields.cell_quadrature(w.mesh, sel, 5)
    tab = om.tables(sel)
    xi = (pts - om.geo.cen[sel][:, None, :]) / om.geo.h[sel][:, None, None]
    phi = monomials(xi, om.exps) - tab["psibar"][:, None, :]
    vals = w.U[sel][:, None, :] + np.einsum("cqk,ckv->cqv", phi, info["a_cw"][sel])
    mean = np.einsum("cqv,cq->cv", vals, wq) / wq.sum(1)[:, None]
    assert np.abs(mean - w.U[sel]).max() < 1e-13 * np.abs(w.U).max()
    # the solution varies across the jump: the weights move off the linear ones
    assert np.abs(info["om1"] - info["lam1"]).max() > 1e-3
    # across the jump the central weight must drop well below lambda_1
    assert info["om1"].min() < 0.5


def _weight_deviation(n, b):
    """Largest |omega - lambda| over the cells and their valid stencils of the
    smooth periodic field, and the largest tau, on the n x n triangle mesh."""
    w = configs.c1_density_jump(n, 2, jump=False)
    om = OracleModel(w.mesh, w.stencils, w.params.with_(scheme_mode=ALL_CWENOZ, b_w=b))
    cells = np.arange(w.mesh.n_cells)
    _, info = om.cwenoz(cells, w.U)
    valid = np.arange(info["oms"].shape[1])[None, :] < w.stencils.n_dir[cells][:, None]
    dev = max(np.abs(info["om1"] - info["lam1"]).max(),
              np.abs(info["oms"] - info["lams"][:, None, None])[valid].max())
    return dev, info["tau"].max(), info["SI1"].max()


def test_cwenoz_weights_converge_to_linear_weights():
    """On smooth data the nonlinear weights tend to the linear weights
    (Section 2.3) at a rate fixed by the exponent b.

    In the reference frame the degree-1 directional fits and the central fit
    agree on the gradient to O(h^2), so every SI is h^2 |grad u|^2 + O(h^3)
    and tau = mean |SI_s - SI_1| = O(h^3); with eps fixed, the ratio
    tau / (eps + SI_s) is O(h^3) and the weights' departure from lambda,
    which is O(ratio^b), falls at rate >= 3 b under refinement."""
    ns = (16, 32, 64)
    for b, use in ((4.0, (16, 32)), (2.0, ns)):
        devs, taus, sis = zip(*[_weight_deviation(n, b) for n in use])
        rate_tau = np.log2(np.array(taus[:-1]) / np.array(taus[1:]))
        rate_si = np.log2(np.array(sis[:-1]) / np.array(sis[1:]))
        rate_w = np.log2(np.array(devs[:-1]) / np.array(devs[1:]))
        assert np.all(rate_tau > 2.9), rate_tau
        assert np.all(rate_si > 1.5) and np.all(rate_si < 2.5), rate_si
        assert np.all(rate_w >= 3 * b), (b, rate_w)


def test_nad_smooth_vortex_all_linear():
    """Section 3.1 and Table 1: no troubled cells on the smooth isentropic vortex."""
    for n in (16, 32, 64):
        w = configs.vortex_2d(n, 2)
        om = OracleModel(w.mesh, w.stencils, w.params)
        cls, _ = om.cell_classes(np.arange(w.mesh.n_cells), w.U)
        assert np.all(cls == LIN)


def test_nad_step_tags_jump_cells():
    w = configs.c1_density_jump(32, 2)
    mesh = w.mesh
    om = OracleModel(mesh, w.stencils, w.params)
    cells = np.arange(mesh.n_cells)
    cls, extra = om.cell_classes(cells, w.U)
    # faces on the jump x = 0.5 (and the periodic wrap x = 0)
    fx = np.array([mesh.vertices[mesh.face_vertices(f)][:, 0] for f in range(mesh.n_faces)])
    on_jump = np.all(np.isclose(fx, 0.5), 1) | np.all(np.isclose(fx, 0.0), 1) | np.all(np.isclose(fx, 1.0), 1)
    touching = np.unique(mesh.face_cells[on_jump].ravel())
    assert np.all(cls[touching] >= CW)
    # preset (d): linear and MUSCL only, the jump cells are MUSCL
    om_d = OracleModel(mesh, w.stencils, w.params.with_(**dict(preset("d_linear_muscl").__dict__,
                                                              order_r=2)))
    cls_d, _ = om_d.cell_classes(cells, w.U)
    assert np.all(cls_d[touching] == MU)
    assert not np.any(cls_d == CW)
    # dilation: a cell's class is at least its face neighbours' own class
    own = extra["own"]
    for j in range(om.nbr.shape[1]):
        nb = om.nbr[:, j]
        ok = nb >= 0
        assert np.all(cls[ok] >= own[nb[ok]])


@pytest.mark.parametrize("name", ["c_linear_cwenoz", "d_linear_muscl", "e_muscl_cwenoz"])
def test_nad_presets(name):
    """Section 2.5, Fig. NADMargin (c)-(e): each two-scheme preset removes one scheme."""
    w = configs.c2_riemann(24, 3)
    cells = np.arange(w.mesh.n_cells)
    om = OracleModel(w.mesh, w.stencils, preset(name, order_r=3, kappa=0.0))
    own, info = om.own_class(cells, w.U)
    cls, _ = om.cell_classes(cells, w.U)
    if name == "c_linear_cwenoz":
        assert not np.any(cls == MU) and np.any(cls == CW)
    if name == "d_linear_muscl":
        assert not np.any(cls == CW) and np.any(cls == MU)
    if name == "e_muscl_cwenoz":
        # no linear cell unless every variable sits exactly at its interval midpoint
        assert not np.any(own == LIN)


def test_muscl_bj_bounds_and_affine_exactness():
    w = configs.c1_density_jump(16, 2)
    om = OracleModel(w.mesh, w.stencils, w.params.with_(scheme_mode=ALL_MUSCL))
    cells = np.arange(w.mesh.n_cells)
    fv, info = om.muscl(cells, w.U)
    m, M = om.nad_bounds(cells, w.U)
    assert np.all(fv >= m[:, None, :] - 1e-14) and np.all(fv <= M[:, None, :] + 1e-14)
    assert np.all((info["theta"] >= 0) & (info["theta"] <= 1))
    # uniform quads + affine data: the limiter is inactive
    mesh = quad_tri_2d(8, 8, lo=(0, 0), hi=(1, 1))
    st = build_stencils(mesh, 2)
    U = fields.cell_average(mesh, lambda p: np.array([1.0, 0.2, 0.1, 3.0]) + p @ np.array(
        [[0.5, 0.1, 0.0, 1.0], [0.25, 0.0, 0.3, -0.5]]), nq=3)
    om2 = OracleModel(mesh, st, Params(order_r=2, scheme_mode=ALL_MUSCL))
    inner = interior_cells(om2, 0.1)
    _, info2 = om2.muscl(inner, U)
    assert np.allclose(info2["theta"], 1.0, atol=1e-12)


def test_harten_check_and_first_order_fallback():
    w = configs.c1_density_jump(16, 2)
    U = w.U.copy()
    U[37, 0] = -0.5  # non-physical density in one cell
    om = OracleModel(w.mesh, w.stencils, w.params)
    fv, cls = om.reconstruct_cells(np.arange(w.mesh.n_cells), U)
    assert cls[37] == FO
    assert np.all(fv[37, :om.geo.c_ngp[37]] == U[37])
    # every accepted reconstruction satisfies the bound on density and pressure
    ok = cls != FO
    g = w.params.gamma
    rho = fv[..., 0]
    rb = U[:, 0][:, None]
    valid = np.arange(fv.shape[1])[None, :] < om.geo.c_ngp[:, None]
    assert np.all(~valid[ok] | (np.abs(rho - rb)[ok] <= 0.9 * np.abs(rb)[ok] + 1e-15))


def test_free_stream_preservation():
    w = configs.c2_riemann(16, 3)
    U = np.tile(fields.prim_to_cons(np.array([1.3, 0.4, -0.2, 2.0])), (w.mesh.n_cells, 1))
    om = OracleModel(w.mesh, w.stencils, w.params)
    R, fs, cls = flux.residual(om, U)
    assert np.all(cls == LIN)
    assert np.allclose(fs, U[0][None, :, None], rtol=0, atol=1e-13)
    assert np.abs(R).max() < 1e-12


def test_free_stream_on_mixed_3d_box():
    """A uniform state gives zero residual on every element type: each cell's
    face normals weighted by area close (including pyramid apex faces and
    prism sides), and the transmissive boundary ghost equals the state."""
    w = configs.c4_mixed("small")
    U = np.tile(fields.prim_to_cons(np.array([1.3, 0.4, -0.2, 0.3, 2.0])), (w.mesh.n_cells, 1))
    om = OracleModel(w.mesh, w.stencils, w.params)
    R, fs, cls = flux.residual(om, U)
    assert np.all(cls == LIN)
    assert np.abs(R).max() < 1e-11


def test_conservation_telescopes_on_periodic_mesh():
    for w in (configs.c1_density_jump(16, 2), configs.vortex_2d(16, 3)):
        om = OracleModel(w.mesh, w.stencils, w.params)
        R, _, _ = flux.residual(om, w.U)
        tot = (R * om.geo.vol[None, :]).sum(1)
        assert np.abs(tot).max() < 1e-12 * np.abs(R * om.geo.vol).max() * w.mesh.n_cells


@pytest.mark.parametrize("r", [2, 3])
def test_convergence_order_smooth(r):
    """Face-state error against exact point values decays at order r + 1."""
    errs = []
    ns = (16, 32, 64)
    for n in ns:
        w = configs.c1_density_jump(n, r, jump=False)
        om = OracleModel(w.mesh, w.stencils, w.params.with_(scheme_mode=ALL_LINEAR))
        cells = np.arange(w.mesh.n_cells)
        _, fv, _ = om.linear(cells, w.U)
        ex = fields.density_jump_2d(om.geo.c_x, jump=False)
        e = np.abs(fv - ex)[..., 0]
        errs.append(e.max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders[-1] > r + 1 - 0.3


def test_independent_least_squares_brute_force():
    """The linear coefficients equal a least-squares solve assembled with a Gauss
    rule instead of the exact simplex integrals, and solved by QR."""
    mesh = mixed_2d(8)
    r = 3
    st = build_stencils(mesh, r)
    rng = np.random.default_rng(11)
    U = rng.normal(size=(mesh.n_cells, 4))
    om = OracleModel(mesh, st, Params(order_r=r))
    cells = np.array([5, 30, 41])
    a, fv, tab = om.linear(cells, U)
    for i, c in enumerate(cells):
        xc, h = om.geo.cen[c], om.geo.h[c]
        pts0, w0 = fields.cell_quadrature(mesh, np.array([c]), 6)
        xi0 = (pts0[0] - xc) / h
        w0 = w0[0] / h ** 2
        mean = (monomials(xi0, om.exps) * w0[:, None]).sum(0) / w0.sum()
        rows, rhs = [], []
        for m in st.central[c]:
            pts, wq = fields.cell_quadrature(mesh, np.array([m]), 6)
            xi = (pts[0] - xc) / h
            wq = wq[0] / h ** 2
            rows.append(((monomials(xi, om.exps) - mean) * wq[:, None]).sum(0))
            rhs.append(wq.sum() * (U[m] - U[c]))
        A = np.array(rows)
        q_, r_ = np.linalg.qr(A)
        sol = np.linalg.solve(r_, q_.T @ np.array(rhs))
        assert np.allclose(sol, a[i], rtol=1e-10, atol=1e-10 * np.abs(sol).max())


def test_rankine_hugoniot_matches_paper_post_shock_state():
    path = __file__.replace("test_oracle_recon.py", "golden/shu_osher_post_shock.txt")
    rho, u, p = np.loadtxt(path)
    r2, u2, p2 = fields.rankine_hugoniot(3.0)
    assert r2 == pytest.approx(rho, abs=1e-6)
    assert u2 == pytest.approx(u, abs=1e-6)
    assert p2 == pytest.approx(p, abs=1e-4)


def test_riemann_states_match_paper():
    path = __file__.replace("test_oracle_recon.py", "golden/riemann_2d_states.txt")
    rows = [l.split() for l in open(path) if not l.startswith("#")]
    for key, *vals in rows:
        assert tuple(float(v) for v in vals) == fields.RIEMANN_2D[key]


def test_hllc_hll_consistency_and_symmetry():
    rng = np.random.default_rng(4)
    for d in (2, 3):
        prim = np.concatenate([rng.uniform(0.5, 2, (50, 1)), rng.normal(size=(50, d)),
                               rng.uniform(0.5, 2, (50, 1))], 1)
        UL = fields.prim_to_cons(prim)
        prim2 = prim * rng.uniform(0.8, 1.2, prim.shape)
        UR = fields.prim_to_cons(prim2)
        n = rng.normal(size=(50, d))
        n /= np.linalg.norm(n, axis=1, keepdims=True)
        for fn in (flux.hllc, flux.hll):
            assert np.allclose(fn(UL, UL, n, 1.4), flux.euler_flux(UL, n, 1.4), rtol=1e-13, atol=1e-13)
            assert np.allclose(fn(UL, UR, n, 1.4), -fn(UR, UL, -n, 1.4), rtol=1e-12, atol=1e-12)
        # supersonic to the right: the upwind (left) flux
        prim_s = prim.copy()
        prim_s[:, 1:1 + d] = 10.0 * n
        prim_s2 = prim2.copy()
        prim_s2[:, 1:1 + d] = 10.0 * n
        Ls, Rs = fields.prim_to_cons(prim_s), fields.prim_to_cons(prim_s2)
        for fn in (flux.hllc, flux.hll):
            assert np.allclose(fn(Ls, Rs, n, 1.4), flux.euler_flux(Ls, n, 1.4), rtol=1e-13)


def _subsonic_states(rng, d, n):
    prim = np.concatenate([rng.uniform(0.5, 2, (n, 1)), 0.3 * rng.normal(size=(n, d)),
                           rng.uniform(0.5, 2, (n, 1))], 1)
    prim2 = np.concatenate([rng.uniform(0.5, 2, (n, 1)), 0.3 * rng.normal(size=(n, d)),
                            rng.uniform(0.5, 2, (n, 1))], 1)
    nrm = rng.normal(size=(n, d))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return fields.prim_to_cons(prim), fields.prim_to_cons(prim2), nrm


def test_hllc_star_states_satisfy_integral_conservation():
    """Toro's HLLC (Section 2.4): over the wave fan [S_L t, S_R t] the two
    star states hold exactly the conserved quantity the integral form of the
    conservation law leaves there,
        (S* - S_L) U*_L + (S_R - S*) U*_R = S_R U_R - S_L U_L - (F_R - F_L),
    both move with normal velocity S*, and each keeps its side's tangential
    velocity."""
    rng = np.random.default_rng(21)
    for d in (2, 3):
        UL, UR, nrm = _subsonic_states(rng, d, 400)
        SL, SR, Ss, UsL, UsR, FL, FR = flux.hllc_star_states(UL, UR, nrm, 1.4)
        assert np.all(SL < 0) and np.all(SR > 0)
        lhs = (Ss - SL)[:, None] * UsL + (SR - Ss)[:, None] * UsR
        rhs = SR[:, None] * UR - SL[:, None] * UL - (FR - FL)
        assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()
        for U, Us in ((UL, UsL), (UR, UsR)):
            vs = Us[:, 1:-1] / Us[:, :1]
            v = U[:, 1:-1] / U[:, :1]
            assert np.allclose((vs * nrm).sum(1), Ss, rtol=0, atol=1e-12)
            tang = lambda x: x - (x * nrm).sum(1, keepdims=True) * nrm
            assert np.allclose(tang(vs), tang(v), rtol=0, atol=1e-12)


def test_hll_flux_is_the_wave_fan_average():
    """HLL (Section 2.4): the single intermediate state is the wave-fan
    average U* = (S_R U_R - S_L U_L - (F_R - F_L)) / (S_R - S_L) of the
    integral conservation law, and the flux across the face follows from
    either outer wave's Rankine-Hugoniot relation:
        F = F_L + S_L (U* - U_L) = F_R + S_R (U* - U_R)."""
    rng = np.random.default_rng(22)
    for d in (2, 3):
        UL, UR, nrm = _subsonic_states(rng, d, 400)
        _, _, SL, SR = flux._speeds(UL, UR, nrm, 1.4)
        FL, FR = flux.euler_flux(UL, nrm, 1.4), flux.euler_flux(UR, nrm, 1.4)
        Us = (SR[:, None] * UR - SL[:, None] * UL - (FR - FL)) / (SR - SL)[:, None]
        F = flux.hll(UL, UR, nrm, 1.4)
        scale = np.abs(F).max()
        assert np.abs(F - (FL + SL[:, None] * (Us - UL))).max() < 1e-12 * scale
        assert np.abs(F - (FR + SR[:, None] * (Us - UR))).max() < 1e-12 * scale


def test_stationary_and_moving_contacts():
    """A contact (equal pressure and velocity, different density) is resolved
    exactly by HLLC, which carries the contact wave, and smeared by HLL:
    at rest HLLC gives the flux (0, p n, 0) and HLL moves mass from the
    dense side to the light side; a contact moving with normal velocity u
    gets HLLC's upwind flux F(U_L) for u > 0 and F(U_R) for u < 0."""
    rng = np.random.default_rng(23)
    for d in (2, 3):
        n = 200
        nrm = rng.normal(size=(n, d))
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        p = rng.uniform(0.5, 2.0, n)
        rl, rr = rng.uniform(0.2, 3.0, n), rng.uniform(0.2, 3.0, n)
        zero = np.zeros((n, d))
        UL = fields.prim_to_cons(np.concatenate([rl[:, None], zero, p[:, None]], 1))
        UR = fields.prim_to_cons(np.concatenate([rr[:, None], zero, p[:, None]], 1))
        F = flux.hllc(UL, UR, nrm, 1.4)
        assert np.abs(F[:, 0]).max() < 1e-14 and np.abs(F[:, -1]).max() < 1e-14
        assert np.allclose(F[:, 1:-1], p[:, None] * nrm, rtol=0, atol=1e-14)
        Fh = flux.hll(UL, UR, nrm, 1.4)
        assert np.all(Fh[:, 0] * (rr - rl) < 0)                         # dense -> light
        assert np.allclose(Fh[:, 1:-1], p[:, None] * nrm, rtol=0, atol=1e-13)
        # moving contact: velocity u n plus a tangential part, subsonic
        t = rng.normal(size=(n, d))
        t -= (t * nrm).sum(1, keepdims=True) * nrm
        for sgn in (1.0, -1.0):
            u = sgn * rng.uniform(0.05, 0.5, n)
            vel = u[:, None] * nrm + 0.3 * t
            UL = fields.prim_to_cons(np.concatenate([rl[:, None], vel, p[:, None]], 1))
            UR = fields.prim_to_cons(np.concatenate([rr[:, None], vel, p[:, None]], 1))
            F = flux.hllc(UL, UR, nrm, 1.4)
            up = flux.euler_flux(UL if sgn > 0 else UR, nrm, 1.4)
            assert np.abs(F - up).max() < 1e-13 * np.abs(up).max()


def test_venkatakrishnan_limiter_function():
    """Venkatakrishnan's function at eps = 0 is (y^2 + 2y)/(y^2 + y + 2) of
    y = room / increment: 0 at y = 0, 3/4 at y = 1, 1 at y = 2, tending to 1,
    increasing on [0, 2] and never above Barth-Jespersen's min(1, y) there;
    a large eps switches limiting off."""
    from oracle.reconstruction import venkatakrishnan
    y = np.linspace(0.0, 2.0, 201)
    phi = venkatakrishnan(np.ones_like(y), y, 0.0)
    assert abs(phi[0]) < 1e-15 and abs(phi[100] - 0.75) < 1e-15 and abs(phi[-1] - 1.0) < 1e-15
    assert np.all(np.diff(phi) > 0) and np.all(phi <= np.minimum(1.0, y) + 1e-15)
    assert abs(venkatakrishnan(1.0, 1e6, 0.0) - 1.0) < 1e-5
    # scale invariance at eps = 0, sign symmetry
    assert abs(venkatakrishnan(-2.0, -1.0, 0.0) - venkatakrishnan(1.0, 0.5, 0.0)) < 1e-15
    assert abs(venkatakrishnan(1e-3, 0.0, 1e3) - 1.0) < 1e-6


def test_venkatakrishnan_muscl_is_exact_on_affine_data_without_limiting():
    """With a huge kappa (eps^2 dominating every increment) the
    Venkatakrishnan-limited MUSCL reproduces affine data exactly; with the
    paper's kappa = 5 on a fine mesh it limits, and theta stays in (0, 1]."""
    from paper_2510_25906_amd.inputs.params import ALL_MUSCL, VENKAT
    w = configs.c1_density_jump(8, 2)
    cells = np.arange(w.mesh.n_cells)
    om = OracleModel(w.mesh, w.stencils, w.params.with_(scheme_mode=ALL_MUSCL, limiter=VENKAT, kappa=1e4))
    a = np.array([[0.3, -0.2], [0.1, 0.4], [-0.5, 0.2], [0.2, 0.1]])   # [nvar, d]
    b = np.array([2.0, 0.5, 0.7, 3.0])
    x0 = np.array([0.5, 0.5])
    cen = om.geo.cen
    # cell averages of an affine field are its centroid values; the mesh is periodic, so
    # use the field on a patch away from the wrap (interior cells only)
    U = b[None, :] + (cen - x0) @ a.T
    fv, info = om.muscl(cells, U)
    inner = np.all(np.abs(cen - 0.5) < 0.3, axis=1)
    x = om.geo.c_x[cells]
    exact = b[None, None, :] + np.einsum("ngd,vd->ngv", x - x0, a)
    valid = np.arange(x.shape[1])[None, :] < om.geo.c_ngp[cells][:, None]
    err = np.abs(fv - exact)[inner][valid[inner]]
    assert err.max() < 1e-10
    om5 = OracleModel(w.mesh, w.stencils, w.params.with_(scheme_mode=ALL_MUSCL, limiter=VENKAT))
    _, info5 = om5.muscl(cells, U)
    assert np.all(info5["theta"] > 0) and np.all(info5["theta"] <= 1.0)


# --- near_margin: distance of each class decision to its threshold -----------

def test_near_margin_free_stream_closed_form():
    """Constant state: no variable has a range (no NAD threshold), dU = 0 so
    the deactivation margin is |0 - thr| / thr = 1, and every Gauss point
    equals the average so the Harten margin is |0 - theta s| / s = theta."""
    w = configs.c1_density_jump(8, 2)
    U = np.tile(fields.prim_to_cons(np.array([1.3, 0.4, -0.2, 2.0])), (w.mesh.n_cells, 1))
    om = OracleModel(w.mesh, w.stencils, w.params)
    parts = om.near_margin(np.arange(w.mesh.n_cells), U, parts=True)
    assert np.all(np.isinf(parts["nad"]))
    assert np.all(parts["deact"] == 1.0)
    assert np.abs(parts["harten"] - 0.9).max() <= 1e-15
    assert np.abs(parts["total"] - 0.9).max() <= 1e-15
    for mode in (ALL_CWENOZ, ALL_MUSCL):
        om.p = w.params.with_(scheme_mode=mode)
        assert np.all(np.isinf(om.near_margin(np.arange(10), w.U)))


def _margin_case():
    w = configs.c1_density_jump(16, 2)
    # delta_w = 0.1 R and delta_m = 0.5 R exactly (no absolute floors), so a
    # change of beta moves a threshold by a known amount
    p = w.params.with_(alpha_w=0.0, beta_w=0.1, alpha_m=0.0, beta_m=0.5)
    return w, p


def test_near_margin_nad_part_by_threshold_shifts():
    """Shifting a variable's NAD threshold toward its excursion d by (1 + 1e-6)
    times the margin changes that variable's class; by (1 - 1e-6) times it,
    no shift of either threshold does (the margin is the distance from d to
    the nearer threshold, in units of S = max(|m|, |M|, R))."""
    w, p = _margin_case()
    om = OracleModel(w.mesh, w.stencils, p)
    cells = np.arange(w.mesh.n_cells)
    parts = om.near_margin(cells, w.U, parts=True)
    _, info = om.own_class(cells, w.U)
    nad = parts["nad"]
    live = np.isfinite(nad).any(1)
    assert live.sum() > 50
    assert set(np.unique(info["cls_v"][live])) >= {0, 1, 2}
    rng = np.random.default_rng(0)
    for c in rng.choice(np.nonzero(live)[0], 40, replace=False):
        v = int(np.argmin(nad[c]))
        mu = nad[c, v]
        m, M, R = info["m"][c, v], info["M"][c, v], info["R"][c, v]
        S = max(abs(m), abs(M), R)
        base = info["cls_v"][c, v]
        changed = []
        for scale in (1 - 1e-6, 1 + 1e-6):
            db = mu * S / R * scale          # threshold shift mu S (scaled), as a change of beta
            flips = False
            for key in ("beta_w", "beta_m"):
                for sgn in (-1.0, 1.0):
                    om.p = p.with_(**{key: getattr(p, key) + sgn * db})
                    _, inf2 = om.own_class(np.array([c]), w.U)
                    flips |= inf2["cls_v"][0, v] != base
            changed.append(flips)
        om.p = p
        assert changed == [False, True], (c, v, mu, changed)


def test_near_margin_deactivation_part_by_kappa_shift():
    """The deactivation decision dU < (kappa h)^n flips when the threshold
    moves by (1 + 1e-6) times the margin toward dU, and not at (1 - 1e-6)."""
    w, p = _margin_case()
    om = OracleModel(w.mesh, w.stencils, p)
    cells = np.arange(w.mesh.n_cells)
    parts = om.near_margin(cells, w.U, parts=True)
    _, info = om.own_class(cells, w.U)
    assert info["deact"].any() and (~info["deact"]).any()
    n = p.n_exp
    for c in np.concatenate([np.nonzero(info["deact"])[0][:15], np.nonzero(~info["deact"])[0][:15]]):
        mu = parts["deact"][c]
        got = []
        for scale in (1 - 1e-6, 1 + 1e-6):
            # deactivated (thr > dU): lower thr to thr (1 - mu s); active: raise it to thr / (1 - mu s)
            f = (1 - mu * scale) if info["deact"][c] else 1 / (1 - mu * scale)
            om.p = p.with_(kappa=p.kappa * f ** (1 / n))
            _, inf2 = om.own_class(np.array([c]), w.U)
            got.append(bool(inf2["deact"][0] != info["deact"][c]))
        om.p = p
        assert got == [False, True], (c, mu, got)


def test_near_margin_harten_part_by_theta_shift():
    """For cells whose linear candidate passes the Harten check, the margin
    is theta minus the largest relative density / pressure deviation: the
    check still passes with theta lowered by (1 - 1e-6) times the margin and
    fails when it is lowered by (1 + 1e-6) times it."""
    w, p = _margin_case()
    p = p.with_(scheme_mode=ALL_LINEAR)
    om = OracleModel(w.mesh, w.stencils, p)
    cells = np.arange(w.mesh.n_cells)
    parts = om.near_margin(cells, w.U, parts=True)
    assert np.array_equal(parts["total"], parts["harten"])
    _, fv, _ = om.linear(cells, w.U)
    ngp = om.geo.c_ngp[cells]
    ok = om.harten_ok(fv, w.U[cells], ngp)
    assert ok.sum() > 100
    rng = np.random.default_rng(1)
    for c in rng.choice(np.nonzero(ok)[0], 40, replace=False):
        mu = parts["harten"][c]
        got = []
        for scale in (1 - 1e-6, 1 + 1e-6):
            om.p = p.with_(tvd_theta=p.tvd_theta - mu * scale)
            got.append(bool(om.harten_ok(fv[c:c + 1], w.U[c:c + 1], ngp[c:c + 1])[0]))
        om.p = p
        assert got == [True, False], (c, mu, got)
