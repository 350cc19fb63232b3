"""Pins of the oracle's quadrature and exact integrals against closed forms."""
from math import factorial

import numpy as np
import pytest

from oracle import quadrature as Q
from oracle.geometry import cell_simplices, compute_geometry
from paper_2510_25906_amd.inputs.mesh import quad_tri_2d, hex_3d


def test_reference_triangle_monomials():
    S = np.array([[[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]])
    for p in range(7):
        for q in range(7 - p):
            got = Q.simplex_monomial_integrals(S, np.array([[p, q]]))[0, 0]
            assert got == pytest.approx(factorial(p) * factorial(q) / factorial(p + q + 2), rel=1e-13)


def test_reference_tet_monomials():
    S = np.array([[[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]])
    for a in range(5):
        for b in range(5 - a):
            for c in range(5 - a - b):
                got = Q.simplex_monomial_integrals(S, np.array([[a, b, c]]))[0, 0]
                ref = factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)
                assert got == pytest.approx(ref, rel=1e-13)


def test_box_monomials_through_tiling():
    """Rectangles and boxes, integrated through the oracle's simplex tiling."""
    m2 = quad_tri_2d(1, 1, lo=(0.5, -1.0), hi=(2.0, 0.25))
    S, own = cell_simplices(m2, np.array([0]))
    for p in range(6):
        for q in range(6 - p):
            got = Q.simplex_monomial_integrals(S, np.array([[p, q]])).sum()
            ref = (2.0 ** (p + 1) - 0.5 ** (p + 1)) / (p + 1) * (0.25 ** (q + 1) - (-1.0) ** (q + 1)) / (q + 1)
            assert got == pytest.approx(ref, rel=1e-12, abs=1e-14)
    m3 = hex_3d(1, 1, 1, lo=(0.0, -0.5, 1.0), hi=(1.5, 0.5, 2.0))
    S, own = cell_simplices(m3, np.array([0]))
    for a in range(4):
        for b in range(4 - a):
            for c in range(4 - a - b):
                got = Q.simplex_monomial_integrals(S, np.array([[a, b, c]])).sum()
                ref = (1.5 ** (a + 1)) / (a + 1) * (0.5 ** (b + 1) - (-0.5) ** (b + 1)) / (b + 1) \
                    * (2.0 ** (c + 1) - 1.0) / (c + 1)
                assert got == pytest.approx(ref, rel=1e-12, abs=1e-14)


def test_affine_simplex_against_change_of_variables():
    """A random triangle: integrate x^2 y by pulling back to the reference triangle
    with a tensor Gauss rule on the collapsed square (independent of the
    Dirichlet expansion)."""
    rng = np.random.default_rng(5)
    V = rng.normal(size=(3, 2))
    S = V[None]
    got = Q.simplex_monomial_integrals(S, np.array([[2, 1]]))[0, 0]
    x, w = np.polynomial.legendre.leggauss(8)
    x, w = 0.5 * (x + 1), 0.5 * w
    s, t = np.meshgrid(x, x, indexing="ij")
    W = np.outer(w, w) * (1 - s)
    a, b = s, t * (1 - s)
    P = V[0] + a[..., None] * (V[1] - V[0]) + b[..., None] * (V[2] - V[0])
    J = abs(np.linalg.det(np.stack([V[1] - V[0], V[2] - V[0]], 1)))
    ref = (W * P[..., 0] ** 2 * P[..., 1]).sum() * J
    assert got == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_triangle_rules_exact_to_degree_r(r):
    bc, w = Q.triangle_rule(r)
    assert np.all(w > 0) and w.sum() == pytest.approx(1.0, rel=1e-15)
    assert np.all(bc > 0) and np.allclose(bc.sum(1), 1.0)
    deg = 2 if r <= 2 else 4
    x, y = bc[:, 1], bc[:, 2]
    for p in range(deg + 1):
        for q in range(deg + 1 - p):
            ref = 2.0 * factorial(p) * factorial(q) / factorial(p + q + 2)
            assert (w * x ** p * y ** q).sum() == pytest.approx(ref, rel=1e-14)
    # and not beyond (so the point count is the minimal reading)
    errs = [abs((w * x ** p * y ** (deg + 1 - p)).sum() - 2.0 * factorial(p) * factorial(deg + 1 - p)
                / factorial(deg + 3)) for p in range(deg + 2)]
    assert max(errs) > 1e-8


def test_gauss_legendre_exactness():
    for n in range(1, 4):
        x, w = Q.gauss_legendre_01(n)
        for p in range(2 * n):
            assert (w * x ** p).sum() == pytest.approx(1.0 / (p + 1), rel=1e-14)


def test_geometry_closure_and_measure():
    m = quad_tri_2d(6, 5, lo=(-0.5, -0.5), hi=(0.5, 0.5),
                    split=np.random.default_rng(0).random((5, 6)) < 0.4)
    g = compute_geometry(m, 3)
    assert g.vol.sum() == pytest.approx(1.0, rel=1e-14)
    # every cell is closed: sum of outward n |S| vanishes
    acc = np.zeros((m.n_cells, 2))
    np.add.at(acc, m.face_cells[:, 0], g.normal * g.area[:, None])
    inner = m.face_cells[:, 1] >= 0
    np.add.at(acc, m.face_cells[inner, 1], -(g.normal * g.area[:, None])[inner])
    assert np.abs(acc).max() < 1e-14
    # quadrature weights sum to the face measure
    s = np.add.reduceat(g.gp_wS, g.gp_off[:-1])
    assert np.allclose(s, g.area, rtol=1e-14)
    m3 = hex_3d(3, 3, 4, hi=(3.0, 1.0, 2.0), periodic=True)
    g3 = compute_geometry(m3, 4)
    assert g3.vol.sum() == pytest.approx(6.0, rel=1e-14)
    assert np.allclose(np.add.reduceat(g3.gp_wS, g3.gp_off[:-1]), g3.area, rtol=1e-14)
    assert np.diff(g3.gp_off).max() == 9


def test_fast_and_expanded_simplex_integrals_agree():
    rng = np.random.default_rng(9)
    for d in (2, 3):
        S = rng.normal(size=(7, d + 1, d))
        exps = np.array([e for e in np.ndindex(*([5] * d)) if sum(e) <= 4])
        a = Q.simplex_monomial_integrals(S, exps)
        b = Q.simplex_monomial_integrals_expanded(S, exps)
        assert np.allclose(a, b, rtol=1e-11, atol=1e-13)
