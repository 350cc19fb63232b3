"""Oracle quadrature and exact simplex integrals (test infrastructure only).

* Face rules follow Section 2 (paragraph after Eq. EulerEquationsDetails):
  Gauss-Legendre on edges and tensor-product (quadrilateral) faces, symmetric
  Gauss rules on triangular faces.  The number of points is not given; the
  reading used is n = ceil((r+1)/2) Gauss-Legendre points per direction and a
  symmetric triangle rule of degree >= r (3 points up to r = 2, 6 points for
  r = 3, 4).
* Volume integrals of monomials are exact, from the Dirichlet integral of
  barycentric monomials over a simplex,
  int_T prod_l lambda_l^{k_l} = d! |T| prod_l k_l! / (d + sum k)!,
  after expanding x = sum_l lambda_l v_l by the multinomial theorem.
"""
from __future__ import annotations

import itertools
from functools import lru_cache
from math import factorial, ceil

import numpy as np
from scipy.optimize import least_squares


def gauss_legendre_01(n: int):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def n_line_points(r: int) -> int:
    return int(ceil((r + 1) / 2))


@lru_cache(maxsize=None)
def triangle_rule(r: int):
    """Symmetric triangle rule exact to degree >= r.

    Returns barycentric points [q, 3] (ordered orbit by orbit, each orbit
    (a, a, 1-2a) listed as (1-2a, a, a), (a, 1-2a, a), (a, a, 1-2a)) and
    weights [q] summing to one.
    """
    if r <= 2:
        orbits = [(1.0 / 6.0, 1.0 / 3.0)]
    elif r <= 4:
        # Two orbits (a_i, a_i, 1 - 2 a_i) with weights w_i per point; solve the
        # moment equations of all monomials x^p y^q, p + q <= 4.
        mons = [(p, q) for p in range(5) for q in range(5) if p + q <= 4]
        exact = np.array([2.0 * factorial(p) * factorial(q) / factorial(p + q + 2) for p, q in mons])

        def resid(z):
            a1, a2, w1, w2 = z
            res = np.zeros(len(mons))
            for a, w in ((a1, w1), (a2, w2)):
                for bc in ((1 - 2 * a, a, a), (a, 1 - 2 * a, a), (a, a, 1 - 2 * a)):
                    x, y = bc[1], bc[2]
                    res += w * np.array([x ** p * y ** q for p, q in mons])
            return res - exact

        sol = least_squares(resid, x0=[0.42, 0.1, 0.2, 0.12], xtol=1e-15, ftol=1e-15, gtol=1e-15)
        a1, a2, w1, w2 = sol.x
        if max(abs(resid(sol.x))) > 1e-14 or not (0 < a2 < a1 < 0.5):
            raise RuntimeError("triangle rule did not converge")
        orbits = [(a1, w1), (a2, w2)]
    else:
        raise ValueError("triangle faces supported up to r = 4")
    pts, wts = [], []
    for a, w in orbits:
        for bc in ((1 - 2 * a, a, a), (a, 1 - 2 * a, a), (a, a, 1 - 2 * a)):
            pts.append(bc)
            wts.append(w)
    return np.array(pts), np.array(wts)


def _compositions(n: int, parts: int):
    if parts == 1:
        yield (n,)
        return
    for first in range(n + 1):
        for rest in _compositions(n - first, parts - 1):
            yield (first,) + rest


@lru_cache(maxsize=None)
def _dirichlet_terms(alpha: tuple, d: int):
    """Expansion terms of prod_j (sum_l lambda_l v_lj)^alpha_j: (coef [T], exps [T, d+1, d])."""
    per_axis = [list(_compositions(a, d + 1)) for a in alpha]
    coefs, exps = [], []
    deg = sum(alpha)
    for combo in itertools.product(*per_axis):
        c = 1.0
        E = np.zeros((d + 1, d), np.int64)
        for j, comp in enumerate(combo):
            m = factorial(alpha[j])
            for l, k in enumerate(comp):
                m //= factorial(k)
                E[l, j] = k
            c *= m
        ktot = E.sum(1)
        num = 1
        for k in ktot:
            num *= factorial(int(k))
        coefs.append(c * num / factorial(d + deg))
        exps.append(E)
    return np.array(coefs), np.array(exps)


def simplex_monomial_integrals(S: np.ndarray, exps: np.ndarray) -> np.ndarray:
    """Exact integrals of x^alpha over simplices.

    S: [n, d+1, d] simplex vertices; exps: [K, d] exponents.  Returns [n, K].
    """
    n, dp1, d = S.shape
    J = S[:, 1:] - S[:, :1]
    vol = np.abs(np.linalg.det(J)) / factorial(d)
    maxdeg = int(exps.sum(1).max()) if len(exps) else 0
    pw = np.ones((n, dp1, d, maxdeg + 1))
    for p in range(1, maxdeg + 1):
        pw[..., p] = pw[..., p - 1] * S
    out = np.zeros((n, exps.shape[0]))
    li = np.arange(dp1)[:, None]
    ji = np.arange(d)[None, :]
    for k, alpha in enumerate(exps):
        coef, E = _dirichlet_terms(tuple(int(a) for a in alpha), d)
        acc = np.zeros(n)
        for c, e in zip(coef, E):
            acc += c * np.prod(pw[:, li, ji, e].reshape(n, -1), axis=1)
        out[:, k] = factorial(d) * vol * acc
    return out
