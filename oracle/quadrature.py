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


def simplex_monomial_integrals_expanded(S: np.ndarray, exps: np.ndarray) -> np.ndarray:
    """Exact integrals of x^alpha over simplices by the full multinomial
    expansion in the barycentric coordinates of all d+1 vertices.

    S: [n, d+1, d] simplex vertices; exps: [K, d] exponents.  Returns [n, K].
    (Slow; kept as an independent check of ``simplex_monomial_integrals``.)
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


@lru_cache(maxsize=None)
def _ref_simplex_tables(d: int, deg: int):
    """Exponents kappa (|kappa| <= deg) of the reference-simplex coordinates,
    their exact integrals kappa! / (d + |kappa|)! over the unit simplex, and the
    index shift tables for multiplying by one coordinate."""
    ks = [k for k in itertools.product(range(deg + 1), repeat=d) if sum(k) <= deg]
    ks.sort(key=lambda k: (sum(k), tuple(-x for x in k)))
    index = {k: i for i, k in enumerate(ks)}
    ref = np.array([np.prod([factorial(x) for x in k]) / factorial(d + sum(k)) for k in ks])
    # up[l][i] = index of kappa_i + e_l (or -1 when the degree would exceed deg)
    up = np.full((d, len(ks)), -1, np.int64)
    for i, k in enumerate(ks):
        for l in range(d):
            kk = list(k)
            kk[l] += 1
            up[l, i] = index.get(tuple(kk), -1)
    return ks, ref, up


def simplex_monomial_integrals(S: np.ndarray, exps: np.ndarray) -> np.ndarray:
    """Exact integrals of x^alpha over simplices.

    With x = v_0 + J lam (lam the coordinates of the reference simplex), x^alpha
    is a polynomial in lam, built exactly by multiplying one affine factor
    x_j = v_0j + sum_l J_jl lam_l at a time; every lam^kappa then integrates to
    kappa! / (d + |kappa|)! over the reference simplex (the Dirichlet
    integral), and the result is scaled by |det J|.

    S: [n, d+1, d] simplex vertices; exps: [K, d] exponents.  Returns [n, K].
    """
    n, dp1, d = S.shape
    if len(exps) == 0:
        return np.zeros((n, 0))
    J = S[:, 1:] - S[:, :1]           # J[:, l, j] = v_{l+1, j} - v_{0, j}
    detJ = np.abs(np.linalg.det(J))
    maxdeg = int(exps.sum(1).max())
    ks, ref, up = _ref_simplex_tables(d, maxdeg)
    nk = len(ks)
    # polynomials are stored coefficient-major: [n_kappa, n_simplices]
    polys = {(0,) * d: np.zeros((nk, n))}
    polys[(0,) * d][0, :] = 1.0
    srcs = [np.nonzero(up[l] >= 0)[0] for l in range(d)]

    def mul_coord(P, j):
        """P(lam) * (v_0j + sum_l J_lj lam_l)."""
        out = P * S[:, 0, j][None, :]
        for l in range(d):
            src = srcs[l]
            out[up[l, src]] += P[src] * J[:, l, j][None, :]
        return out

    def get(alpha):
        if alpha in polys:
            return polys[alpha]
        j = next(i for i, a in enumerate(alpha) if a > 0)
        lower = list(alpha)
        lower[j] -= 1
        P = mul_coord(get(tuple(lower)), j)
        polys[alpha] = P
        return P

    out = np.empty((n, exps.shape[0]))
    for k, alpha in enumerate(exps):
        out[:, k] = detJ * (ref @ get(tuple(int(a) for a in alpha)))
    return out
