"""Seeded initial fields as cell averages of conserved variables.

The workloads are the analytic initial conditions of the paper's test cases
(Section 3): the isentropic vortex (Section 3.1, Eq. 2DVortex), the
two-dimensional Riemann problem (Section 3.5, Eq. 2DRiemannProblem), the
Taylor-Green vortex (Section 3.6, Eqs. tgveq1-tgveq5) and the Shu-Osher
post-shock state (Section 3.2, Eq. 2DShuOsherProblem), plus random
polynomials for exactness checks.  Cell averages are computed by Gauss
quadrature on each element (tensor rules on quads and hexahedra, collapsed
rules on simplices, prisms and pyramids through their simplex tiling).
"""
from __future__ import annotations

import numpy as np

from . import pool
from .mesh import Mesh, TRI, QUAD, TET, PYR, PRISM, HEX, TYPE_NVTX, simplex_decomposition

GAMMA = 1.4


def _gl01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _ref_rule(cell_type, n):
    """Reference-element points (in the element's own vertex weights) and weights.

    Returns shape functions N [nq, nv] and a callable computing |J| per point.
    """
    x, w = _gl01(n)
    if cell_type == QUAD:
        s, t = np.meshgrid(x, x, indexing="ij")
        ws = np.outer(w, w).ravel()
        s, t = s.ravel(), t.ravel()
        N = np.stack([(1 - s) * (1 - t), s * (1 - t), s * t, (1 - s) * t], 1)
        dNs = np.stack([-(1 - t), (1 - t), t, -t], 1)
        dNt = np.stack([-(1 - s), -s, s, (1 - s)], 1)
        return N, ws, (dNs, dNt)
    if cell_type == HEX:
        s, t, u = [a.ravel() for a in np.meshgrid(x, x, x, indexing="ij")]
        ws = np.einsum("i,j,k->ijk", w, w, w).ravel()
        a = [(1 - s), s]
        b = [(1 - t), t]
        c = [(1 - u), u]
        idx = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]
        N = np.stack([a[i] * b[j] * c[k] for i, j, k in idx], 1)
        da = [-np.ones_like(s), np.ones_like(s)]
        dNs = np.stack([da[i] * b[j] * c[k] for i, j, k in idx], 1)
        dNt = np.stack([a[i] * da[j] * c[k] for i, j, k in idx], 1)
        dNu = np.stack([a[i] * b[j] * da[k] for i, j, k in idx], 1)
        return N, ws, (dNs, dNt, dNu)
    raise ValueError(cell_type)


def _simplex_rule(d, n):
    """Collapsed Gauss rule on the unit simplex: barycentric weights, weights."""
    x, w = _gl01(n)
    if d == 2:
        s, t = [a.ravel() for a in np.meshgrid(x, x, indexing="ij")]
        ws = np.outer(w, w).ravel() * (1 - s)
        px, py = s, t * (1 - s)
        B = np.stack([1 - px - py, px, py], 1)
        return B, ws
    s, t, u = [a.ravel() for a in np.meshgrid(x, x, x, indexing="ij")]
    ws = np.einsum("i,j,k->ijk", w, w, w).ravel() * (1 - s) ** 2 * (1 - t)
    px = s
    py = t * (1 - s)
    pz = u * (1 - s) * (1 - t)
    B = np.stack([1 - px - py - pz, px, py, pz], 1)
    return B, ws


def cell_quadrature(mesh: Mesh, cells: np.ndarray, n: int):
    """Quadrature points [nc, nq, d] and weights [nc, nq] (weights sum to |V|).

    All requested cells must share one element type.
    """
    t = int(mesh.cell_type[cells[0]])
    if np.any(mesh.cell_type[cells] != t):
        raise ValueError("cell_quadrature needs cells of one type")
    nv = TYPE_NVTX[t]
    cv = np.stack([mesh.cell_vtx[mesh.cell_vtx_off[cells] + k] for k in range(nv)], 1)
    X = mesh.vertices[cv]  # [nc, nv, d]
    d = mesh.dim
    if t in (QUAD, HEX):
        N, ws, dN = _ref_rule(t, n)
        pts = np.einsum("qv,cvd->cqd", N, X)
        J = np.stack([np.einsum("qv,cvd->cqd", g, X) for g in dN], -1)  # [nc,nq,d,d]
        det = np.abs(np.linalg.det(J))
        return pts, det * ws
    B, ws = _simplex_rule(d, n)
    fact = 2.0 if d == 2 else 6.0
    P_all, W_all = [], []
    for simp in simplex_decomposition(t):
        S = X[:, list(simp)]
        vol = np.abs(np.linalg.det(S[:, 1:] - S[:, :1])) / fact
        P_all.append(np.einsum("qv,cvd->cqd", B, S))
        W_all.append(vol[:, None] * ws[None, :] * fact)
    return np.concatenate(P_all, 1), np.concatenate(W_all, 1)


def _average_block(cc):
    mesh, func, nq = pool.SHARED
    pts, w = cell_quadrature(mesh, cc, nq)
    vals = func(pts)  # [nc, nq, nvar]
    return np.einsum("cqv,cq->cv", vals, w) / w.sum(1)[:, None]


def cell_average(mesh: Mesh, func, nq: int = 6, workers: int = 1) -> np.ndarray:
    """Cell averages of ``func(points [..., d]) -> [..., nvar]`` for all cells
    (in ``workers`` forked processes when workers > 1)."""
    blocks = []
    for t in np.unique(mesh.cell_type):
        cells = np.nonzero(mesh.cell_type == t)[0]
        blocks += [cells[a:a + 32768] for a in range(0, cells.size, 32768)]
    parts = pool.pool_map(_average_block, blocks, workers, (mesh, func, nq))
    out = np.zeros((mesh.n_cells, parts[0].shape[1]))
    for cc, avg in zip(blocks, parts):
        out[cc] = avg
    return out


def prim_to_cons(prim: np.ndarray, gamma: float = GAMMA) -> np.ndarray:
    """(rho, u, v[, w], p) -> (rho, rho u, rho v[, rho w], E) along the last axis."""
    rho = prim[..., 0]
    vel = prim[..., 1:-1]
    p = prim[..., -1]
    E = p / (gamma - 1.0) + 0.5 * rho * (vel ** 2).sum(-1)
    return np.concatenate([rho[..., None], rho[..., None] * vel, E[..., None]], -1)


def cons_to_prim(U: np.ndarray, gamma: float = GAMMA) -> np.ndarray:
    rho = U[..., 0]
    vel = U[..., 1:-1] / rho[..., None]
    p = (gamma - 1.0) * (U[..., -1] - 0.5 * rho * (vel ** 2).sum(-1))
    return np.concatenate([rho[..., None], vel, p[..., None]], -1)


# ---------------------------------------------------------------------------
# initial conditions, as functions of points
# ---------------------------------------------------------------------------

def density_jump_2d(pts, jump=True):
    """rho = 1 + 2 H(x - 1/2) + 0.2 sin(2 pi x) sin(2 pi y), u = v = 1/2, p = 1."""
    x, y = pts[..., 0], pts[..., 1]
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)
    if jump:
        rho = rho + 2.0 * (x > 0.5)
    prim = np.stack([rho, np.full_like(x, 0.5), np.full_like(x, 0.5), np.ones_like(x)], -1)
    return prim_to_cons(prim)


def isentropic_vortex_2d(pts, eps=5.0, centre=(5.0, 5.0), gamma=GAMMA):
    """Mean flow (1, 1, 1, 1) plus the vortex of Section 3.1 (Eq. 2DVortex)."""
    x = pts[..., 0] - centre[0]
    y = pts[..., 1] - centre[1]
    r2 = x * x + y * y
    du = eps / (2 * np.pi) * np.exp(0.5 * (1 - r2)) * (-y)
    dv = eps / (2 * np.pi) * np.exp(0.5 * (1 - r2)) * x
    dT = -(gamma - 1) * eps ** 2 / (8 * gamma * np.pi ** 2) * np.exp(1 - r2)
    T = 1.0 + dT
    rho = T ** (1.0 / (gamma - 1.0))  # isentropic: p / rho^gamma = 1
    p = rho * T
    prim = np.stack([rho, 1.0 + du, 1.0 + dv, p], -1)
    return prim_to_cons(prim)


RIEMANN_2D = {  # Section 3.5, Eq. 2DRiemannProblem: (rho, u, v, p) per quadrant
    "ne": (1.5, 0.0, 0.0, 1.5),
    "nw": (0.5323, 1.206, 0.0, 0.3),
    "sw": (0.138, 1.206, 1.206, 0.029),
    "se": (0.5323, 0.0, 1.206, 0.3),
}


def riemann_2d_prim(pts):
    x, y = pts[..., 0], pts[..., 1]
    out = np.zeros(x.shape + (4,))
    for key, st in RIEMANN_2D.items():
        m = ((x >= 0) if key[1] == "e" else (x < 0)) & ((y >= 0) if key[0] == "n" else (y < 0))
        out[m] = st
    return out


def tgv_prim(pts, mach=1.25, gamma=GAMMA, k=1.0, perturb=None):
    """Taylor-Green vortex of Section 3.6 (Eqs. tgveq1-tgveq5); rho = gamma M^2 p / T, T = 1."""
    x, y, z = pts[..., 0], pts[..., 1], pts[..., 2]
    u = np.sin(k * x) * np.cos(k * y) * np.cos(k * z)
    v = -np.cos(k * x) * np.sin(k * y) * np.cos(k * z)
    w = np.zeros_like(x)
    p = 1.0 / (gamma * mach ** 2) + (np.cos(2 * z) + 2.0) * (np.cos(2 * x) + np.cos(2 * y)) / 16.0
    rho = gamma * mach ** 2 * p
    if perturb is not None:
        kv, ph, amp = perturb
        for c, comp in enumerate((u, v, w)):
            acc = np.zeros_like(x)
            for m in range(kv.shape[0]):
                acc += np.sin(kv[m, 0] * x + kv[m, 1] * y + kv[m, 2] * z + ph[c, m])
            comp += amp / kv.shape[0] * acc
    return np.stack([rho, u, v, w, p], -1)


def tgv_perturbation(seed=1, n_modes=8, amp=0.05):
    rng = np.random.default_rng(seed)
    kv = np.zeros((n_modes, 3), np.int64)
    m = 0
    while m < n_modes:
        k = rng.integers(-4, 5, size=3)
        if np.any(k != 0):
            kv[m] = k
            m += 1
    ph = rng.uniform(0, 2 * np.pi, size=(3, n_modes))
    return kv.astype(np.float64), ph, amp


def rankine_hugoniot(mach, gamma=GAMMA, rho1=1.0, p1=1.0):
    """Post-shock (rho, u, p) behind a normal shock moving at Mach ``mach`` into rest."""
    c1 = np.sqrt(gamma * p1 / rho1)
    s = mach * c1
    rho2 = rho1 * (gamma + 1) * mach ** 2 / ((gamma - 1) * mach ** 2 + 2)
    p2 = p1 * (2 * gamma * mach ** 2 - (gamma - 1)) / (gamma + 1)
    u2 = s * (1 - rho1 / rho2)
    return rho2, u2, p2


# Three smooth vortices (axis along z) for the shock-vortex workload: centre
# (x, y) as fractions of the box, radius and peak speed in units of the
# upstream sound speed.
SHOCK_VORTICES = ((0.25, 0.35, 0.08, 0.3), (0.55, 0.60, 0.08, 0.3), (0.80, 0.40, 0.08, 0.3))


def shock_vortices_prim(pts, length, x_shock, mach=3.0, gamma=GAMMA, vortices=SHOCK_VORTICES, ambient=1e-3):
    """A planar normal shock moving in +x at Mach ``mach`` into gas at rest
    (rho = p = 1 ahead, x > x_shock; Rankine-Hugoniot state behind it) plus
    Gaussian vortices u_theta = s (r/R) exp((1 - r^2/R^2)/2) around z-parallel
    axes, on the box [0, length] x [0, 1] x [0, 1]; returns (rho, u, v, w, p).
    ``ambient`` adds weak smooth waves uniform in x on both sides (density
    factor 1 + a sin 2pi y sin 2pi z, transverse velocities a sin 2pi z and
    a sin 2pi y) so that no conserved variable is constant up to rounding
    anywhere; at the default a = 1e-3 they stay below the NAD deactivation
    threshold on the meshes used here, so they break ties without adding flow
    features."""
    x, y, z = pts[..., 0], pts[..., 1], pts[..., 2]
    rho2, u2, p2 = rankine_hugoniot(mach, gamma)
    behind = x < x_shock
    rho = np.where(behind, rho2, 1.0) * (1.0 + ambient * np.sin(2 * np.pi * y) * np.sin(2 * np.pi * z))
    p = np.where(behind, p2, 1.0)
    u = np.where(behind, u2, 0.0)
    v = ambient * np.sin(2 * np.pi * z)
    w = ambient * np.sin(2 * np.pi * y)
    c1 = np.sqrt(gamma)
    for fx, fy, R, s in vortices:
        dx, dy = x - fx * length, y - fy
        g = s * c1 / R * np.exp(0.5 * (1.0 - (dx * dx + dy * dy) / (R * R)))
        u = u - g * dy
        v = v + g * dx
    return np.stack([rho, u, v, w, p], -1)


def random_polynomial(d, r, nvar, seed, scale=1.0):
    """A seeded random polynomial of total degree <= r per variable.

    Returns (exponents [T, d], coefficients [T, nvar]) and an evaluator.
    """
    rng = np.random.default_rng(seed)
    exps = [e for e in np.ndindex(*([r + 1] * d)) if sum(e) <= r]
    exps = np.array(exps, np.int64)
    coef = rng.normal(size=(exps.shape[0], nvar)) * scale
    coef[0] += 5.0  # keep values away from zero

    def ev(pts):
        mon = np.ones(pts.shape[:-1] + (exps.shape[0],))
        for j in range(d):
            mon = mon * pts[..., j:j + 1] ** exps[:, j]
        return mon @ coef
    return exps, coef, ev
