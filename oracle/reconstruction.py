"""Oracle of the hybrid reconstruction (test infrastructure only).

Plain FP64 NumPy, step by step in the order of the method's flowchart
(Section 2.5, Fig. HybridWENOFlowchart): linear least-squares candidate for
every cell, numerical admissibility detector (NAD) with deactivation, tagging
of the flagged cells' von Neumann neighbourhood, CWENOZ on weakly non-smooth
cells, MUSCL with the Barth-Jespersen limiter on discontinuous cells, and the
Harten bound check with first-order fallback on every cell.

Readings of the paper used here (each is also listed in the design notes):

* Reference frame xi = (x - x_c) / h_c with h_c = |V|^(1/d), so |V_0'| = 1
  (Section 2.1, Eq. AVGVariables2; the transformation itself is only cited).
* Basis psi_k = monomials xi^alpha, 1 <= |alpha| <= r, by degree and then in
  descending lexicographic order; phi_k = psi_k - mean of psi_k over V_0'
  (Section 2.1).  Face states, smoothness indicators and weights do not depend
  on the choice of polynomial basis.
* K = C(r+d, d) - 1 unknowns, M = 2K stencil neighbours (Section 2.1).
* Least-squares rows are integrals over V_m' (Eq. dofMatrix); the
  pseudo-inverse is taken with an SVD-based library routine.
* Smoothness indicator (Eq. SI1) with derivatives in the xi frame, where the
  h_c factor is 1; OI from exact moments of cell 0.
* CWENOZ weights: by default the Z form w~_s = lambda_s (1 + (tau/(eps+SI_s))^b)
  with tau the mean |SI_s - SI_1| over s >= 2; ``LITERAL`` keeps the printed
  placement of the exponent (tau^b / (eps + SI_s)).  SI_1 is the indicator of
  p_1.  lambda_1 = 1 - 1/lambda_1'.
* NAD: with V_i the cell and its face neighbours, m and M their minimum and
  maximum, and d the largest excursion max(m - U(x), U(x) - M) of the linear
  candidate over the cell's face Gauss points: linear if d <= delta_w, else
  MUSCL if d >= delta_m, else CWENOZ (Eqs. DMP, NADMUSCL, NADCWENOZ, marginm,
  marginw); per conserved variable, the cell taking the most dissipative class.
  sign(0) = 0 in delta_w.
* Deactivation (Eq. NADDeactivatedCriteria): 2-norm over the conserved
  variables, face neighbours, strict inequality, dx = h_c.
* Tagging: one max-dilation over face neighbours, after deactivation.
* MUSCL: degree-1 least squares over the face neighbours (padded from the
  central stencil to d+1 cells), Barth-Jespersen limited per variable at the
  face Gauss points against the NAD bounds m, M (Section 2.2); optionally
  Venkatakrishnan's limiter (compared in Section 3.2, kappa = 5) with
  eps^2 = (kappa h_c)^3, the same kappa as the deactivation.
* Harten check on density and pressure at every face Gauss point of the final
  reconstruction, for every class (Eq. harten_jump_fix).
"""
from __future__ import annotations

from math import comb

import numpy as np

from .geometry import compute_geometry, cell_simplices
from .quadrature import simplex_monomial_integrals

LIN, CW, MU, FO = 0, 1, 2, 3
HYBRID, ALL_LINEAR, ALL_CWENOZ, ALL_MUSCL = 0, 1, 2, 3
BJ, VENKAT = 0, 1


def basis_exponents(d: int, r: int) -> np.ndarray:
    """Exponents of the non-constant monomials of degree <= r (hierarchical order)."""
    out = []
    for deg in range(1, r + 1):
        es = [e for e in np.ndindex(*([deg + 1] * d)) if sum(e) == deg]
        es.sort(reverse=True)
        out += es
    return np.array(out, np.int64).reshape(-1, d)


def all_exponents(d: int, deg: int) -> np.ndarray:
    out = []
    for k in range(0, deg + 1):
        es = [e for e in np.ndindex(*([k + 1] * d)) if sum(e) == k]
        es.sort(reverse=True)
        out += es
    return np.array(out, np.int64)


def monomials(xi: np.ndarray, exps: np.ndarray) -> np.ndarray:
    """xi [..., d] -> [..., K] values of xi^alpha."""
    out = np.ones(xi.shape[:-1] + (exps.shape[0],))
    for j in range(xi.shape[-1]):
        out = out * xi[..., j:j + 1] ** exps[:, j]
    return out


def _deriv_coef(alpha, beta):
    c = 1.0
    for a, b in zip(alpha, beta):
        if b > a:
            return 0.0
        for t in range(b):
            c *= (a - t)
    return c


def venkatakrishnan(dm, dp, eps2):
    """Venkatakrishnan's limiter function (J. Comput. Phys. 118, 1995) for an
    unlimited increment dm (nonzero) towards a face point and the room dp to
    the neighbourhood bound in the same direction:
        phi = (dp^2 + 2 dm dp + eps^2) / (dp^2 + 2 dm^2 + dm dp + eps^2),
    which for eps = 0 is the function (y^2 + 2y) / (y^2 + y + 2) of y = dp/dm."""
    with np.errstate(divide="ignore", invalid="ignore"):
        return (dp * dp + 2.0 * dm * dp + eps2) / (dp * dp + 2.0 * dm * dm + dm * dp + eps2)


class OracleModel:
    """Precomputed geometry and per-cell tables for one mesh and stencil set."""

    def __init__(self, mesh, st, params):
        self.mesh = mesh
        self.st = st
        self.p = params
        self.r = params.order_r
        self.d = mesh.dim
        self.nvar = self.d + 2
        self.exps = basis_exponents(self.d, self.r)
        self.K = self.exps.shape[0]
        if self.K != comb(self.r + self.d, self.d) - 1:
            raise AssertionError
        self.geo = compute_geometry(mesh, self.r)
        self.period = mesh.period if mesh.period is not None else np.zeros(self.d)
        self._tab = {}
        # face neighbours per cell (padded)
        NF = 4 if self.d == 2 else 6
        nfc = np.diff(mesh.cell_face_off)
        self.nbr = np.full((mesh.n_cells, NF), -1, np.int64)
        for j in range(int(nfc.max())):
            cells = np.nonzero(nfc > j)[0]
            f = mesh.cell_face[mesh.cell_face_off[cells] + j]
            side = mesh.cell_face_side[mesh.cell_face_off[cells] + j]
            l, r_ = mesh.face_cells[f, 0], mesh.face_cells[f, 1]
            self.nbr[cells, j] = np.where(side == 0, r_, l)

    # ------------------------------------------------------------------
    # Section 2.1: least-squares tables (computed once per cell)
    # ------------------------------------------------------------------
    def _member_integrals(self, cells, ids, shifts, exps):
        """int over V_m' of xi^alpha in the frame of each owner cell.

        cells [n]; ids [n, Mm]; shifts [n, Mm, d].  Returns (I [n, Mm, K'], Vp [n, Mm]).
        """
        n, Mm = ids.shape
        flat = ids.reshape(-1)
        S, own = cell_simplices(self.mesh, flat)
        owner_cell = np.repeat(cells, Mm)[own]
        sh = shifts.reshape(-1, self.d)[own].astype(np.float64) * self.period
        xc = self.geo.cen[owner_cell]
        hh = self.geo.h[owner_cell]
        Sx = (S + sh[:, None, :] - xc[:, None, :]) / hh[:, None, None]
        E = np.concatenate([np.zeros((1, self.d), np.int64), exps], 0)
        I = simplex_monomial_integrals(Sx, E)
        out = np.zeros((n * Mm, E.shape[0]))
        np.add.at(out, own, I)
        out = out.reshape(n, Mm, -1)
        return out[..., 1:], out[..., 0]

    def _compute_tables(self, cells):
        d, r, K = self.d, self.r, self.K
        n = cells.size
        st = self.st
        # own moments up to degree 2r (for the basis means and OI)
        E2 = all_exponents(d, max(r, 2 * r - 2))
        S, own = cell_simplices(self.mesh, cells)
        xc = self.geo.cen[cells][own]
        hh = self.geo.h[cells][own]
        Sx = (S - xc[:, None, :]) / hh[:, None, None]
        mom = np.zeros((n, E2.shape[0]))
        np.add.at(mom, own, simplex_monomial_integrals(Sx, E2))
        eidx = {tuple(e): i for i, e in enumerate(E2)}
        V0 = mom[:, eidx[(0,) * d]]
        psibar = np.stack([mom[:, eidx[tuple(e)]] for e in self.exps], 1) / V0[:, None]
        # OI_kq = sum_{1<=|beta|<=r} int D^beta phi_k D^beta phi_q  (Section 2.3)
        betas = basis_exponents(d, r)
        OI = np.zeros((n, K, K))
        for k, ak in enumerate(self.exps):
            for q, aq in enumerate(self.exps):
                acc = np.zeros(n)
                for b in betas:
                    c = _deriv_coef(ak, b) * _deriv_coef(aq, b)
                    if c != 0.0:
                        acc += c * mom[:, eidx[tuple(ak + aq - 2 * b)]]
                OI[:, k, q] = acc
        # central least squares (Eq. dofMatrix)
        I, Vp = self._member_integrals(cells, st.central[cells], st.central_shift[cells], self.exps)
        A = I - Vp[..., None] * psibar[:, None, :]
        Ad = np.linalg.pinv(A)                      # [n, K, M]
        P = Ad * Vp[:, None, :]
        sv = np.linalg.svd(A, compute_uv=False)
        cond = sv[:, 0] / sv[:, -1]
        if np.any(~(cond < 1e12)):
            bad = int(cells[np.argmax(~(cond < 1e12))])
            raise np.linalg.LinAlgError(f"central least-squares system of cell {bad} is rank deficient")
        # directional degree-1 fits (Section 2.3, r = 1 for directional stencils)
        NF = st.dir.shape[1]
        Md = st.dir.shape[2]
        ids = np.where(st.dir[cells] >= 0, st.dir[cells], cells[:, None, None])
        Id, Vd = self._member_integrals(cells, ids.reshape(n, NF * Md),
                                        st.dir_shift[cells].reshape(n, NF * Md, d), self.exps[:d])
        Ad_dir = Id.reshape(n, NF, Md, d) - Vd.reshape(n, NF, Md)[..., None] * psibar[:, None, None, :d]
        Pdir = np.linalg.pinv(Ad_dir) * Vd.reshape(n, NF, 1, Md)   # [n, NF, d, Md]
        # padding slots (cells with fewer faces than NF) hold no stencil
        Pdir = Pdir * (np.arange(NF)[None, :] < st.n_dir[cells][:, None])[..., None, None]
        # MUSCL degree-1 fit over face neighbours
        NM = st.muscl.shape[1]
        mid = np.where(st.muscl[cells] >= 0, st.muscl[cells], cells[:, None])
        Im, Vm = self._member_integrals(cells, mid, st.muscl_shift[cells], self.exps[:d])
        Am = Im - Vm[..., None] * psibar[:, None, :d]
        valid = np.arange(NM)[None, :] < st.n_muscl[cells][:, None]
        Am = Am * valid[..., None]
        Pmus = np.linalg.pinv(Am) * (Vm * valid)[:, None, :]           # [n, d, NM]
        # Gauss points in the cell frame
        xi = (self.geo.c_x[cells] - self.geo.cen[cells][:, None, :]) / self.geo.h[cells][:, None, None]
        return dict(P=P, psibar=psibar, OI=OI, cond=cond, Pdir=Pdir, Pmus=Pmus, xi=xi, V0=V0)

    def tables(self, cells):
        cells = np.asarray(cells, np.int64)
        need = [c for c in np.unique(cells) if c not in self._tab]
        if need:
            need = np.array(need)
            chunk = max(1, 400000 // (self.st.M * 6))
            for a in range(0, need.size, chunk):
                cc = need[a:a + chunk]
                t = self._compute_tables(cc)
                for i, c in enumerate(cc):
                    self._tab[int(c)] = {k: v[i] for k, v in t.items()}
        keys = self._tab[int(cells[0])].keys() if cells.size else []
        return {k: np.stack([self._tab[int(c)][k] for c in cells]) for k in keys}

    # ------------------------------------------------------------------
    def phi_at_gp(self, tab):
        """Basis values phi_k at each cell's Gauss points: [n, NGPC, K]."""
        return monomials(tab["xi"], self.exps) - tab["psibar"][:, None, :]

    def linear(self, cells, U):
        """Linear candidate (Section 2.1): coefficients [n, K, nvar] and face values."""
        tab = self.tables(cells)
        dU = U[self.st.central[cells]] - U[cells][:, None, :]       # [n, M, nvar]
        a = np.einsum("nkm,nmv->nkv", tab["P"], dU)
        phi = self.phi_at_gp(tab)
        fv = U[cells][:, None, :] + np.einsum("ngk,nkv->ngv", phi, a)
        return a, fv, tab

    def nad_bounds(self, cells, U):
        nb = self.nbr[cells]
        vals = np.where((nb >= 0)[..., None], U[np.maximum(nb, 0)], U[cells][:, None, :])
        allv = np.concatenate([U[cells][:, None, :], vals], 1)
        return allv.min(1), allv.max(1)

    def own_class(self, cells, U):
        """NAD own class (Section 2.5, Eqs. DMP to NADDeactivatedCriteria_2).

        Returns (class [n], margin info dict)."""
        p = self.p
        _, fv, _ = self.linear(cells, U)
        ngp = self.geo.c_ngp[cells]
        valid = np.arange(fv.shape[1])[None, :] < ngp[:, None]
        m, M = self.nad_bounds(cells, U)
        R = M - m
        dmarg = np.maximum(p.alpha_m, p.beta_m * R)
        wmarg = np.sign(p.beta_w) * np.maximum(p.alpha_w, np.abs(p.beta_w * R))
        exc = np.maximum(m[:, None, :] - fv, fv - M[:, None, :])
        exc = np.where(valid[..., None], exc, -np.inf)
        dv = exc.max(1)                                              # [n, nvar]
        cls_v = np.where(dv <= wmarg, LIN, np.where(dv >= dmarg, MU, CW))
        own = cls_v.max(1)
        # deactivation
        nb = self.nbr[cells]
        has = nb >= 0
        diff = np.linalg.norm(U[np.maximum(nb, 0)] - U[cells][:, None, :], axis=2)
        dmax = np.where(has, diff, -np.inf).max(1)
        dmin = np.where(has, diff, np.inf).min(1)
        dU = np.where(has.any(1), dmax - dmin, 0.0)
        thr = (p.kappa * self.geo.h[cells]) ** p.n_exp
        deact = dU < thr
        own = np.where(deact, LIN, own)
        info = dict(dv=dv, wmarg=wmarg, dmarg=dmarg, dU=dU, thr=thr, deact=deact, R=R, m=m, M=M, cls_v=cls_v)
        return own, info

    def near_margin(self, cells, U, parts=False):
        """Relative distance of each cell's class decisions to their
        thresholds, the smallest over the decisions (the library's
        near_margin output); +inf where no decision is taken.

        NAD (Eqs. NADMUSCL, NADCWENOZ with marginm, marginw), hybrid mode,
        per conserved variable whose range R = M - m over the cell and its
        face neighbours is non-zero: min(|d - delta_w|, |d - delta_m|) / S,
        S = max(|m|, |M|, R).  Deactivation (Eq. NADDeactivatedCriteria),
        hybrid mode: |dU - (kappa h)^n| / max(dU, (kappa h)^n), 0 when both
        vanish.  Harten (Eq. harten_jump_fix), hybrid and all-linear modes,
        density and pressure at every face Gauss point of the linear
        candidate: | |q - q_bar| - theta s | / s with s = max(|q_bar|, eps).
        All-CWENOZ and all-MUSCL modes take no such decision: +inf.
        parts=True returns the pieces as well: dict(nad [n, nvar],
        deact [n], harten [n], total [n]), +inf where a piece does not apply."""
        cells = np.asarray(cells, np.int64)
        p = self.p
        out = np.full(cells.size, np.inf)
        nad = np.full((cells.size, self.nvar), np.inf)
        deact = np.full(cells.size, np.inf)
        harten = np.full(cells.size, np.inf)
        mode = p.scheme_mode
        if mode not in (HYBRID, ALL_LINEAR):
            return dict(nad=nad, deact=deact, harten=harten, total=out) if parts else out
        if mode == HYBRID:
            _, info = self.own_class(cells, U)
            m, M, R, dv = info["m"], info["M"], info["R"], info["dv"]
            S = np.maximum(np.maximum(np.abs(m), np.abs(M)), R)
            with np.errstate(divide="ignore", invalid="ignore"):
                nad = np.where(R > 0, np.minimum(np.abs(dv - info["wmarg"]), np.abs(dv - info["dmarg"])) / S, np.inf)
            den = np.maximum(info["dU"], info["thr"])
            with np.errstate(divide="ignore", invalid="ignore"):
                deact = np.where(den > 0, np.abs(info["dU"] - info["thr"]) / den, 0.0)
            out = np.fmin(np.fmin(out, nad.min(1)), deact)
        _, fv, _ = self.linear(cells, U)
        g = p.gamma
        ngp = self.geo.c_ngp[cells]
        valid = np.arange(fv.shape[1])[None, :] < ngp[:, None]
        Ub = U[cells]
        rho_b = Ub[:, 0]
        pres_b = (g - 1) * (Ub[:, -1] - 0.5 * (Ub[:, 1:-1] ** 2).sum(1) / rho_b)
        sr = np.maximum(np.abs(rho_b), p.tvd_eps)[:, None]
        sp = np.maximum(np.abs(pres_b), p.tvd_eps)[:, None]
        with np.errstate(divide="ignore", invalid="ignore"):
            pres = (g - 1) * (fv[..., -1] - 0.5 * (fv[..., 1:-1] ** 2).sum(-1) / fv[..., 0])
            hr = np.abs(np.abs(fv[..., 0] - rho_b[:, None]) - p.tvd_theta * sr) / sr
            hp = np.abs(np.abs(pres - pres_b[:, None]) - p.tvd_theta * sp) / sp
        h = np.where(valid, np.fmin(hr, hp), np.inf)
        harten = np.where(np.isnan(h), np.inf, h).min(1)
        out = np.fmin(out, harten)
        return dict(nad=nad, deact=deact, harten=harten, total=out) if parts else out

    def harten_ok(self, fv, Ucell, ngp):
        """Harten bound check on density and pressure (Eq. harten_jump_fix)."""
        p = self.p
        g = p.gamma
        valid = np.arange(fv.shape[1])[None, :] < ngp[:, None]
        rho_b = Ucell[:, 0]
        pres_b = (g - 1) * (Ucell[:, -1] - 0.5 * (Ucell[:, 1:-1] ** 2).sum(1) / rho_b)
        rho = fv[..., 0]
        ok_r = np.abs(rho - rho_b[:, None]) <= p.tvd_theta * np.maximum(np.abs(rho_b), p.tvd_eps)[:, None]
        with np.errstate(divide="ignore", invalid="ignore"):
            pres = (g - 1) * (fv[..., -1] - 0.5 * (fv[..., 1:-1] ** 2).sum(-1) / rho)
        ok_p = np.abs(pres - pres_b[:, None]) <= p.tvd_theta * np.maximum(np.abs(pres_b), p.tvd_eps)[:, None]
        return np.all(~valid | (ok_r & ok_p), axis=1)

    def cwenoz(self, cells, U):
        """CWENOZ reconstruction (Section 2.3): face values [n, NGPC, nvar].

        Conserved variables (default): every conserved variable on its own.
        Characteristic variables (cweno_vars = 1): per face, on the
        projection W = L U of reading in oracle/characteristic.py, mapped
        back at the face's Gauss points."""
        if self.p.cweno_vars == 1:
            return self.cwenoz_characteristic(cells, U)
        tab, a1, a_hat, svalid, nd, lam1, lams = self.cwenoz_fits(cells, U)
        om1, oms, SI1, SIs, tau, a_cw = self.cwenoz_weights(a1, a_hat, tab["OI"], svalid, nd, lam1, lams)
        phi = self.phi_at_gp(tab)
        fv = U[cells][:, None, :] + np.einsum("ngk,nkv->ngv", phi, a_cw)
        return fv, dict(om1=om1, oms=oms, SI1=SI1, SIs=SIs, tau=tau, lam1=lam1, lams=lams, a_cw=a_cw)

    def cwenoz_fits(self, cells, U):
        """The candidate polynomials of Section 2.3 in conserved variables:
        p_1's coefficients a1 [n, K, nvar] (from the central fit a_opt =
        lam_1 p_1 + sum_s lam_s p_s) and the directional degree-1 fits a_hat
        [n, NF, K, nvar] (zero past degree 1 and past the cell's count)."""
        p = self.p
        d, K = self.d, self.K
        a_opt, _, tab = self.linear(cells, U)
        n = cells.size
        nd = self.st.n_dir[cells]                                   # s_t - 1
        NF = self.st.dir.shape[1]
        ids = np.where(self.st.dir[cells] >= 0, self.st.dir[cells], cells[:, None, None])
        dUd = U[ids] - U[cells][:, None, None, :]                   # [n, NF, Md, nvar]
        a_dir = np.einsum("nfjm,nfmv->nfjv", tab["Pdir"], dUd)       # [n, NF, d, nvar]
        a_hat = np.zeros((n, NF, K, self.nvar))
        a_hat[:, :, :d] = a_dir
        lam1 = 1.0 - 1.0 / p.lambda1_prime
        lams = (1.0 - lam1) / nd                                    # [n]
        svalid = np.arange(NF)[None, :] < nd[:, None]               # [n, NF]
        a_hat = a_hat * svalid[..., None, None]
        a1 = (a_opt - lams[:, None, None] * a_hat.sum(1)) / lam1
        return tab, a1, a_hat, svalid, nd, lam1, lams

    def cwenoz_weights(self, a1, a_hat, OI, svalid, nd, lam1, lams):
        """Smoothness indicators SI = a^T OI a, tau, nonlinear weights and the
        combined coefficients, per variable (last axis), for any leading
        shape: a1 [..., K, V], a_hat [..., NF, K, V], OI [..., K, K],
        svalid [..., NF], nd and lams [...]."""
        p = self.p
        SI1 = np.einsum("...kv,...kq,...qv->...v", a1, OI, a1)
        SIs = np.einsum("...fkv,...kq,...fqv->...fv", a_hat, OI, a_hat)
        tau = (np.abs(SIs - SI1[..., None, :]) * svalid[..., None]).sum(-2) / nd[..., None]
        lams = lams[..., None, None]
        if p.cweno_form == 0:
            w1 = lam1 * (1.0 + (tau / (p.eps_w + SI1)) ** p.b_w)
            ws = lams * (1.0 + (tau[..., None, :] / (p.eps_w + SIs)) ** p.b_w)
        else:
            tb = tau ** p.b_w
            w1 = lam1 * (1.0 + tb / (p.eps_w + SI1))
            ws = lams * (1.0 + tb[..., None, :] / (p.eps_w + SIs))
        ws = ws * svalid[..., None]
        tot = w1 + ws.sum(-2)
        om1 = w1 / tot
        oms = ws / tot[..., None, :]
        a_cw = om1[..., None, :] * a1 + np.einsum("...fv,...fkv->...kv", oms, a_hat)
        return om1, oms, SI1, SIs, tau, a_cw

    def cwenoz_characteristic(self, cells, U, eig=None):
        """CWENOZ in characteristic variables, face by face (reading in
        oracle/characteristic.py): every Gauss-point slot of a cell takes the
        projection of its face.  The fits are linear in the data, so the
        characteristic fits are L times the conserved ones; the weights are
        taken per characteristic field; the face values are U_i + R dW(x).
        `eig(UL, UR, n) -> (R, L)` replaces the eigenvectors (tests)."""
        from .characteristic import roe_average, eigenvectors
        g = self.p.gamma
        geo, mesh = self.geo, self.mesh
        tab, a1, a_hat, svalid, nd, lam1, lams = self.cwenoz_fits(cells, U)
        gidx = np.maximum(geo.c_gidx[cells], 0)                     # [n, S]
        side = geo.c_side[cells]
        face = np.searchsorted(geo.gp_off, gidx, side="right") - 1
        nrm = geo.normal[face] * np.where(side == 0, 1.0, -1.0)[..., None]
        other = mesh.face_cells[face, 1 - side]
        other = np.where(other >= 0, other, cells[:, None])
        UL = np.broadcast_to(U[cells][:, None, :], other.shape + (self.nvar,))
        UR = U[other]
        if eig is None:
            v, H, c = roe_average(UL, UR, g)
            Rm, Lm, _ = eigenvectors(v, H, c, nrm, g)               # [n, S, nv, nv]
        else:
            Rm, Lm = eig(UL, UR, nrm)
        a1W = np.einsum("nsvu,nku->nskv", Lm, a1)
        ahW = np.einsum("nsvu,nfku->nsfkv", Lm, a_hat)
        S = gidx.shape[1]
        rep = lambda x: np.repeat(x[:, None], S, axis=1)
        om1, oms, SI1, SIs, tau, a_cw = self.cwenoz_weights(a1W, ahW, rep(tab["OI"]), rep(svalid), rep(nd),
                                                           lam1, rep(lams))
        phi = self.phi_at_gp(tab)                                   # [n, S, K]
        dW = np.einsum("nsk,nskv->nsv", phi, a_cw)
        fv = U[cells][:, None, :] + np.einsum("nsuv,nsv->nsu", Rm, dW)
        return fv, dict(om1=om1, oms=oms, SI1=SI1, SIs=SIs, tau=tau, a_cw=a_cw)

    def muscl(self, cells, U):
        """MUSCL (Section 2.2) with the Barth-Jespersen limiter, or with
        Venkatakrishnan's (the comparison of Section 3.2), eps^2 = (kappa h)^3."""
        tab = self.tables(cells)
        d = self.d
        ids = np.where(self.st.muscl[cells] >= 0, self.st.muscl[cells], cells[:, None])
        dU = U[ids] - U[cells][:, None, :]
        g = np.einsum("njm,nmv->njv", tab["Pmus"], dU)               # [n, d, nvar]
        phi = self.phi_at_gp(tab)[..., :d]
        delta = np.einsum("ngj,njv->ngv", phi, g)
        m, M = self.nad_bounds(cells, U)
        Ui = U[cells]
        up = (M - Ui)[:, None, :]
        dn = (m - Ui)[:, None, :]
        if self.p.limiter == VENKAT:
            room = np.where(delta > 0, up, dn)
            eps2 = ((self.p.kappa * self.geo.h[cells]) ** 3)[:, None, None]
            ratio = np.where(delta != 0, venkatakrishnan(delta, room, eps2), 1.0)
        else:
            with np.errstate(divide="ignore", invalid="ignore"):
                ratio = np.where(delta > 0, np.minimum(1.0, up / delta),
                                 np.where(delta < 0, np.minimum(1.0, dn / delta), 1.0))
        valid = np.arange(delta.shape[1])[None, :] < self.geo.c_ngp[cells][:, None]
        ratio = np.where(valid[..., None], ratio, 1.0)
        theta = np.minimum(1.0, ratio.min(1))
        fv = Ui[:, None, :] + theta[:, None, :] * delta
        return fv, dict(theta=theta, g=g)

    def cell_classes(self, cells, U):
        """Final class before the Harten check (mode, NAD, dilation)."""
        mode = self.p.scheme_mode
        if mode == ALL_LINEAR:
            return np.full(cells.size, LIN), None
        if mode == ALL_CWENOZ:
            return np.full(cells.size, CW), None
        if mode == ALL_MUSCL:
            return np.full(cells.size, MU), None
        nb = self.nbr[cells]
        closure = np.unique(np.concatenate([cells, nb[nb >= 0]]))
        own_c, info = self.own_class(closure, U)
        own = np.zeros(self.mesh.n_cells, np.int64)
        own[closure] = own_c
        cls = own[cells].copy()
        for j in range(nb.shape[1]):
            ok = nb[:, j] >= 0
            cls[ok] = np.maximum(cls[ok], own[nb[ok, j]])
        return cls, dict(closure=closure, own=own_c, info=info)

    def reconstruct_cells(self, cells, U):
        """Final face values [n, NGPC, nvar] and classes [n] of the given cells."""
        cells = np.asarray(cells, np.int64)
        cls, _ = self.cell_classes(cells, U)
        _, fv, _ = self.linear(cells, U)
        fv = fv.copy()
        for c, fn in ((CW, self.cwenoz), (MU, self.muscl)):
            sel = np.nonzero(cls == c)[0]
            if sel.size:
                fv[sel] = fn(cells[sel], U)[0]
        ok = self.harten_ok(fv, U[cells], self.geo.c_ngp[cells])
        cls = np.where(ok, cls, FO)
        fv = np.where(ok[:, None, None], fv, U[cells][:, None, :])
        return fv, cls

    def reconstruct(self, U):
        """All cells: face states [2, nvar, NGPT] and classes [N] (Section 2.5)."""
        N = self.mesh.n_cells
        cells = np.arange(N)
        fv, cls = self.reconstruct_cells(cells, U)
        fs = self.scatter_face_states(cells, fv)
        return fs, cls

    def scatter_face_states(self, cells, fv):
        geo = self.geo
        fs = np.full((2, self.nvar, geo.n_gp), np.nan)
        for i, c in enumerate(cells):
            k = geo.c_ngp[c]
            g = geo.c_gidx[c, :k]
            s = geo.c_side[c, :k]
            fs[s, :, g] = fv[i, :k]
        # boundary faces: transmissive ghost state on the right side
        bnd = self.mesh.face_cells[:, 1] < 0
        for f in np.nonzero(bnd)[0]:
            a, b = geo.gp_off[f], geo.gp_off[f + 1]
            fs[1, :, a:b] = fs[0, :, a:b]
        return fs
