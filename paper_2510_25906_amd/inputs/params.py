"""Scheme parameters and the NAD margin presets of Section 2.5 (Fig. NADMargin).

Plain values only; shared by the library binding, its oracle and the tests.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

# scheme modes
HYBRID, ALL_LINEAR, ALL_CWENOZ, ALL_MUSCL = 0, 1, 2, 3
MODE_NAMES = {HYBRID: "hybrid", ALL_LINEAR: "linear", ALL_CWENOZ: "cwenoz", ALL_MUSCL: "muscl"}
# Riemann solvers
HLLC, HLL = 0, 1
# CWENOZ weight forms: the Z form (default) and the text's literal form
WENOZ_POW, LITERAL = 0, 1
# MUSCL slope limiters (Sections 2.2, 3.2): Barth-Jespersen, Venkatakrishnan
BJ, VENKAT = 0, 1
# variables CWENOZ reconstructs (Section 2.3): conserved, or characteristic
# (per face, eigenvectors of the flux Jacobian at the Roe average across it)
CONSERVED, CHARACTERISTIC = 0, 1
# cell classes, ordered by dissipation
LINEAR_CLASS, CWENOZ_CLASS, MUSCL_CLASS, FIRST_ORDER_CLASS = 0, 1, 2, 3


@dataclass(frozen=True)
class Params:
    order_r: int = 2
    scheme_mode: int = HYBRID
    riemann: int = HLLC
    cweno_form: int = WENOZ_POW
    limiter: int = BJ
    cweno_vars: int = CONSERVED
    gamma: float = 1.4
    # NAD margins (Eqs. marginm, marginw); default preset (a)
    alpha_m: float = 5e-3
    beta_m: float = 0.5
    alpha_w: float = 0.0
    beta_w: float = 0.0
    # NAD deactivation (Eq. NADDeactivatedCriteria): delta U < (kappa dx)^n
    kappa: float = 5.0
    n_exp: float = 2.0
    # CWENOZ (Section 2.3)
    lambda1_prime: float = 1e3
    eps_w: float = 1e-3
    b_w: float = 4.0
    # Harten bound check (Eq. harten_jump_fix)
    tvd_theta: float = 0.9
    tvd_eps: float = 1e-14
    # Navier-Stokes viscous fluxes (Section 2, Eqs. sutherlandlaw, HeatConduct,
    # Stresses; Section 2.4, Eq. viscous_jump); off by default (Euler).
    # Temperature T = p / rho; Sutherland mu = mu0 (T/T0)^1.5 (T0+S)/(T+S);
    # S = 110.4 K over a 273.15 K reference; penalty alpha = 4/3
    viscous: int = 0
    mu0: float = 0.0
    T0: float = 1.0
    sutherland_S: float = 110.4 / 273.15
    prandtl: float = 0.72
    visc_alpha: float = 4.0 / 3.0

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)


PRESETS = {
    "a_default": dict(alpha_m=5e-3, beta_m=0.5, alpha_w=0.0, beta_w=0.0),
    "b_relaxed": dict(alpha_m=1e-4, beta_m=1e-1, alpha_w=1e-4, beta_w=1e-3),
    "c_linear_cwenoz": dict(alpha_m=1e6, beta_m=1e9, alpha_w=0.0, beta_w=0.0),
    "d_linear_muscl": dict(alpha_m=0.0, beta_m=0.0, alpha_w=0.0, beta_w=0.0),
    "e_muscl_cwenoz": dict(alpha_m=0.0, beta_m=0.0, alpha_w=0.0, beta_w=-0.5),
}


def preset(name: str, **kw) -> Params:
    return Params(**{**PRESETS[name], **kw})
