"""Explicit time integration of dU/dt = R(U) around the library's residual.

The paper advances its semi-discrete system with the five-stage, fourth-order
strong-stability-preserving Runge-Kutta method of Spiteri and Ruuth (Section
2.4).  In Shu-Osher form every stage is a convex combination of earlier
stages and forward-Euler steps of them:

    u_i = sum_j alpha_ij u_j + dt beta_ij R(u_j),   u_0 = U^n,  U^{n+1} = u_5,

with the published coefficients below (Spiteri and Ruuth, SIAM J. Numer.
Anal. 40 (2002), the SSP(5,4) scheme).  Each stage costs one residual
evaluation (hfv_residual) and one stage combination (hfv_rk_stage) on the
device, two for the last stage, which has five terms; nothing in the loop
runs on the host.
"""
from __future__ import annotations

import numpy as np

# (alpha_ij, beta_ij) of stage i, keyed by source stage j
SSP54 = (
    {0: (1.0, 0.391752226571890)},
    {0: (0.444370493651235, 0.0), 1: (0.555629506348765, 0.368410593050371)},
    {0: (0.620101851488403, 0.0), 2: (0.379898148511597, 0.251891774271694)},
    {0: (0.178079954393132, 0.0), 3: (0.821920045606868, 0.544974750228521)},
    {2: (0.517231671970585, 0.0), 3: (0.096059710526147, 0.063692468666290),
     4: (0.386708617503269, 0.226007483236906)},
)


def cfl_dt(ctx, U_host, cfl, gamma=1.4):
    """cfl * min over cells of h_c / (|u| + c) for cell averages U_host
    [n_cells][nvar] (h_c = |V|^(1/d), from the context's geometry table)."""
    d = ctx.dim
    h = ctx.table("GEOM")[d + 1]
    rho = U_host[:, 0]
    vel = U_host[:, 1:1 + d] / rho[:, None]
    p = (gamma - 1.0) * (U_host[:, -1] - 0.5 * rho * (vel ** 2).sum(1))
    speed = np.sqrt((vel ** 2).sum(1)) + np.sqrt(gamma * p / rho)
    return float(cfl * (h / speed).min())


class SSPRK54:
    """Advances a device state U [nvar][n_cells] in place through the
    library: `step(U, dt)` takes one step, `run(U, t_end, dt_max)` takes
    ceil(t_end / dt_max) equal steps ending exactly at t_end."""

    def __init__(self, ctx, stream=None):
        import torch
        self.ctx = ctx
        self.stream = stream
        shape = (ctx.nvar, ctx.n_cells)
        self.u = [None] + [torch.empty(shape, dtype=ctx.dtype, device="cuda") for _ in range(4)]
        self.r = [torch.empty(shape, dtype=ctx.dtype, device="cuda") for _ in range(2)]
        self.steps = 0

    def step(self, U, dt):
        """One step in place.  Stages 1-4 each combine u_0 with the previous
        stage and its residual; the last combines u_2, u_3, R(u_3), u_4 and
        R(u_4), in two stage calls.  Residual buffers alternate, so R(u_3)
        is still held when R(u_4) is computed."""
        ctx, s, u, r = self.ctx, self.stream, self.u, self.r
        u[0] = U
        for i in range(1, 5):
            j = i - 1                                   # source stage of the forward-Euler term
            a0 = SSP54[i - 1][0][0]
            aj, bj = SSP54[i - 1][j]
            Rj = ctx.residual(u[j], r[j % 2], stream=s)
            if j == 0:
                ctx.rk_stage(u[i], a0, u[0], 0.0, None, dt * bj, Rj, stream=s)
            else:
                ctx.rk_stage(u[i], a0, u[0], aj, u[j], dt * bj, Rj, stream=s)
        last = SSP54[4]
        # u_1 is free: (a_52 u_2 + a_53 u_3) + dt b_53 R(u_3), with R(u_3) in r[1]
        ctx.rk_stage(u[1], last[2][0], u[2], last[3][0], u[3], dt * last[3][1], r[1], stream=s)
        R4 = ctx.residual(u[4], r[0], stream=s)
        ctx.rk_stage(U, 1.0, u[1], last[4][0], u[4], dt * last[4][1], R4, stream=s)
        u[0] = None
        self.steps += 1
        return U

    def run(self, U, t_end, dt_max):
        n = max(1, int(np.ceil(t_end / dt_max - 1e-12)))
        dt = t_end / n
        for _ in range(n):
            self.step(U, dt)
        return n, dt
