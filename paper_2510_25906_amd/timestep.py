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


def cfl_dt(ctx, U, cfl):
    """Step size cfl / rate for the device state U, with the library's
    spectral-radius rate max_i (|u_i| + c_i) sum_f |S_f| / |V_i|."""
    r = float(ctx.cfl_rate(U).item())
    if not np.isfinite(r) or r <= 0.0:
        raise FloatingPointError("non-physical state")
    return cfl / r


class SSPRK54:
    """Advances a device state U [nvar][n_cells] in place through the
    library: `step(U, dt)` takes one step, `run(U, t_end, dt_max)` takes
    ceil(t_end / dt_max) equal steps ending exactly at t_end."""

    def __init__(self, ctx, stream=None):
        """Stage buffers are allocated here, once."""
        import torch
        self.ctx = ctx
        self.stream = stream
        shape = (ctx.nvar, ctx.n_cells)
        self.u = [None] + [torch.empty(shape, dtype=ctx.dtype, device="cuda") for _ in range(4)]
        self.r = [torch.empty(shape, dtype=ctx.dtype, device="cuda") for _ in range(2)]
        # classes of the last stage's evaluation, R(u_4), of the latest step
        self.cls = torch.empty(ctx.n_cells, dtype=torch.uint8, device="cuda")
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
        R4 = ctx.residual(u[4], r[0], cell_class=self.cls, stream=s)
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

    def run_cfl(self, U, t_end, cfl, max_steps=1_000_000, on_step=None, collapse=1e-3):
        """Steps of dt = cfl / rate(U) (hfv_cfl_rate, read back once per
        step), the last one shortened to end at t_end.  Raises
        FloatingPointError if the state stops being physical or the step
        size collapses below `collapse` times the first one (a blowing-up
        solution).  on_step(n, t) is called after each step."""
        import torch
        rate = torch.empty(1, dtype=torch.float64, device="cuda")
        t, n, dt0 = 0.0, 0, None
        while t < t_end * (1 - 1e-14):
            r = float(self.ctx.cfl_rate(U, rate, stream=self.stream).item())
            if not np.isfinite(r) or r <= 0.0:
                raise FloatingPointError(f"non-physical state after {n} steps at t = {t:.6g}")
            dt0 = cfl / r if dt0 is None else dt0
            if cfl / r < collapse * dt0:
                raise FloatingPointError(f"step size collapsed after {n} steps at t = {t:.6g}")
            dt = min(cfl / r, t_end - t)
            self.step(U, dt)
            t += dt
            n += 1
            if on_step is not None:
                on_step(n, t)
            if n >= max_steps:
                raise RuntimeError(f"more than {max_steps} steps")
        return n, t
