"""Pins of the oracle's time integrator (Section 2.4: the SSP(5,4)
Runge-Kutta method of Spiteri and Ruuth), checked against what the
mathematics fixes rather than against its own coefficients."""
import numpy as np

from oracle import OracleModel, timestep
from paper_2510_25906_amd.inputs import configs


def test_fourth_order_conditions():
    """The eight order conditions of a fourth-order Runge-Kutta method hold
    for the Butcher tableau derived from the Shu-Osher coefficients."""
    A, b, c = timestep.butcher()
    conds = [(b.sum(), 1.0), (b @ c, 1 / 2), (b @ c ** 2, 1 / 3), (b @ (A @ c), 1 / 6), (b @ c ** 3, 1 / 4),
             (b @ (c * (A @ c)), 1 / 8), (b @ (A @ c ** 2), 1 / 12), (b @ (A @ (A @ c)), 1 / 24)]
    for got, want in conds:
        assert abs(got - want) < 1e-13, (got, want)
    # and it is not fifth order: one fifth-order condition fails
    assert abs(b @ c ** 4 - 1 / 5) > 1e-4


def test_strong_stability_form():
    """Convex combinations of forward-Euler steps: nonnegative coefficients,
    rows of alpha summing to one, and the SSP coefficient min alpha/beta of
    about 1.508, the stability limit the paper quotes (CFL about 1.5)."""
    al, be = timestep.ALPHA, timestep.BETA
    assert np.all(al >= 0) and np.all(be >= 0)
    assert np.allclose(al.sum(1), 1.0, atol=1e-14)
    ratio = min(al[i, j] / be[i, j] for i in range(5) for j in range(5) if be[i, j] > 0)
    assert abs(ratio - 1.508) < 1e-3


def test_ode_convergence_order():
    """u' = -u^2, u(0) = 1, exact u = 1/(1 + t): halving dt divides the
    error at t = 2 by about 2^4."""
    L = lambda u: -u * u
    errs = []
    for n in (10, 20, 40, 80):
        dt, u = 2.0 / n, np.array([1.0])
        for _ in range(n):
            u = timestep.step(L, u, dt)
        errs.append(abs(u[0] - 1.0 / 3.0))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 3.8) and np.all(orders < 4.3), orders


def test_time_loop_keeps_free_stream_and_conserves():
    """On a periodic mesh a uniform state stays uniform, and the total of
    every conserved variable (sum of |V| U) is constant, through the
    hybrid residual inside the time loop."""
    w = configs.vortex_2d(8, 2)
    om = OracleModel(w.mesh, w.stencils, w.params)
    U0 = np.tile(w.U.mean(0), (w.mesh.n_cells, 1))
    U1 = timestep.advance(om, U0, 0.05, 2)
    assert np.abs(U1 - U0).max() <= 1e-13 * np.abs(U0).max()
    vol = om.geo.vol
    U2 = timestep.advance(om, w.U, 0.05, 2)
    tot0, tot2 = vol @ w.U, vol @ U2
    assert np.abs(tot2 - tot0).max() <= 1e-12 * np.abs(tot0).max()
    assert np.abs(U2 - w.U).max() > 1e-4          # the vortex did move
