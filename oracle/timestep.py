"""Oracle time integration (test infrastructure only): explicit
strong-stability-preserving Runge-Kutta in Shu-Osher form, FP64 NumPy.

The paper integrates in time with the five-stage, fourth-order SSP method of
Spiteri and Ruuth (Section 2.4).  A Shu-Osher method is given by
lower-triangular stage matrices alpha and beta: with u_0 = U^n,

    u_i = sum_{j<i} ( alpha[i-1, j] u_j + dt beta[i-1, j] L(u_j) ),  i = 1..s,

and U^{n+1} = u_s.  ALPHA and BETA below are the published SSP(5,4)
coefficients (SIAM J. Numer. Anal. 40 (2002)).  The pins in the tests check
them through the equivalent Butcher tableau (`butcher`) against the
fourth-order conditions and against an ODE with a known solution, so a
mistyped digit fails there.
"""
import numpy as np

ALPHA = np.array([
    [1.0, 0, 0, 0, 0],
    [0.444370493651235, 0.555629506348765, 0, 0, 0],
    [0.620101851488403, 0, 0.379898148511597, 0, 0],
    [0.178079954393132, 0, 0, 0.821920045606868, 0],
    [0, 0, 0.517231671970585, 0.096059710526147, 0.386708617503269],
])
BETA = np.array([
    [0.391752226571890, 0, 0, 0, 0],
    [0, 0.368410593050371, 0, 0, 0],
    [0, 0, 0.251891774271694, 0, 0],
    [0, 0, 0, 0.544974750228521, 0],
    [0, 0, 0, 0.063692468666290, 0.226007483236906],
])


def butcher(alpha=ALPHA, beta=BETA):
    """Butcher tableau (A, b, c) of a Shu-Osher method whose rows of alpha
    sum to one: writing every stage as u_i = u_0 + dt sum_j A[i, j] L(u_j)
    (stage s is the new value), row i of A is sum_j alpha[i-1, j] A[j] plus
    beta[i-1] by induction over the stages."""
    s = alpha.shape[0]
    A = np.zeros((s + 1, s + 1))            # stage 0 = u_0: no L terms
    for i in range(1, s + 1):
        for j in range(i):
            A[i, :] += alpha[i - 1, j] * A[j, :]
            A[i, j] += beta[i - 1, j]
    b = A[s, :s]
    Ab = A[:s, :s]
    return Ab, b, Ab.sum(1)


def step(L, u0, dt, alpha=ALPHA, beta=BETA):
    """One step of u' = L(u) from u0."""
    s = alpha.shape[0]
    u = [u0]
    Lu = [L(u0)]
    for i in range(1, s + 1):
        ui = np.zeros_like(u0)
        for j in range(i):
            if alpha[i - 1, j] != 0.0:
                ui = ui + alpha[i - 1, j] * u[j]
            if beta[i - 1, j] != 0.0:
                ui = ui + dt * beta[i - 1, j] * Lu[j]
        u.append(ui)
        if i < s:
            Lu.append(L(ui))
    return u[s]


def advance(model, U, dt, n_steps):
    """n_steps steps of dU/dt = R(U) for the oracle model (U [N, nvar])."""
    from .flux import residual
    L = lambda V: residual(model, V)[0].T
    for _ in range(n_steps):
        U = step(L, U, dt)
    return U
