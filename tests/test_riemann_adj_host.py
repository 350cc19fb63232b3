"""The hand-written reverse mode of the HLLC and HLL fluxes (Section 2.4), built
for the host with g++, against the oracle's Riemann solver differentiated by
PyTorch autograd in FP64, on seeded states that reach every branch:
supersonic either way, the HLL average, and both HLLC star regions."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import torch

from oracle.adjoint import riemann

HERE = os.path.dirname(os.path.abspath(__file__))
GAMMA = 1.4


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("radj") / "riemann_adj_host")
    subprocess.run([gxx, "-O1", "-std=c++17", os.path.join(HERE, "riemann_adj_host.cpp"), "-o", out], check=True)
    return out


def cases(dim, count, seed):
    """Primitive states with Mach numbers up to about 3 along and against the
    normal, converted to conserved variables."""
    rng = np.random.default_rng(seed)
    n = rng.normal(size=(count, dim))
    n /= np.linalg.norm(n, axis=1, keepdims=True)

    def side():
        rho = rng.uniform(0.3, 3.0, count)
        p = rng.uniform(0.2, 5.0, count)
        c = np.sqrt(GAMMA * p / rho)
        mach = rng.uniform(-3.0, 3.0, count)
        v = mach[:, None] * c[:, None] * n + rng.normal(scale=0.5, size=(count, dim))
        E = p / (GAMMA - 1.0) + 0.5 * rho * (v ** 2).sum(1)
        return np.concatenate([rho[:, None], rho[:, None] * v, E[:, None]], 1)

    return side(), side(), n, rng.normal(size=(count, dim + 2))


def branches(qL, qR, n, hllc):
    """Which branch of the flux each case takes (0 left flux, 1 HLL average or
    left star, 2 right star, 3 right flux), from the primal wave speeds."""
    def prim(q):
        v = q[:, 1:-1] / q[:, :1]
        p = (GAMMA - 1.0) * (q[:, -1] - 0.5 * q[:, 0] * (v ** 2).sum(1))
        return q[:, 0], (v * n).sum(1), p, np.sqrt(GAMMA * p / q[:, 0])
    rL, uL, pL, cL = prim(qL)
    rR, uR, pR, cR = prim(qR)
    SL, SR = np.minimum(uL - cL, uR - cR), np.maximum(uL + cL, uR + cR)
    Ss = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) / (rL * (SL - uL) - rR * (SR - uR))
    if hllc:
        return np.where(SL >= 0, 0, np.where(Ss >= 0, 1, np.where(SR > 0, 2, 3)))
    return np.where(SL >= 0, 0, np.where(SR <= 0, 3, 1))


@pytest.mark.parametrize("dim,hllc", [(2, 1), (2, 0), (3, 1), (3, 0)])
def test_reverse_flux_matches_autograd(exe, dim, hllc):
    count = 4000
    qL, qR, n, gF = cases(dim, count, 100 * dim + hllc)
    lines = [f"{dim} {hllc} {count}"]
    for i in range(count):
        lines.append(" ".join(f"{x:.17g}" for x in np.concatenate([qL[i], qR[i], n[i], gF[i]])))
    res = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
    got = np.array([[float(x) for x in ln.split()] for ln in res.stdout.strip().split("\n")])
    assert got.shape == (count, 2 * (dim + 2))

    tL = torch.tensor(qL, requires_grad=True)
    tR = torch.tensor(qR, requires_grad=True)
    F = riemann(tL, tR, torch.tensor(n), GAMMA, hllc)
    (F * torch.tensor(gF)).sum().backward()
    want = np.concatenate([tL.grad.numpy(), tR.grad.numpy()], 1)

    br = branches(qL, qR, n, hllc)
    seen = np.bincount(br, minlength=4)
    print(f"dim {dim} hllc {hllc}: cases per branch {seen}")
    assert (seen[[0, 1, 3]] > 100).all() and (not hllc or seen[2] > 100)
    scale = np.abs(want).max(1) + np.abs(gF).max(1)
    err = np.abs(got - want).max(1) / scale
    print(f"worst relative difference {err.max():.2e}")
    assert err.max() <= 1e-11
