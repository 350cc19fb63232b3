"""Navier-Stokes viscous fluxes (Section 2, Eqs. Terms1, sutherlandlaw,
HeatConduct, Stresses; Section 2.4, Eq. viscous_jump), GPU path through the
C ABI against the FP64 oracle: periodic triangles with the density jump (2D,
r = 2, 3: jumps exercise the penalty term), the mixed Riemann mesh
(transmissive boundaries), the mixed tetrahedron / pyramid / prism /
hexahedron box (3D, r = 3) and periodic hexahedra at r = 4 (the largest fits
of the FP64 slot-gradient pass).  FP64: classes bit-exact, residual within 1e-11 of the
variable's largest |R|; FP32: residual within 1e-4 of it (the viscous flux
differences gradients, about 1e-3 of the convective flux here, so its FP32
rounding sits near 1e-7 / 1e-3 of its own scale)."""
import json

import numpy as np
import pytest

from helpers import rel_err, near_threshold
from oracle import OracleModel, flux
from paper_2510_25906_amd.inputs import configs
from paper_2510_25906_amd.inputs.params import HYBRID, ALL_CWENOZ, ALL_LINEAR, ALL_MUSCL

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

VISC = dict(viscous=1, mu0=0.01, T0=1.0, sutherland_S=0.4, prandtl=0.72, visc_alpha=4.0 / 3.0)


@pytest.fixture(scope="module")
def hfv():
    from paper_2510_25906_amd import hfv as H
    H.load()
    assert torch.cuda.is_available()
    return H


def to_dev(U, dtype):
    return torch.tensor(np.ascontiguousarray(U.T), dtype=dtype, device="cuda")


CASES = {
    "c1_r2": lambda: configs.c1_density_jump(16, 2),
    "c1_r3": lambda: configs.c1_density_jump(16, 3),
    "c2_r3": lambda: configs.c2_riemann(32, 3),
    "c4_small": lambda: configs.c4_mixed("small"),
    "tgv_r4": lambda: configs.tgv_hex(8, 4),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("mode", [HYBRID, ALL_LINEAR, ALL_CWENOZ, ALL_MUSCL])
def test_viscous_residual_matches_oracle(hfv, case, mode):
    w = CASES[case]()
    p = w.params.with_(scheme_mode=mode, **VISC)
    om = OracleModel(w.mesh, w.stencils, p)
    R_o, fs_o, cls_o = flux.residual(om, w.U)
    om_e = OracleModel(w.mesh, w.stencils, p.with_(viscous=0))
    om_e._tab = om._tab
    R_e, _, _ = flux.residual(om_e, w.U)
    vis = float(np.abs(R_o - R_e).max() / np.abs(R_o).max())
    N = w.mesh.n_cells
    assert not near_threshold(om, w.U, np.arange(N), 1e-12).any()
    scale = np.abs(R_o).max(1)[:, None]
    for prec in (64, 32):
        ctx = hfv.Context(w.mesh, w.stencils, p, prec)
        for cfg in (dict(cwenoz_reuse=0, fused_residual=0), dict(cwenoz_reuse=1, fused_residual=1, linear_split=0,
                                                                 linear_lanes=1)):
            ctx.set_launch(**cfg)
            cls = torch.empty(N, dtype=torch.uint8, device="cuda")
            R = ctx.residual(to_dev(w.U, torch.float64 if prec == 64 else torch.float32), cell_class=cls)
            torch.cuda.synchronize()
            er = rel_err(R.double().cpu().numpy(), R_o, scale)
            print(f"{case} mode {mode} fp{prec} {cfg}: viscous part {vis:.2e} of |R|, residual error {er:.2e}",
                  flush=True)
            if prec == 64:
                assert np.array_equal(cls.cpu().numpy(), cls_o)
                assert er <= 1e-11
            else:
                assert er <= 1e-4
        ctx.close()
    assert vis > 1e-4          # the viscous fluxes are really in the residual


def test_viscous_frozen_residual_and_refusals(hfv):
    """The frozen residual with the forward's classes includes the viscous
    fluxes (equals the residual); the VJP and the allocation-free residual,
    which cover inviscid residuals only, refuse."""
    w = configs.c2_riemann(32, 3)
    p = w.params.with_(**VISC)
    ctx = hfv.Context(w.mesh, w.stencils, p, 64)
    ctx.set_launch(cwenoz_reuse=0)
    U = to_dev(w.U, torch.float64)
    cls = torch.empty(w.mesh.n_cells, dtype=torch.uint8, device="cuda")
    fs = ctx.new_face_states()
    R = ctx.residual(U, face_states=fs, cell_class=cls)
    R2 = ctx.residual_frozen(U, cls)
    torch.cuda.synchronize()
    assert float((R2 - R).abs().max() / R.abs().max()) <= 1e-13
    for call in (lambda: ctx.residual_vjp(U, cls, torch.ones_like(U)),
                 lambda: ctx.residual_noalloc(U, torch.empty_like(U), fs, cls)):
        with pytest.raises(hfv.HfvError) as ei:
            call()
        assert "HFV_ERR_STATE" in str(ei.value)
    ctx.close()


def test_viscous_tgv_time_loop_matches_oracle(hfv):
    """The study's supersonic viscous Taylor-Green setting (Section 3.6: Re =
    1600, M_ref = 1.25, periodic hexahedra) advanced two SSP(5,4) steps on the
    GPU equals the oracle's time loop (FP64 states within 1e-12 of each
    variable's largest value)."""
    from oracle import timestep as otime
    from paper_2510_25906_amd.timestep import SSPRK54, cfl_dt
    from paper_2510_25906_amd.tgv_study import viscous_params
    w = configs.tgv_hex(8, 2, perturb=False)
    p = viscous_params(w.params)
    ctx = hfv.Context(w.mesh, w.stencils, p, 64)
    U = to_dev(w.U, torch.float64)
    dt = cfl_dt(ctx, U, 1.4)
    rk = SSPRK54(ctx)
    for _ in range(2):
        rk.step(U, dt)
    torch.cuda.synchronize()
    om = OracleModel(w.mesh, w.stencils, p)
    U_o = otime.advance(om, w.U, dt, 2)
    err = (np.abs(U.cpu().numpy().T - U_o) / np.abs(U_o).max(0)).max()
    print(f"viscous TGV 8^3 r=2: dt {dt:.4g}, 2 steps, max relative state error {err:.2e}", flush=True)
    assert err <= 1e-12
    ctx.close()


def test_tgv_study_runs(hfv, capsys):
    """The time-integrated study on a tiny mesh: both modes in both precisions
    finish, class fractions sum to one, and the kinetic energy decays."""
    from paper_2510_25906_amd import tgv_study
    out = tgv_study.main(["--n", "8", "--r", "2", "--t-end", "0.2", "--prec", "64,32"])
    assert len(out) == 4
    for rec in out.values():
        assert rec["status"] == "ok" and rec["steps"] > 0
        assert abs(sum(rec["class_fractions"].values()) - 1.0) < 1e-9
        assert rec["kinetic_energy"][0] == (0.0, 1.0)
        assert 0.9 < rec["kinetic_energy"][-1][1] < 1.0
    summary = json.loads(capsys.readouterr().out.strip().splitlines()[-1])["summary"]
    assert set(summary) == {f"fp{p}_{k}" for p in (32, 64) for k in ("cwenoz_time_over_hybrid",
                                                                    "cwenoz_ms_per_step_over_hybrid")}
