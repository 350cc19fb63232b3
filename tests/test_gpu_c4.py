"""GPU path against the FP64 oracle on the mixed tetrahedron / prism / pyramid /
hexahedron box with a Mach-3 shock and three vortices, r = 3: the 4,488-cell
layout in full, with every launch mapping, and cells sampled from the
51,772-cell layout of the same recipe."""
import numpy as np
import pytest

from helpers import state_scale, rel_err, near_threshold, gpu_cell_values, states_err
from oracle import OracleModel, flux
from paper_2510_25906_amd.inputs import configs
from paper_2510_25906_amd.inputs.mesh import TET, PYR, PRISM, HEX
from paper_2510_25906_amd.inputs.params import HYBRID, ALL_CWENOZ, ALL_MUSCL

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hfv():
    from paper_2510_25906_amd import hfv as H
    H.load()
    assert torch.cuda.is_available()
    return H


@pytest.fixture(scope="module")
def small():
    w = configs.c4_mixed("small")
    assert set(np.unique(w.mesh.cell_type)) == {TET, PYR, PRISM, HEX}
    om = OracleModel(w.mesh, w.stencils, w.params)
    return w, om


def to_dev(U, dtype):
    return torch.tensor(np.ascontiguousarray(U.T), dtype=dtype, device="cuda")


def dilated(om, flags):
    nb = om.nbr
    return flags | np.array([flags[nb[c][nb[c] >= 0]].any() for c in range(len(flags))])


# (linear split, linear lanes, CWENOZ reuse, MUSCL lanes, class-list lanes,
# MUSCL and first-order lists merged into the CWENOZ launch, CWENOZ's OI
# read from its cell-major copy)
@pytest.mark.parametrize("split,lanes,reuse,mlanes,cwl,merged,cm", [(0, 5, 0, 0, 1, 0, 0), (0, 1, 1, 1, 1, 0, 0),
                                                                    (1, 4, 0, 5, 1, 0, 0), (2, 2, 1, 0, 1, 0, 0),
                                                                    (2, 4, 0, 1, 1, 0, 0), (0, 5, 0, 0, 5, 1, 0),
                                                                    (1, 4, 1, 0, 5, 1, 0), (2, 2, 0, 0, 1, 1, 0),
                                                                    (0, 5, 1, 0, 5, 1, 1), (1, 4, 0, 0, 1, 0, 1)])
def test_c4_small_fp64_hybrid(hfv, small, split, lanes, reuse, mlanes, cwl, merged, cm):
    w, om = small
    R_o, fs_o, cls_o = flux.residual(om, w.U)
    counts = np.bincount(cls_o, minlength=4)
    print(f"c4 small: N={w.mesh.n_cells} classes={counts}", flush=True)
    assert counts[1] > 0 and counts[2] > 0
    assert not near_threshold(om, w.U, np.arange(w.mesh.n_cells), 1e-12).any()
    ctx = hfv.Context(w.mesh, w.stencils, w.params, 64)
    ctx.set_launch(linear_split=split, linear_lanes=lanes, cwenoz_reuse=reuse, list_blocks=0 if reuse else 64,
                   muscl_lanes=mlanes, lanes=cwl, merged_lists=merged, lists_cell_major=cm)
    fs = ctx.new_face_states()
    cls = torch.empty(w.mesh.n_cells, dtype=torch.uint8, device="cuda")
    R = ctx.residual(to_dev(w.U, torch.float64), face_states=fs, cell_class=cls)
    torch.cuda.synchronize()
    cls_g = cls.cpu().numpy()
    assert np.array_equal(cls_g, cls_o), np.nonzero(cls_g != cls_o)[0][:20]
    S = state_scale(w.U)
    es = states_err(fs, fs_o, om.geo, S)
    er = rel_err(R.cpu().numpy(), R_o, np.abs(R_o).max(1)[:, None])
    print(f"state error {es:.2e}, residual error {er:.2e}", flush=True)
    assert es <= 1e-12 and er <= 1e-11
    ctx.close()


@pytest.mark.parametrize("mode", [ALL_CWENOZ, ALL_MUSCL])
def test_c4_small_fp64_forced_modes(hfv, small, mode):
    w, om0 = small
    p = w.params.with_(scheme_mode=mode)
    om = OracleModel(w.mesh, w.stencils, p)
    om._tab = om0._tab
    R_o, fs_o, cls_o = flux.residual(om, w.U)
    ctx = hfv.Context(w.mesh, w.stencils, p, 64)
    S = state_scale(w.U)
    for cm in (0, 1):       # CWENOZ's OI from the [entry][cell] table or its cell-major copy
        ctx.set_launch(lists_cell_major=cm)
        fs = ctx.new_face_states()
        cls = torch.empty(w.mesh.n_cells, dtype=torch.uint8, device="cuda")
        R = ctx.residual(to_dev(w.U, torch.float64), face_states=fs, cell_class=cls)
        torch.cuda.synchronize()
        assert np.array_equal(cls.cpu().numpy(), cls_o)
        es = states_err(fs, fs_o, om.geo, S)
        er = rel_err(R.cpu().numpy(), R_o, np.abs(R_o).max(1)[:, None])
        print(f"cell-major OI {cm}: state error {es:.2e}, residual error {er:.2e}", flush=True)
        assert es <= 1e-12 and er <= 1e-11
    ctx.close()


def test_c4_small_fp32(hfv, small):
    w, om = small
    fs_o, cls_o = om.reconstruct(w.U)
    cells = np.arange(w.mesh.n_cells)
    flags = dilated(om, near_threshold(om, w.U, cells, 1e-6))
    ctx = hfv.Context(w.mesh, w.stencils, w.params, 32)
    fs, cls = ctx.reconstruct(to_dev(w.U, torch.float32))
    torch.cuda.synchronize()
    cls_g = cls.cpu().numpy()
    flip = cls_g != cls_o
    print(f"fp32 flips {flip.sum()} (flagged {flags.sum()})", flush=True)
    assert not np.any(flip & ~flags), np.nonzero(flip & ~flags)[0][:10]
    fv_g = gpu_cell_values(fs.cpu().numpy(), om.geo, cells)
    from helpers import oracle_cell_values
    fv_o = oracle_cell_values(fs_o, om.geo, cells)
    e = rel_err(fv_g[~flip], fv_o[~flip], state_scale(w.U)[None, None, :])
    print(f"fp32 state error {e:.2e}", flush=True)
    assert e <= 1e-5
    ctx.close()


def test_c4_medium_sampled(hfv):
    """The 51,772-cell layout: sampled cells of every element type against the oracle."""
    w = configs.c4_mixed("medium")
    om = OracleModel(w.mesh, w.stencils, w.params)
    rng = np.random.default_rng(11)
    cells = np.unique(np.concatenate([rng.choice(np.nonzero(w.mesh.cell_type == t)[0], 40, replace=False)
                                      for t in (TET, PYR, PRISM, HEX)]))
    fv_o, cls_o = om.reconstruct_cells(cells, w.U)
    print(f"c4 medium: N={w.mesh.n_cells} sampled classes {np.bincount(cls_o, minlength=4)}", flush=True)
    for prec in (64, 32):
        flags = near_threshold(om, w.U, cells, 1e-12 if prec == 64 else 1e-6)
        ctx = hfv.Context(w.mesh, w.stencils, w.params, prec)
        fs, cls = ctx.reconstruct(to_dev(w.U, torch.float64 if prec == 64 else torch.float32))
        torch.cuda.synchronize()
        cls_g = cls.cpu().numpy()[cells]
        flip = cls_g != cls_o
        if prec == 64:
            assert not flip.any(), cells[flip][:10]
        else:
            assert not np.any(flip & ~flags)
        fv_g = gpu_cell_values(fs.cpu().numpy(), om.geo, cells)
        e = rel_err(fv_g[~flip], fv_o[~flip], state_scale(w.U)[None, None, :])
        print(f"fp{prec} sampled state error {e:.2e}", flush=True)
        assert e <= (1e-12 if prec == 64 else 1e-5)
        ctx.close()


@pytest.mark.parametrize("cfg", [dict(), dict(linear_split=1, linear_lanes=4, list_blocks=64, fused_residual=1),
                                 dict(linear_split=2, linear_lanes=8, lanes=1, cwenoz_reuse=1, list_blocks=0)])
def test_c4_block_order_does_not_change_results(hfv, small, cfg):
    """XCD-contiguous and plain block orders give bitwise identical classes,
    face states and residuals (the remap only permutes block ids)."""
    w, _ = small
    ctx = hfv.Context(w.mesh, w.stencils, w.params, 64)
    Ud = to_dev(w.U, torch.float64)
    out = []
    for remap in (0, 1):
        ctx.set_launch(xcd_remap=remap, **cfg)
        fs = torch.zeros_like(ctx.new_face_states())   # slots past a cell's Gauss points stay 0
        cls = torch.empty(w.mesh.n_cells, dtype=torch.uint8, device="cuda")
        R = ctx.residual(Ud, face_states=fs, cell_class=cls)
        torch.cuda.synchronize()
        out.append((fs, cls, R))
    assert torch.equal(out[0][1], out[1][1])
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][2], out[1][2])
    ctx.close()


def test_c4_small_near_margin(hfv, small):
    """near_margin on the mixed 3D box (four element types, ragged Gauss-point
    counts) under two linear mappings equals the oracle's in FP64, to the
    state bar 1e-12 carried through the margin's local normalisation
    (helpers.margin_tolerance)."""
    from helpers import margin_tolerance
    w, om = small
    N = w.mesh.n_cells
    ref = om.near_margin(np.arange(N), w.U)
    tol = margin_tolerance(om, w.U, np.arange(N), 1e-12)
    ctx = hfv.Context(w.mesh, w.stencils, w.params, 64)
    Ud = to_dev(w.U, torch.float64)
    for split, ll in ((0, 5), (2, 8)):
        ctx.set_launch(linear_split=split, linear_lanes=ll)
        mg = torch.empty(N, dtype=torch.float64, device="cuda")
        ctx.reconstruct(Ud, near_margin=mg)
        torch.cuda.synchronize()
        got = mg.cpu().numpy()
        fin = np.isfinite(ref)
        assert np.array_equal(np.isfinite(got), fin)
        err = float(np.abs(got[fin] - ref[fin]).max())
        worst = float((np.abs(got[fin] - ref[fin]) / tol[fin]).max())
        print(f"split {split}: margin error {err:.2e}, largest error / bound {worst:.2f}", flush=True)
        assert worst <= 1.0
    ctx.close()
