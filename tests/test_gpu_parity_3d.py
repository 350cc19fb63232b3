"""3D GPU path against the FP64 oracle: tetrahedra (triangular faces), a
bounded hexahedral box, the periodic Taylor-Green vortex at r = 2 and r = 4,
and sampled cells of the 262,144-cell periodic hexahedral workloads."""
import numpy as np
import pytest

from helpers import state_scale, rel_err, near_threshold, gpu_cell_values, oracle_cell_values, states_err
from oracle import OracleModel, flux
from paper_2510_25906_amd.inputs import configs, fields
from paper_2510_25906_amd.inputs.mesh import hex_3d, tet_box
from paper_2510_25906_amd.inputs.stencil import build_stencils, cell_centroids
from paper_2510_25906_amd.inputs.params import Params, HYBRID, ALL_LINEAR, ALL_CWENOZ, ALL_MUSCL

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hfv():
    from paper_2510_25906_amd import hfv as H
    H.load()
    assert torch.cuda.is_available()
    return H


def to_dev(U, dtype):
    return torch.tensor(np.ascontiguousarray(U.T), dtype=dtype, device="cuda")


def with_jump(mesh, U, axis=0, at=None, factor=3.0):
    """Scale all conserved variables by ``factor`` beyond a plane (a contact jump)."""
    cen, _ = cell_centroids(mesh)
    at = np.median(cen[:, axis]) if at is None else at
    U = U.copy()
    U[cen[:, axis] > at] *= factor
    return U


def case(name):
    if name.startswith("tet"):
        r = int(name[-1])
        mesh = tet_box(4, 4, 4, jitter=0.2, seed=0)
        st = build_stencils(mesh, r)
        _, _, ev = fields.random_polynomial(3, 2, 5, seed=4, scale=0.2)
        U = fields.cell_average(mesh, lambda p: fields.prim_to_cons(
            np.concatenate([1.0 + 0.1 * np.tanh(ev(p)[..., :1]), 0.3 * np.sin(ev(p)[..., 1:4]),
                            1.0 + 0.1 * np.tanh(ev(p)[..., 4:5])], -1)), nq=4)
        return mesh, st, with_jump(mesh, U), Params(order_r=r)
    if name.startswith("hexbox"):
        r = int(name[-1])
        mesh = hex_3d(6, 6, 6, lo=(0, 0, 0), hi=(1.0, 1.2, 0.9))
        st = build_stencils(mesh, r)
        U = fields.cell_average(mesh, lambda p: fields.prim_to_cons(fields.tgv_prim(p * 6.0)), nq=4)
        return mesh, st, with_jump(mesh, U, axis=1), Params(order_r=r, riemann=1)
    if name.startswith("tgv"):
        n, r = int(name[3:5]), int(name[-1])
        w = configs.tgv_hex(n, r)
        return w.mesh, w.stencils, with_jump(w.mesh, w.U), w.params
    raise KeyError(name)


@pytest.mark.parametrize("name", ["tet4_r2", "tet4_r3", "hexbox6_r3", "tgv10_r2", "tgv10_r4"])
def test_3d_fp64_hybrid_residual(hfv, name):
    mesh, st, U, p = case(name)
    om = OracleModel(mesh, st, p)
    R_o, fs_o, cls_o = flux.residual(om, U)
    print(f"{name}: N={mesh.n_cells} classes={np.bincount(cls_o, minlength=4)}", flush=True)
    assert not near_threshold(om, U, np.arange(mesh.n_cells), 1e-12).any()
    for split in (0, 1, 2):
        ctx = hfv.Context(mesh, st, p, 64)
        ctx.set_launch(linear_split=split, linear_lanes=5 if split == 0 else 4, cwenoz_reuse=int(split > 0),
                       fused_residual=int(split != 1))
        fs = ctx.new_face_states()
        cls = torch.empty(mesh.n_cells, dtype=torch.uint8, device="cuda")
        R = ctx.residual(to_dev(U, torch.float64), face_states=fs, cell_class=cls)
        torch.cuda.synchronize()
        cls_g = cls.cpu().numpy()
        assert np.array_equal(cls_g, cls_o), np.nonzero(cls_g != cls_o)[0][:20]
        S = state_scale(U)
        assert states_err(fs, fs_o, om.geo, S) <= 1e-12
        assert rel_err(R.cpu().numpy(), R_o, np.abs(R_o).max(1)[:, None]) <= 1e-11
        ctx.close()


@pytest.mark.parametrize("name,mode", [("tet4_r3", ALL_CWENOZ), ("tet4_r3", ALL_MUSCL), ("tgv10_r4", ALL_CWENOZ),
                                       ("hexbox6_r3", ALL_MUSCL), ("tgv10_r2", ALL_LINEAR)])
def test_3d_fp64_forced_modes(hfv, name, mode):
    mesh, st, U, p = case(name)
    p = p.with_(scheme_mode=mode)
    om = OracleModel(mesh, st, p)
    R_o, fs_o, cls_o = flux.residual(om, U)
    ctx = hfv.Context(mesh, st, p, 64)
    fs = ctx.new_face_states()
    cls = torch.empty(mesh.n_cells, dtype=torch.uint8, device="cuda")
    R = ctx.residual(to_dev(U, torch.float64), face_states=fs, cell_class=cls)
    torch.cuda.synchronize()
    assert np.array_equal(cls.cpu().numpy(), cls_o)
    S = state_scale(U)
    assert states_err(fs, fs_o, om.geo, S) <= 1e-12
    assert rel_err(R.cpu().numpy(), R_o, np.abs(R_o).max(1)[:, None]) <= 1e-11
    ctx.close()


@pytest.mark.parametrize("lanes,split,lin_lanes", [(1, 0, 1), (5, 0, 5), (5, 1, 4), (5, 1, 8), (5, 2, 2),
                                                    (5, 2, 4), (1, 2, 8), (1, 0, 5)])
def test_3d_fp32_and_lane_shapes(hfv, lanes, split, lin_lanes):
    mesh, st, U, p = case("tgv10_r4")
    om = OracleModel(mesh, st, p)
    R_o, fs_o, cls_o = flux.residual(om, U)
    cells = np.arange(mesh.n_cells)
    flags = near_threshold(om, U, cells, 1e-6)
    ctx = hfv.Context(mesh, st, p, 32)
    ctx.set_launch(lanes=lanes, linear_split=split, linear_lanes=lin_lanes, cwenoz_reuse=int(split == 2))
    fs, cls = ctx.reconstruct(to_dev(U, torch.float32))
    torch.cuda.synchronize()
    cls_g = cls.cpu().numpy()
    flip = cls_g != cls_o
    nb = om.nbr
    near = flags | np.array([flags[nb[c][nb[c] >= 0]].any() for c in cells])
    assert not np.any(flip & ~near)
    fv_g = gpu_cell_values(fs.cpu().numpy(), om.geo, cells)
    fv_o = oracle_cell_values(fs_o, om.geo, cells)
    S = state_scale(U)
    assert rel_err(fv_g[~flip], fv_o[~flip], S[None, None, :]) <= 1e-5
    ctx.close()


@pytest.mark.parametrize("r,precs", [(2, (64, 32)), (4, (32,))])
def test_tgv64_sampled_full_size(hfv, r, precs):
    """The 262,144-cell periodic TGV workloads (r = 2 and r = 4) at full size, sampled."""
    w = configs.tgv_hex(64, r)
    U = w.U
    rng = np.random.default_rng(3)
    cells = np.unique(rng.choice(w.mesh.n_cells, 120, replace=False))
    om = OracleModel(w.mesh, w.stencils, w.params)
    fv_o, cls_o = om.reconstruct_cells(cells, U)
    for prec in precs:
        flags = near_threshold(om, U, cells, 1e-12 if prec == 64 else 1e-6)
        ctx = hfv.Context(w.mesh, w.stencils, w.params, prec)
        fs, cls = ctx.reconstruct(to_dev(U, torch.float64 if prec == 64 else torch.float32))
        torch.cuda.synchronize()
        cls_g = cls.cpu().numpy()[cells]
        print(f"tgv64 r={r} prec={prec} classes(sample)={np.bincount(cls_o, minlength=4)}", flush=True)
        flip = cls_g != cls_o
        if prec == 64:
            assert not flip.any()
        else:
            assert not np.any(flip & ~flags)
        fv_g = gpu_cell_values(fs.cpu().numpy(), om.geo, cells)
        S = state_scale(U)
        assert rel_err(fv_g[~flip], fv_o[~flip], S[None, None, :]) <= (1e-12 if prec == 64 else 1e-5)
        ctx.close()
