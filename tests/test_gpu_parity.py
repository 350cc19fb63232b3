"""GPU path (through the C ABI) against the FP64 oracle.

FP64: classes bit-exact, states within 1e-12 relative
(|x - x_ref| <= 1e-12 max(|x_ref|, S_v), S_v = max_cells |U_v|); residuals
within 1e-11 of the variable's largest |R|: R_i sums face fluxes that cancel
to a small difference, so a rounding of the fluxes at the 1e-16 level becomes
1e-13 - 1e-12 of the largest residual, and the bound keeps a factor of ten.
FP32: states within 1e-5 relative, class flips only in cells flagged within
1e-6 of a threshold (or their face neighbours, through the tagging step).
"""
import numpy as np
import pytest

from helpers import state_scale, rel_err, near_threshold, gpu_cell_values, oracle_cell_values, states_err
from oracle import OracleModel, flux
from paper_2510_25906_amd.inputs import configs, fields
from paper_2510_25906_amd.inputs.params import HYBRID, ALL_LINEAR, ALL_CWENOZ, ALL_MUSCL, preset

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


def dilated_flags(om, flags_cells, cells):
    out = flags_cells.copy()
    idx = {int(c): i for i, c in enumerate(cells)}
    for i, c in enumerate(cells):
        for j in om.nbr[c]:
            if j >= 0 and int(j) in idx and flags_cells[idx[int(j)]]:
                out[i] = True
    return out


@pytest.fixture(scope="module")
def c1():
    w = configs.c1_density_jump(32, 2)
    om = OracleModel(w.mesh, w.stencils, w.params)
    return w, om


@pytest.mark.parametrize("mode", [HYBRID, ALL_LINEAR, ALL_CWENOZ, ALL_MUSCL])
def test_c1_fp64_reconstruct_and_residual(hfv, c1, mode):
    w, om0 = c1
    p = w.params.with_(scheme_mode=mode)
    om = OracleModel(w.mesh, w.stencils, p)
    om._tab = om0._tab
    R_o, fs_o, cls_o = flux.residual(om, w.U)
    print(f"c1 fp64 mode={mode} classes={np.bincount(cls_o, minlength=4)}", flush=True)
    flags = near_threshold(om, w.U, np.arange(w.mesh.n_cells), 1e-12)
    assert not flags.any(), "seed has FP64 near-ties; choose another"
    ctx = hfv.Context(w.mesh, w.stencils, p, 64)
    Ud = to_dev(w.U, torch.float64)
    fs = ctx.new_face_states()
    cls = torch.empty(w.mesh.n_cells, dtype=torch.uint8, device="cuda")
    R = ctx.residual(Ud, face_states=fs, cell_class=cls)
    torch.cuda.synchronize()
    cls_g = cls.cpu().numpy()
    assert np.array_equal(cls_g, cls_o), np.nonzero(cls_g != cls_o)[0][:20]
    S = state_scale(w.U)
    assert states_err(fs, fs_o, om.geo, S) <= 1e-12
    assert rel_err(R.cpu().numpy(), R_o, np.abs(R_o).max(1)[:, None]) <= 1e-11
    # the two residual kernels (fused owner-computes, face fluxes + gather) agree bit for bit
    fused = ctx.get_launch()["fused_residual"]
    ctx.set_launch(fused_residual=1 - fused)
    R2 = ctx.residual(Ud, face_states=fs, cell_class=cls)
    torch.cuda.synchronize()
    assert torch.equal(R, R2)
    ctx.close()


def test_face_slot_table(hfv, c1):
    """Each face's first Gauss point sits at the published slot of both of its
    cells in the oracle's per-cell Gauss-point lists (faces in increasing id)."""
    w, om = c1
    ctx = hfv.Context(w.mesh, w.stencils, w.params, 64)
    t = ctx.table("FACE_SLOTS")
    geo = om.geo
    fc = w.mesh.face_cells
    for f in range(w.mesh.n_faces):
        g0 = geo.gp_off[f]
        for side in (0, 1):
            c = fc[f, side]
            if c < 0:
                assert (t[f] >> 8) & 255 == t[f] & 255
                continue
            slot = (t[f] >> (8 * side)) & 255
            assert geo.c_gidx[c, slot] == g0 and geo.c_side[c, slot] == side
    ctx.close()


def test_c1_tables_match_oracle(hfv, c1):
    w, om = c1
    ctx = hfv.Context(w.mesh, w.stencils, w.params, 64)
    cells = np.arange(w.mesh.n_cells)
    tab = om.tables(cells)
    def relmax(a, b):
        return float(np.abs(a - b).max() / np.abs(b).max())
    e_p = relmax(ctx.table("PINV"), np.transpose(tab["P"], (1, 2, 0)))          # [K, M, N]
    K = om.K
    iu = np.triu_indices(K)
    e_oi = relmax(ctx.table("OI"), tab["OI"][:, iu[0], iu[1]].T)
    geom = ctx.table("GEOM")
    e_c = float(np.abs(geom[:2].T - om.geo.cen).max())
    e_v = relmax(geom[2], om.geo.vol)
    e_d = relmax(ctx.table("PDIR"), np.transpose(tab["Pdir"], (1, 2, 3, 0)))     # [NFM, d, Md, N]
    e_m = relmax(ctx.table("PMUS"), np.transpose(tab["Pmus"], (1, 2, 0)))        # [d, NFM, N]
    print(f"table errors: P {e_p:.2e} OI {e_oi:.2e} centroid {e_c:.2e} vol {e_v:.2e} "
          f"Pdir {e_d:.2e} Pmus {e_m:.2e}", flush=True)
    assert e_p <= 1e-12 and e_oi <= 1e-12 and e_c <= 1e-14 and e_v <= 1e-13
    assert e_d <= 1e-11 and e_m <= 1e-11
    ctx.close()


@pytest.mark.parametrize("lanes,split,lin_lanes,reuse,mlanes,merged,cm",
                         [(1, 0, 1, 0, 0, 0, 0), (2, 0, 2, 1, 4, 0, 0), (4, 0, 4, 0, 1, 0, 0), (4, 1, 2, 1, 2, 0, 0),
                          (4, 1, 4, 0, 0, 0, 0), (2, 1, 8, 1, 1, 0, 0), (2, 2, 2, 1, 0, 0, 0), (2, 2, 4, 0, 4, 0, 0),
                          (1, 2, 8, 1, 2, 0, 0), (1, 0, 1, 0, 0, 1, 0), (2, 1, 2, 0, 4, 1, 0), (4, 0, 2, 1, 0, 1, 0),
                          (2, 2, 8, 1, 0, 1, 0), (1, 0, 1, 1, 0, 0, 1), (2, 1, 2, 0, 0, 1, 1), (4, 0, 2, 1, 0, 1, 1)])
def test_c1_launch_shapes_agree(hfv, c1, lanes, split, lin_lanes, reuse, mlanes, merged, cm):
    """Every work mapping, with and without the CWENOZ reuse of the linear
    pass's central fits, with CWENOZ's OI from its cell-major copy, with the
    MUSCL pass on its own lane count or with
    the MUSCL and first-order lists merged into the CWENOZ launch, gives the
    oracle's classes and states."""
    w, om = c1
    fs_o, cls_o = om.reconstruct(w.U)
    assert (cls_o == 2).sum() > 0
    ctx = hfv.Context(w.mesh, w.stencils, w.params, 64)
    ctx.set_launch(lanes=lanes, block=128, list_blocks=0 if reuse else 3, linear_split=split, linear_lanes=lin_lanes,
                   cwenoz_reuse=reuse, muscl_lanes=mlanes, merged_lists=merged, lists_cell_major=cm)
    assert ctx.get_launch()["cwenoz_reuse"] == reuse and ctx.get_launch()["merged_lists"] == merged
    assert ctx.get_launch()["lists_cell_major"] == cm
    fs, cls = ctx.reconstruct(to_dev(w.U, torch.float64))
    torch.cuda.synchronize()
    assert ctx.query("COUNT_CWENOZ") == int((cls_o == 1).sum()) > 0
    fs, cls = ctx.reconstruct(to_dev(w.U, torch.float64))
    torch.cuda.synchronize()
    assert np.array_equal(cls.cpu().numpy(), cls_o)
    S = state_scale(w.U)
    assert states_err(fs, fs_o, om.geo, S) <= 1e-12
    ctx.close()


def test_c1_fp32(hfv, c1):
    w, om = c1
    R_o, fs_o, cls_o = flux.residual(om, w.U)
    cells = np.arange(w.mesh.n_cells)
    flags = dilated_flags(om, near_threshold(om, w.U, cells, 1e-6), cells)
    ctx = hfv.Context(w.mesh, w.stencils, w.params, 32)
    Ud = to_dev(w.U, torch.float32)
    fs = ctx.new_face_states()
    cls = torch.empty(w.mesh.n_cells, dtype=torch.uint8, device="cuda")
    R = ctx.residual(Ud, face_states=fs, cell_class=cls)
    torch.cuda.synchronize()
    cls_g = cls.cpu().numpy()
    flip = cls_g != cls_o
    assert not np.any(flip & ~flags), np.nonzero(flip & ~flags)[0][:10]
    ok = ~flip
    S = state_scale(w.U)
    fv_g = gpu_cell_values(fs.cpu().numpy(), om.geo, cells)
    fv_o = oracle_cell_values(fs_o, om.geo, cells)
    assert rel_err(fv_g[ok], fv_o[ok], S[None, None, :]) <= 1e-5
    ctx.close()


def test_c2_sampled_full_size(hfv):
    """85k-cell mixed mesh, r = 3, in the benchmark's launch shape: sampled cells."""
    w = configs.c2_riemann(256, 3)
    rng = np.random.default_rng(7)
    for prec, tol in ((64, 1e-12), (32, 1e-5)):
        for mode in (HYBRID, ALL_CWENOZ, ALL_LINEAR):
            p = w.params.with_(scheme_mode=mode)
            om = OracleModel(w.mesh, w.stencils, p)
            cells = np.unique(np.concatenate([rng.choice(w.mesh.n_cells, 300, replace=False),
                                              np.arange(0, 40)]))
            fv_o, cls_o = om.reconstruct_cells(cells, w.U)
            flags = dilated_flags(om, near_threshold(om, w.U, cells, 1e-12 if prec == 64 else 1e-6), cells)
            print(f"c2 prec={prec} mode={mode} sampled={cells.size} flagged={flags.sum()}", flush=True)
            ctx = hfv.Context(w.mesh, w.stencils, p, prec)
            if mode == HYBRID:
                ctx.set_launch(linear_split=1 if prec == 64 else 2, linear_lanes=4, cwenoz_reuse=1)
            Ud = to_dev(w.U, torch.float64 if prec == 64 else torch.float32)
            fs, cls = ctx.reconstruct(Ud)
            torch.cuda.synchronize()
            cls_g = cls.cpu().numpy()[cells]
            flip = cls_g != cls_o
            if prec == 64:
                assert not flip.any(), cells[flip][:10]
            else:
                assert not np.any(flip & ~flags)
            fv_g = gpu_cell_values(fs.cpu().numpy(), om.geo, cells)
            S = state_scale(w.U)
            ok = ~flip
            assert rel_err(fv_g[ok], fv_o[ok], S[None, None, :]) <= tol
            ctx.close()


def test_free_stream_and_conservation(hfv):
    w = configs.c1_density_jump(32, 2)
    ctx = hfv.Context(w.mesh, w.stencils, w.params, 64)
    U = np.tile(fields.prim_to_cons(np.array([1.3, 0.4, -0.2, 2.0])), (w.mesh.n_cells, 1))
    R = ctx.residual(to_dev(U, torch.float64)).cpu().numpy()
    assert np.abs(R).max() < 1e-12
    R2 = ctx.residual(to_dev(w.U, torch.float64)).cpu().numpy()
    vol = ctx.table("GEOM")[2]
    assert np.abs((R2 * vol).sum(1)).max() < 1e-12 * np.abs(R2 * vol).sum()
    ctx.close()


def test_harten_fallback_on_negative_density(hfv):
    w = configs.c1_density_jump(32, 2)
    U = w.U.copy()
    U[37, 0] = -0.5
    ctx = hfv.Context(w.mesh, w.stencils, w.params, 64)
    fs, cls = ctx.reconstruct(to_dev(U, torch.float64))
    torch.cuda.synchronize()
    assert int(cls[37]) == 3
    ctx.close()


def test_rank_deficient_stencil_is_reported(hfv):
    w = configs.c1_density_jump(8, 2)
    st = w.stencils
    bad = st.central.copy()
    bad[5, :] = bad[5, 0]  # every stencil member the same cell
    from dataclasses import replace
    shift = st.central_shift.copy()
    shift[5, :] = shift[5, 0]
    st2 = replace(st, central=bad, central_shift=shift)
    with pytest.raises(hfv.HfvError) as ei:
        hfv.Context(w.mesh, st2, w.params, 64)
    assert "HFV_ERR_RANK" in str(ei.value) and "cell 5" in str(ei.value)


def test_set_launch_rejects_invalid_fields(hfv, c1):
    """An invalid launch field is refused with HFV_ERR_PARAM and leaves the
    configuration as it was."""
    w, _ = c1
    ctx = hfv.Context(w.mesh, w.stencils, w.params, 64)
    ctx.set_launch(lists_cell_major=1, merged_lists=1)
    before = ctx.get_launch()
    for bad in (dict(lists_cell_major=2), dict(lists_cell_major=-1), dict(merged_lists=2), dict(linear_lanes=3),
                dict(lanes=3), dict(block=96), dict(list_blocks=-1), dict(linear_split=3), dict(cwenoz_reuse=2)):
        with pytest.raises(hfv.HfvError) as ei:
            ctx.set_launch(**bad)
        assert "HFV_ERR_PARAM" in str(ei.value)
        assert ctx.get_launch() == before
    ctx.close()


def test_autotune_keeps_results(hfv, c1):
    """The autotuner applies the fastest configuration it timed, and the
    results under it are still the oracle's."""
    w, om = c1
    fs_o, cls_o = om.reconstruct(w.U)
    ctx = hfv.Context(w.mesh, w.stencils, w.params, 64)
    Ud = to_dev(w.U, torch.float64)
    best, recs = ctx.autotune(Ud, reps=3)
    assert ctx.get_launch() == best
    assert len(recs) >= 10 and all(np.isfinite(ms) and ms > 0 for _, ms in recs)
    # the last four records are the confirmation timings of the four fastest
    # configurations; the chosen one is the fastest of those
    last = recs[-4:]
    assert len({tuple(sorted(cfg.items())) for cfg, _ in last}) == 4
    assert min(last, key=lambda r: r[1])[0] == best
    fs, cls = ctx.reconstruct(Ud)
    torch.cuda.synchronize()
    assert np.array_equal(cls.cpu().numpy(), cls_o)
    assert states_err(fs, fs_o, om.geo, state_scale(w.U)) <= 1e-12
    ctx.close()


def test_gauss_point_frame_table(hfv, c1):
    """HFV_T_GP_XI: every cell's Gauss-point slots in its own frame,
    (x - x_c) / h_c, against the oracle's per-cell Gauss points; padded slots
    hold 0."""
    w, om = c1
    ctx = hfv.Context(w.mesh, w.stencils, w.params, 64)
    xi = ctx.table("GP_XI")                              # [NGPC][d][N]
    geo = om.geo
    want = (geo.c_x - geo.cen[:, None, :]) / geo.h[:, None, None]   # [N][NGPC][d]
    valid = np.arange(xi.shape[0])[None, :] < geo.c_ngp[:, None]
    got = xi.transpose(2, 0, 1)
    assert np.abs(np.where(valid[..., None], got - want, 0.0)).max() <= 1e-12
    assert np.all(np.where(valid[..., None], 0.0, got) == 0.0)
    ctx.close()


@pytest.mark.parametrize("prec", [64, 32])
def test_graph_replays_match_eager(hfv, c1, prec):
    """A residual captured into a HIP graph and replayed several times, with
    eager work and synchronisations between the replays and a new state
    written into the captured input each time, gives the eager residual bit
    for bit every time."""
    w, _ = c1
    dt = torch.float64 if prec == 64 else torch.float32
    ctx = hfv.Context(w.mesh, w.stencils, w.params, prec)
    U = to_dev(w.U, dt)
    R = torch.empty_like(U)
    fs = ctx.new_face_states()
    cls = torch.empty(w.mesh.n_cells, dtype=torch.uint8, device="cuda")
    g = ctx.graph_residual(U, R, fs, cls)
    rng = np.random.default_rng(5)
    for k in range(4):
        Uk = w.U * (1.0 + 0.01 * k * rng.uniform(-1, 1, size=w.U.shape))
        U.copy_(to_dev(Uk, dt))
        g.replay()
        torch.cuda.synchronize()
        R_graph, cls_graph = R.clone(), cls.clone()
        R_eager = ctx.residual(U.clone())                 # eager evaluation on the same state
        cls_eager = torch.empty_like(cls)
        ctx.residual(U.clone(), cell_class=cls_eager)
        torch.cuda.synchronize()
        assert torch.equal(R_graph, R_eager), k
        assert torch.equal(cls_graph, cls_eager), k
    ctx.close()


@pytest.mark.parametrize("mode", [HYBRID, ALL_LINEAR, ALL_CWENOZ])
def test_c1_near_margin_matches_oracle(hfv, c1, mode):
    """near_margin in FP64 under every linear mapping equals the oracle's to
    1e-12 (it is a relative distance, of order 1e-3 to 1 here); +inf exactly
    where the oracle has no decision."""
    w, om0 = c1
    p = w.params.with_(scheme_mode=mode)
    om = OracleModel(w.mesh, w.stencils, p)
    om._tab = om0._tab
    N = w.mesh.n_cells
    ref = om.near_margin(np.arange(N), w.U)
    ctx = hfv.Context(w.mesh, w.stencils, p, 64)
    Ud = to_dev(w.U, torch.float64)
    for split, ll in ((0, 1), (0, 4), (1, 2), (1, 8), (2, 4)):
        ctx.set_launch(linear_split=split, linear_lanes=ll)
        mg = torch.full((N,), -1.0, dtype=torch.float64, device="cuda")
        ctx.reconstruct(Ud, near_margin=mg)
        torch.cuda.synchronize()
        got = mg.cpu().numpy()
        fin = np.isfinite(ref)
        assert np.array_equal(np.isfinite(got), fin), (split, ll)
        err = float(np.abs(got[fin] - ref[fin]).max()) if fin.any() else 0.0
        print(f"mode {mode} split {split} lanes {ll}: margin error {err:.2e}, min margin "
              f"{ref[fin].min() if fin.any() else np.inf:.3e}", flush=True)
        assert err <= 1e-12
    ctx.close()


def test_fp32_flips_only_where_the_library_margin_is_small(hfv):
    """FP32 class flips against the FP64 path occur only in cells whose FP64
    near_margin (or a face neighbour's) is within 1e-6, on the 64 x 64
    mixed Riemann mesh with its seeded 1 % noise."""
    w = configs.c2_riemann(64, 3)
    om = OracleModel(w.mesh, w.stencils, w.params)
    N = w.mesh.n_cells
    out = {}
    for prec in (64, 32):
        dt = torch.float64 if prec == 64 else torch.float32
        ctx = hfv.Context(w.mesh, w.stencils, w.params, prec)
        mg = torch.empty(N, dtype=dt, device="cuda")
        fs, cls = ctx.reconstruct(to_dev(w.U, dt), near_margin=mg)
        torch.cuda.synchronize()
        out[prec] = (cls.cpu().numpy(), mg.double().cpu().numpy())
        ctx.close()
    flip = out[64][0] != out[32][0]
    small = out[64][1] <= 1e-6
    flagged = dilated_flags(om, small, np.arange(N))
    print(f"flips {flip.sum()}, cells with margin <= 1e-6: {small.sum()}", flush=True)
    assert not np.any(flip & ~flagged)
    # the FP32 margins track the FP64 ones to FP32 rounding of the states
    fin = np.isfinite(out[64][1]) & np.isfinite(out[32][1])
    assert fin.sum() > 0.99 * N
    assert np.abs(out[32][1][fin] - out[64][1][fin]).max() <= 1e-4


@pytest.mark.parametrize("r", [5, 6])
def test_2d_high_order_matches_oracle(hfv, r):
    """Degrees 5 and 6 in 2D (Table 1's P7 runs r = 6): K = 20 and 27
    unknowns, M = 40 and 54 stencil members.  Periodic triangles with the
    density jump, FP64, hybrid and all-CWENOZ: classes bit-exact, states
    within 1e-12, residual within 1e-11; FP32 hybrid with the flip allowance."""
    w = configs.c1_density_jump(24, r)
    N = w.mesh.n_cells
    for mode in (HYBRID, ALL_CWENOZ):
        p = w.params.with_(scheme_mode=mode)
        om = OracleModel(w.mesh, w.stencils, p)
        R_o, fs_o, cls_o = flux.residual(om, w.U)
        print(f"r={r} mode={mode}: classes {np.bincount(cls_o, minlength=4)}", flush=True)
        assert not near_threshold(om, w.U, np.arange(N), 1e-12).any()
        for prec in (64, 32):
            ctx = hfv.Context(w.mesh, w.stencils, p, prec)
            for cfg in (dict(linear_split=0, linear_lanes=1, lanes=1),
                        dict(linear_split=2, linear_lanes=4, lanes=4, cwenoz_reuse=1, list_blocks=0)):
                ctx.set_launch(**cfg)
                fs = ctx.new_face_states()
                cls = torch.empty(N, dtype=torch.uint8, device="cuda")
                Ud = to_dev(w.U, torch.float64 if prec == 64 else torch.float32)
                R = ctx.residual(Ud, face_states=fs, cell_class=cls)
                torch.cuda.synchronize()
                cls_g = cls.cpu().numpy()
                S = state_scale(w.U)
                if prec == 64:
                    assert np.array_equal(cls_g, cls_o)
                    es = states_err(fs, fs_o, om.geo, S)
                    er = rel_err(R.cpu().numpy(), R_o, np.abs(R_o).max(1)[:, None])
                    print(f"  fp64 {cfg}: state error {es:.2e}, residual error {er:.2e}", flush=True)
                    assert es <= 1e-12 and er <= 1e-11
                else:
                    cells = np.arange(N)
                    flip = cls_g != cls_o
                    flags = dilated_flags(om, near_threshold(om, w.U, cells, 1e-6), cells)
                    assert not np.any(flip & ~flags)
                    fv_g = gpu_cell_values(fs.cpu().numpy(), om.geo, cells)
                    fv_o = oracle_cell_values(fs_o, om.geo, cells)
                    e = rel_err(fv_g[~flip], fv_o[~flip], S[None, None, :])
                    print(f"  fp32 {cfg}: flips {flip.sum()}, state error {e:.2e}", flush=True)
                    assert e <= 1e-5
            ctx.close()
