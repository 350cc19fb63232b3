"""Host-side helpers of the benchmark (no GPU): the FP32-against-FP64 error
and the byte model's invariants."""
import numpy as np

import bench


def test_fp32_error_masks_padding_and_class_flips():
    rng = np.random.default_rng(0)
    ngpc, nvar, n = 4, 3, 10
    fs64 = rng.normal(size=(ngpc, nvar, n))
    fs32 = (fs64 + 1e-6).astype(np.float32)
    ngp = np.array([4, 4, 3, 3, 2, 4, 4, 1, 4, 4])
    for c in range(n):                      # garbage past each cell's Gauss points is ignored
        fs32[ngp[c]:, :, c] = 1e9
    cls64 = np.zeros(n, np.uint8)
    cls32 = cls64.copy()
    cls32[5] = 1                            # a flipped cell is left out and counted
    fs32[:, :, 5] = 1e9
    U = np.ones((n, nvar)) * 2.0
    out = bench.fp32_error((fs64, cls64), fs32, cls32, ngp, U)
    assert out["fp32_class_flips"] == 1
    assert 1e-7 < out["fp32_state_err_vs_fp64"] < 1e-6    # about 1e-6 / 2, FP32 rounding aside


def test_workloads_are_described():
    for key, (text, tag, prec) in bench.WORKLOADS.items():
        assert prec in (32, 64) and tag and "cells" in text


def test_scope_byte_model_per_cell():
    """The scope definition's bytes on a uniform periodic triangle mesh, where
    every cell has 3 faces, 3 vertices and the same Gauss-point count, against
    the per-cell formulas written out."""
    from types import SimpleNamespace
    from paper_2510_25906_amd.inputs import configs
    w = configs.c1_density_jump(8, 2)
    m, st = w.mesh, w.stencils
    ctx = SimpleNamespace(K=5, M=10, nvar=4)
    for prec, s in ((64, 8), (32, 4)):
        bm = bench.ByteModel(m, st, ctx, prec, 2)
        N, NF = m.n_cells, m.n_faces
        ngp = 3 * 2                                   # 3 edges x 2 Gauss-Legendre points (r = 2)
        K, M, nv, d, Md, nf = 5, 10, 4, 2, 4, 3
        lin = s * K * M + 4 * M + s * nv + s * K + s * d * 3 + s * nv * ngp + 1
        assert bm.s_linear() == N * lin
        allc = np.ones(N, bool)
        cw = s * K * (K + 1) // 2 + nf * (s * d * Md + 4 * Md) + s * nv * ngp
        assert bm.s_cwenoz_extra(allc) == N * cw
        assert bm.s_muscl_extra(allc) == N * (s * d * nf + s * nv * ngp)
        assert bm.s_flux() == NF * 2 * (2 * s * nv + s) + NF * (s * d + s * nv)
        assert bm.s_gather() == 2 * NF * s * nv + N * s * nv
        # the kernels as built never move fewer bytes than the scope definition
        cls = np.zeros(N, np.uint8)
        cls[: N // 3] = 1
        cls[N // 3: N // 2] = 2
        for mode in ("hybrid", "cwenoz", "linear"):
            sb = bm.s_per_kernel(mode, cls, False)
            mb = bm.per_kernel(mode, cls, False, False)
            assert sum(sb.values()) <= sum(mb.values())


def test_fp32_flips_split_by_margin():
    """A flip in a cell next to a near-threshold cell is flagged; a flip far
    from one is not."""
    n, ngpc, nvar = 6, 2, 1
    fs = np.zeros((ngpc, nvar, n))
    ngp = np.full(n, 2)
    cls64 = np.zeros(n, np.uint8)
    cls32 = cls64.copy()
    cls32[[1, 4]] = 1
    margin = np.full(n, 0.3)
    margin[0] = 1e-7                            # cell 0 near a threshold; cell 1 its neighbour
    face_cells = np.array([[0, 1], [1, 2], [2, 3], [3, 4], [4, 5], [5, -1]])
    out = bench.fp32_error((fs, cls64, margin), fs.astype(np.float32), cls32, ngp, np.ones((n, nvar)),
                           face_cells)
    assert out["fp32_class_flips"] == 2 and out["fp32_flips_unflagged"] == 1
    assert out["cells_margin_le_1e-6"] == 1
    # flip 1 sits next to cell 0 (margin 1e-7), flip 4 among cells at 0.3
    assert out["fp32_flip_margin_max"] == 0.3


def test_kernel_names_follow_the_launch():
    assert bench.kernel_name("linear", {"linear_split": 1}) == "k_linear_ms"
    assert bench.kernel_name("linear", {"linear_split": 2}) == "k_linear_ks"
    assert bench.kernel_name("cwenoz", {"cwenoz_reuse": 1}) == "k_cwenoz"
    assert bench.kernel_name("flux", {"fused_residual": 1}) == "k_residual"


def test_measured_traffic_matches_sources_and_kernel_instance(tmp_path, monkeypatch):
    """A counter record counts only for the sources it was taken on and, when
    a kernel instance is given, for that instance; a file may hold several
    records."""
    import json
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    assert bench.launch_string(dict(lanes_per_cell=4, block=256)) == "lanes_per_cell=4,block=256"
    h = bench.source_hash()
    recs = [dict(kernel="k_x<1>", source_hash=h, bytes_per_launch=100),
            dict(kernel="k_x<2>", source_hash="0" * 16, bytes_per_launch=200)]
    (tmp_path / "profiles" / "traffic_k_x_w.json").write_text(json.dumps({"records": recs}))
    assert bench.measured_traffic("k_x", "w", "k_x<1>") == 100
    assert bench.measured_traffic("k_x", "w", "k_x<2>") is None          # other sources
    assert bench.measured_traffic("k_x", "w", "k_x<3>") is None
    assert bench.measured_traffic("k_x", "w") == 100                     # any instance
    assert bench.measured_traffic("k_y", "w", "k_x<1>") is None          # no record
    (tmp_path / "profiles" / "traffic_k_z_w.json").write_text(json.dumps(recs[0]))   # a single record
    assert bench.measured_traffic("k_z", "w", "k_x<1>") == 100


def test_kernel_instance_names_match_the_profiler():
    """The instances the committed counter records were taken on, rebuilt from their launches."""
    import json
    import os
    for f in ("traffic_k_cwenoz_mixed2d_85k_r3.json", "traffic_k_linear_mixed3d_1m_r3.json"):
        rec = json.load(open(os.path.join(os.path.dirname(bench.__file__), "profiles", f)))
        for r in rec.get("records", [rec]):
            launch = {k: int(v) for k, v in (kv.split("=") for kv in r["launch"].split(","))}
            slot = "cwenoz" if "cwenoz" in f else "linear"
            dim, prec = (2, 64) if "2d" in r["workload"] else (3, 32)
            assert bench.kernel_instance(slot, launch, dim, 3, prec) == r["kernel"]
