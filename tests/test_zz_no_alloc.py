"""hfv_residual_noalloc (scratch in the library's fixed per-device array)
against hfv_residual, through the C ABI: two calls in a row, the second on a
smaller mesh, then the first mesh again, so that a call reading what an
earlier call left in the shared array would show.

Bars: classes bit-exact; with cwenoz_reuse 0 (both entry points run the same
kernels on the same operands) states and residuals bit for bit; with
cwenoz_reuse 1 (the allocation-free call refits CWENOZ's central polynomial
instead of reading the kept fit, summing in another order) FP64 states within
1e-12 of max(|x|, S_v) and residuals within 1e-11 of the variable's largest
|R|, FP32 states within 1e-5.
"""
import numpy as np
import pytest

from paper_2510_25906_amd.inputs import configs

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


def run_both(ctx, w, prec):
    dt = torch.float64 if prec == 64 else torch.float32
    U = to_dev(w.U, dt)
    N = w.mesh.n_cells
    out = []
    for call in ("residual", "residual_noalloc"):
        R = torch.full_like(U, float("nan"))
        fs = torch.zeros_like(ctx.new_face_states())       # slots past a cell's points stay 0 in both
        cls = torch.full((N,), 255, dtype=torch.uint8, device="cuda")
        if call == "residual":
            ctx.residual(U, R=R, face_states=fs, cell_class=cls)
        else:
            ctx.residual_noalloc(U, R, fs, cls)
        torch.cuda.synchronize()
        out.append((R.double().cpu().numpy(), fs.double().cpu().numpy(), cls.cpu().numpy()))
    return out


def compare(ctx, w, prec, reuse, label):
    (R1, fs1, c1), (R2, fs2, c2) = run_both(ctx, w, prec)
    S = np.abs(w.U).max(0)
    es = float(np.max(np.abs(fs2 - fs1) / np.maximum(np.abs(fs1), S[None, :, None])))
    er = float(np.max(np.abs(R2 - R1) / np.abs(R1).max(1)[:, None]))
    print(f"{label}: fp{prec} reuse {reuse} N={w.mesh.n_cells} classes {np.bincount(c1, minlength=4)} "
          f"state diff {es:.2e} residual diff {er:.2e}", flush=True)
    assert np.array_equal(c1, c2)
    assert np.all(np.isfinite(R2))
    if reuse == 0:
        assert np.array_equal(fs1, fs2) and np.array_equal(R1, R2)
    elif prec == 64:
        assert es <= 1e-12 and er <= 1e-11
    else:
        assert es <= 1e-5


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("reuse", [0, 1])
def test_noalloc_matches_residual_large_then_small(hfv, prec, reuse):
    big = configs.c2_riemann(128, 3)
    small = configs.c1_density_jump(16, 2)
    ctx_b = hfv.Context(big.mesh, big.stencils, big.params, prec)
    ctx_s = hfv.Context(small.mesh, small.stencils, small.params, prec)
    for c in (ctx_b, ctx_s):
        assert 0 < c.query("NOALLOC_BYTES") <= hfv.NOALLOC_SCRATCH_BYTES
        c.set_launch(cwenoz_reuse=reuse, list_blocks=0 if reuse else 512)
    assert ctx_s.query("NOALLOC_BYTES") < ctx_b.query("NOALLOC_BYTES")
    compare(ctx_b, big, prec, reuse, "first call, 128x128 mixed r=3")
    compare(ctx_s, small, prec, reuse, "second call, smaller 16x16 r=2")
    compare(ctx_b, big, prec, reuse, "third call, the first mesh again")
    ctx_b.close()
    ctx_s.close()


def test_noalloc_every_mode(hfv):
    """All-CWENOZ, all-MUSCL and all-linear modes clear the list lengths by
    their own kernels too."""
    from paper_2510_25906_amd.inputs.params import ALL_CWENOZ, ALL_MUSCL, ALL_LINEAR, HYBRID
    w = configs.c2_riemann(64, 3)
    ctx = hfv.Context(w.mesh, w.stencils, w.params, 64)
    ctx.set_launch(cwenoz_reuse=0)
    for mode in (ALL_CWENOZ, HYBRID, ALL_MUSCL, ALL_LINEAR, HYBRID):
        ctx.set_params(w.params.with_(scheme_mode=mode))
        compare(ctx, w, 64, 0, f"mode {mode}")
    ctx.close()
