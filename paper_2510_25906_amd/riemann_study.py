"""Time-integrated four-quadrant Riemann problem (Section 3.5, Eq.
2DRiemannProblem) on one GPU: the hybrid scheme with each NAD margin preset
of Fig. NADMargin (and the default one with the Venkatakrishnan limiter of the
comparison in Section 3.2), against all-CWENOZ and all-MUSCL, with CWENOZ on
conserved variables and (the `_char` variants) on characteristic variables
(Section 2.3), integrated in time at
CFL 0.6 with HLL fluxes and the SSP(5,4) time loop.

For every variant it reports the device time of the whole integration (the
per-step read-back of the CFL rate and of the class counts included), the
number of steps, the time-averaged fractions of the cell classes (the
library's list counts after each step's last residual evaluation) and the
cost relative to the default hybrid and to all-CWENOZ: the quantities the
paper quotes as a 41.67 % efficiency gain of the default hybrid over CWENOZ
and a 118 % extra cost of the MUSCL-CWENOZ preset over the default, on its
own meshes and CPUs (to t = 1).  The mesh is the seeded 256 x 256 mixed quad/triangle
mesh of the benchmark, without the benchmark's noise.  Prints one JSON line
per variant, then a summary line.  A variant whose solution blows up (a
non-physical state, or a step size collapsing) is reported with that status.

    python -m paper_2510_25906_amd.riemann_study [--n 256] [--r 3] [--t-end 0.25] [--prec 64]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from .inputs import configs
from .inputs.params import HYBRID, ALL_CWENOZ, ALL_MUSCL, PRESETS, VENKAT, CHARACTERISTIC

CHAR = dict(cweno_vars=CHARACTERISTIC)
VARIANTS = [(name, HYBRID, PRESETS[name]) for name in PRESETS] + \
           [("a_default_venkat", HYBRID, dict(PRESETS["a_default"], limiter=VENKAT)),
            ("all_cwenoz", ALL_CWENOZ, {}), ("all_muscl", ALL_MUSCL, {})] + \
           [(name + "_char", HYBRID, dict(PRESETS[name], **CHAR)) for name in PRESETS] + \
           [("all_cwenoz_char", ALL_CWENOZ, CHAR)]


def run_variant(w, name, mode, margins, t_end, cfl, prec, tune=True):
    import torch
    from . import hfv
    from .timestep import SSPRK54
    params = w.params.with_(scheme_mode=mode, **margins)
    ctx = hfv.Context(w.mesh, w.stencils, params, prec)
    dt = torch.float64 if prec == 64 else torch.float32
    U = torch.tensor(np.ascontiguousarray(w.U.T), dtype=dt, device="cuda")
    if tune:
        ctx.autotune(U.clone(), reps=3)
    N = w.mesh.n_cells
    rk = SSPRK54(ctx)
    # class counts summed on the device over the steps, from the classes the
    # residual returns (after the Harten fallback), read back once at the end
    acc = torch.zeros(4, dtype=torch.int64, device="cuda")

    def on_step(n, t):
        acc.add_(torch.bincount(rk.cls.to(torch.int64), minlength=4))
        if n % 2000 == 0:
            print(f"[riemann] {name}: step {n}, t = {t:.4f}", file=sys.stderr, flush=True)

    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.record()
    status = "ok"
    try:
        steps, t = rk.run_cfl(U, t_end, cfl, on_step=on_step)
    except FloatingPointError as e:
        steps, t, status = rk.steps, float("nan"), str(e)
    b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    Uh = U.double().cpu().numpy().T
    _, cls = ctx.reconstruct(U)
    final = np.bincount(cls.cpu().numpy(), minlength=4) / N
    ctx.close()
    # time average of the classes of each step's last stage evaluation
    fr = acc.cpu().numpy() / max(steps, 1) / N
    fracs = dict(linear=fr[0], cwenoz=fr[1], muscl=fr[2], first_order=fr[3])
    rec = dict(variant=name, mode=int(mode), margins=margins, status=status, steps=int(steps),
               ms_total=round(a.elapsed_time(b), 2), s_wall=round(wall, 3),
               ms_per_step=round(a.elapsed_time(b) / max(steps, 1), 4),
               class_fractions={k: round(float(v), 5) for k, v in fracs.items()},
               final_class_fractions=[round(float(x), 5) for x in final],
               rho_min=float(Uh[:, 0].min()), rho_max=float(Uh[:, 0].max()))
    return rec, Uh


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--r", type=int, default=3)
    ap.add_argument("--t-end", type=float, default=0.25)
    ap.add_argument("--cfl", type=float, default=0.6)
    ap.add_argument("--prec", type=int, choices=(32, 64), default=64)
    ap.add_argument("--variants", default=",".join(v[0] for v in VARIANTS))
    args = ap.parse_args(argv)
    w = configs.c2_riemann(args.n, args.r, noise=0.0)
    from . import hfv
    hfv.load()
    want = args.variants.split(",")
    out = {}
    for name, mode, margins in VARIANTS:
        if name not in want:
            continue
        rec, _ = run_variant(w, name, mode, margins, args.t_end, args.cfl, args.prec)
        rec.update(n_cells=w.mesh.n_cells, order_r=args.r, prec=args.prec, t_end=args.t_end, cfl=args.cfl)
        out[name] = rec
        print(json.dumps(rec), flush=True)
    summ = {}
    for tag in ("", "_char"):
        d = out.get("a_default" + tag)
        c = out.get("all_cwenoz" + tag)
        if d and c and d["status"] == "ok" and c["status"] == "ok":
            summ[f"cwenoz{tag}_time_over_default{tag}"] = round(c["ms_total"] / d["ms_total"], 3)
        if d and d["status"] == "ok":
            for k, v in out.items():
                if v["status"] == "ok" and k.endswith(tag) and (tag or not k.endswith("_char")):
                    summ[f"{k}_time_over_default{tag}"] = round(v["ms_total"] / d["ms_total"], 3)
    print(json.dumps({"summary": summ}), flush=True)
    return out


if __name__ == "__main__":
    main(sys.argv[1:])
