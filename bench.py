"""Throughput of the CT-MHD step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--config turb128|turb256|turb512]
                [--precision fp64|fp32] [--emf q26|b25a] [--no-cpu-baseline]

Prints one JSON line.  A step is one full RK2-SSP step with first-order flux
correction (dt reduction, ghost wrap, both stages: primitives,
reconstruction, Riemann fluxes, edge EMFs, LD04, Ohmic terms, CT and
conserved updates, invalid-state flagging) on a seeded synthetic state
resident in HBM.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CONFIGS = {
    # the 128^3 driven-free turbulent box: rms Mach 5, b = (0.1,0,0) + curl A, PPM
    "turb128": dict(n=128, recipe="turbulent_mach5", recon="ppm", eta=0.0,
                    name="turbulent-box-128^3-mach5"),
    # the throughput sweep: rms Mach 2, beta 1, eta 1e-3, PPM
    "turb256": dict(n=256, recipe="turbulent_mach2_beta1", recon="ppm", eta=1e-3,
                    name="turbulent-box-256^3-mach2-beta1-eta1e-3"),
    "turb512": dict(n=512, recipe="turbulent_mach2_beta1", recon="ppm", eta=1e-3,
                    name="turbulent-box-512^3-mach2-beta1-eta1e-3"),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="turb128", choices=sorted(CONFIGS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--emf", default="q26", choices=["q26", "b25a", "fs18"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2609_10816_amd import ctmhd, inputs

    cfg = CONFIGS[args.config]
    t0 = time.time()
    cons, bf, info = getattr(inputs, cfg["recipe"])(cfg["n"])
    print(f"[bench] input {cfg['name']} generated in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    P = ctmhd.make_params(recon=cfg["recon"], emf=args.emf, eta=cfg["eta"], cfl=0.3,
                          precision=args.precision)
    ng = ctmhd.required_ghosts(P)
    st = ctmhd.BoxState.from_numpy(cons, bf, ng, info["dx"])
    del cons, bf
    S = ctmhd.Stepper(P, st)
    dev = st.cons[0].device
    K, W = args.steps, args.warmup
    dts = torch.zeros(max(K, W, 1), dtype=torch.float64, device=dev)
    diag = torch.zeros(4 * max(K, W, 1), dtype=torch.int64, device=dev)
    if W:
        S.step(W, None, dts, diag)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    S.step(K, None, dts, diag)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    ncell = cfg["n"] ** 3
    value = ncell * K / el / 1e6
    dg = diag[: 4 * K].view(K, 4).cpu().numpy()
    out = {
        "metric": "Mcell-updates/s on 1 MI355X",
        "value": value,
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": el / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "recon": cfg["recon"], "riemann": "hlld",
                   "emf": args.emf, "averaging": "ld04", "fofc": True, "cfl": 0.3,
                   "eta": cfg["eta"], "precision": args.precision},
        "fofc_flagged_cells": int(dg[:, :2].sum()),
        "hll_fallbacks": int(dg[:, 2].sum()),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
