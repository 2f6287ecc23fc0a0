"""Throughput of the CT-MHD step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--config turb512|turb256|turb128]
                [--precision fp64|fp32|fp32_r64] [--emf q26|b25a|fs18] [--no-cpu-baseline]
                [--no-fp32] [--no-sweep] [--no-batched] [--no-adjoint] [--copy-calibration]

Prints ONE JSON line.  A step is one full RK2-SSP step with first-order flux
correction on a seeded synthetic state already resident in HBM: CFL dt
reduction, ghost wrap, and for both stages primitives, reconstruction, HLLD
fluxes, edge EMFs, LD04 averaging, Ohmic terms, CT and conserved updates and
invalid-state flagging.  `value` is FP64 cell-updates per second of the
default workload, the primary throughput box: 512^3, resistive (eta 1e-3),
rms Mach 2, beta 1, PPM + HLLD + Q26 + LD04, FP64, K steps after W warm-up
steps.

roofline: the dominant kernel is the face kernel (reconstruction + HLLD at
every x_a face of one stage).  Its algorithmic work is face_flops (from
tests/golden/flops_per_unit.json, the oracle's operation count with each
reconstruction charged once) times the 3 n^3 interior faces (all three
directions) one launch resolves; its duration is measured with HIP events
recorded by the library around every launch inside the timed region.  The
path is bound by FP64 vector ALU throughput (peak 78.6 TFLOP/s on MI355X),
not by HBM.  traffic: HBM bytes per launch from the committed rocprofv3
counter summary of the same kernel source and workload, or null if the
kernel source has changed since.  step_hbm_measured: the counters' bytes of
every kernel of one step over the measured step time, against the 8 TB/s
HBM peak (same guard).

Beside the headline the same JSON line carries: fp32_form and
fp32_r64_form (the headline workload in the FP32 form, and in the FP32 form
with its Riemann solve in FP64), sweep (Q26 and B25a, FP64 and FP32 at 512^3 and
256^3, and the 128^3 Mach-5 box), level_form (the 128^3 box cut into 64
boxes of 32^3 that exchange ghost layers), batched_form (2000 AMR-like
boxes, both FP32 forms and FP64, 50 steps replayed from one HIP graph, against one
ctmhd_step call per box), adjoint_form (64^3 gradient of the kinetic energy
after 20 steps through the hand-written adjoint) and cpu_baseline (the
oracle on a 128^3 box of the headline recipe, on the host's cores, with the
CPU model).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CONFIGS = {
    # the 128^3 driven-free turbulent box: rms Mach 5, b = (0.1,0,0) + curl A, PPM
    "turb128": dict(n=128, recipe="turbulent_mach5", recon="ppm", eta=0.0,
                    name="turbulent-box-128^3-mach5-ppm"),
    # the throughput sweep: rms Mach 2, beta 1, eta 1e-3, PPM
    "turb256": dict(n=256, recipe="turbulent_mach2_beta1", recon="ppm", eta=1e-3,
                    name="turbulent-box-256^3-mach2-beta1-eta1e-3-ppm"),
    "turb512": dict(n=512, recipe="turbulent_mach2_beta1", recon="ppm", eta=1e-3,
                    name="turbulent-box-512^3-mach2-beta1-eta1e-3-ppm"),
}
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
ALG_BYTES_PER_CELL_UPDATE = 128.0  # 8 float64 fields read + written
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_face_kernel.txt")
FLOPS_FILE = os.path.join(ROOT, "tests", "golden", "flops_per_unit.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# the files the face kernel is compiled from
FACE_KERNEL_SOURCES = ("ctmhd.hip", "ctmhd_device.h", "ctmhd_host.h", "ctmhd_math.h")


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2609_10816_amd", "csrc")
    for name in FACE_KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(config, precision, emf, what="bytes_per_launch"):
    """HBM bytes from the committed counter summary (`bytes_per_launch`: one
    launch of the face kernel; `bytes_per_step`: every kernel of one step), if
    it was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha") != kernel_source_hash():
        return None
    key = f"{config}/{precision}/{emf}"
    v = kv.get(f"{what}[{key}]")
    return float(v) if v else None


def make_state(cfg):
    from paper_2609_10816_amd import inputs

    t0 = time.time()
    state = getattr(inputs, cfg["recipe"])(cfg["n"])
    log(f"input {cfg['name']} generated in {time.time() - t0:.1f}s")
    return state


def run_gpu(cfg, state, precision, emf, K, W, timer_pairs=0, copy_calibration=False):
    import torch

    from paper_2609_10816_amd import ctmhd

    cons, bf, info = state
    P = ctmhd.make_params(recon=cfg["recon"], emf=emf, eta=cfg["eta"], cfl=0.3,
                          precision=precision)
    ng = ctmhd.required_ghosts(P)
    st = ctmhd.BoxState.from_numpy(cons, bf, ng, info["dx"])
    S = ctmhd.Stepper(P, st)
    dev = st.cons[0].device
    if copy_calibration:
        # a plain copy of known size (1 GiB read + 1 GiB written) for scaling
        # the HBM byte counters of a profiler run
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    dts = torch.zeros(max(K, W, 1), dtype=torch.float64, device=dev)
    diag = torch.zeros(4 * max(K, W, 1), dtype=torch.int64, device=dev)
    if W:
        S.step(W, None, dts, diag)
    torch.cuda.synchronize()
    timer = ctmhd.KernelTimer(timer_pairs) if timer_pairs else None
    if timer:
        timer.start()
    t1 = time.perf_counter()
    S.step(K, None, dts, diag)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    kernel_ms = None
    nlaunch = 0
    if timer:
        nlaunch = timer.stop()
        d = timer.durations_ms(nlaunch)
        kernel_ms = sum(d) / len(d) if d else None
        timer.close()
    dg = diag[: 4 * K].view(K, 4).cpu().numpy()
    res = dict(elapsed=el, kernel_ms=kernel_ms, nlaunch=nlaunch,
               flagged=int(dg[:, :2].sum()), hll=int(dg[:, 2].sum()),
               dt_first=float(dts[0].item()))
    del S, st
    torch.cuda.empty_cache()
    return res


def run_batched_form(K, W, log_tune=True):
    """The batched AMR-like workload: 2000 periodic boxes with edges drawn
    per axis from {8, 16, 32, 64}, 4 ghost layers, PPM + HLLD + Q26 + LD04,
    global CFL dt.  The tile knob is picked by the autotuner; K steps are
    captured in one HIP graph and replayed once inside the timed region.
    Also times the same boxes stepped one ctmhd_step call at a time (the
    per-box loop the batched launch replaces)."""
    import torch

    from paper_2609_10816_amd import autotune, ctmhd, inputs

    t0 = time.time()
    states = inputs.amr_like_boxes(2000, seed=4)
    cells = sum(c[0].size for c, _, _ in states)
    log(f"batched input: 2000 boxes, {cells / 1e6:.2f} M cells, generated in "
        f"{time.time() - t0:.1f}s")
    out = {"workload": "amr-like-2000-boxes-8..64-ppm", "boxes": len(states), "cells": cells,
           "steps": K}
    for precision in ("fp32", "fp32_r64", "fp64"):
        P = ctmhd.make_params(recon="ppm", emf="q26", cfl=0.3, precision=precision)
        st = ctmhd.BatchedState.from_numpy(states, ctmhd.required_ghosts(P))
        if precision == "fp32":
            tile, tms = autotune.tune_batched(P, st, steps=2, reps=1)
            log("autotune (ms/step): " + ", ".join(
                f"{'persistent' if int(k) >> 16 else 'per-phase'} chunk {int(k) & 255}"
                f"/strips {(int(k) >> 8) & 255}: {v:.2f}" for k, v in tms.items()))
        P.tile = tile
        S = ctmhd.BatchedStepper(P, st)
        dev = st.cons[0].device
        dts = torch.zeros(max(K, W, 1), dtype=torch.float64, device=dev)
        diag = torch.zeros(4 * max(K, W, 1), dtype=torch.int64, device=dev)
        if W:
            S.step(W, dt_out=dts, diag=diag)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g):
                S.step(K, dt_out=dts, diag=diag)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.replay()
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        dg = diag[: 4 * K].view(K, 4).cpu().numpy()
        v = cells * K / el / 1e6
        log(f"batched {precision}: {v:.1f} Mcell-updates/s ({el / K * 1e3:.2f} ms/step, "
            f"flagged {int(dg[:, :2].sum())}, wait timeouts {int((dg[:, 3] & 2).any())})")
        out[precision] = {"value": v, "unit": "Mcell-updates/s", "ms_per_step": el / K * 1e3,
                          "fofc_flagged_cells": int(dg[:, :2].sum()),
                          "queue_wait_timeout": bool((dg[:, 3] & 2).any())}
        if precision == "fp32":
            out["tile"] = {"chunk": tile & 255 or 32, "strips": ((tile >> 8) & 255) or 1,
                           "schedule": "persistent" if tile >> 16 else "per-phase"}
            out["autotune_ms_per_step"] = {
                f"{'persistent' if int(k) >> 16 else 'per-phase'}/chunk{int(k) & 255}"
                f"/strips{(int(k) >> 8) & 255}": v for k, v in tms.items()}
            # the same boxes, one ctmhd_step call per box and step
            ws = torch.empty(max(ctmhd.workspace_bytes(P, ctmhd.make_box(b.n, b.ng, b.dx))
                                 for b in st.boxes), dtype=torch.uint8, device=dev)
            single = [ctmhd.make_box(tuple(b.n), b.ng, tuple(b.dx)) for b in st.boxes]
            views = [([st._view(t, k) for t in st.cons], [st._view(t, k) for t in st.bface])
                     for k in range(len(single))]
            Ploop = ctmhd.make_params(recon="ppm", emf="q26", cfl=0.3, precision=precision)
            Ploop.tile = tile
            nl = 2
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for n in range(nl):
                for k, bx in enumerate(single):
                    ctmhd.ctmhd_step(Ploop, bx, views[k][0], views[k][1], 1, dts[n:n + 1], None,
                                     None, ws)
            torch.cuda.synchronize()
            el_loop = time.perf_counter() - t1
            out["per_box_loop_fp32"] = {"value": cells * nl / el_loop / 1e6,
                                        "unit": "Mcell-updates/s",
                                        "ms_per_step": el_loop / nl * 1e3,
                                        "steps": nl}
            del ws, views
        del S, st, g
        torch.cuda.empty_cache()
    return out


def run_level_form(cfg, emf, state, K, W, box=32):
    """A box cut into a level of box^3 boxes (ctmhd_step_level:
    ghosts exchanged between the boxes after every update), FP64, the same
    scheme and steps as the single-box run of that box."""
    import torch

    from paper_2609_10816_amd import ctmhd

    cons, bf, info = state
    n = cfg["n"]
    cuts = (tuple(range(0, n + 1, box)),) * 3
    P = ctmhd.make_params(recon=cfg["recon"], emf=emf, eta=cfg["eta"], cfl=0.3)
    states, origin = ctmhd.split_level(cons, bf, info["dx"], cuts)
    st = ctmhd.BatchedState.from_numpy(states, ctmhd.required_ghosts(P))
    S = ctmhd.LevelStepper(P, st, origin, (n, n, n))
    dev = st.cons[0].device
    dts = torch.zeros(max(K, W, 1), dtype=torch.float64, device=dev)
    diag = torch.zeros(4 * max(K, W, 1), dtype=torch.int64, device=dev)
    if W:
        S.step(W, dt_out=dts, diag=diag)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    S.step(K, dt_out=dts, diag=diag)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    v = n ** 3 * K / el / 1e6
    log(f"level of {len(states)} boxes of {box}^3: {v:.1f} Mcell-updates/s "
        f"({el / K * 1e3:.3f} ms/step)")
    del S, st
    torch.cuda.empty_cache()
    return {"value": v, "unit": "Mcell-updates/s", "ms_per_step": el / K * 1e3,
            "workload": f"{cfg['name']} as a level of {len(states)} boxes of {box}^3",
            "precision": "fp64", "steps": K}


def _adjoint_step_times(P, cons, bf, dx, calls=20):
    """Mean time of one forward step (ctmhd_step with a frozen dt) and of one
    adjoint step (ctmhd_step_adjoint) on the same box, over `calls` calls
    each after a warm-up call.  The dt is the CFL dt of the first step."""
    import torch

    from paper_2609_10816_amd import ctmhd

    ng = ctmhd.required_ghosts(P)
    S = ctmhd.BoxState.from_numpy(cons, bf, ng, dx)
    G = ctmhd.BoxState.from_numpy(cons, bf, ng, dx)  # any cotangent
    O = ctmhd.BoxState(S.n, ng, dx)
    dev = S.cons[0].device
    ws_f = torch.empty(ctmhd.workspace_bytes(P, S.box), dtype=torch.uint8, device=dev)
    ws_a = torch.empty(ctmhd.adjoint_workspace_bytes(P, S.box), dtype=torch.uint8, device=dev)
    dtt = torch.zeros(1, dtype=torch.float64, device=dev)
    ctmhd.ctmhd_step(P, S.box, S.cons, S.bface, 1, None, dtt, None, ws_f)

    def fwd():
        ctmhd.ctmhd_step(P, S.box, S.cons, S.bface, 1, dtt, None, None, ws_f)

    def adj():
        ctmhd.ctmhd_step_adjoint(P, S.box, S.cons, S.bface, dtt, G.cons, G.bface, O.cons,
                                 O.bface, ws_a)

    out = []
    for f in (fwd, adj):
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(calls):
            f()
        torch.cuda.synchronize()
        out.append((time.perf_counter() - t0) / calls * 1e3)
    return out


def run_adjoint_form(nsteps=20, every=5, reps=3):
    """The derivative workload: 64^3 smooth periodic box (3 sine modes of
    amplitude 0.05 per field, beta = 1), PLM-MC or PPM + HLLD + Q26 + LD04,
    FP64 (also PLM-MC with the B25a and FS18 EMFs, and PLM-MC in the FP32 form), no
    flux correction; loss = total kinetic energy after `nsteps`
    steps; the gradient with respect to the initial velocity and face field
    through the hand-written adjoint with a checkpoint every `every` steps.
    Times the forward rollout alone and the backward pass (recomputation +
    adjoint steps), the fastest of `reps` repetitions each, and one adjoint
    step against one forward step of the same box."""
    import numpy as np
    import torch

    from paper_2609_10816_amd import autograd as ad
    from paper_2609_10816_amd import ctmhd, inputs

    n = 64
    cons, bf, info = inputs.smooth_modes_box(n, amp=0.05, beta=1.0, seed=5)
    dx = info["dx"]
    dev = "cuda"
    rho = torch.tensor(cons[0], device=dev)
    u0 = torch.tensor(cons[1:4] / cons[0], device=dev)
    bc = np.stack([0.5 * (bf[a] + np.roll(bf[a], -1, axis=2 - a)) for a in range(3)])
    p = torch.tensor((5.0 / 3.0 - 1.0) * (cons[4] - 0.5 * (cons[1:4] ** 2).sum(0) / cons[0] -
                                          0.5 * (bc ** 2).sum(0)), device=dev)
    b0 = torch.tensor(bf, device=dev)
    out = {"workload": "smooth-64^3-amp0.05-beta1-hlld-q26-ld04", "dtype": "f64",
           "steps": nsteps, "checkpoint_every": every,
           "loss": "total kinetic energy after the steps",
           "gradient": "d loss / d (initial velocity, initial face field)",
           "timing": f"fastest of {reps} repetitions"}
    for recon, prec, emf, tape in (("plm", "fp64", "q26", False), ("ppm", "fp64", "q26", False),
                                   ("plm", "fp64", "b25a", False), ("plm", "fp64", "fs18", False),
                                   ("plm", "fp32", "q26", False), ("plm", "fp64", "q26", True),
                                   ("ppm", "fp64", "q26", True)):
        P = ctmhd.make_params(recon=recon, riemann="hlld", emf=emf, eta=0.0, fofc=False,
                              precision=prec)
        kw = dict(tape=True) if tape else dict(every=every)
        tf_best = tb_best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with torch.no_grad():
                ad.rollout(ad.conserved_from_primitives(rho, u0, p, b0), b0, P, dx, nsteps, **kw)
            torch.cuda.synchronize()
            tf = time.perf_counter() - t0
            u = u0.clone().requires_grad_(True)
            b = b0.clone().requires_grad_(True)
            c, _ = ad.rollout(ad.conserved_from_primitives(rho, u, p, b), b, P, dx, nsteps, **kw)
            ke = ad.kinetic_energy(c, dx)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ke.backward()
            torch.cuda.synchronize()
            tb = time.perf_counter() - t1
            tf_best = tf if tf_best is None else min(tf_best, tf)
            tb_best = tb if tb_best is None else min(tb_best, tb)
        key = recon if prec == "fp64" else f"{recon}_fp32_form"
        if emf != "q26":
            key += f"_{emf}"
        if tape:
            key += "_tape"
        out[key] = {"forward_ms": tf_best * 1e3, "backward_ms": tb_best * 1e3,
                    "ratio_backward_to_forward": tb_best / tf_best,
                    "grad_norm_u": float(u.grad.norm()), "grad_norm_b": float(b.grad.norm())}
        msg = (f"adjoint form {key}: rollout forward {tf_best * 1e3:.1f} ms, backward "
               f"{tb_best * 1e3:.1f} ms (ratio {tb_best / tf_best:.2f})")
        if tape:
            out[key]["note"] = ("every forward step records its tape (ctmhd_step_record); the "
                                "backward reverses each step from its tape, no recomputation")
            if recon in out:
                plain = out[recon]["forward_ms"]
                out[key]["ratio_backward_to_plain_forward"] = tb_best * 1e3 / plain
                msg += f"; backward / plain forward {tb_best * 1e3 / plain:.2f}"
        elif prec == "fp64":
            f_ms, a_ms = _adjoint_step_times(P, cons, bf, dx)
            out[key].update({"step_forward_ms": f_ms, "step_adjoint_ms": a_ms,
                             "ratio_adjoint_step_to_forward_step": a_ms / f_ms})
            msg += f"; one step {f_ms:.3f} ms, its adjoint {a_ms:.3f} ms (ratio {a_ms / f_ms:.2f})"
        else:
            out[key]["note"] = ("forward and recomputation in the FP32 form, adjoint steps in "
                                "FP64 at the FP32-form states")
        log(msg)
    return out


def cpu_model():
    """The host CPU's model name and logical CPU count, from /proc/cpuinfo."""
    name, n = "unknown", 0
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                n += 1
                if name == "unknown":
                    name = line.split(":", 1)[1].strip()
    except OSError:
        pass
    return name, n or os.cpu_count()


def cpu_baseline(cfg, emf, n=128, min_seconds=12.0, max_steps=20):
    """The oracle (plain FP64 C++, OpenMP over z-planes, all the threads it is
    given) on an n^3 box of the headline recipe: the same scheme, rms Mach,
    beta and eta, at a size the host holds in seconds per step.  Steps one at
    a time until at least `min_seconds` of CPU work (at most `max_steps`)."""
    import oracle
    from paper_2609_10816_amd import inputs
    cons, bf, info = getattr(inputs, cfg["recipe"])(n)
    Q = oracle.make_params(recon=cfg["recon"], emf=emf, eta=cfg["eta"], cfl=0.3)
    n3 = n ** 3
    el, steps = 0.0, 0
    c, b = cons, bf
    while el < min_seconds and steps < max_steps:
        t0 = time.perf_counter()
        c, b, _, _ = oracle.step(Q, c, b, info["dx"], nsteps=1)
        el += time.perf_counter() - t0
        steps += 1
    model, ncpu = cpu_model()
    return {"value": n3 * steps / el / 1e6, "unit": "Mcell-updates/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{steps} steps of a {n}^3 box of the same recipe "
                      f"({n3 * steps / 1e6:.2f} M cell-updates, {el:.1f} s)",
            "cpu_model": model, "host_logical_cpus": ncpu}


def cpu_baseline_one_core(cfg, emf, n=64):
    """The oracle on one thread: one step of the n^3 box of the same recipe."""
    import oracle
    from paper_2609_10816_amd import inputs
    cons, bf, info = getattr(inputs, cfg["recipe"])(n)
    Q = oracle.make_params(recon=cfg["recon"], emf=emf, eta=cfg["eta"], cfl=0.3)
    nthr = oracle.num_threads()
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.step(Q, cons, bf, info["dx"], nsteps=1)
        el = time.perf_counter() - t0
    finally:
        oracle.set_threads(nthr)
    return {"value": n ** 3 / el / 1e6, "unit": "Mcell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"1 step of a {n}^3 box of the same recipe ({n ** 3 / 1e6:.2f} M "
                      f"cell-updates), {el:.1f} s"}


def run_sweep(primary, primary_state, emf, K, W, out):
    """The throughput sweep beside the headline: both EMF schemes (Q26 and
    B25a) and both forms (FP64, FP32) at 512^3 and 256^3 of the resistive
    Mach-2 box, and the 128^3 Mach-5 box (Q26), each for K timed steps after
    W warm-up steps."""
    sweep = {}
    for name in ("turb512", "turb256", "turb128"):
        cfg = CONFIGS[name]
        state = primary_state if name == primary else make_state(cfg)
        for e in (("q26", "b25a") if name != "turb128" else ("q26",)):
            row = {}
            for prec in ("fp64", "fp32"):
                if name == primary and e == emf and prec == "fp64":
                    row[prec] = out["value"]
                    continue
                r = run_gpu(cfg, state, prec, e, K, W)
                row[prec] = cfg["n"] ** 3 * K / r["elapsed"] / 1e6
                log(f"sweep {name} {e} {prec}: {row[prec]:.1f} Mcell-updates/s")
            row["fp32_speedup"] = row["fp32"] / row["fp64"]
            sweep[f"{name}/{e}"] = row
        if name == "turb128":
            out["level_form"] = run_level_form(cfg, emf, state, K, W)
            out["level_form"]["vs_single_box"] = (out["level_form"]["value"] /
                                                  sweep["turb128/q26"]["fp64"])
        del state
    sweep["unit"] = "Mcell-updates/s"
    sweep["steps"] = K
    return sweep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="turb512", choices=sorted(CONFIGS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "fp32_r64"])
    ap.add_argument("--emf", default="q26", choices=["q26", "b25a", "fs18"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=50)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    cfg = CONFIGS[args.config]
    K, W = args.steps, args.warmup
    n3 = cfg["n"] ** 3
    state = make_state(cfg)
    res = run_gpu(cfg, state, args.precision, args.emf, K, W, timer_pairs=64 * K,
                  copy_calibration=args.copy_calibration)
    value = n3 * K / res["elapsed"] / 1e6
    log(f"{args.precision}: {value:.1f} Mcell-updates/s, face kernel "
        f"{res['kernel_ms']:.4f} ms avg over {res['nlaunch']} launches")

    flops_tab = json.load(open(FLOPS_FILE))["entries"]
    fkey = f"{cfg['recon']}/{args.emf}/eta{'>0' if cfg['eta'] > 0 else '=0'}"
    face_flops = flops_tab[fkey]["face_flops"]
    cell_update_flops = flops_tab[fkey]["cell_update_flops"]
    achieved = face_flops * 3 * n3 / (res["kernel_ms"] * 1e-3) / 1e12
    traffic = read_traffic(args.config, args.precision, args.emf)
    out = {
        "metric": "Mcell-updates/s on 1 MI355X",
        "value": value,
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": res["elapsed"] / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "cells": n3, "recon": cfg["recon"],
                   "riemann": "hlld", "emf": args.emf, "averaging": "ld04", "fofc": True,
                   "cfl": 0.3, "eta": cfg["eta"], "precision": args.precision},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "kernel": "face (reconstruction + Riemann, all three directions, one stage)",
                     "kernel_ms": res["kernel_ms"], "flops_per_face": face_flops,
                     "faces_per_launch": 3 * n3},
        "step_alu_frac": value * 1e6 * cell_update_flops / (PEAK_FP64_TFLOPS * 1e12),
        "hbm_frac_algorithmic": value * 1e6 * ALG_BYTES_PER_CELL_UPDATE / (PEAK_HBM_GBS * 1e9),
        "step_hbm_measured": None,
        "fofc_flagged_cells": res["flagged"],
        "hll_fallbacks": res["hll"],
        "paper_context": ">50 M cell-updates/s per GPU (one MI250X GCD, PPM-EP + HLLD + Q26, "
                         "512^3 on 4 GCDs); context, not the target",
    }
    step_bytes = read_traffic(args.config, args.precision, args.emf, "bytes_per_step")
    if step_bytes:
        gbs = step_bytes / (res["elapsed"] / K) / 1e9
        out["step_hbm_measured"] = {"bytes_per_step": step_bytes, "achieved_GBs": gbs,
                                    "peak_GBs": PEAK_HBM_GBS, "frac": gbs / PEAK_HBM_GBS,
                                    "source": "rocprofv3 FETCH_SIZE + WRITE_SIZE of every "
                                              "kernel of a step, profiles/traffic_face_kernel.txt"}
    if args.precision == "fp64" and not args.no_fp32:
        r32 = run_gpu(cfg, state, "fp32", args.emf, K, W)
        v32 = n3 * K / r32["elapsed"] / 1e6
        out["fp32_form"] = {"value": v32, "unit": "Mcell-updates/s", "speedup": v32 / value}
        r3r = run_gpu(cfg, state, "fp32_r64", args.emf, K, W)
        v3r = n3 * K / r3r["elapsed"] / 1e6
        out["fp32_r64_form"] = {"value": v3r, "unit": "Mcell-updates/s", "speedup": v3r / value,
                                "riemann": "fp64"}
        log(f"fp32: {v32:.1f}, fp32 with FP64 Riemann: {v3r:.1f} Mcell-updates/s")
    if args.precision == "fp64" and not args.no_sweep:
        out["sweep"] = run_sweep(args.config, state, args.emf, K, W, out)
    del state
    if not args.no_batched:
        bf = run_batched_form(args.batched_steps, W)
        bf["speedup_fp32_vs_fp64_single_box_step"] = bf["fp32"]["value"] / value
        bf["speedup_vs_per_box_loop"] = bf["fp32"]["value"] / bf["per_box_loop_fp32"]["value"]
        out["batched_form"] = bf
    if not args.no_adjoint:
        out["adjoint_form"] = run_adjoint_form()
    if rank == 0 and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.emf)
        out["cpu_baseline_one_core"] = cpu_baseline_one_core(cfg, args.emf)
        log(f"oracle: {out['cpu_baseline']['value']:.3f} Mcell-updates/s on "
            f"{out['cpu_baseline']['cores']} threads ({out['cpu_baseline']['cpu_model']}), "
            f"{out['cpu_baseline_one_core']['value']:.3f} on one")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
