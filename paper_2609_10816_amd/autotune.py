"""Tile-shape autotuner for the CT-MHD step.

The library exposes two tuning knobs through ``ctmhd_params.tile``:

* ``chunk``  - minimum number of faces one workgroup marches along the y and
  z normals before a new march starts (shorter chunks give more workgroups
  and more warm-up reconstructions; longer chunks give fewer, longer
  workgroups);
* ``strips`` - 256-cell strips per work item of the batched call (more
  strips give fewer, longer work items);
* ``schedule`` - the batched call launches once per phase over all boxes
  (the persistent-queue schedule is switched off in the library and is not
  searched by default).

All only change how work is distributed: any choice computes the same step
(to round-off for ``chunk``, bitwise for ``strips`` and ``schedule``).  The
batched search is coordinate-wise: per schedule, the chunk at the default
strips, then the strips at the best chunk.  The tuner times whole
steps on a copy of the caller's state, on the stream the library launches on,
and returns the fastest knob value; results are cached per
(scheme, precision, box-shape signature) for the life of the process and,
optionally, in a JSON file.
"""
from __future__ import annotations

import hashlib
import json
import os

from . import ctmhd

CHUNKS = (8, 16, 32, 64)
STRIPS = (1, 2, 4, 8)

_cache: dict[str, dict] = {}


def _signature(params: ctmhd.Params, shapes) -> str:
    h = hashlib.sha1()
    h.update(repr((params.recon, params.riemann, params.emf_compute, params.fofc,
                   params.precision, params.eta > 0)).encode())
    for n in shapes:
        h.update(repr(tuple(int(v) for v in n)).encode())
    return h.hexdigest()[:20]


def _time_calls(prepare, fn, reps):
    """Best time in ms of fn() over reps runs, each after prepare() (untimed)."""
    import torch
    prepare()
    fn()  # warm-up (first-use costs, code loading)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        prepare()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def _load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _store(path, key, entry):
    if not path:
        return
    data = _load(path)
    data[key] = entry
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_batched(params: ctmhd.Params, state: "ctmhd.BatchedState", steps=2, reps=2,
                 chunks=CHUNKS, strips=STRIPS, schedules=(False,), cache_file=None,
                 verbose=False):
    """Pick ``tile`` for ctmhd_step_batched on these boxes.  The caller's
    state is left as it was.  Returns (tile, {tile: ms per step})."""
    import torch
    key = "batched/" + _signature(params, state.shapes)
    if key in _cache:
        return _cache[key]["tile"], _cache[key]["ms"]
    disk = _load(cache_file)
    if key in disk:
        _cache[key] = disk[key]
        return disk[key]["tile"], disk[key]["ms"]
    saved = [t.clone() for t in state.cons + state.bface]
    dev = state.cons[0].device
    dt = torch.zeros(steps * len(state.shapes), dtype=torch.float64, device=dev)
    timings = {}

    def restore():
        for t, v in zip(state.cons + state.bface, saved):
            t.copy_(v)

    def measure(c, s_, persistent):
        tile = ctmhd.make_tile(chunk=c, strips=s_, persistent=persistent)
        if tile not in timings:
            P = ctmhd.Params.from_buffer_copy(params)
            P.tile = tile
            S = ctmhd.BatchedStepper(P, state)
            timings[tile] = _time_calls(restore, lambda: S.step(steps, dt_out=dt), reps) / steps
            if verbose:
                print(f"[autotune] {'persistent' if persistent else 'per-phase'} chunk {c:3d} "
                      f"strips {s_}: {timings[tile]:.3f} ms/step", flush=True)
            del S
        return timings[tile]

    s0 = strips[0]
    for persistent in schedules:
        c_best = min(chunks, key=lambda c: measure(c, s0, persistent))
        for s_ in strips:
            measure(c_best, s_, persistent)
    restore()
    best = min(timings, key=timings.get)
    entry = {"tile": best, "ms": {str(k): v for k, v in timings.items()}}
    _cache[key] = entry
    _store(cache_file, key, entry)
    return best, entry["ms"]


def tune_single(params: ctmhd.Params, state: "ctmhd.BoxState", steps=2, reps=2, chunks=CHUNKS,
                cache_file=None, verbose=False):
    """Pick ``tile`` (the chunk knob) for ctmhd_step on this machine."""
    import torch
    key = "single/" + _signature(params, [state.n])
    if key in _cache:
        return _cache[key]["tile"], _cache[key]["ms"]
    disk = _load(cache_file)
    if key in disk:
        _cache[key] = disk[key]
        return disk[key]["tile"], disk[key]["ms"]
    saved = [t.clone() for t in state.cons + state.bface]
    dev = state.cons[0].device
    dt = torch.zeros(steps, dtype=torch.float64, device=dev)
    timings = {}
    for c in chunks:
        tile = ctmhd.make_tile(chunk=c)
        P = ctmhd.Params.from_buffer_copy(params)
        P.tile = tile
        S = ctmhd.Stepper(P, state)

        def restore():
            for t, v in zip(state.cons + state.bface, saved):
                t.copy_(v)

        ms = _time_calls(restore, lambda: S.step(steps, None, dt), reps) / steps
        timings[tile] = ms
        if verbose:
            print(f"[autotune] chunk {c:3d}: {ms:.3f} ms/step", flush=True)
        del S
    for t, v in zip(state.cons + state.bface, saved):
        t.copy_(v)
    best = min(timings, key=timings.get)
    entry = {"tile": best, "ms": {str(k): v for k, v in timings.items()}}
    _cache[key] = entry
    _store(cache_file, key, entry)
    return best, entry["ms"]
