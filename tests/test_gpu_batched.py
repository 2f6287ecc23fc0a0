"""The batched form (ctmhd_step_batched): many periodic boxes of uneven sizes
in one persistent launch per step.  Each box is checked against the oracle
run on that box alone (same dt sequence), and against the single-box GPU
path; the launch sequence is replayed from a captured HIP graph."""
import math

import numpy as np
import pytest

import oracle
from helpers import compare_fields, divb_rel, field_errors, rel_l1

FIELDS = ["rho", "m0", "m1", "m2", "e", "b0", "b1", "b2"]
from paper_2609_10816_amd import ctmhd, inputs

pytestmark = pytest.mark.gpu


def _small_boxes(seed=5, nbox=7):
    states = inputs.amr_like_boxes(nbox=nbox, seed=seed, sizes=(4, 8, 12, 16))
    # one degenerate box (1D in 3D): a cold flow diverging at 10 times the
    # sound speed, whose first stage leaves cells with negative pressure that
    # the first-order flux correction must fix
    shape = (1, 1, 16)
    x = (np.arange(16) + 0.5) / 16
    rho = np.ones(shape)
    u = np.zeros((3,) + shape)
    u[0] = (10.0 * np.sin(2.0 * np.pi * x)).reshape(shape)
    p = np.full(shape, 1e-3)
    bf = np.zeros((3,) + shape)
    bf[0] = 1.0
    bf[1] = 0.5
    states.append((inputs.from_primitives(rho, u, p, bf), bf, (1 / 16, 1.0, 1.0)))
    return states


def _params(**kw):
    ok = {k: v for k, v in kw.items() if k not in ("precision", "tile")}
    return ctmhd.make_params(**kw), oracle.make_params(**ok)


def _cmp_box(cg, bg, co, bo, tol, label):
    """The float64 parity bar of the single-box tests, plus a pointwise bound
    (max difference over the mean magnitude, 100 times looser)."""
    _, worst = compare_fields(cg, bg, co, bo, tol, label)
    point = 0.0
    for m in range(5):
        point = max(point, np.abs(cg[m] - co[m]).max() / max(np.abs(co[m]).mean(),
                                                             np.abs(co[0]).mean()))
    for a in range(3):
        point = max(point, np.abs(bg[a] - bo[a]).max() / max(np.abs(bo).mean(), 1e-300))
    assert point <= 100 * tol, (label, point)
    return worst


@pytest.mark.parametrize("emf,precision", [("q26", "fp64"), ("b25a", "fp64"), ("q26", "fp32")])
def test_batched_equals_single_box_path(emf, precision):
    states = _small_boxes()
    P, _ = _params(recon="ppm", emf=emf, eta=1e-3, precision=precision)
    outs, dts, dg = ctmhd.run_batched(P, states, nsteps=3)
    for b, (c, bf, dx) in enumerate(states):
        cg, bg, _, _ = ctmhd.run(P, c, bf, dx, 3, dt_fixed=dts[:, 0])
        diff = max(np.abs(outs[b][0] - cg).max(), np.abs(outs[b][1] - bg).max())
        assert np.array_equal(outs[b][0], cg) and np.array_equal(outs[b][1], bg), (b, diff)


@pytest.mark.skip(reason="the persistent-queue schedule is disabled in the library: a launch of "
                         "it did not finish (cause not found); must not run on a GPU until the "
                         "cause is shown")
@pytest.mark.parametrize("fofc", [True, False])
def test_batched_schedules_agree(fofc):
    """The persistent-queue schedule and the per-phase schedule compute the
    same step bit for bit (global dt, 3 steps, FOFC on and off)."""
    states = _small_boxes(seed=14)
    Pq, _ = _params(recon="ppm", emf="b25a", eta=1e-3, fofc=fofc,
                    tile=ctmhd.make_tile(strips=2, persistent=True))
    Pp, _ = _params(recon="ppm", emf="b25a", eta=1e-3, fofc=fofc,
                    tile=ctmhd.make_tile(strips=2))
    a, da, ga = ctmhd.run_batched(Pq, states, nsteps=3)
    b, db, gb = ctmhd.run_batched(Pp, states, nsteps=3)
    assert np.array_equal(da, db) and np.array_equal(ga[:, :3], gb[:, :3])
    assert int(ga[:, 3].max()) == 0 and int(gb[:, 3].max()) == 0
    for x, y in zip(a, b):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])


def test_batched_deterministic():
    """Two runs of the same batched call agree bit for bit (the schedule of
    the work queue differs between runs; the arithmetic must not)."""
    states = _small_boxes(seed=12)
    P, _ = _params(recon="ppm", emf="q26", eta=1e-3)
    a, da, ga = ctmhd.run_batched(P, states, nsteps=3)
    b, db, gb = ctmhd.run_batched(P, states, nsteps=3)
    assert np.array_equal(da, db) and np.array_equal(ga, gb)
    for x, y in zip(a, b):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])


@pytest.mark.parametrize("emf", ["q26", "b25a", "fs18"])
def test_batched_vs_oracle_global_dt(emf):
    states = _small_boxes()
    P, Q = _params(recon="ppm", emf=emf, eta=1e-3)
    outs, dts, dg = ctmhd.run_batched(P, states, nsteps=2)
    # the global dt is the CFL dt of the box with the largest signal speed
    dt0 = min(oracle.cfl_dt(Q, c, bf, dx) for c, bf, dx in states)
    assert dts[0, 0] == pytest.approx(dt0, rel=1e-13)
    nflag = 0
    worst = 0.0
    for b, (c, bf, dx) in enumerate(states):
        co, bo, _, do = oracle.step(Q, c, bf, dx, nsteps=2, dt_fixed=dts[:, 0])
        nflag += do[0] + do[1]
        worst = max(worst, _cmp_box(outs[b][0], outs[b][1], co, bo, 1e-12, f"box {b}"))
        assert divb_rel(outs[b][1], dx) < 1e-13
    assert int(dg[:, :2].sum()) == nflag
    assert nflag > 0  # the diverging-flow box exercises the flux correction
    print(f"[batched] {len(states)} boxes {emf}: worst field relative L1 {worst:.2e}, "
          f"flagged {nflag}", flush=True)


def test_batched_per_box_dt():
    states = _small_boxes(seed=6)
    P, Q = _params(recon="plm", emf="q26")
    outs, dts, dg = ctmhd.run_batched(P, states, nsteps=2, dt_mode=ctmhd.DT_PER_BOX)
    for b, (c, bf, dx) in enumerate(states):
        co, bo, dto, _ = oracle.step(Q, c, bf, dx, nsteps=2)
        np.testing.assert_allclose(dts[:, b], dto, rtol=1e-13)
        _cmp_box(outs[b][0], outs[b][1], co, bo, 1e-12, f"box {b}")


def _fp32_boxes(precision, states, nsteps):
    """The FP32 forms on AMR-like boxes, per box against the FP64 oracle run
    with the batch's dt sequence.  Per box also: its flux-correction flag
    count on the GPU (the box stepped alone with that dt sequence, which must
    give the batch's result bitwise), the oracle's flag count, and the
    oracle's own response to the dt sequence scaled by 1 + 1e-7 (how strongly
    the box amplifies a perturbation of that size)."""
    P, Q = _params(recon="ppm", emf="q26", precision=precision)
    outs, dts, _ = ctmhd.run_batched(P, states, nsteps=nsteps)
    rows = []
    for b, (c, bf, dx) in enumerate(states):
        alone, _, dga = ctmhd.run_batched(P, [(c, bf, dx)], nsteps=nsteps, dt_fixed=dts[:, 0])
        for m in range(5):
            assert np.array_equal(alone[0][0][m], outs[b][0][m]), (b, m)
        co, bo, _, do = oracle.step(Q, c, bf, dx, nsteps=nsteps, dt_fixed=dts[:, 0])
        cp, bp, _, _ = oracle.step(Q, c, bf, dx, nsteps=nsteps, dt_fixed=dts[:, 0] * (1 + 1e-7))
        errs = field_errors(outs[b][0], outs[b][1], co, bo)
        cond = max(v[1] for v in field_errors(cp, bp, co, bo))
        gf, of = int(dga[:, :2].sum()), int(do[0] + do[1])
        print(f"[batched] {precision} {nsteps} steps box {b} {c.shape[1:]} flags gpu {gf} oracle "
              f"{of}, oracle response to 1e-7 dt {cond:.1e}: " +
              " ".join(f"{n}={v[0]:.1e}/{v[1]:.1e}" for n, v in zip(FIELDS, errs)), flush=True)
        for m in range(5):
            s0, s1 = c[m].sum(), outs[b][0][m].sum()
            assert abs(s1 - s0) <= 1e-13 * (np.abs(c[m]).sum() + np.abs(outs[b][0][m]).sum())
        assert divb_rel(outs[b][1], dx) < 1e-13
        rows.append(dict(errs=errs, gpu_flags=gf, oracle_flags=of, cond=cond))
    return rows


def _fp32_bar(rows, bar, plain=False):
    """Holds each box to `bar` (plain or normalised relative L1, worst field)
    unless the box is ill-conditioned at the FP32 scale (the oracle moves by
    more than 1e-5 under the 1e-7 dt change: a stage update there sits at the
    edge of the flux-correction test, and which cells the correction flags
    depends on rounding) or its flag count differs from the oracle's (a flag
    decided by FP32 rounding; its first-order replacement moves the box off the
    oracle's trajectory by O(the flux difference), bounded here by 1e-3).  At
    most one box of a set may be exempt."""
    k = 0 if plain else 1
    exempt = 0
    for b, r in enumerate(rows):
        e = max(v[k] for v in r["errs"])
        if r["cond"] > 1e-5:
            exempt += 1
        elif r["gpu_flags"] != r["oracle_flags"]:
            exempt += 1
            assert max(v[1] for v in r["errs"]) <= 1e-3, (b, r)
        else:
            assert e <= bar, (b, e)
    assert exempt <= 1, rows


def test_batched_fp32_vs_oracle():
    """The FP32 form in a batch, 10 steps: smooth AMR-like boxes, one 4^3 box
    and a 1-cell-wide diverging flow that the flux correction must fix, each
    within 1e-5 of the FP64 oracle per field (normalisation of the float64
    parity bar: fields that carry only a perturbation on the scale of the
    fluxes that update them); conservation and div b at FP64 round-off."""
    rows = _fp32_boxes("fp32", _small_boxes(seed=7), 10)
    _fp32_bar(rows, 1e-5)


def test_batched_fp32_100_steps_vs_oracle():
    """The FP32 form in a batch over 100 steps of AMR-like boxes of 8 and 16
    cells per axis (one or two wavelengths of supersonic, low-to-high beta
    flow): the FP32 Riemann solve's error grows to about 1e-5 in 100 steps
    (the 128^3 and 48^3 turbulent boxes stay near 1e-6), bound 1e-4
    normalised."""
    rows = _fp32_boxes("fp32", inputs.amr_like_boxes(nbox=6, seed=11, sizes=(8, 16)), 100)
    _fp32_bar(rows, 1e-4)


def test_batched_fp32_r64_100_steps_vs_oracle():
    """The FP32 form with its Riemann solve in FP64 (CTMHD_FP32_R64) on the
    same boxes over 100 steps: the remaining error is the FP32
    reconstruction and edge arithmetic, and every well-conditioned box is
    held to a plain relative L1 error of 1e-5 per field."""
    rows = _fp32_boxes("fp32_r64", inputs.amr_like_boxes(nbox=6, seed=11, sizes=(8, 16)), 100)
    _fp32_bar(rows, 1e-5, plain=True)


def test_batched_tile_knob_same_result():
    """The strips knob only regroups work items: bitwise the same result.  The
    chunk knob moves where the y/z face marches start, so a face's
    reconstruction may be evaluated with another grouping of fused
    multiply-adds: the same result to round-off, in the single-box path too."""
    states = _small_boxes(seed=8)
    P0, Q = _params(recon="ppm")
    a, da, _ = ctmhd.run_batched(P0, states, nsteps=2)
    P1, _ = _params(recon="ppm", tile=ctmhd.make_tile(strips=3))
    b, db, _ = ctmhd.run_batched(P1, states, nsteps=2)
    assert np.array_equal(da, db)
    for x, y in zip(a, b):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
    P2, _ = _params(recon="ppm", tile=ctmhd.make_tile(chunk=8, strips=3))
    c2, dc, _ = ctmhd.run_batched(P2, states, nsteps=2)
    assert np.array_equal(da, dc)
    for k, (x, y) in enumerate(zip(a, c2)):
        _cmp_box(y[0], y[1], x[0], x[1], 1e-14, f"box {k}")
        c, bf, dx = states[k]
        single = ctmhd.run(P2, c, bf, dx, 2, dt_fixed=da[:, 0])
        assert np.array_equal(single[0], y[0]) and np.array_equal(single[1], y[1])


def test_batched_hipgraph_replay():
    """Capture a 2-step batched call in a HIP graph; replay it three times from
    the same initial state with eager work in between; every replay equals
    the eager result."""
    import torch
    states = _small_boxes(seed=9)
    P, _ = _params(recon="ppm", emf="q26")
    st = ctmhd.BatchedState.from_numpy(states, ctmhd.required_ghosts(P))
    S = ctmhd.BatchedStepper(P, st)
    init_c = [t.clone() for t in st.cons]
    init_b = [t.clone() for t in st.bface]
    dts = torch.zeros(2, dtype=torch.float64, device="cuda")
    diag = torch.zeros(8, dtype=torch.int64, device="cuda")

    def reset():
        for t, s in zip(st.cons + st.bface, init_c + init_b):
            t.copy_(s)

    reset()
    S.step(2, dt_out=dts, diag=diag)
    torch.cuda.synchronize()
    ref_c = [t.clone() for t in st.cons]
    ref_b = [t.clone() for t in st.bface]
    ref_dt = dts.clone()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        reset()
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            S.step(2, dt_out=dts, diag=diag)
    torch.cuda.synchronize()
    for rep in range(3):
        reset()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for t, r in zip(st.cons + st.bface, ref_c + ref_b):
            assert torch.equal(t, r), rep
        assert torch.equal(dts, ref_dt), rep
        del junk


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_amr_like_2000_boxes_sampled(precision):
    """The 2000-box AMR-like workload (edges from {8,16,32,64}, 4 ghost
    layers, PPM + Q26), 2 steps; 24 sampled boxes of every size class against
    the oracle on each box alone with the same dt; invariants on every
    sampled box."""
    import torch
    states = inputs.amr_like_boxes(2000, seed=4)
    P, Q = _params(recon="ppm", emf="q26", precision=precision)
    outs, dts, dg = ctmhd.run_batched(P, states, nsteps=2)
    rng = np.random.default_rng(11)
    by_size = {}
    for b, (c, _, _) in enumerate(states):
        by_size.setdefault(max(c.shape[1:]), []).append(b)
    sample = []
    for sz in sorted(by_size):
        sample += list(rng.choice(by_size[sz], size=min(6, len(by_size[sz])), replace=False))
    tol = 1e-12 if precision == "fp64" else 1e-5
    worst = 0.0
    for b in sample:
        c, bf, dx = states[b]
        co, bo, _, _ = oracle.step(Q, c, bf, dx, nsteps=2, dt_fixed=dts[:, 0])
        if precision == "fp64":
            worst = max(worst, _cmp_box(outs[b][0], outs[b][1], co, bo, tol, f"box {b}"))
        else:
            e = max(v[1] for v in field_errors(outs[b][0], outs[b][1], co, bo))
            worst = max(worst, e)
            assert e <= tol, (b, e)
        for m in range(5):
            s0, s1 = c[m].sum(), outs[b][0][m].sum()
            assert abs(s1 - s0) <= 1e-13 * (np.abs(c[m]).sum() + np.abs(outs[b][0][m]).sum())
        assert divb_rel(outs[b][1], dx) < 1e-13
    print(f"[batched] 2000 boxes {precision}: {len(sample)} sampled boxes, worst {worst:.2e}, "
          f"dt {dts[0, 0]:.4e}, flagged {int(dg[:, :2].sum())}, timeout flag {int(dg[:, 3].max())}",
          flush=True)
    assert int(dg[:, 3].max()) == 0
    torch.cuda.empty_cache()


def test_batched_refuses_plan_of_other_boxes():
    """A plan built for other boxes is refused on the device: diag[3] bit 4,
    the state is left untouched, and the kernels exit normally."""
    import torch
    states = _small_boxes(seed=10, nbox=4)
    P, _ = _params(recon="plm")
    st = ctmhd.BatchedState.from_numpy(states, ctmhd.required_ghosts(P))
    S = ctmhd.BatchedStepper(P, st)
    other = [ctmhd.make_box(tuple(b.n), b.ng, tuple(b.dx), b.offset) for b in st.boxes]
    last = other[-1]
    other[-1] = ctmhd.make_box((last.n[0], last.n[1], last.n[2]), last.ng,
                               (last.dx[0] * 2, last.dx[1], last.dx[2]), last.offset)
    S.plan = torch.from_numpy(ctmhd.batch_plan(P, other)).to("cuda")
    before = [t.clone() for t in st.cons + st.bface]
    diag = torch.zeros(4, dtype=torch.int64, device="cuda")
    S.step(1, diag=diag)
    torch.cuda.synchronize()
    assert int(diag[3]) & 4
    for t, r in zip(st.cons + st.bface, before):
        assert torch.equal(t, r)


def test_persistent_schedule_is_refused():
    """Schedule 1 is switched off: the call returns CTMHD_EUNSUPPORTED before
    any launch."""
    states = _small_boxes(seed=15, nbox=2)
    P, _ = _params(recon="plm", tile=ctmhd.make_tile(persistent=True))
    with pytest.raises(ctmhd.CtmhdError, match="persistent"):
        ctmhd.run_batched(P, states, nsteps=1)


def test_autotuner_picks_valid_tile_and_keeps_state(tmp_path):
    import torch
    from paper_2609_10816_amd import autotune
    states = _small_boxes(seed=13)
    P, _ = _params(recon="ppm", emf="q26")
    st = ctmhd.BatchedState.from_numpy(states, ctmhd.required_ghosts(P))
    before = [t.clone() for t in st.cons + st.bface]
    cache = str(tmp_path / "tiles.json")
    tile, ms = autotune.tune_batched(P, st, steps=1, reps=1, chunks=(8, 32), strips=(1, 2),
                                     cache_file=cache)
    valid = [ctmhd.make_tile(chunk=c, strips=s) for c in (8, 32) for s in (1, 2)]
    assert tile in valid and all(int(k) in valid for k in ms)
    assert len(ms) == 3 and all(v > 0 for v in ms.values())  # 2 chunks, then 1 more strips
    for t, r in zip(st.cons + st.bface, before):
        assert torch.equal(t, r)
    # served from the cache file in a fresh process-level cache
    autotune._cache.clear()
    tile2, _ = autotune.tune_batched(P, st, cache_file=cache)
    assert tile2 == tile
    # the tuned step equals the default step to round-off
    P.tile = tile
    outs, dts, _ = ctmhd.run_batched(P, states, nsteps=1)
    P0, Q = _params(recon="ppm", emf="q26")
    ref, dts0, _ = ctmhd.run_batched(P0, states, nsteps=1)
    assert np.array_equal(dts, dts0)
    for k, (x, y) in enumerate(zip(outs, ref)):
        _cmp_box(x[0], x[1], y[0], y[1], 1e-14, f"box {k}")
