"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs, element by element.

Tolerances (float64 path), after every step: the relative error of eq.
error:relative over all 8 fields <= 1e-12, and for each field at its own
scale both the relative L1 difference and the largest element difference
over the largest element <= 1e-12 (helpers.compare_fields).  The momentum of
a linear eigenmode carries only the perturbation (amplitude delta) on an O(1)
background whose fluxes set its round-off, so its two per-field bars are
1e-13 / delta (1e-7 for delta = 1e-6, 1e-10 for delta = 1e-3); observed about
2e-9 and 8e-12.  Discrete div b <= 1e-13 relative and conservation to
round-off on the GPU result itself.  The HLL fallback count of the GPU is the
oracle's times the number of solved copies of each face (the ghost shell).
"""
import math

import numpy as np
import pytest

import oracle
from helpers import compare_fields, divb_rel
from paper_2609_10816_amd import ctmhd, inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12


MOMENTA = (1, 2, 3)


def _compare(cg, bg, co, bo, tol=TOL, label="", pert=None):
    return compare_fields(cg, bg, co, bo, tol, label, pert)


def _conserved(c0, c1, tol=1e-13):
    for m in range(5):
        scale = np.abs(c0[m]).sum() + np.abs(c1[m]).sum() + 1e-300
        assert abs(c1[m].sum() - c0[m].sum()) <= tol * scale, m


def _params(**kw):
    ok = {k: v for k, v in kw.items() if k != "precision"}
    return ctmhd.make_params(**kw), oracle.make_params(**ok)


def _stepwise(P, Q, cons, bf, dx, nsteps, label, dt_fixed=None, tol=TOL, force=None,
              pert=None):
    """Advance both sides one step at a time from their own states, compare
    after every step."""
    cg, bg = cons, bf
    co, bo = cons, bf
    for s in range(nsteps):
        dtf = None if dt_fixed is None else [dt_fixed]
        cg1, bg1, dtg, dg = ctmhd.run(P, cg, bg, dx, 1, dt_fixed=dtf)
        co1, bo1, dto, do = oracle.step(Q, co, bo, dx, nsteps=1, dt_fixed=dtf,
                                        force=None if force is None else force)
        assert dtg[0] == pytest.approx(dto[0], rel=1e-13), (dtg, dto)
        assert dg[0, 0] == do[0] and dg[0, 1] == do[1], (dg, do)
        _compare(cg1, bg1, co1, bo1, tol, f"{label} step {s}", pert)
        assert divb_rel(bg1, dx) < 1e-13
        _conserved(cg, cg1)
        cg, bg, co, bo = cg1, bg1, co1, bo1
    return cg, bg


@pytest.mark.parametrize("emf", ["q26", "b25a", "fs18"])
def test_linear_wave_32(emf):
    """The linear fast-wave workload: 32^3, PLM + HLLD, CFL 0.3, 10 steps."""
    cons, bf, info = inputs.linear_fast_wave_32(32)
    P, Q = _params(recon="plm", emf=emf)
    _stepwise(P, Q, cons, bf, info["dx"], 10, f"fastwave32 {emf}",
              pert={m: 1e-6 for m in MOMENTA})


@pytest.mark.parametrize("recon", ["pc", "plm", "plm_minmod", "ppm"])
@pytest.mark.parametrize("emf", ["q26", "b25a", "fs18"])
def test_turbulent_small(recon, emf):
    """Mach-5 turbulent box at 24^3 with eta > 0: every reconstruction and
    EMF scheme, two steps."""
    cons, bf, info = inputs.turbulent_box((24, 24, 24), mach=5.0, b0=(0.1, 0.0, 0.0),
                                          db_rms=0.05, seed_v=31, seed_a=32)
    P, Q = _params(recon=recon, emf=emf, eta=1e-3)
    _stepwise(P, Q, cons, bf, info["dx"], 2, f"turb24 {recon} {emf}")


@pytest.mark.parametrize("shape", [(13, 7, 5), (17, 1, 1), (9, 11, 1), (1, 6, 10), (33, 20, 18)])
def test_ragged_shapes(shape):
    """Non-cubic and degenerate (1-cell) axes, odd sizes that leave ragged
    tails in every launch."""
    cons, bf, info = inputs.turbulent_box(shape, mach=2.0, b0=(0.5, 0.3, -0.2), db_rms=0.2,
                                          seed_v=33, seed_a=34) if min(shape) > 4 else \
        inputs.fast_wave(shape, kvec=tuple(1 if s > 1 else 0 for s in shape), delta=1e-3)
    dx = [1.0 / s for s in shape]
    pert = None if min(shape) > 4 else {m: 1e-3 for m in MOMENTA}
    for recon in ["plm", "ppm"]:
        P, Q = _params(recon=recon, emf="q26", eta=5e-4)
        _stepwise(P, Q, cons, bf, dx, 2, f"ragged {shape} {recon}", pert=pert)


def test_llf_riemann():
    cons, bf, info = inputs.turbulent_box((16, 12, 10), mach=3.0, seed_v=35, seed_a=36)
    dx = [1 / 16, 1 / 12, 1 / 10]
    P, Q = _params(recon="plm", riemann="llf", emf="q26")
    _stepwise(P, Q, cons, bf, dx, 2, "llf")


def test_fofc_forced_masks():
    """Random forced flags (5% per stage): first-order replacement on the
    GPU follows the oracle."""
    import torch
    cons, bf, info = inputs.turbulent_box((16, 14, 12), mach=3.0, seed_v=37, seed_a=38)
    dx = [1 / 16, 1 / 14, 1 / 12]
    rng = np.random.default_rng(39)
    force = (rng.random((2, 12, 14, 16)) < 0.05).astype(np.uint8)
    ft = torch.from_numpy(force.reshape(-1).copy()).cuda()
    for emf in ["q26", "b25a", "fs18"]:
        P, Q = _params(recon="ppm", emf=emf, eta=1e-3)
        P.force_flags = ft.data_ptr()
        _stepwise(P, Q, cons, bf, dx, 2, f"fofc-forced {emf}", force=force)


def test_fofc_forced_masks_beyond_one_grid():
    """A box of more than 2048 x 256 cells with random forced flags: the
    first-order and fix-up launches stride over it with a capped grid (more
    than one tile per workgroup) and still follow the oracle."""
    import torch
    shape = (96, 80, 72)
    assert shape[0] * shape[1] * shape[2] > 2048 * 256
    cons, bf, info = inputs.turbulent_box(shape, mach=3.0, seed_v=44, seed_a=45)
    dx = [1 / 96, 1 / 80, 1 / 72]
    rng = np.random.default_rng(46)
    force = (rng.random((2, 72, 80, 96)) < 0.02).astype(np.uint8)
    ft = torch.from_numpy(force.reshape(-1).copy()).cuda()
    P, Q = _params(recon="ppm", emf="q26", eta=1e-3)
    P.force_flags = ft.data_ptr()
    _stepwise(P, Q, cons, bf, dx, 1, "fofc-forced large", force=force)


def test_fofc_all_cells():
    import torch
    cons, bf, info = inputs.turbulent_box((12, 12, 12), mach=3.0, seed_v=40, seed_a=41)
    force = np.ones((2, 12, 12, 12), np.uint8)
    ft = torch.from_numpy(force.reshape(-1).copy()).cuda()
    P, Q = _params(recon="ppm", emf="q26")
    P.force_flags = ft.data_ptr()
    _stepwise(P, Q, cons, bf, info["dx"], 1, "fofc-all", force=force)


def test_fofc_natural_trigger():
    """A strong blast (pressure jump 1e4, low-beta field) produces negative
    pressures in the high-order update: the flagged cells and the corrected
    state agree with the oracle."""
    n = 24
    shape = (n, n, n)
    x = [(np.arange(n) + 0.5) / n - 0.5] * 3
    Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    rho = np.ones(shape)
    p = np.where(r < 0.1, 1e3, 0.1)
    u = np.zeros((3,) + shape)
    bf = np.zeros((3,) + shape)
    bf[0] = 10.0 / math.sqrt(2)
    bf[1] = 10.0 / math.sqrt(2)
    cons = inputs.from_primitives(rho, u, p, bf)
    dx = [1 / n] * 3
    P, Q = _params(recon="ppm", emf="q26", cfl=0.3)
    c, b = cons, bf
    flagged = 0
    for s in range(6):
        cg, bg, dtg, dg = ctmhd.run(P, c, b, dx, 1)
        co, bo, dto, do = oracle.step(Q, c, b, dx, nsteps=1)
        assert dg[0, 0] == do[0] and dg[0, 1] == do[1]
        flagged += do[0] + do[1]
        _compare(cg, bg, co, bo, TOL, f"blast step {s} flags {do[:2]}")
        # continue both from the oracle state so that round-off differences
        # do not move flags between steps
        c, b = co, bo
    print(f"[parity] blast total flagged cells {flagged}", flush=True)


def test_nonfinite_dt_stops():
    import torch
    cons, bf, info = inputs.turbulent_box((8, 8, 8), mach=1.0, seed_v=42, seed_a=43)
    cons = cons.copy()
    cons[4, 3, 3, 3] = np.nan
    P, _ = _params(recon="plm")
    cg, bg, dts, dg = ctmhd.run(P, cons, bf, info["dx"], 3)
    assert dg[:, 3].tolist() == [1, 1, 1]
    np.testing.assert_array_equal(cg[0], cons[0])
    np.testing.assert_array_equal(bg, bf)
    del torch


def _strong_rarefaction_box(n0=32, n1=4, U=2.0, p0=0.01):
    """Two cold streams separating at x = 0 (u_x = +U on [0, 1/2), -U on
    [1/2, 1)) with a weak field: at the x = 0 face the HLLD star total
    pressure p_T - rho c U (symmetric case) is negative, so both sides take
    the HLL fallback there in every stage (Sec. 2.2)."""
    shape = (1, n1, n0)
    x = (np.arange(n0) + 0.5) / n0
    y = (np.arange(n1) + 0.5) / n1
    Y, X = np.meshgrid(y, x, indexing="ij")
    rho = (1.0 + 0.1 * np.cos(2 * np.pi * Y)).reshape(shape)
    ux = np.where(X < 0.5, U, -U).reshape(shape)
    u = np.stack([ux, (0.1 * np.sin(2 * np.pi * X)).reshape(shape), np.zeros(shape)])
    p = np.full(shape, p0)
    bf = np.stack([np.full(shape, 0.05), np.full(shape, 0.1), np.full(shape, 0.02)])
    return inputs.from_primitives(rho, u, p, bf), bf, [1.0 / n0, 1.0 / n1, 1.0]


def _shell_rows(shape, recon, emf):
    """Rows of x faces (transverse positions) the face pass solves: across
    each transverse axis the ghost shell the edges read, n + 2 + 2r rows for
    Q26 (u* reconstructed to the edges) and n + 2 otherwise (edge speeds);
    along the normal the faces x = 0..n0 (face n0 is the periodic image of
    face 0, so the x = 0 face is solved twice per row)."""
    r = {"pc": 0, "plm": 1, "ppm": 2}[recon]
    w = r if emf == "q26" else 0
    return (shape[1] + 2 + 2 * w) * (shape[0] + 2 + 2 * w)


@pytest.mark.parametrize("recon", ["plm", "ppm"])
@pytest.mark.parametrize("emf", ["q26", "b25a", "fs18"])
def test_hll_fallback_parity(recon, emf):
    """Both sides fall back to HLL at the x = 0 face of every row in both
    stages and reach the same state; the GPU counts every solved copy of
    those faces."""
    cons, bf, dx = _strong_rarefaction_box()
    P, Q = _params(recon=recon, emf=emf, eta=1e-3)
    shape = cons.shape[1:]
    rows = shape[0] * shape[1]
    c, b = cons, bf
    for s in range(3):
        cg, bg, dtg, dg = ctmhd.run(P, c, b, dx, 1)
        co, bo, dto, do = oracle.step(Q, c, b, dx, nsteps=1)
        print(f"[parity] fallback {recon} {emf} step {s}: HLL fallbacks gpu {dg[0, 2]} "
              f"oracle {do[2]}", flush=True)
        # one fallback face (x = 0) per row and stage on both sides
        assert do[2] == 2 * rows
        assert dg[0, 2] == 2 * 2 * _shell_rows(shape, recon, emf)
        assert dg[0, 0] == do[0] and dg[0, 1] == do[1]
        assert dtg[0] == pytest.approx(dto[0], rel=1e-13)
        _compare(cg, bg, co, bo, TOL, f"fallback {recon} {emf} step {s}")
        assert divb_rel(bg, dx) < 1e-13
        _conserved(c, cg)
        c, b = cg, bg
