"""The adjoint form (ctmhd_step_adjoint): reverse-mode derivative of one step
with frozen dt and no flux correction.

1. Against the oracle's forward-mode (dual-number) derivative: for random
   tangents dS and cotangents g, <g, J dS> (oracle) = <J^T g, dS> (GPU), to
   FP64 round-off.  Non-cubic box, unequal dx, every supported scheme, on a
   state where every field varies (the derivative is taken on the branches
   the forward step takes; it is unique only away from ties).
2. Against central finite differences of the GPU forward step (16^3).
3. Unsupported configurations are refused before any launch.
"""
import numpy as np
import pytest

import oracle
from paper_2609_10816_amd import ctmhd, inputs

pytestmark = pytest.mark.gpu

CONFIGS = [
    ("pc", "llf", 0.0),
    ("plm", "llf", 0.0),
    ("plm", "hlld", 0.0),
    ("plm", "hlld", 1e-3),
    ("plm_minmod", "hlld", 1e-3),
    ("pc", "hlld", 1e-3),
]


def _state(n=(12, 10, 8), seed=3):
    """Non-cubic box, unequal cell widths, every field varying (amplitude 0.3,
    so limiters, min/max selections and the HLLD regions all vary).  A state
    with exactly uniform fields would put limiters at ties, where the one-sided
    derivative depends on round-off (the derivative is not unique there)."""
    cons, bf, info = inputs.smooth_modes_box(n, amp=0.3, beta=1.0, seed=seed, L=(1.0, 1.1, 0.9))
    return cons, bf, info["dx"]


def adjoint(P, cons, bf, dx, dt, gc, gb):
    import torch
    ng = ctmhd.required_ghosts(P)
    S = ctmhd.BoxState.from_numpy(cons, bf, ng, dx)
    G = ctmhd.BoxState.from_numpy(gc, gb, ng, dx)
    O = ctmhd.BoxState(S.n, ng, dx)
    nbytes = ctmhd.adjoint_workspace_bytes(P, S.box)
    assert nbytes > 0
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dtt = torch.tensor([dt], dtype=torch.float64, device="cuda")
    ctmhd.ctmhd_step_adjoint(P, S.box, S.cons, S.bface, dtt, G.cons, G.bface, O.cons, O.bface, ws)
    torch.cuda.synchronize()
    return O.to_numpy()


def _dot(a, b):
    return float(np.sum(a * b)), float(np.sum(np.abs(a * b)))


@pytest.mark.parametrize("recon,riemann,eta", CONFIGS)
def test_adjoint_dot_product_vs_oracle_dual(recon, riemann, eta):
    cons, bf, dx = _state()
    Q = oracle.make_params(recon=recon, riemann=riemann, eta=eta, fofc=False)
    P = ctmhd.make_params(recon=recon, riemann=riemann, eta=eta, fofc=False)
    dt = 0.5 * oracle.cfl_dt(Q, cons, bf, dx)
    rng = np.random.default_rng(7)
    worst = 0.0
    for rep in range(3):
        tc = rng.standard_normal(cons.shape)
        tb = rng.standard_normal(bf.shape)
        gc = rng.standard_normal(cons.shape)
        gb = rng.standard_normal(bf.shape)
        _, _, jc, jb = oracle.step_dual(Q, cons, bf, tc, tb, dx, [dt])
        l1, s1 = _dot(gc, jc)
        l2, s2 = _dot(gb, jb)
        ac, ab = adjoint(P, cons, bf, dx, dt, gc, gb)
        r1, t1 = _dot(ac, tc)
        r2, t2 = _dot(ab, tb)
        lhs, rhs = l1 + l2, r1 + r2
        scale = max(s1 + s2, t1 + t2)
        err = abs(lhs - rhs) / scale
        worst = max(worst, err)
        print(f"[adjoint] {recon} {riemann} eta={eta} rep {rep}: <g, J t> = {lhs:.12e}, "
              f"<J^T g, t> = {rhs:.12e}, relative {err:.2e}", flush=True)
    assert worst <= 1e-12, worst


def test_adjoint_gradient_vs_central_differences_16():
    """Loss L(S) = <w, step(S)> on the 16^3 smooth box (amplitude 0.05,
    beta = 1; FP64, PLM-MC + HLLD + Q26 + LD04, eta = 1e-3, no flux
    correction, frozen dt).  Sampled entries of dL/dS from the adjoint against
    fourth-order central differences of the GPU forward step, one entry at a
    time (a dense random direction would cross limiter kinks somewhere in the
    box; one entry moves only the limiters around one cell)."""
    n = 16
    cons, bf, info = inputs.smooth_modes_box(n, amp=0.05, beta=1.0, seed=5)
    dx = info["dx"]
    P = ctmhd.make_params(recon="plm", riemann="hlld", eta=1e-3, fofc=False)
    Q = oracle.make_params(recon="plm", riemann="hlld", eta=1e-3, fofc=False)
    dt = oracle.cfl_dt(Q, cons, bf, dx)
    rng = np.random.default_rng(11)
    wc = rng.standard_normal(cons.shape)
    wb = rng.standard_normal(bf.shape)
    ac, ab = adjoint(P, cons, bf, dx, dt, wc, wb)
    gscale = float(np.abs(np.concatenate([ac, ab])).mean())

    def loss(c, b):
        c1, b1, _, _ = ctmhd.run(P, c, b, dx, 1, dt_fixed=[dt])
        return float(np.sum(wc * c1) + np.sum(wb * b1))

    worst = 0.0
    for rep in range(16):
        m = int(rng.integers(0, 8))
        k, j, i = (int(v) for v in rng.integers(0, n, 3))
        dc = np.zeros(cons.shape)
        db = np.zeros(bf.shape)
        if m < 5:
            dc[m, k, j, i] = 1.0
            h = 1e-5 * float(np.abs(cons[m]).mean())
            an = ac[m, k, j, i]
        else:
            db[m - 5, k, j, i] = 1.0
            h = 1e-5 * float(np.abs(bf).mean())
            an = ab[m - 5, k, j, i]
        f = {s_: loss(cons + s_ * h * dc, bf + s_ * h * db) for s_ in (-2, -1, 1, 2)}
        fd = (-f[2] + 8.0 * f[1] - 8.0 * f[-1] + f[-2]) / (12.0 * h)
        err = abs(fd - an) / (abs(fd) + 1e-3 * gscale)
        worst = max(worst, err)
        print(f"[adjoint] 16^3 entry field {m} cell {(k, j, i)}: adjoint {an:.12e}, "
              f"central difference {fd:.12e}, relative {err:.2e}", flush=True)
    assert worst <= 1e-6, worst


@pytest.mark.parametrize("kw", [dict(recon="ppm"), dict(precision="fp32"), dict(emf="b25a")])
def test_adjoint_refuses_unsupported(kw):
    import torch
    P = ctmhd.make_params(**kw)
    b = ctmhd.make_box((8, 8, 8), ctmhd.required_ghosts(P), (0.1, 0.1, 0.1))
    assert ctmhd.adjoint_workspace_bytes(P, b) == 0
    x = torch.zeros(ctmhd.lib().ctmhd_box_elems(b), dtype=torch.float64, device="cuda")
    with pytest.raises(ctmhd.CtmhdError, match="adjoint"):
        ctmhd.ctmhd_step_adjoint(P, b, [x] * 5, [x] * 3, x, [x] * 5, [x] * 3, [x] * 5, [x] * 3,
                                 torch.zeros(256, dtype=torch.uint8, device="cuda"))
