"""Shared test helpers: diagnostics defined from the paper, axis permutations.

Array layout: cons (5, n2, n1, n0), bface (3, n2, n1, n0); box axis d is
numpy axis 2 - d of a field.
"""
import numpy as np


def ax(d):
    return 2 - d


def divb(bface, dx):
    """Discrete divergence at cell centres: sum_a (b_a[p+e_a] - b_a[p]) / dx_a."""
    return sum((np.roll(bface[a], -1, axis=ax(a)) - bface[a]) / dx[a] for a in range(3))


def divb_rel(bface, dx):
    """max |div b| / max sum_a (|b_a[+]| + |b_a[-]|)/dx_a (the relative measure)."""
    num = np.abs(divb(bface, dx)).max()
    den = sum((np.abs(np.roll(bface[a], -1, axis=ax(a))) + np.abs(bface[a])) / dx[a]
              for a in range(3)).max()
    return num / den


def relative_error(sim, exact):
    """Eqs. error:absolute, error:normalisation and error:relative: sim and exact
    are lists of arrays (one per element of the state vector)."""
    num = 0.0
    den = 0.0
    for s, e in zip(sim, exact):
        n = s.size
        err = np.abs(e - s).mean()
        nrm = np.abs(e).mean()
        num += (err * n) ** 2
        den += (nrm * n) ** 2
    return np.sqrt(num / den)


def state_list(cons, bface):
    return [cons[m] for m in range(5)] + [bface[a] for a in range(3)]


def rel_l1(a, b):
    """Relative L1 difference of two arrays."""
    den = np.abs(b).sum()
    if den == 0:
        return np.abs(a - b).sum()
    return np.abs(a - b).sum() / den


def permute_cyclic(cons, bface):
    """Relabel axes cyclically: new axis d+1 holds old axis d.  Fields are
    (.., n2, n1, n0); vector components rotate the same way."""
    def tr(f):
        # old numpy axes (z, y, x) = old box axes (2, 1, 0); new box axis
        # (d+1)%3 = old d, i.e. new x1 = old x0, new x2 = old x1, new x0 = old x2.
        # new numpy layout (new2, new1, new0) = (old1, old0, old2)
        return np.transpose(f, (1, 2, 0))
    c = np.stack([tr(cons[0]), tr(cons[3]), tr(cons[1]), tr(cons[2]), tr(cons[4])])
    b = np.stack([tr(bface[2]), tr(bface[0]), tr(bface[1])])
    return np.ascontiguousarray(c), np.ascontiguousarray(b)


def permute_dx(dx):
    return [dx[2], dx[0], dx[1]]


def reflect(cons, bface):
    """Point reflection x -> L - x: cell i (spanning [i, i+1] dx) -> N-1-i,
    the lower face of cell j takes old face (N-j) mod N; u -> -u, b -> -b."""
    def fc(f):
        return f[::-1, ::-1, ::-1]
    c = np.stack([fc(cons[0]), -fc(cons[1]), -fc(cons[2]), -fc(cons[3]), fc(cons[4])])
    b = np.stack([-np.roll(fc(bface[a]), 1, axis=ax(a)) for a in range(3)])
    return np.ascontiguousarray(c), np.ascontiguousarray(b)


FIELDS = ("rho", "m0", "m1", "m2", "e", "b0", "b1", "b2")


def compare_fields(cg, bg, co, bo, tol, label="", pert=None):
    """The float64 parity bar, three checks at once:
      - the relative error of eq. error:relative over all 8 fields <= tol;
      - per field, the plain relative L1 difference sum|d| / sum|oracle| <= tol;
      - per field, element by element, max|d| / max|oracle| <= tol.
    Each field is measured at its own scale.  `pert` maps the index of a
    field that carries only a perturbation of amplitude delta on an O(1)
    background (the momentum of a linear eigenmode) to delta: FP64 round-off
    of the O(1) fluxes that update it is about 1e-16 of 1, i.e. 1e-16/delta of
    the field itself per operation, so its two per-field bars are
    max(tol, 1e-13 / delta) instead.  Returns (relative error, worst
    per-element value over the fields held to tol)."""
    pert = pert or {}
    rel = relative_error(state_list(cg, bg), state_list(co, bo))
    g = state_list(cg, bg)
    o = state_list(co, bo)
    worst = 0.0
    msgs = []
    for f, (x, y) in enumerate(zip(g, o)):
        d = np.abs(x - y)
        if np.abs(y).max() == 0.0:
            # a field that is exactly zero in the oracle (a component no
            # force drives): measured on the scale of its vector's components
            grp = o[1:4] if 1 <= f <= 3 else o[5:8] if f >= 5 else [y]
            ref = max(float(np.abs(v).max()) for v in grp)
            el = float(d.max() / max(ref, 1e-300))
            l1 = float(d.sum() / max(ref * d.size, 1e-300))
        else:
            el = float(d.max() / np.abs(y).max())
            l1 = float(d.sum() / np.abs(y).sum())
        bar = max(tol, 1e-13 / pert[f]) if f in pert else tol
        msgs.append(f"{FIELDS[f]} {el:.1e}/{l1:.1e}" + ("*" if f in pert else ""))
        assert el <= bar and l1 <= bar, (label, FIELDS[f], el, l1, bar)
        if f not in pert:
            worst = max(worst, el)
    print(f"[parity] {label} rel_err={rel:.3e} per field max/L1: " + " ".join(msgs), flush=True)
    assert rel <= tol, (label, rel)
    return rel, worst


def field_errors(cg, bg, co, bo):
    """Per field (rho, m0, m1, m2, e, b0, b1, b2): (plain relative L1,
    relative L1 with the normalisation of compare_fields)."""
    rho_l1 = np.abs(co[0]).sum()
    u = np.sqrt((co[1:4] ** 2).sum(0)) / co[0]
    smax = float(u.max()) + 1.0
    out = []
    for m in range(5):
        d = np.abs(cg[m] - co[m]).sum()
        den = max(np.abs(co[m]).sum(), rho_l1 * smax * (1.0 if m in (1, 2, 3) else 0.0), 1e-300)
        out.append((d / max(np.abs(co[m]).sum(), 1e-300), d / den))
    for a in range(3):
        d = np.abs(bg[a] - bo[a]).sum()
        den = max(np.abs(bo[a]).sum(), np.abs(bo).sum() / 3, 1e-300)
        out.append((d / max(np.abs(bo[a]).sum(), 1e-300), d / den))
    return out
