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
