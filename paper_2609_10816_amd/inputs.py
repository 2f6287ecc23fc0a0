"""Seeded synthetic initial states for the CT-MHD step.

This module holds only input construction: plane-wave eigenmodes, seeded
random-phase spectral fields and the discrete curl of an edge-centred vector
potential.  It contains none of the step's arithmetic and is the one piece of
code that both the GPU path's callers and the CPU oracle's callers use.

Layout (host, numpy float64, periodic box, interior cells only):
  cons  (5, n2, n1, n0): rho, m0, m1, m2, e_tot at cell centres
  bface (3, n2, n1, n0): b_a on the lower x_a face of each cell
Index order [k, j, i] with i (x0) fastest.  Cell (i,j,k) has its centre at
((i+1/2) dx0, (j+1/2) dx1, (k+1/2) dx2) on the domain [0, L)^3.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

GAMMA = 5.0 / 3.0


def _coords(n, L=(1.0, 1.0, 1.0), shift=(0.5, 0.5, 0.5)):
    """Coordinates (x0, x1, x2) of shape (n2, n1, n0) at index + shift."""
    n0, n1, n2 = n
    dx = [L[d] / n[d] for d in range(3)]
    k, j, i = np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij")
    return ((i + shift[0]) * dx[0], (j + shift[1]) * dx[1], (k + shift[2]) * dx[2])


def face_coords(n, a, L=(1.0, 1.0, 1.0)):
    s = [0.5, 0.5, 0.5]
    s[a] = 0.0
    return _coords(n, L, s)


def edge_coords(n, c, L=(1.0, 1.0, 1.0)):
    s = [0.0, 0.0, 0.0]
    s[c] = 0.5
    return _coords(n, L, s)


def curl_edges(A, dx):
    """Face field from an edge-centred vector potential by the discrete curl:
    b_a[p] = (A_c[p+e_b] - A_c[p])/dx_b - (A_b[p+e_c] - A_b[p])/dx_c,
    with (a, b, c) cyclic and A_c stored at the lower-left edge of each cell.
    Arrays are (3, n2, n1, n0); axis d of the box is numpy axis 2-d."""
    B = np.zeros_like(A)
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        dAc = np.roll(A[c], -1, axis=2 - b) - A[c]
        dAb = np.roll(A[b], -1, axis=2 - c) - A[b]
        B[a] = dAc / dx[b] - dAb / dx[c]
    return B


def from_primitives(rho, u, p, bface, gamma=GAMMA):
    """Conserved cell state from primitive cell values and face fields; the
    cell field is the mean of the two faces and e_tot = p/(gamma-1) +
    (rho u^2 + b^2)/2."""
    bc = np.stack([0.5 * (bface[a] + np.roll(bface[a], -1, axis=2 - a)) for a in range(3)])
    cons = np.empty((5,) + rho.shape)
    cons[0] = rho
    for d in range(3):
        cons[1 + d] = rho * u[d]
    cons[4] = p / (gamma - 1.0) + 0.5 * rho * (u ** 2).sum(0) + 0.5 * (bc ** 2).sum(0)
    return cons


def uniform(n, rho=1.0, u=(0.0, 0.0, 0.0), p=0.6, b=(0.0, 0.0, 0.0), gamma=GAMMA):
    shape = (n[2], n[1], n[0])
    rr = np.full(shape, float(rho))
    uu = np.stack([np.full(shape, float(v)) for v in u])
    pp = np.full(shape, float(p))
    bf = np.stack([np.full(shape, float(v)) for v in b])
    return from_primitives(rr, uu, pp, bf, gamma), bf


# ---------------------------------------------------------------------------
# Linear waves (paper Sec. 3.1): background (eq. wave:background) plus a
# plane-wave eigenmode; the face field comes from the curl of an edge
# potential so that the discrete divergence vanishes to round-off.
# ---------------------------------------------------------------------------
def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def _plane_potential(n, L, kvec, terms, t_phase):
    """Edge potential whose curl is sum_t c_t * f_t(k.x - omega t) with f_t in
    {cos, sin}; each c_t must be orthogonal to k."""
    kk = 2.0 * np.pi * np.asarray(kvec, np.float64) / np.asarray(L, np.float64)
    knorm = np.linalg.norm(kk)
    nk = kk / knorm
    A = np.zeros((3, n[2], n[1], n[0]))
    for c in range(3):
        x = edge_coords(n, c, L)
        s = kk[0] * x[0] + kk[1] * x[1] + kk[2] * x[2] - t_phase
        for vec, kind in terms:
            a = np.cross(np.asarray(vec, np.float64), nk) / knorm
            if kind == "cos":
                A[c] += a[c] * np.sin(s)
            else:
                A[c] -= a[c] * np.cos(s)
    return A


def fast_wave(n, kvec=(1, 1, 1), delta=1e-6, rho0=1.0, p0=0.6, b0=(1.0, 1.414, 0.5),
              gamma=GAMMA, t=0.0, L=(1.0, 1.0, 1.0), slow=False):
    """Fast (or slow) magnetosonic eigenmode (paper Sec. 3.1.3 / 3.1.4):
    drho = phi1 rho, du = c (phi1 n_k - phi2 n_perp) [fast] or
    c (-phi1 n_k + phi2 n_perp) [slow], db = b n_perp, all times
    delta cos(omega t - k.x); dp = c_s^2 drho (adiabatic).  n_perp lies in the
    (n_k, n_bg) plane with sin(theta) >= 0.  e_tot from its definition.
    Returns (cons, bface, info)."""
    b0 = np.asarray(b0, np.float64)
    bmag = np.linalg.norm(b0)
    kk = 2.0 * np.pi * np.asarray(kvec, np.float64) / np.asarray(L, np.float64)
    nk = kk / np.linalg.norm(kk)
    nbg = b0 / bmag
    cos_t = float(np.dot(nbg, nk))
    perp = nbg - cos_t * nk
    nperp = perp / np.linalg.norm(perp)
    sin_t = float(np.dot(nbg, nperp))
    cs2 = gamma * p0 / rho0
    ca2 = bmag ** 2 / rho0
    disc = math.sqrt((cs2 + ca2) ** 2 - 4.0 * cs2 * ca2 * cos_t ** 2)
    c2 = 0.5 * (cs2 + ca2 + (-disc if slow else disc))
    cw = math.sqrt(c2)
    phi1 = (c2 - ca2 * cos_t ** 2) / (c2 * sin_t)
    phi2 = ca2 / c2 * cos_t
    omega = cw * np.linalg.norm(kk)
    x = _coords(n, L)
    ph = omega * t - (kk[0] * x[0] + kk[1] * x[1] + kk[2] * x[2])
    amp = delta * np.cos(ph)
    rho = rho0 * (1.0 + phi1 * amp)
    uvec = cw * (phi1 * nk - phi2 * nperp) * (-1.0 if slow else 1.0)
    u = np.stack([uvec[d] * amp for d in range(3)])
    p = p0 + cs2 * rho0 * phi1 * amp
    A = _plane_potential(n, L, kvec, [(bmag * delta * nperp, "cos")], omega * t)
    dx = [L[d] / n[d] for d in range(3)]
    bf = curl_edges(A, dx)
    for a in range(3):
        bf[a] += b0[a]
    cons = from_primitives(rho, u, p, bf, gamma)
    info = dict(omega=omega, period=2.0 * np.pi / omega, speed=cw, phi1=phi1, phi2=phi2,
                theta=math.degrees(math.acos(max(-1.0, min(1.0, cos_t)))), dx=dx)
    return cons, bf, info


def alfven_wave(n, kvec=(1, 0, 0), delta=1e-6, rho0=1.0, p0=1.0 / GAMMA, b0=(1.0, 0.0, 0.0),
                nperp=(0.0, 0.0, 1.0), gamma=GAMMA, t=0.0, L=(1.0, 1.0, 1.0), decay=0.0,
                omega=None):
    """Linearly polarised Alfven wave (paper Sec. 3.1.1):
    du = -c_A n_perp, db = b n_perp, times delta cos(omega t - k.x); optional
    amplitude factor exp(-decay t) and frequency override (resistive closed
    form of Sec. 4, eqs. resistivity:alfven-decay/frequency)."""
    b0 = np.asarray(b0, np.float64)
    bmag = np.linalg.norm(b0)
    kk = 2.0 * np.pi * np.asarray(kvec, np.float64) / np.asarray(L, np.float64)
    nk = kk / np.linalg.norm(kk)
    ca = bmag / math.sqrt(rho0)
    if omega is None:
        omega = ca * np.linalg.norm(kk) * abs(float(np.dot(b0 / bmag, nk)))
    npp = _unit(nperp)
    x = _coords(n, L)
    shape = x[0].shape
    fac = delta * math.exp(-decay * t)
    amp = fac * np.cos(omega * t - (kk[0] * x[0] + kk[1] * x[1] + kk[2] * x[2]))
    rho = np.full(shape, rho0)
    u = np.stack([-ca * npp[d] * amp for d in range(3)])
    p = np.full(shape, p0)
    A = _plane_potential(n, L, kvec, [(bmag * fac * npp, "cos")], omega * t)
    dx = [L[d] / n[d] for d in range(3)]
    bf = curl_edges(A, dx)
    for a in range(3):
        bf[a] += b0[a]
    cons = from_primitives(rho, u, p, bf, gamma)
    return cons, bf, dict(omega=omega, period=2 * np.pi / omega, dx=dx, ca=ca, k=np.linalg.norm(kk))


def circular_alfven(n, kvec=(1, 0, 0), delta=0.1, rho0=1.0, p0=1.0 / GAMMA, bmag=1.0,
                    n1=(0.0, 1.0, 0.0), n2=(0.0, 0.0, 1.0), gamma=GAMMA, t=0.0,
                    L=(1.0, 1.0, 1.0)):
    """Circularly polarised Alfven wave (paper Sec. 3.1.2), an exact nonlinear
    solution: b_bg along n_k, du = -c_A delta (sin phi n1 + cos phi n2),
    db = b delta (sin phi n1 + cos phi n2), phi = omega t - k.x."""
    kk = 2.0 * np.pi * np.asarray(kvec, np.float64) / np.asarray(L, np.float64)
    nk = kk / np.linalg.norm(kk)
    ca = bmag / math.sqrt(rho0)
    omega = ca * np.linalg.norm(kk)
    e1, e2 = _unit(n1), _unit(n2)
    x = _coords(n, L)
    ph = omega * t - (kk[0] * x[0] + kk[1] * x[1] + kk[2] * x[2])
    shape = ph.shape
    rho = np.full(shape, rho0)
    u = np.stack([-ca * delta * (np.sin(ph) * e1[d] + np.cos(ph) * e2[d]) for d in range(3)])
    p = np.full(shape, p0)
    # db = b delta (-sin(s - wt) e1 + cos(s - wt) e2) with s = k.x
    A = _plane_potential(n, L, kvec, [(-bmag * delta * e1, "sin"), (bmag * delta * e2, "cos")],
                         omega * t)
    dx = [L[d] / n[d] for d in range(3)]
    bf = curl_edges(A, dx)
    for a in range(3):
        bf[a] += bmag * nk[a]
    cons = from_primitives(rho, u, p, bf, gamma)
    return cons, bf, dict(omega=omega, period=2 * np.pi / omega, dx=dx)


# ---------------------------------------------------------------------------
# Seeded random-phase spectral fields (turbulent boxes).
# ---------------------------------------------------------------------------
def _kshell(kmin, kmax):
    r = int(math.floor(kmax))
    ks = [k for k in itertools.product(range(-r, r + 1), repeat=3)
          if kmin <= math.sqrt(k[0] ** 2 + k[1] ** 2 + k[2] ** 2) <= kmax]
    return np.array(sorted(ks), dtype=np.int64)


def _spectral_vector(n, seed, kmin, kmax, slope, solenoidal, shifts):
    """Real vector field sum_k Re(c_k exp(2 pi i k.x)) with |c_k| ~ |k|^slope,
    random phases (complex normal), optionally projected solenoidal.
    Component d is evaluated at grid index + shifts[d] (a 3-vector)."""
    rng = np.random.default_rng(seed)
    ks = _kshell(kmin, kmax)
    coef = rng.normal(size=(len(ks), 3)) + 1j * rng.normal(size=(len(ks), 3))
    kn = np.linalg.norm(ks, axis=1)
    if solenoidal:
        kh = ks / kn[:, None]
        coef = coef - kh * (kh * coef).sum(1)[:, None]
    coef *= (kn ** slope)[:, None]
    n0, n1, n2 = n
    out = np.empty((3, n2, n1, n0))
    for d in range(3):
        spec = np.zeros((n2, n1, n0), np.complex128)
        sh = shifts[d]
        phase = np.exp(2j * np.pi * (ks[:, 0] * sh[0] / n0 + ks[:, 1] * sh[1] / n1 +
                                     ks[:, 2] * sh[2] / n2))
        np.add.at(spec, (ks[:, 2] % n2, ks[:, 1] % n1, ks[:, 0] % n0), coef[:, d] * phase)
        out[d] = np.real(np.fft.ifftn(spec)) * (n0 * n1 * n2)
        del spec
    return out


def turbulent_box(n, mach=5.0, b0=(0.1, 0.0, 0.0), db_rms=0.05, seed_v=1, seed_a=2,
                  rho0=1.0, gamma=GAMMA, kmin=1.0, kmax=4.0):
    """Driven-free turbulent box: rho = 1, p = 1/gamma (c_s = 1), seeded
    random-phase solenoidal velocity with per-mode |u_k| ~ k^-2 on
    kmin <= |k| <= kmax scaled to rms |u| = mach, field b0 plus the curl of a
    seeded edge potential with |A_k| ~ k^-3 scaled to rms |db| = db_rms."""
    n = tuple(int(v) for v in n)
    dx = [1.0 / n[d] for d in range(3)]
    cs = [(0.5, 0.5, 0.5)] * 3
    u = _spectral_vector(n, seed_v, kmin, kmax, -2.0, True, cs)
    u *= mach / math.sqrt(float((u ** 2).sum(0).mean()))
    es = [tuple(0.5 if d == c else 0.0 for d in range(3)) for c in range(3)]
    A = _spectral_vector(n, seed_a, kmin, kmax, -3.0, False, es)
    db = curl_edges(A, dx)
    rms = math.sqrt(float((db ** 2).sum(0).mean()))
    db *= db_rms / rms if rms > 0 else 0.0
    bf = db
    for a in range(3):
        bf[a] += b0[a]
    shape = (n[2], n[1], n[0])
    rho = np.full(shape, rho0)
    p = np.full(shape, rho0 / gamma)
    cons = from_primitives(rho, u, p, bf, gamma)
    return cons, bf, dict(dx=dx)


# ---------------------------------------------------------------------------
# The named workloads.
# ---------------------------------------------------------------------------
def linear_fast_wave_32(n=32):
    """32^3 periodic ideal MHD, gamma 5/3: rho 1, p 0.6, b (1, 1.414, 0.5),
    u 0, fast eigenmode of amplitude 1e-6 along (1,1,1)."""
    cons, bf, info = fast_wave((n, n, n), kvec=(1, 1, 1), delta=1e-6, rho0=1.0, p0=0.6,
                               b0=(1.0, 1.414, 0.5))
    return cons, bf, info


def turbulent_mach5(n=128):
    """Driven-free turbulent box, rms Mach 5, b = (0.1, 0, 0) + curl A."""
    return turbulent_box((n, n, n), mach=5.0, b0=(0.1, 0.0, 0.0), db_rms=0.05, seed_v=1, seed_a=2)


def turbulent_mach2_beta1(n=256):
    """The turbulent recipe at rms Mach 2 and plasma beta 1 (|b0| = sqrt(2p)
    along x0), rms |db| = |b0|/2."""
    b = math.sqrt(2.0 / GAMMA)
    return turbulent_box((n, n, n), mach=2.0, b0=(b, 0.0, 0.0), db_rms=0.5 * b, seed_v=1, seed_a=2)


def amr_like_boxes(nbox=2000, seed=4, dx=1.0 / 64.0, sizes=(8, 16, 32, 64), gamma=GAMMA):
    """Many small periodic boxes of uneven sizes (one AMR level, common dx).
    Per box: edge lengths drawn per axis from `sizes`; rho = 1 + 0.2 S_rho,
    u_d = 0.5 S_ud, edge potential A_c = 0.1 |b0| L_min / (2 pi) S_Ac (so that
    each mode's field perturbation is at most 0.1 |b0| |k|), where each S is a sum
    of 3 sine modes with integer per-box-periodic wave vectors (components in
    {0,1,2}, not all zero) and uniform random phases; p = 1/gamma; b0 along a
    random axis with |b0| = sqrt(2p/beta), log10 beta uniform in [-1, 1].
    Returns a list of (cons, bface, dx)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nbox):
        n = tuple(int(v) for v in rng.choice(sizes, size=3))
        L = tuple(n[d] * dx for d in range(3))

        def modes():
            ks = []
            while len(ks) < 3:
                k = rng.integers(0, 3, size=3)
                if k.any():
                    ks.append(k)
            return ks, rng.uniform(0.0, 2.0 * np.pi, size=3)

        def series(ks, ph, x):
            return sum(np.sin(2.0 * np.pi * (k[0] * x[0] / L[0] + k[1] * x[1] / L[1] +
                                             k[2] * x[2] / L[2]) + f) for k, f in zip(ks, ph))

        xc = _coords(n, L)
        ks, ph = modes()
        rho = 1.0 + 0.2 * series(ks, ph, xc)
        u = np.stack([0.5 * series(*modes(), xc) for _ in range(3)])
        p0 = 1.0 / gamma
        beta = 10.0 ** rng.uniform(-1.0, 1.0)
        bmag = math.sqrt(2.0 * p0 / beta)
        axis = int(rng.integers(0, 3))
        A = np.zeros((3, n[2], n[1], n[0]))
        amp = 0.1 * bmag * min(L) / (2.0 * np.pi)
        for c in range(3):
            A[c] = amp * series(*modes(), edge_coords(n, c, L))
        bf = curl_edges(A, [dx, dx, dx])
        bf[axis] += bmag
        p = np.full(rho.shape, p0)
        out.append((from_primitives(rho, u, p, bf, gamma), bf, (dx, dx, dx)))
    return out


def smooth_modes_box(n, amp=0.05, beta=1.0, seed=5, nmodes=3, L=(1.0, 1.0, 1.0), gamma=GAMMA):
    """A smooth periodic box for the derivative workload: rho = 1 + amp S,
    u_d = amp S_d, p = p0 (1 + amp S_p) with p0 = 1/gamma (sound speed 1),
    b = b0 x + curl A with |b0| = sqrt(2 p0 / beta) and
    A_c = amp |b0| L_min / (2 pi) S_Ac, where each S is a sum of `nmodes` sine
    modes with integer wave vectors whose components are all non-zero (each
    +-1 or +-2) and uniform random phases.  Every field varies along every
    axis, so no limiter or min/max of the step sits exactly at a tie (a field
    constant along an axis puts every limiter along it at dl = dr = 0, where
    the derivative of the step is not unique).  Returns (cons, bface, info)."""
    n = (n, n, n) if np.isscalar(n) else tuple(int(v) for v in n)
    L = tuple(float(v) for v in L)
    rng = np.random.default_rng(seed)

    def modes():
        ks = [rng.integers(1, 3, size=3) * rng.choice([-1, 1], size=3) for _ in range(nmodes)]
        return ks, rng.uniform(0.0, 2.0 * np.pi, size=nmodes)

    def series(ks, ph, x):
        return sum(np.sin(2.0 * np.pi * (k[0] * x[0] / L[0] + k[1] * x[1] / L[1] +
                                         k[2] * x[2] / L[2]) + f) for k, f in zip(ks, ph))

    xc = _coords(n, L)
    rho = 1.0 + amp * series(*modes(), xc)
    u = np.stack([amp * series(*modes(), xc) for _ in range(3)])
    p0 = 1.0 / gamma
    p = p0 * (1.0 + amp * series(*modes(), xc))
    bmag = math.sqrt(2.0 * p0 / beta)
    dx = [L[d] / n[d] for d in range(3)]
    A = np.zeros((3, n[2], n[1], n[0]))
    for c in range(3):
        A[c] = amp * bmag * min(L) / (2.0 * np.pi) * series(*modes(), edge_coords(n, c, L))
    bf = curl_edges(A, dx)
    bf[0] += bmag
    return from_primitives(rho, u, p, bf, gamma), bf, {"dx": dx, "b0": bmag}


def field_loop(n=(96, 64, 32), radius=0.5, db=1e-3, gamma=GAMMA):
    """Field-loop advection (Sec. 4.6): the domain [-1.5, 1.5] x [-1, 1] x
    [-0.5, 0.5], rho = 1, p = 1, a uniform velocity (3, 2, 1)/sqrt(13) and a
    weak loop of field db inside the cylinder r = sqrt(x0^2 + x1^2) < radius,
    from the edge potential A_2 = db max(radius - r, 0) (b = db (-x1, x0)/r
    inside), so that the discrete divergence is zero to round-off.
    Returns (cons, bface, info)."""
    L = (3.0, 2.0, 1.0)
    dx = tuple(L[d] / n[d] for d in range(3))
    A = np.zeros((3, n[2], n[1], n[0]))
    x0, x1, _ = edge_coords(n, 2, L)
    r = np.sqrt((x0 - 1.5) ** 2 + (x1 - 1.0) ** 2)
    A[2] = db * np.maximum(radius - r, 0.0)
    bf = curl_edges(A, dx)
    shp = (n[2], n[1], n[0])
    u = np.zeros((3,) + shp)
    for d, v in enumerate((3.0, 2.0, 1.0)):
        u[d] = v / math.sqrt(13.0)
    cons = from_primitives(np.ones(shp), u, np.ones(shp), bf, gamma)
    return cons, bf, {"dx": dx, "L": L, "gamma": gamma}
