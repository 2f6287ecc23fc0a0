"""Pins of the oracle's building blocks against closed forms and textbook
properties (CPU only).

Reconstruction (paper Sec. 2.2): PLM with the MC / minmod limiters and the
Colella-Woodward PPM; Riemann solvers (Sec. 2.2): HLLD, HLL and LLF; fast
speed (eq. waves:fast-speed).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle

GAMMA = 5.0 / 3.0
HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- reconstruction
@pytest.mark.parametrize("method", ["pc", "plm_mc", "plm_minmod", "ppm"])
def test_linear_data_exact(method):
    q = 2.0 + 0.75 * np.arange(-2, 3)
    qm, qp = oracle.recon1d(method, q)
    if method == "pc":
        assert qm == qp == q[2]
    else:
        assert qm == pytest.approx(q[2] - 0.375, abs=1e-15)
        assert qp == pytest.approx(q[2] + 0.375, abs=1e-15)


def test_limiter_tables():
    # Hand values of the limited slope: Delta- = 1, Delta+ = 2.
    qm, qp = oracle.recon1d("plm_mc", [9.0, 0.0, 1.0, 3.0, 9.0])
    assert (qm, qp) == (1.0 - 0.75, 1.0 + 0.75)  # MC: min(2, 4, 1.5) = 1.5
    qm, qp = oracle.recon1d("plm_minmod", [9.0, 0.0, 1.0, 3.0, 9.0])
    assert (qm, qp) == (0.5, 1.5)  # minmod: min(1, 2) = 1
    # Delta- = 1, Delta+ = 10: MC picks 2|Delta-| = 2.
    qm, qp = oracle.recon1d("plm_mc", [9.0, 0.0, 1.0, 11.0, 9.0])
    assert (qm, qp) == (0.0, 2.0)
    # Extremum: slope zero for every limiter, PPM flattens.
    for m in ["plm_mc", "plm_minmod", "ppm"]:
        assert oracle.recon1d(m, [0.0, 1.0, 2.0, 1.0, 0.0]) == (2.0, 2.0)


def _cubic_avg(c, lo, hi):
    # exact cell average of c0 + c1 x + c2 x^2 + c3 x^3 over [lo, hi]
    F = lambda x: c[0] * x + c[1] * x ** 2 / 2 + c[2] * x ** 3 / 3 + c[3] * x ** 4 / 4
    return (F(hi) - F(lo)) / (hi - lo)


def test_ppm_fourth_order_interface_on_cubic():
    """With the limiters inactive the CW interface value is the 4th-order one,
    exact for cell averages of a cubic."""
    c = (1.0, 0.3, 0.02, 0.001)
    q = np.array([_cubic_avg(c, i - 0.5, i + 0.5) for i in range(-2, 3)])
    qm, qp = oracle.recon1d("ppm", q)
    f = lambda x: c[0] + c[1] * x + c[2] * x ** 2 + c[3] * x ** 3
    assert qm == pytest.approx(f(-0.5), abs=1e-14)
    assert qp == pytest.approx(f(0.5), abs=1e-14)


def test_ppm_parabola_monotone_constraint():
    """A steep one-sided jump: the parabola must stay within the neighbours'
    range and be monotone inside the cell (|q6| <= (qR-qL)^2/6 after the fix)."""
    rng = np.random.default_rng(0)
    for _ in range(4000):
        q = rng.normal(size=5) * rng.choice([1e-3, 1.0, 1e3])
        for m in ["plm_mc", "plm_minmod", "ppm"]:
            qm, qp = oracle.recon1d(m, q)
            lo1, hi1 = min(q[1], q[2]), max(q[1], q[2])
            lo2, hi2 = min(q[2], q[3]), max(q[2], q[3])
            tol = 1e-12 * max(1.0, np.abs(q).max())
            assert lo1 - tol <= qm <= hi1 + tol
            assert lo2 - tol <= qp <= hi2 + tol
            if m == "ppm" and qp != qm:
                dq = qp - qm
                q6 = 6.0 * (q[2] - 0.5 * (qm + qp))
                assert abs(q6) <= abs(dq) * (1 + 1e-9) + tol


# ----------------------------------------------------------------- fast speed
def test_fast_speed_golden():
    """Directional fast speeds of the 32^3 fast-wave background
    (rho 1, p 0.6, b (1, 1.414, 0.5), gamma 5/3), from eq. waves:fast-speed
    with cos^2(theta) = b_d^2 / b^2; values in tests/golden/fast_speed_c1.json."""
    g = json.load(open(os.path.join(HERE, "golden", "fast_speed_c1.json")))
    b = g["b"]
    for d in range(3):
        cf = oracle.fast_speed(g["rho"], g["p"], b[d], b[(d + 1) % 3], b[(d + 2) % 3], GAMMA)
        assert cf == pytest.approx(g["cf"][d], abs=5e-6)


def test_fast_speed_limits():
    # b = 0: sound speed; p -> 0: Alfven speed along b_n when b = b_n only
    assert oracle.fast_speed(2.0, 3.0, 0.0, 0.0, 0.0, GAMMA) == pytest.approx(
        math.sqrt(GAMMA * 3.0 / 2.0), rel=1e-15)
    assert oracle.fast_speed(4.0, 1e-30, 2.0, 0.0, 0.0, GAMMA) == pytest.approx(1.0, rel=1e-12)
    # perpendicular field: sqrt(c_s^2 + c_A^2)
    assert oracle.fast_speed(1.0, 0.6, 0.0, 1.0, 0.0, GAMMA) == pytest.approx(math.sqrt(2.0),
                                                                             rel=1e-14)


# ------------------------------------------------------------ Riemann solvers
def physical_flux(s, bn, gamma=GAMMA):
    """Ideal-MHD flux of (rho, m_n, m_t1, m_t2, e_tot) normal to a face,
    eq. mhd:conservation-laws, for a face-local state (rho, un, ut1, ut2, p,
    bt1, bt2)."""
    rho, un, v, w, p, by, bz = s
    b2 = bn * bn + by * by + bz * bz
    e = p / (gamma - 1) + 0.5 * rho * (un * un + v * v + w * w) + 0.5 * b2
    pt = p + 0.5 * b2
    vb = un * bn + v * by + w * bz
    F = np.array([rho * un, rho * un * un + pt - bn * bn, rho * un * v - bn * by,
                  rho * un * w - bn * bz, (e + pt) * un - bn * vb])
    U = np.array([rho, rho * un, rho * v, rho * w, e])
    return F, U


def _rand_state(rng):
    return np.array([rng.uniform(0.2, 3.0), rng.normal() * 2, rng.normal(), rng.normal(),
                     rng.uniform(0.05, 3.0), rng.normal(), rng.normal()])


@pytest.mark.parametrize("solver", ["hlld", "hll", "llf"])
def test_consistency(solver):
    rng = np.random.default_rng(1)
    for _ in range(300):
        s = _rand_state(rng)
        bn = rng.normal()
        if solver == "hlld":
            F, _, _, fb = oracle.hlld(s, s, bn, GAMMA)
            assert fb == 0
        elif solver == "hll":
            F = oracle.hll(s, s, bn, GAMMA)
        else:
            F, _ = oracle.llf(s, s, bn, GAMMA)
        Fx, _ = physical_flux(s, bn)
        np.testing.assert_allclose(F, Fx, rtol=1e-12, atol=1e-12 * np.abs(Fx).max())


def test_supersonic_upwind():
    rng = np.random.default_rng(2)
    for _ in range(100):
        L = _rand_state(rng)
        R = _rand_state(rng)
        L[1] = R[1] = 50.0
        bn = rng.normal()
        F, SL, SR, _ = oracle.hlld(L, R, bn, GAMMA)
        assert SL > 0
        np.testing.assert_array_equal(F, physical_flux(L, bn)[0])


def _mirror(s):
    rho, un, v, w, p, by, bz = s
    return np.array([rho, -un, v, w, p, by, bz])


@pytest.mark.parametrize("solver", ["hlld", "hll", "llf"])
def test_reflection_symmetry(solver):
    """x_n -> -x_n maps (L, R, b_n) to (mirror R, mirror L, -b_n), with
    mirror: u_n -> -u_n (b treated as a vector, so b_n -> -b_n).  The fluxes
    of rho, transverse momentum and e_tot change sign; the normal-momentum
    flux does not."""
    rng = np.random.default_rng(3)
    for _ in range(300):
        L, R = _rand_state(rng), _rand_state(rng)
        bn = rng.normal()
        if solver == "hlld":
            F1 = oracle.hlld(L, R, bn, GAMMA)[0]
            F2 = oracle.hlld(_mirror(R), _mirror(L), -bn, GAMMA)[0]
        elif solver == "hll":
            F1 = oracle.hll(L, R, bn, GAMMA)
            F2 = oracle.hll(_mirror(R), _mirror(L), -bn, GAMMA)
        else:
            F1 = oracle.llf(L, R, bn, GAMMA)[0]
            F2 = oracle.llf(_mirror(R), _mirror(L), -bn, GAMMA)[0]
        expect = np.array([-F1[0], F1[1], -F1[2], -F1[3], -F1[4]])
        np.testing.assert_allclose(F2, expect, rtol=1e-11, atol=1e-11 * np.abs(F1).max())


def test_hlld_stationary_contact_exact():
    """An isolated stationary contact (rho jump only, b_n != 0) is resolved
    exactly by HLLD: zero mass and energy flux, F_m = (p_T - b_n^2, -b_n b_t)."""
    bn, by, bz, p = 0.7, 0.3, -0.2, 1.0
    L = np.array([1.0, 0.0, 0.0, 0.0, p, by, bz])
    R = np.array([0.25, 0.0, 0.0, 0.0, p, by, bz])
    F, SL, SR, fb = oracle.hlld(L, R, bn, GAMMA)
    pt = p + 0.5 * (bn * bn + by * by + bz * bz)
    assert fb == 0
    np.testing.assert_allclose(F, [0.0, pt - bn * bn, -bn * by, -bn * bz, 0.0], atol=1e-14)
    # HLL smears the same contact: its mass flux is non-zero.
    assert abs(oracle.hll(L, R, bn, GAMMA)[0]) > 1e-3


@pytest.mark.parametrize("bn,direction", [(1.0, -1), (1.0, 1), (-0.8, -1), (-0.8, 1)])
def test_hlld_rotational_discontinuity_exact(bn, direction):
    """An isolated rotational (Alfven) discontinuity moving at -/+ c_An with
    u_n = 0: the Rankine-Hugoniot jump [v_t] = -direction sgn(b_n) [b_t]/sqrt(rho)
    makes the exact flux at x = 0 equal to F(U_R) (left-going) or F(U_L)
    (right-going).  HLLD must reproduce it through its double-star states."""
    rho, p = 1.3, 0.9
    phi = 1.0
    btL = np.array([0.6, 0.0])
    btR = 0.6 * np.array([math.cos(phi), math.sin(phi)])
    vtL = np.array([0.2, -0.1])
    vtR = vtL - direction * np.sign(bn) * (btR - btL) / math.sqrt(rho)
    L = np.array([rho, 0.0, vtL[0], vtL[1], p, btL[0], btL[1]])
    R = np.array([rho, 0.0, vtR[0], vtR[1], p, btR[0], btR[1]])
    FL, UL = physical_flux(L, bn)
    FR, UR = physical_flux(R, bn)
    lam = direction * abs(bn) / math.sqrt(rho)
    # the construction satisfies the jump condition lam [U] = [F]
    np.testing.assert_allclose(lam * (UR - UL), FR - FL, atol=1e-14)
    F, SL, SR, fb = oracle.hlld(L, R, bn, GAMMA)
    assert fb == 0
    exact = FR if direction < 0 else FL
    np.testing.assert_allclose(F, exact, atol=2e-14)


def test_hll_llf_relation():
    """With symmetric speeds S_R = -S_L = s, HLL equals LLF with the same s."""
    rng = np.random.default_rng(4)
    for _ in range(100):
        L, R = _rand_state(rng), _rand_state(rng)
        L[1] = R[1] = 0.0  # symmetric outer speeds need max|u| = min|u|
        bn = rng.normal()
        F_hll = oracle.hll(L, R, bn, GAMMA)
        F_llf, s = oracle.llf(L, R, bn, GAMMA)
        np.testing.assert_allclose(F_hll, F_llf, rtol=1e-12, atol=1e-13)


def test_hlld_bounded_by_hll_speeds():
    """alpha^{+/-} (eq. emf:alpha-pm) are the outer HLLD speeds."""
    rng = np.random.default_rng(5)
    for _ in range(50):
        L, R = _rand_state(rng), _rand_state(rng)
        bn = rng.normal()
        _, SL, SR, _ = oracle.hlld(L, R, bn, GAMMA)
        cf = max(oracle.fast_speed(L[0], L[4], bn, L[5], L[6], GAMMA),
                 oracle.fast_speed(R[0], R[4], bn, R[5], R[6], GAMMA))
        assert SL == min(L[1], R[1]) - cf
        assert SR == max(L[1], R[1]) + cf


def _mhd_flux7(st, bn, pt):
    """Physical flux of (rho, m_n, m_t1, m_t2, e_tot, b_t1, b_t2) for a state
    given as (rho, u_n, u_t1, u_t2, b_t1, b_t2, e_tot) with total pressure pt
    (eq. mhd:conservation-laws; induction flux u_n b_t - b_n u_t)."""
    rho, un, v, w, by, bz, e = st
    vb = un * bn + v * by + w * bz
    U = np.array([rho, rho * un, rho * v, rho * w, e, by, bz])
    F = np.array([rho * un, rho * un * un + pt - bn * bn, rho * un * v - bn * by,
                  rho * un * w - bn * bz, (e + pt) * un - bn * vb, un * by - bn * v,
                  un * bz - bn * w])
    return U, F


def test_hlld_fan_rankine_hugoniot():
    """Every wave of the HLLD fan satisfies the Rankine-Hugoniot conditions for
    all seven conserved quantities (mass, momentum, energy, transverse b):
    S [U] = [F] across S_L, S*_L, S_M, S*_R and S_R, with u_n = S_M and
    p_T = p_T* inside the fan.  These are the conditions the HLLD states are
    built from (Miyoshi & Kusano 2005)."""
    rng = np.random.default_rng(6)
    nchecked = 0
    for _ in range(400):
        L, R = _rand_state(rng), _rand_state(rng)
        bn = rng.normal()
        sp, st, fb = oracle.hlld_fan(L, R, bn, GAMMA)
        if fb or not (sp["SL"] < 0 < sp["SR"]):
            continue
        nchecked += 1
        # outer states in the same 7-vector form
        outer = []
        for s in (L, R):
            rho, un, v, w, p, by, bz = s
            e = p / (GAMMA - 1) + 0.5 * rho * (un * un + v * v + w * w) + 0.5 * (
                bn * bn + by * by + bz * bz)
            pt = p + 0.5 * (bn * bn + by * by + bz * bz)
            outer.append(_mhd_flux7((rho, un, v, w, by, bz, e), bn, pt))
        fan = [_mhd_flux7(st[q], bn, sp["pTs"]) for q in range(4)]
        chain = [outer[0]] + fan + [outer[1]]
        speeds = [sp["SL"], sp["SsL"], sp["SM"], sp["SsR"], sp["SR"]]
        for q, S in enumerate(speeds):
            (Ua, Fa), (Ub, Fb) = chain[q], chain[q + 1]
            scale = np.abs(Fa).max() + np.abs(Fb).max() + abs(S) * (np.abs(Ua).max() + np.abs(Ub).max())
            np.testing.assert_allclose(S * (Ub - Ua), Fb - Fa, atol=1e-12 * scale)
    assert nchecked > 200


# ------------------------------------------------------------ HLL fallback
def _hll_numpy(L, R, bn, SL, SR):
    """The HLL flux (Harten, Lax & van Leer) with given outer speeds, from
    the physical fluxes of the two states: F_L if S_L >= 0, F_R if S_R <= 0,
    else (S_R F_L - S_L F_R + S_L S_R (U_R - U_L)) / (S_R - S_L)."""
    FL, UL = physical_flux(L, bn)
    FR, UR = physical_flux(R, bn)
    if SL >= 0:
        return FL
    if SR <= 0:
        return FR
    return (SR * FL - SL * FR + SL * SR * (UR - UL)) / (SR - SL)


def _symmetric_rarefaction(rho, u, p, vt, bt, bn):
    """Left state moving at -u, right state at +u, equal transverse state."""
    L = np.array([rho, -u, vt[0], vt[1], p, bt[0], bt[1]])
    R = np.array([rho, u, vt[0], vt[1], p, bt[0], bt[1]])
    return L, R


@pytest.mark.parametrize("rho,p,vt,bt,bn", [
    (1.0, 0.01, (0.0, 0.0), (0.1, 0.0), 0.05),
    (0.3, 0.2, (0.4, -0.2), (0.5, -0.3), 0.8),
    (2.0, 1e-3, (0.0, 0.1), (0.0, 0.0), -0.3),
])
def test_hlld_symmetric_rarefaction_falls_back_at_closed_form_threshold(rho, p, vt, bt, bn):
    """Two equal states separating at -u and +u.  By symmetry S_M = 0 and the
    HLLD star total pressure (Miyoshi & Kusano 2005) reduces to
    p_T* = p_T - rho c u, with c the common fast speed (S_L = -u - c,
    S_R = u + c).  The fan is unphysical for u > p_T / (rho c): there HLLD
    must return the HLL flux with the same outer speeds and count a fallback;
    just below the threshold it must not fall back."""
    pt = p + 0.5 * (bn * bn + bt[0] ** 2 + bt[1] ** 2)
    c = oracle.fast_speed(rho, p, bn, bt[0], bt[1], GAMMA)
    u_star = pt / (rho * c)
    for u, expect_fb in ((0.97 * u_star, 0), (1.03 * u_star, 1), (5.0 * u_star, 1),
                         (50.0 * u_star, 1)):
        L, R = _symmetric_rarefaction(rho, u, p, vt, bt, bn)
        F, SL, SR, fb = oracle.hlld(L, R, bn, GAMMA)
        assert fb == expect_fb, (u / u_star, fb)
        assert SL == pytest.approx(-u - c, rel=1e-14) and SR == pytest.approx(u + c, rel=1e-14)
        if expect_fb:
            Fh = _hll_numpy(L, R, bn, SL, SR)
            np.testing.assert_allclose(F, Fh, rtol=1e-13, atol=1e-13 * np.abs(Fh).max())
            np.testing.assert_allclose(F, oracle.hll(L, R, bn, GAMMA), rtol=1e-13,
                                       atol=1e-13 * np.abs(Fh).max())
            # symmetric HLL: zero mass flux, energy flux -b_n (v_t . b_t),
            # normal momentum flux p_T - b_n^2 - rho u c (it can be negative)
            vb = vt[0] * bt[0] + vt[1] * bt[1]
            assert abs(F[0]) <= 1e-14 * rho * u
            assert F[4] == pytest.approx(-bn * vb, rel=1e-12, abs=1e-13 * np.abs(Fh).max())
            assert F[1] == pytest.approx(pt - bn * bn - rho * u * c, rel=1e-12,
                                         abs=1e-13 * pt)
        else:
            # below the threshold the HLLD flux differs from HLL (it resolves
            # the rotational and contact structure HLL smears)
            sp, st, _ = oracle.hlld_fan(L, R, bn, GAMMA)
            assert sp["pTs"] == pytest.approx(pt - rho * c * u, rel=1e-12)


def test_hlld_cold_dust_at_rest_falls_back():
    """p = 0, b = 0, u_n = 0 on both sides: every signal speed is zero, the
    star states are undefined (0/0), and the solver must fall back to HLL,
    whose S_L >= 0 branch returns the left physical flux (zero for dust at
    rest), and count the fallback."""
    L = np.array([1.0, 0.0, 0.3, -0.2, 0.0, 0.0, 0.0])
    R = np.array([2.5, 0.0, -0.1, 0.4, 0.0, 0.0, 0.0])
    F, SL, SR, fb = oracle.hlld(L, R, 0.0, GAMMA)
    assert fb == 1
    assert SL == 0.0 and SR == 0.0
    np.testing.assert_array_equal(F, physical_flux(L, 0.0)[0])


def test_hlld_fallback_flux_is_hll_in_strong_rarefactions():
    """Asymmetric strong rarefactions (random states pulled apart at several
    times their sound speed): whenever HLLD reports a fallback its flux is
    the HLL flux with the same outer speeds; and fallbacks do occur."""
    rng = np.random.default_rng(8)
    nfb = 0
    for _ in range(400):
        L, R = _rand_state(rng), _rand_state(rng)
        L[4] *= 1e-2
        R[4] *= 1e-2
        L[1] = -abs(L[1]) - rng.uniform(2.0, 20.0)
        R[1] = abs(R[1]) + rng.uniform(2.0, 20.0)
        bn = 0.3 * rng.normal()
        F, SL, SR, fb = oracle.hlld(L, R, bn, GAMMA)
        if fb:
            nfb += 1
            Fh = _hll_numpy(L, R, bn, SL, SR)
            np.testing.assert_allclose(F, Fh, rtol=1e-12, atol=1e-12 * np.abs(Fh).max())
    assert nfb > 100, nfb
