// ctmhd_adjoint_math.h -- reverse-mode (adjoint) arithmetic of the per-point
// pieces of the CT-MHD step: limited reconstruction, fast magnetosonic speed,
// ideal-MHD flux, LLF and HLLD Riemann fluxes with the face outputs alpha+,
// alpha- and u*, and LD04 averaging of Q26 corner EMFs.
//
// Every *_adj function recomputes the forward values of ctmhd_math.h with the
// same operations and adds to the adjoints of its inputs the product of the
// given output adjoints with the derivative taken on the branch the forward
// takes at these inputs (limiter case, min / max selections, HLLD region,
// degenerate star states, HLL fallback).  Adjoint arguments accumulate (+=).
#pragma once

#include <type_traits>

#include "ctmhd_math.h"

namespace ctmhd {

// ---------------------------------------------------------------------------
// Reconstruction (Sec. 2.2).  Partial derivatives of the full limited slope s
// of plm_slope<M>(qm, q0, qp) with respect to (qm, q0, qp).
// ---------------------------------------------------------------------------
template <int M, typename T>
CTMHD_HD void plm_slope_partials(T qm, T q0, T qp, T& dm, T& d0, T& dp) {
  const T dl = q0 - qm, dr = qp - q0;
  T gl = T(0), gr = T(0);  // ds/d(dl), ds/d(dr)
  if (dl * dr > T(0)) {
    if (M == kPLM_MC) {
      // s = sign * min(2|dl|, 2|dr|, |dl + dr| / 2); all three carry the sign
      // of dr when dl * dr > 0, so each candidate is linear in (dl, dr)
      const T a1 = T(2) * tabs(dl), a2 = T(2) * tabs(dr), a3 = T(0.5) * tabs(dl + dr);
      const T m12 = tmin(a1, a2);
      if (m12 <= a3) {
        if (a1 <= a2) gl = T(2); else gr = T(2);
      } else {
        gl = T(0.5);
        gr = T(0.5);
      }
    } else {
      if (tabs(dl) <= tabs(dr)) gl = T(1); else gr = T(1);
    }
  }
  dm = -gl;
  d0 = gl - gr;
  dp = gr;
}

// Adjoint of the lower / upper face values of the centre cell of (qm, q0, qp)
// (recon_cell for PC and PLM): adds to qmb, q0b, qpb.
template <int M, typename T>
CTMHD_HD void recon_cell_adj(T qm, T q0, T qp, T lob, T hib, T& qmb, T& q0b, T& qpb) {
  q0b += lob + hib;
  if constexpr (M == kPLM_MC || M == kPLM_MM) {
    T dm, d0, dp;
    plm_slope_partials<M>(qm, q0, qp, dm, d0, dp);
    const T sb = T(0.5) * (hib - lob);  // lo = q0 - s/2, hi = q0 + s/2
    qmb += sb * dm;
    q0b += sb * d0;
    qpb += sb * dp;
  } else {
    (void)qm;
    (void)qp;
    (void)qmb;
    (void)qpb;
  }
}

// Partial derivatives of the PPM limited slope ppm_slope(qm, q0, qp) with
// respect to (qm, q0, qp): the centred difference where it is the smaller
// candidate, else twice the smaller one-sided difference (Sec. 2.2).
template <typename T>
CTMHD_HD void ppm_slope_partials(T qm, T q0, T qp, T& dm, T& d0, T& dp) {
  const T dl = q0 - qm, dr = qp - q0, dc = T(0.5) * (qp - qm);
  dm = d0 = dp = T(0);
  if (dl * dr > T(0)) {
    // dl, dr and dc share one sign, so each candidate is linear in the values
    if (tabs(dc) <= T(2) * tmin(tabs(dl), tabs(dr))) {
      dm = T(-0.5);
      dp = T(0.5);
    } else if (tabs(dl) <= tabs(dr)) {  // s = 2 dl
      dm = T(-2);
      d0 = T(2);
    } else {  // s = 2 dr
      d0 = T(-2);
      dp = T(2);
    }
  }
}

// Adjoint of the PPM face values of the centre cell of q[0..4] (recon_cell):
// interface values from the limited slopes of the three middle cells, then
// the Colella-Woodward constraints in the branch the forward takes.
template <typename T>
CTMHD_HD void ppm_cell_adj(const T q[5], T lob, T hib, T qb[5]) {
  const T sixth = T(1) / T(6);
  const T d1 = ppm_slope(q[0], q[1], q[2]);
  const T d2 = ppm_slope(q[1], q[2], q[3]);
  const T d3 = ppm_slope(q[2], q[3], q[4]);
  const T qL = ppm_iface(q[1], q[2], d1, d2);
  const T qR = ppm_iface(q[2], q[3], d2, d3);
  T qLb = T(0), qRb = T(0);  // adjoints of the unconstrained interface values
  if ((qR - q[2]) * (q[2] - qL) <= T(0)) {
    qb[2] += lob + hib;  // local extremum: both values set to the centre
  } else {
    const T dq = qR - qL;
    const T q6 = dq * (q[2] - T(0.5) * (qL + qR));
    const T d6 = dq * dq * sixth;
    if (q6 > d6) {  // lower value reset to 3 q0 - 2 qR
      qb[2] += T(3) * lob;
      qRb += hib - T(2) * lob;
    } else if (-d6 > q6) {  // upper value reset to 3 q0 - 2 qL
      qb[2] += T(3) * hib;
      qLb += lob - T(2) * hib;
    } else {
      qLb += lob;
      qRb += hib;
    }
  }
  // qL = (q1 + q2)/2 - (d2 - d1)/6, qR = (q2 + q3)/2 - (d3 - d2)/6
  qb[1] += T(0.5) * qLb;
  qb[2] += T(0.5) * (qLb + qRb);
  qb[3] += T(0.5) * qRb;
  const T db[3] = {qLb * sixth, (qRb - qLb) * sixth, -qRb * sixth};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    T pm, p0, pp;
    ppm_slope_partials(q[j], q[j + 1], q[j + 2], pm, p0, pp);
    qb[j] += db[j] * pm;
    qb[j + 1] += db[j] * p0;
    qb[j + 2] += db[j] * pp;
  }
}

// Adjoint of the lower / upper face values of the centre cell of q[0..4]
// (recon_cell, any scheme): adds to qb[0..4].
template <int M, typename T>
CTMHD_HD void recon_cell_adj5(const T q[5], T lob, T hib, T qb[5]) {
  if constexpr (M == kPPM)
    ppm_cell_adj(q, lob, hib, qb);
  else
    recon_cell_adj<M>(q[1], q[2], q[3], lob, hib, qb[1], qb[2], qb[3]);
}

// ---------------------------------------------------------------------------
// Fast magnetosonic speed (eq. waves:fast-speed).
// ---------------------------------------------------------------------------
template <typename T>
CTMHD_HD void fast_speed_adj(T rho, T p, T bn, T bt1, T bt2, T gamma, T cb, T& rhob, T& pb,
                             T& bnb, T& bt1b, T& bt2b) {
  const T irho = trcp(rho);
  const T gp = gamma * p;
  const T tot = gp + bn * bn + bt1 * bt1 + bt2 * bt2;
  const T a = tot * irho;
  T disc = a * a - T(4) * gp * bn * bn * irho * irho;
  const bool pos = disc > T(0);
  disc = pos ? disc : T(0);
  const T sd = tsqrt(disc);
  const T h = T(0.5) * (a + sd);
  const T cf = tsqrt(h);
  // cf = sqrt(h), h = (a + sd) / 2, sd = sqrt(disc)
  const T hb = cb / (T(2) * cf);
  T ab = T(0.5) * hb;
  const T sdb = T(0.5) * hb;
  const T discb = pos ? sdb / (T(2) * sd) : T(0);
  // disc = a^2 - 4 gp bn^2 irho^2
  ab += T(2) * a * discb;
  T gpb = -T(4) * bn * bn * irho * irho * discb;
  bnb += -T(8) * gp * bn * irho * irho * discb;
  T irhob = -T(8) * gp * bn * bn * irho * discb;
  // a = tot * irho
  const T totb = ab * irho;
  irhob += ab * tot;
  gpb += totb;
  bnb += T(2) * bn * totb;
  bt1b += T(2) * bt1 * totb;
  bt2b += T(2) * bt2 * totb;
  rhob += -irho * irho * irhob;
  pb += gamma * gpb;
}

// ---------------------------------------------------------------------------
// Ideal-MHD conserved state and normal flux (phys_flux).
// ---------------------------------------------------------------------------
template <typename T>
CTMHD_HD void phys_flux_adj(const FState<T>& s, T bn, T gm1inv, const T Ub[5], const T Fb[5],
                            T pTb, FState<T>& sb, T& bnb) {
  const T b2 = bn * bn + s.bt1 * s.bt1 + s.bt2 * s.bt2;
  const T v2 = s.un * s.un + s.ut1 * s.ut1 + s.ut2 * s.ut2;
  const T e = s.p * gm1inv + T(0.5) * (s.rho * v2 + b2);
  const T pT = s.p + T(0.5) * b2;
  const T vb = s.un * bn + s.ut1 * s.bt1 + s.ut2 * s.bt2;
  const T mn = s.rho * s.un;
  T eb = Ub[4], mnb = Ub[1] + Fb[0], vbb = T(0), b2b = T(0), v2b = T(0);
  // F4 = (e + pT) un - bn vb
  eb += Fb[4] * s.un;
  pTb += Fb[4] * s.un;
  sb.un += Fb[4] * (e + pT);
  bnb -= Fb[4] * vb;
  vbb -= Fb[4] * bn;
  // F3 = mn ut2 - bn bt2, F2 = mn ut1 - bn bt1
  mnb += Fb[3] * s.ut2 + Fb[2] * s.ut1;
  sb.ut2 += Fb[3] * mn;
  sb.ut1 += Fb[2] * mn;
  bnb -= Fb[3] * s.bt2 + Fb[2] * s.bt1;
  sb.bt2 -= Fb[3] * bn;
  sb.bt1 -= Fb[2] * bn;
  // F1 = mn un + pT - bn^2
  mnb += Fb[1] * s.un;
  sb.un += Fb[1] * mn;
  pTb += Fb[1];
  bnb -= T(2) * bn * Fb[1];
  // U = (rho, mn, rho ut1, rho ut2, e)
  sb.rho += Ub[0] + Ub[2] * s.ut1 + Ub[3] * s.ut2;
  sb.ut1 += Ub[2] * s.rho;
  sb.ut2 += Ub[3] * s.rho;
  // mn = rho un
  sb.rho += mnb * s.un;
  sb.un += mnb * s.rho;
  // vb = un bn + ut1 bt1 + ut2 bt2
  sb.un += vbb * bn;
  bnb += vbb * s.un;
  sb.ut1 += vbb * s.bt1;
  sb.bt1 += vbb * s.ut1;
  sb.ut2 += vbb * s.bt2;
  sb.bt2 += vbb * s.ut2;
  // pT = p + b2 / 2, e = p gm1inv + (rho v2 + b2) / 2
  sb.p += pTb + eb * gm1inv;
  b2b += T(0.5) * pTb + T(0.5) * eb;
  sb.rho += T(0.5) * eb * v2;
  v2b += T(0.5) * eb * s.rho;
  sb.un += T(2) * s.un * v2b;
  sb.ut1 += T(2) * s.ut1 * v2b;
  sb.ut2 += T(2) * s.ut2 * v2b;
  bnb += T(2) * bn * b2b;
  sb.bt1 += T(2) * s.bt1 * b2b;
  sb.bt2 += T(2) * s.bt2 * b2b;
}

template <typename T>
CTMHD_HD void fstate_zero(FState<T>& s) {
  s.rho = s.un = s.ut1 = s.ut2 = s.p = s.bt1 = s.bt2 = T(0);
}

// d = s where c (per lane), d unchanged elsewhere.
template <typename T>
CTMHD_HD void fstate_select(bool c, const FState<T>& s, FState<T>& d) {
  d.rho = c ? s.rho : d.rho;
  d.un = c ? s.un : d.un;
  d.ut1 = c ? s.ut1 : d.ut1;
  d.ut2 = c ? s.ut2 : d.ut2;
  d.p = c ? s.p : d.p;
  d.bt1 = c ? s.bt1 : d.bt1;
  d.bt2 = c ? s.bt2 : d.bt2;
}

// ---------------------------------------------------------------------------
// LLF flux (llf_flux): adjoint of F[5] and of the returned signal speed s.
// ---------------------------------------------------------------------------
template <typename T>
CTMHD_HD void llf_flux_adj(const FState<T>& L, const FState<T>& R, T bn, T gamma, const T Fb[5],
                           T sbar, FState<T>& Lb, FState<T>& Rb, T& bnb) {
  const T gm1inv = T(1) / (gamma - T(1));
  T UL[5], FL[5], UR[5], FR[5], pL, pR;
  phys_flux(L, bn, gm1inv, UL, FL, pL);
  phys_flux(R, bn, gm1inv, UR, FR, pR);
  const T cL = fast_speed(L.rho, L.p, bn, L.bt1, L.bt2, gamma);
  const T cR = fast_speed(R.rho, R.p, bn, R.bt1, R.bt2, gamma);
  const T xL = tabs(L.un) + cL, xR = tabs(R.un) + cR;
  const T s = tmax(xL, xR);
  T ULb[5], FLb[5], URb[5], FRb[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    // F = (FL + FR) / 2 - s (UR - UL) / 2
    FLb[m] = T(0.5) * Fb[m];
    FRb[m] = T(0.5) * Fb[m];
    URb[m] = -T(0.5) * s * Fb[m];
    ULb[m] = T(0.5) * s * Fb[m];
    sbar -= T(0.5) * Fb[m] * (UR[m] - UL[m]);
  }
  const bool left = xL >= xR;
  const T xLb = left ? sbar : T(0), xRb = left ? T(0) : sbar;
  // |un|: the derivative of x < 0 ? -x : x (+1 at zero)
  Lb.un += (L.un < T(0) ? T(-1) : T(1)) * xLb;
  Rb.un += (R.un < T(0) ? T(-1) : T(1)) * xRb;
  fast_speed_adj(L.rho, L.p, bn, L.bt1, L.bt2, gamma, xLb, Lb.rho, Lb.p, bnb, Lb.bt1, Lb.bt2);
  fast_speed_adj(R.rho, R.p, bn, R.bt1, R.bt2, gamma, xRb, Rb.rho, Rb.p, bnb, Rb.bt1, Rb.bt2);
  phys_flux_adj(L, bn, gm1inv, ULb, FLb, T(0), Lb, bnb);
  phys_flux_adj(R, bn, gm1inv, URb, FRb, T(0), Rb, bnb);
}

// Adds the adjoint of the ideal-MHD flux F of side K (K = L where left, R
// elsewhere; one path, chosen per lane) onto that side's state adjoint.
template <typename T>
CTMHD_HD void side_flux_adj(bool left, const FState<T>& L, const FState<T>& R, T bn, T gm1inv,
                            const T Ub[5], const T Fb[5], FState<T>& Lb, FState<T>& Rb, T& bnb) {
  const FState<T> K{left ? L.rho : R.rho, left ? L.un : R.un,   left ? L.ut1 : R.ut1,
                    left ? L.ut2 : R.ut2, left ? L.p : R.p,     left ? L.bt1 : R.bt1,
                    left ? L.bt2 : R.bt2};
  FState<T> Kb{left ? Lb.rho : Rb.rho, left ? Lb.un : Rb.un,   left ? Lb.ut1 : Rb.ut1,
               left ? Lb.ut2 : Rb.ut2, left ? Lb.p : Rb.p,     left ? Lb.bt1 : Rb.bt1,
               left ? Lb.bt2 : Rb.bt2};
  phys_flux_adj(K, bn, gm1inv, Ub, Fb, T(0), Kb, bnb);
  fstate_select(left, Kb, Lb);
  fstate_select(!left, Kb, Rb);
}

// x unchanged, as a value the compiler cannot trace to its computation: a
// forward value formed again from such copies is not merged with the first
// computation (whose register would then stay live until this use).
template <typename T>
CTMHD_HD T opaque(T x) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(x));
#endif
  return x;
}
template <typename T>
CTMHD_HD FState<T> opaque(const FState<T>& s) {
  return FState<T>{opaque(s.rho), opaque(s.un), opaque(s.ut1), opaque(s.ut2),
                   opaque(s.p),   opaque(s.bt1), opaque(s.bt2)};
}

// ---------------------------------------------------------------------------
// HLLD flux (hlld_flux): adjoint of F[5] and of the outer speeds SL, SR.
// ---------------------------------------------------------------------------
template <typename T>
CTMHD_HD void hlld_flux_adj(const FState<T>& L, const FState<T>& R, T bn, T gamma, const T Fb[5],
                            T SLbar, T SRbar, FState<T>& Lb, FState<T>& Rb, T& bnb) {
  const T gm1inv = T(1) / (gamma - T(1));
  // The outer conserved states and fluxes (phys_flux) are formed where the
  // reverse reads them rather than kept live across the fan; the fan needs
  // only their total pressures and energies.  Their adjoints go through
  // phys_flux_adj as soon as they are complete (it is linear in them).
  T pTL, pTR, eL, eR;
  {
    T U[5], F[5];
    phys_flux(L, bn, gm1inv, U, F, pTL);
    eL = U[4];
    phys_flux(R, bn, gm1inv, U, F, pTR);
    eR = U[4];
  }
  const T cfL = fast_speed(L.rho, L.p, bn, L.bt1, L.bt2, gamma);
  const T cfR = fast_speed(R.rho, R.p, bn, R.bt1, R.bt2, gamma);
  const T cmax = tmax(cfL, cfR);
  const T SL = tmin(L.un, R.un) - cmax;
  const T SR = tmax(L.un, R.un) + cmax;
  T pTLb = T(0), pTRb = T(0), eLb = T(0), eRb = T(0);
  const T zero5[5] = {T(0), T(0), T(0), T(0), T(0)};

  if (SL > T(0) || SR < T(0)) {
    side_flux_adj(SL > T(0), L, R, bn, gm1inv, zero5, Fb, Lb, Rb, bnb);
  } else {
    // ---- forward of the fan (same operations as hlld_flux) ----
    const T bn2 = bn * bn;
    const T dL = SL - L.un, dR = SR - R.un;
    const T mL = dL * L.rho, mR = dR * R.rho;
    const T iden = trcp(mR - mL);
    const T NS = mR * R.un - mL * L.un - pTR + pTL;
    const T SM = NS * iden;
    const T NP = mR * pTL - mL * pTR + mL * mR * (R.un - L.un);
    const T pTs = NP * iden;
    const T dsL = SL - SM, dsR = SR - SM;
    const T idsL = trcp(dsL), idsR = trcp(dsR);
    const T rsL = mL * idsL, rsR = mR * idsR;
    T vsL, wsL, bysL, bzsL, vsR, wsR, bysR, bzsR;
    T qL, iqL, fvL, fbL, qR, iqR, fvR, fbR;
    bool degL, degR;
    {
      qL = mL * dsL - bn2;
      degL = tabs(qL) <= T(1e-12) * (tabs(mL * dsL) + bn2);
      iqL = trcp(qL);
      fvL = bn * (SM - L.un) * iqL;
      fbL = (mL * dL - bn2) * iqL;
      vsL = degL ? L.ut1 : L.ut1 - L.bt1 * fvL;
      wsL = degL ? L.ut2 : L.ut2 - L.bt2 * fvL;
      bysL = degL ? L.bt1 : L.bt1 * fbL;
      bzsL = degL ? L.bt2 : L.bt2 * fbL;
    }
    {
      qR = mR * dsR - bn2;
      degR = tabs(qR) <= T(1e-12) * (tabs(mR * dsR) + bn2);
      iqR = trcp(qR);
      fvR = bn * (SM - R.un) * iqR;
      fbR = (mR * dR - bn2) * iqR;
      vsR = degR ? R.ut1 : R.ut1 - R.bt1 * fvR;
      wsR = degR ? R.ut2 : R.ut2 - R.bt2 * fvR;
      bysR = degR ? R.bt1 : R.bt1 * fbR;
      bzsR = degR ? R.bt2 : R.bt2 * fbR;
    }
    const T vbL = L.un * bn + L.ut1 * L.bt1 + L.ut2 * L.bt2;
    const T vbR = R.un * bn + R.ut1 * R.bt1 + R.ut2 * R.bt2;
    const T vbsL = SM * bn + vsL * bysL + wsL * bzsL;
    const T vbsR = SM * bn + vsR * bysR + wsR * bzsR;
    const T NeL = dL * eL - pTL * L.un + pTs * SM + bn * (vbL - vbsL);
    const T NeR = dR * eR - pTR * R.un + pTs * SM + bn * (vbR - vbsR);
    const T esL = NeL * idsL, esR = NeR * idsR;
    const bool bad = !(rsL > T(0)) || !(rsR > T(0)) || !(pTs > T(0)) || !(SL < SM) ||
                     !(SM < SR) || !tfinite(SM) || !tfinite(vsL + wsL + bysL + bzsL + esL) ||
                     !tfinite(vsR + wsR + bysR + bzsR + esR);
    if (bad) {
      if (SL >= T(0) || SR <= T(0)) {
        side_flux_adj(SL >= T(0), L, R, bn, gm1inv, zero5, Fb, Lb, Rb, bnb);
      } else {
        // F = (SR FL - SL FR + SL SR (UR - UL)) / (SR - SL)
        T UL[5], FL[5], UR[5], FR[5], pd;
        phys_flux(L, bn, gm1inv, UL, FL, pd);
        phys_flux(R, bn, gm1inv, UR, FR, pd);
        const T iw = trcp(SR - SL);
        T ULb[5], FLb[5], URb[5], FRb[5];
#pragma unroll
        for (int m = 0; m < 5; ++m) {
          const T N = SR * FL[m] - SL * FR[m] + SL * SR * (UR[m] - UL[m]);
          FLb[m] = Fb[m] * SR * iw;
          FRb[m] = -Fb[m] * SL * iw;
          URb[m] = Fb[m] * SL * SR * iw;
          ULb[m] = -Fb[m] * SL * SR * iw;
          SRbar += Fb[m] * (FL[m] + SL * (UR[m] - UL[m])) * iw - Fb[m] * N * iw * iw;
          SLbar += Fb[m] * (-FR[m] + SR * (UR[m] - UL[m])) * iw + Fb[m] * N * iw * iw;
        }
        phys_flux_adj(L, bn, gm1inv, ULb, FLb, T(0), Lb, bnb);
        phys_flux_adj(R, bn, gm1inv, URb, FRb, T(0), Rb, bnb);
      }
    } else {
      T SsL = SM, SsR = SM;
      const bool dstar = !(bn2 <= T(1e-12) * pTs);
      T sg = T(0), sqL = T(0), sqR = T(0), abn = T(0), isum = T(0);
      T vss = T(0), wss = T(0), byss = T(0), bzss = T(0), vbss = T(0);
      T Nv = T(0), Nw = T(0), Nby = T(0), Nbz = T(0);
      if (dstar) {
        sg = bn > T(0) ? T(1) : (bn < T(0) ? T(-1) : T(0));
        const T yL = trsqrt(rsL), yR = trsqrt(rsR);
        sqL = rsL * yL;
        sqR = rsR * yR;
        abn = tabs(bn);
        SsL = SM - abn * yL;
        SsR = SM + abn * yR;
        isum = trcp(sqL + sqR);
        Nv = sqL * vsL + sqR * vsR + (bysR - bysL) * sg;
        Nw = sqL * wsL + sqR * wsR + (bzsR - bzsL) * sg;
        Nby = sqL * bysR + sqR * bysL + sqL * sqR * (vsR - vsL) * sg;
        Nbz = sqL * bzsR + sqR * bzsL + sqL * sqR * (wsR - wsL) * sg;
        vss = Nv * isum;
        wss = Nw * isum;
        byss = Nby * isum;
        bzss = Nbz * isum;
        vbss = SM * bn + vss * byss + wss * bzss;
      }
      // ---- reverse ----
      T UsLb[5], UsRb[5], UssLb[5], UssRb[5];
#pragma unroll
      for (int m = 0; m < 5; ++m) UsLb[m] = UsRb[m] = UssLb[m] = UssRb[m] = T(0);
      T SsLb = T(0), SsRb = T(0);
      // The flux is taken from one side K: F = FK + SK (UsK - UK), plus
      // SsK (UssK - UsK) in the inner regions.  The outer, star and
      // double-star conserved states of K are formed here, where the reverse
      // reads them, instead of being kept live across the fan.
      auto side = [&](auto left_tag, bool inner) {
        constexpr bool LEFT = decltype(left_tag)::value;
        const FState<T>& K = LEFT ? L : R;
        const T SK = LEFT ? SL : SR, SsK = LEFT ? SsL : SsR;
        const T rs = LEFT ? rsL : rsR, vs = LEFT ? vsL : vsR, ws = LEFT ? wsL : wsR;
        const T es = LEFT ? esL : esR;
        T UK[5], FK[5], pd;
        phys_flux(K, bn, gm1inv, UK, FK, pd);
        const T Us[5] = {rs, rs * SM, rs * vs, rs * ws, es};
        T Uss[5] = {Us[0], Us[1], Us[2], Us[3], Us[4]};
        if (dstar) {
          Uss[2] = rs * vss;
          Uss[3] = rs * wss;
          Uss[4] = LEFT ? esL - sqL * (vbsL - vbss) * sg : esR + sqR * (vbsR - vbss) * sg;
        }
        T SKbar = T(0), SsKb = T(0);
#pragma unroll
        for (int m = 0; m < 5; ++m) {
          SKbar += Fb[m] * (Us[m] - UK[m]);
          if (inner) {
            (LEFT ? UsLb : UsRb)[m] += Fb[m] * (SK - SsK);
            SsKb += Fb[m] * (Uss[m] - Us[m]);
            (LEFT ? UssLb : UssRb)[m] += Fb[m] * SsK;
          } else {
            (LEFT ? UsLb : UsRb)[m] += Fb[m] * SK;
          }
        }
        if constexpr (LEFT) {
          SLbar += SKbar;
          SsLb += SsKb;
        } else {
          SRbar += SKbar;
          SsRb += SsKb;
        }
      };
      // the side whose flux and conserved state F takes (FK - SK UK); their
      // adjoints go onto that side's state at the end of the reverse
      const bool left = SsL >= T(0) || SM >= T(0);
      if (SsL >= T(0))
        side(std::integral_constant<bool, true>(), false);
      else if (SM >= T(0))
        side(std::integral_constant<bool, true>(), true);
      else if (SsR >= T(0))
        side(std::integral_constant<bool, false>(), true);
      else
        side(std::integral_constant<bool, false>(), false);
      T SMb = T(0), rsLb = T(0), rsRb = T(0), esLb = T(0), esRb = T(0);
      T vsLb = T(0), wsLb = T(0), bysLb = T(0), bzsLb = T(0);
      T vsRb = T(0), wsRb = T(0), bysRb = T(0), bzsRb = T(0);
      T vbsLb = T(0), vbsRb = T(0);
      if (dstar) {
        T sqLb = T(0), sqRb = T(0), abnb = T(0), isumb = T(0);
        T vssb = T(0), wssb = T(0), byssb = T(0), bzssb = T(0), vbssb = T(0);
        // SsL = SM - abn / sqL, SsR = SM + abn / sqR
        SMb += SsLb + SsRb;
        abnb += -SsLb / sqL + SsRb / sqR;
        sqLb += SsLb * abn / (sqL * sqL);
        sqRb -= SsRb * abn / (sqR * sqR);
        // UssL = (rsL, rsL SM, rsL vss, rsL wss, esL - sqL (vbsL - vbss) sg)
        rsLb += UssLb[0] + UssLb[1] * SM + UssLb[2] * vss + UssLb[3] * wss;
        SMb += UssLb[1] * rsL;
        vssb += UssLb[2] * rsL;
        wssb += UssLb[3] * rsL;
        esLb += UssLb[4];
        sqLb -= UssLb[4] * (vbsL - vbss) * sg;
        vbsLb -= UssLb[4] * sqL * sg;
        vbssb += UssLb[4] * sqL * sg;
        // UssR = (rsR, rsR SM, rsR vss, rsR wss, esR + sqR (vbsR - vbss) sg)
        rsRb += UssRb[0] + UssRb[1] * SM + UssRb[2] * vss + UssRb[3] * wss;
        SMb += UssRb[1] * rsR;
        vssb += UssRb[2] * rsR;
        wssb += UssRb[3] * rsR;
        esRb += UssRb[4];
        sqRb += UssRb[4] * (vbsR - vbss) * sg;
        vbsRb += UssRb[4] * sqR * sg;
        vbssb -= UssRb[4] * sqR * sg;
        // vbss = SM bn + vss byss + wss bzss
        SMb += vbssb * bn;
        bnb += vbssb * SM;
        vssb += vbssb * byss;
        byssb += vbssb * vss;
        wssb += vbssb * bzss;
        bzssb += vbssb * wss;
        // vss = Nv isum, wss = Nw isum
        isumb += vssb * Nv + wssb * Nw + byssb * Nby + bzssb * Nbz;
        const T vb_ = vssb * isum, wb_ = wssb * isum, byb_ = byssb * isum, bzb_ = bzssb * isum;
        sqLb += vb_ * vsL + wb_ * wsL;
        sqRb += vb_ * vsR + wb_ * wsR;
        vsLb += vb_ * sqL;
        vsRb += vb_ * sqR;
        wsLb += wb_ * sqL;
        wsRb += wb_ * sqR;
        bysRb += vb_ * sg;
        bysLb -= vb_ * sg;
        bzsRb += wb_ * sg;
        bzsLb -= wb_ * sg;
        // byss = (sqL bysR + sqR bysL + sqL sqR (vsR - vsL) sg) isum
        sqLb += byb_ * (bysR + sqR * (vsR - vsL) * sg);
        sqRb += byb_ * (bysL + sqL * (vsR - vsL) * sg);
        bysRb += byb_ * sqL;
        bysLb += byb_ * sqR;
        vsRb += byb_ * sqL * sqR * sg;
        vsLb -= byb_ * sqL * sqR * sg;
        // bzss = (sqL bzsR + sqR bzsL + sqL sqR (wsR - wsL) sg) isum
        sqLb += bzb_ * (bzsR + sqR * (wsR - wsL) * sg);
        sqRb += bzb_ * (bzsL + sqL * (wsR - wsL) * sg);
        bzsRb += bzb_ * sqL;
        bzsLb += bzb_ * sqR;
        wsRb += bzb_ * sqL * sqR * sg;
        wsLb -= bzb_ * sqL * sqR * sg;
        // isum = 1 / (sqL + sqR)
        sqLb -= isumb * isum * isum;
        sqRb -= isumb * isum * isum;
        // sq = sqrt(rs), abn = |bn|
        rsLb += sqLb / (T(2) * sqL);
        rsRb += sqRb / (T(2) * sqR);
        bnb += abnb * sg;
      } else {
        SMb += SsLb + SsRb;
#pragma unroll
        for (int m = 0; m < 5; ++m) {
          UsLb[m] += UssLb[m];
          UsRb[m] += UssRb[m];
        }
      }
      // UsL = (rsL, rsL SM, rsL vsL, rsL wsL, esL)
      rsLb += UsLb[0] + UsLb[1] * SM + UsLb[2] * vsL + UsLb[3] * wsL;
      SMb += UsLb[1] * rsL;
      vsLb += UsLb[2] * rsL;
      wsLb += UsLb[3] * rsL;
      esLb += UsLb[4];
      rsRb += UsRb[0] + UsRb[1] * SM + UsRb[2] * vsR + UsRb[3] * wsR;
      SMb += UsRb[1] * rsR;
      vsRb += UsRb[2] * rsR;
      wsRb += UsRb[3] * rsR;
      esRb += UsRb[4];
      // The forward values of the fan that the rest of the reverse reads are
      // formed again here (the same operations on the same values), from
      // copies the compiler cannot trace, instead of being held in registers
      // across the reverse.
      const FState<T> Lo = opaque(L), Ro = opaque(R);
      const T bno = opaque(bn), SLo = opaque(SL), SRo = opaque(SR), SMo = opaque(SM);
      T pTL, pTR, eL, eR;
      {
        T U[5], F[5];
        phys_flux(Lo, bno, gm1inv, U, F, pTL);
        eL = U[4];
        phys_flux(Ro, bno, gm1inv, U, F, pTR);
        eR = U[4];
      }
      const T bn2r = bno * bno;
      const T dL = SLo - Lo.un, dR = SRo - Ro.un;
      const T mL = dL * Lo.rho, mR = dR * Ro.rho;
      const T iden = trcp(mR - mL);
      const T NS = mR * Ro.un - mL * Lo.un - pTR + pTL;
      const T NP = mR * pTL - mL * pTR + mL * mR * (Ro.un - Lo.un);
      const T pTs = NP * iden;
      const T dsL = SLo - SMo, dsR = SRo - SMo;
      const T idsL = trcp(dsL), idsR = trcp(dsR);
      const T iqL = trcp(mL * dsL - bn2r), iqR = trcp(mR * dsR - bn2r);
      const T fvL = bno * (SMo - Lo.un) * iqL, fbL = (mL * dL - bn2r) * iqL;
      const T fvR = bno * (SMo - Ro.un) * iqR, fbR = (mR * dR - bn2r) * iqR;
      const T vbL = Lo.un * bno + Lo.ut1 * Lo.bt1 + Lo.ut2 * Lo.bt2;
      const T vbR = Ro.un * bno + Ro.ut1 * Ro.bt1 + Ro.ut2 * Ro.bt2;
      const T vbsL = SMo * bno + opaque(vsL) * opaque(bysL) + opaque(wsL) * opaque(bzsL);
      const T vbsR = SMo * bno + opaque(vsR) * opaque(bysR) + opaque(wsR) * opaque(bzsR);
      const T NeL = dL * eL - pTL * Lo.un + pTs * SMo + bno * (vbL - vbsL);
      const T NeR = dR * eR - pTR * Ro.un + pTs * SMo + bno * (vbR - vbsR);
      // esL = NeL idsL, NeL = dL UL4 - pTL unL + pTs SM + bn (vbL - vbsL)
      T dLb = T(0), dRb = T(0), pTsb = T(0), idsLb = T(0), idsRb = T(0), vbLb = T(0), vbRb = T(0);
      {
        const T g = esLb * idsL;
        dLb += g * eL;
        eLb += g * dL;
        pTLb -= g * L.un;
        Lb.un -= g * pTL;
        pTsb += g * SM;
        SMb += g * pTs;
        bnb += g * (vbL - vbsL);
        vbLb += g * bn;
        vbsLb -= g * bn;
        idsLb += esLb * NeL;
      }
      {
        const T g = esRb * idsR;
        dRb += g * eR;
        eRb += g * dR;
        pTRb -= g * R.un;
        Rb.un -= g * pTR;
        pTsb += g * SM;
        SMb += g * pTs;
        bnb += g * (vbR - vbsR);
        vbRb += g * bn;
        vbsRb -= g * bn;
        idsRb += esRb * NeR;
      }
      // vbs = SM bn + vs bys + ws bzs
      SMb += (vbsLb + vbsRb) * bn;
      bnb += (vbsLb + vbsRb) * SM;
      vsLb += vbsLb * bysL;
      bysLb += vbsLb * vsL;
      wsLb += vbsLb * bzsL;
      bzsLb += vbsLb * wsL;
      vsRb += vbsRb * bysR;
      bysRb += vbsRb * vsR;
      wsRb += vbsRb * bzsR;
      bzsRb += vbsRb * wsR;
      // vb = un bn + ut1 bt1 + ut2 bt2
      Lb.un += vbLb * bn;
      Lb.ut1 += vbLb * L.bt1;
      Lb.bt1 += vbLb * L.ut1;
      Lb.ut2 += vbLb * L.bt2;
      Lb.bt2 += vbLb * L.ut2;
      Rb.un += vbRb * bn;
      Rb.ut1 += vbRb * R.bt1;
      Rb.bt1 += vbRb * R.ut1;
      Rb.ut2 += vbRb * R.bt2;
      Rb.bt2 += vbRb * R.ut2;
      bnb += vbLb * L.un + vbRb * R.un;
      // star transverse states
      T mLb = T(0), mRb = T(0), dsLb = T(0), dsRb = T(0), bn2b = T(0);
      if (degL) {
        Lb.ut1 += vsLb;
        Lb.ut2 += wsLb;
        Lb.bt1 += bysLb;
        Lb.bt2 += bzsLb;
      } else {
        Lb.ut1 += vsLb;
        Lb.ut2 += wsLb;
        Lb.bt1 += -vsLb * fvL + bysLb * fbL;
        Lb.bt2 += -wsLb * fvL + bzsLb * fbL;
        const T fvLb = -vsLb * L.bt1 - wsLb * L.bt2;
        const T fbLb = bysLb * L.bt1 + bzsLb * L.bt2;
        // fv = bn (SM - un) iq, fb = (m d - bn^2) iq
        bnb += fvLb * (SM - L.un) * iqL;
        SMb += fvLb * bn * iqL;
        Lb.un -= fvLb * bn * iqL;
        T iqLb = fvLb * bn * (SM - L.un) + fbLb * (mL * dL - bn2);
        mLb += fbLb * dL * iqL;
        dLb += fbLb * mL * iqL;
        bn2b -= fbLb * iqL;
        const T qLb = -iqLb * iqL * iqL;  // q = m ds - bn^2
        mLb += qLb * dsL;
        dsLb += qLb * mL;
        bn2b -= qLb;
      }
      if (degR) {
        Rb.ut1 += vsRb;
        Rb.ut2 += wsRb;
        Rb.bt1 += bysRb;
        Rb.bt2 += bzsRb;
      } else {
        Rb.ut1 += vsRb;
        Rb.ut2 += wsRb;
        Rb.bt1 += -vsRb * fvR + bysRb * fbR;
        Rb.bt2 += -wsRb * fvR + bzsRb * fbR;
        const T fvRb = -vsRb * R.bt1 - wsRb * R.bt2;
        const T fbRb = bysRb * R.bt1 + bzsRb * R.bt2;
        bnb += fvRb * (SM - R.un) * iqR;
        SMb += fvRb * bn * iqR;
        Rb.un -= fvRb * bn * iqR;
        T iqRb = fvRb * bn * (SM - R.un) + fbRb * (mR * dR - bn2);
        mRb += fbRb * dR * iqR;
        dRb += fbRb * mR * iqR;
        bn2b -= fbRb * iqR;
        const T qRb = -iqRb * iqR * iqR;
        mRb += qRb * dsR;
        dsRb += qRb * mR;
        bn2b -= qRb;
      }
      // rs = m ids, ids = 1 / ds, ds = S - SM
      mLb += rsLb * idsL;
      idsLb += rsLb * mL;
      mRb += rsRb * idsR;
      idsRb += rsRb * mR;
      dsLb -= idsLb * idsL * idsL;
      dsRb -= idsRb * idsR * idsR;
      SLbar += dsLb;
      SRbar += dsRb;
      SMb -= dsLb + dsRb;
      // pTs = NP iden, SM = NS iden
      T idenb = pTsb * NP + SMb * NS;
      {
        const T g = pTsb * iden;  // NP = mR pTL - mL pTR + mL mR (unR - unL)
        mRb += g * (pTL + mL * (R.un - L.un));
        mLb += g * (-pTR + mR * (R.un - L.un));
        pTLb += g * mR;
        pTRb -= g * mL;
        Rb.un += g * mL * mR;
        Lb.un -= g * mL * mR;
      }
      {
        const T g = SMb * iden;  // NS = mR unR - mL unL - pTR + pTL
        mRb += g * R.un;
        Rb.un += g * mR;
        mLb -= g * L.un;
        Lb.un -= g * mL;
        pTRb -= g;
        pTLb += g;
      }
      // iden = 1 / (mR - mL)
      mRb -= idenb * iden * iden;
      mLb += idenb * iden * iden;
      // m = d rho, d = S - un
      dLb += mLb * L.rho;
      Lb.rho += mLb * dL;
      dRb += mRb * R.rho;
      Rb.rho += mRb * dR;
      SLbar += dLb;
      Lb.un -= dLb;
      SRbar += dRb;
      Rb.un -= dRb;
      bnb += T(2) * bn * bn2b;
      {
        // F = FK - SK UK + ...: the adjoints of FK and UK onto side K
        const T SK = left ? SL : SR;
        T UKb[5];
#pragma unroll
        for (int m = 0; m < 5; ++m) UKb[m] = -Fb[m] * SK;
        side_flux_adj(left, L, R, bn, gm1inv, UKb, Fb, Lb, Rb, bnb);
      }
    }
  }
  // SL = min(unL, unR) - cmax, SR = max(unL, unR) + cmax.  At unL = unR the
  // minimum and the maximum have no unique derivative; both go to the left
  // state, the convention of the selections a <= b ? a : b and a >= b ? a : b
  // (as for cmax and the limiters).  Such ties are not rare: PLM-MC gives
  // exactly equal face values next to every extremum whose neighbour's slope
  // is the doubled one-sided difference.
  const T cmaxb = SRbar - SLbar;
  if (L.un <= R.un)
    Lb.un += SLbar;
  else
    Rb.un += SLbar;
  if (L.un >= R.un)
    Lb.un += SRbar;
  else
    Rb.un += SRbar;
  {
    // cmax = max(cfL, cfR): onto the side that gives it (one path, chosen per lane)
    const bool cl = cfL >= cfR;
    T rb = cl ? Lb.rho : Rb.rho, pb = cl ? Lb.p : Rb.p, b1 = cl ? Lb.bt1 : Rb.bt1,
      b2 = cl ? Lb.bt2 : Rb.bt2;
    fast_speed_adj(cl ? L.rho : R.rho, cl ? L.p : R.p, bn, cl ? L.bt1 : R.bt1, cl ? L.bt2 : R.bt2,
                   gamma, cmaxb, rb, pb, bnb, b1, b2);
    Lb.rho = cl ? rb : Lb.rho;
    Lb.p = cl ? pb : Lb.p;
    Lb.bt1 = cl ? b1 : Lb.bt1;
    Lb.bt2 = cl ? b2 : Lb.bt2;
    Rb.rho = cl ? Rb.rho : rb;
    Rb.p = cl ? Rb.p : pb;
    Rb.bt1 = cl ? Rb.bt1 : b1;
    Rb.bt2 = cl ? Rb.bt2 : b2;
  }
  // the energies and total pressures the fan read
  const T eLv[5] = {T(0), T(0), T(0), T(0), eLb}, eRv[5] = {T(0), T(0), T(0), T(0), eRb};
  phys_flux_adj(L, bn, gm1inv, eLv, zero5, pTLb, Lb, bnb);
  phys_flux_adj(R, bn, gm1inv, eRv, zero5, pTRb, Rb, bnb);
}

// ---------------------------------------------------------------------------
// Face outputs of one face: the 5 fluxes, alpha+ = max(0, SR), alpha- =
// max(0, -SL) and u* = (alpha+ unL + alpha- unR) / (alpha+ + alpha-) (eqs.
// emf:alpha-pm, emf:q26-facevel); LLF uses alpha+ = alpha- = s.  Adjoint of
// the face-local states and of bn.
// ---------------------------------------------------------------------------
template <int RIEMANN, typename T>
CTMHD_HD void face_outputs_adj(const FState<T>& L, const FState<T>& R, T bn, T gamma, const T Fb[5],
                               T apb, T amb, T usb, FState<T>& Lb, FState<T>& Rb, T& bnb) {
  if (RIEMANN == kHLLD) {
    // the outer speeds with the operations of hlld_flux (eq. emf:alpha-pm)
    const T cmax = tmax(fast_speed(L.rho, L.p, bn, L.bt1, L.bt2, gamma),
                        fast_speed(R.rho, R.p, bn, R.bt1, R.bt2, gamma));
    const T SL = tmin(L.un, R.un) - cmax, SR = tmax(L.un, R.un) + cmax;
    const T ap = tmax(T(0), SR), am = tmax(T(0), -SL);
    const T isum = trcp(ap + am);
    const T us = (ap * L.un + am * R.un) * isum;
    apb += usb * (L.un - us) * isum;
    amb += usb * (R.un - us) * isum;
    Lb.un += usb * ap * isum;
    Rb.un += usb * am * isum;
    const T SRb = SR > T(0) ? apb : T(0);
    const T SLb = -SL > T(0) ? -amb : T(0);
    hlld_flux_adj(L, R, bn, gamma, Fb, SLb, SRb, Lb, Rb, bnb);
  } else {
    // u* = (s unL + s unR) / (2 s): no dependence on s
    Lb.un += T(0.5) * usb;
    Rb.un += T(0.5) * usb;
    llf_flux_adj(L, R, bn, gamma, Fb, apb + amb, Lb, Rb, bnb);
  }
}

// ---------------------------------------------------------------------------
// Edge EMF (Q26 corners, eq. emf:q26; LD04 averaging, eq. emf:ld04).
// In: the edge-reconstructed face velocities (uaB, uaT, ubL, ubR) and fields
// (baB, baT, bbL, bbR), the edge speeds (apa, ama, apb, amb) and the adjoint
// Eb of the averaged EMF.  Out (+=): adjoints in the same order.
// ---------------------------------------------------------------------------
template <typename T>
CTMHD_HD void q26_ld04_adj(const T u[4], const T b[4], const T al[4], T Eb, T ub[4], T bb[4],
                           T alb[4]) {
  const T uaB = u[0], uaT = u[1], ubL = u[2], ubR = u[3];
  const T baB = b[0], baT = b[1], bbL = b[2], bbR = b[3];
  const T apa = al[0], ama = al[1], apb = al[2], amb = al[3];
  const T e0 = -uaB * bbL + ubL * baB, e1 = -uaB * bbR + ubR * baB;
  const T e2 = -uaT * bbL + ubL * baT, e3 = -uaT * bbR + ubR * baT;
  const T sa = apa + ama, sb = apb + amb;
  const T iab = T(1) / (sa * sb);
  const T P = apa * apb * e0 + ama * apb * e1 + apa * amb * e2 + ama * amb * e3;
  // E = P / (sa sb) - apb amb / sb (baT - baB) + apa ama / sa (bbR - bbL)
  const T e0b = Eb * apa * apb * iab, e1b = Eb * ama * apb * iab;
  const T e2b = Eb * apa * amb * iab, e3b = Eb * ama * amb * iab;
  const T dba = baT - baB, dbb = bbR - bbL;
  alb[0] += Eb * ((apb * e0 + amb * e2) * iab - P * iab / sa + ama * ama / (sa * sa) * dbb);
  alb[1] += Eb * ((apb * e1 + amb * e3) * iab - P * iab / sa + apa * apa / (sa * sa) * dbb);
  alb[2] += Eb * ((apa * e0 + ama * e1) * iab - P * iab / sb - amb * amb / (sb * sb) * dba);
  alb[3] += Eb * ((apa * e2 + ama * e3) * iab - P * iab / sb - apb * apb / (sb * sb) * dba);
  const T cb = apb * amb / sb, ca = apa * ama / sa;
  bb[1] += -Eb * cb;  // baT
  bb[0] += Eb * cb;   // baB
  bb[3] += Eb * ca;   // bbR
  bb[2] += -Eb * ca;  // bbL
  // corners
  ub[0] += -(e0b * bbL + e1b * bbR);
  ub[1] += -(e2b * bbL + e3b * bbR);
  ub[2] += e0b * baB + e2b * baT;
  ub[3] += e1b * baB + e3b * baT;
  bb[2] += -(e0b * uaB + e2b * uaT);
  bb[3] += -(e1b * uaB + e3b * uaT);
  bb[0] += e0b * ubL + e1b * ubR;
  bb[1] += e2b * ubL + e3b * ubR;
}

// ---------------------------------------------------------------------------
// LD04 averaging alone (eq. emf:ld04), for corner EMFs that do not depend on
// the edge-reconstructed fields (B25a).  In: the four corner EMFs (LB, RB,
// LT, RT), the edge fields (baB, baT, bbL, bbR), the edge speeds (apa, ama,
// apb, amb) and the adjoint Eb of the averaged EMF.  Out (+=): adjoints in
// the same order.
// ---------------------------------------------------------------------------
template <typename T>
CTMHD_HD void ld04_adj(const T e[4], const T b[4], const T al[4], T Eb, T eb[4], T bb[4],
                       T alb[4]) {
  const T baB = b[0], baT = b[1], bbL = b[2], bbR = b[3];
  const T apa = al[0], ama = al[1], apb = al[2], amb = al[3];
  const T sa = apa + ama, sb = apb + amb;
  const T iab = T(1) / (sa * sb);
  const T P = apa * apb * e[0] + ama * apb * e[1] + apa * amb * e[2] + ama * amb * e[3];
  const T dba = baT - baB, dbb = bbR - bbL;
  eb[0] += Eb * apa * apb * iab;
  eb[1] += Eb * ama * apb * iab;
  eb[2] += Eb * apa * amb * iab;
  eb[3] += Eb * ama * amb * iab;
  alb[0] += Eb * ((apb * e[0] + amb * e[2]) * iab - P * iab / sa + ama * ama / (sa * sa) * dbb);
  alb[1] += Eb * ((apb * e[1] + amb * e[3]) * iab - P * iab / sa + apa * apa / (sa * sa) * dbb);
  alb[2] += Eb * ((apa * e[0] + ama * e[1]) * iab - P * iab / sb - amb * amb / (sb * sb) * dba);
  alb[3] += Eb * ((apa * e[2] + ama * e[3]) * iab - P * iab / sb - apb * apb / (sb * sb) * dba);
  const T cb = apb * amb / sb, ca = apa * ama / sa;
  bb[0] += Eb * cb;
  bb[1] += -Eb * cb;
  bb[2] += -Eb * ca;
  bb[3] += Eb * ca;
}

}  // namespace ctmhd
