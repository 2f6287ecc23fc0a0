// ctmhd_math.h -- per-point arithmetic of the CT-MHD step for gfx950.
//
// Device functions only; templated on the stencil type T (double for the
// FP64 form, float for the FP32 form).  Cited sections and equations are those
// of Kriel et al., "Magnetising the Quokka code with fast, second-order
// accurate, error-correcting schemes for MHD on GPUs".
#pragma once

#include <hip/hip_runtime.h>

// per-point arithmetic is callable from device and host code (the host
// instances serve CPU checks of the derivative code)
#define CTMHD_HD __host__ __device__ __forceinline__

namespace ctmhd {

enum : int { kPC = 0, kPLM_MC = 1, kPLM_MM = 2, kPPM = 3 };
// Riemann solvers; kHLLD64 / kLLF64 solve in float64 from face states of
// the stencil type (the FP32 form with a float64 Riemann solve)
enum : int { kHLLD = 0, kLLF = 1, kHLLD64 = 2, kLLF64 = 3 };
enum : int { kQ26 = 0, kB25A = 1, kFS18 = 2 };

// Reconstruction half-width r of each method; ghost layers needed = r + 2.
__host__ __device__ constexpr int recon_halfwidth(int m) {
  return m == kPC ? 0 : (m == kPPM ? 2 : 1);
}

// abs / min / max / sign transfer as single instructions (v_max_f64 etc.);
// on non-NaN operands they return the same values as the comparisons
// a >= b ? a : b and x < 0 ? -x : x (up to the sign of a zero).
CTMHD_HD double tabs(double x) { return __builtin_fabs(x); }
CTMHD_HD float tabs(float x) { return __builtin_fabsf(x); }
CTMHD_HD double tmax(double a, double b) { return __builtin_fmax(a, b); }
CTMHD_HD float tmax(float a, float b) { return __builtin_fmaxf(a, b); }
CTMHD_HD double tmin(double a, double b) { return __builtin_fmin(a, b); }
CTMHD_HD float tmin(float a, float b) { return __builtin_fminf(a, b); }
CTMHD_HD double tsign(double mag, double s) { return __builtin_copysign(mag, s); }
CTMHD_HD float tsign(float mag, float s) { return __builtin_copysignf(mag, s); }
CTMHD_HD double tsqrt(double x) { return __builtin_sqrt(x); }
CTMHD_HD float tsqrt(float x) { return __builtin_sqrtf(x); }
CTMHD_HD bool tfinite(double x) { return __builtin_isfinite(x); }
CTMHD_HD bool tfinite(float x) { return __builtin_isfinite(x); }

// Reciprocal and reciprocal square root of a finite, normal x (x > 0 for
// trsqrt), within about one unit in the last place.  On the GPU: the
// hardware estimates (v_rcp_f64, v_rsq_f64 to about 2^-23; v_rcp_f32,
// v_rsq_f32 to one unit) refined by Newton steps, two in double and one in
// float, against about twice the instructions of the correctly rounded
// division and square root, which also handle denormal and infinite
// operands.  A zero x gives NaN (the callers reject such a state anyway).  On
// the host (CPU checks of the derivative code): the plain operations.
CTMHD_HD double trcp(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
#else
  return 1.0 / x;
#endif
}
CTMHD_HD float trcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
#else
  return 1.0f / x;
#endif
}
CTMHD_HD double trsqrt(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  // y <- y + y (1/2 - (x/2) y^2)
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = __builtin_fma(y, __builtin_fma(-h * y, y, 0.5), y);
  return __builtin_fma(y, __builtin_fma(-h * y, y, 0.5), y);
#else
  return 1.0 / __builtin_sqrt(x);
#endif
}
// Square root of the wave-speed terms.  On the GPU: the hardware reciprocal
// square root estimate (refined by one Newton step in double; one unit in the
// last place in float) times x, then one correction by the residual x - s^2
// (Markstein's form), within about one unit in the last place for x >= 2^-900
// (double) or 2^-100 (float); |x| below that gives 0 and x < 0 NaN.  The
// library square root adds the range scaling of denormal operands and the
// special cases of zero and infinity.  On the host: the library square root.
CTMHD_HD double twsqrt(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = __builtin_fma(y, __builtin_fma(-h * y, y, 0.5), y);
  double s = x * y;
  s = __builtin_fma(0.5 * y, __builtin_fma(-s, s, x), s);
  return __builtin_fabs(x) < 0x1p-900 ? 0.0 : s;
#else
  return __builtin_sqrt(x);
#endif
}
CTMHD_HD float twsqrt(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const float y = __builtin_amdgcn_rsqf(x);
  float s = x * y;
  s = __builtin_fmaf(0.5f * y, __builtin_fmaf(-s, s, x), s);
  return __builtin_fabsf(x) < 0x1p-100f ? 0.0f : s;
#else
  return __builtin_sqrtf(x);
#endif
}
CTMHD_HD float trsqrt(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const float y = __builtin_amdgcn_rsqf(x);
  return __builtin_fmaf(y, __builtin_fmaf(-0.5f * x * y, y, 0.5f), y);
#else
  return 1.0f / __builtin_sqrtf(x);
#endif
}

// ---------------------------------------------------------------------------
// 1D reconstruction (Sec. 2.2).  q[0..4] centred on q[2]; returns the values
// at the lower (qm) and upper (qp) face of the centre cell.  PLM uses the
// monotonised-central or minmod limited slope; PPM uses the Colella-Woodward
// limited-slope interface value and their monotonicity constraints.
// ---------------------------------------------------------------------------
template <int M, typename T>
CTMHD_HD T plm_slope(T qm, T q0, T qp) {
  T dl = q0 - qm, dr = qp - q0;
  T s;
  if (M == kPLM_MC)
    s = tmin(tmin(T(2) * tabs(dl), T(2) * tabs(dr)), T(0.5) * tabs(dl + dr));
  else
    s = tmin(tabs(dl), tabs(dr));
  s = tsign(s, dr);  // dl * dr > 0: dr carries the common sign
  return dl * dr > T(0) ? s : T(0);
}

template <typename T>
CTMHD_HD T ppm_slope(T qm, T q0, T qp) {
  T dl = q0 - qm, dr = qp - q0;
  T dc = T(0.5) * (qp - qm);
  T s = tmin(tabs(dc), T(2) * tmin(tabs(dl), tabs(dr)));
  s = tsign(s, dc);  // dl * dr > 0: dc carries the common sign
  return dl * dr > T(0) ? s : T(0);
}

// PPM interface value between cells with values qa, qb and limited slopes
// da, db (Colella-Woodward).
template <typename T>
CTMHD_HD T ppm_iface(T qa, T qb, T da, T db) {
  return T(0.5) * (qa + qb) - (db - da) * (T(1) / T(6));
}

// Colella-Woodward monotonicity constraints on a cell with centre value q0
// and face values qL, qR (in place).
template <typename T>
CTMHD_HD void ppm_constrain(T q0, T& qL, T& qR) {
  const T sixth = T(1) / T(6);
  if ((qR - q0) * (q0 - qL) <= T(0)) {
    qL = q0;
    qR = q0;
  } else {
    T dq = qR - qL;
    T q6 = dq * (q0 - T(0.5) * (qL + qR));
    T d6 = dq * dq * sixth;
    if (q6 > d6)
      qL = T(3) * q0 - T(2) * qR;
    else if (-d6 > q6)
      qR = T(3) * q0 - T(2) * qL;
  }
}

template <int M, typename T>
CTMHD_HD void recon_cell(const T* q, T& qm, T& qp) {
  if constexpr (M == kPC) {
    qm = q[2];
    qp = q[2];
  } else if constexpr (M == kPLM_MC || M == kPLM_MM) {
    T s = T(0.5) * plm_slope<M>(q[1], q[2], q[3]);
    qm = q[2] - s;
    qp = q[2] + s;
  } else {
    T d1 = ppm_slope(q[0], q[1], q[2]);
    T d2 = ppm_slope(q[1], q[2], q[3]);
    T d3 = ppm_slope(q[2], q[3], q[4]);
    T qL = ppm_iface(q[1], q[2], d1, d2);
    T qR = ppm_iface(q[2], q[3], d2, d3);
    ppm_constrain(q[2], qL, qR);
    qm = qL;
    qp = qR;
  }
}

// Streaming reconstruction along a line of cells: push the cell values in
// order; after the warm-up each push completes the cell r behind the newest
// one and returns its lower / upper face values.  Every limited slope and
// interface value is formed once and gives the same numbers as recon_cell.
template <int M, typename T>
struct ReconStream {
  T q1 = T(0), q2 = T(0);  // the previous two cells (q1 newest)
  T dm1 = T(0);            // PPM: limited slope of the cell behind q1
  T ilo = T(0);            // PPM: interface below the cell completed next
  CTMHD_HD void push(T v, T& qm, T& qp) {
    if constexpr (M == kPC) {
      qm = v;
      qp = v;
    } else if constexpr (M == kPLM_MC || M == kPLM_MM) {
      // completes cell q1 (values q2, q1, v)
      T s = T(0.5) * plm_slope<M>(q2, q1, v);
      qm = q1 - s;
      qp = q1 + s;
      q2 = q1;
      q1 = v;
    } else {
      // slope of cell q1, interface between q2 and q1, completes cell q2
      T dm = ppm_slope(q2, q1, v);
      T ihi = ppm_iface(q2, q1, dm1, dm);
      T qL = ilo, qR = ihi;
      ppm_constrain(q2, qL, qR);
      qm = qL;
      qp = qR;
      ilo = ihi;
      dm1 = dm;
      q2 = q1;
      q1 = v;
    }
  }
};

// Whether entry m of the six-point sequence q[0..5] below enters the
// reconstruction at the q[2]|q[3] interface: m in [2 - r, 3 + r].
template <int M>
__host__ __device__ constexpr bool stencil_uses(int m) {
  return m >= 2 - recon_halfwidth(M) && m <= 3 + recon_halfwidth(M);
}

// Values on the two sides of the interface between q[2] and q[3] of a
// six-point sequence q[0..5]: lo = upper value of cell 2, hi = lower value of
// cell 3.
template <int M, typename T>
CTMHD_HD void recon_iface(const T* q, T& lo, T& hi) {
  if constexpr (M == kPPM) {
    // cells 2 and 3 share slopes d2, d3 and the interface between them
    T d1 = ppm_slope(q[0], q[1], q[2]);
    T d2 = ppm_slope(q[1], q[2], q[3]);
    T d3 = ppm_slope(q[2], q[3], q[4]);
    T d4 = ppm_slope(q[3], q[4], q[5]);
    T i1 = ppm_iface(q[1], q[2], d1, d2);
    T i2 = ppm_iface(q[2], q[3], d2, d3);
    T i3 = ppm_iface(q[3], q[4], d3, d4);
    T aL = i1, aR = i2, bL = i2, bR = i3;
    ppm_constrain(q[2], aL, aR);
    ppm_constrain(q[3], bL, bR);
    lo = aR;
    hi = bL;
  } else {
    T d;
    recon_cell<M>(q, d, lo);
    recon_cell<M>(q + 1, hi, d);
  }
}

// ---------------------------------------------------------------------------
// Fast magnetosonic speed along the face normal (eq. waves:fast-speed).
// ---------------------------------------------------------------------------
template <typename T>
CTMHD_HD T fast_speed(T rho, T p, T bn, T bt1, T bt2, T gamma) {
  T irho = trcp(rho);
  T gp = gamma * p;
  T a = (gp + bn * bn + bt1 * bt1 + bt2 * bt2) * irho;
  T disc = a * a - T(4) * gp * bn * bn * irho * irho;
  disc = disc > T(0) ? disc : T(0);
  return twsqrt(T(0.5) * (a + twsqrt(disc)));
}

// Face-local primitive state: normal velocity un, transverse ut1/ut2 and the
// transverse field bt1/bt2 (t1, t2 in cyclic order after the normal).
template <typename T> struct FState { T rho, un, ut1, ut2, p, bt1, bt2; };

// Conserved state and ideal-MHD flux normal to a face (eq.
// mhd:conservation-laws), (rho, m_n, m_t1, m_t2, e_tot) only.
template <typename T>
CTMHD_HD void phys_flux(const FState<T>& s, T bn, T gm1inv, T* U, T* F, T& pT) {
  T b2 = bn * bn + s.bt1 * s.bt1 + s.bt2 * s.bt2;
  T v2 = s.un * s.un + s.ut1 * s.ut1 + s.ut2 * s.ut2;
  T e = s.p * gm1inv + T(0.5) * (s.rho * v2 + b2);
  pT = s.p + T(0.5) * b2;
  T vb = s.un * bn + s.ut1 * s.bt1 + s.ut2 * s.bt2;
  T mn = s.rho * s.un;
  U[0] = s.rho;
  U[1] = mn;
  U[2] = s.rho * s.ut1;
  U[3] = s.rho * s.ut2;
  U[4] = e;
  F[0] = mn;
  F[1] = mn * s.un + pT - bn * bn;
  F[2] = mn * s.ut1 - bn * s.bt1;
  F[3] = mn * s.ut2 - bn * s.bt2;
  F[4] = (e + pT) * s.un - bn * vb;
}

// Local Lax-Friedrichs flux; returns the signal speed s used as alpha^{+/-}.
template <typename T>
CTMHD_HD T llf_flux(const FState<T>& L, const FState<T>& R, T bn, T gamma,
                                      T* F) {
  const T gm1inv = T(1) / (gamma - T(1));
  T UL[5], FL[5], UR[5], FR[5], pL, pR;
  phys_flux(L, bn, gm1inv, UL, FL, pL);
  phys_flux(R, bn, gm1inv, UR, FR, pR);
  T s = tmax(tabs(L.un) + fast_speed(L.rho, L.p, bn, L.bt1, L.bt2, gamma),
             tabs(R.un) + fast_speed(R.rho, R.p, bn, R.bt1, R.bt2, gamma));
#pragma unroll
  for (int m = 0; m < 5; ++m) F[m] = T(0.5) * (FL[m] + FR[m]) - T(0.5) * s * (UR[m] - UL[m]);
  return s;
}

// HLLD (Miyoshi & Kusano 2005) with the outer speeds of eq. emf:alpha-pm.
// Degenerate star states fall back to the outer transverse state; the
// double-star states are skipped when bn^2 <= 1e-12 p_T*; an unphysical fan
// (rho* <= 0, p_T* <= 0, S_M outside (S_L, S_R), non-finite values) falls
// back to HLL with the same outer speeds.  Returns 1 on fallback.
template <typename T>
CTMHD_HD int hlld_flux(const FState<T>& L, const FState<T>& R, T bn, T gamma,
                                         T* F, T& SL, T& SR) {
  T gm1inv = T(1) / (gamma - T(1));
  T UL[5], FL[5], UR[5], FR[5], pTL, pTR;
  phys_flux(L, bn, gm1inv, UL, FL, pTL);
  phys_flux(R, bn, gm1inv, UR, FR, pTR);
  T cmax = tmax(fast_speed(L.rho, L.p, bn, L.bt1, L.bt2, gamma),
                fast_speed(R.rho, R.p, bn, R.bt1, R.bt2, gamma));
  SL = tmin(L.un, R.un) - cmax;
  SR = tmax(L.un, R.un) + cmax;
  if (SL > T(0)) {
#pragma unroll
    for (int m = 0; m < 5; ++m) F[m] = FL[m];
    return 0;
  }
  if (SR < T(0)) {
#pragma unroll
    for (int m = 0; m < 5; ++m) F[m] = FR[m];
    return 0;
  }
  const T bn2 = bn * bn;
  T dL = SL - L.un, dR = SR - R.un;
  T mL = dL * L.rho, mR = dR * R.rho;  // (S - u) rho
  T iden = trcp(mR - mL);
  T SM = (mR * R.un - mL * L.un - pTR + pTL) * iden;
  T pTs = (mR * pTL - mL * pTR + mL * mR * (R.un - L.un)) * iden;
  T dsL = SL - SM, dsR = SR - SM;
  T idsL = trcp(dsL), idsR = trcp(dsR);
  T rsL = mL * idsL, rsR = mR * idsR;

  // star transverse states
  T vsL, wsL, bysL, bzsL, vsR, wsR, bysR, bzsR;
  {
    T q = mL * dsL - bn2;
    T ref = tabs(mL * dsL) + bn2;
    bool deg = tabs(q) <= T(1e-12) * ref;
    T iq = trcp(q);
    T fv = bn * (SM - L.un) * iq;
    T fb = (mL * dL - bn2) * iq;
    vsL = deg ? L.ut1 : L.ut1 - L.bt1 * fv;
    wsL = deg ? L.ut2 : L.ut2 - L.bt2 * fv;
    bysL = deg ? L.bt1 : L.bt1 * fb;
    bzsL = deg ? L.bt2 : L.bt2 * fb;
  }
  {
    T q = mR * dsR - bn2;
    T ref = tabs(mR * dsR) + bn2;
    bool deg = tabs(q) <= T(1e-12) * ref;
    T iq = trcp(q);
    T fv = bn * (SM - R.un) * iq;
    T fb = (mR * dR - bn2) * iq;
    vsR = deg ? R.ut1 : R.ut1 - R.bt1 * fv;
    wsR = deg ? R.ut2 : R.ut2 - R.bt2 * fv;
    bysR = deg ? R.bt1 : R.bt1 * fb;
    bzsR = deg ? R.bt2 : R.bt2 * fb;
  }
  T vbL = L.un * bn + L.ut1 * L.bt1 + L.ut2 * L.bt2;
  T vbR = R.un * bn + R.ut1 * R.bt1 + R.ut2 * R.bt2;
  T vbsL = SM * bn + vsL * bysL + wsL * bzsL;
  T vbsR = SM * bn + vsR * bysR + wsR * bzsR;
  T esL = (dL * UL[4] - pTL * L.un + pTs * SM + bn * (vbL - vbsL)) * idsL;
  T esR = (dR * UR[4] - pTR * R.un + pTs * SM + bn * (vbR - vbsR)) * idsR;

  bool bad = !(rsL > T(0)) || !(rsR > T(0)) || !(pTs > T(0)) || !(SL < SM) || !(SM < SR) ||
             !tfinite(SM) || !tfinite(vsL + wsL + bysL + bzsL + esL) ||
             !tfinite(vsR + wsR + bysR + bzsR + esR);
  if (bad) {
    if (SL >= T(0)) {
#pragma unroll
      for (int m = 0; m < 5; ++m) F[m] = FL[m];
    } else if (SR <= T(0)) {
#pragma unroll
      for (int m = 0; m < 5; ++m) F[m] = FR[m];
    } else {
      T iw = trcp(SR - SL);
#pragma unroll
      for (int m = 0; m < 5; ++m) F[m] = (SR * FL[m] - SL * FR[m] + SL * SR * (UR[m] - UL[m])) * iw;
    }
    return 1;
  }

  T UsL[5] = {rsL, rsL * SM, rsL * vsL, rsL * wsL, esL};
  T UsR[5] = {rsR, rsR * SM, rsR * vsR, rsR * wsR, esR};
  T SsL = SM, SsR = SM;
  T UssL[5], UssR[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    UssL[m] = UsL[m];
    UssR[m] = UsR[m];
  }
  if (!(bn2 <= T(1e-12) * pTs)) {
    T sg = bn > T(0) ? T(1) : (bn < T(0) ? T(-1) : T(0));
    // rs > 0 here: sqrt(rs) = rs / sqrt(rs)
    T yL = trsqrt(rsL), yR = trsqrt(rsR);
    T sqL = rsL * yL, sqR = rsR * yR;
    T abn = tabs(bn);
    SsL = SM - abn * yL;
    SsR = SM + abn * yR;
    T isum = trcp(sqL + sqR);
    T vss = (sqL * vsL + sqR * vsR + (bysR - bysL) * sg) * isum;
    T wss = (sqL * wsL + sqR * wsR + (bzsR - bzsL) * sg) * isum;
    T byss = (sqL * bysR + sqR * bysL + sqL * sqR * (vsR - vsL) * sg) * isum;
    T bzss = (sqL * bzsR + sqR * bzsL + sqL * sqR * (wsR - wsL) * sg) * isum;
    T vbss = SM * bn + vss * byss + wss * bzss;
    UssL[2] = rsL * vss;
    UssL[3] = rsL * wss;
    UssL[4] = esL - sqL * (vbsL - vbss) * sg;
    UssR[2] = rsR * vss;
    UssR[3] = rsR * wss;
    UssR[4] = esR + sqR * (vbsR - vbss) * sg;
  }
  if (SsL >= T(0)) {
#pragma unroll
    for (int m = 0; m < 5; ++m) F[m] = FL[m] + SL * (UsL[m] - UL[m]);
  } else if (SM >= T(0)) {
#pragma unroll
    for (int m = 0; m < 5; ++m) F[m] = FL[m] + SL * (UsL[m] - UL[m]) + SsL * (UssL[m] - UsL[m]);
  } else if (SsR >= T(0)) {
#pragma unroll
    for (int m = 0; m < 5; ++m) F[m] = FR[m] + SR * (UsR[m] - UR[m]) + SsR * (UssR[m] - UsR[m]);
  } else {
#pragma unroll
    for (int m = 0; m < 5; ++m) F[m] = FR[m] + SR * (UsR[m] - UR[m]);
  }
  return 0;
}

// LD04 averaging (eq. emf:ld04) of four corner EMFs (LB, RB, LT, RT) with the
// edge wavespeeds of eq. emf:alpha-edge and the edge-reconstructed fields.
template <typename T>
CTMHD_HD T ld04(T eLB, T eRB, T eLT, T eRT, T apa, T ama, T apb, T amb, T baB,
                                  T baT, T bbL, T bbR) {
  T sa = apa + ama, sb = apb + amb;
  T iab = T(1) / (sa * sb);
  return (apa * apb * eLB + ama * apb * eRB) * iab + (apa * amb * eLT + ama * amb * eRT) * iab -
         apb * amb / sb * (baT - baB) + apa * ama / sa * (bbR - bbL);
}

}  // namespace ctmhd
