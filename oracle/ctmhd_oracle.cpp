// ctmhd_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, scalar FP64 reference for one second-order constrained-
// transport (CT) MHD time step on a periodic Cartesian box, written from the
// paper (Kriel et al., "Magnetising the Quokka code with fast, second-order
// accurate, error-correcting schemes for MHD on GPUs"):
//   Sec. 2.1 mesh (eq. state:conserved), Sec. 2.2 fluxes (eq. state:primitive,
//   reconstruction, HLLD, LLF), Sec. 2.3 EMFs (eqs. emf:fs18-average, emf:fs18,
//   emf:b25a-*, emf:q26-facevel, emf:alpha-pm, emf:q26, emf:alpha-edge,
//   emf:ld04), Sec. 2.4 resistivity (eqs. resistivity:*), Sec. 2.5 RK2-SSP with
//   first-order flux correction (eqs. rk:increment-state, rk:increment-bfield,
//   rk1:update, rk2:update).
//
// Only the test suite, the smoke check and the CPU-baseline leg of the bench
// may load this library.  It shares no code with the GPU path.  Arrays are
// interior-only (no ghost layers): every index is wrapped periodically.
//
// Everything is templated on the scalar type R:
//   double -- the reference itself,
//   Dual   -- forward-mode derivative (one tangent), for gradient checks,
//   Count  -- a flop counter (add/sub, mul, div, sqrt, compare) per phase.
// Compiled with -ffp-contract=off: no fused multiply-add anywhere.
//
// Readings of points the paper leaves open are marked "reading:" below.

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

namespace orc {

// --------------------------------------------------------------------------
// Scalar types
// --------------------------------------------------------------------------
struct Dual {
  double v = 0.0, d = 0.0;
  Dual() = default;
  Dual(double x) : v(x), d(0.0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
inline double val(Dual a) { return a.v; }
inline Dual rsqrt_(Dual a) {
  double s = std::sqrt(a.v);
  return {s, s > 0.0 ? a.d / (2.0 * s) : 0.0};
}

// Flop counter.  Counts go to per-phase tallies; phase set by the caller.
enum { OP_ADD = 0, OP_MUL, OP_DIV, OP_SQRT, OP_CMP, OP_N };
enum { PH_DT = 0, PH_PRIM, PH_FACE, PH_EMF, PH_UPDATE, PH_FOFC, PH_RECON, PH_N };
static int64_t g_count[PH_N][OP_N];
static int g_phase = 0;
static int64_t g_recon_calls = 0;  // 1D reconstructions (each gives both faces of a cell)
struct Count {
  double v = 0.0;
  Count() = default;
  Count(double x) : v(x) {}
};
inline Count cnt(double x, int op) { g_count[g_phase][op]++; return Count(x); }
inline Count operator+(Count a, Count b) { return cnt(a.v + b.v, OP_ADD); }
inline Count operator-(Count a, Count b) { return cnt(a.v - b.v, OP_ADD); }
inline Count operator-(Count a) { return Count(-a.v); }
inline Count operator*(Count a, Count b) { return cnt(a.v * b.v, OP_MUL); }
inline Count operator/(Count a, Count b) { return cnt(a.v / b.v, OP_DIV); }
inline bool operator<(Count a, Count b) { g_count[g_phase][OP_CMP]++; return a.v < b.v; }
inline bool operator>(Count a, Count b) { g_count[g_phase][OP_CMP]++; return a.v > b.v; }
inline bool operator<=(Count a, Count b) { g_count[g_phase][OP_CMP]++; return a.v <= b.v; }
inline bool operator>=(Count a, Count b) { g_count[g_phase][OP_CMP]++; return a.v >= b.v; }
inline double val(Count a) { return a.v; }
inline Count rsqrt_(Count a) { return cnt(std::sqrt(a.v), OP_SQRT); }

inline double val(double a) { return a; }
inline double rsqrt_(double a) { return std::sqrt(a); }

template <class R> inline R rsqrt(R a) { return rsqrt_(a); }
template <class R> inline R rabs(R a) { return a < R(0.0) ? -a : a; }
template <class R> inline R rmax(R a, R b) { return a >= b ? a : b; }
template <class R> inline R rmin(R a, R b) { return a <= b ? a : b; }
template <class R> inline bool finite(R a) { return std::isfinite(val(a)); }

// --------------------------------------------------------------------------
// Parameters (mirrored by a ctypes Structure in oracle.py)
// --------------------------------------------------------------------------
enum { RECON_PC = 0, RECON_PLM_MC = 1, RECON_PLM_MINMOD = 2, RECON_PPM = 3 };
enum { RIEMANN_HLLD = 0, RIEMANN_LLF = 1 };
enum { EMF_Q26 = 0, EMF_B25A = 1, EMF_FS18 = 2 };
enum { FLAG_RHO = 1, FLAG_P = 2, FLAG_NONFINITE = 4 };

struct Params {
  double gamma;
  double eta;
  double cfl;
  int recon;
  int riemann;
  int emf;
  int fofc;
  int flag_mask;
  int pad_;
};

// --------------------------------------------------------------------------
// Periodic 3D arrays, x fastest.  Interior only.
// --------------------------------------------------------------------------
struct Grid {
  int n[3];
  double dx[3];
  int64_t size() const { return (int64_t)n[0] * n[1] * n[2]; }
  int64_t idx(int i, int j, int k) const {
    i %= n[0]; if (i < 0) i += n[0];
    j %= n[1]; if (j < 0) j += n[1];
    k %= n[2]; if (k < 0) k += n[2];
    return ((int64_t)k * n[1] + j) * n[0] + i;
  }
  int64_t idx(const int p[3]) const { return idx(p[0], p[1], p[2]); }
};

template <class R> using Arr = std::vector<R>;
// Loops over z-planes run in parallel (OpenMP) except for the counting type,
// whose tallies are global.  Every cell's arithmetic is unchanged.
template <class R> constexpr bool kPar = !std::is_same<R, Count>::value;

struct P3 {
  int v[3];
  P3 sh(int a, int s) const { P3 q = *this; q.v[a] += s; return q; }
};

// Cell-centred primitive state, eq. state:primitive.
template <class R> struct Prim { Arr<R> rho, u[3], p, b[3]; };
// Conserved state (eq. state:conserved) plus face-centred normal field.
template <class R> struct State { Arr<R> c[5]; Arr<R> bf[3]; };

// Per-direction face data and per-direction edge EMFs.
template <class R> struct FaceData {
  Arr<R> F[3][5];     // flux of (rho, m0, m1, m2, e_tot) across x_a faces
  Arr<R> ap[3], am[3]; // bounding wavespeed magnitudes alpha_a^{+/-}
  Arr<R> us[3];       // Q26 face-normal velocity u_a^*
};
template <class R> struct Fluxes {
  Arr<R> F[3][5];
  Arr<R> E[3];  // edge EMF eps_c at the lower-left edge of each cell
};

// --------------------------------------------------------------------------
// Conserved -> primitive (Sec. 2.2, eq. state:primitive).  The cell-averaged
// field is the mean of the two faces; pressure from e_tot = e_int +
// (rho u^2 + b^2)/2 with e_int = p/(gamma-1).
// --------------------------------------------------------------------------
template <class R>
void to_prim(const Grid& g, const Params& P, const State<R>& S, Prim<R>& W) {
  const int64_t N = g.size();
  W.rho.assign(N, R(0.0)); W.p.assign(N, R(0.0));
  for (int d = 0; d < 3; ++d) { W.u[d].assign(N, R(0.0)); W.b[d].assign(N, R(0.0)); }
  const R gm1 = R(P.gamma - 1.0);
#pragma omp parallel for if (kPar<R>)
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        int64_t c = g.idx(i, j, k);
        R rho = S.c[0][c];
        R u[3], b[3];
        for (int d = 0; d < 3; ++d) u[d] = S.c[1 + d][c] / rho;
        for (int d = 0; d < 3; ++d) {
          P3 q{{i, j, k}};
          q.v[d] += 1;
          b[d] = R(0.5) * (S.bf[d][c] + S.bf[d][g.idx(q.v)]);
        }
        R ke = R(0.5) * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        R me = R(0.5) * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
        W.rho[c] = rho;
        W.p[c] = gm1 * (S.c[4][c] - ke - me);
        for (int d = 0; d < 3; ++d) { W.u[d][c] = u[d]; W.b[d][c] = b[d]; }
      }
}

// --------------------------------------------------------------------------
// Fast magnetosonic speed along the normal direction (eq. waves:fast-speed
// with c_A^2 cos^2(theta) = b_n^2 / rho).
// --------------------------------------------------------------------------
template <class R>
R fast_speed(R rho, R p, R bn, R bt1, R bt2, R gamma) {
  R b2 = bn * bn + bt1 * bt1 + bt2 * bt2;
  R gp = gamma * p;
  R a = (gp + b2) / rho;
  R disc = a * a - R(4.0) * gp * bn * bn / (rho * rho);
  if (disc < R(0.0)) disc = R(0.0);
  return rsqrt(R(0.5) * (a + rsqrt(disc)));
}

// --------------------------------------------------------------------------
// Time step (Sec. 2.4, eq. resistivity:cfl and the text after it).
// reading: dt = CFL / max over cells of max( max_d (|u_d| + c_f,d)/dx_d ,
// 2 eta / dx_min^2 ); the resistive signal speed 2 eta/dx_min enters the same
// per-cell maximum as the wave speeds.
// --------------------------------------------------------------------------
template <class R>
R compute_dt(const Grid& g, const Params& P, const Prim<R>& W) {
  const R gamma = R(P.gamma);
  double dxmin = std::min(g.dx[0], std::min(g.dx[1], g.dx[2]));
  R smax = R(0.0);
  if (P.eta > 0.0) smax = R(2.0 * P.eta / (dxmin * dxmin));
  for (int64_t c = 0; c < g.size(); ++c) {
    for (int d = 0; d < 3; ++d) {
      R cf = fast_speed(W.rho[c], W.p[c], W.b[d][c], W.b[(d + 1) % 3][c],
                        W.b[(d + 2) % 3][c], gamma);
      R s = (rabs(W.u[d][c]) + cf) / R(g.dx[d]);
      smax = rmax(smax, s);
    }
  }
  return R(P.cfl) / smax;
}

// --------------------------------------------------------------------------
// 1D reconstruction (Sec. 2.2): given five consecutive values q[0..4] centred
// on q[2], return the values at the lower (qm) and upper (qp) faces of the
// centre cell.  PC: constant.  PLM: monotonised-central or minmod slope.
// PPM: reading: the textbook Colella-Woodward interface value with the
// limited centred slope and the CW monotonicity constraints, no
// characteristic tracing (the scheme is method-of-lines under RK2).
// --------------------------------------------------------------------------
template <class R> R sgn(R x) { return x > R(0.0) ? R(1.0) : (x < R(0.0) ? R(-1.0) : R(0.0)); }

template <class R>
R plm_slope(int method, R qm, R q0, R qp) {
  R dl = q0 - qm, dr = qp - q0;
  if (dl * dr <= R(0.0)) return R(0.0);
  R s;
  if (method == RECON_PLM_MC)
    s = rmin(rmin(R(2.0) * rabs(dl), R(2.0) * rabs(dr)), R(0.5) * rabs(dl + dr));
  else
    s = rmin(rabs(dl), rabs(dr));
  return dr > R(0.0) ? s : -s;
}

template <class R>
R ppm_limited_slope(R qm, R q0, R qp) {
  R dl = q0 - qm, dr = qp - q0;
  if (dl * dr <= R(0.0)) return R(0.0);
  R dc = R(0.5) * (qp - qm);
  R s = rmin(rabs(dc), rmin(R(2.0) * rabs(dl), R(2.0) * rabs(dr)));
  return dc > R(0.0) ? s : -s;
}

// interface value between q[i] and q[i+1] from q[i-1..i+2]
template <class R>
R ppm_interface(R qa, R qb, R qc, R qd) {
  R dmb = ppm_limited_slope(qa, qb, qc);
  R dmc = ppm_limited_slope(qb, qc, qd);
  return R(0.5) * (qb + qc) - (dmc - dmb) / R(6.0);
}

template <class R>
void recon1d_(int method, const R q[5], R& qm, R& qp);

// Counting type: tally reconstruction arithmetic under its own phase.
template <class R>
void recon1d(int method, const R q[5], R& qm, R& qp) {
  if (std::is_same<R, Count>::value) {
    int save = g_phase;
    g_phase = PH_RECON;
    ++g_recon_calls;
    recon1d_(method, q, qm, qp);
    g_phase = save;
  } else {
    recon1d_(method, q, qm, qp);
  }
}

template <class R>
void recon1d_(int method, const R q[5], R& qm, R& qp) {
  if (method == RECON_PC) { qm = q[2]; qp = q[2]; return; }
  if (method == RECON_PLM_MC || method == RECON_PLM_MINMOD) {
    R s = plm_slope(method, q[1], q[2], q[3]);
    qm = q[2] - R(0.5) * s;
    qp = q[2] + R(0.5) * s;
    return;
  }
  // PPM
  R qL = ppm_interface(q[0], q[1], q[2], q[3]);
  R qR = ppm_interface(q[1], q[2], q[3], q[4]);
  R q0 = q[2];
  if ((qR - q0) * (q0 - qL) <= R(0.0)) {
    qL = q0; qR = q0;
  } else {
    R dq = qR - qL;
    R q6 = dq * (q0 - R(0.5) * (qL + qR));
    R d2 = dq * dq / R(6.0);
    if (q6 > d2) qL = R(3.0) * q0 - R(2.0) * qR;
    else if (-d2 > q6) qR = R(3.0) * q0 - R(2.0) * qL;
  }
  qm = qL; qp = qR;
}

// Gather five values of an array along axis a centred on p.
template <class R>
void gather5(const Grid& g, const Arr<R>& A, const P3& p, int a, R q[5]) {
  for (int m = 0; m < 5; ++m) q[m] = A[g.idx(p.sh(a, m - 2).v)];
}
// Values of array A on either side of the interface at the lower face of p
// along axis a: lo = upper value of cell p - e_a, hi = lower value of cell p.
template <class R>
void iface(const Grid& g, int method, const Arr<R>& A, const P3& p, int a, R& lo, R& hi) {
  R q[5], dummy;
  gather5(g, A, p.sh(a, -1), a, q);
  recon1d(method, q, dummy, lo);
  gather5(g, A, p, a, q);
  recon1d(method, q, hi, dummy);
}

// --------------------------------------------------------------------------
// Riemann solvers (Sec. 2.2).  Face-local frame: n = normal, t1/t2 the two
// transverse directions in cyclic order.  Only the (rho, m, e_tot) part of the
// flux is returned; the face-normal field bn is the stored face value.
// --------------------------------------------------------------------------
template <class R> struct FState { R rho, un, ut1, ut2, p, bt1, bt2; };

template <class R>
void phys(const FState<R>& s, R bn, R gamma, R U[5], R F[5], R& pT) {
  R b2 = bn * bn + s.bt1 * s.bt1 + s.bt2 * s.bt2;
  R v2 = s.un * s.un + s.ut1 * s.ut1 + s.ut2 * s.ut2;
  R e = s.p / (gamma - R(1.0)) + R(0.5) * s.rho * v2 + R(0.5) * b2;
  pT = s.p + R(0.5) * b2;
  R vb = s.un * bn + s.ut1 * s.bt1 + s.ut2 * s.bt2;
  U[0] = s.rho; U[1] = s.rho * s.un; U[2] = s.rho * s.ut1; U[3] = s.rho * s.ut2; U[4] = e;
  F[0] = s.rho * s.un;
  F[1] = s.rho * s.un * s.un + pT - bn * bn;
  F[2] = s.rho * s.un * s.ut1 - bn * s.bt1;
  F[3] = s.rho * s.un * s.ut2 - bn * s.bt2;
  F[4] = (e + pT) * s.un - bn * vb;
}

// Local Lax-Friedrichs (Rusanov): F = (F_L+F_R)/2 - s (U_R-U_L)/2 with
// s = max(|u_L|+c_fL, |u_R|+c_fR).  Returns s.
template <class R>
R llf(const FState<R>& L, const FState<R>& Rs, R bn, R gamma, R F[5]) {
  R UL[5], FL[5], UR[5], FR[5], pTL, pTR;
  phys(L, bn, gamma, UL, FL, pTL);
  phys(Rs, bn, gamma, UR, FR, pTR);
  R cfL = fast_speed(L.rho, L.p, bn, L.bt1, L.bt2, gamma);
  R cfR = fast_speed(Rs.rho, Rs.p, bn, Rs.bt1, Rs.bt2, gamma);
  R s = rmax(rabs(L.un) + cfL, rabs(Rs.un) + cfR);
  for (int m = 0; m < 5; ++m) F[m] = R(0.5) * (FL[m] + FR[m]) - R(0.5) * s * (UR[m] - UL[m]);
  return s;
}

// HLL with the same outer speeds as HLLD (fallback; reading of the "HLL
// fallback" of the benchmark spec).
template <class R>
void hll(const R UL[5], const R FL[5], const R UR[5], const R FR[5], R SL, R SR, R F[5]) {
  if (SL >= R(0.0)) { for (int m = 0; m < 5; ++m) F[m] = FL[m]; return; }
  if (SR <= R(0.0)) { for (int m = 0; m < 5; ++m) F[m] = FR[m]; return; }
  for (int m = 0; m < 5; ++m)
    F[m] = (SR * FL[m] - SL * FR[m] + SL * SR * (UR[m] - UL[m])) / (SR - SL);
}

// HLLD (Miyoshi & Kusano 2005), restated from the published method.
// Outer speeds S_L, S_R as in eq. emf:alpha-pm (their eq. 67).  Returns 1 if
// the HLL fallback was taken.
// reading (degeneracies): the star transverse state equals the outer state if
// |rho_a (S_a-u_a)(S_a-S_M) - bn^2| <= 1e-12 (|rho_a (S_a-u_a)(S_a-S_M)| +
// bn^2); the double-star states are skipped (U** = U*) if bn^2 <= 1e-12 p_T*;
// HLL is used if rho*_L<=0, rho*_R<=0, p_T*<=0, S_L>=S_M, S_M>=S_R or any star
// quantity is not finite.  Flux selection order: S_L>0, S*_L>=0, S_M>=0,
// S*_R>=0, S_R>=0, else right.
// fan (optional, test hook): S_L, S_M, S_R, S*_L, S*_R, p_T*, then the states
// U*_L, U**_L, U**_R, U*_R as (rho, u_n, u_t1, u_t2, b_t1, b_t2, e_tot).
template <class R>
int hlld(const FState<R>& L, const FState<R>& Rs, R bn, R gamma, R F[5], R& SL, R& SR,
         R* fan = nullptr) {
  R UL[5], FL[5], UR[5], FR[5], pTL, pTR;
  phys(L, bn, gamma, UL, FL, pTL);
  phys(Rs, bn, gamma, UR, FR, pTR);
  R cfL = fast_speed(L.rho, L.p, bn, L.bt1, L.bt2, gamma);
  R cfR = fast_speed(Rs.rho, Rs.p, bn, Rs.bt1, Rs.bt2, gamma);
  R cmax = rmax(cfL, cfR);
  SL = rmin(L.un, Rs.un) - cmax;
  SR = rmax(L.un, Rs.un) + cmax;
  if (SL > R(0.0)) { for (int m = 0; m < 5; ++m) F[m] = FL[m]; return 0; }
  if (SR < R(0.0)) { for (int m = 0; m < 5; ++m) F[m] = FR[m]; return 0; }

  R dL = SL - L.un, dR = SR - Rs.un;
  R den = dR * Rs.rho - dL * L.rho;
  R SM = (dR * Rs.rho * Rs.un - dL * L.rho * L.un - pTR + pTL) / den;
  R pTs = (dR * Rs.rho * pTL - dL * L.rho * pTR + L.rho * Rs.rho * dR * dL * (Rs.un - L.un)) / den;
  R rsL = L.rho * dL / (SL - SM);
  R rsR = Rs.rho * dR / (SR - SM);

  bool bad = !(rsL > R(0.0)) || !(rsR > R(0.0)) || !(pTs > R(0.0)) || !(SL < SM) ||
             !(SM < SR) || !finite(SM) || !finite(pTs);
  R bn2 = bn * bn;

  // Star states on each side.
  auto star = [&](const FState<R>& s, const R U[5], R pT, R S, R rs, R& vs, R& ws, R& bys,
                  R& bzs, R& es) {
    R d = S - s.un;
    R dsm = S - SM;
    R q = s.rho * d * dsm - bn2;
    R ref = rabs(s.rho * d * dsm) + bn2;
    if (rabs(q) <= R(1e-12) * ref) {
      vs = s.ut1; ws = s.ut2; bys = s.bt1; bzs = s.bt2;
    } else {
      vs = s.ut1 - bn * s.bt1 * (SM - s.un) / q;
      ws = s.ut2 - bn * s.bt2 * (SM - s.un) / q;
      R f = (s.rho * d * d - bn2) / q;
      bys = s.bt1 * f;
      bzs = s.bt2 * f;
    }
    R vb = s.un * bn + s.ut1 * s.bt1 + s.ut2 * s.bt2;
    R vbs = SM * bn + vs * bys + ws * bzs;
    es = (d * U[4] - pT * s.un + pTs * SM + bn * (vb - vbs)) / dsm;
    (void)rs;
  };
  R vsL, wsL, bysL, bzsL, esL, vsR, wsR, bysR, bzsR, esR;
  star(L, UL, pTL, SL, rsL, vsL, wsL, bysL, bzsL, esL);
  star(Rs, UR, pTR, SR, rsR, vsR, wsR, bysR, bzsR, esR);
  bad = bad || !finite(vsL) || !finite(wsL) || !finite(bysL) || !finite(bzsL) || !finite(esL) ||
        !finite(vsR) || !finite(wsR) || !finite(bysR) || !finite(bzsR) || !finite(esR);
  if (bad) { hll(UL, FL, UR, FR, SL, SR, F); return 1; }

  R UsL[5] = {rsL, rsL * SM, rsL * vsL, rsL * wsL, esL};
  R UsR[5] = {rsR, rsR * SM, rsR * vsR, rsR * wsR, esR};

  R sqL = rsqrt(rsL), sqR = rsqrt(rsR);
  R SsL = SM, SsR = SM;
  R UssL[5], UssR[5];
  for (int m = 0; m < 5; ++m) { UssL[m] = UsL[m]; UssR[m] = UsR[m]; }
  R vssL = vsL, wssL = wsL, byssL = bysL, bzssL = bzsL;  // double-star transverse
  R vssR = vsR, wssR = wsR, byssR = bysR, bzssR = bzsR;  // (equal to star if skipped)
  if (!(bn2 <= R(1e-12) * pTs)) {
    R sg = sgn(bn);
    SsL = SM - rabs(bn) / sqL;
    SsR = SM + rabs(bn) / sqR;
    R sum = sqL + sqR;
    R vss = (sqL * vsL + sqR * vsR + (bysR - bysL) * sg) / sum;
    R wss = (sqL * wsL + sqR * wsR + (bzsR - bzsL) * sg) / sum;
    R byss = (sqL * bysR + sqR * bysL + sqL * sqR * (vsR - vsL) * sg) / sum;
    R bzss = (sqL * bzsR + sqR * bzsL + sqL * sqR * (wsR - wsL) * sg) / sum;
    R vbss = SM * bn + vss * byss + wss * bzss;
    R vbsL = SM * bn + vsL * bysL + wsL * bzsL;
    R vbsR = SM * bn + vsR * bysR + wsR * bzsR;
    R essL = esL - sqL * (vbsL - vbss) * sg;
    R essR = esR + sqR * (vbsR - vbss) * sg;
    UssL[2] = rsL * vss; UssL[3] = rsL * wss; UssL[4] = essL;
    UssR[2] = rsR * vss; UssR[3] = rsR * wss; UssR[4] = essR;
    vssL = vssR = vss; wssL = wssR = wss; byssL = byssR = byss; bzssL = bzssR = bzss;
  }
  if (fan) {
    R hdr[6] = {SL, SM, SR, SsL, SsR, pTs};
    R st[4][7] = {{rsL, SM, vsL, wsL, bysL, bzsL, esL},
                  {rsL, SM, vssL, wssL, byssL, bzssL, UssL[4]},
                  {rsR, SM, vssR, wssR, byssR, bzssR, UssR[4]},
                  {rsR, SM, vsR, wsR, bysR, bzsR, esR}};
    for (int m = 0; m < 6; ++m) fan[m] = hdr[m];
    for (int q = 0; q < 4; ++q)
      for (int m = 0; m < 7; ++m) fan[6 + 7 * q + m] = st[q][m];
  }

  if (SsL >= R(0.0)) {
    for (int m = 0; m < 5; ++m) F[m] = FL[m] + SL * (UsL[m] - UL[m]);
  } else if (SM >= R(0.0)) {
    for (int m = 0; m < 5; ++m) F[m] = FL[m] + SL * (UsL[m] - UL[m]) + SsL * (UssL[m] - UsL[m]);
  } else if (SsR >= R(0.0)) {
    for (int m = 0; m < 5; ++m) F[m] = FR[m] + SR * (UsR[m] - UR[m]) + SsR * (UssR[m] - UsR[m]);
  } else {
    for (int m = 0; m < 5; ++m) F[m] = FR[m] + SR * (UsR[m] - UR[m]);
  }
  return 0;
}

// --------------------------------------------------------------------------
// Face pass (Sec. 2.2 + eqs. emf:q26-facevel, emf:alpha-pm): for every x_a face
// reconstruct (rho, u_a, u_b, u_c, p, b_b, b_c) from both sides, solve the
// Riemann problem with the stored normal field, and keep F, alpha^{+/-} and
// the Q26 face-normal velocity u_a^*.
// --------------------------------------------------------------------------
template <class R>
int64_t face_pass(const Grid& g, const Params& P, int recon, int riemann, const State<R>& S,
                  const Prim<R>& W, FaceData<R>& FD) {
  const int64_t N = g.size();
  const R gamma = R(P.gamma);
  int64_t nfallback = 0;
  for (int a = 0; a < 3; ++a) {
    for (int m = 0; m < 5; ++m) FD.F[a][m].assign(N, R(0.0));
    FD.ap[a].assign(N, R(0.0)); FD.am[a].assign(N, R(0.0)); FD.us[a].assign(N, R(0.0));
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const Arr<R>* q[7] = {&W.rho, &W.u[a], &W.u[b], &W.u[c], &W.p, &W.b[b], &W.b[c]};
#pragma omp parallel for if (kPar<R>) reduction(+ : nfallback)
    for (int k = 0; k < g.n[2]; ++k)
      for (int j = 0; j < g.n[1]; ++j)
        for (int i = 0; i < g.n[0]; ++i) {
          P3 p{{i, j, k}};
          R lo[7], hi[7];
          for (int v = 0; v < 7; ++v) iface(g, recon, *q[v], p, a, lo[v], hi[v]);
          FState<R> sL{lo[0], lo[1], lo[2], lo[3], lo[4], lo[5], lo[6]};
          FState<R> sR{hi[0], hi[1], hi[2], hi[3], hi[4], hi[5], hi[6]};
          R bn = S.bf[a][g.idx(p.v)];
          R F[5], apv, amv;
          if (riemann == RIEMANN_HLLD) {
            R SL, SR;
            nfallback += hlld(sL, sR, bn, gamma, F, SL, SR);
            apv = rmax(R(0.0), SR);
            amv = rmax(R(0.0), -SL);
          } else {
            R s = llf(sL, sR, bn, gamma, F);
            apv = s; amv = s;  // reading: the FO EMF uses alpha^+ = alpha^- = s
          }
          // Face-local (n, t1, t2) momentum components back to (x0, x1, x2).
          int64_t f = g.idx(p.v);
          FD.F[a][0][f] = F[0];
          FD.F[a][1 + a][f] = F[1];
          FD.F[a][1 + b][f] = F[2];
          FD.F[a][1 + c][f] = F[3];
          FD.F[a][4][f] = F[4];
          FD.ap[a][f] = apv;
          FD.am[a][f] = amv;
          FD.us[a][f] = (apv * sL.un + amv * sR.un) / (apv + amv);
        }
  }
  return nfallback;
}

// --------------------------------------------------------------------------
// Edge EMFs (Sec. 2.3).  Edge c sits at the lower corner of cell p in the
// (a,b) plane with a = c+1, b = c+2 (cyclic).  "L/R" = sides along x_a,
// "B/T" = sides along x_b.  Corner order: LB, RB, LT, RT.
// --------------------------------------------------------------------------
template <class R>
void recon_pair_along(const Grid& g, int recon, const Arr<R>& A, const P3& p, int dir, R& lo,
                      R& hi) {
  iface(g, recon, A, p, dir, lo, hi);
}

// Two-step reconstruction of a cell-centred quantity to the edge, first along
// d1 to the x_d1 face through p, then along d2 to the edge.  Returns the
// value on the (s1, s2) side, s = 0 lower, 1 upper.
template <class R>
R recon_two_step(const Grid& g, int recon, const Arr<R>& A, const P3& p, int d1, int d2,
                 int s1, int s2) {
  R seq[6];
  for (int m = 0; m < 6; ++m) {
    P3 q = p.sh(d2, m - 3);
    R lo, hi;
    iface(g, recon, A, q, d1, lo, hi);
    seq[m] = s1 == 0 ? lo : hi;
  }
  // seq[m] sits at d2-offset m-3 relative to p; interface at p's lower d2 face.
  R dummy, lo, hi;
  recon1d(recon, seq + 0, dummy, lo);  // cell at offset -1: seq[0..4]
  recon1d(recon, seq + 1, hi, dummy);  // cell at offset  0: seq[1..5]
  return s2 == 0 ? lo : hi;
}

template <class R>
void edge_pass(const Grid& g, const Params& P, int recon, const State<R>& S, const Prim<R>& W,
               const FaceData<R>& FD, Arr<R> E[3]) {
  const int64_t N = g.size();
  for (int c = 0; c < 3; ++c) {
    E[c].assign(N, R(0.0));
    const int a = (c + 1) % 3, b = (c + 2) % 3;
    // Cell-centred EMF for the B25a scheme (eqs. emf:b25a-b-avg, b25a-emf-centre).
    Arr<R> ecell;
    if (P.emf == EMF_B25A) {
      ecell.assign(N, R(0.0));
      for (int64_t x = 0; x < N; ++x)
        ecell[x] = -W.u[a][x] * W.b[b][x] + W.u[b][x] * W.b[a][x];
    }
#pragma omp parallel for if (kPar<R>)
    for (int k = 0; k < g.n[2]; ++k)
      for (int j = 0; j < g.n[1]; ++j)
        for (int i = 0; i < g.n[0]; ++i) {
          P3 p{{i, j, k}};
          // Face field reconstructed to the edge (common to all schemes).
          R baB, baT, bbL, bbR;
          recon_pair_along(g, recon, S.bf[a], p, b, baB, baT);
          recon_pair_along(g, recon, S.bf[b], p, a, bbL, bbR);
          R eps[4];  // LB, RB, LT, RT
          if (P.emf == EMF_Q26) {
            // eq. emf:q26: u_a^* along x_b, u_b^* along x_a.
            R uaB, uaT, ubL, ubR;
            recon_pair_along(g, recon, FD.us[a], p, b, uaB, uaT);
            recon_pair_along(g, recon, FD.us[b], p, a, ubL, ubR);
            eps[0] = -uaB * bbL + ubL * baB;
            eps[1] = -uaB * bbR + ubR * baB;
            eps[2] = -uaT * bbL + ubL * baT;
            eps[3] = -uaT * bbR + ubR * baT;
          } else if (P.emf == EMF_B25A) {
            // eq. emf:b25a-average: mean of the [x_a x_b] and [x_b x_a] orders.
            for (int q = 0; q < 4; ++q) {
              int sa = q & 1, sb = q >> 1;
              R e_ab = recon_two_step(g, recon, ecell, p, a, b, sa, sb);
              R e_ba = recon_two_step(g, recon, ecell, p, b, a, sb, sa);
              eps[q] = R(0.5) * (e_ab + e_ba);
            }
          } else {
            // FS18, eqs. emf:fs18-average and emf:fs18.
            for (int q = 0; q < 4; ++q) {
              int sa = q & 1, sb = q >> 1;
              R ua = R(0.5) * (recon_two_step(g, recon, W.u[a], p, a, b, sa, sb) +
                               recon_two_step(g, recon, W.u[a], p, b, a, sb, sa));
              R ub = R(0.5) * (recon_two_step(g, recon, W.u[b], p, a, b, sa, sb) +
                               recon_two_step(g, recon, W.u[b], p, b, a, sb, sa));
              R bbX = sa == 0 ? bbL : bbR;
              R baY = sb == 0 ? baB : baT;
              eps[q] = -ua * bbX + ub * baY;
            }
          }
          // Edge wavespeeds, eq. emf:alpha-edge.
          int64_t fa0 = g.idx(p.sh(b, -1).v), fa1 = g.idx(p.v);
          int64_t fb0 = g.idx(p.sh(a, -1).v), fb1 = g.idx(p.v);
          R apa = rmax(FD.ap[a][fa0], FD.ap[a][fa1]);
          R ama = rmax(FD.am[a][fa0], FD.am[a][fa1]);
          R apb = rmax(FD.ap[b][fb0], FD.ap[b][fb1]);
          R amb = rmax(FD.am[b][fb0], FD.am[b][fb1]);
          // LD04 averaging, eq. emf:ld04.
          R e = (apa * apb * eps[0] + ama * apb * eps[1]) / ((apa + ama) * (apb + amb)) +
                (apa * amb * eps[2] + ama * amb * eps[3]) / ((apa + ama) * (apb + amb)) -
                apb * amb / (apb + amb) * (baT - baB) + apa * ama / (apa + ama) * (bbR - bbL);
          // Ohmic term, eqs. resistivity:current-stencil and emf-update.
          if (P.eta > 0.0) {
            R jc = (S.bf[b][g.idx(p.v)] - S.bf[b][g.idx(p.sh(a, -1).v)]) / R(g.dx[a]) -
                   (S.bf[a][g.idx(p.v)] - S.bf[a][g.idx(p.sh(b, -1).v)]) / R(g.dx[b]);
            e = e + R(P.eta) * jc;
          }
          E[c][g.idx(p.v)] = e;
        }
  }
}

// Joule-heating energy flux (Sec. 2.4, last paragraph).  reading: at an x_a
// face, F_E += ebar_b * bbar_c - ebar_c * bbar_b, with ebar the mean of
// eta j over the face's two bounding edges of that direction and bbar the mean
// of the two adjacent cells' cell-averaged field.
template <class R>
void joule_flux(const Grid& g, const Params& P, const State<R>& S, const Prim<R>& W,
                Arr<R> F[3][5]) {
  if (!(P.eta > 0.0)) return;
  const int64_t N = g.size();
  Arr<R> ej[3];
  for (int c = 0; c < 3; ++c) {
    ej[c].assign(N, R(0.0));
    const int a = (c + 1) % 3, b = (c + 2) % 3;
    for (int k = 0; k < g.n[2]; ++k)
      for (int j = 0; j < g.n[1]; ++j)
        for (int i = 0; i < g.n[0]; ++i) {
          P3 p{{i, j, k}};
          R jc = (S.bf[b][g.idx(p.v)] - S.bf[b][g.idx(p.sh(a, -1).v)]) / R(g.dx[a]) -
                 (S.bf[a][g.idx(p.v)] - S.bf[a][g.idx(p.sh(b, -1).v)]) / R(g.dx[b]);
          ej[c][g.idx(p.v)] = R(P.eta) * jc;
        }
  }
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    for (int k = 0; k < g.n[2]; ++k)
      for (int j = 0; j < g.n[1]; ++j)
        for (int i = 0; i < g.n[0]; ++i) {
          P3 p{{i, j, k}};
          int64_t f = g.idx(p.v);
          R eb = R(0.5) * (ej[b][f] + ej[b][g.idx(p.sh(c, 1).v)]);
          R ec = R(0.5) * (ej[c][f] + ej[c][g.idx(p.sh(b, 1).v)]);
          int64_t cl = g.idx(p.sh(a, -1).v);
          R bb = R(0.5) * (W.b[b][cl] + W.b[b][f]);
          R bc = R(0.5) * (W.b[c][cl] + W.b[c][f]);
          F[a][4][f] = F[a][4][f] + (eb * bc - ec * bb);
        }
  }
}

// Full flux and EMF evaluation on one state (Sec. 2.2-2.4).
template <class R>
int64_t fluxes(const Grid& g, const Params& P, int recon, int riemann, const State<R>& S,
               Fluxes<R>& out) {
  Prim<R> W;
  g_phase = PH_PRIM;
  to_prim(g, P, S, W);
  FaceData<R> FD;
  g_phase = PH_FACE;
  int64_t nfb = face_pass(g, P, recon, riemann, S, W, FD);
  g_phase = PH_EMF;
  edge_pass(g, P, recon, S, W, FD, out.E);
  joule_flux(g, P, S, W, FD.F);
  for (int a = 0; a < 3; ++a)
    for (int m = 0; m < 5; ++m) out.F[a][m] = std::move(FD.F[a][m]);
  return nfb;
}

// Increments D[S_c] (eq. rk:increment-state) and D[b] (eq. rk:increment-bfield).
template <class R>
void increments(const Grid& g, R dt, const Fluxes<R>& X, Arr<R> DS[5], Arr<R> DB[3]) {
  const int64_t N = g.size();
  for (int m = 0; m < 5; ++m) DS[m].assign(N, R(0.0));
  for (int a = 0; a < 3; ++a) DB[a].assign(N, R(0.0));
#pragma omp parallel for if (kPar<R>)
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        P3 p{{i, j, k}};
        int64_t c = g.idx(p.v);
        int64_t up[3] = {g.idx(p.sh(0, 1).v), g.idx(p.sh(1, 1).v), g.idx(p.sh(2, 1).v)};
        for (int m = 0; m < 5; ++m) {
          R s = (X.F[0][m][c] - X.F[0][m][up[0]]) / R(g.dx[0]) +
                (X.F[1][m][c] - X.F[1][m][up[1]]) / R(g.dx[1]) +
                (X.F[2][m][c] - X.F[2][m][up[2]]) / R(g.dx[2]);
          DS[m][c] = dt * s;
        }
        // face b_a at the lower x_a face of p; b = a+1, c = a+2
        for (int a = 0; a < 3; ++a) {
          const int b = (a + 1) % 3, cc = (a + 2) % 3;
          R dxb = R(g.dx[b]), dxc = R(g.dx[cc]);
          R circ = dxc * X.E[cc][c] + dxb * X.E[b][g.idx(p.sh(cc, 1).v)] -
                   dxc * X.E[cc][g.idx(p.sh(b, 1).v)] - dxb * X.E[b][c];
          DB[a][c] = dt / (dxb * dxc) * circ;
        }
      }
}

// Invalid-state test (Sec. 2.5).  reading: rho <= 0, p <= 0 or any
// non-finite value (bitmask of the enabled criteria).
template <class R>
void flag_cells(const Grid& g, const Params& P, const State<R>& S, std::vector<uint8_t>& flag) {
  const int64_t N = g.size();
  flag.assign(N, 0);
  const double gm1 = P.gamma - 1.0;
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        int64_t c = g.idx(i, j, k);
        double rho = val(S.c[0][c]);
        double m2 = 0.0, b2 = 0.0;
        bool nonfinite = false;
        for (int m = 0; m < 5; ++m) nonfinite |= !std::isfinite(val(S.c[m][c]));
        for (int d = 0; d < 3; ++d) {
          P3 q{{i, j, k}};
          double bl = val(S.bf[d][c]);
          double bu = val(S.bf[d][g.idx(q.sh(d, 1).v)]);
          nonfinite |= !std::isfinite(bl) || !std::isfinite(bu);
          double bc = 0.5 * (bl + bu);
          double u = val(S.c[1 + d][c]) / rho;
          m2 += rho * u * u;
          b2 += bc * bc;
        }
        double p = gm1 * (val(S.c[4][c]) - 0.5 * m2 - 0.5 * b2);
        bool bad = false;
        if ((P.flag_mask & FLAG_RHO) && !(rho > 0.0)) bad = true;
        if ((P.flag_mask & FLAG_P) && !(p > 0.0)) bad = true;
        if ((P.flag_mask & FLAG_NONFINITE) && (nonfinite || !std::isfinite(p))) bad = true;
        flag[c] = bad ? 1 : 0;
      }
}

// Replace fluxes on faces touching a flagged cell, and EMFs on edges touching
// one, by the first-order values (Sec. 2.5).  Marks what was replaced.
template <class R>
void replace_fo(const Grid& g, const std::vector<uint8_t>& flag, const Fluxes<R>& FO,
                Fluxes<R>& X, std::vector<uint8_t>& face_rep, std::vector<uint8_t>& edge_rep) {
  const int64_t N = g.size();
  face_rep.assign(3 * N, 0);
  edge_rep.assign(3 * N, 0);
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        P3 p{{i, j, k}};
        int64_t c = g.idx(p.v);
        for (int a = 0; a < 3; ++a) {
          if (flag[c] || flag[g.idx(p.sh(a, -1).v)]) {
            for (int m = 0; m < 5; ++m) X.F[a][m][c] = FO.F[a][m][c];
            face_rep[a * N + c] = 1;
          }
          const int ea = (a + 1) % 3, eb = (a + 2) % 3;  // edge along a
          P3 q1 = p.sh(ea, -1), q2 = p.sh(eb, -1), q3 = q1.sh(eb, -1);
          if (flag[c] || flag[g.idx(q1.v)] || flag[g.idx(q2.v)] || flag[g.idx(q3.v)]) {
            X.E[a][c] = FO.E[a][c];
            edge_rep[a * N + c] = 1;
          }
        }
      }
}

// --------------------------------------------------------------------------
// One full step (Sec. 2.5, eqs. rk1:update and rk2:update with FOFC).
// force1/force2: optional per-cell masks OR-ed into the flags of each stage
// (test hook).  diag: [flagged stage 1, flagged stage 2, HLL fallbacks,
// non-finite].
// --------------------------------------------------------------------------
template <class R>
void step(const Grid& g, const Params& P, State<R>& S, R dt, const uint8_t* force1,
          const uint8_t* force2, int64_t diag[4]) {
  const int64_t N = g.size();
  State<R> Sn = S;

  Fluxes<R> FO;
  if (P.fofc) {
    g_phase = PH_FOFC;
    Prim<R> W;
    to_prim(g, P, Sn, W);
    FaceData<R> FD;
    face_pass(g, P, RECON_PC, RIEMANN_LLF, Sn, W, FD);
    edge_pass(g, P, RECON_PC, Sn, W, FD, FO.E);
    joule_flux(g, P, Sn, W, FD.F);
    for (int a = 0; a < 3; ++a)
      for (int m = 0; m < 5; ++m) FO.F[a][m] = std::move(FD.F[a][m]);
  }

  // Stage 1.
  Fluxes<R> H1;
  diag[2] += fluxes(g, P, P.recon, P.riemann, Sn, H1);
  g_phase = PH_UPDATE;
  Arr<R> D1S[5], D1B[3];
  increments(g, dt, H1, D1S, D1B);
  State<R> Sh = Sn;
  for (int m = 0; m < 5; ++m)
    for (int64_t x = 0; x < N; ++x) Sh.c[m][x] = Sn.c[m][x] + D1S[m][x];
  for (int a = 0; a < 3; ++a)
    for (int64_t x = 0; x < N; ++x) Sh.bf[a][x] = Sn.bf[a][x] + D1B[a][x];

  std::vector<uint8_t> flag, frep, erep;
  if (P.fofc) {
    flag_cells(g, P, Sh, flag);
    if (force1)
      for (int64_t x = 0; x < N; ++x) flag[x] |= force1[x];
    int64_t nflag = 0;
    for (int64_t x = 0; x < N; ++x) nflag += flag[x];
    diag[0] += nflag;
    if (nflag) {
      replace_fo(g, flag, FO, H1, frep, erep);
      // Recompute the stage from the final fluxes; unaffected cells and
      // faces reproduce their values exactly.
      increments(g, dt, H1, D1S, D1B);
      for (int m = 0; m < 5; ++m)
        for (int64_t x = 0; x < N; ++x) Sh.c[m][x] = Sn.c[m][x] + D1S[m][x];
      for (int a = 0; a < 3; ++a)
        for (int64_t x = 0; x < N; ++x) Sh.bf[a][x] = Sn.bf[a][x] + D1B[a][x];
    }
  }

  // Stage 2.
  Fluxes<R> H2;
  diag[2] += fluxes(g, P, P.recon, P.riemann, Sh, H2);
  g_phase = PH_UPDATE;
  Arr<R> D2S[5], D2B[3];
  increments(g, dt, H2, D2S, D2B);
  for (int m = 0; m < 5; ++m)
    for (int64_t x = 0; x < N; ++x) S.c[m][x] = Sn.c[m][x] + R(0.5) * (D1S[m][x] + D2S[m][x]);
  for (int a = 0; a < 3; ++a)
    for (int64_t x = 0; x < N; ++x) S.bf[a][x] = Sn.bf[a][x] + R(0.5) * (D1B[a][x] + D2B[a][x]);

  if (P.fofc) {
    flag_cells(g, P, S, flag);
    if (force2)
      for (int64_t x = 0; x < N; ++x) flag[x] |= force2[x];
    int64_t nflag = 0;
    for (int64_t x = 0; x < N; ++x) nflag += flag[x];
    diag[1] += nflag;
    if (nflag) {
      // RK-averaged fluxes and EMFs, replaced outright by FO where needed.
      Fluxes<R> Avg;
      for (int a = 0; a < 3; ++a) {
        for (int m = 0; m < 5; ++m) {
          Avg.F[a][m].assign(N, R(0.0));
          for (int64_t x = 0; x < N; ++x)
            Avg.F[a][m][x] = R(0.5) * (H1.F[a][m][x] + H2.F[a][m][x]);
        }
        Avg.E[a].assign(N, R(0.0));
        for (int64_t x = 0; x < N; ++x) Avg.E[a][x] = R(0.5) * (H1.E[a][x] + H2.E[a][x]);
      }
      replace_fo(g, flag, FO, Avg, frep, erep);
      Arr<R> DAS[5], DAB[3];
      increments(g, dt, Avg, DAS, DAB);
      // Cells with a replaced face, faces with a replaced bounding edge.
      for (int k = 0; k < g.n[2]; ++k)
        for (int j = 0; j < g.n[1]; ++j)
          for (int i = 0; i < g.n[0]; ++i) {
            P3 p{{i, j, k}};
            int64_t c = g.idx(p.v);
            bool cell_aff = false;
            for (int a = 0; a < 3; ++a)
              cell_aff = cell_aff || frep[a * N + c] || frep[a * N + g.idx(p.sh(a, 1).v)];
            if (cell_aff)
              for (int m = 0; m < 5; ++m) S.c[m][c] = Sn.c[m][c] + DAS[m][c];
            for (int a = 0; a < 3; ++a) {
              const int b = (a + 1) % 3, cc = (a + 2) % 3;
              bool face_aff = erep[cc * N + c] || erep[cc * N + g.idx(p.sh(b, 1).v)] ||
                              erep[b * N + c] || erep[b * N + g.idx(p.sh(cc, 1).v)];
              if (face_aff) S.bf[a][c] = Sn.bf[a][c] + DAB[a][c];
            }
          }
    }
  }
  g_phase = PH_DT;
}

template <class R>
void load_state(const Grid& g, const double* cons, const double* bface, State<R>& S) {
  const int64_t N = g.size();
  for (int m = 0; m < 5; ++m) {
    S.c[m].resize(N);
    for (int64_t x = 0; x < N; ++x) S.c[m][x] = R(cons[m * N + x]);
  }
  for (int a = 0; a < 3; ++a) {
    S.bf[a].resize(N);
    for (int64_t x = 0; x < N; ++x) S.bf[a][x] = R(bface[a * N + x]);
  }
}

}  // namespace orc

using namespace orc;

extern "C" {

// Advance nsteps.  cons: 5*N doubles (rho, m0, m1, m2, e_tot), bface: 3*N
// (b_a at the lower x_a face of each cell); both x-fastest, interior only.
// dt_fixed: nsteps values or NULL (CFL dt).  dt_out: nsteps values or NULL.
// diag: 4 int64 accumulated over the steps.  force: 2*N uint8 (stage 1 mask,
// stage 2 mask) applied to every step, or NULL.
int oracle_step(const Params* P, const int n[3], const double dx[3], double* cons, double* bface,
                int nsteps, const double* dt_fixed, double* dt_out, int64_t* diag,
                const uint8_t* force) {
  Grid g{{n[0], n[1], n[2]}, {dx[0], dx[1], dx[2]}};
  const int64_t N = g.size();
  State<double> S;
  load_state(g, cons, bface, S);
  int64_t dg[4] = {0, 0, 0, 0};
  for (int s = 0; s < nsteps; ++s) {
    double dt;
    if (dt_fixed) {
      dt = dt_fixed[s];
    } else {
      Prim<double> W;
      to_prim(g, *P, S, W);
      dt = compute_dt(g, *P, W);
    }
    if (dt_out) dt_out[s] = dt;
    if (!std::isfinite(dt)) { dg[3] += 1; break; }
    step(g, *P, S, dt, force ? force : nullptr, force ? force + N : nullptr, dg);
  }
  for (int m = 0; m < 5; ++m) std::memcpy(cons + m * N, S.c[m].data(), N * sizeof(double));
  for (int a = 0; a < 3; ++a) std::memcpy(bface + a * N, S.bf[a].data(), N * sizeof(double));
  if (diag)
    for (int q = 0; q < 4; ++q) diag[q] = dg[q];
  return 0;
}

// Forward-mode derivative through nsteps with frozen dt values: on entry
// (cons, bface) is the state and (tcons, tbface) its tangent; on exit both
// are advanced.
int oracle_step_dual(const Params* P, const int n[3], const double dx[3], double* cons,
                     double* bface, double* tcons, double* tbface, int nsteps,
                     const double* dt_fixed) {
  Grid g{{n[0], n[1], n[2]}, {dx[0], dx[1], dx[2]}};
  const int64_t N = g.size();
  State<Dual> S;
  for (int m = 0; m < 5; ++m) {
    S.c[m].resize(N);
    for (int64_t x = 0; x < N; ++x) S.c[m][x] = Dual(cons[m * N + x], tcons[m * N + x]);
  }
  for (int a = 0; a < 3; ++a) {
    S.bf[a].resize(N);
    for (int64_t x = 0; x < N; ++x) S.bf[a][x] = Dual(bface[a * N + x], tbface[a * N + x]);
  }
  int64_t dg[4] = {0, 0, 0, 0};
  for (int s = 0; s < nsteps; ++s) step(g, *P, S, Dual(dt_fixed[s]), nullptr, nullptr, dg);
  for (int m = 0; m < 5; ++m)
    for (int64_t x = 0; x < N; ++x) { cons[m * N + x] = S.c[m][x].v; tcons[m * N + x] = S.c[m][x].d; }
  for (int a = 0; a < 3; ++a)
    for (int64_t x = 0; x < N; ++x) { bface[a * N + x] = S.bf[a][x].v; tbface[a * N + x] = S.bf[a][x].d; }
  return (int)(dg[0] + dg[1]);
}

// Count the arithmetic of one step (dt from the CFL condition included).
// counts: PH_N x OP_N int64, phases (dt, prim, face, emf, update, fofc,
// recon) and ops (add/sub, mul, div, sqrt, compare); recon_calls: number of
// 1D reconstructions performed.
int oracle_count_step(const Params* P, const int n[3], const double dx[3], const double* cons,
                      const double* bface, int64_t* counts, int64_t* recon_calls) {
  Grid g{{n[0], n[1], n[2]}, {dx[0], dx[1], dx[2]}};
  std::memset(g_count, 0, sizeof(g_count));
  g_recon_calls = 0;
  State<Count> S;
  load_state(g, cons, bface, S);
  g_phase = PH_PRIM;
  Prim<Count> W;
  to_prim(g, *P, S, W);
  g_phase = PH_DT;
  Count dt = compute_dt(g, *P, W);
  // The prim conversion used for dt is part of the dt pass.
  for (int o = 0; o < OP_N; ++o) { g_count[PH_DT][o] += g_count[PH_PRIM][o]; g_count[PH_PRIM][o] = 0; }
  int64_t dg[4] = {0, 0, 0, 0};
  step(g, *P, S, dt, nullptr, nullptr, dg);
  std::memcpy(counts, g_count, sizeof(g_count));
  if (recon_calls) *recon_calls = g_recon_calls;
  return 0;
}

// Threads the parallel loops use.
int oracle_num_threads(void) { return omp_get_max_threads(); }
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

// ---- unit-level entry points used by the pinning tests -------------------
void oracle_recon1d(int method, const double q[5], double* qm, double* qp) {
  recon1d<double>(method, q, *qm, *qp);
}

// The HLLD wave fan (34 values, see hlld()); returns 1 on HLL fallback.
int oracle_hlld_fan(const double* L, const double* Rr, double bn, double gamma, double* fan) {
  FState<double> a{L[0], L[1], L[2], L[3], L[4], L[5], L[6]};
  FState<double> b{Rr[0], Rr[1], Rr[2], Rr[3], Rr[4], Rr[5], Rr[6]};
  double F[5], SL, SR;
  return hlld<double>(a, b, bn, gamma, F, SL, SR, fan);
}

// state: rho, un, ut1, ut2, p, bt1, bt2
int oracle_hlld(const double* L, const double* Rr, double bn, double gamma, double* F,
                double* SL, double* SR) {
  FState<double> a{L[0], L[1], L[2], L[3], L[4], L[5], L[6]};
  FState<double> b{Rr[0], Rr[1], Rr[2], Rr[3], Rr[4], Rr[5], Rr[6]};
  return hlld<double>(a, b, bn, gamma, F, *SL, *SR);
}

double oracle_llf(const double* L, const double* Rr, double bn, double gamma, double* F) {
  FState<double> a{L[0], L[1], L[2], L[3], L[4], L[5], L[6]};
  FState<double> b{Rr[0], Rr[1], Rr[2], Rr[3], Rr[4], Rr[5], Rr[6]};
  return llf<double>(a, b, bn, gamma, F);
}

void oracle_hll(const double* L, const double* Rr, double bn, double gamma, double* F) {
  FState<double> a{L[0], L[1], L[2], L[3], L[4], L[5], L[6]};
  FState<double> b{Rr[0], Rr[1], Rr[2], Rr[3], Rr[4], Rr[5], Rr[6]};
  double UL[5], FL[5], UR[5], FR[5], pL, pR;
  phys(a, bn, gamma, UL, FL, pL);
  phys(b, bn, gamma, UR, FR, pR);
  double cfL = fast_speed(a.rho, a.p, bn, a.bt1, a.bt2, gamma);
  double cfR = fast_speed(b.rho, b.p, bn, b.bt1, b.bt2, gamma);
  double cm = std::max(cfL, cfR);
  hll<double>(UL, FL, UR, FR, std::min(a.un, b.un) - cm, std::max(a.un, b.un) + cm, F);
}

double oracle_fast_speed(double rho, double p, double bn, double bt1, double bt2, double gamma) {
  return fast_speed<double>(rho, p, bn, bt1, bt2, gamma);
}

// CFL time step of a state (no step taken).
double oracle_dt(const Params* P, const int n[3], const double dx[3], const double* cons,
                 const double* bface) {
  Grid g{{n[0], n[1], n[2]}, {dx[0], dx[1], dx[2]}};
  State<double> S;
  load_state(g, cons, bface, S);
  Prim<double> W;
  to_prim(g, *P, S, W);
  return compute_dt(g, *P, W);
}

// Edge EMFs and face fluxes of one state (for component-level checks):
// F: 3*5*N, E: 3*N.
int oracle_fluxes(const Params* P, const int n[3], const double dx[3], const double* cons,
                  const double* bface, int recon, int riemann, double* F, double* E) {
  Grid g{{n[0], n[1], n[2]}, {dx[0], dx[1], dx[2]}};
  const int64_t N = g.size();
  State<double> S;
  load_state(g, cons, bface, S);
  Fluxes<double> X;
  int64_t nfb = fluxes(g, *P, recon, riemann, S, X);
  for (int a = 0; a < 3; ++a) {
    for (int m = 0; m < 5; ++m) std::memcpy(F + (a * 5 + m) * N, X.F[a][m].data(), N * sizeof(double));
    std::memcpy(E + a * N, X.E[a].data(), N * sizeof(double));
  }
  return (int)nfb;
}

}  // extern "C"
