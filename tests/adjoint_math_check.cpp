// CPU check of the reverse-mode per-point arithmetic of the HIP path
// (ctmhd_adjoint_math.h) against central finite differences of the forward
// per-point arithmetic (ctmhd_math.h): for random inputs x, output weights
// yb and directions dx, the adjoint xb must satisfy
//   xb . dx = d/dh [ yb . f(x + h dx) ]  (central difference, h small).
// Built as host code by tests/test_adjoint_math.py; exit status 0 = pass.
#include <cmath>
#include <cstdio>
#include <random>

#include "ctmhd_adjoint_math.h"

using namespace ctmhd;

static std::mt19937_64 rng(12345);
static double U(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }

static int g_fail = 0;
static void report(const char* what, double worst, double tol) {
  std::printf("%-34s worst relative mismatch %.3e (tol %.0e) %s\n", what, worst, tol,
              worst <= tol ? "ok" : "FAIL");
  if (!(worst <= tol)) ++g_fail;
}

// mismatch relative to the L1 size sc of the terms of the directional
// derivative (a sum of terms may cancel; its error scales with the terms)
static double relmis(double ad, double fd, double sc) {
  return std::fabs(ad - fd) / (sc + 1e-12);
}

static FState<double> rand_state(double umax) {
  FState<double> s;
  s.rho = U(0.3, 2.0);
  s.un = U(-umax, umax);
  s.ut1 = U(-1, 1);
  s.ut2 = U(-1, 1);
  s.p = U(0.2, 2.0);
  s.bt1 = U(-1.5, 1.5);
  s.bt2 = U(-1.5, 1.5);
  return s;
}

static double* fs_ptr(FState<double>& s, int k) {
  double* p[7] = {&s.rho, &s.un, &s.ut1, &s.ut2, &s.p, &s.bt1, &s.bt2};
  return p[k];
}

// ---- fast speed ----
static void check_fast() {
  double worst = 0;
  for (int it = 0; it < 2000; ++it) {
    double x[5] = {U(0.3, 2), U(0.1, 2), U(-1.5, 1.5), U(-1.5, 1.5), U(-1.5, 1.5)};
    double dx[5];
    for (double& d : dx) d = U(-1, 1);
    const double g = 5.0 / 3.0, cb = U(-1, 1);
    double xb[5] = {0, 0, 0, 0, 0};
    fast_speed_adj(x[0], x[1], x[2], x[3], x[4], g, cb, xb[0], xb[1], xb[2], xb[3], xb[4]);
    double ad = 0, sc = 0;
    for (int k = 0; k < 5; ++k) {
      ad += xb[k] * dx[k];
      sc += std::fabs(xb[k] * dx[k]);
    }
    const double h = 1e-6;
    double xp[5], xm[5];
    for (int k = 0; k < 5; ++k) {
      xp[k] = x[k] + h * dx[k];
      xm[k] = x[k] - h * dx[k];
    }
    double fd = cb * (fast_speed(xp[0], xp[1], xp[2], xp[3], xp[4], g) -
                      fast_speed(xm[0], xm[1], xm[2], xm[3], xm[4], g)) / (2 * h);
    worst = std::fmax(worst, relmis(ad, fd, sc));
  }
  report("fast_speed_adj", worst, 1e-7);
}

// ---- ideal-MHD flux ----
static void check_phys() {
  double worst = 0;
  const double g = 5.0 / 3.0, gm1inv = 1.0 / (g - 1.0);
  for (int it = 0; it < 2000; ++it) {
    FState<double> s = rand_state(2), ds = rand_state(1);
    double bn = U(-1.5, 1.5), dbn = U(-1, 1);
    double Ub[5], Fb[5], pTb = U(-1, 1);
    for (int m = 0; m < 5; ++m) {
      Ub[m] = U(-1, 1);
      Fb[m] = U(-1, 1);
    }
    FState<double> sb;
    fstate_zero(sb);
    double bnb = 0;
    phys_flux_adj(s, bn, gm1inv, Ub, Fb, pTb, sb, bnb);
    double ad = bnb * dbn, sc = std::fabs(bnb * dbn);
    for (int k = 0; k < 7; ++k) {
      ad += *fs_ptr(sb, k) * *fs_ptr(ds, k);
      sc += std::fabs(*fs_ptr(sb, k) * *fs_ptr(ds, k));
    }
    auto J = [&](double h) {
      FState<double> t = s;
      for (int k = 0; k < 7; ++k) *fs_ptr(t, k) += h * *fs_ptr(ds, k);
      double UU[5], FF[5], pT;
      phys_flux(t, bn + h * dbn, gm1inv, UU, FF, pT);
      double j = pTb * pT;
      for (int m = 0; m < 5; ++m) j += Ub[m] * UU[m] + Fb[m] * FF[m];
      return j;
    };
    const double h = 1e-6;
    worst = std::fmax(worst, relmis(ad, (J(h) - J(-h)) / (2 * h), sc));
  }
  report("phys_flux_adj", worst, 1e-7);
}

// HLLD region of an input pair, for the coverage census: 0 F = FL, 1 left
// star, 2 left double star, 3 right double star, 4 right star, 5 F = FR
// (the double-star regions only when the double-star states exist).
static int hlld_region(const FState<double>& L, const FState<double>& R, double bn, double g) {
  const double gm1inv = 1.0 / (g - 1.0);
  double UL[5], FL[5], UR[5], FR[5], pTL, pTR;
  phys_flux(L, bn, gm1inv, UL, FL, pTL);
  phys_flux(R, bn, gm1inv, UR, FR, pTR);
  const double c = std::fmax(fast_speed(L.rho, L.p, bn, L.bt1, L.bt2, g),
                             fast_speed(R.rho, R.p, bn, R.bt1, R.bt2, g));
  const double SL = std::fmin(L.un, R.un) - c, SR = std::fmax(L.un, R.un) + c;
  if (SL > 0) return 0;
  if (SR < 0) return 5;
  const double mL = (SL - L.un) * L.rho, mR = (SR - R.un) * R.rho;
  const double SM = (mR * R.un - mL * L.un - pTR + pTL) / (mR - mL);
  const double pTs = (mR * pTL - mL * pTR + mL * mR * (R.un - L.un)) / (mR - mL);
  const double rsL = mL / (SL - SM), rsR = mR / (SR - SM);
  double SsL = SM, SsR = SM;
  if (!(bn * bn <= 1e-12 * pTs)) {
    SsL = SM - std::fabs(bn) / std::sqrt(rsL);
    SsR = SM + std::fabs(bn) / std::sqrt(rsR);
  }
  if (SsL >= 0) return 1;
  if (SM >= 0) return 2;
  if (SsR >= 0) return 3;
  return 4;
}

// ---- face outputs (Riemann solver + alpha +- + u*) ----
template <int RIEMANN>
static void check_face(const char* name, double umax, double bnmax, int* regions) {
  double worst = 0;
  const double g = 5.0 / 3.0;
  int n = 0;
  for (int it = 0; it < 20000 && n < 4000; ++it) {
    FState<double> L = rand_state(umax), R = rand_state(umax);
    double bn = U(-bnmax, bnmax);
    // classify the HLLD region; skip inputs within a finite-difference step
    // of a region boundary or of the fallback
    double F[5], SL, SR;
    int fb = hlld_flux(L, R, bn, g, F, SL, SR);
    if (RIEMANN == kHLLD) {
      if (fb) continue;
      if (std::fabs(SL) < 1e-3 || std::fabs(SR) < 1e-3) continue;
    }
    FState<double> dL = rand_state(1), dR = rand_state(1);
    double dbn = U(-1, 1);
    double Fb[5];
    for (double& v : Fb) v = U(-1, 1);
    double apb = U(-1, 1), amb = U(-1, 1), usb = U(-1, 1);
    auto J = [&](double h) {
      FState<double> l = L, r = R;
      for (int k = 0; k < 7; ++k) {
        *fs_ptr(l, k) += h * *fs_ptr(dL, k);
        *fs_ptr(r, k) += h * *fs_ptr(dR, k);
      }
      double b = bn + h * dbn, FF[5], ap, am;
      if (RIEMANN == kHLLD) {
        double sl, sr;
        hlld_flux(l, r, b, g, FF, sl, sr);
        ap = std::fmax(0.0, sr);
        am = std::fmax(0.0, -sl);
      } else {
        ap = am = llf_flux(l, r, b, g, FF);
      }
      double us = (ap * l.un + am * r.un) / (ap + am);
      double j = apb * ap + amb * am + usb * us;
      for (int m = 0; m < 5; ++m) j += Fb[m] * FF[m];
      return j;
    };
    const double h = 1e-7;
    double jp = J(h), jm = J(-h), j0 = J(0);
    // skip kinks (a branch change inside [-h, h]): second difference large
    if (std::fabs(jp - 2 * j0 + jm) > 1e-9 * (std::fabs(j0) + 1)) continue;
    FState<double> Lb, Rb;
    fstate_zero(Lb);
    fstate_zero(Rb);
    double bnb = 0;
    face_outputs_adj<RIEMANN>(L, R, bn, g, Fb, apb, amb, usb, Lb, Rb, bnb);
    double ad = bnb * dbn, sc = std::fabs(bnb * dbn);
    for (int k = 0; k < 7; ++k) {
      ad += *fs_ptr(Lb, k) * *fs_ptr(dL, k) + *fs_ptr(Rb, k) * *fs_ptr(dR, k);
      sc += std::fabs(*fs_ptr(Lb, k) * *fs_ptr(dL, k)) + std::fabs(*fs_ptr(Rb, k) * *fs_ptr(dR, k));
    }
    const double fd = (jp - jm) / (2 * h);
    const double e = relmis(ad, fd, sc);
    if (e > 1e-5 && g_fail < 50)
      std::printf("  %s mismatch %.3e: ad %.10e fd %.10e (SL %.3f SR %.3f bn %.3f)\n", name, e, ad,
                  fd, SL, SR, bn);
    worst = std::fmax(worst, e);
    ++n;
    if (regions && RIEMANN == kHLLD) regions[hlld_region(L, R, bn, g)]++;
  }
  char label[64];
  std::snprintf(label, sizeof(label), "%s (%d samples)", name, n);
  report(label, worst, 1e-6);
}

// ---- LD04 with Q26 corners ----
static void check_ld04() {
  double worst = 0;
  for (int it = 0; it < 2000; ++it) {
    double u[4], b[4], al[4], du[4], db[4], dal[4];
    for (int k = 0; k < 4; ++k) {
      u[k] = U(-2, 2);
      b[k] = U(-2, 2);
      al[k] = U(0.2, 3);
      du[k] = U(-1, 1);
      db[k] = U(-1, 1);
      dal[k] = U(-1, 1);
    }
    const double Eb = U(-1, 1);
    auto E = [&](double h) {
      double uu[4], bb[4], aa[4];
      for (int k = 0; k < 4; ++k) {
        uu[k] = u[k] + h * du[k];
        bb[k] = b[k] + h * db[k];
        aa[k] = al[k] + h * dal[k];
      }
      double e0 = -uu[0] * bb[2] + uu[2] * bb[0], e1 = -uu[0] * bb[3] + uu[3] * bb[0];
      double e2 = -uu[1] * bb[2] + uu[2] * bb[1], e3 = -uu[1] * bb[3] + uu[3] * bb[1];
      return Eb * ld04(e0, e1, e2, e3, aa[0], aa[1], aa[2], aa[3], bb[0], bb[1], bb[2], bb[3]);
    };
    double ub[4] = {0, 0, 0, 0}, bb[4] = {0, 0, 0, 0}, alb[4] = {0, 0, 0, 0};
    q26_ld04_adj(u, b, al, Eb, ub, bb, alb);
    double ad = 0, sc = 0;
    for (int k = 0; k < 4; ++k) {
      ad += ub[k] * du[k] + bb[k] * db[k] + alb[k] * dal[k];
      sc += std::fabs(ub[k] * du[k]) + std::fabs(bb[k] * db[k]) + std::fabs(alb[k] * dal[k]);
    }
    const double h = 1e-6;
    worst = std::fmax(worst, relmis(ad, (E(h) - E(-h)) / (2 * h), sc));
  }
  report("q26_ld04_adj", worst, 1e-7);
}

// ---- LD04 alone (corner EMFs as inputs, as for B25a) ----
static void check_ld04_alone() {
  double worst = 0;
  for (int it = 0; it < 2000; ++it) {
    double e[4], b[4], al[4], de[4], db[4], dal[4];
    for (int k = 0; k < 4; ++k) {
      e[k] = U(-2, 2);
      b[k] = U(-2, 2);
      al[k] = U(0.2, 3);
      de[k] = U(-1, 1);
      db[k] = U(-1, 1);
      dal[k] = U(-1, 1);
    }
    const double Eb = U(-1, 1);
    auto E = [&](double h) {
      double ee[4], bb[4], aa[4];
      for (int k = 0; k < 4; ++k) {
        ee[k] = e[k] + h * de[k];
        bb[k] = b[k] + h * db[k];
        aa[k] = al[k] + h * dal[k];
      }
      return Eb * ld04(ee[0], ee[1], ee[2], ee[3], aa[0], aa[1], aa[2], aa[3], bb[0], bb[1], bb[2],
                       bb[3]);
    };
    double eb[4] = {0, 0, 0, 0}, bb[4] = {0, 0, 0, 0}, alb[4] = {0, 0, 0, 0};
    ld04_adj(e, b, al, Eb, eb, bb, alb);
    double ad = 0, sc = 0;
    for (int k = 0; k < 4; ++k) {
      ad += eb[k] * de[k] + bb[k] * db[k] + alb[k] * dal[k];
      sc += std::fabs(eb[k] * de[k]) + std::fabs(bb[k] * db[k]) + std::fabs(alb[k] * dal[k]);
    }
    const double h = 1e-6;
    worst = std::fmax(worst, relmis(ad, (E(h) - E(-h)) / (2 * h), sc));
  }
  report("ld04_adj", worst, 1e-7);
}

// ---- reconstruction ----
// A line of 13 values; the centres 2 .. 10 (whose five-point windows lie in
// the line) carry random adjoints of their lower and upper values; the
// adjoint (recon_cell_adj5 per centre, summed) is checked against central
// differences.
template <int M>
static void check_recon(const char* name, int* branches) {
  constexpr int L = 13;
  double worst = 0;
  int n = 0;
  for (int it = 0; it < 40000 && n < 4000; ++it) {
    double q[L], dq[L], lob[L] = {0}, hib[L] = {0};
    for (int k = 0; k < L; ++k) {
      q[k] = U(-1, 1);
      dq[k] = U(-1, 1);
    }
    for (int c = 2; c <= L - 3; ++c) {
      lob[c] = U(-1, 1);
      hib[c] = U(-1, 1);
    }
    auto J = [&](double h) {
      double j = 0;
      for (int c = 2; c <= L - 3; ++c) {
        double qq[5], lo, hi;
        for (int k = 0; k < 5; ++k) qq[k] = q[c - 2 + k] + h * dq[c - 2 + k];
        recon_cell<M>(qq, lo, hi);
        j += lob[c] * lo + hib[c] * hi;
      }
      return j;
    };
    const double h = 1e-7;
    double jp = J(h), jm = J(-h), j0 = J(0);
    if (std::fabs(jp - 2 * j0 + jm) > 1e-10) continue;  // limiter kink inside [-h, h]
    double qs[L] = {0};
    for (int c = 2; c <= L - 3; ++c) {
      double qb[5] = {0, 0, 0, 0, 0};
      recon_cell_adj5<M>(q + c - 2, lob[c], hib[c], qb);
      for (int k = 0; k < 5; ++k) qs[c - 2 + k] += qb[k];
      if (branches && M == kPPM) {
        // census of the constraint branches (extremum, lower reset, upper reset, none)
        const double* w = q + c - 2;
        const double d1 = ppm_slope(w[0], w[1], w[2]), d2 = ppm_slope(w[1], w[2], w[3]);
        const double d3 = ppm_slope(w[2], w[3], w[4]);
        const double a = ppm_iface(w[1], w[2], d1, d2), b = ppm_iface(w[2], w[3], d2, d3);
        const double dqq = b - a, q6 = dqq * (w[2] - 0.5 * (a + b)), d6 = dqq * dqq / 6.0;
        ++branches[(b - w[2]) * (w[2] - a) <= 0 ? 0 : (q6 > d6 ? 1 : (-d6 > q6 ? 2 : 3))];
      }
    }
    double ad = 0, sc = 0;
    for (int k = 0; k < L; ++k) {
      ad += qs[k] * dq[k];
      sc += std::fabs(qs[k] * dq[k]);
    }
    const double fd = (jp - jm) / (2 * h);
    worst = std::fmax(worst, relmis(ad, fd, sc));
    ++n;
  }
  report(name, worst, 1e-7);
  if (n < 1000) {
    std::printf("%s: only %d samples away from limiter kinks\n", name, n);
    ++g_fail;
  }
}

int main() {
  check_fast();
  check_phys();
  check_ld04();
  check_ld04_alone();
  check_recon<kPC>("recon PC", nullptr);
  check_recon<kPLM_MC>("recon PLM-MC", nullptr);
  check_recon<kPLM_MM>("recon PLM-minmod", nullptr);
  int ppmb[4] = {0};
  check_recon<kPPM>("recon PPM", ppmb);
  std::printf("PPM constraint branches (extremum, lower reset, upper reset, none): %d %d %d %d\n",
              ppmb[0], ppmb[1], ppmb[2], ppmb[3]);
  for (int k = 0; k < 4; ++k)
    if (ppmb[k] < 500) {
      std::printf("PPM constraint branch %d covered by fewer than 500 samples\n", k);
      ++g_fail;
    }
  int reg[6] = {0};
  check_face<kLLF>("LLF face outputs", 2.0, 1.5, nullptr);
  check_face<kHLLD>("HLLD face outputs (subsonic)", 1.0, 1.5, reg);
  check_face<kHLLD>("HLLD face outputs (supersonic)", 6.0, 1.5, reg);
  check_face<kHLLD>("HLLD face outputs (weak bn)", 1.0, 1e-7, reg);
  check_face<kHLLD>("HLLD face outputs (strong bn)", 1.0, 3.0, reg);
  std::printf("HLLD regions covered (FL, *L, **L, **R, *R, FR): %d %d %d %d %d %d\n", reg[0],
              reg[1], reg[2], reg[3], reg[4], reg[5]);
  for (int r = 0; r < 6; ++r)
    if (reg[r] < 50) {
      std::printf("HLLD region %d covered by fewer than 50 samples\n", r);
      ++g_fail;
    }
  std::printf("%s\n", g_fail ? "FAILED" : "ALL OK");
  return g_fail ? 1 : 0;
}
