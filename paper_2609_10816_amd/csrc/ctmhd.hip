// ctmhd.hip -- kernels and C ABI of libctmhd for gfx950 (MI355X).
//
// One RK2-SSP step with first-order flux correction (Sec. 2.5 of Kriel et al.)
// is a short sequence of stream-ordered kernels on a ghosted box:
//   k_begin      zero the per-step reduction slots
//   k_wrap       periodic ghost fill of the 8 fields
//   k_dt         CFL signal speed per cell -> wavefront max -> device max
//   k_dt_final   dt = CFL / max (or the caller's dt); non-finite dt stops
//   per stage:
//   k_prim       conserved -> primitive (pressure recovery in FP64)
//   k_face<a>    reconstruction + Riemann solve at x_a faces (flux, alpha, u*)
//   k_emf<c>     edge EMFs (Q26 / B25a / FS18) + LD04 + eta j
//   k_update     flux divergence and CT curl; RK combination
//   k_flag       invalid-state flags (FOFC)
//   k_fo_face/k_fo_edge  first-order fluxes / EMFs from S^n where flagged
//   k_update     again, only when something was flagged
// Face arrays hold the x_a face on the lower side of each cell, edge arrays
// the edge at the lower corner in the two transverse directions.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>

#include "ctmhd.h"
#include "ctmhd_math.h"

using namespace ctmhd;

namespace {

// ---------------------------------------------------------------------------
// Geometry of one ghosted box.
// ---------------------------------------------------------------------------
struct Geom {
  int n[3];    // interior cells
  int g;       // ghost layers
  int N[3];    // n + 2g
  int st[3];   // strides: 1, N0, N0*N1
  int elems;   // N0*N1*N2
  double dx[3];
  double idx[3];
};

Geom make_geom(const ctmhd_box& b) {
  Geom G;
  for (int d = 0; d < 3; ++d) {
    G.n[d] = b.n[d];
    G.N[d] = b.n[d] + 2 * b.ng;
    G.dx[d] = b.dx[d];
    G.idx[d] = 1.0 / b.dx[d];
  }
  G.g = b.ng;
  G.st[0] = 1;
  G.st[1] = G.N[0];
  G.st[2] = G.N[0] * G.N[1];
  G.elems = G.N[0] * G.N[1] * G.N[2];
  return G;
}

// A 3D index range [lo, lo+len) mapped onto a 1D grid, x fastest.
struct Range {
  int lo[3];
  int len[3];
  int count() const { return len[0] * len[1] * len[2]; }
};

__device__ __forceinline__ bool range_pos(const Range& r, int t, int s[3]) {
  if (t >= r.len[0] * r.len[1] * r.len[2]) return false;
  int i = t % r.len[0];
  int q = t / r.len[0];
  int j = q % r.len[1];
  int k = q / r.len[1];
  s[0] = r.lo[0] + i;
  s[1] = r.lo[1] + j;
  s[2] = r.lo[2] + k;
  return true;
}

__device__ __forceinline__ int gidx() { return blockIdx.x * blockDim.x + threadIdx.x; }

struct State {
  double* c[5];
  double* b[3];
};

template <typename T>
struct Work {
  T* prim[8];       // rho, u0, u1, u2, p, bc0, bc1, bc2
  T* ecell[3];      // cell-centred ideal EMF (B25a)
  T* F[2][3][5];    // per stage, direction, component (global momentum order)
  T* ap[3];
  T* am[3];
  T* us[3];
  T* E[2][3];       // per stage, edge EMFs
  uint8_t* flag;    // interior cells
  unsigned long long* smax;  // CFL signal-speed maximum (bits of a non-negative double)
  double* dt;       // the step's dt
  int* stop;        // 1 once a non-finite dt was seen
  int* nflag;       // flagged cells of the current stage
};

// Per-step diagnostic slot pointer (may be null).
struct Diag {
  long long* d;  // 4 counters of this step or null
};

constexpr int kBlock = 256;

inline int nblocks(long long n) { return (int)((n + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------
__global__ void k_init(int* stop) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *stop = 0;
}

__global__ void k_begin(unsigned long long* smax, int* nflag, long long* diag, const int* stop) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *smax = 0ull;
    nflag[0] = 0;
    nflag[1] = 0;
    if (diag) {
      diag[0] = 0;
      diag[1] = 0;
      diag[2] = 0;
      diag[3] = *stop ? 1 : 0;
    }
  }
}

__device__ __forceinline__ int pwrap(int s, int g, int n) {
  int q = (s - g) % n;
  if (q < 0) q += n;
  return q + g;
}

// Periodic ghost fill of all 8 fields (faces follow the same rule: the face at
// storage index s is the lower face of cell s).
__global__ void k_wrap(State S, Geom G, const int* stop) {
  if (*stop) return;
  int t = gidx();
  if (t >= G.elems) return;
  int i = t % G.N[0];
  int q = t / G.N[0];
  int j = q % G.N[1];
  int k = q / G.N[1];
  bool inter = i >= G.g && i < G.g + G.n[0] && j >= G.g && j < G.g + G.n[1] && k >= G.g &&
               k < G.g + G.n[2];
  if (inter) return;
  int src = pwrap(i, G.g, G.n[0]) + G.st[1] * pwrap(j, G.g, G.n[1]) + G.st[2] * pwrap(k, G.g, G.n[2]);
#pragma unroll
  for (int m = 0; m < 5; ++m) S.c[m][t] = S.c[m][src];
#pragma unroll
  for (int a = 0; a < 3; ++a) S.b[a][t] = S.b[a][src];
}

__global__ void k_copy(State dst, State src, int elems, const int* only_if_stop) {
  if (only_if_stop && !*only_if_stop) return;
  int t = gidx();
  if (t >= elems) return;
#pragma unroll
  for (int m = 0; m < 5; ++m) dst.c[m][t] = src.c[m][t];
#pragma unroll
  for (int a = 0; a < 3; ++a) dst.b[a][t] = src.b[a][t];
}

// ---------------------------------------------------------------------------
// CFL time step (eq. resistivity:cfl and the signal-speed treatment of the
// resistive term): max over cells of max_d (|u_d| + c_f,d) / dx_d and
// 2 eta / dx_min^2, reduced across the wavefront, the block and the grid.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__global__ void __launch_bounds__(kBlock) k_dt(State S, Geom G, double gamma, double sres,
                                               unsigned long long* smax, const int* stop) {
  if (*stop) return;
  __shared__ double red[kBlock / 64];
  int t = gidx();
  double s = 0.0;
  int ninter = G.n[0] * G.n[1] * G.n[2];
  if (t < ninter) {
    int i = t % G.n[0] + G.g;
    int q = t / G.n[0];
    int j = q % G.n[1] + G.g;
    int k = q / G.n[1] + G.g;
    int c = i + G.st[1] * j + G.st[2] * k;
    double rho = S.c[0][c];
    double ir = 1.0 / rho;
    double u[3], b[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      u[d] = S.c[1 + d][c] * ir;
      b[d] = 0.5 * (S.b[d][c] + S.b[d][c + G.st[d]]);
    }
    double p = (gamma - 1.0) *
               (S.c[4][c] - 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) -
                0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]));
    s = sres;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double cf = fast_speed<double>(rho, p, b[d], b[(d + 1) % 3], b[(d + 2) % 3], gamma);
      double sd = (fabs(u[d]) + cf) * G.idx[d];
      // NaN-propagating max: a NaN signal speed must surface as a NaN dt
      s = (sd > s || sd != sd) ? sd : s;
    }
  }
  // NaN-aware: fmax drops NaN, so reduce bit patterns instead for the final
  // atomic (a NaN has larger bits than +inf as an unsigned integer).
  unsigned long long bits = (unsigned long long)__double_as_longlong(s);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long ob = __shfl_xor(bits, o, 64);
    bits = ob > bits ? ob : bits;
  }
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = __longlong_as_double((long long)bits);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = 0;
    for (int q = 0; q < kBlock / 64; ++q) {
      unsigned long long v = (unsigned long long)__double_as_longlong(red[q]);
      m = v > m ? v : m;
    }
    atomicMax(smax, m);
  }
}

__global__ void k_dt_final(const unsigned long long* smax, double cfl, const double* dt_fixed,
                           double* dt, double* dt_out, int* stop, long long* diag) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (*stop) {
    *dt = 0.0;
    if (dt_out) *dt_out = 0.0;
    return;
  }
  double v;
  if (dt_fixed) {
    v = *dt_fixed;
  } else {
    double s = __longlong_as_double((long long)*smax);
    v = cfl / s;
  }
  if (!(v > 0.0) || !__builtin_isfinite(v)) {
    *stop = 1;
    if (diag) diag[3] = 1;
  }
  *dt = v;
  if (dt_out) *dt_out = v;
}

// ---------------------------------------------------------------------------
// Conserved -> primitive (eq. state:primitive).  Pressure recovery is always
// FP64; results are rounded to the stencil type T.  Cells whose upper faces
// are stored (index < N-1 on every axis).
// ---------------------------------------------------------------------------
template <typename T, int EMF>
__global__ void __launch_bounds__(kBlock) k_prim(State S, Geom G, Work<T> W, double gamma,
                                                 const int* stop) {
  if (*stop) return;
  int t = gidx();
  if (t >= G.elems) return;
  int i = t % G.N[0];
  int q = t / G.N[0];
  int j = q % G.N[1];
  int k = q / G.N[1];
  if (i >= G.N[0] - 1 || j >= G.N[1] - 1 || k >= G.N[2] - 1) return;
  double rho = S.c[0][t];
  double ir = 1.0 / rho;
  double u[3], b[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    u[d] = S.c[1 + d][t] * ir;
    b[d] = 0.5 * (S.b[d][t] + S.b[d][t + G.st[d]]);
  }
  double p = (gamma - 1.0) * (S.c[4][t] - 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) -
                              0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]));
  W.prim[0][t] = (T)rho;
  W.prim[1][t] = (T)u[0];
  W.prim[2][t] = (T)u[1];
  W.prim[3][t] = (T)u[2];
  W.prim[4][t] = (T)p;
  W.prim[5][t] = (T)b[0];
  W.prim[6][t] = (T)b[1];
  W.prim[7][t] = (T)b[2];
  if (EMF == kB25A) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      int a = (c + 1) % 3, bb = (c + 2) % 3;
      // eq. emf:b25a-emf-centre in the stencil type
      W.ecell[c][t] = -(T)u[a] * (T)b[bb] + (T)u[bb] * (T)b[a];
    }
  }
}

// eta j_c at the edge stored at s (lower corner in a and b), eq.
// resistivity:current-stencil.
template <typename T>
__device__ __forceinline__ T eta_j(const State& S, const Geom& G, int s, int c, T eta) {
  int a = (c + 1) % 3, b = (c + 2) % 3;
  double j = (S.b[b][s] - S.b[b][s - G.st[a]]) * G.idx[a] - (S.b[a][s] - S.b[a][s - G.st[b]]) * G.idx[b];
  return eta * (T)j;
}

// Joule energy flux at the x_a face stored at s (Sec. 2.4): (eta j x b).n_a
// with eta j averaged over the face's bounding edges and b the mean of the two
// adjacent cells' cell-averaged field.
template <typename T>
__device__ __forceinline__ T joule(const State& S, const Geom& G, const T* const* prim, int s,
                                   int a, T eta) {
  int b = (a + 1) % 3, c = (a + 2) % 3;
  T eb = T(0.5) * (eta_j<T>(S, G, s, b, eta) + eta_j<T>(S, G, s + G.st[c], b, eta));
  T ec = T(0.5) * (eta_j<T>(S, G, s, c, eta) + eta_j<T>(S, G, s + G.st[b], c, eta));
  int l = s - G.st[a];
  T bb = T(0.5) * (prim[5 + b][l] + prim[5 + b][s]);
  T bc = T(0.5) * (prim[5 + c][l] + prim[5 + c][s]);
  return eb * bc - ec * bb;
}

// ---------------------------------------------------------------------------
// Face pass (Sec. 2.2, eqs. emf:alpha-pm, emf:q26-facevel): reconstruct the
// seven face-local primitives from both sides, solve the Riemann problem with
// the stored normal field, store the flux, alpha^{+/-} and u_a^*.
// ---------------------------------------------------------------------------
template <typename T, int RECON, int RIEMANN>
__global__ void __launch_bounds__(kBlock)
    k_face(State S, Geom G, Work<T> W, Range R, int a, int stage, double gamma_d, double eta_d,
           Range upd, long long* diag, const int* stop) {
  if (*stop) return;
  int s3[3];
  int fb = 0;
  if (range_pos(R, gidx(), s3)) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const int sa = G.st[a];
    const int s = s3[0] + G.st[1] * s3[1] + G.st[2] * s3[2];
    const T gamma = (T)gamma_d;
    const int var[7] = {0, 1 + a, 1 + b, 1 + c, 4, 5 + b, 5 + c};
    T lo[7], hi[7];
#pragma unroll
    for (int v = 0; v < 7; ++v) {
      const T* P = W.prim[var[v]];
      T q[6];
#pragma unroll
      for (int m = 0; m < 6; ++m) q[m] = stencil_uses<RECON>(m) ? P[s + (m - 3) * sa] : T(0);
      recon_iface<RECON>(q, lo[v], hi[v]);
    }
    FState<T> L{lo[0], lo[1], lo[2], lo[3], lo[4], lo[5], lo[6]};
    FState<T> Rr{hi[0], hi[1], hi[2], hi[3], hi[4], hi[5], hi[6]};
    T bn = (T)S.b[a][s];
    T F[5], ap, am;
    if (RIEMANN == kHLLD) {
      T SL, SR;
      fb = hlld_flux(L, Rr, bn, gamma, F, SL, SR);
      ap = tmax(T(0), SR);
      am = tmax(T(0), -SL);
    } else {
      ap = am = llf_flux(L, Rr, bn, gamma, F);
    }
    bool in_upd = s3[0] >= upd.lo[0] && s3[0] < upd.lo[0] + upd.len[0] && s3[1] >= upd.lo[1] &&
                  s3[1] < upd.lo[1] + upd.len[1] && s3[2] >= upd.lo[2] && s3[2] < upd.lo[2] + upd.len[2];
    if (eta_d > 0.0 && in_upd) F[4] += joule<T>(S, G, W.prim, s, a, (T)eta_d);
    W.F[stage][a][0][s] = F[0];
    W.F[stage][a][1 + a][s] = F[1];
    W.F[stage][a][1 + b][s] = F[2];
    W.F[stage][a][1 + c][s] = F[3];
    W.F[stage][a][4][s] = F[4];
    W.ap[a][s] = ap;
    W.am[a][s] = am;
    W.us[a][s] = (ap * L.un + am * Rr.un) / (ap + am);
  }
  if (diag) {
    unsigned long long m = __ballot(fb);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd((unsigned long long*)&diag[2], (unsigned long long)__popcll(m));
  }
}

// ---------------------------------------------------------------------------
// Edge pass (Sec. 2.3): face field reconstructed to the edge, four corner
// EMFs of the chosen compute scheme, LD04 averaging, plus eta j.
// ---------------------------------------------------------------------------
template <int RECON, typename T>
__device__ __forceinline__ void iface_along(const T* A, int s, int stride, T& lo, T& hi) {
  T q[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) q[m] = stencil_uses<RECON>(m) ? A[s + (m - 3) * stride] : T(0);
  recon_iface<RECON>(q, lo, hi);
}

template <int RECON, typename T>
__device__ __forceinline__ void iface_along_d(const double* A, int s, int stride, T& lo, T& hi) {
  T q[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) q[m] = stencil_uses<RECON>(m) ? (T)A[s + (m - 3) * stride] : T(0);
  recon_iface<RECON>(q, lo, hi);
}

// Two-step reconstruction of a cell-centred field to the four corners of the
// edge at s: first along d1 to the x_d1 face, then along d2 to the edge.
// out[s1 + 2*s2] with s = 0 lower side, 1 upper side along each direction.
template <int RECON, typename T>
__device__ __forceinline__ void two_step(const T* A, int s, int st1, int st2, T out[4]) {
  T seqlo[6], seqhi[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    if (!stencil_uses<RECON>(m)) {
      seqlo[m] = seqhi[m] = T(0);
    } else {
      iface_along<RECON>(A, s + (m - 3) * st2, st1, seqlo[m], seqhi[m]);
    }
  }
  T l0, l1, h0, h1;
  recon_iface<RECON>(seqlo, l0, l1);
  recon_iface<RECON>(seqhi, h0, h1);
  out[0] = l0;  // (lower along d1, lower along d2)
  out[1] = h0;  // (upper, lower)
  out[2] = l1;  // (lower, upper)
  out[3] = h1;  // (upper, upper)
}

template <typename T, int RECON, int EMF>
__global__ void __launch_bounds__(kBlock)
    k_emf(State S, Geom G, Work<T> W, Range R, int c, int stage, double eta_d, const int* stop) {
  if (*stop) return;
  int s3[3];
  if (!range_pos(R, gidx(), s3)) return;
  const int a = (c + 1) % 3, b = (c + 2) % 3;
  const int sa = G.st[a], sb = G.st[b];
  const int s = s3[0] + G.st[1] * s3[1] + G.st[2] * s3[2];
  T baB, baT, bbL, bbR;
  iface_along_d<RECON>(S.b[a], s, sb, baB, baT);
  iface_along_d<RECON>(S.b[b], s, sa, bbL, bbR);
  T e[4];  // LB, RB, LT, RT
  if (EMF == kQ26) {
    T uaB, uaT, ubL, ubR;
    iface_along<RECON>(W.us[a], s, sb, uaB, uaT);
    iface_along<RECON>(W.us[b], s, sa, ubL, ubR);
    e[0] = -uaB * bbL + ubL * baB;
    e[1] = -uaB * bbR + ubR * baB;
    e[2] = -uaT * bbL + ubL * baT;
    e[3] = -uaT * bbR + ubR * baT;
  } else if (EMF == kB25A) {
    T ab[4], ba[4];
    two_step<RECON>(W.ecell[c], s, sa, sb, ab);  // [x_a x_b]: index sa_side + 2 sb_side
    two_step<RECON>(W.ecell[c], s, sb, sa, ba);  // [x_b x_a]: index sb_side + 2 sa_side
    e[0] = T(0.5) * (ab[0] + ba[0]);
    e[1] = T(0.5) * (ab[1] + ba[2]);
    e[2] = T(0.5) * (ab[2] + ba[1]);
    e[3] = T(0.5) * (ab[3] + ba[3]);
  } else {
    const T* ua = W.prim[1 + a];
    const T* ub = W.prim[1 + b];
    T ua_ab[4], ua_ba[4], ub_ab[4], ub_ba[4];
    two_step<RECON>(ua, s, sa, sb, ua_ab);
    two_step<RECON>(ua, s, sb, sa, ua_ba);
    two_step<RECON>(ub, s, sa, sb, ub_ab);
    two_step<RECON>(ub, s, sb, sa, ub_ba);
    const int perm[4] = {0, 2, 1, 3};  // corner q = sa_side + 2 sb_side -> [x_b x_a] index
    const T bbX[2] = {bbL, bbR}, baY[2] = {baB, baT};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      T u1 = T(0.5) * (ua_ab[q] + ua_ba[perm[q]]);
      T u2 = T(0.5) * (ub_ab[q] + ub_ba[perm[q]]);
      e[q] = -u1 * bbX[q & 1] + u2 * baY[q >> 1];
    }
  }
  T apa = tmax(W.ap[a][s - sb], W.ap[a][s]);
  T ama = tmax(W.am[a][s - sb], W.am[a][s]);
  T apb = tmax(W.ap[b][s - sa], W.ap[b][s]);
  T amb = tmax(W.am[b][s - sa], W.am[b][s]);
  T eps = ld04(e[0], e[1], e[2], e[3], apa, ama, apb, amb, baB, baT, bbL, bbR);
  if (eta_d > 0.0) eps += eta_j<T>(S, G, s, c, (T)eta_d);
  W.E[stage][c][s] = eps;
}

// ---------------------------------------------------------------------------
// Update (eqs. rk:increment-state, rk:increment-bfield, rk1:update,
// rk2:update).  stage 0: out = S^n + D^n.  stage 1: out = S^n + (D^n + D^{n+1/2})/2.
// Increments are formed in FP64 from the stored fluxes and EMFs.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void incr(const Geom& G, const Work<T>& W, int st, int s, double dt,
                                     double dc[5], double db[3]) {
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    double f = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T* Fa = W.F[st][a][m];
      f += ((double)Fa[s] - (double)Fa[s + G.st[a]]) * G.idx[a];
    }
    dc[m] = dt * f;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const T* Ec = W.E[st][c];
    const T* Eb = W.E[st][b];
    double circ = ((double)Ec[s] - (double)Ec[s + G.st[b]]) * G.idx[b] +
                  ((double)Eb[s + G.st[c]] - (double)Eb[s]) * G.idx[c];
    db[a] = dt * circ;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_update(State base, State out, Geom G, Work<T> W, int stage, int only_if_flagged,
             const int* stop) {
  if (*stop) return;
  if (only_if_flagged && W.nflag[stage] == 0) return;
  int t = gidx();
  int ninter = G.n[0] * G.n[1] * G.n[2];
  if (t >= ninter) return;
  int i = t % G.n[0] + G.g;
  int q = t / G.n[0];
  int j = q % G.n[1] + G.g;
  int k = q / G.n[1] + G.g;
  int s = i + G.st[1] * j + G.st[2] * k;
  double dt = *W.dt;
  double d1c[5], d1b[3];
  incr(G, W, 0, s, dt, d1c, d1b);
  if (stage == 0) {
#pragma unroll
    for (int m = 0; m < 5; ++m) out.c[m][s] = base.c[m][s] + d1c[m];
#pragma unroll
    for (int a = 0; a < 3; ++a) out.b[a][s] = base.b[a][s] + d1b[a];
  } else {
    double d2c[5], d2b[3];
    incr(G, W, 1, s, dt, d2c, d2b);
#pragma unroll
    for (int m = 0; m < 5; ++m) out.c[m][s] = base.c[m][s] + 0.5 * (d1c[m] + d2c[m]);
#pragma unroll
    for (int a = 0; a < 3; ++a) out.b[a][s] = base.b[a][s] + 0.5 * (d1b[a] + d2b[a]);
  }
}

// ---------------------------------------------------------------------------
// First-order flux correction (Sec. 2.5).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
    k_flag(State X, Geom G, uint8_t* flag, const uint8_t* force, int crit, double gamma,
           int* nflag, long long* diag, const int* stop) {
  if (*stop) return;
  int t = gidx();
  int ninter = G.n[0] * G.n[1] * G.n[2];
  int bad = 0;
  if (t < ninter) {
    int i0 = t % G.n[0];
    int q = t / G.n[0];
    int j0 = q % G.n[1];
    int k0 = q / G.n[1];
    int i = i0 + G.g, j = j0 + G.g, k = k0 + G.g;
    int s = i + G.st[1] * j + G.st[2] * k;
    int up[3] = {((i0 + 1) % G.n[0]) + G.g + G.st[1] * j + G.st[2] * k,
                 i + G.st[1] * (((j0 + 1) % G.n[1]) + G.g) + G.st[2] * k,
                 i + G.st[1] * j + G.st[2] * (((k0 + 1) % G.n[2]) + G.g)};
    double rho = X.c[0][s];
    bool nonfin = false;
#pragma unroll
    for (int m = 0; m < 5; ++m) nonfin |= !__builtin_isfinite(X.c[m][s]);
    double m2 = 0.0, b2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double bl = X.b[d][s], bu = X.b[d][up[d]];
      nonfin |= !__builtin_isfinite(bl) || !__builtin_isfinite(bu);
      double bc = 0.5 * (bl + bu);
      double u = X.c[1 + d][s] / rho;
      m2 += rho * u * u;
      b2 += bc * bc;
    }
    double p = (gamma - 1.0) * (X.c[4][s] - 0.5 * m2 - 0.5 * b2);
    if ((crit & CTMHD_FLAG_RHO) && !(rho > 0.0)) bad = 1;
    if ((crit & CTMHD_FLAG_P) && !(p > 0.0)) bad = 1;
    if ((crit & CTMHD_FLAG_NONFINITE) && (nonfin || !__builtin_isfinite(p))) bad = 1;
    if (force && force[t]) bad = 1;
    flag[t] = (uint8_t)bad;
  }
  unsigned long long m = __ballot(bad);
  if ((threadIdx.x & 63) == 0 && m) {
    int cnt = __popcll(m);
    atomicAdd(nflag, cnt);
    if (diag) atomicAdd((unsigned long long*)diag, (unsigned long long)cnt);
  }
}

__device__ __forceinline__ int interior_id(const Geom& G, int s0, int s1, int s2) {
  int i = (s0 - G.g) % G.n[0];
  if (i < 0) i += G.n[0];
  int j = (s1 - G.g) % G.n[1];
  if (j < 0) j += G.n[1];
  int k = (s2 - G.g) % G.n[2];
  if (k < 0) k += G.n[2];
  return i + G.n[0] * (j + G.n[1] * k);
}

// PC face state from the conserved state of cell l (left) or r (right).
template <typename T>
__device__ __forceinline__ void pc_cell(const State& S, const Geom& G, int s, double gamma, T& rho,
                                        T u[3], T& p, T bc[3]) {
  double r = S.c[0][s];
  double ir = 1.0 / r;
  double uu[3], bb[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    uu[d] = S.c[1 + d][s] * ir;
    bb[d] = 0.5 * (S.b[d][s] + S.b[d][s + G.st[d]]);
  }
  double pp = (gamma - 1.0) * (S.c[4][s] - 0.5 * r * (uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]) -
                               0.5 * (bb[0] * bb[0] + bb[1] * bb[1] + bb[2] * bb[2]));
  rho = (T)r;
  p = (T)pp;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    u[d] = (T)uu[d];
    bc[d] = (T)bb[d];
  }
}

// First-order (PC + LLF) flux at the x_a face s; returns s_LLF and u*.
template <typename T>
__device__ __forceinline__ T fo_face(const State& S, const Geom& G, int s, int a, double gamma_d,
                                     T F[5], T& ustar) {
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  T rl, ul[3], pl, bl[3], rr, ur[3], pr, br[3];
  pc_cell<T>(S, G, s - G.st[a], gamma_d, rl, ul, pl, bl);
  pc_cell<T>(S, G, s, gamma_d, rr, ur, pr, br);
  FState<T> L{rl, ul[a], ul[b], ul[c], pl, bl[b], bl[c]};
  FState<T> R{rr, ur[a], ur[b], ur[c], pr, br[b], br[c]};
  T Fl[5];
  T sp = llf_flux(L, R, (T)S.b[a][s], (T)gamma_d, Fl);
  F[0] = Fl[0];
  F[1 + a] = Fl[1];
  F[1 + b] = Fl[2];
  F[1 + c] = Fl[3];
  F[4] = Fl[4];
  ustar = (sp * L.un + sp * R.un) / (sp + sp);
  return sp;
}

// Joule flux at the x_a face s with cell fields from the conserved state.
template <typename T>
__device__ __forceinline__ T joule_sn(const State& S, const Geom& G, int s, int a, T eta) {
  int b = (a + 1) % 3, c = (a + 2) % 3;
  T eb = T(0.5) * (eta_j<T>(S, G, s, b, eta) + eta_j<T>(S, G, s + G.st[c], b, eta));
  T ec = T(0.5) * (eta_j<T>(S, G, s, c, eta) + eta_j<T>(S, G, s + G.st[b], c, eta));
  int l = s - G.st[a];
  T bbl = (T)(0.5 * (S.b[b][l] + S.b[b][l + G.st[b]]));
  T bbr = (T)(0.5 * (S.b[b][s] + S.b[b][s + G.st[b]]));
  T bcl = (T)(0.5 * (S.b[c][l] + S.b[c][l + G.st[c]]));
  T bcr = (T)(0.5 * (S.b[c][s] + S.b[c][s + G.st[c]]));
  return eb * (T(0.5) * (bcl + bcr)) - ec * (T(0.5) * (bbl + bbr));
}

// Replace the flux at every interior x_a face that touches a flagged cell by
// the first-order flux from S^n (stage 0: the stage-1 flux; stage 1: both
// stored fluxes, so that their RK average is the FO flux).
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_fo_face(State Sn, Geom G, Work<T> W, int a, int stage, double gamma, double eta_d,
              const int* stop) {
  if (*stop) return;
  if (W.nflag[stage] == 0) return;
  int t = gidx();
  int nf = G.n[0] * G.n[1] * G.n[2];
  if (t >= nf) return;
  int s3[3] = {t % G.n[0] + G.g, (t / G.n[0]) % G.n[1] + G.g, t / (G.n[0] * G.n[1]) + G.g};
  int s = s3[0] + G.st[1] * s3[1] + G.st[2] * s3[2];
  int l3[3] = {s3[0], s3[1], s3[2]};
  l3[a] -= 1;
  if (!W.flag[interior_id(G, s3[0], s3[1], s3[2])] && !W.flag[interior_id(G, l3[0], l3[1], l3[2])]) return;
  T F[5], us;
  fo_face<T>(Sn, G, s, a, gamma, F, us);
  if (eta_d > 0.0) F[4] += joule_sn<T>(Sn, G, s, a, (T)eta_d);
  // periodic images: the update reads faces s and s + e_a of interior cells,
  // so the face at the upper boundary (s_a = g + n_a) holds the same value
#pragma unroll
  for (int rep = 0; rep < 2; ++rep) {
    int sw = s + (rep ? G.n[a] * G.st[a] : 0);
    if (rep && s3[a] != G.g) break;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      W.F[stage][a][m][sw] = F[m];
      if (stage == 1) W.F[0][a][m][sw] = F[m];
    }
  }
}

template <typename T, int EMF>
__device__ __forceinline__ T fo_corner_cell(const State& Sn, const Geom& G, int s, int a, int b,
                                            double gamma, T baY, T bbX) {
  // ideal EMF of a cell (PC): -u_a b_b + u_b b_a, from cell-centred values
  T rho, u[3], p, bc[3];
  pc_cell<T>(Sn, G, s, gamma, rho, u, p, bc);
  if (EMF == kB25A) return -u[a] * bc[b] + u[b] * bc[a];
  return -u[a] * bbX + u[b] * baY;  // FS18 with PC: cell velocity, edge field
}

// Replace the EMF at every interior edge that touches a flagged cell by the
// first-order EMF from S^n.
template <typename T, int EMF>
__global__ void __launch_bounds__(kBlock)
    k_fo_edge(State Sn, Geom G, Work<T> W, int c, int stage, double gamma, double eta_d,
              const int* stop) {
  if (*stop) return;
  if (W.nflag[stage] == 0) return;
  int t = gidx();
  int nf = G.n[0] * G.n[1] * G.n[2];
  if (t >= nf) return;
  const int a = (c + 1) % 3, b = (c + 2) % 3;
  int s3[3] = {t % G.n[0] + G.g, (t / G.n[0]) % G.n[1] + G.g, t / (G.n[0] * G.n[1]) + G.g};
  int s = s3[0] + G.st[1] * s3[1] + G.st[2] * s3[2];
  int fl = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int p3[3] = {s3[0], s3[1], s3[2]};
    p3[a] -= (q & 1);
    p3[b] -= (q >> 1);
    fl |= W.flag[interior_id(G, p3[0], p3[1], p3[2])];
  }
  if (!fl) return;
  const int sa = G.st[a], sb = G.st[b];
  T F[5];
  T usaB, usaT, usbL, usbR;
  T apB = fo_face<T>(Sn, G, s - sb, a, gamma, F, usaB);
  T apT = fo_face<T>(Sn, G, s, a, gamma, F, usaT);
  T bpL = fo_face<T>(Sn, G, s - sa, b, gamma, F, usbL);
  T bpR = fo_face<T>(Sn, G, s, b, gamma, F, usbR);
  T baB = (T)Sn.b[a][s - sb], baT = (T)Sn.b[a][s];
  T bbL = (T)Sn.b[b][s - sa], bbR = (T)Sn.b[b][s];
  T e[4];
  if (EMF == kQ26) {
    e[0] = -usaB * bbL + usbL * baB;
    e[1] = -usaB * bbR + usbR * baB;
    e[2] = -usaT * bbL + usbL * baT;
    e[3] = -usaT * bbR + usbR * baT;
  } else {
    // corner XY is the cell on side X along a and side Y along b
    e[0] = fo_corner_cell<T, EMF>(Sn, G, s - sa - sb, a, b, gamma, baB, bbL);
    e[1] = fo_corner_cell<T, EMF>(Sn, G, s - sb, a, b, gamma, baB, bbR);
    e[2] = fo_corner_cell<T, EMF>(Sn, G, s - sa, a, b, gamma, baT, bbL);
    e[3] = fo_corner_cell<T, EMF>(Sn, G, s, a, b, gamma, baT, bbR);
  }
  T aa = tmax(apB, apT), ab = tmax(bpL, bpR);
  T eps = ld04(e[0], e[1], e[2], e[3], aa, aa, ab, ab, baB, baT, bbL, bbR);
  if (eta_d > 0.0) eps += eta_j<T>(Sn, G, s, c, (T)eta_d);
  // the update reads edges s, s + e_a, s + e_b: also write the periodic images
  // on the upper boundary rows
#pragma unroll
  for (int qa = 0; qa < 2; ++qa)
#pragma unroll
    for (int qb = 0; qb < 2; ++qb) {
      if ((qa && s3[a] != G.g) || (qb && s3[b] != G.g)) continue;
      int sw = s + (qa ? G.n[a] * sa : 0) + (qb ? G.n[b] * sb : 0);
      W.E[stage][c][sw] = eps;
      if (stage == 1) W.E[0][c][sw] = eps;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
thread_local char g_err[256] = "";

int fail(int code, const char* msg) {
  snprintf(g_err, sizeof(g_err), "%s", msg);
  return code;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int check_params(const ctmhd_params* p) {
  if (!p) return fail(CTMHD_EARG, "params is NULL");
  if (!(p->gamma > 1.0)) return fail(CTMHD_EARG, "gamma must be > 1");
  if (!(p->eta >= 0.0)) return fail(CTMHD_EARG, "eta must be >= 0");
  if (!(p->cfl > 0.0 && p->cfl < 1.0)) return fail(CTMHD_EARG, "cfl must be in (0, 1)");
  if (p->eta > 0.0 && !(p->cfl < 1.0 / 3.0))
    return fail(CTMHD_EARG, "cfl must be < 1/3 with eta > 0 (3D diffusive limit)");
  if (p->recon < 0 || p->recon > 3) return fail(CTMHD_EARG, "unknown reconstruction");
  if (p->riemann < 0 || p->riemann > 1) return fail(CTMHD_EARG, "unknown Riemann solver");
  if (p->emf_compute < 0 || p->emf_compute > 2) return fail(CTMHD_EARG, "unknown EMF scheme");
  if (p->emf_average != CTMHD_AVG_LD04) return fail(CTMHD_EUNSUPPORTED, "only LD04 averaging is built");
  if (p->precision != CTMHD_FP64 && p->precision != CTMHD_FP32) return fail(CTMHD_EARG, "unknown precision");
  return CTMHD_OK;
}

int check_box(const ctmhd_params* p, const ctmhd_box* b) {
  if (!b) return fail(CTMHD_EARG, "box is NULL");
  for (int d = 0; d < 3; ++d) {
    if (b->n[d] < 1) return fail(CTMHD_EARG, "box dimensions must be >= 1");
    if (!(b->dx[d] > 0.0)) return fail(CTMHD_EARG, "dx must be > 0");
  }
  if (b->ng < recon_halfwidth(p->recon) + 2) return fail(CTMHD_EARG, "too few ghost layers");
  long long e = 1;
  for (int d = 0; d < 3; ++d) e *= (long long)(b->n[d] + 2 * b->ng);
  if (e * 6 >= (1LL << 31)) return fail(CTMHD_EARG, "box too large for 32-bit indexing");
  return CTMHD_OK;
}

// Workspace of one box for stencil type of `tbytes` bytes.
size_t box_ws_bytes(const ctmhd_box& b, size_t tbytes) {
  size_t e = 1;
  for (int d = 0; d < 3; ++d) e *= (size_t)(b.n[d] + 2 * b.ng);
  size_t ninter = (size_t)b.n[0] * b.n[1] * b.n[2];
  size_t bytes = 0;
  bytes += 2 * 8 * align256(e * 8);        // two state buffers
  bytes += (8 + 3) * align256(e * tbytes); // prim + B25a cell EMF
  bytes += 2 * 15 * align256(e * tbytes);  // fluxes, two stages
  bytes += 9 * align256(e * tbytes);       // alpha+, alpha-, u*
  bytes += 6 * align256(e * tbytes);       // EMFs, two stages
  bytes += align256(ninter);               // flags
  bytes += 256;                            // scalars
  return bytes;
}

template <typename T>
struct Carve {
  char* p;
  char* end;
  template <typename U>
  U* take(size_t n) {
    U* r = (U*)p;
    p += align256(n * sizeof(U));
    return r;
  }
};

template <typename T>
int build_work(void* ws, size_t ws_bytes, const ctmhd_box& b, Work<T>& W, State& A2, State& H) {
  size_t need = box_ws_bytes(b, sizeof(T));
  if (!ws || ws_bytes < need) return fail(CTMHD_EARG, "workspace too small");
  if (((uintptr_t)ws & 255) != 0) return fail(CTMHD_EARG, "workspace must be 256-byte aligned");
  size_t e = 1;
  for (int d = 0; d < 3; ++d) e *= (size_t)(b.n[d] + 2 * b.ng);
  size_t ninter = (size_t)b.n[0] * b.n[1] * b.n[2];
  Carve<T> cv{(char*)ws, (char*)ws + ws_bytes};
  for (int m = 0; m < 5; ++m) A2.c[m] = cv.template take<double>(e);
  for (int a = 0; a < 3; ++a) A2.b[a] = cv.template take<double>(e);
  for (int m = 0; m < 5; ++m) H.c[m] = cv.template take<double>(e);
  for (int a = 0; a < 3; ++a) H.b[a] = cv.template take<double>(e);
  for (int v = 0; v < 8; ++v) W.prim[v] = cv.template take<T>(e);
  for (int c = 0; c < 3; ++c) W.ecell[c] = cv.template take<T>(e);
  for (int st = 0; st < 2; ++st)
    for (int a = 0; a < 3; ++a)
      for (int m = 0; m < 5; ++m) W.F[st][a][m] = cv.template take<T>(e);
  for (int a = 0; a < 3; ++a) W.ap[a] = cv.template take<T>(e);
  for (int a = 0; a < 3; ++a) W.am[a] = cv.template take<T>(e);
  for (int a = 0; a < 3; ++a) W.us[a] = cv.template take<T>(e);
  for (int st = 0; st < 2; ++st)
    for (int c = 0; c < 3; ++c) W.E[st][c] = cv.template take<T>(e);
  W.flag = cv.template take<uint8_t>(ninter);
  char* sc = cv.p;
  W.smax = (unsigned long long*)sc;
  W.dt = (double*)(sc + 8);
  W.stop = (int*)(sc + 16);
  W.nflag = (int*)(sc + 24);
  return CTMHD_OK;
}

// Timing hook state (host only).
void* const* g_prof_events = nullptr;
int g_prof_pairs = 0;
int g_prof_used = 0;

inline void prof_begin(hipStream_t st) {
  if (g_prof_events && g_prof_used < g_prof_pairs)
    hipEventRecord((hipEvent_t)g_prof_events[2 * g_prof_used], st);
}
inline void prof_end(hipStream_t st) {
  if (g_prof_events && g_prof_used < g_prof_pairs) {
    hipEventRecord((hipEvent_t)g_prof_events[2 * g_prof_used + 1], st);
    ++g_prof_used;
  }
}

#define LAUNCH(kern, blocks, ...)                                                  \
  do {                                                                             \
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), 0, st, __VA_ARGS__);      \
    if (hipGetLastError() != hipSuccess) return fail(CTMHD_EHIP, "kernel launch failed: " #kern); \
  } while (0)

// Dispatch helpers: template kernels selected at run time.
template <typename T, int RECON>
int launch_face(hipStream_t st, const ctmhd_params* p, State S, const Geom& G, const Work<T>& W,
                Range R, int a, int stage, Range upd, long long* diag) {
  if (R.count() <= 0) return CTMHD_OK;
  prof_begin(st);
  if (p->riemann == CTMHD_RIEMANN_HLLD)
    LAUNCH((k_face<T, RECON, kHLLD>), nblocks(R.count()), S, G, W, R, a, stage, p->gamma, p->eta, upd,
           diag, W.stop);
  else
    LAUNCH((k_face<T, RECON, kLLF>), nblocks(R.count()), S, G, W, R, a, stage, p->gamma, p->eta, upd,
           diag, W.stop);
  prof_end(st);
  return CTMHD_OK;
}

template <typename T, int RECON>
int launch_emf(hipStream_t st, const ctmhd_params* p, State S, const Geom& G, const Work<T>& W,
               Range R, int c, int stage) {
  if (p->emf_compute == CTMHD_EMF_Q26)
    LAUNCH((k_emf<T, RECON, kQ26>), nblocks(R.count()), S, G, W, R, c, stage, p->eta, W.stop);
  else if (p->emf_compute == CTMHD_EMF_B25A)
    LAUNCH((k_emf<T, RECON, kB25A>), nblocks(R.count()), S, G, W, R, c, stage, p->eta, W.stop);
  else
    LAUNCH((k_emf<T, RECON, kFS18>), nblocks(R.count()), S, G, W, R, c, stage, p->eta, W.stop);
  return CTMHD_OK;
}

template <typename T>
int launch_prim(hipStream_t st, const ctmhd_params* p, State S, const Geom& G, const Work<T>& W) {
  if (p->emf_compute == CTMHD_EMF_B25A)
    LAUNCH((k_prim<T, kB25A>), nblocks(G.elems), S, G, W, p->gamma, W.stop);
  else
    LAUNCH((k_prim<T, kQ26>), nblocks(G.elems), S, G, W, p->gamma, W.stop);
  return CTMHD_OK;
}

template <typename T>
int launch_fo_edge(hipStream_t st, const ctmhd_params* p, State Sn, const Geom& G, const Work<T>& W,
                   int c, int stage, int ninter) {
  if (p->emf_compute == CTMHD_EMF_Q26)
    LAUNCH((k_fo_edge<T, kQ26>), nblocks(ninter), Sn, G, W, c, stage, p->gamma, p->eta, W.stop);
  else if (p->emf_compute == CTMHD_EMF_B25A)
    LAUNCH((k_fo_edge<T, kB25A>), nblocks(ninter), Sn, G, W, c, stage, p->gamma, p->eta, W.stop);
  else
    LAUNCH((k_fo_edge<T, kFS18>), nblocks(ninter), Sn, G, W, c, stage, p->gamma, p->eta, W.stop);
  return CTMHD_OK;
}

// One stage: fluxes and EMFs of `in`, update into `out` from `base` = S^n.
template <typename T, int RECON>
int run_stage(hipStream_t st, const ctmhd_params* p, const Geom& G, const Work<T>& W, State in,
              State base, State out, int stage, const uint8_t* force, long long* diag) {
  int rc;
  if ((rc = launch_prim<T>(st, p, in, G, W))) return rc;
  const int r = recon_halfwidth(RECON);
  const int g = G.g;
  Range upd;
  for (int d = 0; d < 3; ++d) {
    upd.lo[d] = g;
    upd.len[d] = G.n[d];
  }
  for (int a = 0; a < 3; ++a) {
    Range R, U = upd;
    for (int d = 0; d < 3; ++d) {
      if (d == a) {
        R.lo[d] = g - 1;
        R.len[d] = G.n[d] + 2;  // [g-1, g+n]
      } else {
        R.lo[d] = 0;
        R.len[d] = g + G.n[d] + r + 1;  // [0, g+n+r]
      }
    }
    U.len[a] = G.n[a] + 1;  // faces g .. g+n along a are read by the update
    if ((rc = launch_face<T, RECON>(st, p, in, G, W, R, a, stage, U, diag))) return rc;
  }
  for (int c = 0; c < 3; ++c) {
    Range R;
    for (int d = 0; d < 3; ++d) {
      R.lo[d] = g;
      R.len[d] = G.n[d] + (d == c ? 0 : 1);
    }
    if ((rc = launch_emf<T, RECON>(st, p, in, G, W, R, c, stage))) return rc;
  }
  const int ninter = G.n[0] * G.n[1] * G.n[2];
  LAUNCH(k_update<T>, nblocks(ninter), base, out, G, W, stage, 0, W.stop);
  if (p->fofc) {
    LAUNCH(k_flag, nblocks(ninter), out, G, W.flag, force ? force + (size_t)stage * ninter : nullptr,
           p->flag_criteria, p->gamma, W.nflag + stage, diag ? diag + stage : nullptr, W.stop);
    for (int a = 0; a < 3; ++a)
      LAUNCH(k_fo_face<T>, nblocks(ninter), base, G, W, a, stage, p->gamma, p->eta, W.stop);
    for (int c = 0; c < 3; ++c)
      if ((rc = launch_fo_edge<T>(st, p, base, G, W, c, stage, ninter))) return rc;
    LAUNCH(k_update<T>, nblocks(ninter), base, out, G, W, stage, 1, W.stop);
  }
  return CTMHD_OK;
}

template <typename T, int RECON>
int step_box(const ctmhd_params* p, const ctmhd_box* box, double* const cons[5],
             double* const bface[3], int nsteps, const double* dt_fixed, double* dt_out,
             int64_t* diag, void* ws, size_t ws_bytes, hipStream_t st) {
  Geom G = make_geom(*box);
  Work<T> W;
  State B, H;
  int rc = build_work<T>(ws, ws_bytes, *box, W, B, H);
  if (rc) return rc;
  State A;
  for (int m = 0; m < 5; ++m) A.c[m] = cons[m];
  for (int a = 0; a < 3; ++a) A.b[a] = bface[a];
  const State user = A;
  double dxmin = fmin(G.dx[0], fmin(G.dx[1], G.dx[2]));
  double sres = p->eta > 0.0 ? 2.0 * p->eta / (dxmin * dxmin) : 0.0;
  const int ninter = G.n[0] * G.n[1] * G.n[2];
  LAUNCH(k_init, 1, W.stop);
  for (int n = 0; n < nsteps; ++n) {
    long long* dg = diag ? (long long*)diag + 4 * n : nullptr;
    LAUNCH(k_begin, 1, W.smax, W.nflag, dg, W.stop);
    LAUNCH(k_wrap, nblocks(G.elems), A, G, W.stop);
    if (!dt_fixed) LAUNCH(k_dt, nblocks(ninter), A, G, p->gamma, sres, W.smax, W.stop);
    LAUNCH(k_dt_final, 1, W.smax, p->cfl, dt_fixed ? dt_fixed + n : nullptr, W.dt,
           dt_out ? dt_out + n : nullptr, W.stop, dg);
    if ((rc = run_stage<T, RECON>(st, p, G, W, A, A, H, 0, p->force_flags, dg))) return rc;
    LAUNCH(k_wrap, nblocks(G.elems), H, G, W.stop);
    if ((rc = run_stage<T, RECON>(st, p, G, W, H, A, B, 1, p->force_flags, dg))) return rc;
    // a stopped step leaves the state where it was: carry it to the next buffer
    LAUNCH(k_copy, nblocks(G.elems), B, A, G.elems, W.stop);
    State tmp = A;
    A = B;
    B = tmp;
  }
  if (A.c[0] != user.c[0]) LAUNCH(k_copy, nblocks(G.elems), user, A, G.elems, (const int*)nullptr);
  // ghosts of the result hold the periodic copy on return
  LAUNCH(k_init, 1, W.stop);
  LAUNCH(k_wrap, nblocks(G.elems), user, G, W.stop);
  return CTMHD_OK;
}

template <typename T>
int step_box_t(const ctmhd_params* p, const ctmhd_box* box, double* const cons[5],
               double* const bface[3], int nsteps, const double* dt_fixed, double* dt_out,
               int64_t* diag, void* ws, size_t ws_bytes, hipStream_t st) {
  switch (p->recon) {
    case CTMHD_RECON_PC:
      return step_box<T, kPC>(p, box, cons, bface, nsteps, dt_fixed, dt_out, diag, ws, ws_bytes, st);
    case CTMHD_RECON_PLM_MC:
      return step_box<T, kPLM_MC>(p, box, cons, bface, nsteps, dt_fixed, dt_out, diag, ws, ws_bytes, st);
    case CTMHD_RECON_PLM_MINMOD:
      return step_box<T, kPLM_MM>(p, box, cons, bface, nsteps, dt_fixed, dt_out, diag, ws, ws_bytes, st);
    default:
      return step_box<T, kPPM>(p, box, cons, bface, nsteps, dt_fixed, dt_out, diag, ws, ws_bytes, st);
  }
}

}  // namespace

extern "C" {

int ctmhd_required_ghosts(const ctmhd_params* p) {
  int rc = check_params(p);
  if (rc) return rc;
  return recon_halfwidth(p->recon) + 2;
}

int64_t ctmhd_box_elems(const ctmhd_box* b) {
  if (!b) return 0;
  int64_t e = 1;
  for (int d = 0; d < 3; ++d) e *= (int64_t)(b->n[d] + 2 * b->ng);
  return e;
}

size_t ctmhd_workspace_bytes(const ctmhd_params* p, const ctmhd_box* boxes, int nbox) {
  if (check_params(p) || !boxes || nbox < 1) return 0;
  size_t tb = p->precision == CTMHD_FP32 ? 4 : 8;
  if (nbox == 1) return box_ws_bytes(boxes[0], tb);
  return 0;
}

int ctmhd_step(const ctmhd_params* p, const ctmhd_box* box, double* const cons[5],
               double* const bface[3], int nsteps, const double* dt_fixed, double* dt_out,
               int64_t* diag, void* workspace, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  int rc = check_params(p);
  if (rc) return rc;
  if ((rc = check_box(p, box))) return rc;
  if (!cons || !bface) return fail(CTMHD_EARG, "state pointers are NULL");
  for (int m = 0; m < 5; ++m)
    if (!cons[m]) return fail(CTMHD_EARG, "a cons pointer is NULL");
  for (int a = 0; a < 3; ++a)
    if (!bface[a]) return fail(CTMHD_EARG, "a bface pointer is NULL");
  if (nsteps < 0) return fail(CTMHD_EARG, "nsteps must be >= 0");
  if (nsteps == 0) return CTMHD_OK;
  hipStream_t st = (hipStream_t)stream;
  if (p->precision == CTMHD_FP32)
    return step_box_t<float>(p, box, cons, bface, nsteps, dt_fixed, dt_out, diag, workspace,
                             ws_bytes, st);
  return step_box_t<double>(p, box, cons, bface, nsteps, dt_fixed, dt_out, diag, workspace,
                            ws_bytes, st);
}

int ctmhd_step_batched(const ctmhd_params* p, int nbox, const ctmhd_box* boxes,
                       double* const cons[5], double* const bface[3], int nsteps, int dt_mode,
                       const double* dt_fixed, double* dt_out, int64_t* diag, void* workspace,
                       size_t ws_bytes, void* stream) {
  (void)p; (void)nbox; (void)boxes; (void)cons; (void)bface; (void)nsteps; (void)dt_mode;
  (void)dt_fixed; (void)dt_out; (void)diag; (void)workspace; (void)ws_bytes; (void)stream;
  return fail(CTMHD_EUNSUPPORTED, "ctmhd_step_batched is not built yet");
}

int ctmhd_step_adjoint(const ctmhd_params* p, const ctmhd_box* box, const double* const cons_n[5],
                       const double* const bface_n[3], const double* dt,
                       const double* const g_cons[5], const double* const g_bface[3],
                       double* const g_cons_out[5], double* const g_bface_out[3], void* workspace,
                       size_t ws_bytes, void* stream) {
  (void)p; (void)box; (void)cons_n; (void)bface_n; (void)dt; (void)g_cons; (void)g_bface;
  (void)g_cons_out; (void)g_bface_out; (void)workspace; (void)ws_bytes; (void)stream;
  return fail(CTMHD_EUNSUPPORTED, "ctmhd_step_adjoint is not built yet");
}

int ctmhd_profile_events(void* const* events, int npairs) {
  if (npairs < 0) return fail(CTMHD_EARG, "npairs must be >= 0");
  g_prof_events = npairs > 0 ? events : nullptr;
  g_prof_pairs = events ? npairs : 0;
  g_prof_used = 0;
  return CTMHD_OK;
}

int ctmhd_profile_recorded(void) { return g_prof_used; }

const char* ctmhd_last_error(void) { return g_err; }

}  // extern "C"
