// ctmhd_device.h -- device-side structures and functions of libctmhd
// (gfx950), shared by the forward and the adjoint translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <type_traits>

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

__device__ __forceinline__ int gidx() { return blockIdx.x * blockDim.x + threadIdx.x; }

// Storage stride of axis d.  The x stride is 1 by construction; returning it
// as a constant (d is known at compile time at every call site) lets the
// compiler fold x-neighbour offsets into the load instructions.
__device__ __forceinline__ int gstride(const Geom& G, int d) { return d == 0 ? 1 : G.st[d]; }

// Workgroups are dispatched to the 8 XCDs of the chip round-robin (workgroup
// i on XCD i mod 8), and each XCD has its own L2.  This permutation of the
// tiles of a launch gives each XCD a contiguous run of them, so that the
// neighbouring rows and planes a stencil reads were brought into the same
// L2.  It is a bijection on [0, gridDim.x): results do not depend on it.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile() {
  const int nb = (int)gridDim.x, b = (int)blockIdx.x;
  const int per = nb / kXcds;
  if (b >= per * kXcds) return b;
  return (b % kXcds) * per + b / kXcds;
}

// The banded alternative: XCD x takes tiles [j C + x m, j C + (x+1) m) of
// every chunk j of C = 8 m consecutive tiles, so that all XCDs sweep the box
// together, each on its own band of the same chunk.  With a chunk about one
// plane of a large box, the planes a z stencil re-reads are then shared by the
// whole chip in the Infinity Cache instead of being re-fetched from HBM by
// each XCD on its own.  A bijection on [0, gridDim.x) (the tail beyond the
// last complete chunk keeps its order); m = 0 gives xcd_tile().
__device__ __forceinline__ int xcd_band_tile(int m) {
  if (m <= 0) return xcd_tile();
  const int nb = (int)gridDim.x, b = (int)blockIdx.x;
  const int C = kXcds * m;
  if (b >= nb / C * C) return b;
  const int k = b / kXcds;
  return (k / m) * C + (b % kXcds) * m + k % m;
}

struct State {
  double* c[5];
  double* b[3];
};

constexpr int kBlock = 256;
constexpr int kMaxSlots = 64;  // spread of the CFL maximum over atomics

template <typename T>
struct Work {
  T* prim[8];       // rho, u0, u1, u2, p, bc0, bc1, bc2 (B25a / FS18 only)
  T* ecell[3];      // cell-centred ideal EMF (B25a)
  // Stored first steps of the two-step corner reconstructions (when
  // first_step_stored), the values on both sides (0 lower, 1 upper) of the
  // interface at each position.  B25a: ecell[c] with order 0 along a = c+1
  // first, order 1 along b = c+2 first.  FS18: velocity u_v along axis d.
  T* b25f[3][2][2];
  T* fsf[3][3][2];
  T* F[2][3][5];    // per stage, direction, component (global momentum order)
  T* ap[3];
  T* am[3];
  T* us[3];
  T* E[2][3];       // per stage, edge EMFs
  uint8_t* flag;    // interior cells, x0 fastest; a level of boxes: every storage position
  // CFL maxima (bits of non-negative doubles), kMaxSlots each: [0] fused into
  // the stage-2 update, [1] recomputed by a stage-2 fix-up
  unsigned long long* smax;
  double* dt;       // the step's dt
  int* stop;        // 1 once a non-finite dt was seen
  int* nflag;       // flagged cells of stage 0 / 1; nflag[2]: stage-2 fix-up ran
};

inline int nblocks(long long n) { return (int)((n + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------
__global__ void k_init(int* stop, unsigned long long* smax, int* nflag) {
  int t = threadIdx.x;
  if (blockIdx.x != 0) return;
  if (t == 0) {
    *stop = 0;
    nflag[0] = nflag[1] = nflag[2] = 0;
  }
  if (t < 2 * kMaxSlots) smax[t] = 0ull;
}

__device__ __forceinline__ int pwrap(int s, int g, int n) {
  int q = (s - g) % n;
  if (q < 0) q += n;
  return q + g;
}

// Periodic ghost fill of all 8 fields (faces follow the same rule: the face at
// storage index s is the lower face of cell s).  Used on the caller's state at
// the start of a call; later states get their ghost images from k_update.
__device__ __forceinline__ void wrap_at(const State& S, const Geom& G, int t) {
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

__global__ void k_wrap(State S, Geom G, const int* stop) {
  if (*stop) return;
  wrap_at(S, G, gidx());
}

// Grid-stride copy of a state (any grid size).
__global__ void k_copy(State dst, State src, int elems, const int* only_if_stop) {
  if (only_if_stop && !*only_if_stop) return;
  for (int t = gidx(); t < elems; t += gridDim.x * blockDim.x) {
#pragma unroll
    for (int m = 0; m < 5; ++m) dst.c[m][t] = src.c[m][t];
#pragma unroll
    for (int a = 0; a < 3; ++a) dst.b[a][t] = src.b[a][t];
  }
}

// ---------------------------------------------------------------------------
// Cell primitives from the conserved state (eq. state:primitive), FP64.
// ---------------------------------------------------------------------------
// The eleven loads behind the primitives of one cell: the conserved state
// and the two faces of the cell along each axis.  Split from the arithmetic
// so that a marching thread can issue the loads of its next cell before the
// stores of the current one (the compiler cannot move loads of the state
// across stores to the workspace, which it must assume may alias).
struct CellRaw {
  double c[5], bl[3], bh[3];
};

__device__ __forceinline__ void cell_load(const State& S, const Geom& G, int s, CellRaw& R) {
#pragma unroll
  for (int m = 0; m < 5; ++m) R.c[m] = S.c[m][s];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    R.bl[d] = S.b[d][s];
    R.bh[d] = S.b[d][s + G.st[d]];
  }
}

__device__ __forceinline__ void raw_prim(const CellRaw& R, double gamma, double& rho, double u[3],
                                         double& p, double bc[3]) {
  rho = R.c[0];
  double ir = trcp(rho);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    u[d] = R.c[1 + d] * ir;
    bc[d] = 0.5 * (R.bl[d] + R.bh[d]);
  }
  p = (gamma - 1.0) * (R.c[4] - 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) -
                       0.5 * (bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]));
}

__device__ __forceinline__ void cell_prim(const State& S, const Geom& G, int s, double gamma,
                                          double& rho, double u[3], double& p, double bc[3]) {
  CellRaw R;
  cell_load(S, G, s, R);
  raw_prim(R, gamma, rho, u, p, bc);
}

// CFL signal speed of one cell (eq. resistivity:cfl; the resistive term
// enters as the speed 2 eta / dx_min, i.e. 2 eta / dx_min^2 per unit length).
// NaN propagates.
__device__ __forceinline__ double cfl_signal(double rho, const double u[3], double p,
                                             const double bc[3], const Geom& G, double gamma,
                                             double sres) {
  double s = sres;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double cf = fast_speed<double>(rho, p, bc[d], bc[(d + 1) % 3], bc[(d + 2) % 3], gamma);
    double sd = (fabs(u[d]) + cf) * G.idx[d];
    s = (sd > s || sd != sd) ? sd : s;
  }
  return s;
}

// Block maximum of a non-negative (or NaN) double, folded into one of
// kMaxSlots device slots by an atomic max on its bit pattern (a NaN has
// larger bits than +inf as an unsigned integer).  All threads must call.
__device__ __forceinline__ void block_max_to_slots(double s, unsigned long long* slots, int slot) {
  __shared__ unsigned long long red[kBlock / 64];
  unsigned long long bits = (unsigned long long)__double_as_longlong(s);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long ob = __shfl_xor(bits, o, 64);
    bits = ob > bits ? ob : bits;
  }
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = bits;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) m = red[q] > m ? red[q] : m;
    atomicMax(&slots[slot], m);
  }
}

// CFL signal of interior cell t (0 for t outside the box).
__device__ __forceinline__ double dt_sig_at(const State& S, const Geom& G, double gamma,
                                            double sres, int t) {
  int ninter = G.n[0] * G.n[1] * G.n[2];
  if (t >= ninter) return 0.0;
  int i = t % G.n[0] + G.g;
  int q = t / G.n[0];
  int j = q % G.n[1] + G.g;
  int k = q / G.n[1] + G.g;
  int c = i + G.st[1] * j + G.st[2] * k;
  double rho, u[3], p, bc[3];
  cell_prim(S, G, c, gamma, rho, u, p, bc);
  return cfl_signal(rho, u, p, bc, G, gamma, sres);
}

// CFL maximum of a whole state (start of a call).
__global__ void __launch_bounds__(kBlock) k_dt(State S, Geom G, double gamma, double sres,
                                               unsigned long long* slots, const int* stop) {
  if (*stop) return;
  int ninter = G.n[0] * G.n[1] * G.n[2];
  double s = 0.0;
  for (int t = gidx(); t < ninter; t += gridDim.x * blockDim.x) {
    double v = dt_sig_at(S, G, gamma, sres, t);
    s = (v > s || v != v) ? v : s;
  }
  block_max_to_slots(s, slots, blockIdx.x % kMaxSlots);
}

// dt of a step.  smax[0..kMaxSlots) holds the CFL maximum of the step's
// starting state unless the previous step's second stage was fixed up
// (nflag[2]), whose recomputed maximum is in smax[kMaxSlots..).  Resets the
// slots, the flag counters and this step's diagnostics.
__global__ void k_dt_final(unsigned long long* smax, int* nflag, double cfl,
                           const double* dt_fixed, double* dt, double* dt_out, int* stop,
                           long long* diag) {
  int t = threadIdx.x;
  __shared__ unsigned long long m;
  if (t == 0) {
    const unsigned long long* src = nflag[2] ? smax + kMaxSlots : smax;
    unsigned long long v = 0;
    for (int q = 0; q < kMaxSlots; ++q) v = src[q] > v ? src[q] : v;
    m = v;
  }
  __syncthreads();
  if (t < 2 * kMaxSlots) smax[t] = 0ull;
  if (t != 0) return;
  nflag[0] = nflag[1] = nflag[2] = 0;
  if (diag) {
    diag[0] = diag[1] = diag[2] = 0;
    diag[3] = *stop ? 1 : 0;
  }
  if (*stop) {
    *dt = 0.0;
    if (dt_out) *dt_out = 0.0;
    return;
  }
  double v = dt_fixed ? *dt_fixed : cfl / __longlong_as_double((long long)m);
  if (!(v > 0.0) || !__builtin_isfinite(v)) {
    *stop = 1;
    if (diag) diag[3] = 1;
  }
  *dt = v;
  if (dt_out) *dt_out = v;
}

// ---------------------------------------------------------------------------
// Cell-centred fields for the two-step EMF schemes (B25a: ideal EMF; FS18:
// velocity), over cells whose upper faces are stored.
// ---------------------------------------------------------------------------
template <typename T, int EMF>
__device__ __forceinline__ void prim_at(const State& S, const Geom& G, const Work<T>& W,
                                        double gamma, int t) {
  if (t >= G.elems) return;
  int i = t % G.N[0];
  int q = t / G.N[0];
  int j = q % G.N[1];
  int k = q / G.N[1];
  if (i >= G.N[0] - 1 || j >= G.N[1] - 1 || k >= G.N[2] - 1) return;
  double rho, u[3], p, b[3];
  cell_prim(S, G, t, gamma, rho, u, p, b);
  if (EMF == kB25A) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      int a = (c + 1) % 3, bb = (c + 2) % 3;
      // eq. emf:b25a-emf-centre in the stencil type
      W.ecell[c][t] = -(T)u[a] * (T)b[bb] + (T)u[bb] * (T)b[a];
    }
  } else {
    W.prim[1][t] = (T)u[0];
    W.prim[2][t] = (T)u[1];
    W.prim[3][t] = (T)u[2];
  }
}

template <typename T, int EMF>
__global__ void __launch_bounds__(kBlock) k_prim(State S, Geom G, Work<T> W, double gamma,
                                                 const int* stop) {
  if (*stop) return;
  prim_at<T, EMF>(S, G, W, gamma, gidx());
}

// eta j_c at the edge stored at s (lower corner in a and b), eq.
// resistivity:current-stencil.
template <typename T>
__device__ __forceinline__ T eta_j(const State& S, const Geom& G, int s, int c, T eta) {
  int a = (c + 1) % 3, b = (c + 2) % 3;
  double j = (S.b[b][s] - S.b[b][s - gstride(G, a)]) * G.idx[a] -
             (S.b[a][s] - S.b[a][s - gstride(G, b)]) * G.idx[b];
  return eta * (T)j;
}

// Joule energy flux at the x_a face stored at s (Sec. 2.4): (eta j x b).n_a
// with eta j averaged over the face's bounding edges and b the mean of the two
// adjacent cells' cell-averaged field.
template <typename T>
__device__ __forceinline__ T joule(const State& S, const Geom& G, int s, int a, T eta) {
  int b = (a + 1) % 3, c = (a + 2) % 3;
  const int sb = gstride(G, b), sc = gstride(G, c);
  T eb = T(0.5) * (eta_j<T>(S, G, s, b, eta) + eta_j<T>(S, G, s + sc, b, eta));
  T ec = T(0.5) * (eta_j<T>(S, G, s, c, eta) + eta_j<T>(S, G, s + sb, c, eta));
  int l = s - gstride(G, a);
  T bbl = (T)(0.5 * (S.b[b][l] + S.b[b][l + sb]));
  T bbr = (T)(0.5 * (S.b[b][s] + S.b[b][s + sb]));
  T bcl = (T)(0.5 * (S.b[c][l] + S.b[c][l + sc]));
  T bcr = (T)(0.5 * (S.b[c][s] + S.b[c][s + sc]));
  return eb * (T(0.5) * (bcl + bcr)) - ec * (T(0.5) * (bbl + bbr));
}

// The same Joule flux at the x_a face between cells lo and hi from values the
// face pass already holds: each cell's transverse face fields
// t = {b_b lower, b_b upper, b_c lower, b_c upper} (b, c cyclic after a),
// the face's normal field bn = b_a, and its four in-plane neighbours
// nb = {b_a at -x_b, +x_b, -x_c, +x_c}.  Every edge current, cell-averaged
// field and product is formed as in joule().
template <typename T>
__device__ __forceinline__ T joule_pair(const Geom& G, int a, const double lo[4],
                                        const double hi[4], double bn, const double nb[4], T eta) {
  // no fused multiply-adds: the single-box and batched face kernels inline
  // this into different code, and must give the same bits
#pragma clang fp contract(off)
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  // eta j_b at the edges s and s + x_c, eta j_c at the edges s and s + x_b
  T eb = T(0.5) * (eta * (T)((bn - nb[2]) * G.idx[c] - (hi[2] - lo[2]) * G.idx[a]) +
                   eta * (T)((nb[3] - bn) * G.idx[c] - (hi[3] - lo[3]) * G.idx[a]));
  T ec = T(0.5) * (eta * (T)((hi[0] - lo[0]) * G.idx[a] - (bn - nb[0]) * G.idx[b]) +
                   eta * (T)((hi[1] - lo[1]) * G.idx[a] - (nb[1] - bn) * G.idx[b]));
  T bbl = (T)(0.5 * (lo[0] + lo[1]));
  T bbr = (T)(0.5 * (hi[0] + hi[1]));
  T bcl = (T)(0.5 * (lo[2] + lo[3]));
  T bcr = (T)(0.5 * (hi[2] + hi[3]));
  return eb * (T(0.5) * (bcl + bcr)) - ec * (T(0.5) * (bbl + bbr));
}

// ---------------------------------------------------------------------------
// Face pass (Sec. 2.2, eqs. emf:alpha-pm, emf:q26-facevel).
// ---------------------------------------------------------------------------
// Face ranges of one stage.  Faces of direction a: s_a in [lo_a, lo_a +
// nf_a), transverse coordinates in [tlo, tlo + tlen) on both axes.
struct FacePlan {
  int lo[3], nf[3];   // along the face normal
  int tlo, tlen[3];   // transverse range start (same on every axis) and length per axis
  int ulo[3], ulen[3];  // faces read by the update (Joule flux only there)
  // x part: one wavefront per (row, segment)
  int xseg, xnseg, xwaves, xrows, xblocks;  // xwaves = items; xrows items per wavefront
  // y and z parts: lane blocks x chunks
  int chunk[3], nchunk[3], lanes[3], lblocks[3], blocks[3];
  int total_blocks;
};

// Face-local primitive of a cell for the face normal a (FP64 recovery, then T).
template <typename T>
__device__ __forceinline__ void face_local_raw(const CellRaw& R, int a, double gamma, T v[7]) {
  double rho, u[3], p, bc[3];
  raw_prim(R, gamma, rho, u, p, bc);
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  v[0] = (T)rho;
  v[1] = (T)u[a];
  v[2] = (T)u[b];
  v[3] = (T)u[c];
  v[4] = (T)p;
  v[5] = (T)bc[b];
  v[6] = (T)bc[c];
}

template <typename T>
__device__ __forceinline__ void face_local(const State& S, const Geom& G, int s, int a, double gamma,
                                           T v[7]) {
  CellRaw R;
  cell_load(S, G, s, R);
  face_local_raw<T>(R, a, gamma, v);
}

template <typename T, int RIEMANN>
__device__ __forceinline__ int solve_and_store(const Work<T>& W, int s, int a, int stage,
                                               const T qL[7], const T qR[7], double bn_d,
                                               double gamma_d, T jflux) {
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  // the solver's arithmetic type: T, or float64 for kHLLD64 / kLLF64
  using RT = typename std::conditional<(RIEMANN >= kHLLD64), double, T>::type;
  FState<RT> L{(RT)qL[0], (RT)qL[1], (RT)qL[2], (RT)qL[3], (RT)qL[4], (RT)qL[5], (RT)qL[6]};
  FState<RT> R{(RT)qR[0], (RT)qR[1], (RT)qR[2], (RT)qR[3], (RT)qR[4], (RT)qR[5], (RT)qR[6]};
  const RT bn = (RT)bn_d;  // normal field of the face, S.b[a][s]
  RT Fr[5];
  T F[5], ap, am;
  int fb = 0;
  if (RIEMANN == kHLLD || RIEMANN == kHLLD64) {
    RT SL, SR;
    fb = hlld_flux(L, R, bn, (RT)gamma_d, Fr, SL, SR);
    ap = (T)tmax(RT(0), SR);
    am = (T)tmax(RT(0), -SL);
  } else {
    ap = am = (T)llf_flux(L, R, bn, (RT)gamma_d, Fr);
  }
#pragma unroll
  for (int m = 0; m < 5; ++m) F[m] = (T)Fr[m];
  F[4] += jflux;  // Joule energy flux (zero outside the faces the update reads, or eta = 0)
  // Streaming stores: no later access of this kernel reads them, and keeping
  // them out of the L2 leaves it to the state rows the marches re-read.
  __builtin_nontemporal_store(F[0], &W.F[stage][a][0][s]);
  __builtin_nontemporal_store(F[1], &W.F[stage][a][1 + a][s]);
  __builtin_nontemporal_store(F[2], &W.F[stage][a][1 + b][s]);
  __builtin_nontemporal_store(F[3], &W.F[stage][a][1 + c][s]);
  __builtin_nontemporal_store(F[4], &W.F[stage][a][4][s]);
  __builtin_nontemporal_store(ap, &W.ap[a][s]);
  __builtin_nontemporal_store(am, &W.am[a][s]);
  __builtin_nontemporal_store((ap * (T)L.un + am * (T)R.un) * trcp(ap + am), &W.us[a][s]);
  return fb;
}

// Whether the face pass's x_a face at s3 is one the update reads: [g, g+n]
// along the normal, [g, g+n) across (the Joule flux is needed only there).
__device__ __forceinline__ bool face_in_update(const FacePlan& FP, const int s3[3], int a) {
  bool in_upd = true;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    in_upd = in_upd && s3[d] >= FP.ulo[d] && s3[d] < FP.ulo[d] + FP.ulen[d] + (d == a ? 1 : 0);
  return in_upd;
}

// A cell's transverse face fields for the normal a, as joule_pair takes them.
__device__ __forceinline__ void cell_tfaces(const CellRaw& R, int a, double t[4]) {
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  t[0] = R.bl[b];
  t[1] = R.bh[b];
  t[2] = R.bl[c];
  t[3] = R.bh[c];
}

// The four in-plane neighbours of the normal field of the x_a face at s, as
// joule_pair takes them.
__device__ __forceinline__ void face_nb(const State& S, const Geom& G, int s, int a,
                                        double nb[4]) {
  const int sb = gstride(G, (a + 1) % 3), sc = gstride(G, (a + 2) % 3);
  const double* ba = S.b[a];
  nb[0] = ba[s - sb];
  nb[1] = ba[s + sb];
  nb[2] = ba[s - sc];
  nb[3] = ba[s + sc];
}

// Value of the neighbouring lane (l - 1 for lane_prev, l + 1 for lane_next)
// by a DPP whole-wavefront shift, a VALU move; lane 0 (63) receives 0.
__device__ __forceinline__ int dpp_prev(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false);  // wave_shr:1
}
__device__ __forceinline__ int dpp_next(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false);  // wave_shl:1
}
__device__ __forceinline__ double lane_prev(double v) {
  return __hiloint2double(dpp_prev(__double2hiint(v)), dpp_prev(__double2loint(v)));
}
__device__ __forceinline__ double lane_next(double v) {
  return __hiloint2double(dpp_next(__double2hiint(v)), dpp_next(__double2loint(v)));
}
__device__ __forceinline__ float lane_prev(float v) {
  return __int_as_float(dpp_prev(__float_as_int(v)));
}
__device__ __forceinline__ float lane_next(float v) {
  return __int_as_float(dpp_next(__float_as_int(v)));
}

// x faces: one wavefront holds 64 consecutive cells of a row; lane l forms
// the primitives, the limited slope and the upper interface value of its own
// cell, neighbours come from whole-wavefront DPP shifts by one lane, and the
// face at lane l takes the upper value of lane l-1.  Faces at lanes [r+1, 63-r] are resolved
// (overlapping segments).
template <int RECON, typename T>
__device__ __forceinline__ void recon_lanes(T q, T& qm, T& qp) {
  if constexpr (RECON == kPC) {
    qm = q;
    qp = q;
  } else if constexpr (RECON == kPLM_MC || RECON == kPLM_MM) {
    T s = T(0.5) * plm_slope<RECON>(lane_prev(q), q, lane_next(q));
    qm = q - s;
    qp = q + s;
  } else {
    T qr = lane_next(q);
    T dm = ppm_slope(lane_prev(q), q, qr);
    T ihi = ppm_iface(q, qr, dm, lane_next(dm));
    T ilo = lane_prev(ihi);
    ppm_constrain(q, ilo, ihi);
    qm = ilo;
    qp = ihi;
  }
}

template <typename T, int RECON, int RIEMANN>
__device__ void faces_x(const State& S, const Geom& G, const Work<T>& W, const FacePlan& FP,
                        int wave, int stage, double gamma, double eta, int& nfb) {
  constexpr int r = recon_halfwidth(RECON);
  const int lane = threadIdx.x & 63;
  // this wavefront takes items [it, end) (item = row * xnseg + segment) and
  // loads the cells of the next item before it resolves the current one
  int it = wave * FP.xrows;
  const int end = it + FP.xrows < FP.xwaves ? it + FP.xrows : FP.xwaves;
  auto locate = [&](int item, int& x, int& y, int& z) {
    const int row = item / FP.xnseg, seg = item % FP.xnseg;
    y = FP.tlo + row % FP.tlen[1];
    z = FP.tlo + row / FP.tlen[1];
    x = FP.lo[0] - (r + 1) + seg * FP.xseg + lane;
    const int xc = x < 0 ? 0 : (x > G.N[0] - 2 ? G.N[0] - 2 : x);  // loads stay in the box
    return xc + G.st[1] * y + G.st[2] * z;
  };
  // whether this lane's face of an item needs the Joule flux; if so its
  // normal-field neighbours are loaded with the item's cell
  auto joule_nb = [&](int x, int y, int z, int s, double nb[4]) {
    const int s3[3] = {x, y, z};
    const bool j = eta > 0.0 && lane >= r + 1 && lane <= 63 - r && x >= FP.lo[0] &&
                   x < FP.lo[0] + FP.nf[0] && face_in_update(FP, s3, 0);
    if (j) face_nb(S, G, s, 0, nb);
    return j;
  };
  int xn, yn, zn;
  int sn = locate(it, xn, yn, zn);
  CellRaw nxt;
  cell_load(S, G, sn, nxt);
  double nb_nxt[4] = {0.0, 0.0, 0.0, 0.0};
  bool j_nxt = joule_nb(xn, yn, zn, sn, nb_nxt);
  for (; it < end; ++it) {  // wavefront-uniform trip count (cross-lane shuffles below)
    const CellRaw cur = nxt;
    const int x = xn, s = sn;
    double nb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) nb[k] = nb_nxt[k];
    const bool jf_need = j_nxt;
    if (it + 1 < end) {
      sn = locate(it + 1, xn, yn, zn);
      cell_load(S, G, sn, nxt);
      j_nxt = joule_nb(xn, yn, zn, sn, nb_nxt);
    }
    T v[7];
    face_local_raw<T>(cur, 0, gamma, v);
    T qm[7], qp[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) recon_lanes<RECON>(v[k], qm[k], qp[k]);
    T qL[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) qL[k] = lane_prev(qp[k]);
    // transverse face fields of this lane's cell and of the cell below it
    double thi[4], tlo[4];
    cell_tfaces(cur, 0, thi);
#pragma unroll
    for (int k = 0; k < 4; ++k) tlo[k] = lane_prev(thi[k]);
    const bool face = lane >= r + 1 && lane <= 63 - r && x >= FP.lo[0] && x < FP.lo[0] + FP.nf[0];
    if (face) {
      const T jf = jf_need ? joule_pair<T>(G, 0, tlo, thi, cur.bl[0], nb, (T)eta) : T(0);
      nfb += solve_and_store<T, RIEMANN>(W, s, 0, stage, qL, qm, cur.bl[0], gamma, jf);
    }
  }
}

// y / z faces: lanes over the transverse plane (x fastest), each thread
// marches along the face normal A through a chunk of faces, streaming the
// cells through a reconstruction pipeline (one slope and one interface value
// per cell); each cell is loaded and reconstructed once.
template <typename T, int RECON, int RIEMANN, int A>
__device__ void faces_march(const State& S, const Geom& G, const Work<T>& W, const FacePlan& FP,
                            int lblock, int chunk, int stage, double gamma, double eta, int& nfb) {
  constexpr int r = recon_halfwidth(RECON);
  const int lane = lblock * kBlock + threadIdx.x;
  if (lane >= FP.lanes[A]) return;
  const int C = A == 1 ? 2 : 1;  // transverse axes: x (fastest) and C
  int s3[3];
  s3[0] = FP.tlo + lane % FP.tlen[0];
  s3[C] = FP.tlo + lane / FP.tlen[0];
  const int f0 = FP.lo[A] + chunk * FP.chunk[A];
  int f1 = f0 + FP.chunk[A];
  if (f1 > FP.lo[A] + FP.nf[A]) f1 = FP.lo[A] + FP.nf[A];
  const int sa = G.st[A];
  const int base = s3[0] + G.st[C] * s3[C];
  ReconStream<RECON, T> rs[7];
  T qprev[7];
  // cells f0-1-r .. f1-1+r; the pushes before cell f0-1+r only warm up the
  // pipeline.  The loads of cell q+1 and the normal field of the face it
  // completes are issued before the stores of the face completed by cell q.
  int q = f0 - 1 - r;
  CellRaw nxt;
  cell_load(S, G, base + q * sa, nxt);
  double bn_next = 0.0;  // read only for the faces f0 .. f1-1
  // Joule flux of face q (between cells q-1 and q), formed when cell q
  // arrives and used r pushes later, when the face is solved: jd[k] holds the
  // flux of face q-k
  double tprev[4] = {0.0, 0.0, 0.0, 0.0};
  T jd[r + 1];
#pragma unroll
  for (int k = 0; k <= r; ++k) jd[k] = T(0);
  // the normal-field neighbours of face q+1 are loaded with cell q+1 when
  // that face needs the Joule flux
  double nb_next[4] = {0.0, 0.0, 0.0, 0.0};
  bool j_next = false;
  for (; q <= f1 - 1 + r; ++q) {
    const CellRaw cur = nxt;
    const double bn = bn_next;
    double nb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) nb[k] = nb_next[k];
    const bool jq = j_next;
    if (q < f1 - 1 + r) {
      cell_load(S, G, base + (q + 1) * sa, nxt);
      if (q + 1 - r >= f0) bn_next = S.b[A][base + (q + 1 - r) * sa];
      j_next = false;
      if (eta > 0.0 && q + 1 >= f0 && q + 1 < f1) {
        s3[A] = q + 1;
        j_next = face_in_update(FP, s3, A);
        if (j_next) face_nb(S, G, base + (q + 1) * sa, A, nb_next);
      }
    }
#pragma unroll
    for (int k = r; k > 0; --k) jd[k] = jd[k - 1];
    double tcur[4];
    cell_tfaces(cur, A, tcur);
    jd[0] = jq ? joule_pair<T>(G, A, tprev, tcur, cur.bl[A], nb, (T)eta) : T(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) tprev[k] = tcur[k];
    T v[7];
    face_local_raw<T>(cur, A, gamma, v);
    const int cell = q - r;  // completed by this push
    T qm[7], qp[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) rs[k].push(v[k], qm[k], qp[k]);
    if (cell >= f0) {
      const int s = base + cell * sa;
      nfb += solve_and_store<T, RIEMANN>(W, s, A, stage, qprev, qm, bn, gamma, jd[r]);
    }
#pragma unroll
    for (int k = 0; k < 7; ++k) qprev[k] = qp[k];
  }
}

// One virtual block (256 threads) of the face pass.
template <typename T, int RECON, int RIEMANN>
__device__ __forceinline__ void faces_block(const State& S, const Geom& G, const Work<T>& W,
                                            const FacePlan& FP, int b, int stage, double gamma,
                                            double eta, int& nfb) {
  // long-running marching blocks first, the short x-face wavefronts fill in
  if (b < FP.blocks[2]) {
    faces_march<T, RECON, RIEMANN, 2>(S, G, W, FP, b / FP.nchunk[2], b % FP.nchunk[2], stage,
                                      gamma, eta, nfb);
  } else if ((b -= FP.blocks[2]) < FP.blocks[1]) {
    faces_march<T, RECON, RIEMANN, 1>(S, G, W, FP, b / FP.nchunk[1], b % FP.nchunk[1], stage,
                                      gamma, eta, nfb);
  } else {
    b -= FP.blocks[1];
    const int wave = b * (kBlock / 64) + (threadIdx.x >> 6);
    if (wave * FP.xrows < FP.xwaves)
      faces_x<T, RECON, RIEMANN>(S, G, W, FP, wave, stage, gamma, eta, nfb);
  }
}

template <typename T, int RECON, int RIEMANN>
__global__ void __launch_bounds__(kBlock)
    k_faces(State S, Geom G, Work<T> W, FacePlan FP, int stage, double gamma, double eta,
            long long* diag, const int* stop) {
  if (*stop) return;
  int nfb = 0;
  faces_block<T, RECON, RIEMANN>(S, G, W, FP, blockIdx.x, stage, gamma, eta, nfb);
  if (diag && nfb) atomicAdd((unsigned long long*)&diag[2], (unsigned long long)nfb);
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

// Whether the two-step corner reconstructions of B25a and FS18 store their
// first step once per stage (PPM) or the edge pass recomputes it for every
// edge that reads it (PC, PLM: there the stored arrays cost more traffic than
// the short stencils they save).
__host__ __device__ constexpr bool first_step_stored(int emf, int recon) {
  return emf != kQ26 && recon == kPPM;
}

// The first step of the two-step corner reconstructions at position t, for
// every field and axis the edges use; 0 where the stencil leaves the box.
template <typename T, int RECON, int EMF>
__device__ __forceinline__ void first_step_at(const Geom& G, const Work<T>& W, int t) {
  if (t >= G.elems) return;
  const int s3[3] = {t % G.N[0], (t / G.N[0]) % G.N[1], t / (G.N[0] * G.N[1])};
  constexpr int r = recon_halfwidth(RECON);
  constexpr int nf = EMF == kB25A ? 2 : 3;  // orders of ecell[c] / axes of u_v
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int o = 0; o < nf; ++o) {
      const int d1 = EMF == kB25A ? (o == 0 ? (c + 1) % 3 : (c + 2) % 3) : o;
      const T* A = EMF == kB25A ? W.ecell[c] : W.prim[1 + c];
      T lo = T(0), hi = T(0);
      if (s3[d1] - 1 - r >= 0 && s3[d1] + r < G.N[d1])
        iface_along<RECON>(A, t, gstride(G, d1), lo, hi);
      T* const* out = EMF == kB25A ? W.b25f[c][o] : W.fsf[c][o];
      __builtin_nontemporal_store(lo, &out[0][t]);  // read by the edge pass only
      __builtin_nontemporal_store(hi, &out[1][t]);
    }
}

template <typename T, int RECON, int EMF>
__global__ void __launch_bounds__(kBlock) k_first_step(Geom G, Work<T> W, const int* stop) {
  if (*stop) return;
  first_step_at<T, RECON, EMF>(G, W, gidx());
}

// Second step of a two-step reconstruction from the stored first-step
// values F[0] (lower side) and F[1] (upper side along d1), along d2 with
// stride st2: the same values as two_step.
template <int RECON, typename T>
__device__ __forceinline__ void second_step(T* const F[2], int s, int st2, T out[4]) {
  T seqlo[6], seqhi[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    seqlo[m] = stencil_uses<RECON>(m) ? F[0][s + (m - 3) * st2] : T(0);
    seqhi[m] = stencil_uses<RECON>(m) ? F[1][s + (m - 3) * st2] : T(0);
  }
  T l0, l1, h0, h1;
  recon_iface<RECON>(seqlo, l0, l1);
  recon_iface<RECON>(seqhi, h0, h1);
  out[0] = l0;
  out[1] = h0;
  out[2] = l1;
  out[3] = h1;
}

// Q26 corner EMFs (eq. emf:q26) from the edge-reconstructed face velocities
// u*_a (B/T along x_b), u*_b (L/R along x_a) and face fields, combined by LD04
// (eq. emf:ld04) with the edge wavespeeds (eq. emf:alpha-edge).
template <typename T>
__device__ __forceinline__ T q26_ld04(T uaB, T uaT, T ubL, T ubR, T baB, T baT, T bbL, T bbR,
                                      T apa, T ama, T apb, T amb) {
  const T e0 = -uaB * bbL + ubL * baB;
  const T e1 = -uaB * bbR + ubR * baB;
  const T e2 = -uaT * bbL + ubL * baT;
  const T e3 = -uaT * bbR + ubR * baT;
  return ld04(e0, e1, e2, e3, apa, ama, apb, amb, baB, baT, bbL, bbR);
}

// The Q26 EMF of the c edge at s from its edge-reconstructed face fields and
// face velocities: edge wave speeds (eq. emf:alpha-edge), Q26 corners with
// LD04, plus eta j.
template <typename T>
__device__ __forceinline__ T q26_edge(const State& S, const Geom& G, const Work<T>& W, int s, int c,
                                      T baB, T baT, T bbL, T bbR, T uaB, T uaT, T ubL, T ubR,
                                      double eta_d) {
  const int a = (c + 1) % 3, b = (c + 2) % 3;
  const int sa = gstride(G, a), sb = gstride(G, b);
  T apa = tmax(W.ap[a][s - sb], W.ap[a][s]);
  T ama = tmax(W.am[a][s - sb], W.am[a][s]);
  T apb = tmax(W.ap[b][s - sa], W.ap[b][s]);
  T amb = tmax(W.am[b][s - sa], W.am[b][s]);
  T eps = q26_ld04(uaB, uaT, ubL, ubR, baB, baT, bbL, bbR, apa, ama, apb, amb);
  if (eta_d > 0.0) eps += eta_j<T>(S, G, s, c, (T)eta_d);
  return eps;
}

template <typename T, int RECON, int EMF>
__device__ __forceinline__ T edge_emf(const State& S, const Geom& G, const Work<T>& W, int s, int c,
                                      double eta_d) {
  const int a = (c + 1) % 3, b = (c + 2) % 3;
  const int sa = gstride(G, a), sb = gstride(G, b);
  T baB, baT, bbL, bbR;
  iface_along_d<RECON>(S.b[a], s, sb, baB, baT);
  iface_along_d<RECON>(S.b[b], s, sa, bbL, bbR);
  if (EMF == kQ26) {
    T uaB, uaT, ubL, ubR;
    iface_along<RECON>(W.us[a], s, sb, uaB, uaT);
    iface_along<RECON>(W.us[b], s, sa, ubL, ubR);
    return q26_edge<T>(S, G, W, s, c, baB, baT, bbL, bbR, uaB, uaT, ubL, ubR, eta_d);
  }
  T apa = tmax(W.ap[a][s - sb], W.ap[a][s]);
  T ama = tmax(W.am[a][s - sb], W.am[a][s]);
  T apb = tmax(W.ap[b][s - sa], W.ap[b][s]);
  T amb = tmax(W.am[b][s - sa], W.am[b][s]);
  T e[4];  // LB, RB, LT, RT
  if (EMF == kB25A) {
    T ab[4], ba[4];  // [x_a x_b]: index sa_side + 2 sb_side; [x_b x_a]: sb_side + 2 sa_side
    if constexpr (first_step_stored(EMF, RECON)) {
      second_step<RECON>(W.b25f[c][0], s, sb, ab);
      second_step<RECON>(W.b25f[c][1], s, sa, ba);
    } else {
      two_step<RECON>(W.ecell[c], s, sa, sb, ab);
      two_step<RECON>(W.ecell[c], s, sb, sa, ba);
    }
    e[0] = T(0.5) * (ab[0] + ba[0]);
    e[1] = T(0.5) * (ab[1] + ba[2]);
    e[2] = T(0.5) * (ab[2] + ba[1]);
    e[3] = T(0.5) * (ab[3] + ba[3]);
  } else {
    T ua_ab[4], ua_ba[4], ub_ab[4], ub_ba[4];
    if constexpr (first_step_stored(EMF, RECON)) {
      second_step<RECON>(W.fsf[a][a], s, sb, ua_ab);
      second_step<RECON>(W.fsf[a][b], s, sa, ua_ba);
      second_step<RECON>(W.fsf[b][a], s, sb, ub_ab);
      second_step<RECON>(W.fsf[b][b], s, sa, ub_ba);
    } else {
      const T* ua = W.prim[1 + a];
      const T* ub = W.prim[1 + b];
      two_step<RECON>(ua, s, sa, sb, ua_ab);
      two_step<RECON>(ua, s, sb, sa, ua_ba);
      two_step<RECON>(ub, s, sa, sb, ub_ab);
      two_step<RECON>(ub, s, sb, sa, ub_ba);
    }
    const int perm[4] = {0, 2, 1, 3};  // corner q = sa_side + 2 sb_side -> [x_b x_a] index
    const T bbX[2] = {bbL, bbR}, baY[2] = {baB, baT};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      T u1 = T(0.5) * (ua_ab[q] + ua_ba[perm[q]]);
      T u2 = T(0.5) * (ub_ab[q] + ub_ba[perm[q]]);
      e[q] = -u1 * bbX[q & 1] + u2 * baY[q >> 1];
    }
  }
  T eps = ld04(e[0], e[1], e[2], e[3], apa, ama, apb, amb, baB, baT, bbL, bbR);
  if (eta_d > 0.0) eps += eta_j<T>(S, G, s, c, (T)eta_d);
  return eps;
}

// All three edge directions at the edge positions [g, g+n] on every axis
// (an edge of direction c exists for s_c < g + n_c).
template <typename T, int RECON, int EMF>
__device__ __forceinline__ void emf_at(const State& S, const Geom& G, const Work<T>& W, int stage,
                                       double eta_d, int t) {
  const int L0 = G.n[0] + 1, L1 = G.n[1] + 1, L2 = G.n[2] + 1;
  if (t >= L0 * L1 * L2) return;
  int s3[3] = {G.g + t % L0, G.g + (t / L0) % L1, G.g + t / (L0 * L1)};
  int s = s3[0] + G.st[1] * s3[1] + G.st[2] * s3[2];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if (s3[c] < G.g + G.n[c]) W.E[stage][c][s] = edge_emf<T, RECON, EMF>(S, G, W, s, c, eta_d);
}

template <typename T, int RECON, int EMF>
__global__ void __launch_bounds__(kBlock)
    k_emf3(State S, Geom G, Work<T> W, int stage, double eta_d, int band, const int* stop) {
  if (*stop) return;
  emf_at<T, RECON, EMF>(S, G, W, stage, eta_d, xcd_band_tile(band) * kBlock + (int)threadIdx.x);
}

// Q26 EMFs of one column of edge positions (x and y fixed, z in [z0, z1)),
// marching up z.  The four reconstructions along z -- B_y and u*_y at the x
// edges, B_x and u*_x at the y edges -- run as streams that take one cell
// and complete one per position, as in the face marches, instead of loading
// and limiting six cells per edge; the other reconstructions, the wave speeds
// and eta j are those of edge_emf.  The streamed values are the same
// arithmetic on the same cells, so the EMFs equal emf_at's.
template <typename T, int RECON>
__device__ __forceinline__ void emf_march_q26(const State& S, const Geom& G, const Work<T>& W,
                                              int stage, double eta_d, int col, int z0, int z1) {
  constexpr int r = recon_halfwidth(RECON);
  const int L0 = G.n[0] + 1;
  const int x = G.g + col % L0, y = G.g + col / L0;
  const int sy = G.st[1], sz = G.st[2];
  const bool xe = x < G.g + G.n[0], ye = y < G.g + G.n[1];  // x / y edges exist here
  const int base = x + sy * y;
  ReconStream<RECON, T> rs[4];  // B_y, u*_y (x edges), B_x, u*_x (y edges)
  T lo[4];                      // upper values of the cell below the next position
  // cells z0-1-r .. z1-1+r; the pushes before cell z0-1+r only fill the
  // pipelines (their streams' cells lie in the ghost layers)
  for (int q = z0 - 1 - r; q <= z1 - 1 + r; ++q) {
    const int sq = base + q * sz;
    const T v[4] = {(T)S.b[1][sq], W.us[1][sq], (T)S.b[0][sq], W.us[0][sq]};
    T qm[4], qp[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) rs[k].push(v[k], qm[k], qp[k]);
    const int z = q - r;  // the cell completed by this push
    if (z >= z0) {
      const int s = base + z * sz;
      if (xe) {  // a = y (streamed along z), b = z (along y)
        T bbL, bbR, ubL, ubR;
        iface_along_d<RECON>(S.b[2], s, sy, bbL, bbR);
        iface_along<RECON>(W.us[2], s, sy, ubL, ubR);
        W.E[stage][0][s] =
            q26_edge<T>(S, G, W, s, 0, lo[0], qm[0], bbL, bbR, lo[1], qm[1], ubL, ubR, eta_d);
      }
      if (ye) {  // a = z (along x), b = x (streamed along z)
        T baB, baT, uaB, uaT;
        iface_along_d<RECON>(S.b[2], s, 1, baB, baT);
        iface_along<RECON>(W.us[2], s, 1, uaB, uaT);
        W.E[stage][1][s] =
            q26_edge<T>(S, G, W, s, 1, baB, baT, lo[2], qm[2], uaB, uaT, lo[3], qm[3], eta_d);
      }
      if (z < G.g + G.n[2]) W.E[stage][2][s] = edge_emf<T, RECON, kQ26>(S, G, W, s, 2, eta_d);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) lo[k] = qp[k];
  }
}

// Q26 edge pass as z marches: workgroup tile = chunk * ctiles + column tile
// (columns x fastest, kBlock per tile), z chunks of zc positions.  Through
// xcd_tile each XCD takes a contiguous run of tiles: a slab of z chunks over
// a band of rows, so the y neighbours a column reads share its XCD's L2.
template <typename T, int RECON>
__global__ void __launch_bounds__(kBlock)
    k_emf_march(State S, Geom G, Work<T> W, int stage, double eta_d, int ctiles, int zc,
                const int* stop) {
  if (*stop) return;
  const int tile = xcd_tile();
  const int col = (tile % ctiles) * kBlock + (int)threadIdx.x;
  if (col >= (G.n[0] + 1) * (G.n[1] + 1)) return;
  const int z0 = G.g + (tile / ctiles) * zc;
  const int zend = G.g + G.n[2] + 1;
  emf_march_q26<T, RECON>(S, G, W, stage, eta_d, col, z0, z0 + zc < zend ? z0 + zc : zend);
}

// ---------------------------------------------------------------------------
// Update (eqs. rk:increment-state, rk:increment-bfield, rk1:update,
// rk2:update).  stage 0: out = S^n + D^n.  stage 1: out = S^n + (D^n +
// D^{n+1/2})/2.  Increments are formed in FP64 from the stored fluxes and
// EMFs (which are single-valued per face and edge: conservation and div b
// hold to FP64 round-off in both precision forms), without contraction into
// fused multiply-adds.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ double dcons(const Geom& G, const Work<T>& W, int st, int s, int m,
                                        double dt) {
#pragma clang fp contract(off)
  double f = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T* Fa = W.F[st][a][m];
    f += ((double)Fa[s] - (double)Fa[s + gstride(G, a)]) * G.idx[a];
  }
  return dt * f;
}

// increment of the face field b_a stored at s
template <typename T>
__device__ __forceinline__ double dface(const Geom& G, const Work<T>& W, int st, int s, int a,
                                        double dt) {
#pragma clang fp contract(off)
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  const T* Ec = W.E[st][c];
  const T* Eb = W.E[st][b];
  double circ = ((double)Ec[s] - (double)Ec[s + gstride(G, b)]) * G.idx[b] +
                ((double)Eb[s + gstride(G, c)] - (double)Eb[s]) * G.idx[c];
  return dt * circ;
}

// New face field.  stage 0: b^n + D^n.  stage 1, main pass: the SSP form
// (b^n + b^{n+1/2} + D^{n+1/2}) / 2, which equals b^n + (D^n + D^{n+1/2}) / 2
// up to round-off and does not re-read the first-stage EMFs; stage 1 after a
// first-order replacement: b^n + (D^n + D^{n+1/2}) / 2 with the replaced
// values of both stages.
template <typename T>
__device__ __forceinline__ double new_face(const State& base, const State& half, const Geom& G,
                                           const Work<T>& W, int stage, int fixup, int s, int a,
                                           double dt) {
#pragma clang fp contract(off)
  if (stage == 0) return base.b[a][s] + dface(G, W, 0, s, a, dt);
  if (!fixup) return 0.5 * (base.b[a][s] + half.b[a][s] + dface(G, W, 1, s, a, dt));
  return base.b[a][s] + 0.5 * (dface(G, W, 0, s, a, dt) + dface(G, W, 1, s, a, dt));
}

struct UpdateCfg {
  int fofc;          // flag the new state
  int crit;          // CTMHD_FLAG_*
  double gamma;
  double sres;       // resistive signal speed term of the CFL maximum
  const uint8_t* force;  // forced flags of this stage or null
  int flag_storage;  // 1: flags indexed by storage position (a level of boxes)
};

// fixup = 0: main update (flags, and for stage 1 the CFL maximum into slot 0)
// fixup = 1: after first-order replacement; runs only if this stage flagged
//            cells; stage 1 recomputes the CFL maximum into slot 1.
// stage and fixup as constants: each form of the update is straight-line
// code, so that every load of a cell can be issued before the first wait.
template <typename T, int stage, int fixup>
__device__ __forceinline__ void update_item_s(const State& base, const State& half,
                                              const State& out, const Geom& G, const Work<T>& W,
                                              const UpdateCfg& U, long long* diag, int vb,
                                              int strips, unsigned long long* slots, int slot) {
  // no fused multiply-adds: the update is memory-bound, and without them its
  // results cannot depend on how a calling kernel is specialised (the main
  // and fix-up calls, the single-box and batched kernels give the same bits)
#pragma clang fp contract(off)
  const int ninter = G.n[0] * G.n[1] * G.n[2];
  const double dt = *W.dt;
  double sigmax = 0.0;
  for (int strip = 0; strip < strips; ++strip) {
  const int t = (vb * strips + strip) * kBlock + (int)threadIdx.x;
  const bool live = t < ninter;
  int bad = 0;
  double sig = 0.0;
  if (live) {
    const int i0 = t % G.n[0];
    const int q = t / G.n[0];
    const int j0 = q % G.n[1];
    const int k0 = q / G.n[1];
    const int p3[3] = {i0, j0, k0};
    const int s = (i0 + G.g) + G.st[1] * (j0 + G.g) + G.st[2] * (k0 + G.g);
    double c[5], bl[3];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      if (stage == 0)
        c[m] = base.c[m][s] + dcons(G, W, 0, s, m, dt);
      else if (!fixup)
        c[m] = 0.5 * (base.c[m][s] + half.c[m][s] + dcons(G, W, 1, s, m, dt));
      else
        c[m] = base.c[m][s] + 0.5 * (dcons(G, W, 0, s, m, dt) + dcons(G, W, 1, s, m, dt));
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) bl[a] = new_face(base, half, G, W, stage, fixup, s, a, dt);
    // upper faces of this cell, recomputed with the same arithmetic as the
    // neighbour that owns them (for the flags and the CFL signal); formed
    // before the stores below, which the compiler cannot move loads across
    const bool need_state = (U.fofc && !fixup) || stage == 1;
    double bu[3] = {0.0, 0.0, 0.0};
    if (need_state) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
        bu[a] = new_face(base, half, G, W, stage, fixup, s + gstride(G, a), a, dt);
    }
    // periodic images: every storage position congruent to this cell
    int mlo[3], mhi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int pos = p3[d] + G.g;
      mlo[d] = -(pos / G.n[d]);
      mhi[d] = (G.N[d] - 1 - pos) / G.n[d];
    }
    for (int mz = mlo[2]; mz <= mhi[2]; ++mz)
      for (int my = mlo[1]; my <= mhi[1]; ++my)
        for (int mx = mlo[0]; mx <= mhi[0]; ++mx) {
          const int sw = s + mx * G.n[0] + my * G.n[1] * G.st[1] + mz * G.n[2] * G.st[2];
#pragma unroll
          for (int m = 0; m < 5; ++m) out.c[m][sw] = c[m];
#pragma unroll
          for (int a = 0; a < 3; ++a) out.b[a][sw] = bl[a];
        }
    if (need_state) {
      const double rho = c[0];
      double u[3], bc[3];
      bool nonfin = false;
#pragma unroll
      for (int m = 0; m < 5; ++m) nonfin |= !__builtin_isfinite(c[m]);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        nonfin |= !__builtin_isfinite(bl[d]) || !__builtin_isfinite(bu[d]);
        bc[d] = 0.5 * (bl[d] + bu[d]);
        u[d] = c[1 + d] / rho;
      }
      const double p = (U.gamma - 1.0) * (c[4] - 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) -
                                          0.5 * (bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]));
      if (U.fofc && !fixup) {
        if ((U.crit & CTMHD_FLAG_RHO) && !(rho > 0.0)) bad = 1;
        if ((U.crit & CTMHD_FLAG_P) && !(p > 0.0)) bad = 1;
        if ((U.crit & CTMHD_FLAG_NONFINITE) && (nonfin || !__builtin_isfinite(p))) bad = 1;
        if (U.force && U.force[t]) bad = 1;
        W.flag[U.flag_storage ? s : t] = (uint8_t)bad;
      }
      if (stage == 1) sig = cfl_signal(rho, u, p, bc, G, U.gamma, U.sres);
    }
  }
  if (U.fofc && !fixup) {
    unsigned long long m = __ballot(bad);
    if ((threadIdx.x & 63) == 0 && m) {
      int cnt = __popcll(m);
      atomicAdd(&W.nflag[stage], cnt);
      if (diag) atomicAdd((unsigned long long*)&diag[stage], (unsigned long long)cnt);
    }
  }
  sigmax = (sig > sigmax || sig != sig) ? sig : sigmax;
  }
  if (stage == 1) {
    if (fixup && threadIdx.x == 0) W.nflag[2] = 1;
    block_max_to_slots(sigmax, slots, slot);
  }
}

template <typename T>
__device__ __forceinline__ void update_item(const State& base, const State& half, const State& out,
                                            const Geom& G, const Work<T>& W, int stage, int fixup,
                                            const UpdateCfg& U, long long* diag, int vb, int strips,
                                            unsigned long long* slots, int slot) {
  if (stage == 0) {
    if (fixup)
      update_item_s<T, 0, 1>(base, half, out, G, W, U, diag, vb, strips, slots, slot);
    else
      update_item_s<T, 0, 0>(base, half, out, G, W, U, diag, vb, strips, slots, slot);
  } else {
    if (fixup)
      update_item_s<T, 1, 1>(base, half, out, G, W, U, diag, vb, strips, slots, slot);
    else
      update_item_s<T, 1, 0>(base, half, out, G, W, U, diag, vb, strips, slots, slot);
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_update(State base, State half, State out, Geom G, Work<T> W, int stage, int fixup,
             UpdateCfg U, long long* diag, int band, const int* stop) {
  if (*stop) return;
  if (!fixup) {
    update_item<T>(base, half, out, G, W, stage, 0, U, diag, xcd_band_tile(band), 1, W.smax,
                   blockIdx.x % kMaxSlots);
    return;
  }
  // fix-up: a capped grid strides over the tiles (usually nothing is flagged
  // and every workgroup returns at once)
  if (W.nflag[stage] == 0) return;
  const int ntiles = (G.n[0] * G.n[1] * G.n[2] + kBlock - 1) / kBlock;
  for (int vb = blockIdx.x; vb < ntiles; vb += (int)gridDim.x)
    update_item<T>(base, half, out, G, W, stage, 1, U, diag, vb, 1, W.smax + kMaxSlots,
                   blockIdx.x % kMaxSlots);
}

// ---------------------------------------------------------------------------
// First-order flux correction (Sec. 2.5): faces touching a flagged cell take
// the PC + LLF flux of S^n, edges touching one the first-order EMF of S^n.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int interior_id(const Geom& G, int s0, int s1, int s2) {
  int i = (s0 - G.g) % G.n[0];
  if (i < 0) i += G.n[0];
  int j = (s1 - G.g) % G.n[1];
  if (j < 0) j += G.n[1];
  int k = (s2 - G.g) % G.n[2];
  if (k < 0) k += G.n[2];
  return i + G.n[0] * (j + G.n[1] * k);
}

// First-order (PC + LLF) flux at the x_a face s; returns s_LLF and u*.
template <typename T>
__device__ __forceinline__ T fo_face(const State& S, const Geom& G, int s, int a, double gamma_d,
                                     T F[5], T& ustar) {
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  T vl[7], vr[7];
  face_local<T>(S, G, s - G.st[a], a, gamma_d, vl);
  face_local<T>(S, G, s, a, gamma_d, vr);
  FState<T> L{vl[0], vl[1], vl[2], vl[3], vl[4], vl[5], vl[6]};
  FState<T> R{vr[0], vr[1], vr[2], vr[3], vr[4], vr[5], vr[6]};
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

template <typename T, int EMF>
__device__ __forceinline__ T fo_corner_cell(const State& Sn, const Geom& G, int s, int a, int b,
                                            double gamma, T baY, T bbX) {
  // ideal EMF of a cell (PC): -u_a b_b + u_b b_a, from cell-centred values
  double rho, u[3], p, bc[3];
  cell_prim(Sn, G, s, gamma, rho, u, p, bc);
  if (EMF == kB25A) return -(T)u[a] * (T)bc[b] + (T)u[b] * (T)bc[a];
  return -(T)u[a] * bbX + (T)u[b] * baY;  // FS18 with PC: cell velocity, edge field
}

// Flag of the cell at storage coordinates p3: periodic box (interior flags,
// wrapped) or a level of boxes (flags at every storage position, the ghost
// layers filled from the neighbouring boxes).
template <typename T>
__device__ __forceinline__ uint8_t flag_of(const Geom& G, const Work<T>& W, bool lvl,
                                           const int p3[3]) {
  if (lvl) return W.flag[p3[0] + G.st[1] * p3[1] + G.st[2] * p3[2]];
  return W.flag[interior_id(G, p3[0], p3[1], p3[2])];
}

// One thread per cell position s: its three lower faces and the three edges
// at its lower corner.  Stage 1 writes both stored flux sets so that their RK
// average is the first-order value.
//   periodic box (lvl false): interior positions; the periodic images of the
//     upper boundary faces / edges are written as well (the update reads them);
//   a level of boxes (lvl true): positions 0..n along each axis, so that the
//     upper boundary faces / edges are computed from this box's ghost cells
//     and flags (bitwise the values the neighbour that owns them computes).
template <typename T, int EMF>
__device__ __forceinline__ void fo_at(const State& Sn, const Geom& G, const Work<T>& W, int stage,
                                      double gamma, double eta_d, int t, bool lvl) {
  const int e = lvl ? 1 : 0;
  const int m0 = G.n[0] + e, m1 = G.n[1] + e;
  if (t >= m0 * m1 * (G.n[2] + e)) return;
  const int s3[3] = {t % m0 + G.g, (t / m0) % m1 + G.g, t / (m0 * m1) + G.g};
  const int s = s3[0] + G.st[1] * s3[1] + G.st[2] * s3[2];
  bool up[3];  // on the upper boundary layer along each axis (level only)
#pragma unroll
  for (int d = 0; d < 3; ++d) up[d] = s3[d] == G.g + G.n[d];
  const bool f0 = flag_of(G, W, lvl, s3) != 0;
  for (int a = 0; a < 3; ++a) {
    if (up[(a + 1) % 3] || up[(a + 2) % 3]) continue;  // not a face of this box
    int l3[3] = {s3[0], s3[1], s3[2]};
    l3[a] -= 1;
    if (!f0 && !flag_of(G, W, lvl, l3)) continue;
    T F[5], us;
    fo_face<T>(Sn, G, s, a, gamma, F, us);
    if (eta_d > 0.0) F[4] += joule<T>(Sn, G, s, a, (T)eta_d);
    for (int rep = 0; rep < 2; ++rep) {
      if (rep && (lvl || s3[a] != G.g)) break;
      const int sw = s + (rep ? G.n[a] * G.st[a] : 0);
      for (int m = 0; m < 5; ++m) {
        W.F[stage][a][m][sw] = F[m];
        if (stage == 1) W.F[0][a][m][sw] = F[m];
      }
    }
  }
  for (int c = 0; c < 3; ++c) {
    const int a = (c + 1) % 3, b = (c + 2) % 3;
    if (up[c]) continue;  // not an edge of this box
    int fl = 0;
    for (int q = 0; q < 4; ++q) {
      int p3[3] = {s3[0], s3[1], s3[2]};
      p3[a] -= (q & 1);
      p3[b] -= (q >> 1);
      fl |= flag_of(G, W, lvl, p3);
    }
    if (!fl) continue;
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
    for (int qa = 0; qa < 2; ++qa)
      for (int qb = 0; qb < 2; ++qb) {
        if ((qa || qb) && lvl) continue;
        if ((qa && s3[a] != G.g) || (qb && s3[b] != G.g)) continue;
        const int sw = s + (qa ? G.n[a] * sa : 0) + (qb ? G.n[b] * sb : 0);
        W.E[stage][c][sw] = eps;
        if (stage == 1) W.E[0][c][sw] = eps;
      }
  }
}

template <typename T, int EMF>
__global__ void __launch_bounds__(kBlock)
    k_fo(State Sn, Geom G, Work<T> W, int stage, double gamma, double eta_d, const int* stop) {
  if (*stop) return;
  if (W.nflag[stage] == 0) return;
  // grid-stride: the launch is capped, so that the usual case (nothing
  // flagged) costs a few workgroups, not one per 256 cells
  const int ninter = G.n[0] * G.n[1] * G.n[2];
  for (int t = gidx(); t < ninter; t += (int)gridDim.x * kBlock)
    fo_at<T, EMF>(Sn, G, W, stage, gamma, eta_d, t, false);
}

// ---------------------------------------------------------------------------
// Batched boxes: one persistent launch per step drains a work queue of
// (phase, box, tile) items.  Items are ordered phase-major (largest boxes
// first inside a phase), so an item only ever waits for items that precede
// it in the queue (the previous phase of its own box): with workgroups that
// claim an item only after finishing the last one, the queue always drains.
// Each box is a periodic box of its own (ghosts wrapped per box), or the boxes
// tile one periodic domain (a level of an AMR hierarchy): then the ghost
// layers of every box are filled from the interiors of the boxes that own
// those cells (exchange phases after every update).
// ---------------------------------------------------------------------------
enum : int { PH_F = 0, PH_E, PH_U, PH_O, PH_X, PH_WRAP, PH_DT, PH_COPY, PH_P, PH_XCHG, PH_FIRST };
constexpr int kMaxPhases = 24;

// Exchange phase argument (PlanHeader::xarg): which state to fill, whether
// the invalid-cell flags travel too, and whether it runs only after a fix-up.
enum : int { XG_HALF = 0, XG_NEXT = 1, XG_CUR = 2, XG_TARGET = 3, XG_FLAGS = 4, XG_IF_FIXUP = 8 };

// One block of a box's ghost region whose cells are owned by one box (possibly
// itself, through the periodic wrap): dst and src are packed element indices
// of the block's first element, in the destination box's ghost region and the
// owner's interior.
struct XBlock {
  long long dst, src;
  int dsy, dsz, ssy, ssz;  // strides along axes 1 and 2 of both boxes
  int ex, ey;              // extents along axes 0 and 1 (axis 2: from the volume)
  int vol_lo;              // first ghost index of the block in its box's list
  int vol;                 // elements of the block
};

struct BoxDesc {
  Geom G;
  FacePlan FP;
  long long off;       // element offset of the box in the packed field arrays
  long long flag_off;  // offset of the box in the packed flag array
  double sres;         // resistive term of the CFL maximum (depends on dx)
};

struct PlanHeader {
  int nbox, nphase, strips, magic;
  unsigned long long key;    // hash of the parameters and boxes the plan was built for
  int kind[kMaxPhases];      // PH_*
  int stage[kMaxPhases];     // RK stage of F/E/U/O/X phases
  int item_off[kMaxPhases];  // first queue index of each phase inside its launch
  int range[3][2];           // phase ranges [lo, hi) of the start, step and copy launches
  int range_items[3];        // items of each launch
  long long order_off, prefix_off, desc_off;  // byte offsets of the arrays below
  int xarg[kMaxPhases];      // XG_* of exchange phases
  int level;                 // 1: the boxes tile one periodic domain
  int nxblk;                 // exchange blocks
  long long xbox_off, xblk_off;
  // int order[nbox]; int prefix[nphase][nbox + 1]; BoxDesc desc[nbox];
  // level only: int xbox[nbox + 1] (first block of each box); XBlock xblk[nxblk]
};
constexpr int kPlanMagic = 0x43544d48;

template <typename T>
struct BatchArgs {
  State user, B, H;   // packed states (box offsets from the plan)
  Work<T> W;          // packed stencil arrays; per-box scalars below
  const char* plan;
  int* cursor;        // queue cursor of this launch
  int* done;          // [nphase][nbox] finished items
  int* nflag;         // [nbox][4]: flagged cells stage 0 / 1, stage-1 fix-up ran
  unsigned long long* slots;  // [nbox][2]: CFL maximum (main pass, fix-up)
  double* dt;         // [nbox] (per-box dt) or [1]
  int* stop;
  int* err;           // set when a dependency wait times out
  long long* diag;    // this step's counters or null
  int dt_per_box;
  const int* loc;     // where the current state lives: 0 `user`, 1 B (flipped by each step that ran)
  int launch;         // 0 start (wrap + CFL), 1 step, 2 copy-back
  unsigned long long key;  // must equal the plan's key
  unsigned long long tab;  // device address of BoxTab<T>[nbox]
  double gamma, eta;
  int fofc, crit;
  int level;          // the boxes tile one periodic domain
};

// Everything one box needs, with its pointers already shifted to the box:
// built once per batched call by k_btab in the workspace and read through the
// constant address space (uniform scalar loads that may be indexed at run
// time, as kernel arguments are in the single-box kernels).
template <typename T>
struct BoxTab {
  State su, sb, sh;  // the box in the caller's arrays, in B, in H
  Work<T> w;         // its stencil arrays and per-box scalars
  Geom G;
  FacePlan FP;
  double sres;
};
#define CTMHD_CONST __attribute__((address_space(4)))

__device__ __forceinline__ State shift_state(const State& S, long long off) {
  State R;
#pragma unroll
  for (int m = 0; m < 5; ++m) R.c[m] = S.c[m] + off;
#pragma unroll
  for (int a = 0; a < 3; ++a) R.b[a] = S.b[a] + off;
  return R;
}

template <typename T>
__device__ __forceinline__ Work<T> shift_work(const Work<T>& W0, long long off) {
  Work<T> W = W0;
#pragma unroll
  for (int v = 0; v < 8; ++v) W.prim[v] = W0.prim[v] ? W0.prim[v] + off : nullptr;
#pragma unroll
  for (int c = 0; c < 3; ++c) W.ecell[c] = W0.ecell[c] ? W0.ecell[c] + off : nullptr;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int o = 0; o < 2; ++o)
#pragma unroll
      for (int k = 0; k < 2; ++k)
        W.b25f[c][o][k] = W0.b25f[c][o][k] ? W0.b25f[c][o][k] + off : nullptr;
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int k = 0; k < 2; ++k)
        W.fsf[v][d][k] = W0.fsf[v][d][k] ? W0.fsf[v][d][k] + off : nullptr;
#pragma unroll
  for (int st = 0; st < 2; ++st)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int m = 0; m < 5; ++m) W.F[st][a][m] = W0.F[st][a][m] + off;
      W.E[st][a] = W0.E[st][a] + off;
    }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    W.ap[a] = W0.ap[a] + off;
    W.am[a] = W0.am[a] + off;
    W.us[a] = W0.us[a] + off;
  }
  return W;
}

// Wait until *cnt >= need.  Thread 0 polls with relaxed loads (an acquire
// per poll would invalidate the XCD's L2 on every iteration and starve the
// working workgroups), then acquires once.  Bounded by wall-clock time
// (100 MHz counter, about 1 s): on a timeout the error flag is raised and
// every later wait returns at once.
__device__ __forceinline__ void wait_count(const int* cnt, int need, int* err) {
  if (threadIdx.x == 0) {
    const unsigned long long t0 = wall_clock64();
    while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
      __builtin_amdgcn_s_sleep(8);
      if (wall_clock64() - t0 > 100000000ull) {
        __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    // the producer may sit on another XCD (another L2): one acquire for the
    // workgroup's CU and XCD caches
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// Every wave releases its own stores at agent scope before thread 0 counts
// the item as done.
__device__ __forceinline__ void signal_count(int* cnt) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Ghost exchange of a level: element r of box b's ghost region takes the
// value of the cell (faces: the lower face of the cell) that owns it, for all
// 8 fields of S and, with `flags`, the invalid-cell flag.  Reads touch only
// interiors and writes only ghost positions, so one launch serves all boxes.
template <typename T>
__device__ __forceinline__ void xchg_at(const BatchArgs<T>& A, const State& S, bool flags, int b,
                                        int r) {
  const PlanHeader* P = (const PlanHeader*)A.plan;
  const int* xbox = (const int*)(A.plan + P->xbox_off);
  const XBlock* xb = (const XBlock*)(A.plan + P->xblk_off);
  int k0 = xbox[b], k1 = xbox[b + 1];
  if (k0 >= k1) return;
  const XBlock& lastb = xb[k1 - 1];
  if (r >= lastb.vol_lo + lastb.vol) return;
  while (k1 - k0 > 1) {  // the block holding r: largest k with vol_lo <= r
    const int mid = (k0 + k1) >> 1;
    if (xb[mid].vol_lo <= r) k0 = mid; else k1 = mid;
  }
  const XBlock& B = xb[k0];
  const int l = r - B.vol_lo;
  const int x = l % B.ex, y = (l / B.ex) % B.ey, z = l / (B.ex * B.ey);
  const long long d = B.dst + x + (long long)B.dsy * y + (long long)B.dsz * z;
  const long long s = B.src + x + (long long)B.ssy * y + (long long)B.ssz * z;
#pragma unroll
  for (int m = 0; m < 5; ++m) S.c[m][d] = S.c[m][s];
#pragma unroll
  for (int a = 0; a < 3; ++a) S.b[a][d] = S.b[a][s];
  if (flags) A.W.flag[d] = A.W.flag[s];
}

// One work item of a batched step: phase kind `kind` (run-time; KIND is its
// compile-time class: PH_U covers PH_U and PH_X, so that the main and the
// fix-up update share one call site as in k_update) of box b, tile `tile`.
template <typename T, int RECON, int RIEMANN, int EMF, int KIND>
__device__ __forceinline__ void batch_item(const BatchArgs<T>& A, int b, int kind, int stage,
                                           int tile, int strips, int cl, int xa) {
  const BoxTab<T>& tb = *(const BoxTab<T>*)((const CTMHD_CONST BoxTab<T>*)A.tab + b);
  const Geom& G = tb.G;
  const State& cur = cl == 0 ? tb.su : tb.sb;
  if constexpr (KIND == PH_COPY) {  // the state of this box back into the caller's arrays
    if (cl == 1)
      for (int s = 0; s < strips; ++s) {
        const int t = (tile * strips + s) * kBlock + threadIdx.x;
        if (t < G.elems) {
#pragma unroll
          for (int m = 0; m < 5; ++m) tb.su.c[m][t] = tb.sb.c[m][t];
#pragma unroll
          for (int a = 0; a < 3; ++a) tb.su.b[a][t] = tb.sb.b[a][t];
        }
      }
    return;
  } else {
    const Work<T>& W = tb.w;
    const State& Hs = tb.sh;
    const State& in = stage == 0 ? cur : Hs;
    if constexpr (KIND == PH_P) {
      for (int s = 0; s < strips; ++s)
        prim_at<T, EMF>(in, G, W, A.gamma, (tile * strips + s) * kBlock + threadIdx.x);
    } else if constexpr (KIND == PH_FIRST) {
      for (int s = 0; s < strips; ++s)
        first_step_at<T, RECON, EMF>(G, W, (tile * strips + s) * kBlock + threadIdx.x);
    } else if constexpr (KIND == PH_F) {
      int nfb = 0;
      faces_block<T, RECON, RIEMANN>(in, G, W, tb.FP, tile, stage, A.gamma, A.eta, nfb);
      if (A.diag && nfb) atomicAdd((unsigned long long*)&A.diag[2], (unsigned long long)nfb);
    } else if constexpr (KIND == PH_E) {
      for (int s = 0; s < strips; ++s)
        emf_at<T, RECON, EMF>(in, G, W, stage, A.eta, (tile * strips + s) * kBlock + threadIdx.x);
    } else if constexpr (KIND == PH_U) {
      const State& oth = cl == 0 ? tb.sb : tb.su;
      UpdateCfg U;
      U.fofc = A.fofc;
      U.crit = A.crit;
      U.gamma = A.gamma;
      U.sres = tb.sres;
      U.force = nullptr;
      U.flag_storage = A.level;
      const int fix = kind == PH_X ? 1 : 0;
      if (!fix || W.nflag[stage])
        update_item<T>(cur, Hs, stage == 0 ? Hs : oth, G, W, stage, fix, U, A.diag, tile, strips,
                       W.smax, fix);
    } else if constexpr (KIND == PH_O) {
      if (W.nflag[stage])
        for (int s = 0; s < strips; ++s)
          fo_at<T, EMF>(cur, G, W, stage, A.gamma, A.eta, (tile * strips + s) * kBlock + threadIdx.x,
                        A.level != 0);
    } else if constexpr (KIND == PH_WRAP) {
      for (int s = 0; s < strips; ++s) wrap_at(cur, G, (tile * strips + s) * kBlock + threadIdx.x);
    } else if constexpr (KIND == PH_XCHG) {
      if ((xa & XG_IF_FIXUP) && !W.nflag[stage]) return;
      const int tg = xa & XG_TARGET;
      // packed (unshifted) arrays: the owner of a ghost block is another box
      const State& dst = tg == XG_HALF ? A.H : tg == XG_CUR ? (cl == 0 ? A.user : A.B)
                                                              : (cl == 0 ? A.B : A.user);
      for (int s = 0; s < strips; ++s)
        xchg_at(A, dst, (xa & XG_FLAGS) != 0, b, (tile * strips + s) * kBlock + threadIdx.x);
    } else if constexpr (KIND == PH_DT) {
      double sig = 0.0;
      for (int s = 0; s < strips; ++s) {
        double v = dt_sig_at(cur, G, A.gamma, tb.sres, (tile * strips + s) * kBlock + threadIdx.x);
        sig = (v > sig || v != v) ? v : sig;
      }
      block_max_to_slots(sig, W.smax, 0);
    }
  }
}

// Per-box tables of a batched call (one thread per box).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_btab(BatchArgs<T> A, int nbox) {
  const PlanHeader* P = (const PlanHeader*)A.plan;
  if (P->magic != kPlanMagic || P->key != A.key) return;  // refused by the step kernels
  const int b = blockIdx.x * kBlock + threadIdx.x;
  if (b >= nbox) return;
  const BoxDesc& d = ((const BoxDesc*)(A.plan + P->desc_off))[b];
  BoxTab<T>* tb = (BoxTab<T>*)A.tab + b;
  tb->su = shift_state(A.user, d.off);
  tb->sb = shift_state(A.B, d.off);
  tb->sh = shift_state(A.H, d.off);
  Work<T> W = shift_work(A.W, d.off);
  W.flag = A.W.flag + d.flag_off;
  W.dt = A.dt + (A.dt_per_box ? b : 0);
  W.nflag = A.nflag + (A.level ? 0 : 4 * b);  // a level flags and fixes up as one domain
  W.smax = A.slots + 2 * b;
  W.stop = A.stop;
  tb->w = W;
  tb->G = d.G;
  tb->FP = d.FP;
  tb->sres = d.sres;
}

// Plan lookup shared by both schedules: true if the plan was built for the
// call's parameters and boxes.
__device__ __forceinline__ bool plan_ok(const char* plan, unsigned long long key, int* err) {
  const PlanHeader* P = (const PlanHeader*)plan;
  if (P->magic == kPlanMagic && P->key == key) return true;
  if (threadIdx.x == 0) atomicOr(err, 2);
  return false;
}

// Box (index into `order`, largest k with pre[k] <= r) of item r of a phase.
__device__ __forceinline__ int item_box(const int* pre, int nbox, int r) {
  int k0 = 0, k1 = nbox;
  while (k1 - k0 > 1) {
    int mid = (k0 + k1) >> 1;
    if (pre[mid] <= r) k0 = mid; else k1 = mid;
  }
  return k0;
}

// Persistent schedule: one launch per step (plus a start and a copy-back
// launch).  Workgroups claim queue items in phase-major order; an item waits
// only for all items of the previous phase of its own box.
template <typename T, int RECON, int RIEMANN, int EMF>
__global__ void __launch_bounds__(kBlock) k_batch(BatchArgs<T> A) {
  if (*A.stop && A.launch != 2) return;  // the copy-back runs even after a stop
  if (!plan_ok(A.plan, A.key, A.err)) return;
  const PlanHeader* P = (const PlanHeader*)A.plan;
  const int* order = (const int*)(A.plan + P->order_off);
  const int* prefix = (const int*)(A.plan + P->prefix_off);
  const int nbox = P->nbox;
  const int lo = P->range[A.launch][0], hi = P->range[A.launch][1];
  const int total = P->range_items[A.launch];
  const int strips = P->strips;
  const int cl = *A.loc;  // fixed for the whole launch
  __shared__ int item_s;
  for (;;) {
    if (threadIdx.x == 0) item_s = atomicAdd(A.cursor, 1);
    __syncthreads();
    const int q = item_s;
    __syncthreads();
    if (q >= total) break;
    int p = lo;
    while (p + 1 < hi && P->item_off[p + 1] <= q) ++p;
    const int* pre = prefix + (long long)p * (nbox + 1);
    const int r = q - P->item_off[p];
    const int k0 = item_box(pre, nbox, r);
    const int b = order[k0];
    const int tile = r - pre[k0];
    if (p > lo) {
      const int* ppre = prefix + (long long)(p - 1) * (nbox + 1);
      wait_count(A.done + (long long)(p - 1) * nbox + b, ppre[k0 + 1] - ppre[k0], A.err);
    }
    const int kind = P->kind[p], stage = P->stage[p];
    switch (kind) {
      case PH_P: batch_item<T, RECON, RIEMANN, EMF, PH_P>(A, b, kind, stage, tile, strips, cl, P->xarg[p]); break;
      case PH_FIRST: batch_item<T, RECON, RIEMANN, EMF, PH_FIRST>(A, b, kind, stage, tile, strips, cl, P->xarg[p]); break;
      case PH_F: batch_item<T, RECON, RIEMANN, EMF, PH_F>(A, b, kind, stage, tile, strips, cl, P->xarg[p]); break;
      case PH_E: batch_item<T, RECON, RIEMANN, EMF, PH_E>(A, b, kind, stage, tile, strips, cl, P->xarg[p]); break;
      case PH_U:
      case PH_X: batch_item<T, RECON, RIEMANN, EMF, PH_U>(A, b, kind, stage, tile, strips, cl, P->xarg[p]); break;
      case PH_O: batch_item<T, RECON, RIEMANN, EMF, PH_O>(A, b, kind, stage, tile, strips, cl, P->xarg[p]); break;
      case PH_WRAP: batch_item<T, RECON, RIEMANN, EMF, PH_WRAP>(A, b, kind, stage, tile, strips, cl, P->xarg[p]); break;
      case PH_DT: batch_item<T, RECON, RIEMANN, EMF, PH_DT>(A, b, kind, stage, tile, strips, cl, P->xarg[p]); break;
      case PH_XCHG: batch_item<T, RECON, RIEMANN, EMF, PH_XCHG>(A, b, kind, stage, tile, strips, cl, P->xarg[p]); break;
      default: batch_item<T, RECON, RIEMANN, EMF, PH_COPY>(A, b, kind, stage, tile, strips, cl, P->xarg[p]); break;
    }
    signal_count(A.done + (long long)p * nbox + b);
  }
}

// Phased schedule: one launch per phase over all boxes; workgroup r runs
// item r of phase p.  Launch boundaries order the phases.
template <typename T, int RECON, int RIEMANN, int EMF, int KIND>
__global__ void __launch_bounds__(kBlock) k_bphase(BatchArgs<T> A, int p) {
  if (KIND != PH_COPY && *A.stop) return;  // the copy-back runs even after a stop
  if (!plan_ok(A.plan, A.key, A.err)) return;
  const PlanHeader* P = (const PlanHeader*)A.plan;
  const int nbox = P->nbox;
  const int* pre = (const int*)(A.plan + P->prefix_off) + (long long)p * (nbox + 1);
  const int r = blockIdx.x;
  if (r >= pre[nbox]) return;
  const int k0 = item_box(pre, nbox, r);
  const int b = ((const int*)(A.plan + P->order_off))[k0];
  batch_item<T, RECON, RIEMANN, EMF, KIND>(A, b, P->kind[p], P->stage[p], r - pre[k0], P->strips,
                                           *A.loc, P->xarg[p]);
}

// dt of a batched step from the per-box CFL maxima (the fix-up maximum where
// a box's second stage was fixed up); resets the per-step counters.
__global__ void __launch_bounds__(kBlock)
    k_bdt_final(int nbox, int nphase, int dt_per_box, int level, unsigned long long* slots, int* nflag,
                int* done, int* cursor, double cfl, const double* dt_fixed, double* dt,
                double* dt_out, int* stop, const int* err, long long* diag) {
  __shared__ unsigned long long red[kBlock];
  const int t = threadIdx.x;
  unsigned long long mx = 0;
  const bool stopped = *stop != 0;
  for (int b = t; b < nbox; b += kBlock) {
    unsigned long long v = nflag[4 * (level ? 0 : b) + 2] ? slots[2 * b + 1] : slots[2 * b];
    mx = v > mx ? v : mx;
    if (dt_per_box) {
      double x = stopped ? 0.0 : (dt_fixed ? dt_fixed[b] : cfl / __longlong_as_double((long long)v));
      if (!stopped && (!(x > 0.0) || !__builtin_isfinite(x))) atomicExch(stop, 1);
      dt[b] = x;
      if (dt_out) dt_out[b] = x;
    }
  }
  red[t] = mx;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (t < o) red[t] = red[t + o] > red[t] ? red[t + o] : red[t];
    __syncthreads();
  }
  if (t == 0 && !dt_per_box) {
    double x = stopped ? 0.0 : (dt_fixed ? dt_fixed[0] : cfl / __longlong_as_double((long long)red[0]));
    if (!stopped && (!(x > 0.0) || !__builtin_isfinite(x))) *stop = 1;
    dt[0] = x;
    if (dt_out) dt_out[0] = x;
  }
  for (int b = t; b < nbox; b += kBlock) {
    slots[2 * b] = slots[2 * b + 1] = 0ull;
    nflag[4 * b] = nflag[4 * b + 1] = nflag[4 * b + 2] = nflag[4 * b + 3] = 0;
  }
  for (int i = t; i < nphase * nbox; i += kBlock) done[i] = 0;
  if (t < 4) cursor[t] = 0;
  __syncthreads();
  if (t == 0 && diag) {
    diag[0] = diag[1] = diag[2] = 0;
    diag[3] = (*stop ? 1 : 0) | (*err << 1);
  }
}

// Reset before a launch of the queue (start / copy launches); init = 1 at the
// start of a call also clears the stop / error flags, the state location and
// the per-box CFL slots.
__global__ void k_breset(int nbox, int nphase, int* done, int* cursor, int init, int* stop,
                         int* err, int* loc, unsigned long long* slots, int* nflag) {
  for (int i = threadIdx.x; i < nphase * nbox; i += kBlock) done[i] = 0;
  if (threadIdx.x < 4) cursor[threadIdx.x] = 0;
  if (!init) return;
  for (int b = threadIdx.x; b < nbox; b += kBlock) {
    slots[2 * b] = slots[2 * b + 1] = 0ull;
    nflag[4 * b] = nflag[4 * b + 1] = nflag[4 * b + 2] = nflag[4 * b + 3] = 0;
  }
  if (threadIdx.x == 0) {
    *stop = 0;
    *err = 0;
    *loc = 0;
  }
}

// After a batched step: the new state is in the other buffer unless the step
// was stopped (non-finite dt), which leaves it where it was.
__global__ void k_bstep_end(int* loc, const int* stop, const int* err, long long* diag) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (diag) diag[3] |= *err << 1;
  if (!*stop) *loc ^= 1;
}

}  // namespace
