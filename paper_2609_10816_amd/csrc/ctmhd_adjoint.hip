// ctmhd_adjoint.hip -- reverse-mode derivative (vector-Jacobian product) of
// one CT-MHD step: the C ABI entry point ctmhd_step_adjoint.
//
// One RK2-SSP step with a frozen dt and no flux correction (eqs. rk1:update,
// rk2:update) is
//   S1 = S0 + D(S0),   S2 = (S0 + S1 + D(S1)) / 2,
// where D(S) is dt times the flux divergence of the cell fields and the CT
// curl of the edge EMFs for the face fields.  Given g2 = dL/dS2,
//   g1 = g2 / 2 + D'(S1)^T (g2 / 2),   g0 = g2 / 2 + g1 + D'(S0)^T g1.
//
// D'(S)^T v is formed in five passes over the ghosted box, each gathering
// (no two threads write one value, except the small Ohmic terms, which use
// atomics):
//   edges  the EMF adjoint from v (transposed curl), then LD04 and the Q26
//          corners in reverse: adjoints of the edge-reconstructed u*, face
//          fields and edge speeds, stored per edge (B25a: the adjoints of the
//          corner values of both two-step reconstructions of the cell EMF)
//   faces  the flux adjoint from v (transposed divergence); the adjoints of
//          u*, alpha+-, and of the face field gathered from the edges that
//          read them (through the reverse of their reconstructions); the
//          Riemann solver in reverse: adjoints of the two face-local states
//          and of the normal field; Joule flux and eta j in reverse
//   cells  face-local state adjoints gathered through the reverse of the
//          cell reconstructions (B25a: also the cell-EMF adjoint, gathered
//          through the reverse of both two-step reconstructions, onto u and
//          the cell field) into primitive adjoints
//   fields primitive -> conserved (Sec. 2.2, eq. state:primitive), and the
//          cell-centred field adjoints onto the two faces of each cell
//   fold   every ghost copy's adjoint added to its interior cell or face
// The forward face arrays (alpha+-, u*) of the state being differentiated come
// from the forward face kernel.
#include "ctmhd_adjoint_math.h"
#include "ctmhd_host.h"

namespace {

struct PrimPtrs {
  double* p[8];
};

struct AdjArrays {
  double* v[8];        // adjoint of D: 5 cell fields, 3 face fields (vval)
  double vs;           // scale of v
  double* ca[5];       // conserved-field adjoint per cell (k_adj_cons)
  double* prim[8];     // rho, u0, u1, u2, p, bc0, bc1, bc2 of the state
  double* ea[3][12];   // per edge direction: adjoints of uaB uaT ubL ubR baB baT bbL bbR
                       // apa ama apb amb
  double* fa[3][14];   // per face direction: adjoints of the left and right face states
  double* bn[3];       // face-field adjoint, gathered per face
  double* bj[3];       // face-field adjoint of the Ohmic terms (atomic accumulation)
  // B25a and FS18 only.  Per edge direction c, the cell fields reconstructed
  // to the corners in two steps: B25a the cell EMF e_c (field 0), FS18 the
  // cell velocities u_a (field 0) and u_b (field 1).  ec[c][8 f + 4 o + q]:
  // adjoint of corner q (LB, RB, LT, RT) of field f in order o ([x_a x_b],
  // then [x_b x_a]); fv / fb[c][f][o][side]: the first-step face values
  // (lower, upper side) and their adjoints; eb[k]: the adjoint of the cell
  // field (B25a: e_k; FS18: u_k)
  double* ec[3][16];
  double* fv[3][2][2][2];
  double* fb[3][2][2][2];
  double* eb[3];
};

// Cell fields of the two-step corner reconstructions of edge direction c.
__host__ __device__ constexpr int corner_fields(int emf) { return emf == kFS18 ? 2 : emf == kB25A ? 1 : 0; }
__host__ __device__ constexpr int corner_comp(int c, int f) { return f == 0 ? (c + 1) % 3 : (c + 2) % 3; }
template <int EMF>
__host__ __device__ const double* corner_src(const Work<double>& W, int c, int f) {
  return EMF == kB25A ? W.ecell[c] : W.prim[1 + corner_comp(c, f)];
}

__device__ __forceinline__ void decode(const Geom& G, int t, int s3[3]) {
  s3[0] = t % G.N[0];
  const int q = t / G.N[0];
  s3[1] = q % G.N[1];
  s3[2] = q / G.N[1];
}

// The adjoint of D at position pos: vs * v on interior positions, 0 on ghost
// positions (whatever the caller's buffer holds there; pos lies in the box).
__device__ __forceinline__ double vval(const AdjArrays& X, int f, int pos, bool inter) {
  // the product masked bitwise rather than selected, so that the load is not
  // moved into a branch of its own (where each load would wait alone)
  const long long keep = inter ? -1ll : 0ll;
  return __longlong_as_double(__double_as_longlong(X.vs * X.v[f][pos]) & keep);
}
// Whether the cell s3 (shifted by -1 along axis d if d >= 0) is an interior cell.
__device__ __forceinline__ bool interior_at(const Geom& G, const int s3[3], int d) {
  bool in = true;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int q = s3[e] - (e == d ? 1 : 0);
    in = in && q >= G.g && q < G.g + G.n[e];
  }
  return in;
}

// ---------------------------------------------------------------------------
// Cell primitives of the state (FP64, as cell_prim); 0 on the last layer of
// each axis, which has no upper face.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
    k_adj_prim(State S, Geom G, AdjArrays X, double gamma, const int* stop) {
  if (*stop) return;
  const int t = gidx();
  if (t >= G.elems) return;
  int s3[3];
  decode(G, t, s3);
  double rho = 0.0, u[3] = {0.0, 0.0, 0.0}, p = 0.0, bc[3] = {0.0, 0.0, 0.0};
  if (s3[0] < G.N[0] - 1 && s3[1] < G.N[1] - 1 && s3[2] < G.N[2] - 1)
    cell_prim(S, G, t, gamma, rho, u, p, bc);
  X.prim[0][t] = rho;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    X.prim[1 + d][t] = u[d];
    X.prim[5 + d][t] = bc[d];
  }
  X.prim[4][t] = p;
}

// Adjoint coef of j_c = (b_b[s] - b_b[s - st_a]) / dx_a - (b_a[s] - b_a[s - st_b]) / dx_b
// (eq. resistivity:current-stencil; a = c+1, b = c+2) onto the face fields.
__device__ __forceinline__ void etaj_adj(double* const bj[3], const Geom& G, int s, int c,
                                         double coef) {
  const int a = (c + 1) % 3, b = (c + 2) % 3;
  atomicAdd(&bj[b][s], coef * G.idx[a]);
  atomicAdd(&bj[b][s - gstride(G, a)], -coef * G.idx[a]);
  atomicAdd(&bj[a][s], -coef * G.idx[b]);
  atomicAdd(&bj[a][s - gstride(G, b)], coef * G.idx[b]);
}

// ---------------------------------------------------------------------------
// Edges: EMF adjoint and the reverse of LD04 + Q26, B25a or FS18 corners
// (edge_emf), one edge direction (blockIdx.y) per thread.
// ---------------------------------------------------------------------------
template <int RECON, int EMF>
__global__ void __launch_bounds__(kBlock)
    k_adj_edge(State S, Geom G, Work<double> W, AdjArrays X, double eta, const int* stop) {
  if (*stop) return;
  const int t = gidx();
  if (t >= G.elems) return;
  const double dt = *W.dt;
  int s3[3];
  decode(G, t, s3);
  bool inside = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) inside = inside && s3[d] >= G.g && s3[d] <= G.g + G.n[d];
  {
    const int c = (int)blockIdx.y;  // edge direction
    if (!inside || s3[c] >= G.g + G.n[c]) {
#pragma unroll
      for (int q = 0; q < 12; ++q) X.ea[c][q][t] = 0.0;
#pragma unroll
      for (int q = 0; q < 8 * corner_fields(EMF); ++q) X.ec[c][q][t] = 0.0;
      return;
    }
    const int a = (c + 1) % 3, b = (c + 2) % 3;
    const int sa = gstride(G, a), sb = gstride(G, b);
    // the EMF enters the new face fields b_a at t, t - sb and b_b at t, t - sa
    const bool i0 = interior_at(G, s3, -1), ia = interior_at(G, s3, a),
               ib = interior_at(G, s3, b);
    const double Eb = dt * ((vval(X, 5 + a, t, i0) - vval(X, 5 + a, t - sb, ib)) * G.idx[b] -
                            (vval(X, 5 + b, t, i0) - vval(X, 5 + b, t - sa, ia)) * G.idx[a]);
    double bv[4], al[4];
    iface_along_d<RECON>(S.b[a], t, sb, bv[0], bv[1]);  // baB, baT
    iface_along_d<RECON>(S.b[b], t, sa, bv[2], bv[3]);  // bbL, bbR
    al[0] = tmax(W.ap[a][t - sb], W.ap[a][t]);
    al[1] = tmax(W.am[a][t - sb], W.am[a][t]);
    al[2] = tmax(W.ap[b][t - sa], W.ap[b][t]);
    al[3] = tmax(W.am[b][t - sa], W.am[b][t]);
    double ub[4] = {0.0, 0.0, 0.0, 0.0}, bb[4] = {0.0, 0.0, 0.0, 0.0};
    double alb[4] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (EMF == kB25A) {
      // corners: the mean of the two two-step reconstructions of the cell EMF
      // (edge_emf); e[q] = (ab[q] + ba[perm q]) / 2
      double ab[4], ba[4];
      two_step<RECON>(W.ecell[c], t, sa, sb, ab);
      two_step<RECON>(W.ecell[c], t, sb, sa, ba);
      const double e[4] = {0.5 * (ab[0] + ba[0]), 0.5 * (ab[1] + ba[2]), 0.5 * (ab[2] + ba[1]),
                           0.5 * (ab[3] + ba[3])};
      double eb[4] = {0.0, 0.0, 0.0, 0.0};
      ld04_adj(e, bv, al, Eb, eb, bb, alb);
      X.ec[c][0][t] = 0.5 * eb[0];
      X.ec[c][1][t] = 0.5 * eb[1];
      X.ec[c][2][t] = 0.5 * eb[2];
      X.ec[c][3][t] = 0.5 * eb[3];
      X.ec[c][4][t] = 0.5 * eb[0];
      X.ec[c][5][t] = 0.5 * eb[2];
      X.ec[c][6][t] = 0.5 * eb[1];
      X.ec[c][7][t] = 0.5 * eb[3];
    } else if constexpr (EMF == kFS18) {
      // corners: -u1 b_b + u2 b_a with u1, u2 the means of the two two-step
      // reconstructions of u_a and u_b (edge_emf)
      double ua_ab[4], ua_ba[4], ub_ab[4], ub_ba[4];
      two_step<RECON>(W.prim[1 + a], t, sa, sb, ua_ab);
      two_step<RECON>(W.prim[1 + a], t, sb, sa, ua_ba);
      two_step<RECON>(W.prim[1 + b], t, sa, sb, ub_ab);
      two_step<RECON>(W.prim[1 + b], t, sb, sa, ub_ba);
      constexpr int perm[4] = {0, 2, 1, 3};  // corner q -> [x_b x_a] index
      double u1[4], u2[4], e[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        u1[q] = 0.5 * (ua_ab[q] + ua_ba[perm[q]]);
        u2[q] = 0.5 * (ub_ab[q] + ub_ba[perm[q]]);
        e[q] = -u1[q] * bv[2 + (q & 1)] + u2[q] * bv[q >> 1];
      }
      double eb[4] = {0.0, 0.0, 0.0, 0.0};
      ld04_adj(e, bv, al, Eb, eb, bb, alb);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        bb[2 + (q & 1)] += -eb[q] * u1[q];
        bb[q >> 1] += eb[q] * u2[q];
        const double u1b = -eb[q] * bv[2 + (q & 1)], u2b = eb[q] * bv[q >> 1];
        X.ec[c][q][t] = 0.5 * u1b;                 // u_a, [x_a x_b]
        X.ec[c][4 + perm[q]][t] = 0.5 * u1b;       // u_a, [x_b x_a]
        X.ec[c][8 + q][t] = 0.5 * u2b;             // u_b, [x_a x_b]
        X.ec[c][12 + perm[q]][t] = 0.5 * u2b;      // u_b, [x_b x_a]
      }
    } else {
      double u[4];
      iface_along<RECON>(W.us[a], t, sb, u[0], u[1]);  // uaB, uaT
      iface_along<RECON>(W.us[b], t, sa, u[2], u[3]);  // ubL, ubR
      q26_ld04_adj(u, bv, al, Eb, ub, bb, alb);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      X.ea[c][q][t] = ub[q];
      X.ea[c][4 + q][t] = bb[q];
      X.ea[c][8 + q][t] = alb[q];
    }
    if (eta > 0.0) etaj_adj(X.bj, G, t, c, eta * Eb);
  }
}

// Adjoint of a face value v[f] read as one of the two arguments of an edge
// speed max(v[e - st], v[e]) at the edges e = f + st and e = f (axis d).
// Every value is loaded (indices kept in the box) before any is compared.
__device__ __forceinline__ double gather_max(const double* V, const double* AB, const Geom& G,
                                             const int s3[3], int f, int d) {
  const int st = G.st[d];
  const bool hi = s3[d] + 1 < G.N[d], lo = s3[d] >= 1;
  const double g1 = AB[hi ? f + st : f], g0 = AB[f];
  const double v0 = V[f], vp = V[hi ? f + st : f], vm = V[lo ? f - st : f];
  // first argument at edge f + st, second argument at edge f (no
  // short-circuit, so that no load waits inside a branch)
  const bool first = hi & (g1 != 0.0) & (v0 >= vp), second = lo & (g0 != 0.0) & !(vm >= v0);
  double acc = 0.0;
  acc += first ? g1 : 0.0;
  acc += second ? g0 : 0.0;
  return acc;
}

// Whether the update reads face s3 of direction a: [g, g+n] along the
// normal, [g, g+n) across.
__device__ __forceinline__ bool face_in_update_adj(const Geom& G, const int s3[3], int a) {
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  return s3[a] >= G.g && s3[a] <= G.g + G.n[a] && s3[b] >= G.g && s3[b] < G.g + G.n[b] &&
         s3[c] >= G.g && s3[c] < G.g + G.n[c];
}
// The flux adjoint of face t of direction a from v (transposed divergence),
// in the face's local order (normal, two transverse momentum components).
__device__ __forceinline__ void face_flux_adj(const Geom& G, const AdjArrays& X, const int s3[3],
                                              int t, int a, double dt, double Fl[5]) {
  double Fb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (face_in_update_adj(G, s3, a)) {
    const int sa = G.st[a];
    const bool i0 = interior_at(G, s3, -1), ia = interior_at(G, s3, a);
#pragma unroll
    for (int m = 0; m < 5; ++m)
      Fb[m] = dt * G.idx[a] * (vval(X, m, t, i0) - vval(X, m, t - sa, ia));
  }
  Fl[0] = Fb[0];
  Fl[1] = Fb[1 + a];
  Fl[2] = Fb[1 + (a + 1) % 3];
  Fl[3] = Fb[1 + (a + 2) % 3];
  Fl[4] = Fb[4];
}

// ---------------------------------------------------------------------------
// Joule flux in reverse (eta > 0), face direction blockIdx.y: the energy
// flux adjoint onto the face fields of the Ohmic terms (atomic accumulation
// into bj).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
    k_adj_joule(State S, Geom G, Work<double> W, AdjArrays X, double eta, const int* stop) {
  if (*stop) return;
  const int t = gidx();
  if (t >= G.elems) return;
  int s3[3];
  decode(G, t, s3);
  const int a = (int)blockIdx.y;
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  if (!face_in_update_adj(G, s3, a)) return;
  double Fl[5];
  face_flux_adj(G, X, s3, t, a, *W.dt, Fl);
  if (Fl[4] == 0.0) return;
  // J = eb (bcl + bcr)/2 - ec (bbl + bbr)/2 (joule)
  const double Jb = Fl[4];
  const int sa = G.st[a], sb = G.st[b], sc = G.st[c], l = t - sa;
  const double eb = 0.5 * (eta_j<double>(S, G, t, b, eta) + eta_j<double>(S, G, t + sc, b, eta));
  const double ec = 0.5 * (eta_j<double>(S, G, t, c, eta) + eta_j<double>(S, G, t + sb, c, eta));
  const double bbl = 0.5 * (S.b[b][l] + S.b[b][l + sb]), bbr = 0.5 * (S.b[b][t] + S.b[b][t + sb]);
  const double bcl = 0.5 * (S.b[c][l] + S.b[c][l + sc]), bcr = 0.5 * (S.b[c][t] + S.b[c][t + sc]);
  const double ebb = Jb * 0.5 * (bcl + bcr), ecb = -Jb * 0.5 * (bbl + bbr);
  const double qc = 0.25 * Jb * eb, qb = -0.25 * Jb * ec;
  atomicAdd(&X.bj[c][l], qc);
  atomicAdd(&X.bj[c][l + sc], qc);
  atomicAdd(&X.bj[c][t], qc);
  atomicAdd(&X.bj[c][t + sc], qc);
  atomicAdd(&X.bj[b][l], qb);
  atomicAdd(&X.bj[b][l + sb], qb);
  atomicAdd(&X.bj[b][t], qb);
  atomicAdd(&X.bj[b][t + sb], qb);
  etaj_adj(X.bj, G, t, b, eta * 0.5 * ebb);
  etaj_adj(X.bj, G, t + sc, b, eta * 0.5 * ebb);
  etaj_adj(X.bj, G, t, c, eta * 0.5 * ecb);
  etaj_adj(X.bj, G, t + sb, c, eta * 0.5 * ecb);
}

// ---------------------------------------------------------------------------
// Faces: the Riemann solver in reverse, one face of direction blockIdx.y per
// thread.  Its output adjoints: the flux adjoint from v (face_flux_adj), the
// alpha adjoints gathered from the edges that read alpha (edges of direction
// c read this face's arrays along b, those of direction b along c), and the
// u* adjoint that face_lines leaves in fa[a][7].  Writes the adjoints of the
// left and right face-local states to fa[a][0..13] and adds the normal-field
// adjoint to bn.
// ---------------------------------------------------------------------------
template <int RECON, int RIEMANN>
__global__ void __launch_bounds__(kBlock)
    k_adj_friemann(State S, Geom G, Work<double> W, AdjArrays X, double gamma, const int* stop) {
  if (*stop) return;
  const int t = gidx();
  if (t >= G.elems) return;
  const int a = (int)blockIdx.y;
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  const int sa = G.st[a];
  int s3[3];
  decode(G, t, s3);
  double Fl[5];
  face_flux_adj(G, X, s3, t, a, *W.dt, Fl);
  const double apb = gather_max(W.ap[a], X.ea[c][8], G, s3, t, b) +
                     gather_max(W.ap[a], X.ea[b][10], G, s3, t, c);
  const double amb = gather_max(W.am[a], X.ea[c][9], G, s3, t, b) +
                     gather_max(W.am[a], X.ea[b][11], G, s3, t, c);
  const double usb = X.fa[a][7][t];
  constexpr int r = recon_halfwidth(RECON);
  const bool inr = s3[a] >= r + 1 && s3[a] + r < G.N[a] - 1;
  // The stencils of the face-local states, loaded together with the inputs
  // above so that the thread waits for memory once: the six-point sequence
  // t - 3 sa .. t + 2 sa of each reconstructed primitive (the offsets fall
  // back to t where the stencil would leave the box; such faces are skipped).
  const int vmap[7] = {0, 1 + a, 1 + b, 1 + c, 4, 5 + b, 5 + c};
  double w[7][6];
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const double* P = X.prim[vmap[q]];
#pragma unroll
    for (int m = 0; m < 6; ++m) w[q][m] = stencil_uses<RECON>(m) ? P[inr ? t + (m - 3) * sa : t] : 0.0;
  }
  const double bn = S.b[a][t];
  __builtin_amdgcn_sched_barrier(0);
  FState<double> Lb, Rb;
  fstate_zero(Lb);
  fstate_zero(Rb);
  double bnb = 0.0;
  const bool any = Fl[0] != 0.0 || Fl[1] != 0.0 || Fl[2] != 0.0 || Fl[3] != 0.0 ||
                   Fl[4] != 0.0 || usb != 0.0 || apb != 0.0 || amb != 0.0;
  if (any && inr) {
    // face-local states as the forward face kernel forms them: the upper
    // value of cell t - sa and the lower value of cell t (shared slopes for
    // PPM)
    double qL[7], qR[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) recon_iface<RECON>(w[q], qL[q], qR[q]);
    const FState<double> L{qL[0], qL[1], qL[2], qL[3], qL[4], qL[5], qL[6]};
    const FState<double> R{qR[0], qR[1], qR[2], qR[3], qR[4], qR[5], qR[6]};
    face_outputs_adj<RIEMANN>(L, R, bn, gamma, Fl, apb, amb, usb, Lb, Rb, bnb);
  }
  X.fa[a][0][t] = Lb.rho;
  X.fa[a][1][t] = Lb.un;
  X.fa[a][2][t] = Lb.ut1;
  X.fa[a][3][t] = Lb.ut2;
  X.fa[a][4][t] = Lb.p;
  X.fa[a][5][t] = Lb.bt1;
  X.fa[a][6][t] = Lb.bt2;
  X.fa[a][7][t] = Rb.rho;
  X.fa[a][8][t] = Rb.un;
  X.fa[a][9][t] = Rb.ut1;
  X.fa[a][10][t] = Rb.ut2;
  X.fa[a][11][t] = Rb.p;
  X.fa[a][12][t] = Rb.bt1;
  X.fa[a][13][t] = Rb.bt2;
  X.bn[a][t] += bnb;
}

// ---------------------------------------------------------------------------
// Line gathers: out[f] (=, or += with acc) the adjoint of X[f] through the
// reconstructions along one axis whose upper / lower values have the adjoints
// UP (stored at the upper face of each centre) and LO (at its lower face):
// the sum over the 2r+1 centres whose stencil holds f, for every position of
// the box.  Each centre's
// reconstruction is reversed once: along x by the 64 lanes of a wavefront
// (stencil values and the five contributions by cross-lane shuffles), along y
// and z by a thread that takes a segment of a line and holds its values, the
// adjoints of its centres and the partial sums in registers.  Centres whose
// stencil leaves the box carry no adjoint.
// ---------------------------------------------------------------------------
struct LineJob {
  const double* X;
  const double* UP;
  const double* LO;
  double* out;
  int acc;
};
constexpr int kMaxLineJobs = 8;
struct LineJobs {
  LineJob j[kMaxLineJobs];
};
// Positions per thread of the y / z gathers (4 was slower at 64^3, 16 no
// faster).
constexpr int kLineChunk = 8;

template <int RECON>
__global__ void __launch_bounds__(kBlock) k_line_x(Geom G, LineJobs J, const int* stop) {
  if (*stop) return;
  constexpr int r = recon_halfwidth(RECON);
  constexpr int seg = 64 - 4 * r;  // positions resolved per wavefront
  const LineJob& L = J.j[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int N = G.N[0];
  const int nseg = (N + seg - 1) / seg;
  if (wave >= nseg * G.N[1] * G.N[2]) return;  // whole wavefronts
  const int row = wave / nseg, sg = wave % nseg;
  const int base = row * N;  // (y, z) row of x-contiguous values
  const int x = sg * seg - 2 * r + lane;  // position of this lane, and the centre it reverses
  const bool in = x >= 0 && x < N;
  const double xv = L.X[base + (in ? x : (x < 0 ? 0 : N - 1))];
  const bool valid = x - r >= 0 && x + r < N;
  const double lo = valid ? L.LO[base + x] : 0.0;
  const double up = valid && x + 1 < N ? L.UP[base + x + 1] : 0.0;
  double q[5], qb[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    q[m] = (m - 2 >= -r && m - 2 <= r) ? __shfl(xv, lane + m - 2, 64) : 0.0;
    qb[m] = 0.0;
  }
  if (lo != 0.0 || up != 0.0) recon_cell_adj5<RECON>(q, lo, up, qb);
  // position x receives qb[m] of the centre at lane - (m - 2); lanes
  // [2r, 63-2r] have every such centre (and its stencil) in the wavefront
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < 5; ++m)
    if (m - 2 >= -r && m - 2 <= r) acc += __shfl(qb[m], lane - (m - 2), 64);
  if (in && lane >= 2 * r && lane < 64 - 2 * r) {
    double* o = L.out + base + x;
    *o = L.acc ? *o + acc : acc;
  }
}

template <int RECON, int D>
__global__ void __launch_bounds__(kBlock) k_line_march(Geom G, LineJobs J, const int* stop) {
  if (*stop) return;
  constexpr int r = recon_halfwidth(RECON);
  constexpr int CH = kLineChunk;
  constexpr int NC = CH + 2 * r;  // centres whose stencil holds a position of the chunk
  constexpr int NV = CH + 4 * r;  // values the stencils of those centres read
  constexpr int C = D == 1 ? 2 : 1;  // transverse axes: x and C
  const LineJob& L = J.j[blockIdx.z];
  const int lane = blockIdx.x * kBlock + threadIdx.x;
  if (lane >= G.N[0] * G.N[C]) return;
  const int base = lane % G.N[0] + (lane / G.N[0]) * G.st[C];
  const int st = G.st[D], N = G.N[D];
  const int p0 = blockIdx.y * CH;
  auto clampN = [N](int p) { return p < 0 ? 0 : (p >= N ? N - 1 : p); };
  // Every load of the chunk is issued before the first reverse, so that a
  // thread waits for memory once (indices clamped into the line): val[j] is
  // position p0 - 2r + j (only centres whose stencil lies in the line read
  // it), lo[i] / up[i] the adjoints of centre p0 - r + i, old[k] the output
  // at p0 + k of an accumulating job.
  double val[NV], lo[NC], up[NC], old[CH];
#pragma unroll
  for (int j = 0; j < NV; ++j) val[j] = L.X[base + clampN(p0 - 2 * r + j) * st];
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    const int c = p0 - r + i;
    const bool valid = c - r >= 0 && c + r < N;
    const double l = L.LO[base + clampN(c) * st];
    const double h = L.UP[base + clampN(c + 1) * st];
    lo[i] = valid ? l : 0.0;
    up[i] = valid && c + 1 < N ? h : 0.0;
  }
#pragma unroll
  for (int k = 0; k < CH; ++k) old[k] = 0.0;
  if (L.acc) {
#pragma unroll
    for (int k = 0; k < CH; ++k) old[k] = L.out[base + clampN(p0 + k) * st];
  }
  __builtin_amdgcn_sched_barrier(0);
  // centres in increasing order, each adding its stencil's adjoints
  double acc[CH];
#pragma unroll
  for (int k = 0; k < CH; ++k) acc[k] = 0.0;
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    if (lo[i] != 0.0 || up[i] != 0.0) {
      double q[5], qb[5];
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        q[m] = (m - 2 >= -r && m - 2 <= r) ? val[i + m - 2 + r] : 0.0;
        qb[m] = 0.0;
      }
      recon_cell_adj5<RECON>(q, lo[i], up[i], qb);
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const int k = i - r + m - 2;  // chunk position of stencil point m
        if (m - 2 >= -r && m - 2 <= r && k >= 0 && k < CH) acc[k] += qb[m];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    if (p0 + k < N) L.out[base + (p0 + k) * st] = L.acc ? old[k] + acc[k] : acc[k];
  }
}

// One line gather launch per axis for up to kMaxLineJobs arrays.
template <int RECON>
int launch_lines(hipStream_t st, const Geom& G, int D, const LineJobs& J, int njobs,
                 const int* stop) {
  if (D == 0) {
    constexpr int seg = 64 - 4 * recon_halfwidth(RECON);
    const long long waves = (long long)((G.N[0] + seg - 1) / seg) * G.N[1] * G.N[2];
    const int blocks = (int)((waves + kBlock / 64 - 1) / (kBlock / 64));
    hipLaunchKernelGGL(k_line_x<RECON>, dim3(blocks, njobs), dim3(kBlock), 0, st, G, J, stop);
  } else {
    const int C = D == 1 ? 2 : 1;
    const int blocks = (G.N[0] * G.N[C] + kBlock - 1) / kBlock;
    const dim3 grid(blocks, (G.N[D] + kLineChunk - 1) / kLineChunk, njobs);
    if (D == 1)
      hipLaunchKernelGGL((k_line_march<RECON, 1>), grid, dim3(kBlock), 0, st, G, J, stop);
    else
      hipLaunchKernelGGL((k_line_march<RECON, 2>), grid, dim3(kBlock), 0, st, G, J, stop);
  }
  if (hipGetLastError() != hipSuccess) return fail(CTMHD_EHIP, "kernel launch failed: line gather");
  return CTMHD_OK;
}

// ---------------------------------------------------------------------------
// Faces, part 0: the u* and face-field adjoints of face direction a gathered
// from the edges that reconstruct them along the two transverse axes: edges
// of direction c read them along b, edges of direction b along c.  Written to
// fa[a][7] and bn[a]; on each axis the faces whose first gather it is write,
// the others add.  Without u* at the edges (B25a) only the face fields are
// gathered, and k_adj_zero3 has cleared fa[a][7].
// ---------------------------------------------------------------------------
template <int RECON>
int face_lines(hipStream_t st, const Geom& G, const State& S, const Work<double>& W,
               const AdjArrays& X, bool ustar, const int* stop) {
  for (int D = 0; D < 3; ++D) {
    LineJobs J{};
    int n = 0;
    for (int a = 0; a < 3; ++a) {
      const int b = (a + 1) % 3, c = (a + 2) % 3;
      if (D == b) {  // the first gather of face direction a when b < c
        const int acc = b > c;
        if (ustar) J.j[n++] = LineJob{W.us[a], X.ea[c][0], X.ea[c][1], X.fa[a][7], acc};
        J.j[n++] = LineJob{S.b[a], X.ea[c][4], X.ea[c][5], X.bn[a], acc};
      } else if (D == c) {
        const int acc = c > b;
        if (ustar) J.j[n++] = LineJob{W.us[a], X.ea[b][2], X.ea[b][3], X.fa[a][7], acc};
        J.j[n++] = LineJob{S.b[a], X.ea[b][6], X.ea[b][7], X.bn[a], acc};
      }
    }
    const int rc = launch_lines<RECON>(st, G, D, J, n, stop);
    if (rc) return rc;
  }
  return CTMHD_OK;
}

// ---------------------------------------------------------------------------
// Cells: face-state adjoints through the reverse of the reconstructions (line
// gathers into the primitive adjoints pb, three axes in turn), then
// primitive -> conserved.
// ---------------------------------------------------------------------------
template <int RECON>
int cell_lines(hipStream_t st, const Geom& G, const AdjArrays& X, double* const pb[8],
               const int* stop) {
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const int vmap[7] = {0, 1 + a, 1 + b, 1 + c, 4, 5 + b, 5 + c};
    LineJobs J{};
    for (int q = 0; q < 7; ++q) {
      // the left state of face e is the upper value of cell e - st, the right
      // state the lower value of cell e; axis 0 writes its seven primitives
      // first, bc0 is first written by axis 1
      J.j[q] = LineJob{X.prim[vmap[q]], X.fa[a][q], X.fa[a][7 + q], pb[vmap[q]],
                       a == 0 ? 0 : (a == 1 ? (vmap[q] != 5) : 1)};
    }
    const int rc = launch_lines<RECON>(st, G, a, J, 7, stop);
    if (rc) return rc;
  }
  return CTMHD_OK;
}

// ---------------------------------------------------------------------------
// B25a cell EMF (eq. emf:b25a-emf-centre), reconstructed to the edge corners
// in two steps in both orders (first along d1 to the x_d1 faces, then along
// d2 to the edge).  In reverse, per edge direction and order: the first-step
// face values (recomputed here), their adjoints gathered along d2 from the
// stored corner adjoints, then the cell-EMF adjoint gathered along d1; all
// through the line gathers above.  Finally the cell-EMF adjoint onto u and
// the cell-centred field.
// ---------------------------------------------------------------------------
// First step along d1 at every position, for every edge direction c, field
// and order (d1 = a then b): the values on both sides of the x_d1 interface
// at t (upper value of the cell t - st_d1, lower value of t), 0 where the
// stencil leaves the box.
template <int RECON, int EMF>
__global__ void __launch_bounds__(kBlock)
    k_adj_iface(Geom G, Work<double> W, AdjArrays X, const int* stop) {
  if (*stop) return;
  const int t = gidx();
  if (t >= G.elems) return;
  int s3[3];
  decode(G, t, s3);
  constexpr int r = recon_halfwidth(RECON);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int f = 0; f < corner_fields(EMF); ++f)
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        const int d1 = o == 0 ? (c + 1) % 3 : (c + 2) % 3;
        double l = 0.0, h = 0.0;
        if (s3[d1] - 1 - r >= 0 && s3[d1] + r < G.N[d1])
          iface_along<RECON>(corner_src<EMF>(W, c, f), t, gstride(G, d1), l, h);
        X.fv[c][f][o][0][t] = l;
        X.fv[c][f][o][1][t] = h;
      }
}

// FS18: the cell-velocity adjoints onto the primitive adjoints.
__global__ void __launch_bounds__(kBlock)
    k_adj_ucell(Geom G, AdjArrays X, PrimPtrs PB, const int* stop) {
  if (*stop) return;
  const int t = gidx();
  if (t >= G.elems) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) PB.p[1 + d][t] += X.eb[d][t];
}

// e_c = -u_a b_b + u_b b_a in reverse, all three directions: adds to the
// primitive adjoints.
__global__ void __launch_bounds__(kBlock)
    k_adj_ecell(Geom G, AdjArrays X, PrimPtrs PB, const int* stop) {
  if (*stop) return;
  const int t = gidx();
  if (t >= G.elems) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double g = X.eb[c][t];
    if (g == 0.0) continue;
    const int a = (c + 1) % 3, b = (c + 2) % 3;
    PB.p[1 + a][t] += -g * X.prim[5 + b][t];
    PB.p[5 + b][t] += -g * X.prim[1 + a][t];
    PB.p[1 + b][t] += g * X.prim[5 + a][t];
    PB.p[5 + a][t] += g * X.prim[1 + b][t];
  }
}

// Per axis D, one launch of the second-step gathers (the orders whose second
// axis is D), then the first-step gathers (the orders whose first axis is D)
// in launches whose jobs write distinct cell-field adjoints; the first gather
// into a cell-field adjoint writes it, the later ones add.
template <int RECON, int EMF>
int cell_corner_adj(hipStream_t st, const Geom& G, const Work<double>& W, const AdjArrays& X,
                    const PrimPtrs& PB, const int* stop) {
  constexpr int NF = corner_fields(EMF);
  const int nb = nblocks(G.elems);
  LAUNCH((k_adj_iface<RECON, EMF>), nb, G, W, X, stop);
  for (int D = 0; D < 3; ++D) {
    LineJobs J{};
    int n = 0;
    for (int c = 0; c < 3; ++c)
      for (int f = 0; f < NF; ++f)
        for (int o = 0; o < 2; ++o) {
          const int d2 = o == 0 ? (c + 2) % 3 : (c + 1) % 3;
          if (d2 != D) continue;
          double* const* E = X.ec[c] + 8 * f + 4 * o;  // LB, RB, LT, RT
          // the lower-d1 face values give the LB / LT corners, the upper RB / RT
          J.j[n++] = LineJob{X.fv[c][f][o][0], E[0], E[2], X.fb[c][f][o][0], 0};
          J.j[n++] = LineJob{X.fv[c][f][o][1], E[1], E[3], X.fb[c][f][o][1], 0};
        }
    if (const int rc = launch_lines<RECON>(st, G, D, J, n, stop)) return rc;
  }
  bool written[3] = {false, false, false};
  for (int D = 0; D < 3; ++D) {
    LineJob pend[12];
    int dst[12], np = 0;
    for (int c = 0; c < 3; ++c)
      for (int f = 0; f < NF; ++f)
        for (int o = 0; o < 2; ++o) {
          const int d1 = o == 0 ? (c + 1) % 3 : (c + 2) % 3;
          if (d1 != D) continue;
          const int k = EMF == kB25A ? c : corner_comp(c, f);
          pend[np] = LineJob{corner_src<EMF>(W, c, f), X.fb[c][f][o][0], X.fb[c][f][o][1], X.eb[k], 0};
          dst[np++] = k;
        }
    while (np > 0) {  // launches with distinct destinations
      LineJobs J{};
      int n = 0;
      bool used[3] = {false, false, false};
      for (int i = 0; i < np;) {
        if (!used[dst[i]] && n < kMaxLineJobs) {
          used[dst[i]] = true;
          J.j[n] = pend[i];
          J.j[n++].acc = written[dst[i]] ? 1 : 0;
          pend[i] = pend[np - 1];
          dst[i] = dst[np - 1];
          --np;
        } else {
          ++i;
        }
      }
      for (int k = 0; k < 3; ++k) written[k] = written[k] || used[k];
      if (const int rc = launch_lines<RECON>(st, G, D, J, n, stop)) return rc;
    }
  }
  if constexpr (EMF == kB25A)
    LAUNCH(k_adj_ecell, nb, G, X, PB, stop);
  else
    LAUNCH(k_adj_ucell, nb, G, X, PB, stop);
  return CTMHD_OK;
}

// Primitive -> conserved adjoints of cell w (Sec. 2.2, eq. state:primitive):
// ca[5] the conserved fields, cb[3] the cell-centred field; 0 on the last
// layer of each axis, which has no upper face.
// p = (gamma - 1) (e - rho |u|^2 / 2 - |bc|^2 / 2), u = m / rho
__device__ __forceinline__ void cell_cons_adj(const AdjArrays& X, const PrimPtrs& PB, double gm1,
                                              int w, bool valid, double ca[5], double cb[3]) {
  if (!valid) {
#pragma unroll
    for (int m = 0; m < 5; ++m) ca[m] = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) cb[d] = 0.0;
    return;
  }
  double pb[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) pb[v] = PB.p[v][w];
  const double rho = X.prim[0][w], p_b = pb[4];
  const double u[3] = {X.prim[1][w], X.prim[2][w], X.prim[3][w]};
  const double bc[3] = {X.prim[5][w], X.prim[6][w], X.prim[7][w]};
  double rb = pb[0] + 0.5 * gm1 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * p_b;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    rb -= pb[1 + d] * u[d] / rho;
    ca[1 + d] = pb[1 + d] / rho - gm1 * p_b * u[d];
    cb[d] = pb[5 + d] - gm1 * p_b * bc[d];
  }
  ca[0] = rb;
  ca[4] = gm1 * p_b;
}

// The cell-centred field adjoint cb[a] of cell w alone (as cell_cons_adj).
__device__ __forceinline__ double cell_cb_adj(const AdjArrays& X, const PrimPtrs& PB, double gm1,
                                              int w, int a, bool valid) {
  return valid ? PB.p[5 + a][w] - gm1 * PB.p[4][w] * X.prim[5 + a][w] : 0.0;
}

// Per position: the conserved-field adjoints into ca (cell_cons_adj), and
// the face-field adjoint bn completed with the Ohmic part (ohm != 0) and half
// of each adjacent cell's cell-centred adjoint (bc_a = (b_a[lower] +
// b_a[upper]) / 2).
__global__ void __launch_bounds__(kBlock)
    k_adj_cons(Geom G, AdjArrays X, PrimPtrs PB, double gamma, int ohm, const int* stop) {
  if (*stop) return;
  const int t = gidx();
  if (t >= G.elems) return;
  int s3[3];
  decode(G, t, s3);
  bool up[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) up[d] = s3[d] < G.N[d] - 1;
  const double gm1 = gamma - 1.0;
  double ca[5], cb[3];
  cell_cons_adj(X, PB, gm1, t, up[0] && up[1] && up[2], ca, cb);
#pragma unroll
  for (int m = 0; m < 5; ++m) X.ca[m][t] = ca[m];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // the lower neighbour along a lies on the last layer of no axis other
    // than those t lies on
    const double cbm =
        s3[a] >= 1 ? cell_cb_adj(X, PB, gm1, t - G.st[a], a, up[(a + 1) % 3] && up[(a + 2) % 3])
                   : 0.0;
    X.bn[a][t] += (ohm ? X.bj[a][t] : 0.0) + 0.5 * (cb[a] + cbm);
  }
}

// out = c2 g2 + c1 g1 + (sum over all periodic copies of the interior
// position of the cell / face adjoints) on interior positions, 0 elsewhere.
// A stopped call (non-finite dt) writes NaN.
__global__ void __launch_bounds__(kBlock)
    k_adj_fold(Geom G, State out, State g2, double c2, State g1, double c1, AdjArrays X,
               const int* stop) {
  const int t = gidx();
  if (t >= G.elems) return;
  int s3[3];
  decode(G, t, s3);
  bool inter = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) inter = inter && s3[d] >= G.g && s3[d] < G.g + G.n[d];
  double vc[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, vb[3] = {0.0, 0.0, 0.0};
  if (inter) {
    if (*stop) {
#pragma unroll
      for (int m = 0; m < 5; ++m) vc[m] = __builtin_nan("");
#pragma unroll
      for (int a = 0; a < 3; ++a) vb[a] = __builtin_nan("");
    } else {
      int mlo[3], mhi[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        mlo[d] = -(s3[d] / G.n[d]);
        mhi[d] = (G.N[d] - 1 - s3[d]) / G.n[d];
      }
      for (int mz = mlo[2]; mz <= mhi[2]; ++mz)
        for (int my = mlo[1]; my <= mhi[1]; ++my)
          for (int mx = mlo[0]; mx <= mhi[0]; ++mx) {
            const int w = t + mx * G.n[0] + my * G.n[1] * G.st[1] + mz * G.n[2] * G.st[2];
#pragma unroll
            for (int m = 0; m < 5; ++m) vc[m] += X.ca[m][w];
#pragma unroll
            for (int a = 0; a < 3; ++a) vb[a] += X.bn[a][w];
          }
#pragma unroll
      for (int m = 0; m < 5; ++m) vc[m] += c2 * g2.c[m][t] + (c1 != 0.0 ? c1 * g1.c[m][t] : 0.0);
#pragma unroll
      for (int a = 0; a < 3; ++a) vb[a] += c2 * g2.b[a][t] + (c1 != 0.0 ? c1 * g1.b[a][t] : 0.0);
    }
  }
#pragma unroll
  for (int m = 0; m < 5; ++m) out.c[m][t] = vc[m];
#pragma unroll
  for (int a = 0; a < 3; ++a) out.b[a][t] = vb[a];
}

// Start of a reverse from a tape: the recorded dt, and the stop flag, set
// where that dt is not a positive finite number.
__global__ void k_adj_tape_dt(const double* tdt, double* dt, int* stop) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double v = *tdt;
  *stop = v > 0.0 && __builtin_isfinite(v) ? 0 : 1;
  *dt = v;
}

// Copy of the forward face arrays alpha+, alpha-, u* (3 directions each).
__global__ void __launch_bounds__(kBlock) k_adj_save9(Geom G, Work<double> W, Work<double> D) {
  const int t = gidx();
  if (t >= G.elems) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    D.ap[a][t] = W.ap[a][t];
    D.am[a][t] = W.am[a][t];
    D.us[a][t] = W.us[a][t];
  }
}

// Clears the Ohmic accumulators, and the u* adjoints when no edge reads u*
// (B25a, FS18), where the face gathers leave them unwritten.  Not launched
// for Q26 without resistivity: nothing then reads either.
__global__ void __launch_bounds__(kBlock) k_adj_zero3(Geom G, AdjArrays X, int zero_us) {
  const int t = gidx();
  if (t >= G.elems) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    X.bj[a][t] = 0.0;
    if (zero_us) X.fa[a][7][t] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
// G1, prim, ea, fa, bn, bj, ca, saved face arrays of S0
constexpr int kAdjArrays = 8 + 8 + 36 + 42 + 3 + 3 + 5 + 9;
// B25a / FS18: per cell field of the corner reconstructions, 24 corner
// adjoints and 12 + 12 first-step values and adjoints; 3 cell-field adjoints
constexpr int kAdjArraysPerField = 24 + 12 + 12;

size_t adj_ws_bytes(const ctmhd_params* p, const ctmhd_box& b) {
  size_t e = 1;
  for (int d = 0; d < 3; ++d) e *= (size_t)(b.n[d] + 2 * b.ng);
  const int nf = p->emf_compute == CTMHD_EMF_FS18 ? 2 : p->emf_compute == CTMHD_EMF_B25A ? 1 : 0;
  const int n = kAdjArrays + nf * kAdjArraysPerField + (nf ? 3 : 0);
  return box_ws_bytes(b, 8, p) + (size_t)n * align256(e * 8);
}

int check_adjoint(const ctmhd_params* p) {
  if (p->precision != CTMHD_FP64)
    return fail(CTMHD_EUNSUPPORTED, "the adjoint is built for the FP64 form only");
  return CTMHD_OK;
}

// The primitive adjoints of vjp_d (in ea[0][0..7] once its face gathers are done).
PrimPtrs prim_adjoints(const AdjArrays& X) {
  PrimPtrs PB;
  for (int v = 0; v < 8; ++v) PB.p[v] = X.ea[0][v];
  return PB;
}

// D'(S)^T v into X.ca / X.bn (ghosted), given the forward face arrays of S in W.
template <int RECON, int RIEMANN, int EMF>
int vjp_d(hipStream_t st, const ctmhd_params* p, State S, const Geom& G, const Work<double>& W,
          const AdjArrays& X) {
  const int nb = nblocks(G.elems);
  if (EMF != kQ26 || p->eta > 0.0) LAUNCH(k_adj_zero3, nb, G, X, EMF != kQ26 ? 1 : 0);
  LAUNCH(k_adj_prim, nb, S, G, X, p->gamma, W.stop);
  if constexpr (EMF != kQ26) LAUNCH((k_prim<double, EMF>), nb, S, G, W, p->gamma, W.stop);
  hipLaunchKernelGGL((k_adj_edge<RECON, EMF>), dim3(nb, 3), dim3(kBlock), 0, st, S, G, W, X,
                     p->eta, W.stop);
  if (hipGetLastError() != hipSuccess) return fail(CTMHD_EHIP, "kernel launch failed: adjoint edges");
  if (const int rc = face_lines<RECON>(st, G, S, W, X, EMF == kQ26, W.stop)) return rc;
  // both face kernels take the direction from blockIdx.y
  if (p->eta > 0.0)
    hipLaunchKernelGGL(k_adj_joule, dim3(nb, 3), dim3(kBlock), 0, st, S, G, W, X, p->eta, W.stop);
  hipLaunchKernelGGL((k_adj_friemann<RECON, RIEMANN>), dim3(nb, 3), dim3(kBlock), 0, st, S, G, W,
                     X, p->gamma, W.stop);
  if (hipGetLastError() != hipSuccess) return fail(CTMHD_EHIP, "kernel launch failed: adjoint faces");
  // the primitive adjoints go to ea[0][0..7], free once the face gathers are done
  const PrimPtrs PB = prim_adjoints(X);
  if (const int rc = cell_lines<RECON>(st, G, X, PB.p, W.stop)) return rc;
  if constexpr (EMF != kQ26)
    if (const int rc = cell_corner_adj<RECON, EMF>(st, G, W, X, PB, W.stop)) return rc;
  LAUNCH(k_adj_cons, nb, G, X, PB, p->gamma, p->eta > 0.0 ? 1 : 0, W.stop);
  return CTMHD_OK;
}

// Everything an adjoint step works in, carved from the caller's workspace.
struct AdjCtx {
  Work<double> W, W0;  // forward work arrays; W0: W with the face arrays of S0
  State A, H;          // S0 with ghosts, S1 (the recomputing form)
  State G1;            // g1
  AdjArrays X;
};

template <int EMF>
int adj_setup(const ctmhd_params* p, const ctmhd_box& box, void* ws, size_t ws_bytes, AdjCtx& C) {
  const Geom G = make_geom(box);
  if (!ws || ws_bytes < adj_ws_bytes(p, box)) return fail(CTMHD_EARG, "workspace too small");
  int rc = build_work<double>(p, ws, ws_bytes, box, C.W, C.A, C.H);
  if (rc) return rc;
  const size_t e = (size_t)G.elems;
  Carve cv{(char*)ws + box_ws_bytes(box, 8, p)};
  AdjArrays& X = C.X;
  for (int m = 0; m < 5; ++m) C.G1.c[m] = cv.take<double>(e);
  for (int a = 0; a < 3; ++a) C.G1.b[a] = cv.take<double>(e);
  for (int v = 0; v < 8; ++v) X.prim[v] = cv.take<double>(e);
  for (int c = 0; c < 3; ++c)
    for (int q = 0; q < 12; ++q) X.ea[c][q] = cv.take<double>(e);
  for (int a = 0; a < 3; ++a)
    for (int q = 0; q < 14; ++q) X.fa[a][q] = cv.take<double>(e);
  for (int a = 0; a < 3; ++a) X.bn[a] = cv.take<double>(e);
  for (int a = 0; a < 3; ++a) X.bj[a] = cv.take<double>(e);
  for (int m = 0; m < 5; ++m) X.ca[m] = cv.take<double>(e);
  X.vs = 1.0;
  constexpr int NF = corner_fields(EMF);
  for (int c = 0; c < 3; ++c) {
    for (int q = 0; q < 16; ++q) X.ec[c][q] = q < 8 * NF ? cv.take<double>(e) : nullptr;
    for (int f = 0; f < 2; ++f)
      for (int o = 0; o < 2; ++o)
        for (int k = 0; k < 2; ++k) {
          X.fv[c][f][o][k] = f < NF ? cv.take<double>(e) : nullptr;
          X.fb[c][f][o][k] = f < NF ? cv.take<double>(e) : nullptr;
        }
  }
  for (int c = 0; c < 3; ++c) X.eb[c] = NF ? cv.take<double>(e) : nullptr;
  C.W0 = C.W;
  for (int a = 0; a < 3; ++a) {
    C.W0.ap[a] = cv.take<double>(e);
    C.W0.am[a] = cv.take<double>(e);
    C.W0.us[a] = cv.take<double>(e);
  }
  return CTMHD_OK;
}

UpdateCfg adj_update_cfg(const ctmhd_params* p) {
  UpdateCfg U;
  U.fofc = 0;
  U.crit = p->flag_criteria;
  U.gamma = p->gamma;
  U.sres = 0.0;
  U.force = nullptr;
  U.flag_storage = 0;
  return U;
}

// Both VJPs of the step and the folds, given S0 (A) and S1 (H) with ghosts
// and the forward face arrays of S1 (in W1) and of S0 (in W0); W1.dt holds dt.
template <int RECON, int RIEMANN, int EMF>
int adj_reverse(hipStream_t st, const ctmhd_params* p, const Geom& G, AdjCtx& C,
                const Work<double>& W1, const Work<double>& W0, State A, State H, State Gin,
                State Gout) {
  const int nb = nblocks(G.elems);
  AdjArrays& X = C.X;
  int rc;
  // stage 2 in reverse at S1: g1 = g2/2 + D'(S1)^T (g2/2), with g2 read in
  // place (its interior values)
  for (int m = 0; m < 5; ++m) X.v[m] = Gin.c[m];
  for (int a = 0; a < 3; ++a) X.v[5 + a] = Gin.b[a];
  X.vs = 0.5;
  if ((rc = vjp_d<RECON, RIEMANN, EMF>(st, p, H, G, W1, X))) return rc;
  LAUNCH(k_adj_fold, nb, G, C.G1, Gin, 0.5, Gin, 0.0, X, W1.stop);
  // stage 1 in reverse at S0: g0 = g2/2 + g1 + D'(S0)^T g1
  for (int m = 0; m < 5; ++m) X.v[m] = C.G1.c[m];
  for (int a = 0; a < 3; ++a) X.v[5 + a] = C.G1.b[a];
  X.vs = 1.0;
  if ((rc = vjp_d<RECON, RIEMANN, EMF>(st, p, A, G, W0, X))) return rc;
  LAUNCH(k_adj_fold, nb, G, Gout, Gin, 0.5, C.G1, 1.0, X, W1.stop);
  return CTMHD_OK;
}

// The tape of one recorded step: S0 and S1 with ghosts, the face arrays
// (alpha+, alpha-, u*) of S0 and of S1, and dt.
struct Tape {
  State S0, S1;
  double* ap[2][3];
  double* am[2][3];
  double* us[2][3];
  double* dt;
};
constexpr int kTapeArrays = 8 + 8 + 18;

size_t tape_bytes_of(const ctmhd_box& b) {
  size_t e = 1;
  for (int d = 0; d < 3; ++d) e *= (size_t)(b.n[d] + 2 * b.ng);
  return (size_t)kTapeArrays * align256(e * 8) + 256;
}

Tape carve_tape(void* tape, const Geom& G) {
  Tape T;
  Carve cv{(char*)tape};
  const size_t e = (size_t)G.elems;
  for (int m = 0; m < 5; ++m) T.S0.c[m] = cv.take<double>(e);
  for (int a = 0; a < 3; ++a) T.S0.b[a] = cv.take<double>(e);
  for (int m = 0; m < 5; ++m) T.S1.c[m] = cv.take<double>(e);
  for (int a = 0; a < 3; ++a) T.S1.b[a] = cv.take<double>(e);
  for (int k = 0; k < 2; ++k)
    for (int a = 0; a < 3; ++a) {
      T.ap[k][a] = cv.take<double>(e);
      T.am[k][a] = cv.take<double>(e);
      T.us[k][a] = cv.take<double>(e);
    }
  T.dt = cv.take<double>(1);
  return T;
}

Work<double> with_face_arrays(const Work<double>& W, const Tape& T, int k) {
  Work<double> R = W;
  for (int a = 0; a < 3; ++a) {
    R.ap[a] = T.ap[k][a];
    R.am[a] = T.am[k][a];
    R.us[a] = T.us[k][a];
  }
  return R;
}

template <int RECON, int RIEMANN, int EMF>
int adjoint_box(const ctmhd_params* p_in, const ctmhd_box* box, const double* const cons_n[5],
                const double* const bface_n[3], const double* dt, const double* const g_cons[5],
                const double* const g_bface[3], double* const g_cons_out[5],
                double* const g_bface_out[3], const void* tape, void* ws, size_t ws_bytes,
                hipStream_t st) {
  ctmhd_params pp = *p_in;
  pp.fofc = 0;  // the differentiated step takes no flux correction
  const ctmhd_params* p = &pp;
  const Geom G = make_geom(*box);
  AdjCtx C;
  int rc = adj_setup<EMF>(p, *box, ws, ws_bytes, C);
  if (rc) return rc;
  Work<double>& W = C.W;
  State Gin, Gout;
  for (int m = 0; m < 5; ++m) {
    Gin.c[m] = const_cast<double*>(g_cons[m]);
    Gout.c[m] = g_cons_out[m];
  }
  for (int a = 0; a < 3; ++a) {
    Gin.b[a] = const_cast<double*>(g_bface[a]);
    Gout.b[a] = g_bface_out[a];
  }
  if (tape) {
    // everything the reverse needs was recorded by ctmhd_step_record
    const Tape T = carve_tape(const_cast<void*>(tape), G);
    LAUNCH(k_adj_tape_dt, 1, T.dt, W.dt, W.stop);
    return adj_reverse<RECON, RIEMANN, EMF>(st, p, G, C, with_face_arrays(W, T, 1),
                                            with_face_arrays(C.W0, T, 0), T.S0, T.S1, Gin, Gout);
  }
  LAUNCH(k_init, 1, W.stop, W.smax, W.nflag);
  State S0;
  for (int m = 0; m < 5; ++m) S0.c[m] = const_cast<double*>(cons_n[m]);
  for (int a = 0; a < 3; ++a) S0.b[a] = const_cast<double*>(bface_n[a]);
  const FacePlan FP = make_face_plan(G, p->recon, p->emf_compute, tile_chunk(p), tile_xrows(p));
  const int ninter = G.n[0] * G.n[1] * G.n[2];
  const int nb = nblocks(G.elems);
  const UpdateCfg U = adj_update_cfg(p);
  State A = C.A, H = C.H;
  // forward: S0 with ghosts, the caller's dt, stage 1 into H = S1
  LAUNCH(k_copy, nb, A, S0, G.elems, (const int*)nullptr);
  LAUNCH(k_wrap, nb, A, G, W.stop);
  LAUNCH(k_dt_final, 1, W.smax, W.nflag, p->cfl, dt, W.dt, (double*)nullptr, W.stop,
         (long long*)nullptr);
  if ((rc = launch_faces<double, RECON>(st, p, A, G, W, FP, 0, nullptr))) return rc;
  LAUNCH(k_adj_save9, nb, G, W, C.W0);
  if constexpr (EMF != kQ26) LAUNCH((k_prim<double, EMF>), nb, A, G, W, p->gamma, W.stop);
  if constexpr (first_step_stored(EMF, RECON))
    LAUNCH((k_first_step<double, RECON, EMF>), nb, G, W, W.stop);
  if ((rc = launch_emf<double, RECON>(st, p, A, G, W, 0))) return rc;
  LAUNCH(k_update<double>, nblocks(ninter), A, A, H, G, W, 0, 0, U, (long long*)nullptr, 0, W.stop);
  if ((rc = launch_faces<double, RECON>(st, p, H, G, W, FP, 1, nullptr))) return rc;
  return adj_reverse<RECON, RIEMANN, EMF>(st, p, G, C, W, C.W0, A, H, Gin, Gout);
}

// One forward step (frozen dt, no flux correction) that records its tape:
// S0 and S1 with ghosts and the face arrays of both stages go to the tape,
// S^{n+1} to the caller's arrays.  The same kernels and arithmetic as
// ctmhd_step.
template <int RECON>
int record_box(const ctmhd_params* p_in, const ctmhd_box* box, double* const cons[5],
               double* const bface[3], const double* dt, void* tape, void* ws, size_t ws_bytes,
               hipStream_t st) {
  ctmhd_params pp = *p_in;
  pp.fofc = 0;
  const ctmhd_params* p = &pp;
  const Geom G = make_geom(*box);
  Work<double> W;
  State A_unused, H_unused;
  int rc = build_work<double>(p, ws, ws_bytes, *box, W, A_unused, H_unused);
  if (rc) return rc;
  const Tape T = carve_tape(tape, G);
  State user;
  for (int m = 0; m < 5; ++m) user.c[m] = cons[m];
  for (int a = 0; a < 3; ++a) user.b[a] = bface[a];
  const FacePlan FP = make_face_plan(G, p->recon, p->emf_compute, tile_chunk(p), tile_xrows(p));
  const int ninter = G.n[0] * G.n[1] * G.n[2];
  const int nb = nblocks(G.elems);
  const UpdateCfg U = adj_update_cfg(p);
  const Work<double> W0 = with_face_arrays(W, T, 0), W1 = with_face_arrays(W, T, 1);
  LAUNCH(k_init, 1, W.stop, W.smax, W.nflag);
  LAUNCH(k_copy, nb, T.S0, user, G.elems, (const int*)nullptr);
  LAUNCH(k_wrap, nb, T.S0, G, W.stop);
  if (!dt) {  // the CFL dt of S^n, as ctmhd_step computes it
    const double dxmin = fmin(G.dx[0], fmin(G.dx[1], G.dx[2]));
    const double sres = p->eta > 0.0 ? 2.0 * p->eta / (dxmin * dxmin) : 0.0;
    int dtb = nblocks(ninter);
    if (dtb > 2048) dtb = 2048;
    LAUNCH(k_dt, dtb, T.S0, G, p->gamma, sres, W.smax, W.stop);
  }
  LAUNCH(k_dt_final, 1, W.smax, W.nflag, p->cfl, dt, W.dt, T.dt, W.stop, (long long*)nullptr);
  if (p->emf_compute == CTMHD_EMF_B25A) {
    LAUNCH((k_prim<double, kB25A>), nb, T.S0, G, W0, p->gamma, W.stop);
    if constexpr (first_step_stored(kB25A, RECON))
      LAUNCH((k_first_step<double, RECON, kB25A>), nb, G, W0, W.stop);
  } else if (p->emf_compute == CTMHD_EMF_FS18) {
    LAUNCH((k_prim<double, kFS18>), nb, T.S0, G, W0, p->gamma, W.stop);
    if constexpr (first_step_stored(kFS18, RECON))
      LAUNCH((k_first_step<double, RECON, kFS18>), nb, G, W0, W.stop);
  }
  if ((rc = launch_faces<double, RECON>(st, p, T.S0, G, W0, FP, 0, nullptr))) return rc;
  if ((rc = launch_emf<double, RECON>(st, p, T.S0, G, W0, 0))) return rc;
  LAUNCH(k_update<double>, nblocks(ninter), T.S0, T.S0, T.S1, G, W0, 0, 0, U,
         (long long*)nullptr, 0, W.stop);
  if (p->emf_compute == CTMHD_EMF_B25A) {
    LAUNCH((k_prim<double, kB25A>), nb, T.S1, G, W1, p->gamma, W.stop);
    if constexpr (first_step_stored(kB25A, RECON))
      LAUNCH((k_first_step<double, RECON, kB25A>), nb, G, W1, W.stop);
  } else if (p->emf_compute == CTMHD_EMF_FS18) {
    LAUNCH((k_prim<double, kFS18>), nb, T.S1, G, W1, p->gamma, W.stop);
    if constexpr (first_step_stored(kFS18, RECON))
      LAUNCH((k_first_step<double, RECON, kFS18>), nb, G, W1, W.stop);
  }
  if ((rc = launch_faces<double, RECON>(st, p, T.S1, G, W1, FP, 1, nullptr))) return rc;
  if ((rc = launch_emf<double, RECON>(st, p, T.S1, G, W1, 1))) return rc;
  // a stopped step (non-finite dt) leaves the caller's state as it was
  LAUNCH(k_update<double>, nblocks(ninter), T.S0, T.S1, user, G, W1, 1, 0, U,
         (long long*)nullptr, 0, W.stop);
  return CTMHD_OK;
}

template <int RECON>
int adjoint_riemann(const ctmhd_params* p, const ctmhd_box* box, const double* const cons_n[5],
                    const double* const bface_n[3], const double* dt,
                    const double* const g_cons[5], const double* const g_bface[3],
                    double* const g_cons_out[5], double* const g_bface_out[3], const void* tape,
                    void* ws, size_t ws_bytes, hipStream_t st) {
#define CTMHD_ADJ(RI, EM) \
  adjoint_box<RECON, RI, EM>(p, box, cons_n, bface_n, dt, g_cons, g_bface, g_cons_out, g_bface_out, tape, ws, ws_bytes, st)
  if (p->emf_compute == CTMHD_EMF_B25A)
    return p->riemann == CTMHD_RIEMANN_HLLD ? CTMHD_ADJ(kHLLD, kB25A) : CTMHD_ADJ(kLLF, kB25A);
  if (p->emf_compute == CTMHD_EMF_FS18)
    return p->riemann == CTMHD_RIEMANN_HLLD ? CTMHD_ADJ(kHLLD, kFS18) : CTMHD_ADJ(kLLF, kFS18);
  return p->riemann == CTMHD_RIEMANN_HLLD ? CTMHD_ADJ(kHLLD, kQ26) : CTMHD_ADJ(kLLF, kQ26);
#undef CTMHD_ADJ
}

int adjoint_dispatch(const ctmhd_params* p, const ctmhd_box* box, const double* const cons_n[5],
                     const double* const bface_n[3], const double* dt,
                     const double* const g_cons[5], const double* const g_bface[3],
                     double* const g_cons_out[5], double* const g_bface_out[3], const void* tape,
                     void* ws, size_t ws_bytes, hipStream_t st) {
  switch (p->recon) {
    case CTMHD_RECON_PC:
      return adjoint_riemann<kPC>(p, box, cons_n, bface_n, dt, g_cons, g_bface, g_cons_out,
                                  g_bface_out, tape, ws, ws_bytes, st);
    case CTMHD_RECON_PLM_MC:
      return adjoint_riemann<kPLM_MC>(p, box, cons_n, bface_n, dt, g_cons, g_bface, g_cons_out,
                                      g_bface_out, tape, ws, ws_bytes, st);
    case CTMHD_RECON_PLM_MINMOD:
      return adjoint_riemann<kPLM_MM>(p, box, cons_n, bface_n, dt, g_cons, g_bface, g_cons_out,
                                      g_bface_out, tape, ws, ws_bytes, st);
    default:
      return adjoint_riemann<kPPM>(p, box, cons_n, bface_n, dt, g_cons, g_bface, g_cons_out,
                                   g_bface_out, tape, ws, ws_bytes, st);
  }
}

int check_gradients(const double* const g_cons[5], const double* const g_bface[3],
                    double* const g_cons_out[5], double* const g_bface_out[3]) {
  if (!g_cons || !g_bface || !g_cons_out || !g_bface_out)
    return fail(CTMHD_EARG, "a pointer argument is NULL");
  for (int m = 0; m < 5; ++m)
    if (!g_cons[m] || !g_cons_out[m]) return fail(CTMHD_EARG, "a cons pointer is NULL");
  for (int a = 0; a < 3; ++a)
    if (!g_bface[a] || !g_bface_out[a]) return fail(CTMHD_EARG, "a bface pointer is NULL");
  return CTMHD_OK;
}

}  // namespace

extern "C" {

size_t ctmhd_adjoint_workspace_bytes(const ctmhd_params* p, const ctmhd_box* box) {
  if (check_params(p) || check_adjoint(p) || check_box(p, box)) return 0;
  return adj_ws_bytes(p, *box);
}

int ctmhd_step_adjoint(const ctmhd_params* p, const ctmhd_box* box, const double* const cons_n[5],
                       const double* const bface_n[3], const double* dt,
                       const double* const g_cons[5], const double* const g_bface[3],
                       double* const g_cons_out[5], double* const g_bface_out[3], void* workspace,
                       size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  int rc = check_params(p);
  if (rc) return rc;
  if ((rc = check_adjoint(p))) return rc;
  if ((rc = check_box(p, box))) return rc;
  if (!cons_n || !bface_n || !dt) return fail(CTMHD_EARG, "a pointer argument is NULL");
  if ((rc = check_gradients(g_cons, g_bface, g_cons_out, g_bface_out))) return rc;
  for (int m = 0; m < 5; ++m)
    if (!cons_n[m]) return fail(CTMHD_EARG, "a cons pointer is NULL");
  for (int a = 0; a < 3; ++a)
    if (!bface_n[a]) return fail(CTMHD_EARG, "a bface pointer is NULL");
  if (((uintptr_t)workspace & 255) != 0) return fail(CTMHD_EARG, "workspace must be 256-byte aligned");
  return adjoint_dispatch(p, box, cons_n, bface_n, dt, g_cons, g_bface, g_cons_out, g_bface_out,
                          nullptr, workspace, ws_bytes, (hipStream_t)stream);
}

size_t ctmhd_tape_bytes(const ctmhd_params* p, const ctmhd_box* box) {
  if (check_params(p) || check_adjoint(p) || check_box(p, box)) return 0;
  return tape_bytes_of(*box);
}

int ctmhd_step_record(const ctmhd_params* p, const ctmhd_box* box, double* const cons[5],
                      double* const bface[3], const double* dt, void* tape, size_t tape_bytes,
                      void* workspace, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  int rc = check_params(p);
  if (rc) return rc;
  if ((rc = check_adjoint(p))) return rc;
  if ((rc = check_box(p, box))) return rc;
  if (!cons || !bface) return fail(CTMHD_EARG, "a pointer argument is NULL");
  for (int m = 0; m < 5; ++m)
    if (!cons[m]) return fail(CTMHD_EARG, "a cons pointer is NULL");
  for (int a = 0; a < 3; ++a)
    if (!bface[a]) return fail(CTMHD_EARG, "a bface pointer is NULL");
  if (!tape || tape_bytes < tape_bytes_of(*box)) return fail(CTMHD_EARG, "tape too small");
  if (((uintptr_t)tape & 255) != 0) return fail(CTMHD_EARG, "tape must be 256-byte aligned");
  if (!workspace || ws_bytes < box_ws_bytes(*box, 8, p))
    return fail(CTMHD_EARG, "workspace too small");
  if (((uintptr_t)workspace & 255) != 0) return fail(CTMHD_EARG, "workspace must be 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  switch (p->recon) {
    case CTMHD_RECON_PC:
      return record_box<kPC>(p, box, cons, bface, dt, tape, workspace, ws_bytes, st);
    case CTMHD_RECON_PLM_MC:
      return record_box<kPLM_MC>(p, box, cons, bface, dt, tape, workspace, ws_bytes, st);
    case CTMHD_RECON_PLM_MINMOD:
      return record_box<kPLM_MM>(p, box, cons, bface, dt, tape, workspace, ws_bytes, st);
    default:
      return record_box<kPPM>(p, box, cons, bface, dt, tape, workspace, ws_bytes, st);
  }
}

int ctmhd_step_adjoint_tape(const ctmhd_params* p, const ctmhd_box* box, const void* tape,
                            size_t tape_bytes, const double* const g_cons[5],
                            const double* const g_bface[3], double* const g_cons_out[5],
                            double* const g_bface_out[3], void* workspace, size_t ws_bytes,
                            void* stream) {
  g_err[0] = 0;
  int rc = check_params(p);
  if (rc) return rc;
  if ((rc = check_adjoint(p))) return rc;
  if ((rc = check_box(p, box))) return rc;
  if ((rc = check_gradients(g_cons, g_bface, g_cons_out, g_bface_out))) return rc;
  if (!tape || tape_bytes < tape_bytes_of(*box)) return fail(CTMHD_EARG, "tape too small");
  if (((uintptr_t)tape & 255) != 0) return fail(CTMHD_EARG, "tape must be 256-byte aligned");
  if (((uintptr_t)workspace & 255) != 0) return fail(CTMHD_EARG, "workspace must be 256-byte aligned");
  return adjoint_dispatch(p, box, nullptr, nullptr, nullptr, g_cons, g_bface, g_cons_out,
                          g_bface_out, tape, workspace, ws_bytes, (hipStream_t)stream);
}

}  // extern "C"
