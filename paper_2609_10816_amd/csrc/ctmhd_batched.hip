// ctmhd_batched.hip -- many periodic boxes of uneven sizes per call
// (ctmhd_step_batched), and boxes that tile one periodic domain (a level,
// ctmhd_step_level): host-built work plan, per-box constant tables, the ghost
// exchange table of a level and the launch sequence of the batched step.
#include <vector>

#include "ctmhd_host.h"

namespace {

// ---------------------------------------------------------------------------
// Batched boxes (host): plan, workspace and launch sequence.
// ---------------------------------------------------------------------------
long long box_elems_ll(const ctmhd_box& b) {
  long long e = 1;
  for (int d = 0; d < 3; ++d) e *= (long long)(b.n[d] + 2 * b.ng);
  return e;
}
long long box_inter_ll(const ctmhd_box& b) { return (long long)b.n[0] * b.n[1] * b.n[2]; }

// A level: the boxes tile the periodic index domain [0, domain) (origin:
// 3 ints per box, the index of the box's first interior cell).
struct LevelSpec {
  const int32_t* origin;
  int32_t domain[3];
};

// Phase lists: start launch (wrap or exchange, CFL), step launch, copy-back
// launch.  A level fills the ghost layers of every state an update writes by
// an exchange phase (with the flags after a main update when fofc is on, and
// again after a fix-up, which then runs on every box).
int plan_phases(const ctmhd_params* p, bool level, int kind[kMaxPhases], int stage[kMaxPhases],
                int xarg[kMaxPhases], int range[3][2]) {
  int n = 0;
  for (int q = 0; q < kMaxPhases; ++q) xarg[q] = 0;
  range[0][0] = n;
  if (level) {
    kind[n] = PH_XCHG; xarg[n] = XG_CUR; stage[n++] = 0;
  } else {
    kind[n] = PH_WRAP; stage[n++] = 0;
  }
  kind[n] = PH_DT; stage[n++] = 0;
  range[0][1] = n;
  range[1][0] = n;
  for (int st = 0; st < 2; ++st) {
    const int target = st == 0 ? XG_HALF : XG_NEXT;
    if (p->emf_compute != CTMHD_EMF_Q26) {
      kind[n] = PH_P; stage[n++] = st;
    }
    if (first_step_stored(p->emf_compute, p->recon)) {
      kind[n] = PH_FIRST; stage[n++] = st;
    }
    kind[n] = PH_F; stage[n++] = st;
    kind[n] = PH_E; stage[n++] = st;
    kind[n] = PH_U; stage[n++] = st;
    if (level) {
      kind[n] = PH_XCHG; xarg[n] = target | (p->fofc ? XG_FLAGS : 0); stage[n++] = st;
    }
    if (p->fofc) {
      kind[n] = PH_O; stage[n++] = st;
      kind[n] = PH_X; stage[n++] = st;
      if (level) {
        kind[n] = PH_XCHG; xarg[n] = target | XG_IF_FIXUP; stage[n++] = st;
      }
    }
  }
  range[1][1] = n;
  range[2][0] = n;
  kind[n] = PH_COPY; stage[n++] = 0;
  range[2][1] = n;
  return n;
}

size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// Work items of one phase of one box.
long long item_count(int kind, const Geom& G, const FacePlan& FP, long long per, bool level) {
  const long long ninter = (long long)G.n[0] * G.n[1] * G.n[2];
  switch (kind) {
    case PH_F: return FP.total_blocks;
    case PH_E: return ((long long)(G.n[0] + 1) * (G.n[1] + 1) * (G.n[2] + 1) + per - 1) / per;
    case PH_XCHG: return ((long long)G.elems - ninter + per - 1) / per;
    case PH_O:
      if (level) return ((long long)(G.n[0] + 1) * (G.n[1] + 1) * (G.n[2] + 1) + per - 1) / per;
      return (ninter + per - 1) / per;
    case PH_P:
    case PH_FIRST:
    case PH_WRAP:
    case PH_COPY: return ((long long)G.elems + per - 1) / per;
    default: return ((long long)G.n[0] * G.n[1] * G.n[2] + per - 1) / per;
  }
}

// FNV-1a over everything a plan depends on: the kernel refuses a plan whose
// key differs from the one computed for the call's own parameters and boxes.
unsigned long long plan_key(const ctmhd_params* p, const ctmhd_box* boxes, int nbox,
                            const LevelSpec* L) {
  unsigned long long h = 0xcbf29ce484222325ull;
  auto mix = [&h](const void* v, size_t n) {
    const unsigned char* c = (const unsigned char*)v;
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 0x100000001b3ull;
  };
  const int f[8] = {p->recon, p->emf_compute, p->fofc, tile_strips(p), tile_chunk(p),
                   tile_xrows(p), nbox, L ? 1 : 0};
  mix(f, sizeof(f));
  if (L) {
    mix(L->domain, sizeof(L->domain));
    mix(L->origin, sizeof(int32_t) * 3 * (size_t)nbox);
  }
  for (int b = 0; b < nbox; ++b) {
    mix(boxes[b].n, sizeof(boxes[b].n));
    mix(&boxes[b].ng, sizeof(boxes[b].ng));
    mix(boxes[b].dx, sizeof(boxes[b].dx));
    mix(&boxes[b].offset, sizeof(boxes[b].offset));
  }
  return h;
}

size_t plan_layout(int nbox, int nphase, long long nxblk, long long* order_off,
                   long long* prefix_off, long long* desc_off, long long* xbox_off,
                   long long* xblk_off) {
  size_t o = align16(sizeof(PlanHeader));
  *order_off = (long long)o;
  o = align16(o + sizeof(int) * (size_t)nbox);
  *prefix_off = (long long)o;
  o = align16(o + sizeof(int) * (size_t)nphase * (nbox + 1));
  *desc_off = (long long)o;
  o = align16(o + sizeof(BoxDesc) * (size_t)nbox);
  *xbox_off = (long long)o;
  if (nxblk > 0) o = align16(o + sizeof(int) * (size_t)(nbox + 1));
  *xblk_off = (long long)o;
  o += sizeof(XBlock) * (size_t)nxblk;
  return o;
}

int check_boxes(const ctmhd_params* p, const ctmhd_box* boxes, int nbox) {
  if (!boxes || nbox < 1) return fail(CTMHD_EARG, "no boxes");
  for (int b = 0; b < nbox; ++b) {
    int rc = check_box(p, &boxes[b]);
    if (rc) return rc;
    if (boxes[b].offset < 0) return fail(CTMHD_EARG, "negative box offset");
  }
  // boxes must not overlap in the packed arrays
  for (int b = 0; b < nbox; ++b) {
    const long long b0 = boxes[b].offset, b1 = b0 + box_elems_ll(boxes[b]);
    for (int c = b + 1; c < nbox; ++c) {
      const long long c0 = boxes[c].offset, c1 = c0 + box_elems_ll(boxes[c]);
      if (b0 < c1 && c0 < b1) return fail(CTMHD_EARG, "boxes overlap in the packed arrays");
    }
  }
  return CTMHD_OK;
}

// A level: one cell size, boxes inside the domain that cover it exactly once
// (no two overlap, also through the periodic wrap, and their cells add up to
// the domain's).
int check_level(const ctmhd_box* boxes, int nbox, const LevelSpec& L) {
  if (!L.origin) return fail(CTMHD_EARG, "origin is NULL");
  long long dom = 1;
  for (int d = 0; d < 3; ++d) {
    if (L.domain[d] < 1) return fail(CTMHD_EARG, "level domain must be >= 1 per axis");
    dom *= L.domain[d];
  }
  long long cells = 0;
  for (int b = 0; b < nbox; ++b) {
    for (int d = 0; d < 3; ++d) {
      const int o = L.origin[3 * b + d];
      if (o < 0 || o >= L.domain[d]) return fail(CTMHD_EARG, "box origin outside the level domain");
      if (boxes[b].n[d] > L.domain[d]) return fail(CTMHD_EARG, "box larger than the level domain");
      if (boxes[b].dx[d] != boxes[0].dx[d]) return fail(CTMHD_EARG, "boxes of a level must share dx");
    }
    cells += box_inter_ll(boxes[b]);
  }
  if (cells != dom) return fail(CTMHD_EARG, "boxes do not cover the level domain exactly");
  // [o, o + n) on a circle of length D: with 0 <= o < D and n <= D, the
  // images by -D, 0, +D are the only ones that can meet another interval
  auto meet = [](int o1, int n1, int o2, int n2, int D) {
    for (int k = -1; k <= 1; ++k)
      if (o1 < o2 + n2 + k * D && o2 + k * D < o1 + n1) return true;
    return false;
  };
  for (int b = 0; b < nbox; ++b)
    for (int c = b + 1; c < nbox; ++c) {
      bool all = true;
      for (int d = 0; d < 3 && all; ++d)
        all = meet(L.origin[3 * b + d], boxes[b].n[d], L.origin[3 * c + d], boxes[c].n[d],
                   L.domain[d]);
      if (all) return fail(CTMHD_EARG, "boxes of the level overlap");
    }
  return CTMHD_OK;
}

// Exchange table of a level: the ghost region of each box cut into blocks,
// each owned by one box's interior (or one periodic image of it).  xbox[b] is
// the first block of box b; xbox[nbox] the number of blocks.
int level_blocks(const ctmhd_box* boxes, int nbox, const LevelSpec& L, std::vector<XBlock>& blk,
                 std::vector<int>& xbox) {
  blk.clear();
  xbox.assign((size_t)nbox + 1, 0);
  struct Piece { int lo, hi, shift; };
  constexpr int kMaxPieces = 32;  // per axis: images k in [-K, K], K = g / D + 2
  for (int b = 0; b < nbox; ++b) {
    xbox[b] = (int)blk.size();
    const ctmhd_box& B = boxes[b];
    const int g = B.ng;
    long long vol = 0;
    for (int c = 0; c < nbox; ++c) {
      const ctmhd_box& C = boxes[c];
      Piece pc[3][kMaxPieces];
      int np[3] = {0, 0, 0};
      bool any = true;
      for (int d = 0; d < 3 && any; ++d) {
        const int D = L.domain[d];
        const int lo = L.origin[3 * b + d] - g, hi = L.origin[3 * b + d] + B.n[d] + g;
        const int K = g / D + 2;
        if (2 * K + 1 > kMaxPieces) return fail(CTMHD_EARG, "ghost width too large for the level domain");
        for (int k = -K; k <= K; ++k) {
          const int clo = L.origin[3 * c + d] + k * D, chi = clo + C.n[d];
          const int a0 = lo > clo ? lo : clo, a1 = hi < chi ? hi : chi;
          if (a0 < a1) pc[d][np[d]++] = Piece{a0, a1, k};
        }
        any = np[d] > 0;
      }
      if (!any) continue;
      for (int iz = 0; iz < np[2]; ++iz)
        for (int iy = 0; iy < np[1]; ++iy)
          for (int ix = 0; ix < np[0]; ++ix) {
            const Piece& x = pc[0][ix];
            const Piece& y = pc[1][iy];
            const Piece& z = pc[2][iz];
            if (c == b && x.shift == 0 && y.shift == 0 && z.shift == 0) continue;  // the interior
            const Piece* q[3] = {&x, &y, &z};
            int dst0[3], src0[3];
            for (int d = 0; d < 3; ++d) {
              dst0[d] = q[d]->lo - (L.origin[3 * b + d] - g);
              src0[d] = q[d]->lo - (L.origin[3 * c + d] + q[d]->shift * L.domain[d]) + C.ng;
            }
            const int BN0 = B.n[0] + 2 * g, BN1 = B.n[1] + 2 * g;
            const int CN0 = C.n[0] + 2 * C.ng, CN1 = C.n[1] + 2 * C.ng;
            XBlock e;
            e.dst = B.offset + dst0[0] + (long long)BN0 * (dst0[1] + (long long)BN1 * dst0[2]);
            e.src = C.offset + src0[0] + (long long)CN0 * (src0[1] + (long long)CN1 * src0[2]);
            e.dsy = BN0;
            e.dsz = BN0 * BN1;
            e.ssy = CN0;
            e.ssz = CN0 * CN1;
            e.ex = x.hi - x.lo;
            e.ey = y.hi - y.lo;
            e.vol = e.ex * e.ey * (z.hi - z.lo);
            e.vol_lo = (int)vol;
            vol += e.vol;
            blk.push_back(e);
          }
    }
    if (vol != box_elems_ll(B) - box_inter_ll(B))
      return fail(CTMHD_EARG, "the level does not cover a box's ghost region exactly once");
  }
  xbox[nbox] = (int)blk.size();
  return CTMHD_OK;
}

long long packed_elems(const ctmhd_box* boxes, int nbox) {
  long long m = 0;
  for (int b = 0; b < nbox; ++b) {
    long long e = boxes[b].offset + box_elems_ll(boxes[b]);
    m = e > m ? e : m;
  }
  return m;
}

size_t batch_ws_bytes(const ctmhd_params* p, const ctmhd_box* boxes, int nbox) {
  const size_t tb = stencil_bytes(p);
  const size_t e = (size_t)packed_elems(boxes, nbox);
  int kind[kMaxPhases], stage[kMaxPhases], xarg[kMaxPhases], range[3][2];
  const int nphase = plan_phases(p, true, kind, stage, xarg, range);  // the longer list
  size_t bytes = 0;
  bytes += 2 * 8 * align256(e * 8);  // B and H states
  if (p->emf_compute != CTMHD_EMF_Q26) bytes += 3 * align256(e * tb);
  if (first_step_stored(p->emf_compute, p->recon))  // stored first steps
    bytes += (p->emf_compute == CTMHD_EMF_B25A ? 12 : 18) * align256(e * tb);
  bytes += (2 * 15 + 9 + 6) * align256(e * tb);
  bytes += align256(e);                                      // flags (packed positions)
  bytes += align256(sizeof(int) * (size_t)nphase * nbox);    // done
  bytes += align256(sizeof(int) * 4 * (size_t)nbox);         // nflag
  bytes += align256(sizeof(unsigned long long) * 2 * (size_t)nbox);  // CFL slots
  bytes += align256(sizeof(double) * (size_t)nbox);          // dt
  bytes += align256((tb == 4 ? sizeof(BoxTab<float>) : sizeof(BoxTab<double>)) * (size_t)nbox);
  bytes += 256;                                              // cursor, stop, err, loc
  return bytes;
}

template <typename T>
int batch_args(const ctmhd_params* p, const ctmhd_box* boxes, int nbox, void* ws, size_t ws_bytes,
               BatchArgs<T>& A, int& nphase) {
  if (!ws || ws_bytes < batch_ws_bytes(p, boxes, nbox)) return fail(CTMHD_EARG, "workspace too small");
  if (((uintptr_t)ws & 255) != 0) return fail(CTMHD_EARG, "workspace must be 256-byte aligned");
  const size_t e = (size_t)packed_elems(boxes, nbox);
  int kind[kMaxPhases], stage[kMaxPhases], xarg[kMaxPhases], range[3][2];
  nphase = plan_phases(p, true, kind, stage, xarg, range);  // sizes the done counters
  Carve cv{(char*)ws};
  for (int m = 0; m < 5; ++m) A.B.c[m] = cv.take<double>(e);
  for (int a = 0; a < 3; ++a) A.B.b[a] = cv.take<double>(e);
  for (int m = 0; m < 5; ++m) A.H.c[m] = cv.take<double>(e);
  for (int a = 0; a < 3; ++a) A.H.b[a] = cv.take<double>(e);
  Work<T>& W = A.W;
  for (int v = 0; v < 8; ++v) W.prim[v] = nullptr;
  for (int c = 0; c < 3; ++c) W.ecell[c] = nullptr;
  for (int c = 0; c < 3; ++c)
    for (int o = 0; o < 2; ++o) W.b25f[c][o][0] = W.b25f[c][o][1] = nullptr;
  for (int v = 0; v < 3; ++v)
    for (int d = 0; d < 3; ++d) W.fsf[v][d][0] = W.fsf[v][d][1] = nullptr;
  const bool first = first_step_stored(p->emf_compute, p->recon);
  if (p->emf_compute == CTMHD_EMF_B25A) {
    for (int c = 0; c < 3; ++c) W.ecell[c] = cv.take<T>(e);
    if (first)
      for (int c = 0; c < 3; ++c)
        for (int o = 0; o < 2; ++o)
          for (int k = 0; k < 2; ++k) W.b25f[c][o][k] = cv.take<T>(e);
  }
  if (p->emf_compute == CTMHD_EMF_FS18) {
    for (int v = 1; v < 4; ++v) W.prim[v] = cv.take<T>(e);
    if (first)
      for (int v = 0; v < 3; ++v)
        for (int d = 0; d < 3; ++d)
          for (int k = 0; k < 2; ++k) W.fsf[v][d][k] = cv.take<T>(e);
  }
  for (int st = 0; st < 2; ++st)
    for (int a = 0; a < 3; ++a)
      for (int m = 0; m < 5; ++m) W.F[st][a][m] = cv.take<T>(e);
  for (int a = 0; a < 3; ++a) W.ap[a] = cv.take<T>(e);
  for (int a = 0; a < 3; ++a) W.am[a] = cv.take<T>(e);
  for (int a = 0; a < 3; ++a) W.us[a] = cv.take<T>(e);
  for (int st = 0; st < 2; ++st)
    for (int c = 0; c < 3; ++c) W.E[st][c] = cv.take<T>(e);
  W.flag = cv.take<uint8_t>(e);
  A.done = cv.take<int>((size_t)nphase * nbox);
  A.nflag = cv.take<int>(4 * (size_t)nbox);
  A.slots = cv.take<unsigned long long>(2 * (size_t)nbox);
  A.dt = cv.take<double>((size_t)nbox);
  A.tab = (unsigned long long)(uintptr_t)cv.take<BoxTab<T>>((size_t)nbox);
  char* sc = cv.p;
  A.cursor = (int*)sc;          // 4 ints
  A.stop = (int*)(sc + 16);
  A.err = (int*)(sc + 20);
  A.loc = (const int*)(sc + 24);
  W.dt = A.dt;
  W.nflag = A.nflag;
  W.smax = A.slots;
  W.stop = A.stop;
  A.gamma = p->gamma;
  A.eta = p->eta;
  A.fofc = p->fofc;
  A.crit = p->flag_criteria;
  A.level = 0;
  return CTMHD_OK;
}

// Persistent grid: every workgroup that can be resident at once.
// The persistent-queue schedule (k_batch) is not built: a launch of it did
// not finish and the cause has not been found.
constexpr bool kPersistentBuilt = false;

template <typename K>
int persistent_blocks(K kernel) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, 0) != hipSuccess) return 0;
  if (per < 1) per = 1;
  return ncu * per;
}

// Items of every phase summed over the boxes (the grid of each phased launch;
// the same counts as the plan's prefix sums).
int phase_items(const ctmhd_params* p, const ctmhd_box* boxes, int nbox, bool level,
                const int* kind, int nphase, long long* items) {
  const long long per = (long long)kBlock * tile_strips(p);
  for (int q = 0; q < nphase; ++q) items[q] = 0;
  for (int b = 0; b < nbox; ++b) {
    const Geom G = make_geom(boxes[b]);
    const FacePlan FP = make_face_plan(G, p->recon, p->emf_compute, tile_chunk(p), tile_xrows(p));
    for (int q = 0; q < nphase; ++q) items[q] += item_count(kind[q], G, FP, per, level);
  }
  for (int q = 0; q < nphase; ++q)
    if (items[q] >= (1LL << 31)) return fail(CTMHD_EARG, "work queue too long");
  return CTMHD_OK;
}

template <typename T, int RECON, int RIEMANN, int EMF>
int launch_bphase(hipStream_t st, int kind, long long items, const BatchArgs<T>& A, int q) {
  if (items <= 0) return CTMHD_OK;
  const unsigned grid = (unsigned)items;
  switch (kind) {
    case PH_P: LAUNCH((k_bphase<T, kPC, kHLLD, EMF, PH_P>), grid, A, q); break;
    case PH_FIRST: LAUNCH((k_bphase<T, RECON, kHLLD, EMF, PH_FIRST>), grid, A, q); break;
    case PH_F: LAUNCH((k_bphase<T, RECON, RIEMANN, kQ26, PH_F>), grid, A, q); break;
    case PH_E: LAUNCH((k_bphase<T, RECON, kHLLD, EMF, PH_E>), grid, A, q); break;
    case PH_U:
    case PH_X: LAUNCH((k_bphase<T, kPC, kHLLD, kQ26, PH_U>), grid, A, q); break;
    case PH_O: LAUNCH((k_bphase<T, kPC, kHLLD, EMF, PH_O>), grid, A, q); break;
    case PH_WRAP: LAUNCH((k_bphase<T, kPC, kHLLD, kQ26, PH_WRAP>), grid, A, q); break;
    case PH_DT: LAUNCH((k_bphase<T, kPC, kHLLD, kQ26, PH_DT>), grid, A, q); break;
    case PH_XCHG: LAUNCH((k_bphase<T, kPC, kHLLD, kQ26, PH_XCHG>), grid, A, q); break;
    default: LAUNCH((k_bphase<T, kPC, kHLLD, kQ26, PH_COPY>), grid, A, q); break;
  }
  return CTMHD_OK;
}

template <typename T, int RECON, int RIEMANN, int EMF>
int batched_run(const ctmhd_params* p, int nbox, const ctmhd_box* boxes, const LevelSpec* L,
                const void* plan, double* const cons[5], double* const bface[3], int nsteps,
                int dt_mode, const double* dt_fixed, double* dt_out, int64_t* diag, void* ws,
                size_t ws_bytes, hipStream_t st) {
  BatchArgs<T> A;
  int nphase = 0;
  int rc = batch_args<T>(p, boxes, nbox, ws, ws_bytes, A, nphase);
  if (rc) return rc;
  for (int m = 0; m < 5; ++m) A.user.c[m] = cons[m];
  for (int a = 0; a < 3; ++a) A.user.b[a] = bface[a];
  A.plan = (const char*)plan;
  A.key = plan_key(p, boxes, nbox, L);
  A.diag = nullptr;
  A.dt_per_box = dt_mode == CTMHD_DT_PER_BOX;
  A.level = L ? 1 : 0;
  // the persistent-queue schedule is switched off (the entry point refuses
  // it); its kernel is not even instantiated
  constexpr bool persistent = kPersistentBuilt;
  int kind[kMaxPhases], stage[kMaxPhases], xarg[kMaxPhases], range[3][2];
  nphase = plan_phases(p, L != nullptr, kind, stage, xarg, range);
  long long items[kMaxPhases];
  int grid = 0;
  if constexpr (persistent) {
    grid = persistent_blocks(k_batch<T, RECON, RIEMANN, EMF>);
    if (grid < 1) return fail(CTMHD_EHIP, "occupancy query failed");
  } else {
    if ((rc = phase_items(p, boxes, nbox, L != nullptr, kind, nphase, items))) return rc;
  }
  // launch l (0 start, 1 step, 2 copy-back) of either schedule
  auto run_launch = [&](int l) -> int {
    if constexpr (persistent) {
      A.launch = l;
      if (l == 1) prof_begin(st);
      LAUNCH((k_batch<T, RECON, RIEMANN, EMF>), grid, A);
      if (l == 1) prof_end(st);
      return CTMHD_OK;
    }
    for (int q = range[l][0]; q < range[l][1]; ++q) {
      if (kind[q] == PH_F) prof_begin(st);
      int r = launch_bphase<T, RECON, RIEMANN, EMF>(st, kind[q], items[q], A, q);
      if (r) return r;
      if (kind[q] == PH_F) prof_end(st);
    }
    return CTMHD_OK;
  };
  const int ndt = A.dt_per_box ? nbox : 1;
  LAUNCH(k_breset, 1, nbox, nphase, A.done, A.cursor, 1, A.stop, A.err, (int*)A.loc, A.slots,
         A.nflag);
  LAUNCH(k_btab<T>, (nbox + kBlock - 1) / kBlock, A, nbox);
  if ((rc = run_launch(0))) return rc;
  for (int n = 0; n < nsteps; ++n) {
    long long* dg = diag ? (long long*)diag + 4 * n : nullptr;
    LAUNCH(k_bdt_final, 1, nbox, nphase, A.dt_per_box, A.level, A.slots, A.nflag, A.done, A.cursor, p->cfl,
           dt_fixed ? dt_fixed + (size_t)n * ndt : nullptr, A.dt,
           dt_out ? dt_out + (size_t)n * ndt : nullptr, A.stop, A.err, dg);
    A.diag = dg;
    if ((rc = run_launch(1))) return rc;
    LAUNCH(k_bstep_end, 1, (int*)A.loc, A.stop, A.err, dg);
  }
  if (persistent)
    LAUNCH(k_breset, 1, nbox, nphase, A.done, A.cursor, 0, A.stop, A.err, (int*)A.loc, A.slots,
           A.nflag);
  A.diag = nullptr;
  return run_launch(2);
}

template <typename T, int RECON>
int batched_emf(const ctmhd_params* p, int nbox, const ctmhd_box* boxes, const LevelSpec* L,
                const void* plan, double* const cons[5], double* const bface[3], int nsteps,
                int dt_mode, const double* dt_fixed, double* dt_out, int64_t* diag, void* ws,
                size_t ws_bytes, hipStream_t st) {
#define CTMHD_BATCH(RI, EM) \
  batched_run<T, RECON, RI, EM>(p, nbox, boxes, L, plan, cons, bface, nsteps, dt_mode, dt_fixed, dt_out, diag, ws, ws_bytes, st)
  if constexpr (std::is_same<T, float>::value) {
    if (p->precision == CTMHD_FP32_R64) {
      if (p->riemann == CTMHD_RIEMANN_HLLD) {
        if (p->emf_compute == CTMHD_EMF_Q26) return CTMHD_BATCH(kHLLD64, kQ26);
        if (p->emf_compute == CTMHD_EMF_B25A) return CTMHD_BATCH(kHLLD64, kB25A);
        return CTMHD_BATCH(kHLLD64, kFS18);
      }
      if (p->emf_compute == CTMHD_EMF_Q26) return CTMHD_BATCH(kLLF64, kQ26);
      if (p->emf_compute == CTMHD_EMF_B25A) return CTMHD_BATCH(kLLF64, kB25A);
      return CTMHD_BATCH(kLLF64, kFS18);
    }
  }
  if (p->riemann == CTMHD_RIEMANN_HLLD) {
    if (p->emf_compute == CTMHD_EMF_Q26) return CTMHD_BATCH(kHLLD, kQ26);
    if (p->emf_compute == CTMHD_EMF_B25A) return CTMHD_BATCH(kHLLD, kB25A);
    return CTMHD_BATCH(kHLLD, kFS18);
  }
  if (p->emf_compute == CTMHD_EMF_Q26) return CTMHD_BATCH(kLLF, kQ26);
  if (p->emf_compute == CTMHD_EMF_B25A) return CTMHD_BATCH(kLLF, kB25A);
  return CTMHD_BATCH(kLLF, kFS18);
#undef CTMHD_BATCH
}

template <typename T>
int batched_t(const ctmhd_params* p, int nbox, const ctmhd_box* boxes, const LevelSpec* L,
              const void* plan, double* const cons[5], double* const bface[3], int nsteps,
              int dt_mode, const double* dt_fixed, double* dt_out, int64_t* diag, void* ws,
              size_t ws_bytes, hipStream_t st) {
  switch (p->recon) {
    case CTMHD_RECON_PC:
      return batched_emf<T, kPC>(p, nbox, boxes, L, plan, cons, bface, nsteps, dt_mode, dt_fixed, dt_out, diag, ws, ws_bytes, st);
    case CTMHD_RECON_PLM_MC:
      return batched_emf<T, kPLM_MC>(p, nbox, boxes, L, plan, cons, bface, nsteps, dt_mode, dt_fixed, dt_out, diag, ws, ws_bytes, st);
    case CTMHD_RECON_PLM_MINMOD:
      return batched_emf<T, kPLM_MM>(p, nbox, boxes, L, plan, cons, bface, nsteps, dt_mode, dt_fixed, dt_out, diag, ws, ws_bytes, st);
    default:
      return batched_emf<T, kPPM>(p, nbox, boxes, L, plan, cons, bface, nsteps, dt_mode, dt_fixed, dt_out, diag, ws, ws_bytes, st);
  }
}

int build_plan(const ctmhd_params* p, const ctmhd_box* boxes, int nbox, const LevelSpec* L,
               void* host_plan, size_t bytes) {
  g_err[0] = 0;
  int rc = check_params(p);
  if (rc) return rc;
  if ((rc = check_boxes(p, boxes, nbox))) return rc;
  std::vector<XBlock> blk;
  std::vector<int> xbox;
  if (L) {
    if ((rc = check_level(boxes, nbox, *L))) return rc;
    if ((rc = level_blocks(boxes, nbox, *L, blk, xbox))) return rc;
  }
  int kind[kMaxPhases], stage[kMaxPhases], xarg[kMaxPhases], range[3][2];
  const int nphase = plan_phases(p, L != nullptr, kind, stage, xarg, range);
  long long order_off, prefix_off, desc_off, xbox_off, xblk_off;
  const size_t need = plan_layout(nbox, nphase, (long long)blk.size(), &order_off, &prefix_off,
                                  &desc_off, &xbox_off, &xblk_off);
  if (!host_plan || bytes < need) return fail(CTMHD_EARG, "plan buffer too small");
  char* base = (char*)host_plan;
  memset(base, 0, need);
  PlanHeader* P = (PlanHeader*)base;
  int* order = (int*)(base + order_off);
  int* prefix = (int*)(base + prefix_off);
  BoxDesc* desc = (BoxDesc*)(base + desc_off);
  P->nbox = nbox;
  P->nphase = nphase;
  P->strips = tile_strips(p);
  P->magic = kPlanMagic;
  P->key = plan_key(p, boxes, nbox, L);
  for (int q = 0; q < nphase; ++q) {
    P->kind[q] = kind[q];
    P->stage[q] = stage[q];
    P->xarg[q] = xarg[q];
  }
  P->level = L ? 1 : 0;
  P->nxblk = (int)blk.size();
  P->xbox_off = xbox_off;
  P->xblk_off = xblk_off;
  if (L) {
    memcpy(base + xbox_off, xbox.data(), sizeof(int) * xbox.size());
    memcpy(base + xblk_off, blk.data(), sizeof(XBlock) * blk.size());
  }
  for (int l = 0; l < 3; ++l) {
    P->range[l][0] = range[l][0];
    P->range[l][1] = range[l][1];
  }
  P->order_off = order_off;
  P->prefix_off = prefix_off;
  P->desc_off = desc_off;
  // largest boxes first (stable), so that the longest items start early
  for (int b = 0; b < nbox; ++b) order[b] = b;
  for (int i = 1; i < nbox; ++i) {
    int v = order[i], j = i;
    long long ev = box_inter_ll(boxes[v]);
    while (j > 0 && box_inter_ll(boxes[order[j - 1]]) < ev) {
      order[j] = order[j - 1];
      --j;
    }
    order[j] = v;
  }
  const int strips = P->strips;
  const long long per = (long long)kBlock * strips;
  long long flag_off = 0;
  for (int b = 0; b < nbox; ++b) {
    const ctmhd_box& bx = boxes[b];
    BoxDesc& d = desc[b];
    d.G = make_geom(bx);
    d.FP = make_face_plan(d.G, p->recon, p->emf_compute, tile_chunk(p), tile_xrows(p));
    d.off = bx.offset;
    d.flag_off = L ? bx.offset : flag_off;  // a level indexes flags by storage position
    flag_off += box_inter_ll(bx);
    double dxmin = fmin(bx.dx[0], fmin(bx.dx[1], bx.dx[2]));
    d.sres = p->eta > 0.0 ? 2.0 * p->eta / (dxmin * dxmin) : 0.0;
  }
  long long items_in_launch = 0;
  int launch = 0;
  for (int q = 0; q < nphase; ++q) {
    while (launch < 2 && q >= range[launch][1]) {
      P->range_items[launch] = (int)items_in_launch;
      ++launch;
      items_in_launch = 0;
    }
    P->item_off[q] = (int)items_in_launch;
    int* pre = prefix + (long long)q * (nbox + 1);
    pre[0] = 0;
    for (int k = 0; k < nbox; ++k) {
      const BoxDesc& d = desc[order[k]];
      const long long cnt = item_count(kind[q], d.G, d.FP, per, L != nullptr);
      if ((long long)pre[k] + cnt >= (1LL << 31)) return fail(CTMHD_EARG, "work queue too long");
      pre[k + 1] = pre[k] + (int)cnt;
    }
    items_in_launch += pre[nbox];
    if (items_in_launch >= (1LL << 31)) return fail(CTMHD_EARG, "work queue too long");
  }
  P->range_items[launch] = (int)items_in_launch;
  return CTMHD_OK;
}

int step_common(const ctmhd_params* p, int nbox, const ctmhd_box* boxes, const LevelSpec* L,
                const void* plan, double* const cons[5], double* const bface[3], int nsteps,
                int dt_mode, const double* dt_fixed, double* dt_out, int64_t* diag,
                void* workspace, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  int rc = check_params(p);
  if (rc) return rc;
  if ((rc = check_boxes(p, boxes, nbox))) return rc;
  if (L && (rc = check_level(boxes, nbox, *L))) return rc;
  if (p->force_flags) return fail(CTMHD_EARG, "force_flags is a single-box test hook");
  if (!plan) return fail(CTMHD_EARG, "plan is NULL");
  if (!cons || !bface) return fail(CTMHD_EARG, "state pointers are NULL");
  for (int m = 0; m < 5; ++m)
    if (!cons[m]) return fail(CTMHD_EARG, "a cons pointer is NULL");
  for (int a = 0; a < 3; ++a)
    if (!bface[a]) return fail(CTMHD_EARG, "a bface pointer is NULL");
  if (dt_mode != CTMHD_DT_GLOBAL && dt_mode != CTMHD_DT_PER_BOX) return fail(CTMHD_EARG, "unknown dt mode");
  // The persistent-queue schedule is switched off: a launch of it with the
  // per-box constant tables did not finish and the cause is not known.
  if (tile_sched(p) == 1)
    return fail(CTMHD_EUNSUPPORTED, "the persistent batched schedule is disabled (a launch of it did not finish; cause not found)");
  if (nsteps < 0) return fail(CTMHD_EARG, "nsteps must be >= 0");
  if (nsteps == 0) return CTMHD_OK;
  if (packed_elems(boxes, nbox) * 6 >= (1LL << 31) * 64LL) return fail(CTMHD_EARG, "packed arrays too large");
  hipStream_t st = (hipStream_t)stream;
  if (p->precision != CTMHD_FP64)
    return batched_t<float>(p, nbox, boxes, L, plan, cons, bface, nsteps, dt_mode, dt_fixed,
                            dt_out, diag, workspace, ws_bytes, st);
  return batched_t<double>(p, nbox, boxes, L, plan, cons, bface, nsteps, dt_mode, dt_fixed,
                           dt_out, diag, workspace, ws_bytes, st);
}

}  // namespace

extern "C" {

size_t ctmhd_workspace_bytes(const ctmhd_params* p, const ctmhd_box* boxes, int nbox) {
  if (check_params(p) || !boxes || nbox < 1) return 0;
  size_t tb = stencil_bytes(p);
  // one box: enough for either entry point
  if (nbox == 1) {
    const size_t one = box_ws_bytes(boxes[0], tb, p);
    if (check_boxes(p, boxes, 1)) return one;
    const size_t bat = batch_ws_bytes(p, boxes, 1);
    return one > bat ? one : bat;
  }
  if (check_boxes(p, boxes, nbox)) return 0;
  return batch_ws_bytes(p, boxes, nbox);
}

size_t ctmhd_batch_plan_bytes(const ctmhd_params* p, const ctmhd_box* boxes, int nbox) {
  if (check_params(p) || check_boxes(p, boxes, nbox)) return 0;
  int kind[kMaxPhases], stage[kMaxPhases], xarg[kMaxPhases], range[3][2];
  const int nphase = plan_phases(p, false, kind, stage, xarg, range);
  long long a, b, c, d, e;
  return plan_layout(nbox, nphase, 0, &a, &b, &c, &d, &e);
}

int ctmhd_batch_plan(const ctmhd_params* p, const ctmhd_box* boxes, int nbox, void* host_plan,
                     size_t bytes) {
  return build_plan(p, boxes, nbox, nullptr, host_plan, bytes);
}

int ctmhd_step_batched(const ctmhd_params* p, int nbox, const ctmhd_box* boxes, const void* plan,
                       double* const cons[5], double* const bface[3], int nsteps, int dt_mode,
                       const double* dt_fixed, double* dt_out, int64_t* diag, void* workspace,
                       size_t ws_bytes, void* stream) {
  return step_common(p, nbox, boxes, nullptr, plan, cons, bface, nsteps, dt_mode, dt_fixed, dt_out,
                     diag, workspace, ws_bytes, stream);
}

size_t ctmhd_level_plan_bytes(const ctmhd_params* p, const ctmhd_box* boxes, const int32_t* origin,
                              int nbox, const int32_t domain[3]) {
  if (check_params(p) || check_boxes(p, boxes, nbox) || !domain) return 0;
  LevelSpec L{origin, {domain[0], domain[1], domain[2]}};
  std::vector<XBlock> blk;
  std::vector<int> xbox;
  if (check_level(boxes, nbox, L) || level_blocks(boxes, nbox, L, blk, xbox)) return 0;
  int kind[kMaxPhases], stage[kMaxPhases], xarg[kMaxPhases], range[3][2];
  const int nphase = plan_phases(p, true, kind, stage, xarg, range);
  long long a, b, c, d, e;
  return plan_layout(nbox, nphase, (long long)blk.size(), &a, &b, &c, &d, &e);
}

int ctmhd_level_plan(const ctmhd_params* p, const ctmhd_box* boxes, const int32_t* origin, int nbox,
                     const int32_t domain[3], void* host_plan, size_t bytes) {
  g_err[0] = 0;
  if (!domain) return fail(CTMHD_EARG, "domain is NULL");
  LevelSpec L{origin, {domain[0], domain[1], domain[2]}};
  return build_plan(p, boxes, nbox, &L, host_plan, bytes);
}

int ctmhd_step_level(const ctmhd_params* p, int nbox, const ctmhd_box* boxes, const int32_t* origin,
                     const int32_t domain[3], const void* plan, double* const cons[5],
                     double* const bface[3], int nsteps, const double* dt_fixed, double* dt_out,
                     int64_t* diag, void* workspace, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!domain) return fail(CTMHD_EARG, "domain is NULL");
  LevelSpec L{origin, {domain[0], domain[1], domain[2]}};
  return step_common(p, nbox, boxes, &L, plan, cons, bface, nsteps, CTMHD_DT_GLOBAL, dt_fixed,
                     dt_out, diag, workspace, ws_bytes, stream);
}

}  // extern "C"
