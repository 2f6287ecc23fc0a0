// ctmhd_host.h -- host-side helpers of libctmhd shared by its translation
// units: error reporting, argument checks, workspace carving, launches.
#pragma once

#include "ctmhd_device.h"

// one error message per host thread, shared by all entry points
extern thread_local char g_err[256];
// kernel timing hook (ctmhd_profile_events)
extern void* const* g_prof_events;
extern int g_prof_pairs;
extern int g_prof_used;

namespace {

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// Bytes of the stencil type of a precision form: float32 for both FP32 forms.
inline size_t stencil_bytes(const ctmhd_params* p) { return p->precision == CTMHD_FP64 ? 8 : 4; }

int fail(int code, const char* msg) {
  snprintf(g_err, sizeof(g_err), "%s", msg);
  return code;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Tuning knobs in ctmhd_params.tile: bits 0-7 minimum faces per marching
// chunk (default 32), bits 8-15 256-element strips per batched work item
// (default 1), bit 16 batched schedule (0 per phase, 1 persistent), bits
// 19-20 XCD mapping, bits 21-22 Q26 edge kernel, bits 24-30 x-face row
// segments per wavefront (default 4).
int tile_chunk(const ctmhd_params* p) {
  int c = p->tile & 0xff;
  return c > 0 ? c : 32;
}
int tile_strips(const ctmhd_params* p) {
  int s = (p->tile >> 8) & 0xff;
  return s > 0 ? s : 1;
}
// bit 16: batched schedule, 0 one launch per phase, 1 persistent queue
int tile_sched(const ctmhd_params* p) { return (p->tile >> 16) & 1; }
// bits 19-20: XCD mapping of the edge and update passes of the single-box
// call: 0 automatic, 1 each XCD a contiguous range of tiles, 2 all XCDs on
// bands of the same plane
int tile_xcd_map(const ctmhd_params* p) { return (p->tile >> 19) & 3; }
// bits 21-22: Q26 edge kernel of the single-box call: 0 automatic, 1 one
// thread per edge position, 2 z marches (the same values)
int tile_emf(const ctmhd_params* p) { return (p->tile >> 21) & 3; }

// Tiles per XCD and chunk of the banded mapping (0: the contiguous mapping)
// for a pass whose tiles of kBlock positions run over planes of
// `plane_positions` positions.
int xcd_band(const ctmhd_params* p, long long plane_positions, long long total_positions) {
  int m = tile_xcd_map(p);
  // automatic: banded once a plane holds 2^15 positions (measured: +6-9% on
  // the step at 512^3, +2% at 256^3, neutral at 128^3)
  if (m == 0) m = plane_positions >= (1LL << 15) ? 2 : 1;
  if (m == 1) return 0;
  (void)total_positions;
  const long long tiles = (plane_positions + kBlock - 1) / kBlock;
  const long long band = (tiles + kXcds - 1) / kXcds;
  return band < 1 ? 1 : (int)band;
}

// bits 24-30: x-face items (row segments) per wavefront (default 4)
int tile_xrows(const ctmhd_params* p) {
  int x = (p->tile >> 24) & 0x7f;
  return x > 0 ? x : 4;
}

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
  if (p->precision != CTMHD_FP64 && p->precision != CTMHD_FP32 && p->precision != CTMHD_FP32_R64)
    return fail(CTMHD_EARG, "unknown precision");
  if (p->tile < 0 || (p->tile & ~0x7f79ffff) != 0 || ((p->tile >> 19) & 3) == 3 ||
      ((p->tile >> 21) & 3) == 3)
    return fail(CTMHD_EARG, "tile knob out of range");
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

// Workspace of one box for the stencil type of `tbytes` bytes.
size_t box_ws_bytes(const ctmhd_box& b, size_t tbytes, const ctmhd_params* p) {
  const int emf = p->emf_compute;
  size_t e = 1;
  for (int d = 0; d < 3; ++d) e *= (size_t)(b.n[d] + 2 * b.ng);
  size_t ninter = (size_t)b.n[0] * b.n[1] * b.n[2];
  size_t bytes = 0;
  bytes += 2 * 8 * align256(e * 8);           // two state buffers
  if (emf == CTMHD_EMF_B25A) bytes += 3 * align256(e * tbytes);  // cell EMF
  if (first_step_stored(emf, p->recon))     // stored first steps
    bytes += (emf == CTMHD_EMF_B25A ? 12 : 18) * align256(e * tbytes);
  if (emf == CTMHD_EMF_FS18) bytes += 3 * align256(e * tbytes);  // cell velocity
  bytes += 2 * 15 * align256(e * tbytes);     // fluxes, two stages
  bytes += 9 * align256(e * tbytes);          // alpha+, alpha-, u*
  bytes += 6 * align256(e * tbytes);          // EMFs, two stages
  bytes += align256(ninter);                  // flags
  bytes += align256(2 * kMaxSlots * 8) + 256; // CFL slots + scalars
  return bytes;
}

struct Carve {
  char* p;
  template <typename U>
  U* take(size_t n) {
    U* r = (U*)p;
    p += align256(n * sizeof(U));
    return r;
  }
};

template <typename T>
int build_work(const ctmhd_params* prm, void* ws, size_t ws_bytes, const ctmhd_box& b, Work<T>& W,
               State& A2, State& H) {
  size_t need = box_ws_bytes(b, sizeof(T), prm);
  if (!ws || ws_bytes < need) return fail(CTMHD_EARG, "workspace too small");
  if (((uintptr_t)ws & 255) != 0) return fail(CTMHD_EARG, "workspace must be 256-byte aligned");
  size_t e = 1;
  for (int d = 0; d < 3; ++d) e *= (size_t)(b.n[d] + 2 * b.ng);
  size_t ninter = (size_t)b.n[0] * b.n[1] * b.n[2];
  Carve cv{(char*)ws};
  for (int m = 0; m < 5; ++m) A2.c[m] = cv.take<double>(e);
  for (int a = 0; a < 3; ++a) A2.b[a] = cv.take<double>(e);
  for (int m = 0; m < 5; ++m) H.c[m] = cv.take<double>(e);
  for (int a = 0; a < 3; ++a) H.b[a] = cv.take<double>(e);
  for (int v = 0; v < 8; ++v) W.prim[v] = nullptr;
  for (int c = 0; c < 3; ++c) W.ecell[c] = nullptr;
  for (int c = 0; c < 3; ++c)
    for (int o = 0; o < 2; ++o) W.b25f[c][o][0] = W.b25f[c][o][1] = nullptr;
  for (int v = 0; v < 3; ++v)
    for (int d = 0; d < 3; ++d) W.fsf[v][d][0] = W.fsf[v][d][1] = nullptr;
  const bool first = first_step_stored(prm->emf_compute, prm->recon);
  if (prm->emf_compute == CTMHD_EMF_B25A) {
    for (int c = 0; c < 3; ++c) W.ecell[c] = cv.take<T>(e);
    if (first)
      for (int c = 0; c < 3; ++c)
        for (int o = 0; o < 2; ++o)
          for (int k = 0; k < 2; ++k) W.b25f[c][o][k] = cv.take<T>(e);
  }
  if (prm->emf_compute == CTMHD_EMF_FS18) {
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
  W.flag = cv.take<uint8_t>(ninter);
  W.smax = cv.take<unsigned long long>(2 * kMaxSlots);
  char* sc = cv.p;
  W.dt = (double*)sc;
  W.stop = (int*)(sc + 8);
  W.nflag = (int*)(sc + 16);
  return CTMHD_OK;
}


inline void prof_begin(hipStream_t st) {
  if (g_prof_events && g_prof_used < g_prof_pairs)
    (void)hipEventRecord((hipEvent_t)g_prof_events[2 * g_prof_used], st);
}
inline void prof_end(hipStream_t st) {
  if (g_prof_events && g_prof_used < g_prof_pairs) {
    (void)hipEventRecord((hipEvent_t)g_prof_events[2 * g_prof_used + 1], st);
    ++g_prof_used;
  }
}

#define LAUNCH(kern, blocks, ...)                                                  \
  do {                                                                             \
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), 0, st, __VA_ARGS__);      \
    if (hipGetLastError() != hipSuccess) return fail(CTMHD_EHIP, "kernel launch failed: " #kern); \
  } while (0)

// Face plan: ranges and launch shape of the fused face kernel.
FacePlan make_face_plan(const Geom& G, int recon, int emf, int chunk_min, int xrows) {
  FacePlan P;
  const int r = recon_halfwidth(recon);
  const int g = G.g;
  // Q26 reconstructs u* along the transverse axes to the edges, which needs
  // faces r+1 beyond the edge range [g, g+n]; the other schemes only need
  // alpha on the faces next to the edges.
  const int tlo = emf == CTMHD_EMF_Q26 ? g - 1 - r : g - 1;
  P.tlo = tlo;
  for (int d = 0; d < 3; ++d) {
    P.lo[d] = g;
    P.nf[d] = G.n[d] + 1;  // faces g .. g+n read by the update and the edges
    P.tlen[d] = (emf == CTMHD_EMF_Q26 ? g + G.n[d] + r : g + G.n[d]) - tlo + 1;
    P.ulo[d] = g;
    P.ulen[d] = G.n[d];
  }
  // x part
  P.xseg = 64 - 2 * r - 1;
  P.xnseg = (P.nf[0] + P.xseg - 1) / P.xseg;
  P.xwaves = P.xnseg * P.tlen[1] * P.tlen[2];
  P.xrows = xrows;
  const int xwf = (P.xwaves + xrows - 1) / xrows;  // wavefronts of the x part
  P.xblocks = (xwf + kBlock / 64 - 1) / (kBlock / 64);
  // y and z parts: enough chunks along the march for ~8192 waves in flight
  P.total_blocks = P.xblocks;
  for (int A = 1; A <= 2; ++A) {
    const int C = A == 1 ? 2 : 1;
    P.lanes[A] = P.tlen[0] * P.tlen[C];
    P.lblocks[A] = (P.lanes[A] + kBlock - 1) / kBlock;
    int want = (8192 * 64 / kBlock) / (P.lblocks[A] > 0 ? P.lblocks[A] : 1);
    int maxch = (P.nf[A] + chunk_min - 1) / chunk_min;  // chunk >= chunk_min faces (warm-up 2r+1)
    if (want > maxch) want = maxch;
    if (want < 1) want = 1;
    P.chunk[A] = (P.nf[A] + want - 1) / want;
    P.nchunk[A] = (P.nf[A] + P.chunk[A] - 1) / P.chunk[A];
    P.blocks[A] = P.lblocks[A] * P.nchunk[A];
    P.total_blocks += P.blocks[A];
  }
  P.chunk[0] = P.nchunk[0] = P.lanes[0] = P.lblocks[0] = P.blocks[0] = 0;
  return P;
}

template <typename T, int RECON>
int launch_faces(hipStream_t st, const ctmhd_params* p, State S, const Geom& G, const Work<T>& W,
                 const FacePlan& FP, int stage, long long* diag) {
  prof_begin(st);
  if constexpr (std::is_same<T, float>::value) {
    if (p->precision == CTMHD_FP32_R64) {
      if (p->riemann == CTMHD_RIEMANN_HLLD)
        LAUNCH((k_faces<T, RECON, kHLLD64>), FP.total_blocks, S, G, W, FP, stage, p->gamma, p->eta,
               diag, W.stop);
      else
        LAUNCH((k_faces<T, RECON, kLLF64>), FP.total_blocks, S, G, W, FP, stage, p->gamma, p->eta,
               diag, W.stop);
      prof_end(st);
      return CTMHD_OK;
    }
  }
  if (p->riemann == CTMHD_RIEMANN_HLLD)
    LAUNCH((k_faces<T, RECON, kHLLD>), FP.total_blocks, S, G, W, FP, stage, p->gamma, p->eta, diag,
           W.stop);
  else
    LAUNCH((k_faces<T, RECON, kLLF>), FP.total_blocks, S, G, W, FP, stage, p->gamma, p->eta, diag,
           W.stop);
  prof_end(st);
  return CTMHD_OK;
}

// Q26 edge pass: the number of workgroups aimed at (many times the number
// that run at once, so that the last, partial round of these equally long
// marches is a small part of the launch) and the shortest z chunk
constexpr int kEmfTiles = 32768;
constexpr int kEmfMinChunk = 8;

// Workgroups of the z-marching edge kernel that the device holds at once (0 if
// the runtime cannot say).  Queried once per instantiation.
template <typename T, int RECON>
int emf_march_resident() {
  static const int n = [] {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_emf_march<T, RECON>, kBlock, 0) !=
        hipSuccess)
      return 0;
    return ncu * per;
  }();
  return n;
}

template <typename T, int RECON>
int launch_emf(hipStream_t st, const ctmhd_params* p, State S, const Geom& G, const Work<T>& W,
               int stage) {
  const int cnt = (G.n[0] + 1) * (G.n[1] + 1) * (G.n[2] + 1);
  const int band = xcd_band(p, (long long)(G.n[0] + 1) * (G.n[1] + 1), cnt);
  if (p->emf_compute == CTMHD_EMF_Q26) {
    // z marches: enough chunks for about kEmfTiles workgroups, at least
    // kEmfMinChunk positions each (the pipelines take 2r + 1 pushes to fill)
    const int ctiles = nblocks((G.n[0] + 1) * (G.n[1] + 1));
    const int L2 = G.n[2] + 1;
    int nch = (kEmfTiles + ctiles - 1) / ctiles;
    if (nch > L2 / kEmfMinChunk) nch = L2 / kEmfMinChunk;
    if (nch < 1) nch = 1;
    const int zc = (L2 + nch - 1) / nch;
    nch = (L2 + zc - 1) / zc;
    // automatic: a small box gives the marches less than about one round of
    // the chip, where the per-edge kernel's many short workgroups fill it
    // better (the two give the same values)
    const int m = tile_emf(p);
    if (m == 2 || (m == 0 && 4LL * ctiles * nch >= 3LL * emf_march_resident<T, RECON>()))
      LAUNCH((k_emf_march<T, RECON>), ctiles * nch, S, G, W, stage, p->eta, ctiles, zc, W.stop);
    else
      LAUNCH((k_emf3<T, RECON, kQ26>), nblocks(cnt), S, G, W, stage, p->eta, band, W.stop);
  } else if (p->emf_compute == CTMHD_EMF_B25A)
    LAUNCH((k_emf3<T, RECON, kB25A>), nblocks(cnt), S, G, W, stage, p->eta, band, W.stop);
  else
    LAUNCH((k_emf3<T, RECON, kFS18>), nblocks(cnt), S, G, W, stage, p->eta, band, W.stop);
  return CTMHD_OK;
}

}  // namespace
