// ctmhd.hip -- kernels and C ABI of libctmhd for gfx950 (MI355X).
//
// One RK2-SSP step with first-order flux correction (Sec. 2.5 of Kriel et al.)
// is a short sequence of stream-ordered kernels on a ghosted box:
//   k_dt_final   dt from the CFL maximum of the step's starting state (or the
//                caller's dt); a non-finite dt stops the call
//   per stage:
//   k_faces      reconstruction + Riemann solve at every face of all three
//                directions in one launch: x faces inside a wavefront (cross-
//                lane shuffles), y and z faces by marching along the face
//                normal with a register window, so that every cell is loaded
//                and reconstructed once per direction; primitives are formed
//                on the fly (pressure recovery in FP64)
//   k_emf_march  Q26 edge EMFs of the three edge directions with LD04
//                averaging and eta j, one thread per column of edges marching
//                up z (the z reconstructions streamed through registers)
//   k_emf3       the same for B25a / FS18, one thread per edge position
//   k_update     flux divergence and CT curl, RK combination, periodic ghost
//                images, invalid-state flags and (second stage) the CFL
//                maximum of the new state for the next step
//   k_fo         first-order fluxes / EMFs from S^n around flagged cells
//   k_update     again (fix-up mode), only when something was flagged
// Face arrays hold the x_a face on the lower side of each cell, edge arrays
// the edge at the lower corner in the two transverse directions.
#include "ctmhd_host.h"

thread_local char g_err[256] = "";
void* const* g_prof_events = nullptr;
int g_prof_pairs = 0;
int g_prof_used = 0;

namespace {

// Workgroups of the first-order and fix-up launches, which stride over the
// box: enough to fill the chip when cells are flagged, few enough that the
// usual launch with nothing flagged costs microseconds.
inline int fix_blocks(int ninter) {
  const int nb = nblocks(ninter);
  return nb < 2048 ? nb : 2048;
}

template <typename T>
int launch_fo(hipStream_t st, const ctmhd_params* p, State Sn, const Geom& G, const Work<T>& W,
              int stage, int ninter) {
  const int nb = fix_blocks(ninter);
  if (p->emf_compute == CTMHD_EMF_Q26)
    LAUNCH((k_fo<T, kQ26>), nb, Sn, G, W, stage, p->gamma, p->eta, W.stop);
  else if (p->emf_compute == CTMHD_EMF_B25A)
    LAUNCH((k_fo<T, kB25A>), nb, Sn, G, W, stage, p->gamma, p->eta, W.stop);
  else
    LAUNCH((k_fo<T, kFS18>), nb, Sn, G, W, stage, p->gamma, p->eta, W.stop);
  return CTMHD_OK;
}

// One stage: fluxes and EMFs of `in`, update into `out` from `base` = S^n.
template <typename T, int RECON>
int run_stage(hipStream_t st, const ctmhd_params* p, const Geom& G, const Work<T>& W,
              const FacePlan& FP, State in, State base, State out, int stage, double sres,
              long long* diag) {
  int rc;
  if (p->emf_compute == CTMHD_EMF_B25A) {
    LAUNCH((k_prim<T, kB25A>), nblocks(G.elems), in, G, W, p->gamma, W.stop);
    if constexpr (first_step_stored(kB25A, RECON))
      LAUNCH((k_first_step<T, RECON, kB25A>), nblocks(G.elems), G, W, W.stop);
  } else if (p->emf_compute == CTMHD_EMF_FS18) {
    LAUNCH((k_prim<T, kFS18>), nblocks(G.elems), in, G, W, p->gamma, W.stop);
    if constexpr (first_step_stored(kFS18, RECON))
      LAUNCH((k_first_step<T, RECON, kFS18>), nblocks(G.elems), G, W, W.stop);
  }
  if ((rc = launch_faces<T, RECON>(st, p, in, G, W, FP, stage, diag))) return rc;
  if ((rc = launch_emf<T, RECON>(st, p, in, G, W, stage))) return rc;
  const int ninter = G.n[0] * G.n[1] * G.n[2];
  UpdateCfg U;
  U.fofc = p->fofc;
  U.crit = p->flag_criteria;
  U.gamma = p->gamma;
  U.sres = sres;
  U.force = p->force_flags ? p->force_flags + (size_t)stage * ninter : nullptr;
  U.flag_storage = 0;
  const int band = xcd_band(p, (long long)G.n[0] * G.n[1], ninter);
  LAUNCH(k_update<T>, nblocks(ninter), base, in, out, G, W, stage, 0, U, diag, band, W.stop);
  if (p->fofc) {
    if ((rc = launch_fo<T>(st, p, base, G, W, stage, ninter))) return rc;
    LAUNCH(k_update<T>, fix_blocks(ninter), base, in, out, G, W, stage, 1, U, diag, band, W.stop);
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
  int rc = build_work<T>(p, ws, ws_bytes, *box, W, B, H);
  if (rc) return rc;
  State A;
  for (int m = 0; m < 5; ++m) A.c[m] = cons[m];
  for (int a = 0; a < 3; ++a) A.b[a] = bface[a];
  const State user = A;
  const FacePlan FP = make_face_plan(G, p->recon, p->emf_compute, tile_chunk(p), tile_xrows(p));
  double dxmin = fmin(G.dx[0], fmin(G.dx[1], G.dx[2]));
  double sres = p->eta > 0.0 ? 2.0 * p->eta / (dxmin * dxmin) : 0.0;
  const int ninter = G.n[0] * G.n[1] * G.n[2];
  LAUNCH(k_init, 1, W.stop, W.smax, W.nflag);
  LAUNCH(k_wrap, nblocks(G.elems), A, G, W.stop);
  int dtb = nblocks(ninter);
  if (dtb > 2048) dtb = 2048;
  LAUNCH(k_dt, dtb, A, G, p->gamma, sres, W.smax, W.stop);
  for (int n = 0; n < nsteps; ++n) {
    long long* dg = diag ? (long long*)diag + 4 * n : nullptr;
    LAUNCH(k_dt_final, 1, W.smax, W.nflag, p->cfl, dt_fixed ? dt_fixed + n : nullptr, W.dt,
           dt_out ? dt_out + n : nullptr, W.stop, dg);
    if ((rc = run_stage<T, RECON>(st, p, G, W, FP, A, A, H, 0, sres, dg))) return rc;
    if ((rc = run_stage<T, RECON>(st, p, G, W, FP, H, A, B, 1, sres, dg))) return rc;
    // a stopped step leaves the state where it was: carry it to the next buffer
    // (a capped grid: the launch almost always finds nothing to do)
    LAUNCH(k_copy, fix_blocks(G.elems), B, A, G.elems, W.stop);
    State tmp = A;
    A = B;
    B = tmp;
  }
  if (A.c[0] != user.c[0]) LAUNCH(k_copy, nblocks(G.elems), user, A, G.elems, (const int*)nullptr);
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
  if (p->precision != CTMHD_FP64)
    return step_box_t<float>(p, box, cons, bface, nsteps, dt_fixed, dt_out, diag, workspace,
                             ws_bytes, st);
  return step_box_t<double>(p, box, cons, bface, nsteps, dt_fixed, dt_out, diag, workspace,
                            ws_bytes, st);
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
