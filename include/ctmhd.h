/* ctmhd.h -- C ABI of libctmhd: one second-order constrained-transport MHD
 * time step on periodic Cartesian boxes, on an AMD Instinct MI355X (gfx950).
 *
 * The method is that of Kriel et al., "Magnetising the Quokka code with fast,
 * second-order accurate, error-correcting schemes for MHD on GPUs":
 *   - state: cell-centred (rho, rho u, e_tot) and the face-centred normal
 *     magnetic field (Sec. 2.1, eq. state:conserved);
 *   - fluxes: PC / PLM / PPM reconstruction of the primitives and the HLLD
 *     Riemann solver with an HLL fallback, or LLF (Sec. 2.2);
 *   - edge EMFs: the Q26 scheme (eqs. emf:q26-facevel, emf:q26) or the B25a /
 *     FS18 schemes (eqs. emf:b25a-*, emf:fs18*), combined by LD04 averaging
 *     (eq. emf:ld04) with edge wavespeeds (eq. emf:alpha-edge);
 *   - constant Ohmic resistivity: eta j added to the EMF and the Joule energy
 *     flux (Sec. 2.4, eqs. resistivity:*);
 *   - RK2-SSP with first-order flux correction (Sec. 2.5, eqs.
 *     rk:increment-state, rk:increment-bfield, rk1:update, rk2:update).
 *
 * Data layout (every array is caller-owned DEVICE memory, float64):
 *   A box has n[3] interior cells and ng ghost layers on every side; each of
 *   the 8 fields is a contiguous (n2+2ng)(n1+2ng)(n0+2ng) array with x0
 *   fastest.  Cell fields: rho, m0, m1, m2, e_tot.  Face field b_a[i,j,k] is
 *   the x_a-face on the LOWER side of cell (i,j,k).  Boundaries are periodic;
 *   ghost layers are library scratch and hold the periodic copy on return.
 *
 * Streams and ownership: every call is enqueued on `stream` (a hipStream_t,
 * NULL for the default stream) and returns without synchronising.  The
 * library allocates and frees nothing: all scratch lives in the caller's
 * `workspace` of at least ctmhd_workspace_bytes() bytes (256-byte aligned).
 * dt values and diagnostic counters stay on the device.
 *
 * Errors: calls return CTMHD_OK (0) or a negative code; ctmhd_last_error()
 * gives a static description of the last failure on the calling thread.
 * Numerical faults are reported asynchronously through `diag`.
 */
#ifndef CTMHD_H_
#define CTMHD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* reconstruction (Sec. 2.2) */
#define CTMHD_RECON_PC 0
#define CTMHD_RECON_PLM_MC 1
#define CTMHD_RECON_PLM_MINMOD 2
#define CTMHD_RECON_PPM 3
/* Riemann solver (Sec. 2.2) */
#define CTMHD_RIEMANN_HLLD 0
#define CTMHD_RIEMANN_LLF 1
/* EMF compute scheme (Sec. 2.3.1) */
#define CTMHD_EMF_Q26 0
#define CTMHD_EMF_B25A 1
#define CTMHD_EMF_FS18 2
/* EMF averaging scheme (Sec. 2.3.2) */
#define CTMHD_AVG_LD04 0
/* invalid-state criteria for first-order flux correction (Sec. 2.5) */
#define CTMHD_FLAG_RHO 1       /* rho <= 0 */
#define CTMHD_FLAG_P 2         /* p <= 0 */
#define CTMHD_FLAG_NONFINITE 4 /* any non-finite value */
/* arithmetic form */
#define CTMHD_FP64 0           /* everything in float64 */
#define CTMHD_FP32 1           /* stencil in float32; pressure recovery, dt and
                                  the state / face-b accumulation in float64 */
#define CTMHD_FP32_R64 2       /* as CTMHD_FP32, with the Riemann solve in float64
                                  (from the float32 face states); its fluxes,
                                  wavespeeds and u* are stored in float32 */
/* dt mode of the batched call */
#define CTMHD_DT_GLOBAL 0
#define CTMHD_DT_PER_BOX 1

/* status codes */
#define CTMHD_OK 0
#define CTMHD_EARG (-1)        /* bad argument (sizes, ghosts, CFL, pointers) */
#define CTMHD_EUNSUPPORTED (-2)/* scheme combination not built */
#define CTMHD_EHIP (-3)        /* a HIP launch or runtime call failed */

typedef struct ctmhd_params {
  double gamma;          /* adiabatic index, > 1 */
  double eta;            /* constant Ohmic resistivity, >= 0 */
  double cfl;            /* CFL number in (0, 1); < 1/3 when eta > 0 (eq. resistivity:cfl) */
  int32_t recon;         /* CTMHD_RECON_* */
  int32_t riemann;       /* CTMHD_RIEMANN_* */
  int32_t emf_compute;   /* CTMHD_EMF_* */
  int32_t emf_average;   /* CTMHD_AVG_LD04 */
  int32_t fofc;          /* 1: first-order flux correction on, 0: off */
  int32_t flag_criteria; /* OR of CTMHD_FLAG_* */
  int32_t precision;     /* CTMHD_FP64, CTMHD_FP32 or CTMHD_FP32_R64 */
  int32_t tile;          /* launch-shape knob (0 = defaults): bits 0-7 minimum faces per
                            marching chunk of the face pass (default 32), bits 8-15
                            256-element strips per work item of the batched call (default 1),
                            bit 16 schedule of the batched call (0 one launch per phase,
                            1 one persistent launch per step), bits 19-20 XCD mapping of
                            the per-position edge and update passes of ctmhd_step (the
                            z-marching edge pass maps its own tiles; 0 automatic, 1 each
                            XCD a contiguous range of tiles, 2 all XCDs on bands of one
                            plane), bits 21-22 Q26 edge kernel of ctmhd_step (0 automatic,
                            1 one thread per edge position, 2 one thread per column of
                            edges marching along z; the same values), bits 24-30 x-face row
                            segments per wavefront of the face pass (default 4); other
                            values are rejected with CTMHD_EARG */
  /* Test hook: NULL, or a DEVICE mask of 2 * n0*n1*n2 bytes (stage-1 mask then
   * stage-2 mask, interior cells, x0 fastest) OR-ed into the invalid-cell
   * flags of every step.  Single-box call only. */
  const uint8_t* force_flags;
} ctmhd_params;

typedef struct ctmhd_box {
  int32_t n[3];    /* interior cells per axis, >= 1 */
  int32_t ng;      /* ghost layers, >= ctmhd_required_ghosts() */
  double dx[3];    /* cell widths, > 0 */
  int64_t offset;  /* element offset of this box in the packed arrays (batched call) */
} ctmhd_box;

/* Ghost layers the scheme needs: reconstruction half-width + 2 (PC 2, PLM 3,
 * PPM 4).  Sec. 2.3.1 (last paragraph): the edge EMFs reconstruct face
 * quantities along the transverse axes, so the Riemann problem is solved in
 * ghost zones next to the box too, and those faces' reconstructions reach
 * further out.  Returns a negative code for bad parameters. */
int ctmhd_required_ghosts(const ctmhd_params* p);

/* Elements (not bytes) of one field array of a box: prod(n_d + 2 ng). */
int64_t ctmhd_box_elems(const ctmhd_box* box);

/* Workspace bytes (device memory, 256-byte aligned, owned by the caller) for
 * ctmhd_step or ctmhd_step_batched on these boxes; with nbox = 1 the size
 * serves either entry point.  0 for bad arguments. */
size_t ctmhd_workspace_bytes(const ctmhd_params* p, const ctmhd_box* boxes, int nbox);

/* Advance one box by `nsteps` RK2 steps (Sec. 2.5).
 *   cons[5]  : host array of 5 device pointers (rho, m0, m1, m2, e_tot), in/out
 *   bface[3] : host array of 3 device pointers (b0, b1, b2), in/out
 *   dt_fixed : device, nsteps values used as dt, or NULL for the CFL dt
 *              computed from each step's starting state (eq. resistivity:cfl)
 *   dt_out   : device, nsteps values written, or NULL
 *   diag     : device, 4*nsteps int64 written per step: [cells flagged in
 *              stage 1, cells flagged in stage 2, HLL fallbacks, non-finite
 *              dt (1: the step and all later steps were skipped)], or NULL
 * The discrete divergence of the face field is preserved to round-off. */
int ctmhd_step(const ctmhd_params* p, const ctmhd_box* box, double* const cons[5],
               double* const bface[3], int nsteps, const double* dt_fixed, double* dt_out,
               int64_t* diag, void* workspace, size_t ws_bytes, void* stream);

/* Batched boxes (the AMR-like form): plan of the work queue.  The plan is
 * built on the host into a caller buffer of ctmhd_batch_plan_bytes() bytes
 * (boxes: HOST array) and must be copied by the caller into device memory
 * before ctmhd_step_batched; it depends on params (scheme, tile knob, fofc)
 * and on the boxes only, so one upload serves every later call. */
size_t ctmhd_batch_plan_bytes(const ctmhd_params* p, const ctmhd_box* boxes, int nbox);
int ctmhd_batch_plan(const ctmhd_params* p, const ctmhd_box* boxes, int nbox, void* host_plan,
                     size_t bytes);

/* Advance `nbox` independent periodic boxes of different sizes by `nsteps`
 * steps.  The work of a step is a list of (phase, box, tile) items in
 * phase-major order, described by the plan.  Two schedules (tile bit 16),
 * with bitwise the same result:
 *   0: one launch per phase over all boxes, workgroup r runs item r; the
 *      launch boundaries order the phases (about 10-14 launches per step);
 *   1: one persistent launch per step whose workgroups claim items from a
 *      device queue; an item waits (acquire) only for the previous phase of
 *      its own box, and publishes its results (release) at agent scope.
 *      Currently DISABLED: returns CTMHD_EUNSUPPORTED (a launch of it did not
 *      finish; the cause has not been found).
 * Box b's 8 fields start at element
 * boxes[b].offset of the packed arrays cons[m] / bface[a] and are laid out as
 * in ctmhd_step (its own ghost layers; each box is periodic on itself);
 * boxes must not overlap.  `boxes` is the HOST array the plan was made from,
 * `plan` its DEVICE copy.  dt_mode CTMHD_DT_GLOBAL: one dt = CFL / (maximum
 * signal speed over all boxes); CTMHD_DT_PER_BOX: each box its own CFL dt.
 * dt_fixed / dt_out hold nsteps values (global) or nsteps*nbox (per box,
 * step-major).  diag as in ctmhd_step, summed over boxes; diag[3] |= 2
 * reports an internal dependency-wait timeout, diag[3] |= 4 a plan that was
 * not built for these params and boxes (the plan carries a hash of them; the
 * kernels then leave the state untouched).  The call enqueues kernels
 * only (no host-device copies), so multi-step sequences can be captured in a
 * hipGraph.  force_flags must be NULL here. */
int ctmhd_step_batched(const ctmhd_params* p, int nbox, const ctmhd_box* boxes, const void* plan,
                       double* const cons[5], double* const bface[3], int nsteps, int dt_mode,
                       const double* dt_fixed, double* dt_out, int64_t* diag, void* workspace,
                       size_t ws_bytes, void* stream);

/* One level of boxes (Sec. 2.6: the cell-centred update couples boxes only
 * through their ghost zones).  The boxes tile the periodic index domain
 * [0, domain[0]) x [0, domain[1]) x [0, domain[2]) exactly once: box b's
 * first interior cell has level index origin[3b .. 3b+2] (0 <= origin <
 * domain), its cells run over n[d] indices from there (wrapping at the domain
 * end), all boxes share dx, and no two boxes overlap, also through the wrap.
 * The ghost layers of every box are filled from the interiors of the boxes
 * that own those cells, at the start of a call and after every update, so
 * that a level advances exactly as one periodic box of the domain size would
 * (bitwise: every face and edge on a box boundary is computed by both boxes
 * from the same values).  Face b_a at the lower face of a box's first cell
 * belongs to that box; its upper boundary face belongs to the next box.
 * With fofc on, the invalid-cell flags of the neighbouring boxes are
 * exchanged too, and a first-order fix-up, when any cell of the level is
 * flagged, runs on every box (as on one box).  Plan: built on the host
 * (boxes, origin, domain: HOST arrays) into a buffer of
 * ctmhd_level_plan_bytes() bytes (0 for bad arguments or a level that does
 * not tile its domain) and copied by the caller to device memory; it also
 * holds the ghost exchange table (one rectangular block per pair of box and
 * owning box image).  Workspace: ctmhd_workspace_bytes() of the same boxes.
 * ctmhd_step_level: as ctmhd_step_batched with dt_mode CTMHD_DT_GLOBAL (a
 * level has one dt); the packed layout, dt_fixed, dt_out, diag and the
 * errors are those of the batched call, and a level that does not tile its
 * domain returns CTMHD_EARG. */
size_t ctmhd_level_plan_bytes(const ctmhd_params* p, const ctmhd_box* boxes, const int32_t* origin,
                              int nbox, const int32_t domain[3]);
int ctmhd_level_plan(const ctmhd_params* p, const ctmhd_box* boxes, const int32_t* origin, int nbox,
                     const int32_t domain[3], void* host_plan, size_t bytes);
int ctmhd_step_level(const ctmhd_params* p, int nbox, const ctmhd_box* boxes, const int32_t* origin,
                     const int32_t domain[3], const void* plan, double* const cons[5],
                     double* const bface[3], int nsteps, const double* dt_fixed, double* dt_out,
                     int64_t* diag, void* workspace, size_t ws_bytes, void* stream);

/* Workspace bytes for ctmhd_step_adjoint on this machine (0 for bad arguments or
 * an unsupported configuration). */
size_t ctmhd_adjoint_workspace_bytes(const ctmhd_params* p, const ctmhd_box* box);

/* Reverse-mode derivative (vector-Jacobian product) of ONE step of
 * ctmhd_step (Sec. 2.5: RK2-SSP, eqs. rk1:update and rk2:update) with a
 * frozen dt and no flux correction taken (params->fofc is ignored):
 *   cons_n, bface_n : device, the box's state S^n in the ctmhd_step layout
 *                     (ghosts need not be filled)
 *   dt              : device, one double, the dt of the step (> 0, finite)
 *   g_cons, g_bface : device, dL/dS^{n+1} (interior values; ghosts ignored)
 *   g_cons_out, g_bface_out : device, written with dL/dS^n (interior; ghosts
 *                     zeroed); may not alias the inputs
 *   workspace       : device, >= ctmhd_adjoint_workspace_bytes(), 256-byte
 *                     aligned, caller-owned
 * The derivative is taken on the branches the forward step takes at S^n
 * (limiter cases, Riemann-fan regions, min / max selections).  Built for the
 * FP64 form with PC, PLM (MC or minmod) or PPM reconstruction, HLLD or LLF,
 * Q26, B25a or FS18 corner EMFs and LD04, eta >= 0; the FP32 form returns
 * CTMHD_EUNSUPPORTED.  A non-finite dt writes NaN.  Deterministic except for
 * the Ohmic terms (eta > 0), whose face-field adjoints are accumulated with
 * atomics.  The call recomputes the step's first stage; a step recorded by
 * ctmhd_step_record is reversed without that by ctmhd_step_adjoint_tape. */
int ctmhd_step_adjoint(const ctmhd_params* p, const ctmhd_box* box,
                       const double* const cons_n[5], const double* const bface_n[3],
                       const double* dt, const double* const g_cons[5],
                       const double* const g_bface[3], double* const g_cons_out[5],
                       double* const g_bface_out[3], void* workspace, size_t ws_bytes,
                       void* stream);

/* Recorded steps for the adjoint (reverse-mode derivative of eqs. rk1:update
 * and rk2:update, as ctmhd_step_adjoint) without recomputing the first
 * stage.  ctmhd_step_record advances the box by ONE step exactly as
 * ctmhd_step with nsteps = 1, dt_fixed = dt and fofc off (bitwise the same
 * S^{n+1}), and writes its tape: S^n and the first-stage state S1 with their
 * ghost layers, the face arrays (alpha+, alpha-, u*) of both stages and dt.
 * ctmhd_step_adjoint_tape then gives dL/dS^n from dL/dS^{n+1} as
 * ctmhd_step_adjoint on S^n would (bitwise the same result), reading that
 * tape instead of recomputing it.
 *   tape       : device, >= ctmhd_tape_bytes() bytes, 256-byte aligned,
 *                caller-owned; one per recorded step that is to be reversed
 *   dt         : device, one double (> 0, finite; a non-finite dt leaves the
 *                state unchanged and makes the adjoint write NaN), or NULL
 *                for the CFL dt of S^n (eq. resistivity:cfl); the tape holds
 *                the dt used, as the double at byte offset
 *                ctmhd_tape_bytes() - 256
 *   workspace  : ctmhd_step_record: >= ctmhd_workspace_bytes(p, box, 1);
 *                ctmhd_step_adjoint_tape: >= ctmhd_adjoint_workspace_bytes()
 * Configurations as ctmhd_step_adjoint (FP64 form; any reconstruction,
 * Riemann solver and EMF scheme); others return CTMHD_EUNSUPPORTED, and
 * ctmhd_tape_bytes returns 0 for them. */
size_t ctmhd_tape_bytes(const ctmhd_params* p, const ctmhd_box* box);
int ctmhd_step_record(const ctmhd_params* p, const ctmhd_box* box, double* const cons[5],
                      double* const bface[3], const double* dt, void* tape, size_t tape_bytes,
                      void* workspace, size_t ws_bytes, void* stream);
int ctmhd_step_adjoint_tape(const ctmhd_params* p, const ctmhd_box* box, const void* tape,
                            size_t tape_bytes, const double* const g_cons[5],
                            const double* const g_bface[3], double* const g_cons_out[5],
                            double* const g_bface_out[3], void* workspace, size_t ws_bytes,
                            void* stream);

/* ctmhd_step without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Arguments, layout, ownership, result and errors
 * are those of ctmhd_step; the workspace is a fixed array of
 * ctmhd_noalloc_scratch_bytes() (256 MiB) in the library's device memory,
 * one per GPU, held from the first call on that GPU until the process ends.
 * The call allocates and frees nothing.  A box whose
 * ctmhd_workspace_bytes(p, box, 1) exceeds that size is rejected with
 * CTMHD_EARG (in FP64 with PPM: up to 73^3 interior cells with Q26, 66^3 with
 * FS18).  Every call on one GPU uses the same array: calls that overlap on
 * one GPU (other host threads, or streams not ordered with each other) race
 * and give wrong results; calls ordered on one stream are safe. */
size_t ctmhd_noalloc_scratch_bytes(void);
int ctmhd_step_noalloc(const ctmhd_params* p, const ctmhd_box* box, double* const cons[5],
                       double* const bface[3], int nsteps, const double* dt_fixed,
                       double* dt_out, int64_t* diag, void* stream);

/* Kernel timing hook (for benchmarks).  `events` holds 2*npairs hipEvent_t
 * handles created by the caller (timing enabled).  During subsequent
 * ctmhd_step calls in this process the library records pair i
 * (events[2i] before, events[2i+1] after) around the i-th launch of its face
 * kernel (reconstruction + Riemann solve, the dominant kernel), for
 * i < npairs.  ctmhd_profile_recorded() returns the pairs recorded so far.
 * npairs = 0 (or events = NULL) switches the hook off.  Not thread-safe. */
int ctmhd_profile_events(void* const* events, int npairs);
int ctmhd_profile_recorded(void);

/* Static description of the last error on this thread ("" if none). */
const char* ctmhd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CTMHD_H_ */
