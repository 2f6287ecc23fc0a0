/* A plain C caller of libctmhd (no Python, no torch): device memory from the
 * HIP runtime, one ctmhd_step call of 5 steps on a 16 x 12 x 8 box, checks
 * on the host.
 *   1. A uniform moving state is a fixed point of the step, bitwise.
 *   2. A density wave advected by a uniform flow through a uniform field:
 *      total mass and energy are conserved to round-off.
 * Exit status 0 = pass.  Built and run by tests/test_c_abi.py. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ctmhd.h"

#define N0 16
#define N1 12
#define N2 8
#define NSTEPS 5
static const double kPi = 3.14159265358979323846;

static int check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return 1;
  }
  return 0;
}

/* Fill the interior of 8 host arrays of the ghosted box. */
static void fill(double* f[8], int ng, int wave) {
  const double gamma = 5.0 / 3.0, u[3] = {0.3, -0.2, 0.1}, b[3] = {1.0, 0.5, 0.25};
  const int S0 = N0 + 2 * ng, S1 = N1 + 2 * ng;
  for (int k = 0; k < N2; ++k)
    for (int j = 0; j < N1; ++j)
      for (int i = 0; i < N0; ++i) {
        const long s = (i + ng) + (long)S0 * ((j + ng) + (long)S1 * (k + ng));
        const double rho = 1.0 + (wave ? 0.2 * sin(2.0 * kPi * (i + 0.5) / N0) : 0.0);
        const double p = 0.6;
        f[0][s] = rho;
        for (int d = 0; d < 3; ++d) f[1 + d][s] = rho * u[d];
        f[4][s] = p / (gamma - 1.0) + 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) +
                  0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
        for (int a = 0; a < 3; ++a) f[5 + a][s] = b[a];
      }
}

static double interior_sum(const double* f, int ng) {
  const int S0 = N0 + 2 * ng, S1 = N1 + 2 * ng;
  double t = 0.0;
  for (int k = 0; k < N2; ++k)
    for (int j = 0; j < N1; ++j)
      for (int i = 0; i < N0; ++i) t += f[(i + ng) + (long)S0 * ((j + ng) + (long)S1 * (k + ng))];
  return t;
}

int main(void) {
  ctmhd_params p;
  memset(&p, 0, sizeof(p));
  p.gamma = 5.0 / 3.0;
  p.eta = 0.0;
  p.cfl = 0.3;
  p.recon = CTMHD_RECON_PLM_MC;
  p.riemann = CTMHD_RIEMANN_HLLD;
  p.emf_compute = CTMHD_EMF_Q26;
  p.emf_average = CTMHD_AVG_LD04;
  p.fofc = 1;
  p.flag_criteria = CTMHD_FLAG_RHO | CTMHD_FLAG_P | CTMHD_FLAG_NONFINITE;
  p.precision = CTMHD_FP64;
  p.tile = 0;
  p.force_flags = NULL;
  const int ng = ctmhd_required_ghosts(&p);
  if (ng < 0) {
    fprintf(stderr, "required_ghosts: %s\n", ctmhd_last_error());
    return 1;
  }
  ctmhd_box box;
  memset(&box, 0, sizeof(box));
  box.n[0] = N0;
  box.n[1] = N1;
  box.n[2] = N2;
  box.ng = ng;
  box.dx[0] = box.dx[1] = box.dx[2] = 1.0 / N0;
  box.offset = 0;
  const int64_t e = ctmhd_box_elems(&box);
  const size_t ws_bytes = ctmhd_workspace_bytes(&p, &box, 1);
  if (ws_bytes == 0) {
    fprintf(stderr, "workspace_bytes: %s\n", ctmhd_last_error());
    return 1;
  }
  double* host[8];
  double* dev[8];
  void* ws = NULL;
  double* dt_out = NULL;
  int64_t* diag = NULL;
  for (int v = 0; v < 8; ++v) {
    host[v] = (double*)calloc((size_t)e, sizeof(double));
    if (check_hip(hipMalloc((void**)&dev[v], (size_t)e * sizeof(double)), "hipMalloc")) return 1;
  }
  if (check_hip(hipMalloc(&ws, ws_bytes), "hipMalloc workspace") ||
      check_hip(hipMalloc((void**)&dt_out, NSTEPS * sizeof(double)), "hipMalloc dt") ||
      check_hip(hipMalloc((void**)&diag, 4 * NSTEPS * sizeof(int64_t)), "hipMalloc diag"))
    return 1;
  int fail = 0;
  for (int wave = 0; wave < 2; ++wave) {
    fill(host, ng, wave);
    double before[8];
    for (int v = 0; v < 8; ++v) {
      before[v] = interior_sum(host[v], ng);
      if (check_hip(hipMemcpy(dev[v], host[v], (size_t)e * sizeof(double), hipMemcpyHostToDevice),
                    "hipMemcpy"))
        return 1;
    }
    double* const cons[5] = {dev[0], dev[1], dev[2], dev[3], dev[4]};
    double* const bface[3] = {dev[5], dev[6], dev[7]};
    const int rc = ctmhd_step(&p, &box, cons, bface, NSTEPS, NULL, dt_out, diag, ws, ws_bytes, NULL);
    if (rc != CTMHD_OK) {
      fprintf(stderr, "ctmhd_step: %d %s\n", rc, ctmhd_last_error());
      return 1;
    }
    if (check_hip(hipDeviceSynchronize(), "synchronize")) return 1;
    double* out = (double*)malloc((size_t)e * sizeof(double));
    double dts[NSTEPS];
    int64_t dg[4 * NSTEPS];
    if (check_hip(hipMemcpy(dts, dt_out, sizeof(dts), hipMemcpyDeviceToHost), "hipMemcpy dt") ||
        check_hip(hipMemcpy(dg, diag, sizeof(dg), hipMemcpyDeviceToHost), "hipMemcpy diag"))
      return 1;
    for (int v = 0; v < 8; ++v) {
      if (check_hip(hipMemcpy(out, dev[v], (size_t)e * sizeof(double), hipMemcpyDeviceToHost),
                    "hipMemcpy back"))
        return 1;
      const double after = interior_sum(out, ng);
      if (wave == 0) {
        /* bitwise fixed point on the interior */
        const int S0 = N0 + 2 * ng, S1 = N1 + 2 * ng;
        for (int k = 0; k < N2; ++k)
          for (int j = 0; j < N1; ++j)
            for (int i = 0; i < N0; ++i) {
              const long s = (i + ng) + (long)S0 * ((j + ng) + (long)S1 * (k + ng));
              if (out[s] != host[v][s]) {
                if (!fail) fprintf(stderr, "uniform state changed: field %d cell %d %d %d\n", v, i, j, k);
                fail = 1;
              }
            }
      } else if (v == 0 || v == 4) {
        const double rel = fabs(after - before[v]) / fabs(before[v]);
        printf("density wave: field %d interior sum %.15e -> %.15e (relative change %.2e)\n", v,
               before[v], after, rel);
        if (!(rel <= 1e-13)) fail = 1;
      }
    }
    for (int n = 0; n < NSTEPS; ++n)
      if (!(dts[n] > 0.0) || dg[4 * n + 3] != 0) fail = 1;
    printf("%s: dt[0] = %.6e, flagged cells %lld\n", wave ? "density wave" : "uniform state", dts[0],
           (long long)(dg[0] + dg[1]));
    free(out);
  }
  for (int v = 0; v < 8; ++v) {
    hipFree(dev[v]);
    free(host[v]);
  }
  hipFree(ws);
  hipFree(dt_out);
  hipFree(diag);
  printf("%s\n", fail ? "FAIL" : "ok");
  return fail;
}
