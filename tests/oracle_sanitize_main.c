/* Host driver that runs the FP64 oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_oracle_sanitizers.py with
 * gcc; test infrastructure only).  It steps every side kind: a walled cavity
 * with a porosity field, a periodic channel with moving walls and a per-node
 * acceleration, an inlet/outlet channel, and the raw-moment (MRT) model. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "clb_oracle.h"

static int run(int nx, int ny, const int bc[4], int model, int hetero, int accel) {
  const int n = nx * ny;
  double *phi = malloc(sizeof(double) * n), *K = malloc(sizeof(double) * n),
         *Fp = malloc(sizeof(double) * n), *acc = accel ? malloc(sizeof(double) * 2 * n) : NULL;
  double *rho = malloc(sizeof(double) * n), *ux = malloc(sizeof(double) * n),
         *uy = malloc(sizeof(double) * n), *T = malloc(sizeof(double) * n);
  double *f = malloc(sizeof(double) * 9 * n), *g = malloc(sizeof(double) * 5 * n);
  for (int i = 0; i < n; ++i) {
    phi[i] = hetero ? 0.4 + 0.5 * (double)((i * 7919) % 101) / 100.0 : 0.6;
    K[i] = 40.0 * phi[i];
    Fp[i] = 0.3;
    rho[i] = 1.0;
    ux[i] = 0.01 * sin(0.3 * i);
    uy[i] = 0.01 * cos(0.2 * i);
    T[i] = 0.5 + 0.2 * sin(0.1 * i);
    if (acc) {
      acc[2 * i] = 1e-6 * (i % ny);
      acc[2 * i + 1] = 2e-6;
    }
  }
  orc_params p = {0};
  p.nx = nx;
  p.ny = ny;
  for (int s = 0; s < 4; ++s) {
    p.bc[s] = bc[s];
    p.bc_T[s] = s == 0 ? 1.0 : 0.0;
  }
  p.bc_u[3] = 0.01;
  p.inlet_U = 0.02;
  p.nu = 0.1;
  p.s0 = p.s1 = 1.0;
  p.s_b = 1.5;
  p.s_v = 1.2;
  p.s3 = 1.2;
  p.s4 = 1.8;
  p.zT = p.ze = p.zn = 1.0;
  p.za = 1.1;
  p.varpi = 0.25;
  p.sigma = 0.9;
  p.T0 = 0.5;
  p.gb[1] = 1e-4;
  p.accel = acc;
  p.phi = phi;
  p.K = K;
  p.Fphi = Fp;
  p.nthreads = 1;
  p.model = model;
  int rc = orc_init_equilibrium(&p, rho, ux, uy, T, f, g);
  if (!rc) rc = orc_step(&p, f, g, 40);
  if (!rc) rc = orc_macros(&p, f, g, rho, ux, uy, T);
  double nu = 0.0;
  for (int s = 0; s < 4 && !rc; ++s)
    if (bc[s] != ORC_PERIODIC) nu += orc_nusselt(&p, f, g, s, 1.0, NULL);
  int bad = rc != 0 || !isfinite(nu);
  for (int i = 0; i < n; ++i) bad |= !isfinite(ux[i]) || !isfinite(T[i]);
  printf("%dx%d bc %d %d %d %d model %d: rc %d nu %.6f\n", nx, ny, bc[0], bc[1], bc[2], bc[3],
         model, rc, nu);
  free(phi), free(K), free(Fp), free(acc), free(rho), free(ux), free(uy), free(T), free(f),
      free(g);
  return bad;
}

int main(void) {
  const int cavity[4] = {ORC_WALL_T, ORC_WALL_T, ORC_WALL_ADIABATIC, ORC_WALL_ADIABATIC};
  const int channel[4] = {ORC_PERIODIC, ORC_PERIODIC, ORC_WALL_T, ORC_WALL_T};
  const int inout[4] = {ORC_INLET, ORC_OUTLET, ORC_WALL_T, ORC_WALL_ADIABATIC};
  const int periodic[4] = {ORC_PERIODIC, ORC_PERIODIC, ORC_PERIODIC, ORC_PERIODIC};
  int bad = 0;
  bad |= run(9, 7, cavity, 0, 1, 0);
  bad |= run(8, 11, channel, 0, 0, 1);
  bad |= run(13, 6, inout, 0, 1, 0);
  bad |= run(5, 5, periodic, 1, 1, 1);
  bad |= run(4, 4, cavity, 1, 0, 0);
  return bad;
}
