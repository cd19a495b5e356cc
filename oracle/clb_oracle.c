/*
 * FP64 CPU oracle for the porous-media cascaded lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark.  It is not part of the product path and
 * shares nothing with the GPU library.
 *
 * Everything below follows Section 2 of Feng, Liu & He (arXiv:2110.05943)
 * with the matrices written out as printed: populations -> raw moments with M
 * (Eq. 13), raw -> central moments with the porous shift matrix N (Eq. 14),
 * relaxation by Eq. 11 with the block-diagonal Lambda of Eq. 15, and back with
 * N^-1 (Eq. A1) and M^-1.  The temperature lattice does the same with M_T
 * (Eq. 30), N_T (Eq. 31), Q (Eq. 28) and N_T^-1 (Eq. A2).  M^-1 and M_T^-1 are
 * not printed in the paper; they are obtained once by Gauss-Jordan elimination.
 *
 * Readings of points the paper leaves open (boundary treatment, corner rule,
 * Nusselt discretisation) are the ones stated next to the code that uses them.
 *
 * Pins (tests/test_oracle_pins.py): matrix identities, a brute-force 4x4 step,
 * consistent forcing, conservation, uniform Darcy-Forchheimer flow, linear
 * decay rates, pure conduction (Nu = 1), the Darcy-Brinkman channel and the
 * paper's mixed-convection channel with second-order convergence, and plane
 * Poiseuille flow between an inlet and an outlet side.  Boundary nodes
 * (tests/test_oracle_walls.py): a brute-force step with population-space
 * reconstruction on small walled lattices over every side kind and every
 * corner branch, and pure conduction with two Dirichlet sides at every corner
 * against its Fourier series (second order in the interior and in the far
 * side's Nusselt number).  The corner temperature between two Dirichlet sides
 * is a convention (no physical quantity fixes it: it only decides which of
 * the two sides books the flux of the corner gap); the brute force pins that
 * the oracle applies the stated one.
 */
#include "clb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D2Q9 velocities of Eq. 6 with c = 1; the D2Q5 set is the first five. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

/* Eq. 13 */
static const double MMAT[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},   {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1}, {0, 1, 0, 1, 0, 1, 1, 1, 1},
    {0, 0, 1, 0, 1, 1, 1, 1, 1},   {0, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 1, 1, -1, -1}, {0, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 1, 1, 1, 1}};

/* Eq. 30 */
static const double MTMAT[5][5] = {
    {1, 1, 1, 1, 1}, {0, 1, 0, -1, 0}, {0, 0, 1, 0, -1}, {0, 1, 0, 1, 0}, {0, 0, 1, 0, 1}};

static double MINV[9][9];
static double MTINV[5][5];
static int inverses_ready = 0;

/* Gauss-Jordan inverse with partial pivoting of an n x n row-major matrix. */
static void invert(int n, const double *a, double *out) {
  double w[9][18];
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < 2 * n; ++c)
      w[r][c] = c < n ? a[r * n + c] : (c - n == r ? 1.0 : 0.0);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(w[r][col]) > fabs(w[piv][col])) piv = r;
    if (piv != col)
      for (int c = 0; c < 2 * n; ++c) {
        double t = w[col][c];
        w[col][c] = w[piv][c];
        w[piv][c] = t;
      }
    double d = w[col][col];
    for (int c = 0; c < 2 * n; ++c) w[col][c] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double m = w[r][col];
      if (m == 0.0) continue;
      for (int c = 0; c < 2 * n; ++c) w[r][c] -= m * w[col][c];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) out[r * n + c] = w[r][n + c];
}

static void ensure_inverses(void) {
  if (inverses_ready) return;
#pragma omp critical(orc_inverse)
  {
    if (!inverses_ready) {
      invert(9, &MMAT[0][0], &MINV[0][0]);
      invert(5, &MTMAT[0][0], &MTINV[0][0]);
      inverses_ready = 1;
    }
  }
}

static void matvec(int n, const double *a, const double *x, double *y) {
  for (int r = 0; r < n; ++r) {
    double s = 0.0;
    for (int c = 0; c < n; ++c) s += a[r * n + c] * x[c];
    y[r] = s;
  }
}

/* ---------------------------------------------------------------- matrices */

void orc_matrix_M(double out[81]) { memcpy(out, MMAT, sizeof(MMAT)); }

void orc_matrix_Minv(double out[81]) {
  ensure_inverses();
  memcpy(out, MINV, sizeof(MINV));
}

void orc_matrix_MT(double out[25]) { memcpy(out, MTMAT, sizeof(MTMAT)); }

void orc_matrix_MTinv(double out[25]) {
  ensure_inverses();
  memcpy(out, MTINV, sizeof(MTINV));
}

/* Porous shift matrix N(u, phi), Eq. 14, entry by entry as printed. */
void orc_matrix_N(double ux, double uy, double phi, double out[81]) {
  const double ux2 = ux * ux, uy2 = uy * uy, p = phi, p2 = phi * phi;
  double N[9][9] = {{0}};
  for (int i = 0; i < 9; ++i) N[i][i] = 1.0;
  N[1][0] = -ux;
  N[2][0] = -uy;
  N[3][0] = ux2 / p;
  N[3][1] = -2.0 * ux / p;
  N[4][0] = uy2 / p;
  N[4][2] = -2.0 * uy / p;
  N[5][0] = ux * uy / p;
  N[5][1] = -uy / p;
  N[5][2] = -ux / p;
  N[6][0] = -ux2 * uy / p;
  N[6][1] = 2.0 * ux * uy / p;
  N[6][2] = ux2 / p;
  N[6][3] = -uy;
  N[6][5] = -2.0 * ux;
  N[7][0] = -uy2 * ux / p;
  N[7][1] = uy2 / p;
  N[7][2] = 2.0 * ux * uy / p;
  N[7][4] = -ux;
  N[7][5] = -2.0 * uy;
  N[8][0] = ux2 * uy2 / p2;
  N[8][1] = -2.0 * ux * uy2 / p2;
  N[8][2] = -2.0 * uy * ux2 / p2;
  N[8][3] = uy2 / p;
  N[8][4] = ux2 / p;
  N[8][5] = 4.0 * ux * uy / p;
  N[8][6] = -2.0 * uy / p;
  N[8][7] = -2.0 * ux / p;
  memcpy(out, N, sizeof(N));
}

/* N^-1 as printed in Appendix A, Eq. A1. */
void orc_matrix_Ninv(double ux, double uy, double phi, double out[81]) {
  const double ux2 = ux * ux, uy2 = uy * uy, p = phi, p2 = phi * phi;
  double A[9][9] = {{0}};
  for (int i = 0; i < 9; ++i) A[i][i] = 1.0;
  A[1][0] = ux;
  A[2][0] = uy;
  A[3][0] = ux2 / p;
  A[3][1] = 2.0 * ux / p;
  A[4][0] = uy2 / p;
  A[4][2] = 2.0 * uy / p;
  A[5][0] = ux * uy / p;
  A[5][1] = uy / p;
  A[5][2] = ux / p;
  A[6][0] = ux2 * uy / p;
  A[6][1] = 2.0 * ux * uy / p;
  A[6][2] = ux2 / p;
  A[6][3] = uy;
  A[6][5] = 2.0 * ux;
  A[7][0] = uy2 * ux / p;
  A[7][1] = uy2 / p;
  A[7][2] = 2.0 * ux * uy / p;
  A[7][4] = ux;
  A[7][5] = 2.0 * uy;
  A[8][0] = ux2 * uy2 / p2;
  A[8][1] = 2.0 * ux * uy2 / p2;
  A[8][2] = 2.0 * uy * ux2 / p2;
  A[8][3] = uy2 / p;
  A[8][4] = ux2 / p;
  A[8][5] = 4.0 * ux * uy / p;
  A[8][6] = 2.0 * uy / p;
  A[8][7] = 2.0 * ux / p;
  memcpy(out, A, sizeof(A));
}

/* Temperature shift matrix N_T(u, sigma), Eq. 31. */
void orc_matrix_NT(double ux, double uy, double sigma, double out[25]) {
  double N[5][5] = {{0}};
  for (int i = 0; i < 5; ++i) N[i][i] = 1.0;
  N[1][0] = -ux / sigma;
  N[2][0] = -uy / sigma;
  N[3][0] = ux * ux / sigma;
  N[3][1] = -2.0 * ux;
  N[4][0] = uy * uy / sigma;
  N[4][2] = -2.0 * uy;
  memcpy(out, N, sizeof(N));
}

/* N_T^-1 as printed in Appendix A, Eq. A2. */
void orc_matrix_NTinv(double ux, double uy, double sigma, double out[25]) {
  double A[5][5] = {{0}};
  for (int i = 0; i < 5; ++i) A[i][i] = 1.0;
  A[1][0] = ux / sigma;
  A[2][0] = uy / sigma;
  A[3][0] = ux * ux / sigma;
  A[3][1] = 2.0 * ux;
  A[4][0] = uy * uy / sigma;
  A[4][2] = 2.0 * uy;
  memcpy(out, A, sizeof(A));
}

/* Block-diagonal relaxation matrix of Eq. 15:
 * diag([s0, s1, s1], [[s+, s-], [s-, s+]], [s_v, s3, s3, s4]),
 * s+ = (s_b + s_v)/2, s- = (s_b - s_v)/2. */
void orc_matrix_Lambda(const orc_params *p, double out[81]) {
  double L[9][9] = {{0}};
  const double sp = 0.5 * (p->s_b + p->s_v), sm = 0.5 * (p->s_b - p->s_v);
  L[0][0] = p->s0;
  L[1][1] = p->s1;
  L[2][2] = p->s1;
  L[3][3] = sp;
  L[3][4] = sm;
  L[4][3] = sm;
  L[4][4] = sp;
  L[5][5] = p->s_v;
  L[6][6] = p->s3;
  L[7][7] = p->s3;
  L[8][8] = p->s4;
  memcpy(out, L, sizeof(L));
}

/* ------------------------------------------------------------ equilibria */

static const double CS2 = 1.0 / 3.0; /* c_s^2 of D2Q9 with c = 1 */

/* Equilibrium raw moments, Eq. 19 (left). */
void orc_meq(double rho, double ux, double uy, double phi, double out[9]) {
  const double ux2 = ux * ux, uy2 = uy * uy;
  out[0] = rho;
  out[1] = rho * ux;
  out[2] = rho * uy;
  out[3] = rho / 3.0 + rho * ux2 / phi;
  out[4] = rho / 3.0 + rho * uy2 / phi;
  out[5] = rho * ux * uy / phi;
  out[6] = rho * uy / 3.0 + rho * ux2 * uy / phi;
  out[7] = rho * ux / 3.0 + rho * ux * uy2 / phi;
  out[8] = rho / 9.0 + rho * (ux2 + uy2) / (3.0 * phi) + rho * ux2 * uy2 / (phi * phi);
}

/* Raw-moment forcing terms, Eq. 19 (right). */
void orc_Sraw(double rho, double ux, double uy, double Fx, double Fy, double phi,
              double out[9]) {
  const double p = phi, p2 = phi * phi;
  out[0] = 0.0;
  out[1] = rho * Fx;
  out[2] = rho * Fy;
  out[3] = 2.0 * rho * ux * Fx / p;
  out[4] = 2.0 * rho * uy * Fy / p;
  out[5] = rho * (ux * Fy + uy * Fx) / p;
  out[6] = rho * Fy / 3.0 + rho * Fy * ux * ux / p + 2.0 * rho * Fx * ux * uy / p;
  out[7] = rho * Fx / 3.0 + rho * Fx * uy * uy / p + 2.0 * rho * Fy * uy * ux / p;
  out[8] = (2.0 / 3.0) * rho * (ux * Fx + uy * Fy) / p + 2.0 * rho * Fx * ux * uy * uy / p2 +
           2.0 * rho * Fy * uy * ux * ux / p2;
}

/* Equilibrium central moments, Eq. 16. */
void orc_mteq(double rho, double out[9]) {
  memset(out, 0, 9 * sizeof(double));
  out[0] = rho;
  out[3] = rho * CS2;
  out[4] = rho * CS2;
  out[8] = rho * CS2 * CS2;
}

/* Central-moment forcing terms, Eq. 17. */
void orc_St(double rho, double Fx, double Fy, double out[9]) {
  memset(out, 0, 9 * sizeof(double));
  out[1] = rho * Fx;
  out[2] = rho * Fy;
  out[6] = CS2 * rho * Fy;
  out[7] = CS2 * rho * Fx;
}

/* f^eq = M^-1 m^eq (text after Eq. 19). */
void orc_feq(double rho, double ux, double uy, double phi, double out[9]) {
  double m[9];
  ensure_inverses();
  orc_meq(rho, ux, uy, phi, m);
  matvec(9, &MINV[0][0], m, out);
}

/* g^eq, Eq. 34 as printed. */
void orc_geq(double T, double ux, double uy, double sigma, double varpi, double out[5]) {
  out[0] = sigma * T - varpi * T - (ux * ux + uy * uy) * T;
  out[1] = 0.25 * varpi * T + 0.5 * ux * T + 0.5 * ux * ux * T;
  out[2] = 0.25 * varpi * T + 0.5 * uy * T + 0.5 * uy * uy * T;
  out[3] = 0.25 * varpi * T - 0.5 * ux * T + 0.5 * ux * ux * T;
  out[4] = 0.25 * varpi * T - 0.5 * uy * T + 0.5 * uy * uy * T;
}

/* Equilibrium raw moments of g, Eq. 33, with c_sT^2 = varpi/2. */
void orc_neq(double T, double ux, double uy, double sigma, double varpi, double out[5]) {
  const double cT2 = 0.5 * varpi;
  out[0] = sigma * T;
  out[1] = ux * T;
  out[2] = uy * T;
  out[3] = (cT2 + ux * ux) * T;
  out[4] = (cT2 + uy * uy) * T;
}

/* -------------------------------------------------------------- collisions */

/* D2Q9: m = M f; m~ = N m; Eq. 11; f* = M^-1 N^-1 m~* (Eqs. 11-18). */
void orc_collide_f(const orc_params *p, const double f[9], double rho, double ux,
                   double uy, double Fx, double Fy, double phi, double out[9]) {
  double m[9], mt[9], N[81], Ninv[81], L[81], eq[9], St[9], diff[9], ms[9], mr[9];
  ensure_inverses();
  matvec(9, &MMAT[0][0], f, m);
  if (p->model == 1) {
    /* MRT: N = I, so the moments, equilibria and forcing are the raw ones */
    memcpy(mt, m, sizeof(mt));
    orc_meq(rho, ux, uy, phi, eq);
    orc_Sraw(rho, ux, uy, Fx, Fy, phi, St);
  } else {
    orc_matrix_N(ux, uy, phi, N);
    matvec(9, N, m, mt);
    orc_mteq(rho, eq);
    orc_St(rho, Fx, Fy, St);
  }
  orc_matrix_Lambda(p, L);
  for (int i = 0; i < 9; ++i) diff[i] = mt[i] - eq[i];
  for (int r = 0; r < 9; ++r) {
    double relax = 0.0, src = 0.0;
    for (int c = 0; c < 9; ++c) {
      relax += L[r * 9 + c] * diff[c];
      src += ((r == c ? 1.0 : 0.0) - 0.5 * L[r * 9 + c]) * St[c];
    }
    ms[r] = mt[r] - relax + src;
  }
  if (p->model == 1) {
    memcpy(mr, ms, sizeof(mr));
  } else {
    orc_matrix_Ninv(ux, uy, phi, Ninv);
    matvec(9, Ninv, ms, mr);
  }
  matvec(9, &MINV[0][0], mr, out);
}

/* D2Q5: n = M_T g; n~ = N_T n; Eq. 28; g* = M_T^-1 N_T^-1 n~* (Eqs. 28-35). */
void orc_collide_g(const orc_params *p, const double g[5], double T, double ux,
                   double uy, double out[5]) {
  double n[5], nt[5], N[25], Ninv[25], eq[5], ns[5], nr[5];
  const double q[5] = {p->zT, p->za, p->za, p->ze, p->zn};
  const double cT2 = 0.5 * p->varpi;
  ensure_inverses();
  matvec(5, &MTMAT[0][0], g, n);
  if (p->model == 1) {
    /* MRT: N_T = I, raw equilibria of Eq. 33 */
    memcpy(nt, n, sizeof(nt));
    orc_neq(T, ux, uy, p->sigma, p->varpi, eq);
  } else {
    orc_matrix_NT(ux, uy, p->sigma, N);
    matvec(5, N, n, nt);
    /* Eq. 32 */
    eq[0] = p->sigma * T;
    eq[1] = 0.0;
    eq[2] = 0.0;
    eq[3] = cT2 * T;
    eq[4] = cT2 * T;
  }
  for (int i = 0; i < 5; ++i) ns[i] = nt[i] - q[i] * (nt[i] - eq[i]);
  if (p->model == 1) {
    memcpy(nr, ns, sizeof(nr));
  } else {
    orc_matrix_NTinv(ux, uy, p->sigma, Ninv);
    matvec(5, Ninv, ns, nr);
  }
  matvec(5, &MTINV[0][0], nr, out);
}

/* ------------------------------------------------------ macroscopic values */

static void body_force(const orc_params *p, int node, double ux, double uy, double T,
                       double *Fx, double *Fy) {
  /* G = -g beta (T - T0) + a (text after Eq. 4); F of Eq. 4. */
  double Gx = p->gb[0] * (T - p->T0) + p->a[0];
  double Gy = p->gb[1] * (T - p->T0) + p->a[1];
  if (p->accel) {
    Gx += p->accel[2 * node];
    Gy += p->accel[2 * node + 1];
  }
  const double phi = p->phi[node], K = p->K[node], Fp = p->Fphi[node];
  const double umag = sqrt(ux * ux + uy * uy);
  *Fx = -phi * p->nu / K * ux - phi * Fp / sqrt(K) * umag * ux + phi * Gx;
  *Fy = -phi * p->nu / K * uy - phi * Fp / sqrt(K) * umag * uy + phi * Gy;
}

void orc_node_macros(const orc_params *p, const double f[9], const double g[5],
                     int32_t node, double out[6]) {
  double rho = 0.0, jx = 0.0, jy = 0.0, sg = 0.0;
  for (int i = 0; i < 9; ++i) {
    rho += f[i];           /* Eq. 20 */
    jx += EX[i] * f[i];
    jy += EY[i] * f[i];
  }
  for (int i = 0; i < 5; ++i) sg += g[i];
  const double T = sg / p->sigma; /* Eq. 36 */
  double Gx = p->gb[0] * (T - p->T0) + p->a[0];
  double Gy = p->gb[1] * (T - p->T0) + p->a[1];
  if (p->accel) {
    Gx += p->accel[2 * node];
    Gy += p->accel[2 * node + 1];
  }
  const double phi = p->phi[node], K = p->K[node], Fp = p->Fphi[node];
  /* Eq. 23 */
  const double vx = jx / rho + 0.5 * phi * Gx;
  const double vy = jy / rho + 0.5 * phi * Gy;
  const double l0 = 0.5 * (1.0 + phi * 0.5 * p->nu / K);
  const double l1 = phi * 0.5 * Fp / sqrt(K);
  const double vmag = sqrt(vx * vx + vy * vy);
  /* Eq. 22 */
  const double den = l0 + sqrt(l0 * l0 + l1 * vmag);
  const double ux = vx / den, uy = vy / den;
  double Fx, Fy;
  body_force(p, node, ux, uy, T, &Fx, &Fy);
  out[0] = rho;
  out[1] = ux;
  out[2] = uy;
  out[3] = T;
  out[4] = Fx;
  out[5] = Fy;
}

/* --------------------------------------------------------------- boundary */

/* Boundary reading used throughout (the paper cites the non-equilibrium
 * extrapolation scheme of its Ref. [55] without writing it out):
 *  - walls lie on the outermost nodes; a node on a non-periodic side is a
 *    boundary node;
 *  - x_f is the inward normal neighbour (the diagonal one at a corner),
 *    x_ff the next node on the same line;
 *  - before the collision all q populations of a boundary node are replaced
 *    by f_i = f_i^eq(rho_b, u_b; phi_b) + [f_i(x_f) - f_i^eq(rho_f, u_f; phi_f)]
 *    and g_i = g_i^eq(T_b, u_b) + [g_i(x_f) - g_i^eq(T_f, u_f)];
 *  - the node then collides with rho_b, u_b, T_b and F(u_b, T_b);
 *  - rho_b = rho_f except at an outlet (rho_b = 1);
 *  - an adiabatic wall takes T_b = (4 T_f - T_ff)/3;
 *  - at a corner u_b = 0 and T_b is the Dirichlet value of the x-side if it
 *    has one, else of the y-side, else the extrapolated value. */
typedef struct {
  int boundary;
  int xf, yf, xff, yff;
  int sx, sy; /* side index on the x / y axis, or -1 */
} bnode_t;

static bnode_t classify(const orc_params *p, int x, int y) {
  bnode_t b;
  memset(&b, 0, sizeof(b));
  b.sx = -1;
  b.sy = -1;
  int dx = 0, dy = 0;
  if (x == 0 && p->bc[0] != ORC_PERIODIC) {
    b.sx = 0;
    dx = 1;
  } else if (x == p->nx - 1 && p->bc[1] != ORC_PERIODIC) {
    b.sx = 1;
    dx = -1;
  }
  if (y == 0 && p->bc[2] != ORC_PERIODIC) {
    b.sy = 2;
    dy = 1;
  } else if (y == p->ny - 1 && p->bc[3] != ORC_PERIODIC) {
    b.sy = 3;
    dy = -1;
  }
  b.boundary = (b.sx >= 0 || b.sy >= 0);
  b.xf = x + dx;
  b.yf = y + dy;
  b.xff = x + 2 * dx;
  b.yff = y + 2 * dy;
  return b;
}

static int is_dirichlet_T(int kind) { return kind == ORC_WALL_T || kind == ORC_INLET; }

/* Boundary values (rho_b, u_b, T_b) of a boundary node from the fluid
 * macroscopic values of x_f and the temperature of x_ff. */
static void boundary_values(const orc_params *p, int x, int y, const bnode_t *b,
                            const double *mf /* rho ux uy T of x_f */, double Tff,
                            double out[4]) {
  const double Textra = (4.0 * mf[3] - Tff) / 3.0;
  if (b->sx >= 0 && b->sy >= 0) { /* corner */
    out[0] = mf[0];
    out[1] = 0.0;
    out[2] = 0.0;
    if (is_dirichlet_T(p->bc[b->sx]))
      out[3] = p->bc_T[b->sx];
    else if (is_dirichlet_T(p->bc[b->sy]))
      out[3] = p->bc_T[b->sy];
    else
      out[3] = Textra;
    return;
  }
  const int s = b->sx >= 0 ? b->sx : b->sy;
  switch (p->bc[s]) {
    case ORC_WALL_T:
      out[0] = mf[0];
      out[1] = p->bc_u[s];
      out[2] = p->bc_v[s];
      out[3] = p->bc_T[s];
      break;
    case ORC_WALL_ADIABATIC:
      out[0] = mf[0];
      out[1] = p->bc_u[s];
      out[2] = p->bc_v[s];
      out[3] = Textra;
      break;
    case ORC_INLET: {
      /* parabolic profile with mean inlet_U along the side, inward normal */
      const double t = (s < 2) ? (double)y / (p->ny - 1) : (double)x / (p->nx - 1);
      const double un = 6.0 * p->inlet_U * t * (1.0 - t);
      out[0] = mf[0];
      out[1] = s == 0 ? un : (s == 1 ? -un : 0.0);
      out[2] = s == 2 ? un : (s == 3 ? -un : 0.0);
      out[3] = p->bc_T[s];
      break;
    }
    default: /* ORC_OUTLET */
      out[0] = 1.0;
      out[1] = mf[1];
      out[2] = mf[2];
      out[3] = mf[3];
      break;
  }
}

/* ---------------------------------------------------------------- lattice */

/* nthreads > 0: that many threads; 0: the process's initial OpenMP default
   (a call with an explicit count does not carry over to later calls). */
static void set_threads(const orc_params *p) {
#ifdef _OPENMP
  static int initial = 0;
  if (initial == 0) initial = omp_get_max_threads();
  omp_set_num_threads(p->nthreads > 0 ? p->nthreads : initial);
#else
  (void)p;
#endif
}

static int check(const orc_params *p) {
  if (p->nx < 3 || p->ny < 3) return -1;
  for (int s = 0; s < 2; ++s)
    if (p->bc[s] != ORC_PERIODIC && p->nx < 4) return -1;
  for (int s = 2; s < 4; ++s)
    if (p->bc[s] != ORC_PERIODIC && p->ny < 4) return -1;
  if ((p->bc[0] == ORC_PERIODIC) != (p->bc[1] == ORC_PERIODIC)) return -1;
  if ((p->bc[2] == ORC_PERIODIC) != (p->bc[3] == ORC_PERIODIC)) return -1;
  return 0;
}

int orc_init_equilibrium(const orc_params *p, const double *rho, const double *ux,
                         const double *uy, const double *T, double *f, double *g) {
  if (check(p)) return -1;
  const long n = (long)p->nx * p->ny;
  ensure_inverses();
  for (long k = 0; k < n; ++k) {
    orc_feq(rho ? rho[k] : 1.0, ux ? ux[k] : 0.0, uy ? uy[k] : 0.0, p->phi[k], f + 9 * k);
    orc_geq(T[k], ux ? ux[k] : 0.0, uy ? uy[k] : 0.0, p->sigma, p->varpi, g + 5 * k);
  }
  return 0;
}

/* Fluid macroscopic values of every node (meaningless at boundary nodes). */
static void all_fluid_macros(const orc_params *p, const double *f, const double *g,
                             double *mac /* 6 per node */) {
  const long n = (long)p->nx * p->ny;
#pragma omp parallel for schedule(static)
  for (long k = 0; k < n; ++k) orc_node_macros(p, f + 9 * k, g + 5 * k, (int32_t)k, mac + 6 * k);
}

/* Replace boundary-node populations and macroscopic values (pre-collision). */
static void apply_boundaries(const orc_params *p, const double *f, const double *g,
                             double *mac, double *fb, double *gb) {
  const int nx = p->nx, ny = p->ny;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const bnode_t b = classify(p, x, y);
      if (!b.boundary) continue;
      const long k = (long)y * nx + x;
      const long kf = (long)b.yf * nx + b.xf;
      const double *mf = mac + 6 * kf;
      double Tff = mf[3];
      if (b.xff >= 0 && b.xff < nx && b.yff >= 0 && b.yff < ny)
        Tff = mac[6 * ((long)b.yff * nx + b.xff) + 3];
      double bv[4];
      boundary_values(p, x, y, &b, mf, Tff, bv);
      double eqb[9], eqf[9], geb[5], gef[5];
      orc_feq(bv[0], bv[1], bv[2], p->phi[k], eqb);
      orc_feq(mf[0], mf[1], mf[2], p->phi[kf], eqf);
      for (int i = 0; i < 9; ++i) fb[9 * k + i] = eqb[i] + (f[9 * kf + i] - eqf[i]);
      orc_geq(bv[3], bv[1], bv[2], p->sigma, p->varpi, geb);
      orc_geq(mf[3], mf[1], mf[2], p->sigma, p->varpi, gef);
      for (int i = 0; i < 5; ++i) gb[5 * k + i] = geb[i] + (g[5 * kf + i] - gef[i]);
      double Fx, Fy;
      body_force(p, (int)k, bv[1], bv[2], bv[3], &Fx, &Fy);
      double *m = mac + 6 * k;
      m[0] = bv[0];
      m[1] = bv[1];
      m[2] = bv[2];
      m[3] = bv[3];
      m[4] = Fx;
      m[5] = Fy;
    }
}

int orc_step(const orc_params *p, double *f, double *g, int64_t nsteps) {
  if (check(p)) return -1;
  ensure_inverses();
  set_threads(p);
  const int nx = p->nx, ny = p->ny;
  const long n = (long)nx * ny;
  double *mac = (double *)malloc(sizeof(double) * 6 * n);
  double *fpre = (double *)malloc(sizeof(double) * 9 * n);
  double *gpre = (double *)malloc(sizeof(double) * 5 * n);
  double *fpost = (double *)malloc(sizeof(double) * 9 * n);
  double *gpost = (double *)malloc(sizeof(double) * 5 * n);
  if (!mac || !fpre || !gpre || !fpost || !gpost) {
    free(mac); free(fpre); free(gpre); free(fpost); free(gpost);
    return -2;
  }
  for (int64_t step = 0; step < nsteps; ++step) {
    /* macroscopic values, then boundary reconstruction */
    all_fluid_macros(p, f, g, mac);
    memcpy(fpre, f, sizeof(double) * 9 * n);
    memcpy(gpre, g, sizeof(double) * 5 * n);
    apply_boundaries(p, f, g, mac, fpre, gpre);
    /* collision at every node */
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) {
      const double *m = mac + 6 * k;
      orc_collide_f(p, fpre + 9 * k, m[0], m[1], m[2], m[4], m[5], p->phi[k], fpost + 9 * k);
      orc_collide_g(p, gpre + 5 * k, m[3], m[1], m[2], gpost + 5 * k);
    }
    /* streaming, Eqs. 18 and 35: f_i(x + e_i) = f_i*(x).  A population whose
     * source lies outside a non-periodic side keeps its post-collision value;
     * it belongs to a boundary node, whose populations are all rebuilt at the
     * next step. */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const long k = (long)y * nx + x;
        for (int i = 0; i < 9; ++i) {
          int sx = x - EX[i], sy = y - EY[i];
          int inside = 1;
          if (sx < 0 || sx >= nx) {
            if (p->bc[0] == ORC_PERIODIC) sx = (sx + nx) % nx;
            else inside = 0;
          }
          if (sy < 0 || sy >= ny) {
            if (p->bc[2] == ORC_PERIODIC) sy = (sy + ny) % ny;
            else inside = 0;
          }
          const long ks = inside ? (long)sy * nx + sx : k;
          f[9 * k + i] = fpost[9 * ks + i];
          if (i < 5) g[5 * k + i] = gpost[5 * ks + i];
        }
      }
  }
  free(mac); free(fpre); free(gpre); free(fpost); free(gpost);
  return 0;
}

int orc_macros(const orc_params *p, const double *f, const double *g, double *rho,
               double *ux, double *uy, double *T) {
  if (check(p)) return -1;
  ensure_inverses();
  set_threads(p);
  const long n = (long)p->nx * p->ny;
  double *mac = (double *)malloc(sizeof(double) * 6 * n);
  double *fb = (double *)malloc(sizeof(double) * 9 * n);
  double *gb = (double *)malloc(sizeof(double) * 5 * n);
  if (!mac || !fb || !gb) {
    free(mac); free(fb); free(gb);
    return -2;
  }
  all_fluid_macros(p, f, g, mac);
  apply_boundaries(p, f, g, mac, fb, gb);
  for (long k = 0; k < n; ++k) {
    if (rho) rho[k] = mac[6 * k];
    if (ux) ux[k] = mac[6 * k + 1];
    if (uy) uy[k] = mac[6 * k + 2];
    if (T) T[k] = mac[6 * k + 3];
  }
  free(mac); free(fb); free(gb);
  return 0;
}

/* Nusselt number (the paper gives only the continuum form
 * Nu(y) = -L (dT/dx)_wall / dT and its mean over the wall).  Reading: the
 * wall-normal derivative is the second-order one-sided difference
 * (-3 T_0 + 4 T_1 - T_2)/2 taken inward from the wall, L is the node count
 * across the domain minus one, and the mean is the trapezoid rule over the
 * wall nodes divided by their span. */
double orc_nusselt(const orc_params *p, const double *f, const double *g, int32_t side,
                   double dT, double *local) {
  if (check(p) || side < 0 || side > 3) return NAN;
  const int nx = p->nx, ny = p->ny;
  double *T = (double *)malloc(sizeof(double) * (long)nx * ny);
  if (!T) return NAN;
  orc_macros(p, f, g, NULL, NULL, NULL, T);
  const int along_y = side < 2; /* W/E walls run along y */
  const int nw = along_y ? ny : nx;
  const double L = along_y ? nx - 1 : ny - 1;
  /* derivative along +x (+y) = sign * inward one-sided difference */
  const double sign = (side == 0 || side == 2) ? 1.0 : -1.0;
  double sum = 0.0;
  for (int j = 0; j < nw; ++j) {
    double t[3];
    for (int d = 0; d < 3; ++d) {
      int x, y;
      if (along_y) {
        y = j;
        x = side == 0 ? d : nx - 1 - d;
      } else {
        x = j;
        y = side == 2 ? d : ny - 1 - d;
      }
      t[d] = T[(long)y * nx + x];
    }
    const double grad = sign * (-3.0 * t[0] + 4.0 * t[1] - t[2]) / 2.0;
    const double nu = -L * grad / dT;
    if (local) local[j] = nu;
    sum += (j == 0 || j == nw - 1) ? 0.5 * nu : nu;
  }
  free(T);
  return sum / (nw - 1);
}
