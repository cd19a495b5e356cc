/*
 * FP64 CPU oracle for the porous-media cascaded lattice Boltzmann (CLB) step
 * of Feng, Liu & He, "Numerical simulations of convection heat transfer in
 * porous media using a cascaded lattice Boltzmann method" (arXiv:2110.05943).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library and never imports it.
 *
 * State convention: the arrays f (9 per node) and g (5 per node) hold the
 * post-streaming populations at time n, node-major (f[node*9 + i]), with
 * node = y*nx + x.  One call of orc_step advances n -> n+1 by: macroscopic
 * quantities (Eqs. 20-23, 36, 4), boundary reconstruction, the D2Q9 collision
 * (Eqs. 11-17, A1), the D2Q5 collision (Eqs. 28-33, A2) and streaming
 * (Eqs. 18, 35).
 */
#ifndef CLB_ORACLE_H
#define CLB_ORACLE_H
#include <stdint.h>

/* Side kinds, one per side W(0) E(1) S(2) N(3). */
enum {
  ORC_PERIODIC = 0,       /* the axis wraps around                                   */
  ORC_WALL_T = 1,         /* wall with velocity (bc_u,bc_v) and temperature bc_T      */
  ORC_WALL_ADIABATIC = 2, /* wall with velocity (bc_u,bc_v), zero normal T gradient   */
  ORC_INLET = 3,          /* parabolic normal inflow of mean inlet_U, temperature bc_T */
  ORC_OUTLET = 4          /* rho = 1, u and T copied from the inner neighbour         */
};

typedef struct {
  int32_t nx, ny;          /* nodes, walls included                                   */
  int32_t bc[4];           /* side kinds for W, E, S, N                               */
  double bc_u[4], bc_v[4]; /* wall velocity per side                                  */
  double bc_T[4];          /* wall temperature per side                               */
  double inlet_U;          /* mean normal velocity of a parabolic inlet               */
  double nu;               /* fluid kinematic viscosity in the Darcy term of Eq. 4    */
  double s0, s1, s_b, s_v, s3, s4;     /* Eq. 15                                       */
  double zT, za, ze, zn;               /* Q of Eq. 28                                  */
  double varpi;            /* D2Q5 parameter, c_sT^2 = varpi/2 (Eq. 34)               */
  double sigma;            /* heat-capacity ratio                                     */
  double T0;               /* reference temperature of the Boussinesq term            */
  double gb[2];            /* G = gb*(T - T0) + a  (gb = -g*beta)                     */
  double a[2];             /* uniform external acceleration                           */
  const double *accel;     /* optional extra acceleration, 2 per node (x,y), or NULL  */
  const double *phi;       /* porosity per node                                       */
  const double *K;         /* permeability per node (INFINITY: no Darcy drag)         */
  const double *Fphi;      /* Forchheimer coefficient per node                        */
  int32_t nthreads;        /* OpenMP threads, <= 0: runtime default                   */
  int32_t model;           /* 0: cascaded (shift matrices N, N_T of Eqs. 14, 31);
                              1: raw-moment MRT, N = N_T = I (end of Section 2 and
                              Table 2): relax M f toward the raw equilibria and
                              forcing moments of Eq. 19, M_T g toward Eq. 33.
                              The single-rate (BGK) case is model 1 with equal
                              rates, chosen by the caller.                          */
} orc_params;

#ifdef __cplusplus
extern "C" {
#endif

/* Matrices as printed in the paper, row-major. */
void orc_matrix_M(double out[81]);                                   /* Eq. 13 */
void orc_matrix_Minv(double out[81]);                                /* M^-1   */
void orc_matrix_N(double ux, double uy, double phi, double out[81]);  /* Eq. 14 */
void orc_matrix_Ninv(double ux, double uy, double phi, double out[81]); /* Eq. A1 */
void orc_matrix_MT(double out[25]);                                  /* Eq. 30 */
void orc_matrix_MTinv(double out[25]);
void orc_matrix_NT(double ux, double uy, double sigma, double out[25]);  /* Eq. 31 */
void orc_matrix_NTinv(double ux, double uy, double sigma, double out[25]); /* Eq. A2 */
void orc_matrix_Lambda(const orc_params *p, double out[81]);          /* Eq. 15 */

/* Equilibria and sources. */
void orc_meq(double rho, double ux, double uy, double phi, double out[9]);   /* Eq. 19 */
void orc_Sraw(double rho, double ux, double uy, double Fx, double Fy, double phi,
              double out[9]);                                                /* Eq. 19 */
void orc_mteq(double rho, double out[9]);                                    /* Eq. 16 */
void orc_St(double rho, double Fx, double Fy, double out[9]);                /* Eq. 17 */
void orc_feq(double rho, double ux, double uy, double phi, double out[9]);   /* M^-1 m^eq */
void orc_geq(double T, double ux, double uy, double sigma, double varpi,
             double out[5]);                                                 /* Eq. 34 */
void orc_neq(double T, double ux, double uy, double sigma, double varpi,
             double out[5]);                                                 /* Eq. 33 */

/* One-node collisions with given macroscopic quantities. */
void orc_collide_f(const orc_params *p, const double f[9], double rho, double ux,
                   double uy, double Fx, double Fy, double phi, double out[9]);
void orc_collide_g(const orc_params *p, const double g[5], double T, double ux,
                   double uy, double out[5]);

/* Macroscopic quantities of one node from its populations (Eqs. 20-23, 36, 4). */
void orc_node_macros(const orc_params *p, const double f[9], const double g[5],
                     int32_t node, double out[6] /* rho ux uy T Fx Fy */);

/* Lattice operations. */
int orc_init_equilibrium(const orc_params *p, const double *rho, const double *ux,
                         const double *uy, const double *T, double *f, double *g);
int orc_step(const orc_params *p, double *f, double *g, int64_t nsteps);
/* Observable macroscopic fields at time n: fluid nodes by Eqs. 20-23/36,
 * boundary nodes report the boundary values used by their collision. */
int orc_macros(const orc_params *p, const double *f, const double *g, double *rho,
               double *ux, double *uy, double *T);
/* Mean Nusselt number on one side (0..3) by a second-order one-sided wall
 * gradient and the trapezoid rule; local values into `local` when non-NULL. */
double orc_nusselt(const orc_params *p, const double *f, const double *g, int32_t side,
                   double dT, double *local);

#ifdef __cplusplus
}
#endif
#endif
