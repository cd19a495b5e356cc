/*
 * clb.h - C ABI of the MI355X (gfx950) porous-media cascaded lattice
 * Boltzmann library.
 *
 * The library advances one or many independent 2-D domains ("cavities") of
 * the coupled method of Feng, Liu & He, "Numerical simulations of convection
 * heat transfer in porous media using a cascaded lattice Boltzmann method"
 * (arXiv:2110.05943):
 *   - flow: D2Q9 central-moment collision whose shift matrix carries the
 *     porosity (Section 2.1, Eqs. 6-23, A1) with the generalized non-Darcy
 *     (Brinkman-Forchheimer) force of Eq. 4;
 *   - temperature: D2Q5 central-moment collision whose shift matrix carries the
 *     heat-capacity ratio sigma (Section 2.2, Eqs. 24-37, A2);
 *   - streaming (Eqs. 18, 35), boundary nodes by non-equilibrium
 *     extrapolation, and FP64 reductions for the Nusselt number (Section 3.2),
 *     residual and mass.
 *
 * Conventions (all entry points):
 *   - Every call returns clb_status; CLB_OK is 0.  No call throws.
 *   - Out-parameters are left untouched when a call fails.
 *   - The caller owns all device memory: clb_create receives one device
 *     workspace of clb_workspace_bytes() bytes and never allocates device
 *     memory itself.  The caller also owns the HIP stream (a hipStream_t passed
 *     as void*); all device work is enqueued on it.  The workspace must stay
 *     allocated until clb_destroy.
 *   - Host arrays of nodal fields are row-major (ny rows of nx values, x
 *     fastest, index y*nx + x), in FP64.  Walls lie on the outermost nodes,
 *     so nx and ny count wall nodes and the characteristic length of a square
 *     cavity is L = nx - 1.
 *   - A context may be used by one host thread at a time.  Calls that return
 *     host values synchronize the stream.
 */
#ifndef CLB_H
#define CLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CLB_OK = 0,
  CLB_ERR_ARG = 1,        /* invalid argument or parameter set                 */
  CLB_ERR_HIP = 2,        /* a HIP runtime call failed (launch, copy, fault)   */
  CLB_ERR_WORKSPACE = 3,  /* workspace too small or misaligned (256 B)         */
  CLB_ERR_DIVERGED = 4,   /* a non-finite value was found in the fields        */
  CLB_ERR_STATE = 5,      /* call not valid in the current state               */
  CLB_NOT_CONVERGED = 6   /* per-domain result of clb_run: still unsteady      */
} clb_status;

/* Side kinds (index 0..3 = W, E, S, N). */
enum {
  CLB_PERIODIC = 0,       /* the axis wraps; both sides of an axis must agree  */
  CLB_WALL_T = 1,         /* wall, velocity (bc_u, bc_v), temperature bc_T      */
  CLB_WALL_ADIABATIC = 2, /* wall, velocity (bc_u, bc_v), zero normal gradient  */
  CLB_INLET = 3,          /* parabolic normal inflow of mean inlet_U, T = bc_T  */
  CLB_OUTLET = 4          /* rho = 1, velocity and T taken from the inner node  */
};

enum { CLB_WEST = 0, CLB_EAST = 1, CLB_SOUTH = 2, CLB_NORTH = 3 };

/* Storage of the populations in device memory.  Every mode stores the
 * deviation of each population from its rest value and rounds stochastically
 * when narrowing (unbiased rounding; bit-reproducible from the step count).
 *   CLB_STORE_F32:   14 FP32 planes (112 B per node update), FP64 arithmetic;
 *   CLB_STORE_F16:   14 FP16 planes (56 B), FP32 arithmetic;
 *   CLB_STORE_MIXED: 9 FP16 flow planes and 5 FP32 temperature planes (76 B),
 *                    FP32 arithmetic;
 *   CLB_STORE_F32C:  14 FP32 planes (112 B), FP32 arithmetic (FP64 only in
 *                    the reductions); the node's heat sum (Eq. 36) and the
 *                    D2Q5 rest population carry the exact errors of their
 *                    FP32 additions (compensated sums), and the rest
 *                    population, the one stored value whose round-to-nearest
 *                    bias the thermal field would accumulate, is rounded
 *                    stochastically from its compensated value; the other
 *                    planes round to nearest. */
enum { CLB_STORE_F32 = 0, CLB_STORE_F16 = 1, CLB_STORE_MIXED = 2, CLB_STORE_F32C = 3 };

/* Collision operator of a domain.
 *   CLB_MODEL_CASCADED: the paper's method, moments shifted by N(u, phi) and
 *                       N_T(u, sigma) (Eqs. 11-17, 28-33);
 *   CLB_MODEL_MRT:      the same with N = N_T = I, i.e. relaxation of the raw
 *                       moments toward the raw equilibria and forcing of
 *                       Eq. 19 and Eq. 33 (the MRT method of Section 2 and
 *                       Table 2);
 *   CLB_MODEL_BGK:      CLB_MODEL_MRT with every D2Q9 rate equal to s_v and
 *                       every D2Q5 rate equal to zeta_alpha (single relaxation
 *                       time; rate overrides are ignored). */
enum { CLB_MODEL_CASCADED = 0, CLB_MODEL_MRT = 1, CLB_MODEL_BGK = 2 };

/* How the lattice parameters follow from the dimensionless groups. */
enum {
  CLB_SCALE_CAVITY = 0,   /* relaxation rates of Eq. 46, u_c = Ma c_s (Section 3.2) */
  CLB_SCALE_CHANNEL = 1   /* 1/s_v = 1/2 + J H u_ref/(c_s^2 Re), Ra gives g beta (Section 3.1) */
};

/* Built-in per-row acceleration of a domain (clb_params.forcing).
 *   CLB_FORCING_NONE:      none;
 *   CLB_FORCING_INJECTION: the y-acceleration of Eq. 42 for the porous channel
 *     with injection of Section 3.1, so that its steady state is that of
 *     Eqs. 43-44.  On row y (0 .. ny-1, H = ny - 1), with the domain's derived
 *     nu, K = Da H^2, alpha_e and g beta dT, and u1 = bc_v[CLB_SOUTH] (the
 *     injection velocity):
 *       a_y(y) = (nu / K) u1 - g beta dT (exp(y u1 / alpha_e) - 1)
 *                                       / (exp(H u1 / alpha_e) - 1)
 *     (the last factor is y / H when u1 = 0).  Needs a uniform medium with
 *     Da > 0, else CLB_ERR_ARG.  Added to a_rows when both are given. */
enum { CLB_FORCING_NONE = 0, CLB_FORCING_INJECTION = 1 };

/*
 * Parameters of one domain.  A field left at 0 takes the paper's default or is
 * derived (Section 3: J = 1, varpi = 1/4, s0 = s1 = 1, s3 = 1.2,
 * s4 = 1.8, zeta_T = zeta_e = zeta_nu = 1; Eq. 46 or the channel relation for
 * s_v and zeta_alpha; Eq. 5 for F_phi).  The bulk rate s_b defaults to 1.5:
 * the paper's value is garbled, and the reading s_b = s_v makes the collision
 * linearly unstable for s_v < 1.19.  Call clb_params_default() first.
 */
typedef struct clb_params {
  int32_t nx, ny;            /* nodes including wall nodes; >= 4 on a walled axis;
                                ny * (nx rounded up to 64, or to 128 with FP16 planes)
                                <= 2^30 (a 32768^2 domain), else CLB_ERR_ARG          */
  int32_t bc[4];             /* side kinds W, E, S, N                                */
  double bc_u[4], bc_v[4];   /* wall velocity per side (lattice units)               */
  double bc_T[4];            /* Dirichlet temperature per side                       */
  double inlet_U;            /* mean velocity of a CLB_INLET side                    */

  /* porous medium (Eqs. 4-5) */
  double phi;                /* uniform porosity in (0, 1], used when eps == NULL    */
  const double *eps;         /* optional porosity per node (host, ny*nx); then
                                K = eps^3 dp^2 / (150 (1-eps)^2) and the Ergun F_phi
                                are evaluated per node (Eq. 5)                        */
  double dp;                 /* particle diameter for the eps field                  */
  double Da;                 /* uniform medium: K = Da Lc^2; <= 0 removes the drag   */
  double F_phi;              /* uniform medium: < 0 Ergun (Eq. 5), 0 none, > 0 value */

  /* dimensionless groups (Eq. 38) and scaling */
  int32_t scaling;           /* CLB_SCALE_*                                          */
  double Ra, Pr, Re, J, Gamma, sigma, Ma;
  double u_ref;              /* channel scaling: velocity in Re = H u_ref / nu       */
  double dT;                 /* temperature difference; default 1                   */
  double T0;                 /* Boussinesq reference temperature; default 0.5        */
  double g_dir[2];           /* unit vector of gravity; default (0, -1)              */
  double a[2];               /* external acceleration (lattice units)                */

  /* lattice overrides (> 0 replaces the derived value) */
  double nu;                 /* fluid viscosity in the Darcy term                    */
  double s_v, s_b, s1, s3, s4, zeta_a, zeta_e, zeta_nu, varpi;
  double gbeta;              /* g beta per unit temperature                           */

  double T_init;             /* initial uniform temperature; default T0              */
  int32_t storage;           /* CLB_STORE_*; must agree over all domains of a context */
  int32_t model;             /* CLB_MODEL_*: collision operator; default cascaded;
                                must agree over all domains of a context         */
  const double *a_rows;      /* optional acceleration per row (host, 2*ny values:
                                a_x, a_y of row y), added to a[] at every node of the
                                row; e.g. the y-dependent a_y of Eq. 42.  Copied
                                during clb_create; NULL for none                     */
  int32_t forcing;           /* CLB_FORCING_*: built-in per-row acceleration          */
} clb_params;

/* Lattice quantities derived from a clb_params (all lattice units). */
typedef struct clb_derived {
  double L;                  /* characteristic length: nx-1 (cavity) or ny-1 (channel) */
  double s_v, s_b, s1, s3, s4, zeta_a, zeta_e, zeta_nu, varpi;
  double nu_e, nu, alpha_e;  /* nu_e = c_s^2 (1/s_v - 1/2); alpha_e of Eq. 37       */
  double gbeta;              /* magnitude of g beta                                  */
  double K, F_phi;           /* uniform medium values (K = inf without drag)          */
  double sigma, T0, dT;
} clb_derived;

typedef struct clb_ctx clb_ctx;

/* Fill *p with the defaults above (square cavity scaling, hot W / cold E walls,
 * adiabatic S / N walls, phi = 1, no drag, FP32 storage, nx = ny = 0). */
void clb_params_default(clb_params *p);

/* Derive the lattice parameters of one domain (host only, no device work).
 * Errors: CLB_ERR_ARG for an invalid parameter set (N < 4 on a walled axis,
 * phi outside (0, 1], sigma <= 0, a relaxation rate outside (0, 2), varpi
 * outside (0, 1), mismatched periodic sides). */
clb_status clb_derive(const clb_params *p, clb_derived *out);

/* The per-row acceleration a domain will carry (host only): rows[2y] and
 * rows[2y + 1] receive a_x and a_y of row y (0 .. ny-1), the sum of
 * p->a_rows and the built-in forcing (clb_params.forcing; Eq. 42 for
 * CLB_FORCING_INJECTION); zeros for a domain with neither.  rows holds 2*ny
 * doubles owned by the caller.  Errors: CLB_ERR_ARG as for clb_derive, or
 * for a NULL pointer. */
clb_status clb_row_accel(const clb_params *p, double *rows);

/* Device bytes needed for `count` domains.  Pure host function. */
clb_status clb_workspace_bytes(const clb_params *p, int32_t count, size_t *bytes);

/* Create a context for `count` domains described by p[0..count-1] on the
 * caller's device workspace (256-byte aligned, >= clb_workspace_bytes) and
 * stream.  Host arrays referenced by p (eps, a_rows) are copied during the
 * call; a non-finite a_rows entry or eps outside (0, 1) is CLB_ERR_ARG.
 * All domains start at rest with T = T_init at every node.
 * Errors: CLB_ERR_ARG, CLB_ERR_WORKSPACE, CLB_ERR_HIP. */
clb_status clb_create(const clb_params *p, int32_t count, void *d_workspace, size_t bytes,
                      void *hip_stream, clb_ctx **out);

/* Enqueue n time steps of every active domain on the stream (asynchronous).
 * One time step (Section 2) is, per node: the populations streamed in (pull
 * form of Eqs. 18 and 35), the macroscopic values and the implicit velocity
 * (Eqs. 20-23 and 36, force of Eq. 4), the boundary reconstruction of wall,
 * inlet and outlet nodes, the D2Q9 cascaded collision with the porous shift
 * (Eqs. 11-17, A1) and the D2Q5 collision with the heat-capacity ratio
 * (Eqs. 28-33, A2).  The last step also records u, v, T for clb_residual.  A
 * kernel fault is reported here or by the next synchronizing call
 * (CLB_ERR_HIP). */
clb_status clb_step(clb_ctx *ctx, int64_t n);

/* Macroscopic fields of one domain at the current time (Eqs. 20-23, 36;
 * boundary nodes report the values used by their collision).  Any pointer may
 * be NULL.  Synchronizes. */
clb_status clb_macros(clb_ctx *ctx, int32_t cavity, double *rho, double *u, double *v,
                      double *T);

/* Mean Nusselt number on one side (CLB_WEST..CLB_NORTH), the heat-transfer
 * measure of Section 3.2 (the wall-normal temperature gradient scaled by L /
 * dT, averaged over the wall): second-order one-sided wall gradient,
 * trapezoid mean over the wall nodes, L and dT of the domain.  nu_local
 * (nullable) receives one value per wall node.  FP64.  Synchronizes. */
clb_status clb_nusselt(clb_ctx *ctx, int32_t cavity, int32_t side, double *nu_mean,
                       double *nu_local);

/* Mean Nusselt number on one side for every domain (count values). */
clb_status clb_nusselt_all(clb_ctx *ctx, int32_t side, double *nu_mean);

/* Relative change per step, r_u = |u^n - u^(n-k)|_2 / (k |u^n|_2) over (u, v),
 * r_T likewise on T, and the mass sum(rho), all in FP64.  k = 1 after
 * clb_step (the change between the last two steps); after clb_run, k is the
 * length of its last round.
 * Returns CLB_ERR_STATE before the first step and CLB_ERR_DIVERGED (with the
 * out-values set) when a field holds a non-finite value.  Synchronizes. */
clb_status clb_residual(clb_ctx *ctx, int32_t cavity, double *res_u, double *res_T,
                        double *mass);

/* Residuals of all domains: arrays of `count` values; status[i] is CLB_OK or
 * CLB_ERR_DIVERGED per domain (any array may be NULL). */
clb_status clb_residual_all(clb_ctx *ctx, double *res_u, double *res_T, double *mass,
                            int32_t *status);

/* Warm start: set every node of one domain to equilibrium, f = f^eq(rho = 1, u)
 * (Eq. 19) and g = g^eq(T, u) (Eq. 34).  NULL u or v means 0; T must be given.
 * The fields pass through FP32.  Synchronizes. */
clb_status clb_set_state(clb_ctx *ctx, int32_t cavity, const double *u, const double *v,
                         const double *T);

/* Warm start from device memory: the same equilibrium initialisation as
 * clb_set_state, from an FP32 device array holding, for node i = y*nx + x,
 * u = u_scale d_fields[i*stride], v = u_scale d_fields[i*stride + 1] and
 * T = T_offset + d_fields[i*stride + 2] (stride >= 3; e.g. a network output
 * with 16 channels per pixel).  Stream-ordered on the context's stream; no
 * synchronization: d_fields must be complete in stream order of the
 * context's stream (e.g. written on that stream) and stay allocated until the
 * work is done. */
clb_status clb_set_state_device(clb_ctx *ctx, int32_t cavity, const float *d_fields,
                                int64_t stride, double u_scale, double T_offset);

/* Choose which domains clb_step advances (active[i] != 0).  A domain that
 * stops has its current state copied into its second buffer, so it reads the
 * same (and later resumes from the same state) whatever the parity of the
 * steps the others take meanwhile.  Synchronizes. */
clb_status clb_set_active(clb_ctx *ctx, const uint8_t *active);

/* Run to steady state with retirement (batched stepping of many domains).
 * Advances the active domains in rounds of `check_every` steps, at most
 * `max_steps` steps in total.  After each round it evaluates, for every
 * domain still running, the relative change per step over the round (the
 * residual of clb_residual with k = the round length); a domain with
 * max(res_u, res_T) <= tol is retired (made inactive) with status CLB_OK, a
 * domain holding a non-finite value is retired with CLB_ERR_DIVERGED.  The
 * paper fixes no steady-state criterion.  Measuring the change over a whole
 * round rather than one step divides the noise floor that stochastic
 * rounding leaves in the single-step change (about 1e-7 in u and 1e-8 in T
 * with FP32 storage) by the round length, while a smooth approach to the
 * steady state gives nearly the same value either way.
 *   steps_taken[count]: steps this call advanced each domain;
 *   status[count]:      CLB_OK (steady), CLB_ERR_DIVERGED, CLB_NOT_CONVERGED
 *                       (still active after max_steps), or CLB_ERR_STATE for
 *                       a domain that was inactive at entry (0 steps);
 *   nu_record:          NULL, or count * max_records values (domain-major):
 *                       the mean Nusselt number of side `nu_side` after round
 *                       r (step (r+1) * check_every) for r < max_records, NaN
 *                       for rounds after the domain retired.  nu_side = -1
 *                       records nothing; otherwise no domain may have a
 *                       periodic side there.
 * Retired domains stay inactive on return (clb_set_active resumes them).
 * Returns CLB_ERR_ARG for invalid arguments (out-arrays untouched), a HIP
 * error if a launch or copy fails, CLB_OK otherwise.  Synchronizes after
 * every round. */
clb_status clb_run(clb_ctx *ctx, int64_t max_steps, int32_t check_every, double tol,
                   int32_t nu_side, double *nu_record, int32_t max_records,
                   int64_t *steps_taken, int32_t *status);

/* Byte-exact checkpoint of all population planes and the step counter.
 * clb_state_bytes gives the size of the host buffer.  Synchronizes. */
clb_status clb_state_bytes(clb_ctx *ctx, size_t *bytes);
clb_status clb_get_state(clb_ctx *ctx, void *host_buf, size_t bytes);
clb_status clb_put_state(clb_ctx *ctx, const void *host_buf, size_t bytes);

/* Time steps taken so far. */
clb_status clb_steps_done(clb_ctx *ctx, int64_t *steps);

/* Launch shape of the node kernels.  tile_x = tile_y = 0 (the default)
 * chooses per domain a tile width of 64, 128 or 256 nodes (the fewest idle
 * lanes per row, the wider on a tie) and stacks rows to 256 threads; otherwise
 * every work tile is tile_x * tile_y nodes (tile_x in {64, 128, 256},
 * tile_x * tile_y in {64, 128, 256, 512}).  One workgroup runs one tile at a
 * time, one thread per node; `blocks` workgroups loop over the tiles (0: one
 * workgroup per tile).  Results do not depend on the shape.  Re-captures the
 * step graph. */
clb_status clb_set_launch(clb_ctx *ctx, int32_t tile_x, int32_t tile_y, int32_t blocks);
clb_status clb_get_launch(clb_ctx *ctx, int32_t *tile_x, int32_t *tile_y, int32_t *blocks);

/* Time steps per kernel launch: 1 or 2 (else CLB_ERR_ARG); 2 is the default,
 * except with CLB_STORE_F16 when some domain is narrower than 128 nodes
 * (there one step per launch is faster).  With 2, the active domains
 * advance in pairs of steps per launch (domains that clb_run retires simply
 * drop out of the launch): each tile (128 x 8 nodes when every domain is at
 * least 128 wide, else 64 x 8) and a one-node ring around it are collided
 * into LDS, then the tile again from there, so that the populations cross
 * HBM once per two node updates.  The per-node arithmetic and rounding are
 * those of single steps in every storage mode: with CLB_STORE_F32, F16 and
 * MIXED the results have been bit-identical in every test; with
 * CLB_STORE_F32C the compiler's separate choices of fused multiply-adds in
 * the two kernels leave differences at the FP32 rounding level.  The
 * residual snapshot of clb_step is written by the last two-step launch; an
 * odd remainder, and the first step of each clb_run round (which records
 * that round's snapshot), run singly.  Re-captures the step graphs. */
clb_status clb_set_steps_per_launch(clb_ctx *ctx, int32_t steps);

/* The launch mode: steps per launch (1 or 2) and the width of the two-step
 * tiles in nodes: 64 or 128 when every domain uses that width, 0 when each
 * domain has its own (128 for the domains at least that wide, else 64; a
 * pair of steps then runs as one launch per width).  At creation: 128 when
 * every domain is at least that wide, else 64; clb_autotune may change it.
 * Either pointer may be NULL. */
clb_status clb_get_steps_per_launch(clb_ctx *ctx, int32_t *steps, int32_t *tile_x);

/* Time the step kernel over the candidate launch shapes on the live state
 * (which the timing runs advance) and keep the fastest; with two steps per
 * launch in effect, also time the two-step kernel with 64-wide tiles for
 * every domain, 128-wide tiles for every domain (when some domain is at
 * least 128 wide) and per-domain widths (when the widths are mixed), and keep
 * the fastest.  When cache_path is non-NULL the choice is read from /
 * appended to that text file (one line per context key: key, tile_x, tile_y,
 * blocks and, when timed, the two-step width: 64, 128, or 1 for per-domain),
 * keyed by storage and domain sizes.
 * Synchronizes. */
clb_status clb_autotune(clb_ctx *ctx, const char *cache_path);

/* Release the context (not the workspace, which the caller owns). */
void clb_destroy(clb_ctx *ctx);

const char *clb_strerror(clb_status s);

#ifdef __cplusplus
}
#endif
#endif /* CLB_H */
