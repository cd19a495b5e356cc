// Internal definitions shared by the host runtime (clb_api.cpp) and the
// kernels (clb_kernels.hip) of the GPU library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace clb {

// Side kinds, same numbering as the public CLB_* enum.
enum : int32_t { kPeriodic = 0, kWallT = 1, kWallAdiabatic = 2, kInlet = 3, kOutlet = 4 };

// Number of planes of one population buffer: 9 (D2Q9) + 5 (D2Q5).
constexpr int kPlanes = 14;
// Partial sums per tile / results per domain of the residual reduction:
// |du|^2, |u|^2, dT^2, T^2, sum(rho - 1), non-finite count, nodes, unused.
constexpr int kRed = 8;

// One work tile: domain index (-1: padding entry, skipped), the origin of a
// tile of nodes, and its index in the list of all tiles (the slot of its
// residual partial sums).
// One tile of a tile list.  id: the slot of the tile's partial sums (one-step
// lists); in the two-step list, 1 when the tile's LDS region reaches a node
// on or next to a side of its domain (boundary nodes, wrapped or skipped ring
// nodes: the general path), 0 for an interior tile.
struct Tile {
  int32_t cav, x0, y0, id;
};

// Per-domain constants in the arithmetic type T of a kernel.  The scalar
// fields are listed once (CLB_DOMAIN_SCALARS) so that the FP32 copy is made
// field by field from the FP64 one.
//   bc_u, bc_v, bc_th: boundary values; temperatures as theta = T - T0
//   inlet_U:  mean velocity of an inlet side
//   phi, ip:  uniform porosity and 1/phi (ignored with a porosity field)
//   cd, cf:   phi nu / K and phi F_phi / sqrt(K)
//   kc_d, kc_f: porosity field: cd = kc_d (1-eps)^2/eps^2, cf = kc_f (1-eps)/eps^2
//             (Kozeny-Carman K and the Ergun F_phi of Eq. 5)
//   s1c, s1f: 1 - s1, 1 - s1/2;  sp, sm: s+, s-;  svc: 1 - s_v (Eq. 15)
//   s3c, s3f: 1 - s3, (1 - s3/2)/3;  s4
//   zac, zec, znc: 1 - zeta_a, 1 - zeta_e, 1 - zeta_nu (Eq. 28)
//   hv:       varpi / 2 = c_sT^2;  sig, isig, sig_mv: sigma, 1/sigma, sigma - varpi
//   T0:       storage reference temperature
//   gbx, gby, ax, ay: body force G = gb theta + a
//   dT:       temperature difference of the Nusselt number
//   l0, l0sq, l1: uniform medium: the coefficients of Eq. 23, l0 = 1/2 + cd/4,
//             its square, and l1 = cf/2
#define CLB_DOMAIN_SCALARS(X)                                                              \
  X(inlet_U) X(phi) X(ip) X(cd) X(cf) X(kc_d) X(kc_f) X(s1c) X(s1f) X(sp) X(sm) X(svc)   \
  X(s3c) X(s3f) X(s4) X(zac) X(zec) X(znc) X(hv) X(sig) X(isig) X(sig_mv) X(T0) X(gbx)   \
  X(gby) X(ax) X(ay) X(dT) X(l0) X(l0sq) X(l1)

template <typename T>
struct DomainConsts {
  T bc_u[4], bc_v[4], bc_th[4];
#define CLB_DECLARE(n) T n;
  CLB_DOMAIN_SCALARS(CLB_DECLARE)
#undef CLB_DECLARE
  template <typename U>
  void assign(const DomainConsts<U> &o) {
    for (int s = 0; s < 4; ++s) {
      bc_u[s] = (T)o.bc_u[s];
      bc_v[s] = (T)o.bc_v[s];
      bc_th[s] = (T)o.bc_th[s];
    }
#define CLB_ASSIGN(n) n = (T)o.n;
    CLB_DOMAIN_SCALARS(CLB_ASSIGN)
#undef CLB_ASSIGN
  }
};

// Per-domain constants and addresses read by every kernel (scalar loads).
// Populations are stored as deviations from their rest values:
//   df_i = f_i - w_i,   dg_i = g_i - g_i^eq(T0, u = 0),
// where T0 here is the storage reference temperature (the initial temperature
// of the domain); the Boussinesq reference enters through the constant part
// of the body force (ax, ay).
struct alignas(16) CavDesc {
  int32_t nx, ny, pitch, plane;   // plane = ny * pitch elements
  int32_t bc[4];
  int32_t has_eps, tile0, ntiles;
  int32_t tw_log2;                // tiles of this domain are (1 << tw_log2) nodes wide
  char *A;                        // population planes, 14 planes (9 f, 5 g)
  char *B;                        // second buffer (A/B double buffering)
  const float *eps;               // porosity plane (pitch layout) or null
  const double *arow;             // (a_x, a_y) per row, added to (ax, ay), or null
  float *snap;                    // u, v, theta planes for the residual (pitch layout)

  // Constants of the domain: FP64, and rounded once to FP32 for the kernels
  // that compute in FP32 (cst<R>() picks the set).
  DomainConsts<double> c;
  DomainConsts<float> c32;
};

// Tile shape of the node kernels.  tile_x = 0 chooses the width per domain
// (the smallest of 64, 128, 256 that covers a row with the fewest idle
// lanes, rows stacked to 256 threads); otherwise every domain uses
// tile_x x tile_y.  Work-groups are flat: thread t of a tile handles node
// (x0 + t % width, y0 + t / width).  blocks = 0: one work-group per tile.
struct LaunchShape {
  int tile_x, tile_y, blocks;
  int threads() const { return tile_x ? tile_x * tile_y : 256; }
};

// Kernel launchers (clb_kernels.hip).  All return hipSuccess or the launch error.
// raw != 0: the raw-moment (MRT) collision instead of the cascaded one.
// rows != 0: some domain carries a per-row acceleration (CavDesc::arow).
hipError_t launch_step(const CavDesc *descs, const Tile *tiles, int32_t *counts,
                       int32_t grid_tiles, int parity, int write_snap, int storage, int raw,
                       int rows, LaunchShape shape, hipStream_t s);
// Two steps per launch over a list of tile_x x kFusedY tiles (any storage
// mode), tile_x = kFusedX (64) or kFusedXWide (128; the kernel masks the
// nodes of a domain narrower than the tile); the list holds the tiles of the
// active domains and may hold padding entries (cav = -1).  ntiles is the grid
// (workgroups); the kernel reads the list length from *len (a device int).
// A context may run two such launches per pair of steps, one per tile width,
// over disjoint sets of domains.  write_snap records (u, v, theta) of the
// second step for the residual.
constexpr int kFusedX = 64, kFusedXWide = 128, kFusedY = 8;
hipError_t launch_step2(const CavDesc *descs, const Tile *tiles, int32_t ntiles, int32_t *counts,
                        const int32_t *len, int parity, int write_snap, int storage, int raw,
                        int rows, int tile_x, hipStream_t s);
hipError_t launch_init(const CavDesc *descs, int32_t cav, int nx, int ny, int parity,
                       const float *uvth /* 3 dense planes or null */, float th_uniform,
                       int storage, hipStream_t s);
// Partial sums of the tiles in `tiles` (padding entries skipped) go to slot
// tiles[t].id of `partials`.
hipError_t launch_residual(const CavDesc *descs, const Tile *tiles, int32_t ntiles, int parity,
                           double *partials, int storage, LaunchShape shape, hipStream_t s);
// Per-domain totals of the partial sums (two fixed-order passes through
// gpart, max_groups >= ceil(ntiles / 256) of every domain).
hipError_t launch_residual_finalize(const CavDesc *descs, int32_t count, int32_t max_groups,
                                    const double *partials, double *gpart, double *results,
                                    hipStream_t s);
hipError_t launch_macros(const CavDesc *descs, const Tile *tiles, int32_t tile0, int32_t ntiles,
                         int parity, float *out /* 4 dense planes */, int storage,
                         LaunchShape shape, hipStream_t s);
// Mean Nusselt number of domains cav0 .. cav0 + ncav - 1 on one side; chunks
// of 256 wall nodes go through nu_part (max_chunks per domain).
hipError_t launch_nusselt(const CavDesc *descs, int32_t cav0, int32_t ncav, int32_t side,
                          int parity, double *nu_mean, double *nu_local, double *nu_part,
                          int32_t max_chunks, int storage, hipStream_t s);

// (clb_state.hip) planes[0..n) = u_scale src[i*stride], planes[n..2n) =
// u_scale src[i*stride + 1], planes[2n..3n) = th_offset + src[i*stride + 2].
hipError_t launch_uvT_planes(const float *src, int64_t stride, int64_t n, double u_scale,
                             double th_offset, float *planes, hipStream_t s);

}  // namespace clb
