// Host runtime of the porous-media cascaded lattice Boltzmann library: the
// C ABI of include/clb.h.  Derives the lattice parameters of each domain from
// the paper's dimensionless groups, lays the caller's device workspace out,
// builds the work-tile lists, captures the time step into HIP graphs and runs
// the reductions.  It never allocates device memory.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <limits>
#include <sstream>
#include <string>
#include <vector>

#include "clb.h"
#include "clb_internal.h"

using clb::CavDesc;
using clb::LaunchShape;
using clb::Tile;

namespace {

thread_local std::string g_last_error;

constexpr size_t kAlign = 256;
constexpr int kGraphSteps = 32;  // steps per captured graph (even)
constexpr double kCs2 = 1.0 / 3.0;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

clb_status hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return CLB_ERR_HIP;
}

#define HIPCHK(expr)                                  \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) return hip_fail(_e, #expr); \
  } while (0)

bool walled_x(const clb_params &p) { return p.bc[0] != CLB_PERIODIC; }
bool walled_y(const clb_params &p) { return p.bc[2] != CLB_PERIODIC; }

// Bytes of the 9 D2Q9 planes and of the 5 D2Q5 planes per element.
bool f32_planes(int storage) { return storage == CLB_STORE_F32 || storage == CLB_STORE_F32C; }
int fbytes(int storage) { return f32_planes(storage) ? 4 : 2; }
int gbytes(int storage) { return storage == CLB_STORE_F16 ? 2 : 4; }
// Bytes of one population buffer per plane element (all 14 planes).
size_t pop_bytes(int storage) { return 9 * (size_t)fbytes(storage) + 5 * (size_t)gbytes(storage); }

// Row pitch in elements: every row starts on a 256-byte boundary.
int pitch_of(const clb_params &p) {
  const int per = f32_planes(p.storage) ? 64 : 128;
  return (p.nx + per - 1) / per * per;
}

}  // namespace

// ------------------------------------------------------------ derivation

extern "C" void clb_params_default(clb_params *p) {
  std::memset(p, 0, sizeof(*p));
  p->bc[0] = CLB_WALL_T;
  p->bc[1] = CLB_WALL_T;
  p->bc[2] = CLB_WALL_ADIABATIC;
  p->bc[3] = CLB_WALL_ADIABATIC;
  p->bc_T[0] = 1.0;
  p->bc_T[1] = 0.0;
  p->phi = 1.0;
  p->F_phi = 0.0;
  p->scaling = CLB_SCALE_CAVITY;
  p->J = 1.0;
  p->Gamma = 1.0;
  p->sigma = 1.0;
  p->Ma = 0.1;
  p->dT = 1.0;
  p->T0 = 0.5;
  p->g_dir[0] = 0.0;
  p->g_dir[1] = -1.0;
  p->T_init = 0.5;
  p->storage = CLB_STORE_F32;
}

static bool rate_ok(double s) { return s > 0.0 && s < 2.0; }

// Relations used (Feng, Liu & He, arXiv:2110.05943):
//   nu_e = c_s^2 (1/s_v - 1/2), below Eq. 15;  J = nu_e / nu, Eq. 38;
//   alpha_e = c_sT^2 (1/zeta_a - 1/2), Eq. 37, c_sT^2 = varpi/2 (Eq. 34);
//   cavity: Eq. 46 for 1/s_v and 1/zeta_a, and u_c = sqrt(g beta dT L) = Ma c_s;
//   channel (Section 3.1): 1/s_v = 1/2 + J H u_ref/(c_s^2 Re), the same
//   zeta_a relation, and g beta dT = Ra nu alpha / H^3 from Eq. 38;
//   Da = K / L^2 (Eq. 38); F_phi of Eq. 5; defaults of Section 3.
extern "C" clb_status clb_derive(const clb_params *pp, clb_derived *out) {
  if (!pp || !out) return CLB_ERR_ARG;
  const clb_params &p = *pp;
  if (p.nx < 3 || p.ny < 3) return CLB_ERR_ARG;
  for (int s = 0; s < 4; ++s)
    if (p.bc[s] < CLB_PERIODIC || p.bc[s] > CLB_OUTLET) return CLB_ERR_ARG;
  if ((p.bc[0] == CLB_PERIODIC) != (p.bc[1] == CLB_PERIODIC)) return CLB_ERR_ARG;
  if ((p.bc[2] == CLB_PERIODIC) != (p.bc[3] == CLB_PERIODIC)) return CLB_ERR_ARG;
  if (walled_x(p) && p.nx < 4) return CLB_ERR_ARG;
  if (walled_y(p) && p.ny < 4) return CLB_ERR_ARG;
  // The kernels address a plane with 32-bit element indices and 32-bit byte
  // offsets from the plane base: at most 2^30 elements (a 32768^2 domain).
  if (p.nx > (1 << 30) || p.ny > (1 << 30)) return CLB_ERR_ARG;
  if ((int64_t)p.ny * pitch_of(p) > (int64_t(1) << 30)) return CLB_ERR_ARG;
  if (p.model < CLB_MODEL_CASCADED || p.model > CLB_MODEL_BGK) return CLB_ERR_ARG;
  if (p.storage != CLB_STORE_F32 && p.storage != CLB_STORE_F16 && p.storage != CLB_STORE_MIXED &&
      p.storage != CLB_STORE_F32C)
    return CLB_ERR_ARG;
  if (p.scaling != CLB_SCALE_CAVITY && p.scaling != CLB_SCALE_CHANNEL) return CLB_ERR_ARG;
  if (!p.eps && !(p.phi > 0.0 && p.phi <= 1.0)) return CLB_ERR_ARG;
  if (p.forcing != CLB_FORCING_NONE && p.forcing != CLB_FORCING_INJECTION) return CLB_ERR_ARG;
  if (p.forcing == CLB_FORCING_INJECTION && (p.eps || !(p.Da > 0.0))) return CLB_ERR_ARG;
  if (p.eps && !(p.dp > 0.0)) return CLB_ERR_ARG;

  clb_derived d;
  std::memset(&d, 0, sizeof(d));
  const double J = p.J > 0 ? p.J : 1.0;
  const double Gamma = p.Gamma > 0 ? p.Gamma : 1.0;
  const double Ma = p.Ma > 0 ? p.Ma : 0.1;
  d.sigma = p.sigma > 0 ? p.sigma : 1.0;
  d.varpi = p.varpi > 0 ? p.varpi : 0.25;
  if (!(d.varpi < 1.0)) return CLB_ERR_ARG;
  d.T0 = p.T0;
  d.dT = p.dT > 0 ? p.dT : 1.0;
  const bool channel = p.scaling == CLB_SCALE_CHANNEL;
  d.L = channel ? p.ny - 1 : p.nx - 1;
  const double cT2 = 0.5 * d.varpi;

  if (p.s_v > 0) {
    d.s_v = p.s_v;
  } else if (!channel) {
    if (!(p.Ra > 0 && p.Pr > 0)) return CLB_ERR_ARG;
    d.s_v = 1.0 / (0.5 + Ma * J * d.L * std::sqrt(3.0 * p.Pr) / std::sqrt(p.Ra));
  } else {
    if (!(p.Re > 0 && p.u_ref > 0)) return CLB_ERR_ARG;
    d.s_v = 1.0 / (0.5 + J * d.L * p.u_ref / (kCs2 * p.Re));
  }
  d.nu_e = kCs2 * (1.0 / d.s_v - 0.5);
  d.nu = p.nu > 0 ? p.nu : d.nu_e / J;
  if (p.zeta_a > 0) {
    d.zeta_a = p.zeta_a;
  } else {
    if (!(p.Pr > 0)) return CLB_ERR_ARG;
    d.zeta_a = 1.0 / (0.5 + Gamma * kCs2 * (1.0 / d.s_v - 0.5) / (J * cT2 * p.Pr));
  }
  d.alpha_e = cT2 * (1.0 / d.zeta_a - 0.5);
  if (p.gbeta > 0) {
    d.gbeta = p.gbeta;
  } else if (!channel) {
    d.gbeta = p.Ra > 0 ? Ma * Ma * kCs2 / d.L / d.dT : 0.0;
  } else {
    const double alpha = p.Pr > 0 ? d.nu / p.Pr : 0.0;
    d.gbeta = p.Ra > 0 ? p.Ra * d.nu * alpha / (d.L * d.L * d.L) / d.dT : 0.0;
  }
  // The bulk rate is garbled in the paper's list of rates; read literally as
  // s_b = s_v, the collision of Eqs. 11-17 with s3 = 1.2, s4 = 1.8 is linearly
  // unstable at rest whenever s_v < 1.19.  s_b = 1.5 lies in the band where it
  // is stable for every s_v in (0.6, 2); s_b only sets the bulk viscosity.
  d.s_b = p.s_b > 0 ? p.s_b : 1.5;
  d.s1 = p.s1 > 0 ? p.s1 : 1.0;
  d.s3 = p.s3 > 0 ? p.s3 : 1.2;
  d.s4 = p.s4 > 0 ? p.s4 : 1.8;
  d.zeta_e = p.zeta_e > 0 ? p.zeta_e : 1.0;
  d.zeta_nu = p.zeta_nu > 0 ? p.zeta_nu : 1.0;
  if (p.model == CLB_MODEL_BGK) {  // single relaxation time
    d.s_b = d.s1 = d.s3 = d.s4 = d.s_v;
    d.zeta_e = d.zeta_nu = d.zeta_a;
  }
  if (!rate_ok(d.s_v) || !rate_ok(d.s_b) || !rate_ok(d.s1) || !rate_ok(d.s3) || !rate_ok(d.s4) ||
      !rate_ok(d.zeta_a) || !rate_ok(d.zeta_e) || !rate_ok(d.zeta_nu))
    return CLB_ERR_ARG;
  d.K = p.Da > 0 ? p.Da * d.L * d.L : std::numeric_limits<double>::infinity();
  const double phi = p.eps ? 0.0 : p.phi;
  if (p.F_phi < 0)
    d.F_phi = p.eps ? -1.0 : 1.75 / std::sqrt(150.0 * phi * phi * phi);
  else
    d.F_phi = p.F_phi;
  *out = d;
  return CLB_OK;
}

namespace {
bool has_rows(const clb_params &p) { return p.a_rows || p.forcing != CLB_FORCING_NONE; }

// Per-row acceleration (a_x, a_y) of a domain: the caller's a_rows plus the
// built-in forcing.  CLB_FORCING_INJECTION: Eq. 42 (Section 3.1) from the
// derived nu, K, alpha_e and g beta dT, with u1 the injection velocity of the
// south side.
std::vector<double> row_accel(const clb_params &p, const clb_derived &d) {
  const size_t ny = (size_t)p.ny;
  std::vector<double> h(2 * ny, 0.0);
  if (p.a_rows) std::copy(p.a_rows, p.a_rows + 2 * ny, h.begin());
  if (p.forcing == CLB_FORCING_INJECTION) {
    const double H = p.ny - 1, u1 = p.bc_v[CLB_SOUTH], k = u1 / d.alpha_e;
    const double gbdT = d.gbeta * d.dT;
    for (size_t y = 0; y < ny; ++y) {
      const double prof = k != 0.0 ? std::expm1((double)y * k) / std::expm1(H * k) : y / H;
      h[2 * y + 1] += d.nu / d.K * u1 - gbdT * prof;
    }
  }
  return h;
}
}  // namespace

extern "C" clb_status clb_row_accel(const clb_params *p, double *rows) {
  if (!p || !rows) return CLB_ERR_ARG;
  clb_derived d;
  const clb_status s = clb_derive(p, &d);
  if (s != CLB_OK) return s;
  const std::vector<double> h = row_accel(*p, d);
  std::copy(h.begin(), h.end(), rows);
  return CLB_OK;
}

// --------------------------------------------------------------- layout

namespace {

struct Layout {
  size_t desc, tiles_all, tiles_active, tiles2, counts, partials, gpart, results, nu, nu_local,
      nu_part, obs;
  std::vector<size_t> A, B, eps, arow, snap;
  size_t total;
  size_t max_tiles, max_tiles2, obs_elems, max_wall;
  int32_t max_chunks;
};

size_t max_tiles_of(const clb_params &p) {
  // smallest tile is 64 x 1
  return (size_t)((p.nx + 63) / 64) * p.ny;
}

// Tiles of the two-step kernel in one domain (the narrow tiles: an upper
// bound for either width).
size_t tiles2_of(const clb_params &p) {
  return (size_t)((p.nx + clb::kFusedX - 1) / clb::kFusedX) *
         ((p.ny + clb::kFusedY - 1) / clb::kFusedY);
}

Layout make_layout(const clb_params *p, int count) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, kAlign);
    return o;
  };
  L.max_tiles = 0;
  L.max_tiles2 = 0;
  L.obs_elems = 0;
  L.max_wall = 0;
  for (int c = 0; c < count; ++c) {
    L.max_tiles += max_tiles_of(p[c]);
    L.max_tiles2 += tiles2_of(p[c]);
    L.obs_elems = std::max(L.obs_elems, (size_t)p[c].nx * p[c].ny);
    L.max_wall = std::max(L.max_wall, (size_t)std::max(p[c].nx, p[c].ny));
  }
  L.desc = take(sizeof(CavDesc) * count);
  L.tiles_all = take(sizeof(Tile) * L.max_tiles);
  L.tiles_active = take(sizeof(Tile) * (L.max_tiles + 8));
  L.tiles2 = take(sizeof(Tile) * 2 * (L.max_tiles2 + 8));  // a 64- and a 128-wide list
  L.counts = take(sizeof(int32_t) * 6);
  L.partials = take(sizeof(double) * clb::kRed * L.max_tiles);
  L.gpart = take(sizeof(double) * clb::kRed * L.max_tiles);
  L.results = take(sizeof(double) * clb::kRed * count);
  L.nu = take(sizeof(double) * count);
  L.nu_local = take(sizeof(double) * L.max_wall);
  L.max_chunks = (int32_t)((L.max_wall + 255) / 256);
  L.nu_part = take(sizeof(double) * (size_t)L.max_chunks * count);
  L.obs = take(sizeof(float) * 4 * L.obs_elems);
  for (int c = 0; c < count; ++c) {
    const size_t plane = (size_t)p[c].ny * pitch_of(p[c]);
    const size_t pop = plane * pop_bytes(p[c].storage);
    L.A.push_back(take(pop));
    L.B.push_back(take(pop));
    L.eps.push_back(p[c].eps ? take(plane * sizeof(float)) : 0);
    L.arow.push_back(has_rows(p[c]) ? take(2 * (size_t)p[c].ny * sizeof(double)) : 0);
    L.snap.push_back(take(3 * plane * sizeof(float)));
  }
  L.total = off;
  return L;
}

}  // namespace

extern "C" clb_status clb_workspace_bytes(const clb_params *p, int32_t count, size_t *bytes) {
  if (!p || count <= 0 || !bytes) return CLB_ERR_ARG;
  for (int c = 0; c < count; ++c) {
    clb_derived d;
    const clb_status s = clb_derive(&p[c], &d);
    if (s != CLB_OK) return s;
    if (p[c].storage != p[0].storage) return CLB_ERR_ARG;
  }
  *bytes = make_layout(p, count).total;
  return CLB_OK;
}

// ---------------------------------------------------------------- context

struct clb_ctx {
  int count = 0;
  int storage = 0;
  int raw = 0;   // raw-moment (MRT / BGK) collision
  int rows = 0;  // some domain has a per-row acceleration
  int fused = 0;  // two steps per launch (FP32 planes, all domains active)
  std::vector<clb_params> p;
  std::vector<clb_derived> der;
  std::vector<CavDesc> desc;
  Layout lay;
  char *ws = nullptr;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  CavDesc *d_desc = nullptr;
  Tile *d_tiles_all = nullptr, *d_tiles_active = nullptr;
  // Two-step tile lists, [0] of 64-wide and [1] of 128-wide tiles.  Their
  // grids (ntiles2) are the XCD-ordered list lengths over all domains of that
  // width; the lists hold the active domains (lengths in counts[4 + i], which
  // the kernel reads, so graphs survive retirement).
  Tile *d_tiles2[2] = {nullptr, nullptr};
  int32_t ntiles2[2] = {0, 0};
  // two-step tile width: 0 = per domain (128 for domains at least 128 wide,
  // else 64), or 64 / 128 for every domain
  int tile2_mode = 0;
  int32_t *d_counts = nullptr;
  double *d_partials = nullptr, *d_gpart = nullptr, *d_results = nullptr, *d_nu = nullptr,
         *d_nu_local = nullptr, *d_nu_part = nullptr;
  float *d_obs = nullptr;
  std::vector<Tile> tiles_all, tiles_active;
  std::vector<int32_t> tile0, ntiles;
  std::vector<uint8_t> active;
  LaunchShape shape{0, 0, 0};
  int64_t steps = 0;
  int parity = 0;
  bool snap_valid = false;
  int64_t snap_span = 1;  // steps between the snapshot and the current state
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t graph2[2] = {nullptr, nullptr};  // two-step launches
};

namespace {

void drop_graphs(clb_ctx *c) {
  for (auto *set : {c->graph, c->graph2})
    for (int k = 0; k < 2; ++k)
      if (set[k]) {
        (void)hipGraphExecDestroy(set[k]);
        set[k] = nullptr;
      }
}

void fill_desc(const clb_params &p, const clb_derived &d, CavDesc &k) {
  std::memset(&k, 0, sizeof(k));
  k.nx = p.nx;
  k.ny = p.ny;
  k.pitch = pitch_of(p);
  k.plane = k.pitch * p.ny;
  // Deviations of the D2Q5 populations are stored about the initial
  // temperature Ts; theta in the kernels is T - Ts, and the Boussinesq
  // reference T0 enters as the constant force -g beta (Ts - T0).
  const double Ts = p.T_init;
  for (int s = 0; s < 4; ++s) {
    k.bc[s] = p.bc[s];
    k.c.bc_u[s] = p.bc_u[s];
    k.c.bc_v[s] = p.bc_v[s];
    k.c.bc_th[s] = (p.bc_T[s] - Ts);
  }
  k.c.inlet_U = p.inlet_U;
  k.has_eps = p.eps != nullptr;
  const double phi = p.eps ? 1.0 : p.phi;
  k.c.phi = phi;
  k.c.ip = (1.0 / phi);
  const bool drag = std::isfinite(d.K);
  k.c.cd = drag ? (phi * d.nu / d.K) : 0.0;
  k.c.cf = drag ? (phi * d.F_phi / std::sqrt(d.K)) : 0.0;
  k.c.l0 = 0.5 + 0.25 * k.c.cd;
  k.c.l0sq = k.c.l0 * k.c.l0;
  k.c.l1 = 0.5 * k.c.cf;
  if (p.eps) {
    k.c.kc_d = (150.0 * d.nu / (p.dp * p.dp));
    k.c.kc_f = p.F_phi == 0.0 ? 0.0 : (1.75 / p.dp);
  }
  k.c.s1c = (1.0 - d.s1);
  k.c.s1f = (1.0 - 0.5 * d.s1);
  k.c.sp = (0.5 * (d.s_b + d.s_v));
  k.c.sm = (0.5 * (d.s_b - d.s_v));
  k.c.svc = (1.0 - d.s_v);
  k.c.s3c = (1.0 - d.s3);
  k.c.s3f = ((1.0 - 0.5 * d.s3) / 3.0);
  k.c.s4 = d.s4;
  k.c.zac = (1.0 - d.zeta_a);
  k.c.zec = (1.0 - d.zeta_e);
  k.c.znc = (1.0 - d.zeta_nu);
  k.c.hv = (0.5 * d.varpi);
  k.c.sig = d.sigma;
  k.c.isig = (1.0 / d.sigma);
  k.c.sig_mv = (d.sigma - d.varpi);
  k.c.T0 = Ts;
  const double gbx = -p.g_dir[0] * d.gbeta, gby = -p.g_dir[1] * d.gbeta;
  k.c.gbx = gbx;
  k.c.gby = gby;
  k.c.ax = (p.a[0] + gbx * (Ts - d.T0));
  k.c.ay = (p.a[1] + gby * (Ts - d.T0));
  k.c.dT = d.dT;
  k.c32.assign(k.c);
}

// Tile width for a row of nx nodes when the shape is chosen per domain: the
// fewest idle lanes per row, the wider width on a tie.
int auto_width(int nx) {
  int best = 64;
  long best_idle = -1;
  for (int w : {64, 128, 256}) {
    const long idle = (long)((nx + w - 1) / w) * w - nx;
    if (best_idle < 0 || idle <= best_idle) {
      best = w;
      best_idle = idle;
    }
  }
  return best;
}

int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// All tiles of every domain in domain order.
void build_tiles(clb_ctx *c) {
  c->tiles_all.clear();
  c->tile0.assign(c->count, 0);
  c->ntiles.assign(c->count, 0);
  for (int k = 0; k < c->count; ++k) {
    const int tx = c->shape.tile_x ? c->shape.tile_x : auto_width(c->p[k].nx);
    const int ty = c->shape.tile_x ? c->shape.tile_y : 256 / tx;
    c->desc[k].tw_log2 = log2i(tx);
    c->tile0[k] = (int32_t)c->tiles_all.size();
    for (int y0 = 0; y0 < c->p[k].ny; y0 += ty)
      for (int x0 = 0; x0 < c->p[k].nx; x0 += tx)
        c->tiles_all.push_back(Tile{k, x0, y0, (int32_t)c->tiles_all.size()});
    c->ntiles[k] = (int32_t)c->tiles_all.size() - c->tile0[k];
    c->desc[k].tile0 = c->tile0[k];
    c->desc[k].ntiles = c->ntiles[k];
  }
}

// Work-groups are dispatched round-robin over the XCDs (8 on gfx950), so
// work-group b runs on XCD b % 8.  The active list is laid out so that each
// XCD receives one contiguous run of tiles: neighbouring tiles share the
// cache lines at their edges (the x-shifted pulls), and those lines then hit
// in that XCD's L2 instead of being fetched once per XCD.  Padding entries
// (cav = -1) are skipped by the kernel.
constexpr int kXcds = 8;

clb_status upload_tiles(clb_ctx *c) {
  std::vector<Tile> order;
  for (int k = 0; k < c->count; ++k)
    if (c->active[k])
      order.insert(order.end(), c->tiles_all.begin() + c->tile0[k],
                   c->tiles_all.begin() + c->tile0[k] + c->ntiles[k]);
  c->tiles_active.clear();
  if (c->shape.blocks == 0 && !order.empty()) {
    const size_t n = order.size(), m = (n + kXcds - 1) / kXcds;
    c->tiles_active.assign(m * kXcds, Tile{-1, 0, 0, 0});
    for (size_t b = 0; b < m * kXcds; ++b) {
      const size_t t = (b % kXcds) * m + b / kXcds;
      if (t < n) c->tiles_active[b] = order[t];
    }
  } else {
    c->tiles_active = order;
  }
  // counts: active list length, all tiles, step index for parity 0 / parity 1
  int32_t counts[4] = {(int32_t)c->tiles_active.size(), (int32_t)c->tiles_all.size(),
                       (int32_t)c->steps, (int32_t)c->steps};
  HIPCHK(hipMemcpyAsync(c->d_desc, c->desc.data(), sizeof(CavDesc) * c->count,
                        hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->d_tiles_all, c->tiles_all.data(), sizeof(Tile) * c->tiles_all.size(),
                        hipMemcpyHostToDevice, c->stream));
  if (!c->tiles_active.empty())
    HIPCHK(hipMemcpyAsync(c->d_tiles_active, c->tiles_active.data(),
                          sizeof(Tile) * c->tiles_active.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->d_counts, counts, sizeof(counts), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return CLB_OK;
}

// Origin of tile i of a two-step tiling along an axis of n nodes: the last
// tile ends at the last node (it overlaps its neighbour when n is not a
// multiple of the tile).  The boundary reconstruction of step two gathers up
// to three nodes inward from a wall; with the wall at the far end of its tile
// those nodes stay inside the tile's LDS region.  Overlapping nodes are
// computed by both tiles with identical results.
int tile2_origin(int i, int tile, int n) { return n >= tile ? std::min(i * tile, n - tile) : 0; }

// Width of domain k's two-step tiles.
int tile2_width(const clb_ctx *c, int k) {
  if (c->tile2_mode) return c->tile2_mode;
  return c->p[k].nx >= clb::kFusedXWide ? clb::kFusedXWide : clb::kFusedX;
}

// The two-step tile lists, one per tile width: every tile of every active
// domain of that width, laid out for the XCDs like the active list, with the
// lengths in counts[4] (64-wide) and counts[5] (128-wide).
clb_status upload_tiles2(clb_ctx *c) {
  for (int wi = 0; wi < 2; ++wi) {
    const int w = wi ? clb::kFusedXWide : clb::kFusedX, h = clb::kFusedY;
    std::vector<Tile> order;
    size_t all = 0;
    for (int k = 0; k < c->count; ++k) {
      if (tile2_width(c, k) != w) continue;
      const int nx = c->p[k].nx, ny = c->p[k].ny;
      const int tx = (nx + w - 1) / w;
      const int ty = (ny + h - 1) / h;
      all += (size_t)tx * ty;
      if (!c->active[k]) continue;
      for (int j = 0; j < ty; ++j)
        for (int i = 0; i < tx; ++i) {
          const int x0 = tile2_origin(i, w, nx), y0 = tile2_origin(j, h, ny);
          // interior: the region [x0 - 1, x0 + w] x [y0 - 1, y0 + h] lies in
          // [1, nx - 2] x [1, ny - 2], so its pulls stay inside the domain
          const bool interior = x0 >= 2 && x0 + w <= nx - 2 && y0 >= 2 && y0 + h <= ny - 2;
          order.push_back(Tile{k, x0, y0, interior ? 0 : 1});
        }
    }
    const size_t n = order.size(), m = (n + kXcds - 1) / kXcds;
    std::vector<Tile> list(m * kXcds, Tile{-1, 0, 0, 0});
    for (size_t b = 0; b < m * kXcds; ++b) {
      const size_t t = (b % kXcds) * m + b / kXcds;
      if (t < n) list[b] = order[t];
    }
    c->ntiles2[wi] = (int32_t)((all + kXcds - 1) / kXcds * kXcds);
    const int32_t n2 = (int32_t)list.size();
    if (!list.empty())
      HIPCHK(hipMemcpyAsync(c->d_tiles2[wi], list.data(), sizeof(Tile) * list.size(),
                            hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->d_counts + 4 + wi, &n2, sizeof(n2), hipMemcpyHostToDevice,
                          c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  return CLB_OK;
}

bool fused_now(const clb_ctx *c) {
  if (!c->fused) return false;
  for (int k = 0; k < c->count; ++k)
    if (c->active[k]) return true;
  return false;
}

bool shape_ok(int tx, int ty) {
  if (tx == 0 && ty == 0) return true;  // width chosen per domain
  if (tx != 64 && tx != 128 && tx != 256) return false;
  const int n = tx * ty;
  return ty >= 1 && (n == 64 || n == 128 || n == 256 || n == 512);
}

// Grid of the step kernel: the padded list length (<= all tiles + 7).
int grid_tiles(const clb_ctx *c) {
  const size_t n = c->tiles_all.size();
  return (int)((n + kXcds - 1) / kXcds * kXcds);
}

clb_status launch_one(clb_ctx *c, int write_snap, hipStream_t s) {
  const hipError_t e =
      clb::launch_step(c->d_desc, c->d_tiles_active, c->d_counts, grid_tiles(c), c->parity,
                       write_snap, c->storage, c->raw, c->rows, c->shape, s);
  if (e != hipSuccess) return hip_fail(e, "step kernel launch");
  return CLB_OK;
}

// The two-step launches of one pair of steps (one per tile width in use).
hipError_t launch_two_lists(clb_ctx *c, int parity, int write_snap, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (int wi = 0; wi < 2 && e == hipSuccess; ++wi)
    if (c->ntiles2[wi] > 0)
      e = clb::launch_step2(c->d_desc, c->d_tiles2[wi], c->ntiles2[wi], c->d_counts,
                            c->d_counts + 4 + wi, parity, write_snap, c->storage, c->raw,
                            c->rows, wi ? clb::kFusedXWide : clb::kFusedX, s);
  return e;
}

clb_status launch_two(clb_ctx *c, int write_snap, hipStream_t s) {
  const hipError_t e = launch_two_lists(c, c->parity, write_snap, s);
  if (e != hipSuccess) return hip_fail(e, "two-step kernel launch");
  return CLB_OK;
}

clb_status capture_graph(clb_ctx *c, int p0) {
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t err = hipSuccess;
  // kGraphSteps steps: single-step launches, or half as many two-step ones
  const bool two = fused_now(c);
  const int launches = two ? kGraphSteps / 2 : kGraphSteps;
  for (int k = 0; k < launches && err == hipSuccess; ++k)
    err = two ? launch_two_lists(c, (p0 + k) & 1, 0, c->cap_stream)
              : clb::launch_step(c->d_desc, c->d_tiles_active, c->d_counts, grid_tiles(c),
                                 (p0 + k) & 1, 0, c->storage, c->raw, c->rows, c->shape,
                                 c->cap_stream);
  const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
  if (err != hipSuccess) return hip_fail(err, "graph capture launch");
  if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
  hipGraphExec_t &slot = two ? c->graph2[p0] : c->graph[p0];
  const hipError_t e3 = hipGraphInstantiate(&slot, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e3 != hipSuccess) {
    slot = nullptr;
    return hip_fail(e3, "hipGraphInstantiate");
  }
  return CLB_OK;
}

}  // namespace

extern "C" clb_status clb_create(const clb_params *p, int32_t count, void *d_workspace,
                                 size_t bytes, void *hip_stream, clb_ctx **out) {
  if (!p || count <= 0 || !out) return CLB_ERR_ARG;
  std::vector<clb_derived> der(count);
  for (int k = 0; k < count; ++k) {
    const clb_status s = clb_derive(&p[k], &der[k]);
    if (s != CLB_OK) return s;
    if (p[k].storage != p[0].storage || p[k].model != p[0].model) return CLB_ERR_ARG;
    if (p[k].a_rows)
      for (size_t i = 0; i < 2 * (size_t)p[k].ny; ++i)
        if (!std::isfinite(p[k].a_rows[i])) return CLB_ERR_ARG;
  }
  Layout lay = make_layout(p, count);
  if (!d_workspace || bytes < lay.total || ((uintptr_t)d_workspace % kAlign) != 0)
    return CLB_ERR_WORKSPACE;

  clb_ctx *c = new clb_ctx();
  c->count = count;
  c->storage = p[0].storage;
  c->raw = p[0].model != CLB_MODEL_CASCADED;
  // 128-wide two-step tiles (fewer partly used cache lines at the tile
  // edges) when no domain would leave most of such a tile idle, else 64-wide
  // ones for every domain (per-domain widths, two launches per pair of steps,
  // measured slower on the 256-cavity batch; clb_autotune times them)
  c->tile2_mode = clb::kFusedXWide;
  for (int k = 0; k < count; ++k)
    if (p[k].nx < clb::kFusedXWide) c->tile2_mode = clb::kFusedX;
  // two steps per launch by default; all-FP16 storage only with 128-wide
  // tiles (its 64-wide two-step kernel, without the interior-tile path, loses
  // to its one-step kernel on the batch of small domains: 470 against 2 x 227
  // us; with 128-wide tiles it wins on the 4096^2 cavity: 323 against 2 x 174)
  c->fused = p[0].storage != CLB_STORE_F16 || c->tile2_mode == clb::kFusedXWide;
  c->p.assign(p, p + count);
  for (auto &q : c->p) {  // host arrays are not kept
    c->rows |= has_rows(q);
    q.eps = nullptr;
    q.a_rows = nullptr;
  }
  c->der = der;
  c->lay = lay;
  c->ws = static_cast<char *>(d_workspace);
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->d_desc = reinterpret_cast<CavDesc *>(c->ws + lay.desc);
  c->d_tiles_all = reinterpret_cast<Tile *>(c->ws + lay.tiles_all);
  c->d_tiles_active = reinterpret_cast<Tile *>(c->ws + lay.tiles_active);
  c->d_tiles2[0] = reinterpret_cast<Tile *>(c->ws + lay.tiles2);
  c->d_tiles2[1] = c->d_tiles2[0] + lay.max_tiles2 + 8;
  c->d_counts = reinterpret_cast<int32_t *>(c->ws + lay.counts);
  c->d_partials = reinterpret_cast<double *>(c->ws + lay.partials);
  c->d_gpart = reinterpret_cast<double *>(c->ws + lay.gpart);
  c->d_nu_part = reinterpret_cast<double *>(c->ws + lay.nu_part);
  c->d_results = reinterpret_cast<double *>(c->ws + lay.results);
  c->d_nu = reinterpret_cast<double *>(c->ws + lay.nu);
  c->d_nu_local = reinterpret_cast<double *>(c->ws + lay.nu_local);
  c->d_obs = reinterpret_cast<float *>(c->ws + lay.obs);
  c->desc.resize(count);
  for (int k = 0; k < count; ++k) {
    fill_desc(p[k], der[k], c->desc[k]);
    c->desc[k].A = c->ws + lay.A[k];
    c->desc[k].B = c->ws + lay.B[k];
    c->desc[k].eps = p[k].eps ? reinterpret_cast<const float *>(c->ws + lay.eps[k]) : nullptr;
    c->desc[k].arow =
        has_rows(p[k]) ? reinterpret_cast<const double *>(c->ws + lay.arow[k]) : nullptr;
    c->desc[k].snap = reinterpret_cast<float *>(c->ws + lay.snap[k]);
  }
  c->active.assign(count, 1);
  auto fail = [&](clb_status s) {
    clb_destroy(c);
    return s;
  };
  {
    const hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(hip_fail(e, "hipStreamCreate"));
  }
  {
    // defined contents everywhere, row padding included (checkpoints are byte exact)
    const hipError_t e = hipMemsetAsync(c->ws, 0, lay.total, c->stream);
    if (e != hipSuccess) return fail(hip_fail(e, "workspace clear"));
  }
  // porosity fields (FP32, pitch layout)
  for (int k = 0; k < count; ++k) {
    if (!p[k].eps) continue;
    const int nx = p[k].nx, ny = p[k].ny, pitch = c->desc[k].pitch;
    std::vector<float> h((size_t)ny * pitch, 1.0f);
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const double e = p[k].eps[(size_t)y * nx + x];
        if (!(e > 0.0 && e < 1.0)) return fail(CLB_ERR_ARG);
        h[(size_t)y * pitch + x] = (float)e;
      }
    hipError_t e = hipMemcpyAsync(c->ws + lay.eps[k], h.data(), h.size() * sizeof(float),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(hip_fail(e, "eps upload"));
  }
  // per-row accelerations (FP64, 2 values per row)
  for (int k = 0; k < count; ++k) {
    if (!has_rows(p[k])) continue;
    const std::vector<double> h = row_accel(p[k], der[k]);
    for (double v : h)
      if (!std::isfinite(v)) return fail(CLB_ERR_ARG);
    hipError_t e = hipMemcpyAsync(c->ws + lay.arow[k], h.data(), h.size() * sizeof(double),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(hip_fail(e, "a_rows upload"));
  }
  build_tiles(c);
  {
    clb_status s = upload_tiles(c);
    if (s == CLB_OK) s = upload_tiles2(c);
    if (s != CLB_OK) return fail(s);
  }
  for (int k = 0; k < count; ++k) {
    const hipError_t e =
        clb::launch_init(c->d_desc, k, p[k].nx, p[k].ny, 0, nullptr, 0.0f, c->storage,
                         c->stream);
    if (e != hipSuccess) return fail(hip_fail(e, "init kernel"));
  }
  {
    const hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(hip_fail(e, "create sync"));
  }
  *out = c;
  return CLB_OK;
}

extern "C" void clb_destroy(clb_ctx *c) {
  if (!c) return;
  drop_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

namespace {
// Enqueues `rest` steps without a snapshot: graphs of kGraphSteps steps, then
// two-step launches (when in effect), then a single step for an odd remainder.
clb_status advance_plain(clb_ctx *c, int64_t rest, bool two) {
  while (rest > 0) {
    if (rest >= kGraphSteps) {
      hipGraphExec_t &g = two ? c->graph2[c->parity] : c->graph[c->parity];
      if (!g) {
        const clb_status s = capture_graph(c, c->parity);
        if (s != CLB_OK) return s;
      }
      HIPCHK(hipGraphLaunch(g, c->stream));
      rest -= kGraphSteps;  // an even number of buffer swaps: parity unchanged
    } else if (two && rest >= 2) {
      const clb_status s = launch_two(c, 0, c->stream);
      if (s != CLB_OK) return s;
      c->parity ^= 1;
      rest -= 2;
    } else {
      const clb_status s = launch_one(c, 0, c->stream);
      if (s != CLB_OK) return s;
      c->parity ^= 1;
      --rest;
    }
  }
  return CLB_OK;
}

// Enqueues n >= 1 steps, one of which records the snapshot of (u, v, theta)
// for the residual: the last one (residual over one step) or, with
// snap_first, the first one (residual over all n steps).  With two steps per
// launch the last step's snapshot is written by the second step of the last
// two-step launch, so that every step of an even request runs two per
// launch; an odd request takes one single step first.
clb_status advance(clb_ctx *c, int64_t n, bool snap_first) {
  const bool two = fused_now(c);
  clb_status s = CLB_OK;
  if (snap_first) {
    s = launch_one(c, 1, c->stream);
    if (s != CLB_OK) return s;
    c->parity ^= 1;
    s = advance_plain(c, n - 1, two);
  } else if (two && n >= 2) {
    s = advance_plain(c, n - 2, two);
    if (s == CLB_OK) s = launch_two(c, 1, c->stream);
    if (s != CLB_OK) return s;
    c->parity ^= 1;
  } else {
    s = advance_plain(c, n - 1, two);
    if (s == CLB_OK) s = launch_one(c, 1, c->stream);
    if (s != CLB_OK) return s;
    c->parity ^= 1;
  }
  if (s != CLB_OK) return s;
  c->steps += n;
  c->snap_valid = true;
  c->snap_span = snap_first ? n : 1;
  return CLB_OK;
}
}  // namespace

extern "C" clb_status clb_step(clb_ctx *c, int64_t n) {
  if (!c || n < 0) return CLB_ERR_ARG;
  if (n == 0) return CLB_OK;
  return advance(c, n, false);
}

extern "C" clb_status clb_macros(clb_ctx *c, int32_t cav, double *rho, double *u, double *v,
                                 double *T) {
  if (!c || cav < 0 || cav >= c->count) return CLB_ERR_ARG;
  const clb_params &p = c->p[cav];
  const size_t n = (size_t)p.nx * p.ny;
  HIPCHK(clb::launch_macros(c->d_desc, c->d_tiles_all, c->tile0[cav], c->ntiles[cav], c->parity,
                            c->d_obs, c->storage, c->shape, c->stream));
  std::vector<float> h(4 * n);
  HIPCHK(hipMemcpyAsync(h.data(), c->d_obs, h.size() * sizeof(float), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  const double T0 = p.T_init;  // storage reference of theta
  for (size_t k = 0; k < n; ++k) {
    if (rho) rho[k] = 1.0 + (double)h[k];
    if (u) u[k] = h[n + k];
    if (v) v[k] = h[2 * n + k];
    if (T) T[k] = T0 + (double)h[3 * n + k];
  }
  return CLB_OK;
}

extern "C" clb_status clb_nusselt(clb_ctx *c, int32_t cav, int32_t side, double *nu_mean,
                                  double *nu_local) {
  if (!c || cav < 0 || cav >= c->count || side < 0 || side > 3 || !nu_mean) return CLB_ERR_ARG;
  const clb_params &p = c->p[cav];
  if (p.bc[side] == CLB_PERIODIC) return CLB_ERR_ARG;
  const int nw = side < 2 ? p.ny : p.nx;
  HIPCHK(clb::launch_nusselt(c->d_desc, cav, 1, side, c->parity, c->d_nu,
                             nu_local ? c->d_nu_local : nullptr, c->d_nu_part, c->lay.max_chunks,
                             c->storage, c->stream));
  double m = 0.0;
  HIPCHK(hipMemcpyAsync(&m, c->d_nu + cav, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (nu_local)
    HIPCHK(hipMemcpyAsync(nu_local, c->d_nu_local, sizeof(double) * nw, hipMemcpyDeviceToHost,
                          c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *nu_mean = m;
  return CLB_OK;
}

extern "C" clb_status clb_nusselt_all(clb_ctx *c, int32_t side, double *nu_mean) {
  if (!c || side < 0 || side > 3 || !nu_mean) return CLB_ERR_ARG;
  for (int k = 0; k < c->count; ++k)
    if (c->p[k].bc[side] == CLB_PERIODIC) return CLB_ERR_ARG;
  HIPCHK(clb::launch_nusselt(c->d_desc, 0, c->count, side, c->parity, c->d_nu, nullptr,
                             c->d_nu_part, c->lay.max_chunks, c->storage, c->stream));
  std::vector<double> h(c->count);
  HIPCHK(hipMemcpyAsync(h.data(), c->d_nu, sizeof(double) * c->count, hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  std::copy(h.begin(), h.end(), nu_mean);
  return CLB_OK;
}

namespace {
// Groups of 256 tile partial sums in the largest domain.
int32_t max_groups(const clb_ctx *c) {
  int32_t m = 1;
  for (int k = 0; k < c->count; ++k) m = std::max(m, (c->ntiles[k] + 255) / 256);
  return m;
}

// Residual sums per domain into h (kRed values per domain).  With
// active_only, only the tiles of active domains are evaluated and the slots
// of the other domains keep their last values.
clb_status residual_sums(clb_ctx *c, std::vector<double> &h, bool active_only = false) {
  if (!c->snap_valid) return CLB_ERR_STATE;
  if (active_only)
    HIPCHK(clb::launch_residual(c->d_desc, c->d_tiles_active, (int)c->tiles_active.size(),
                                c->parity, c->d_partials, c->storage, c->shape, c->stream));
  else
    HIPCHK(clb::launch_residual(c->d_desc, c->d_tiles_all, (int)c->tiles_all.size(), c->parity,
                                c->d_partials, c->storage, c->shape, c->stream));
  HIPCHK(clb::launch_residual_finalize(c->d_desc, c->count, max_groups(c), c->d_partials,
                                       c->d_gpart, c->d_results, c->stream));
  h.assign((size_t)clb::kRed * c->count, 0.0);
  HIPCHK(hipMemcpyAsync(h.data(), c->d_results, sizeof(double) * h.size(), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return CLB_OK;
}

// Relative change per step over the `span` steps since the snapshot.
void residual_values(const double *r, int64_t span, double *ru, double *rT, double *mass,
                     bool *bad) {
  const double inf = std::numeric_limits<double>::infinity();
  *ru = r[1] > 0 ? std::sqrt(r[0] / r[1]) / (double)span : inf;
  *rT = r[3] > 0 ? std::sqrt(r[2] / r[3]) / (double)span : inf;
  *mass = r[6] + r[4];
  *bad = r[5] > 0 || !std::isfinite(r[0]) || !std::isfinite(r[2]) || !std::isfinite(r[4]);
}
}  // namespace

extern "C" clb_status clb_residual(clb_ctx *c, int32_t cav, double *res_u, double *res_T,
                                   double *mass) {
  if (!c || cav < 0 || cav >= c->count) return CLB_ERR_ARG;
  std::vector<double> h;
  const clb_status s = residual_sums(c, h);
  if (s != CLB_OK) return s;
  double ru, rT, m;
  bool bad;
  residual_values(&h[(size_t)clb::kRed * cav], c->snap_span, &ru, &rT, &m, &bad);
  if (res_u) *res_u = ru;
  if (res_T) *res_T = rT;
  if (mass) *mass = m;
  return bad ? CLB_ERR_DIVERGED : CLB_OK;
}

extern "C" clb_status clb_residual_all(clb_ctx *c, double *res_u, double *res_T, double *mass,
                                       int32_t *status) {
  if (!c) return CLB_ERR_ARG;
  std::vector<double> h;
  const clb_status s = residual_sums(c, h);
  if (s != CLB_OK) return s;
  for (int k = 0; k < c->count; ++k) {
    double ru, rT, m;
    bool bad;
    residual_values(&h[(size_t)clb::kRed * k], c->snap_span, &ru, &rT, &m, &bad);
    if (res_u) res_u[k] = ru;
    if (res_T) res_T[k] = rT;
    if (mass) mass[k] = m;
    if (status) status[k] = bad ? CLB_ERR_DIVERGED : CLB_OK;
  }
  return CLB_OK;
}

namespace {
// An inactive domain keeps the same state in both buffers (the parity of the
// others' later steps must not matter): after its state is written, stream-
// ordered, copy the current buffer into the other one.
clb_status mirror_if_inactive(clb_ctx *c, int k) {
  if (c->active[k]) return CLB_OK;
  const char *src = c->parity ? c->desc[k].B : c->desc[k].A;
  char *dst = c->parity ? c->desc[k].A : c->desc[k].B;
  HIPCHK(hipMemcpyAsync(dst, src, (size_t)c->desc[k].plane * pop_bytes(c->storage),
                        hipMemcpyDeviceToDevice, c->stream));
  return CLB_OK;
}
}  // namespace

extern "C" clb_status clb_set_state(clb_ctx *c, int32_t cav, const double *u, const double *v,
                                    const double *T) {
  if (!c || cav < 0 || cav >= c->count || !T) return CLB_ERR_ARG;
  const clb_params &p = c->p[cav];
  const size_t n = (size_t)p.nx * p.ny;
  const double T0 = p.T_init;  // storage reference of theta
  std::vector<float> h(3 * n);
  for (size_t k = 0; k < n; ++k) {
    h[k] = u ? (float)u[k] : 0.0f;
    h[n + k] = v ? (float)v[k] : 0.0f;
    h[2 * n + k] = (float)(T[k] - T0);
  }
  HIPCHK(hipMemcpyAsync(c->d_obs, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice,
                        c->stream));
  HIPCHK(clb::launch_init(c->d_desc, cav, p.nx, p.ny, c->parity, c->d_obs, 0.0f, c->storage,
                          c->stream));
  const clb_status s = mirror_if_inactive(c, cav);
  if (s != CLB_OK) return s;
  HIPCHK(hipStreamSynchronize(c->stream));
  c->snap_valid = false;
  return CLB_OK;
}

extern "C" clb_status clb_set_state_device(clb_ctx *c, int32_t cav, const float *d_fields,
                                           int64_t stride, double u_scale, double T_offset) {
  if (!c || cav < 0 || cav >= c->count || !d_fields || stride < 3) return CLB_ERR_ARG;
  const clb_params &p = c->p[cav];
  const int64_t n = (int64_t)p.nx * p.ny;
  HIPCHK(clb::launch_uvT_planes(d_fields, stride, n, u_scale, T_offset - p.T_init, c->d_obs,
                                c->stream));
  HIPCHK(clb::launch_init(c->d_desc, cav, p.nx, p.ny, c->parity, c->d_obs, 0.0f, c->storage,
                          c->stream));
  c->snap_valid = false;
  return mirror_if_inactive(c, cav);
}

extern "C" clb_status clb_set_active(clb_ctx *c, const uint8_t *active) {
  if (!c || !active) return CLB_ERR_ARG;
  for (int k = 0; k < c->count; ++k) {
    const uint8_t a = active[k] ? 1 : 0;
    const bool stops = c->active[k] && !a;
    c->active[k] = a;
    if (stops) {  // a domain that stops keeps its state in both buffers
      const clb_status s = mirror_if_inactive(c, k);
      if (s != CLB_OK) return s;
    }
  }
  clb_status s = upload_tiles(c);
  if (s == CLB_OK) s = upload_tiles2(c);
  return s;
}

// ------------------------------------------------------ run to steady state

extern "C" clb_status clb_run(clb_ctx *c, int64_t max_steps, int32_t check_every, double tol,
                              int32_t nu_side, double *nu_record, int32_t max_records,
                              int64_t *steps_taken, int32_t *status) {
  if (!c || max_steps < 0 || check_every < 1 || !(tol >= 0.0) || !steps_taken || !status)
    return CLB_ERR_ARG;
  if (nu_side < -1 || nu_side > 3 || (nu_record && (max_records < 1 || nu_side < 0)))
    return CLB_ERR_ARG;
  if (nu_side >= 0)
    for (int k = 0; k < c->count; ++k)
      if (c->p[k].bc[nu_side] == CLB_PERIODIC) return CLB_ERR_ARG;
  const int n = c->count;
  std::vector<uint8_t> live(c->active);
  std::vector<int64_t> taken(n, 0);
  std::vector<int32_t> st(n, CLB_ERR_STATE);
  for (int k = 0; k < n; ++k)
    if (live[k]) st[k] = CLB_NOT_CONVERGED;
  std::vector<double> nu(n), h;
  const double nan = std::numeric_limits<double>::quiet_NaN();
  if (nu_record) std::fill(nu_record, nu_record + (size_t)n * max_records, nan);
  int64_t done = 0;
  int round = 0;
  auto any_live = [&] { return std::find(live.begin(), live.end(), 1) != live.end(); };
  while (done < max_steps && any_live()) {
    const int64_t m = std::min<int64_t>(check_every, max_steps - done);
    clb_status s = advance(c, m, true);
    if (s != CLB_OK) return s;
    done += m;
    s = residual_sums(c, h, true);
    if (s != CLB_OK) return s;
    if (nu_side >= 0) {
      HIPCHK(clb::launch_nusselt(c->d_desc, 0, n, nu_side, c->parity, c->d_nu, nullptr,
                                 c->d_nu_part, c->lay.max_chunks, c->storage, c->stream));
      HIPCHK(hipMemcpyAsync(nu.data(), c->d_nu, sizeof(double) * n, hipMemcpyDeviceToHost,
                            c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
    }
    bool retired = false;
    for (int k = 0; k < n; ++k) {
      if (!live[k]) continue;
      taken[k] += m;
      if (nu_record && round < max_records) nu_record[(size_t)k * max_records + round] = nu[k];
      double ru, rT, mass;
      bool bad;
      residual_values(&h[(size_t)clb::kRed * k], c->snap_span, &ru, &rT, &mass, &bad);
      if (bad)
        st[k] = CLB_ERR_DIVERGED;
      else if (std::max(ru, rT) <= tol)
        st[k] = CLB_OK;
      else
        continue;
      live[k] = 0;
      retired = true;
    }
    ++round;
    if (retired) {
      s = clb_set_active(c, live.data());
      if (s != CLB_OK) return s;
    }
  }
  std::copy(taken.begin(), taken.end(), steps_taken);
  std::copy(st.begin(), st.end(), status);
  return CLB_OK;
}

// ------------------------------------------------------------- checkpoint

namespace {
struct StateHeader {
  char magic[8];
  int32_t count, storage;
  int64_t steps;
  uint64_t payload;
};

size_t payload_bytes(const clb_ctx *c) {
  size_t b = 0;
  for (int k = 0; k < c->count; ++k) b += (size_t)c->desc[k].plane * pop_bytes(c->storage);
  return b;
}
}  // namespace

extern "C" clb_status clb_state_bytes(clb_ctx *c, size_t *bytes) {
  if (!c || !bytes) return CLB_ERR_ARG;
  *bytes = sizeof(StateHeader) + payload_bytes(c);
  return CLB_OK;
}

extern "C" clb_status clb_get_state(clb_ctx *c, void *host_buf, size_t bytes) {
  if (!c || !host_buf || bytes < sizeof(StateHeader) + payload_bytes(c)) return CLB_ERR_ARG;
  StateHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, "CLBSTAT1", 8);
  h.count = c->count;
  h.storage = c->storage;
  h.steps = c->steps;
  h.payload = payload_bytes(c);
  char *dst = static_cast<char *>(host_buf);
  std::memcpy(dst, &h, sizeof(h));
  dst += sizeof(h);
  for (int k = 0; k < c->count; ++k) {
    const size_t b = (size_t)c->desc[k].plane * pop_bytes(c->storage);
    const char *src = c->parity ? c->desc[k].B : c->desc[k].A;
    HIPCHK(hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToHost, c->stream));
    dst += b;
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  return CLB_OK;
}

extern "C" clb_status clb_put_state(clb_ctx *c, const void *host_buf, size_t bytes) {
  if (!c || !host_buf || bytes < sizeof(StateHeader)) return CLB_ERR_ARG;
  StateHeader h;
  std::memcpy(&h, host_buf, sizeof(h));
  if (std::memcmp(h.magic, "CLBSTAT1", 8) != 0 || h.count != c->count ||
      h.storage != c->storage || h.payload != payload_bytes(c) ||
      bytes < sizeof(StateHeader) + h.payload)
    return CLB_ERR_ARG;
  const char *src = static_cast<const char *>(host_buf) + sizeof(h);
  for (int k = 0; k < c->count; ++k) {
    const size_t b = (size_t)c->desc[k].plane * pop_bytes(c->storage);
    char *dst = c->parity ? c->desc[k].B : c->desc[k].A;
    HIPCHK(hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, c->stream));
    const clb_status s = mirror_if_inactive(c, k);
    if (s != CLB_OK) return s;
    src += b;
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  c->steps = h.steps;
  c->snap_valid = false;
  return upload_tiles(c);  // also resets the device step counter
}

extern "C" clb_status clb_steps_done(clb_ctx *c, int64_t *steps) {
  if (!c || !steps) return CLB_ERR_ARG;
  *steps = c->steps;
  return CLB_OK;
}

// ----------------------------------------------------------- launch shape

extern "C" clb_status clb_set_launch(clb_ctx *c, int32_t tx, int32_t ty, int32_t blocks) {
  if (!c || !shape_ok(tx, ty) || blocks < 0) return CLB_ERR_ARG;
  drop_graphs(c);
  c->shape = LaunchShape{tx, ty, blocks};
  build_tiles(c);
  return upload_tiles(c);
}

extern "C" clb_status clb_set_steps_per_launch(clb_ctx *c, int32_t k) {
  if (!c || (k != 1 && k != 2)) return CLB_ERR_ARG;
  drop_graphs(c);
  c->fused = k == 2;
  return CLB_OK;
}

extern "C" clb_status clb_get_steps_per_launch(clb_ctx *c, int32_t *steps, int32_t *tile_x) {
  if (!c) return CLB_ERR_ARG;
  if (steps) *steps = c->fused ? 2 : 1;
  if (tile_x) {
    bool w64 = false, w128 = false;
    for (int k = 0; k < c->count; ++k) (tile2_width(c, k) == clb::kFusedX ? w64 : w128) = true;
    *tile_x = w64 && w128 ? 0 : (w128 ? clb::kFusedXWide : clb::kFusedX);
  }
  return CLB_OK;
}

namespace {
// The autotune cache's code for two-step tiles chosen per domain.
constexpr int kTile2PerDomain = 1;

// Switch the two-step tiles to width w (64 or 128 for every domain, 0 per
// domain): rebuild the lists and drop the graphs that captured the old ones.
clb_status set_tile2_width(clb_ctx *c, int w) {
  if (w != 0 && w != clb::kFusedX && w != clb::kFusedXWide) return CLB_ERR_ARG;
  drop_graphs(c);
  c->tile2_mode = w;
  return upload_tiles2(c);
}
}  // namespace

extern "C" clb_status clb_get_launch(clb_ctx *c, int32_t *tx, int32_t *ty, int32_t *blocks) {
  if (!c) return CLB_ERR_ARG;
  if (tx) *tx = c->shape.tile_x;
  if (ty) *ty = c->shape.tile_y;
  if (blocks) *blocks = c->shape.blocks;
  return CLB_OK;
}

namespace {
std::string tune_key(const clb_ctx *c) {
  std::ostringstream k;
  k << "storage=" << c->storage << ";n=" << c->count;
  size_t nodes = 0;
  for (const auto &p : c->p) nodes += (size_t)p.nx * p.ny;
  k << ";nodes=" << nodes << ";first=" << c->p[0].nx << "x" << c->p[0].ny;
  return k.str();
}
}  // namespace

// Measures the candidate launch shapes with HIP events on the live state.
extern "C" clb_status clb_autotune(clb_ctx *c, const char *cache_path) {
  if (!c) return CLB_ERR_ARG;
  const std::string key = tune_key(c);
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    LaunchShape found{0, 0, -1};
    int found_w = 0;  // two-step tile width; 0: none recorded
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      LaunchShape s;
      if (ls >> k >> s.tile_x >> s.tile_y >> s.blocks && k == key && shape_ok(s.tile_x, s.tile_y)) {
        found = s;
        int w = 0;
        found_w = (ls >> w) ? w : 0;
      }
    }
    if (found.blocks >= 0) {
      const clb_status s = clb_set_launch(c, found.tile_x, found.tile_y, found.blocks);
      if (s != CLB_OK || found_w == 0) return s;
      return set_tile2_width(c, found_w == kTile2PerDomain ? 0 : found_w);
    }
  }
  const int shapes[][2] = {{0, 0},   {64, 1},  {64, 2},  {64, 4},  {64, 8}, {128, 1},
                           {128, 2}, {128, 4}, {256, 1}, {256, 2}};
  size_t nodes = 0;
  for (const auto &p : c->p) nodes += (size_t)p.nx * p.ny;
  // enough steps for ~2 ms of work per candidate at ~50 GLUPS, at least 4
  const int reps = (int)std::max<size_t>(4, std::min<size_t>(200, 100000000 / (nodes + 1)));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  LaunchShape best = c->shape;
  float best_ms = 1e30f;
  for (const auto &sh : shapes) {
    for (int blocks : {0, 2048}) {
      clb_status s = clb_set_launch(c, sh[0], sh[1], blocks);
      if (s != CLB_OK) return s;
      for (int w = 0; w < 2; ++w) {
        s = launch_one(c, 0, c->stream);
        if (s != CLB_OK) return s;
        c->parity ^= 1;
        c->steps += 1;
      }
      HIPCHK(hipEventRecord(e0, c->stream));
      for (int r = 0; r < reps; ++r) {
        s = launch_one(c, 0, c->stream);
        if (s != CLB_OK) return s;
        c->parity ^= 1;
        c->steps += 1;
      }
      HIPCHK(hipEventRecord(e1, c->stream));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms) {
        best_ms = ms;
        best = c->shape;
      }
    }
  }
  clb_status s = clb_set_launch(c, best.tile_x, best.tile_y, best.blocks);
  if (s != CLB_OK) return s;
  // The two-step tile width, when pairs of steps run per launch: 64 for every
  // domain; 128 for every domain if some domain is that wide; per domain if
  // the widths are mixed; timed the same way (each pair of steps advances two
  // steps).  The cache records 64, 128, or kTile2PerDomain.
  int best_w = 0;
  bool have_w = false;
  if (fused_now(c)) {
    bool wide = false, narrow = false;
    for (const auto &p : c->p) (p.nx >= clb::kFusedXWide ? wide : narrow) = true;
    float best2_ms = 1e30f;
    for (int w : {clb::kFusedX, clb::kFusedXWide, 0}) {
      if (w == clb::kFusedXWide && !wide) continue;
      if (w == 0 && !(wide && narrow)) continue;
      s = set_tile2_width(c, w);
      if (s != CLB_OK) return s;
      for (int r = 0; r < 1 + std::max(2, reps / 2); ++r) {
        if (r == 1) HIPCHK(hipEventRecord(e0, c->stream));  // after one warm-up launch
        s = launch_two(c, 0, c->stream);
        if (s != CLB_OK) return s;
        c->parity ^= 1;
        c->steps += 2;
      }
      HIPCHK(hipEventRecord(e1, c->stream));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best2_ms) {
        best2_ms = ms;
        best_w = w;
        have_w = true;
      }
    }
    s = set_tile2_width(c, best_w);
    if (s != CLB_OK) return s;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->snap_valid = false;
  if (cache_path) {
    std::ofstream o(cache_path, std::ios::app);
    o << key << " " << best.tile_x << " " << best.tile_y << " " << best.blocks;
    if (have_w) o << " " << (best_w ? best_w : kTile2PerDomain);
    o << "\n";
  }
  return CLB_OK;
}

extern "C" const char *clb_strerror(clb_status s) {
  switch (s) {
    case CLB_OK: return "ok";
    case CLB_ERR_ARG: return "invalid argument";
    case CLB_ERR_HIP: return g_last_error.empty() ? "HIP error" : g_last_error.c_str();
    case CLB_ERR_WORKSPACE: return "workspace too small or misaligned";
    case CLB_ERR_DIVERGED: return "non-finite value in the fields";
    case CLB_ERR_STATE: return "call not valid in the current state";
    case CLB_NOT_CONVERGED: return "not steady within the step limit";
  }
  return "unknown status";
}
