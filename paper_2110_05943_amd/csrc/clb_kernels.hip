// HIP kernels (gfx950) of the porous-media cascaded lattice Boltzmann step.
//
// Method: Feng, Liu & He, arXiv:2110.05943, Section 2.  One fused kernel per
// time step pulls the 9 + 5 populations of every node from the A buffer
// (streaming, Eqs. 18 and 35), computes the macroscopic values (Eqs. 20-23,
// 36 and the force of Eq. 4), applies the boundary reconstruction at wall
// nodes, collides both lattices in central-moment space (D2Q9: Eqs. 11-17 with
// the porous shift of Eq. 14 and its inverse Eq. A1; D2Q5: Eqs. 28-33 with
// Eq. 31 and Eq. A2) and writes the post-collision populations to the B
// buffer.  The two lattices are coupled node-locally (G needs T, the D2Q5
// shift needs u), so both are handled in one pass: 14 loads and 14 stores per
// node and step.
//
// Storage is the deviation of each population from its rest value
// (df_i = f_i - w_i, dg_i = g_i - g_i^eq(T0, 0)), so every moment below is the
// small deviation of a moment from its rest value.
//
// Precision.  Kernels are templated on a storage policy: FP32 planes are
// computed in FP64, FP16 planes in FP32, and the mixed policy keeps the D2Q9
// planes in FP16 and the D2Q5 planes in FP32.  Stores to a narrower type
// round stochastically.  In a slowly varying field, a deterministic rounding
// repeats the same error at a node step after step; that bias accumulates
// through the long thermal memory of the problem (it dominates the error
// against an FP64 reference after a few thousand steps), while unbiased
// rounding leaves noise that the dynamics damp.  FP64 lanes run at the FP32
// rate on gfx950 (packed FP32 is not used), so the FP64 arithmetic rides
// under the memory traffic.
#include <hip/hip_runtime.h>

#include "clb_internal.h"

#include <type_traits>

namespace clb {

// ---------------------------------------------------------------- storage

// FP16 planes hold 2^12 times the deviation, which keeps deviations down to
// ~1e-8 in the normal FP16 range (the largest, ~0.5, stays far below 65504).
constexpr float kF16Scale = 4096.0f, kF16Unscale = 1.0f / 4096.0f;

// Population planes live in global memory.  The casts below let the compiler
// emit global (not flat) loads and stores, and plane-relative 32-bit offsets
// (at()) let it address them as a uniform base plus a per-lane offset.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
using gcptr = const __attribute__((address_space(1))) T *;

template <typename R>
__device__ __forceinline__ R ldv(const float *p) {
  return (R)__builtin_nontemporal_load((gcptr<float>)p);
}
template <typename R>
__device__ __forceinline__ R ldv(const _Float16 *p) {
  return (R)((float)__builtin_nontemporal_load((gcptr<_Float16>)p) * kF16Unscale);
}

// FP64 -> FP32 with stochastic rounding: 16 random bits are added below the
// FP32 precision of the value (29 bits lie below a normal FP32 significand),
// which is then truncated toward zero.
__device__ __forceinline__ float round_sr(double v, uint32_t r) {
  unsigned long long u = (unsigned long long)__double_as_longlong(v);
  u += (unsigned long long)(r & 0xFFFFu) << 13;
  u &= ~((1ull << 29) - 1ull);
  return (float)__longlong_as_double((long long)u);
}
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
// Per-node state of the encoder: the FP16 conversion below writes one half of
// its destination register and keeps the other, so the conversions of a node
// are chained through one register instead of clearing one per store.
struct EncState {
  half2v k = {};
};

// The stored value of a post-collision deviation v with random word r; the
// pointer argument only selects the storage type.
__device__ __forceinline__ float enc(EncState &, const float *, double v, uint32_t r) {
  return round_sr(v, r);
}
// FP32 -> FP16 with stochastic rounding by the gfx950 conversion
// instruction v_cvt_sr_f16_f32, which adds the top 13 bits of its random
// operand r below the FP16 precision of the value and truncates (unbiased,
// subnormal results included).  v is the value already scaled by kF16Scale
// (the collision folds the scale into its last products).
__device__ __forceinline__ _Float16 enc(EncState &e, const _Float16 *, float v, uint32_t r) {
  e.k = __builtin_amdgcn_cvt_sr_f16_f32(e.k, v, r, false);
  return e.k[0];
}
// FP32 -> FP32: no rounding (FP32 planes computed in FP32).
__device__ __forceinline__ float enc(EncState &, const float *, float v, uint32_t) { return v; }

template <typename T, typename R>
__device__ __forceinline__ void stv(EncState &e, T *p, R v, uint32_t r) {
  __builtin_nontemporal_store(enc(e, p, v, r), (gptr<T>)p);
}

// The deviation a stored value stands for (the inverse scaling of enc).
template <typename R>
__device__ __forceinline__ R dec(float v) { return (R)v; }
template <typename R>
__device__ __forceinline__ R dec(_Float16 v) { return (R)((float)v * kF16Unscale); }

// Storage policy: element types of the 9 D2Q9 planes (F) and the 5 D2Q5
// planes (G) and the arithmetic type R.  A population buffer holds the F
// planes, then the G planes, each plane `plane` elements long.
template <typename SF, typename SG, typename SR>
struct Store {
  using F = SF;
  using G = SG;
  using R = SR;
};
using StoreF32 = Store<float, float, double>;        // FP32 planes, FP64 arithmetic
using StoreF16 = Store<_Float16, _Float16, float>;   // FP16 planes, FP32 arithmetic
using StoreMix = Store<_Float16, float, float>;      // FP16 flow, FP32 temperature
using StoreF32C = Store<float, float, float>;        // FP32 planes, FP32 arithmetic

// With FP32 arithmetic and FP32 planes every stored value is the
// round-to-nearest result of its last operation, a rounding that repeats at a
// node step after step.  Where such a repeated rounding changes a conserved
// quantity, the slow dynamics integrate it: here the node's heat, i.e. the
// sum of the incoming D2Q5 populations and the rest population that closes
// it after the collision (which holds most of the heat).  That policy
// therefore carries the exact errors of those additions (compensated
// arithmetic, all in FP32) and rounds the compensated rest population
// stochastically; the other planes keep round-to-nearest.
template <typename P>
constexpr bool kCompensatedRest = std::is_same<P, StoreF32C>::value;

// s = a + b rounded to nearest, and its exact error e (a + b = s + e):
// Knuth's TwoSum, six FP32 additions with no assumption on |a| and |b|.
__device__ __forceinline__ float two_sum(float a, float b, float &e) {
  const float s = a + b;
  const float bv = s - a, av = s - bv;
  e = (a - av) + (b - bv);
  return s;
}

// s + e (s a rounded value, |e| at most half its last place) rounded
// stochastically to one of the two FP32 neighbours of s + e: with du uniform
// in [-1/2, 1/2) (16 bits of r), s + (e + du ulp(s)) rounded to nearest is
// s + ulp(s) floor(e / ulp(s) + du + 1/2), whose mean is s + e.
__device__ __forceinline__ float round_pair_sr(float s, float e, uint32_t r) {
  const float ulp = __uint_as_float(__float_as_uint(s) & 0x7F800000u) * 0x1p-23f;
  const float du = __uint_as_float(((r & 0xFFFFu) << 7) | 0x3F800000u) - 1.5f;
  return s + __builtin_fmaf(du, ulp, e);
}

// The domain constants in the arithmetic type R of a kernel.
template <typename R>
__device__ __forceinline__ const DomainConsts<R> &cst(const CavDesc &d);
template <>
__device__ __forceinline__ const DomainConsts<double> &cst<double>(const CavDesc &d) {
  return d.c;
}
template <>
__device__ __forceinline__ const DomainConsts<float> &cst<float>(const CavDesc &d) {
  return d.c32;
}

template <typename P>
__device__ __forceinline__ const typename P::F *fplanes(const char *buf) {
  return reinterpret_cast<const typename P::F *>(buf);
}
template <typename P>
__device__ __forceinline__ const typename P::G *gplanes(const char *buf, int plane) {
  return reinterpret_cast<const typename P::G *>(buf + (size_t)9 * plane * sizeof(typename P::F));
}

// Counter-based random bits: an integer hash (xorshift-multiply finaliser)
// of (node, step, domain) gives each node one random word; a run is
// reproducible bit for bit.  Further words of the node: for FP32 storage
// (rounding noise ~1e-8) golden-ratio (Weyl) increments, the cheapest
// sequence; for FP16 storage, whose rounding noise (~1e-4) reaches the wall
// gradient of the Nusselt number, a xorshift32 step, so that the roundings of
// the populations of one node stay uncorrelated.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
template <typename R>
__device__ __forceinline__ uint32_t next_bits(uint32_t x) {
  if (sizeof(R) == 8) return x + 0x9E3779B9u;
  x ^= x << 13;
  x ^= x >> 17;
  x ^= x << 5;
  return x;
}
// The random operand of the rounding of plane i from the node's current word
// w; each word serves two planes.  FP64 arithmetic (round_sr reads the low 16
// bits): w and w >> 16.  FP32 arithmetic (v_cvt_sr_f16_f32 reads the top 13
// bits): w and w << 13, the disjoint fields w[19..31] and w[6..18]; w << 13
// is also the first term of the xorshift step that makes the next word.
template <typename R>
__device__ __forceinline__ uint32_t round_bits(uint32_t w, int i) {
  if (sizeof(R) == 8) return (i & 1) ? (w >> 16) : w;
  return (i & 1) ? (w << 13) : w;
}

// ------------------------------------------------------- fast helpers

// 1/x and sqrt(x) from the hardware FP32 instructions.  rcp_nr refines the
// FP32 reciprocal estimate (about one FP32 unit) by one Newton step in FP64
// arithmetic (relative error about 2^-46); it serves 1/rho and the
// denominator of Eq. 23, whose errors pass into the velocity at first order.
// The square roots inside Eq. 23 (|v| and the root of l0^2 + l1 |v|) and
// 1/phi of a porosity field take the FP32 estimates: measured against the
// FP64 oracle on the 64^2 cavity over 5000 steps, the FP64-arithmetic
// results move by less than 1e-8 relative.  The FP32 overloads (FP16, mixed
// and FP32-arithmetic storage) take the estimates throughout: their error is
// of the order of the FP32 arithmetic itself.
__device__ __forceinline__ double rcp_nr(double x) {
  const double r = (double)__builtin_amdgcn_rcpf((float)x);
  return r * (2.0 - x * r);
}
__device__ __forceinline__ float rcp_nr(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_est(double x) {
  return (double)__builtin_amdgcn_rcpf((float)x);
}
__device__ __forceinline__ float rcp_est(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double sqrt_est(double x) {
  return (double)__builtin_amdgcn_sqrtf((float)x);
}
__device__ __forceinline__ float sqrt_est(float x) { return __builtin_amdgcn_sqrtf(x); }

// A plane base that every lane shares, held in scalar registers and opaque
// to the optimiser: the 14 stores of a node then each take the form
// "scalar base + the node's 32-bit offset" instead of a chain of 64-bit
// vector additions from one base (an empty asm statement with an SGPR
// operand; it emits no instruction).
template <typename T>
__device__ __forceinline__ T *uniform_base(T *p) {
  asm("" : "+s"(p));
  return p;
}

// Element i of a plane as a byte offset below 4 GiB from the plane base.
template <typename T>
__device__ __forceinline__ T *at(T *base, uint32_t i) {
  return (T *)((char *)base + i * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ const T *at(const T *base, uint32_t i) {
  return (const T *)((const char *)base + i * (uint32_t)sizeof(T));
}
// ------------------------------------------------------------- node state

// Deviations of the raw moments of Eq. 9 (k00 - 1, k10, k01, k20 - 1/3,
// k02 - 1/3, k11, k21, k12, k22 - 1/9), the D2Q5 raw moments of Eq. 26
// (k10, k01, k20 - c_sT^2 T0, k02 - c_sT^2 T0 and sigma theta), and the
// macroscopic values the collision uses.
template <typename R>
struct NodeState {
  R dr, jx, jy, k20, k02, k11, k21, k12, k22;
  R n1, n2, n3, n4;
  R sg;                 // sigma theta = sum of the D2Q5 deviations (conserved)
  R sg_lo;              // rounding error of sg (kCompensatedRest policy only)
  R th;                 // theta = T - T0
  R rho, ux, uy, umag;
  R phi, ip, cd, cf;    // medium at this node
  R gax, gay;           // external acceleration at this node (per-row variant only)
};

// Deviation of the equilibrium raw moments of Eq. 19 from their rest values,
// for rho = 1 + drho.
template <typename R>
__device__ __forceinline__ void meq_dev(R drho, R ux, R uy, R ip, R m[9]) {
  const R rho = R(1) + drho;
  const R ux2 = ux * ux, uy2 = uy * uy, rip = rho * ip;
  const R third = R(1) / R(3);
  m[0] = drho;
  m[1] = rho * ux;
  m[2] = rho * uy;
  m[3] = drho * third + rip * ux2;
  m[4] = drho * third + rip * uy2;
  m[5] = rip * ux * uy;
  m[6] = rho * uy * third + rip * ux2 * uy;
  m[7] = rho * ux * third + rip * ux * uy2;
  m[8] = drho * (R(1) / R(9)) + rip * (ux2 + uy2) * third + rip * ip * ux2 * uy2;
}

__device__ __forceinline__ bool dirichlet_T(int kind) { return kind == kWallT || kind == kInlet; }

// Porosity-dependent drag coefficients at one node.
template <typename R>
__device__ __forceinline__ void medium_at(const CavDesc &d, int idx, R &phi, R &ip, R &cd, R &cf) {
  if (d.has_eps) {
    // Eq. 5 (Kozeny-Carman K, Ergun F_phi) folded into phi nu / K and
    // phi F_phi / sqrt(K):  cd = 150 nu (1-phi)^2 / (phi^2 dp^2),
    // cf = 1.75 (1-phi) / (phi^2 dp).
    phi = (R)d.eps[idx];
    ip = rcp_est(phi);
    const R q = (R(1) - phi) * ip;
    cd = cst<R>(d).kc_d * q * q;
    cf = cst<R>(d).kc_f * q * ip;
  } else {
    phi = cst<R>(d).phi;
    ip = cst<R>(d).ip;
    cd = cst<R>(d).cd;
    cf = cst<R>(d).cf;
  }
}

// External acceleration a of row y; ROWS adds the domain's per-row profile
// when it has one.
template <bool ROWS, typename R>
__device__ __forceinline__ void accel_at(const CavDesc &d, int y, R &ax, R &ay) {
  ax = cst<R>(d).ax;
  ay = cst<R>(d).ay;
  if constexpr (ROWS) {
    if (d.arow) {
      ax += (R)d.arow[2 * y];
      ay += (R)d.arow[2 * y + 1];
    }
  }
}

// Where a gather reads populations.  GlobalSrc: the planes of a buffer in
// global memory; (xs, ys) must have all 8 neighbours inside the domain or
// across a periodic side, which wraps (WRAP = false: all 8 inside).  LdsSrc (two-step kernel): FP32
// populations of a rectangular region held in LDS, 14 planes of kRegion
// elements, rows kRegionW long; the region's element 0 is the node (ox, oy)
// of the domain in unwrapped coordinates, and every neighbour read lies in
// the region by construction of the caller.
template <typename P, bool WRAP = true>
struct GlobalSrc {
  const char *buf;

  template <typename R>
  __device__ __forceinline__ void pull(const CavDesc &d, int xs, int ys, R f[9], R g[5]) const {
    const int nx = d.nx, ny = d.ny, pitch = d.pitch, plane = d.plane;
    int xm = xs - 1, xp = xs + 1, ym = ys - 1, yp = ys + 1;
    if (WRAP && d.bc[0] == kPeriodic) {
      xm = xm < 0 ? xm + nx : xm;
      xp = xp >= nx ? xp - nx : xp;
    }
    if (WRAP && d.bc[2] == kPeriodic) {
      ym = ym < 0 ? ym + ny : ym;
      yp = yp >= ny ? yp - ny : yp;
    }
    const int r0 = ys * pitch, rm = ym * pitch, rp = yp * pitch;
    const typename P::F *A = fplanes<P>(buf);
    const typename P::G *G = gplanes<P>(buf, plane);
    // f_i(x) = f_i*(x - e_i), velocities of Eq. 6.
    f[0] = ldv<R>(at(A, r0 + xs));
    f[1] = ldv<R>(at(A + (size_t)plane, r0 + xm));
    f[2] = ldv<R>(at(A + (size_t)2 * plane, rm + xs));
    f[3] = ldv<R>(at(A + (size_t)3 * plane, r0 + xp));
    f[4] = ldv<R>(at(A + (size_t)4 * plane, rp + xs));
    f[5] = ldv<R>(at(A + (size_t)5 * plane, rm + xm));
    f[6] = ldv<R>(at(A + (size_t)6 * plane, rm + xp));
    f[7] = ldv<R>(at(A + (size_t)7 * plane, rp + xp));
    f[8] = ldv<R>(at(A + (size_t)8 * plane, rp + xm));
    g[0] = ldv<R>(at(G, r0 + xs));
    g[1] = ldv<R>(at(G + (size_t)plane, r0 + xm));
    g[2] = ldv<R>(at(G + (size_t)2 * plane, rm + xs));
    g[3] = ldv<R>(at(G + (size_t)3 * plane, r0 + xp));
    g[4] = ldv<R>(at(G + (size_t)4 * plane, rp + xs));
  }

  // Sum of the five pulled D2Q5 populations.
  template <typename R>
  __device__ __forceinline__ R gsum(const CavDesc &d, int xs, int ys) const {
    const int nx = d.nx, ny = d.ny, pitch = d.pitch, plane = d.plane;
    int xm = xs - 1, xp = xs + 1, ym = ys - 1, yp = ys + 1;
    if (d.bc[0] == kPeriodic) {
      xm = xm < 0 ? xm + nx : xm;
      xp = xp >= nx ? xp - nx : xp;
    }
    if (d.bc[2] == kPeriodic) {
      ym = ym < 0 ? ym + ny : ym;
      yp = yp >= ny ? yp - ny : yp;
    }
    const typename P::G *G = gplanes<P>(buf, plane);
    return ldv<R>(at(G, ys * pitch + xs)) +
           ((ldv<R>(at(G + (size_t)plane, ys * pitch + xm)) +
             ldv<R>(at(G + (size_t)3 * plane, ys * pitch + xp))) +
            (ldv<R>(at(G + (size_t)2 * plane, ym * pitch + xs)) +
             ldv<R>(at(G + (size_t)4 * plane, yp * pitch + xs))));
  }
};

// Threads of a two-step workgroup: four per tile column, so that the tile
// takes two passes of the second step.  The 64-wide kernel with FP32 planes
// and FP32 arithmetic takes eight: its 37 KB of LDS and 55 VGPRs then hold
// eight waves per SIMD instead of four (5% faster on the 256-cavity batch;
// slower for the other storage modes and for 128-wide tiles, whose LDS
// allows only two workgroups per CU).
template <typename P, int TX>
constexpr int kThreads2 = (TX == kFusedX && std::is_same<P, StoreF32C>::value) ? 8 * TX : 4 * TX;

// The LDS region of a two-step tile TX x kFusedY: the tile plus a one-node ring.
template <int TX>
struct Region {
  static constexpr int W = TX + 2;
  static constexpr int N = W * (kFusedY + 2);
};

// The LDS region of a two-step tile in the storage types of P: the 9 D2Q9
// planes (P::F) and then the 5 D2Q5 planes (P::G), Region<TX>::N elements
// each, holding the values the stored planes would hold.
template <typename P, int TX>
struct RegionPlanes {
  static constexpr int kBytes =
      Region<TX>::N * (9 * (int)sizeof(typename P::F) + 5 * (int)sizeof(typename P::G));
  __device__ static typename P::F *f(char *lds) { return (typename P::F *)lds; }
  __device__ static typename P::G *g(char *lds) {
    return (typename P::G *)(lds + 9 * Region<TX>::N * sizeof(typename P::F));
  }
};

template <typename P, int TX>
struct LdsSrc {
  static constexpr int kRegionW = Region<TX>::W, kRegion = Region<TX>::N;
  char *lds;
  int ox, oy;

  template <typename R>
  __device__ __forceinline__ void pull(const CavDesc &, int xs, int ys, R f[9], R g[5]) const {
    const int c = (ys - oy) * kRegionW + (xs - ox);
    const int W = kRegionW;
    const typename P::F *F = RegionPlanes<P, TX>::f(lds);
    const typename P::G *G = RegionPlanes<P, TX>::g(lds);
    f[0] = dec<R>(F[c]);
    f[1] = dec<R>(F[kRegion + c - 1]);
    f[2] = dec<R>(F[2 * kRegion + c - W]);
    f[3] = dec<R>(F[3 * kRegion + c + 1]);
    f[4] = dec<R>(F[4 * kRegion + c + W]);
    f[5] = dec<R>(F[5 * kRegion + c - W - 1]);
    f[6] = dec<R>(F[6 * kRegion + c - W + 1]);
    f[7] = dec<R>(F[7 * kRegion + c + W + 1]);
    f[8] = dec<R>(F[8 * kRegion + c + W - 1]);
    g[0] = dec<R>(G[c]);
    g[1] = dec<R>(G[kRegion + c - 1]);
    g[2] = dec<R>(G[2 * kRegion + c - W]);
    g[3] = dec<R>(G[3 * kRegion + c + 1]);
    g[4] = dec<R>(G[4 * kRegion + c + W]);
  }

  template <typename R>
  __device__ __forceinline__ R gsum(const CavDesc &, int xs, int ys) const {
    const int c = (ys - oy) * kRegionW + (xs - ox);
    const int W = kRegionW;
    const typename P::G *G = RegionPlanes<P, TX>::g(lds);
    return dec<R>(G[c]) + ((dec<R>(G[kRegion + c - 1]) + dec<R>(G[3 * kRegion + c + 1])) +
                           (dec<R>(G[2 * kRegion + c - W]) + dec<R>(G[4 * kRegion + c + W])));
  }
};

// Pull the post-streaming populations of node (xs, ys) from `src` and reduce
// them to moments and macroscopic values.
template <typename P, bool ROWS, typename Src, typename R = typename P::R>
__device__ __forceinline__ void gather_moments(const CavDesc &d, const Src &src, int xs, int ys,
                                               NodeState<R> &st) {
  R fv[9], gv[5];
  src.template pull<R>(d, xs, ys, fv, gv);
  const R f0 = fv[0], f1 = fv[1], f2 = fv[2], f3 = fv[3], f4 = fv[4], f5 = fv[5], f6 = fv[6],
          f7 = fv[7], f8 = fv[8];
  const R g0 = gv[0], g1 = gv[1], g2 = gv[2], g3 = gv[3], g4 = gv[4];
  const int r0 = ys * d.pitch;

  // raw moments (Eq. 7 on Eq. 6), as deviations
  const R p13 = f1 + f3, m13 = f1 - f3, p24 = f2 + f4, m24 = f2 - f4;
  const R a = f5 + f7, b = f6 + f8, c = f5 - f7, e = f6 - f8;
  st.k22 = a + b;
  st.k11 = a - b;
  st.k21 = c + e;
  st.k12 = c - e;
  st.jx = m13 + st.k12;
  st.jy = m24 + st.k21;
  st.k20 = p13 + st.k22;
  st.k02 = p24 + st.k22;
  st.dr = f0 + (p13 + p24 + st.k22);
  // D2Q5 raw moments (Eq. 24); theta from Eq. 36
  st.n1 = g1 - g3;
  st.n2 = g2 - g4;
  if constexpr (kCompensatedRest<P>) {
    // the heat sum and the exact error of its four roundings, which the
    // collision returns to the rest population (heat is then conserved
    // without a rounding bias)
    R e3, e4, e5, e6;
    st.n3 = two_sum(g1, g3, e3);
    st.n4 = two_sum(g2, g4, e4);
    const R s = two_sum(st.n3, st.n4, e5);
    st.sg = two_sum(g0, s, e6);
    st.sg_lo = (e3 + e4) + (e5 + e6);
  } else {
    st.n3 = g1 + g3;
    st.n4 = g2 + g4;
    st.sg = g0 + (st.n3 + st.n4);
  }
  st.th = st.sg * cst<R>(d).isig;

  medium_at(d, r0 + xs, st.phi, st.ip, st.cd, st.cf);
  // Eqs. 20-23: rho, the temporal velocity v and the explicit velocity u.
  st.rho = R(1) + st.dr;
  const R irho = rcp_nr(st.rho);
  R gax, gay;
  accel_at<ROWS>(d, ys, gax, gay);
  if constexpr (ROWS) {
    st.gax = gax;
    st.gay = gay;
  }
  const R Gx = cst<R>(d).gbx * st.th + gax, Gy = cst<R>(d).gby * st.th + gay;
  const R hphi = R(0.5) * st.phi;
  const R vx = st.jx * irho + hphi * Gx;
  const R vy = st.jy * irho + hphi * Gy;
  const R vm = sqrt_est(vx * vx + vy * vy);
  R l0, l0sq, l1;  // Eq. 23
  if (d.has_eps) {
    l0 = R(0.5) + R(0.25) * st.cd;
    l0sq = l0 * l0;
    l1 = R(0.5) * st.cf;
  } else {
    l0 = cst<R>(d).l0;
    l0sq = cst<R>(d).l0sq;
    l1 = cst<R>(d).l1;
  }
  const R iD = rcp_nr(l0 + sqrt_est(l0sq + l1 * vm));
  st.ux = vx * iD;
  st.uy = vy * iD;
  st.umag = vm * iD;
}

// theta at node (xs, ys) from its post-streaming D2Q5 populations.
template <typename P, typename Src, typename R = typename P::R>
__device__ __forceinline__ R gather_theta(const CavDesc &d, const Src &src, int xs, int ys) {
  return src.template gsum<R>(d, xs, ys) * cst<R>(d).isig;
}

// Macroscopic state of node (x, y) ready for the collision.  Boundary nodes
// (outermost nodes of a non-periodic side) are rebuilt by non-equilibrium
// extrapolation from their inward neighbour x_f (diagonal at a corner):
// their raw moments become m(x_f) + m^eq(rho_b, u_b; phi_b) - m^eq(rho_f, u_f;
// phi_f), which is M applied to f_i^eq(b) + [f_i(x_f) - f_i^eq(x_f)], and
// likewise for the D2Q5 moments with Eq. 33.  The node then collides with
// (rho_b, u_b, T_b).  Returns true for boundary nodes.
template <typename P, bool ROWS, typename Src, bool EDGE = true, typename R = typename P::R>
__device__ __forceinline__ bool node_state(const CavDesc &d, const Src &A, int x, int y,
                                           NodeState<R> &st) {
  if constexpr (!EDGE) {  // caller guarantees (x, y) is no boundary node
    gather_moments<P, ROWS>(d, A, x, y, st);
    return false;
  }
  int sx = -1, sy = -1, dx = 0, dy = 0;
  if (x == 0 && d.bc[0] != kPeriodic) {
    sx = 0;
    dx = 1;
  } else if (x == d.nx - 1 && d.bc[1] != kPeriodic) {
    sx = 1;
    dx = -1;
  }
  if (y == 0 && d.bc[2] != kPeriodic) {
    sy = 2;
    dy = 1;
  } else if (y == d.ny - 1 && d.bc[3] != kPeriodic) {
    sy = 3;
    dy = -1;
  }
  const bool wall = (sx >= 0) || (sy >= 0);
  gather_moments<P, ROWS>(d, A, x + dx, y + dy, st);
  if (wall) {
    const R drf = st.dr, uxf = st.ux, uyf = st.uy, thf = st.th, ipf = st.ip;
    const bool corner = (sx >= 0) && (sy >= 0);
    const int side = sx >= 0 ? sx : sy;
    const int kind = d.bc[side];
    bool need_ff;
    if (corner)
      need_ff = !dirichlet_T(d.bc[sx]) && !dirichlet_T(d.bc[sy]);
    else
      need_ff = kind == kWallAdiabatic;
    R thff = R(0);
    if (need_ff) thff = gather_theta<P>(d, A, x + 2 * dx, y + 2 * dy);
    // second-order zero normal gradient: theta_b = (4 theta_f - theta_ff) / 3
    const R thx = thf + (thf - thff) * (R(1) / R(3));
    R drb = drf, ubx = R(0), uby = R(0), thb;
    if (corner) {
      thb = dirichlet_T(d.bc[sx]) ? cst<R>(d).bc_th[sx]
                                  : (dirichlet_T(d.bc[sy]) ? cst<R>(d).bc_th[sy] : thx);
    } else if (kind == kWallT || kind == kWallAdiabatic) {
      ubx = cst<R>(d).bc_u[side];
      uby = cst<R>(d).bc_v[side];
      thb = kind == kWallT ? cst<R>(d).bc_th[side] : thx;
    } else if (kind == kInlet) {
      const R t = side < 2 ? (R)y / (R)(d.ny - 1) : (R)x / (R)(d.nx - 1);
      const R un = R(6) * cst<R>(d).inlet_U * t * (R(1) - t);
      ubx = side == 0 ? un : (side == 1 ? -un : R(0));
      uby = side == 2 ? un : (side == 3 ? -un : R(0));
      thb = cst<R>(d).bc_th[side];
    } else {  // outlet
      drb = R(0);
      ubx = uxf;
      uby = uyf;
      thb = thf;
    }
    // the boundary node's own medium and acceleration
    medium_at(d, y * d.pitch + x, st.phi, st.ip, st.cd, st.cf);
    if constexpr (ROWS) accel_at<ROWS>(d, y, st.gax, st.gay);
    R mb[9], mf[9];
    meq_dev(drb, ubx, uby, st.ip, mb);
    meq_dev(drf, uxf, uyf, ipf, mf);
    st.dr += mb[0] - mf[0];
    st.jx += mb[1] - mf[1];
    st.jy += mb[2] - mf[2];
    st.k20 += mb[3] - mf[3];
    st.k02 += mb[4] - mf[4];
    st.k11 += mb[5] - mf[5];
    st.k21 += mb[6] - mf[6];
    st.k12 += mb[7] - mf[7];
    st.k22 += mb[8] - mf[8];
    const R T0 = cst<R>(d).T0, hv = cst<R>(d).hv;
    const R Tb = T0 + thb, Tf = T0 + thf;
    st.n1 += ubx * Tb - uxf * Tf;
    st.n2 += uby * Tb - uyf * Tf;
    st.n3 += (hv * thb + ubx * ubx * Tb) - (hv * thf + uxf * uxf * Tf);
    st.n4 += (hv * thb + uby * uby * Tb) - (hv * thf + uyf * uyf * Tf);
    st.sg = cst<R>(d).sig * thb;
    st.sg_lo = R(0);
    st.th = thb;
    st.rho = R(1) + st.dr;
    st.ux = ubx;
    st.uy = uby;
    st.umag = sqrt_est(ubx * ubx + uby * uby);
  }
  return wall;
}

// Collide one node in central-moment space (RAW: in raw-moment space, the
// MRT form with N = N_T = I): the 14 post-collision deviations, D2Q9 first,
// each in the scale of its stored plane (kF16Scale for FP16 planes, 1 for
// FP32 planes).  The scale rides on the constants of the last products, a
// power-of-two change that leaves every rounding as it was.
template <typename P, bool RAW, bool ROWS, typename R = typename P::R>
__device__ __forceinline__ void collide(const CavDesc &d, const NodeState<R> &st, bool wall,
                                        R out[kPlanes], R &rest_err) {
  const R rho = st.rho, ux = st.ux, uy = st.uy, ip = st.ip, dr = st.dr;
  const R jx = st.jx, jy = st.jy;
  const R ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy;
  const R third = R(1) / R(3), two = R(2), half = R(0.5), quarter = R(0.25);

  // force of Eq. 4 with G = gb theta + a
  R gax = cst<R>(d).ax, gay = cst<R>(d).ay;
  if constexpr (ROWS) {
    gax = st.gax;
    gay = st.gay;
  }
  const R Gx = cst<R>(d).gbx * st.th + gax, Gy = cst<R>(d).gby * st.th + gay;
  const R drag = st.cd + st.cf * st.umag;
  const R rFx = rho * (st.phi * Gx - drag * ux);
  const R rFy = rho * (st.phi * Gy - drag * uy);

  // post-collision raw moments (deviations from their rest values)
  R K10, K01, Q20, Q02, Q11, Q21, Q12, Q22;
  if constexpr (!RAW) {
    // central moments m~ = N m (Eq. 14), as deviations from their rest values
    const R c1 = jx - ux * rho;
    const R c2 = jy - uy * rho;
    const R c3 = st.k20 + ip * ux * (ux * rho - two * jx);
    const R c4 = st.k02 + ip * uy * (uy * rho - two * jy);
    const R c5 = st.k11 + ip * (uxy * rho - uy * jx - ux * jy);
    const R K20 = third + st.k20, K02 = third + st.k02;
    const R c6 = st.k21 - uy * K20 - two * ux * st.k11 + ip * ux * (two * uy * jx + ux * jy - uxy * rho);
    const R c7 = st.k12 - ux * K02 - two * uy * st.k11 + ip * uy * (uy * jx + two * ux * jy - uxy * rho);
    const R c8 = st.k22 +
                 ip * (uy2 * K20 + ux2 * K02 + R(4) * uxy * st.k11 - two * uy * st.k21 -
                       two * ux * st.k12) +
                 ip * ip * uxy * (uxy * rho - two * uy * jx - two * ux * jy);

    // relaxation with consistent forcing (Eqs. 11, 15-17)
    const R e3 = c3 - dr * third, e4 = c4 - dr * third;
    const R sp = cst<R>(d).sp, sm = cst<R>(d).sm, s3c = cst<R>(d).s3c, s3f = cst<R>(d).s3f, s1c = cst<R>(d).s1c,
            s1f = cst<R>(d).s1f;
    // At a fluid node rho u = j + rho F / 2 (Eqs. 21-22), so c1 = -rho F_x / 2
    // and c1s = rho F_x / 2 for any s1 (the consistent forcing of the first
    // moments); a boundary node collides with its prescribed u_b instead.
    const R c1s = wall ? s1c * c1 + s1f * rFx : half * rFx;
    const R c2s = wall ? s1c * c2 + s1f * rFy : half * rFy;
    const R c3s = c3 - sp * e3 - sm * e4;
    const R c4s = c4 - sm * e3 - sp * e4;
    const R c5s = cst<R>(d).svc * c5;
    const R c6s = s3c * c6 + s3f * rFy;
    const R c7s = s3c * c7 + s3f * rFx;
    const R c8s = c8 - cst<R>(d).s4 * (c8 - dr * (R(1) / R(9)));

    // back to raw moments with N^-1 (Eq. A1).  The first moments are
    // rho u + c~*_10.  At a fluid node Eq. 21 makes this j + rho F exactly for
    // any s1; that form is used there because rebuilding it from the rounded u
    // would inject a momentum error every step.
    K10 = wall ? ux * rho + c1s : jx + rFx;
    K01 = wall ? uy * rho + c2s : jy + rFy;
    Q20 = ip * ux * (ux * rho + two * c1s) + c3s;
    Q02 = ip * uy * (uy * rho + two * c2s) + c4s;
    Q11 = ip * (uxy * rho + uy * c1s + ux * c2s) + c5s;
    Q21 = ip * ux * (uxy * rho + two * uy * c1s + ux * c2s) + uy * (third + c3s) +
                  two * ux * c5s + c6s;
    Q12 = ip * uy * (uxy * rho + uy * c1s + two * ux * c2s) + ux * (third + c4s) +
                  two * uy * c5s + c7s;
    Q22 = ip * ip * uxy * (uxy * rho + two * uy * c1s + two * ux * c2s) +
                  ip * (uy2 * (third + c3s) + ux2 * (third + c4s) + R(4) * uxy * c5s +
                        two * uy * c6s + two * ux * c7s) +
                  c8s;

  } else {
    // MRT (N = N_T = I): raw moments relax toward the raw equilibria of
    // Eq. 19 with the raw forcing moments of Eq. 19.  The first moments are
    // the same expressions as in the cascaded branch.
    R me[9];
    meq_dev(dr, ux, uy, ip, me);
    const R s1c = cst<R>(d).s1c, s1f = cst<R>(d).s1f;
    const R S3 = two * ux * rFx * ip, S4 = two * uy * rFy * ip;
    const R S5 = (ux * rFy + uy * rFx) * ip;
    const R S6 = rFy * third + (rFy * ux2 + two * rFx * uxy) * ip;
    const R S7 = rFx * third + (rFx * uy2 + two * rFy * uxy) * ip;
    const R S8 = two * third * (ux * rFx + uy * rFy) * ip +
                 two * ip * ip * uxy * (rFx * uy + rFy * ux);
    K10 = wall ? me[1] + s1c * (jx - me[1]) + s1f * rFx : jx + rFx;
    K01 = wall ? me[2] + s1c * (jy - me[2]) + s1f * rFy : jy + rFy;
    const R sp = cst<R>(d).sp, sm = cst<R>(d).sm;
    const R e3 = st.k20 - me[3], e4 = st.k02 - me[4];
    Q20 = st.k20 - sp * e3 - sm * e4 + S3 - half * (sp * S3 + sm * S4);
    Q02 = st.k02 - sm * e3 - sp * e4 + S4 - half * (sm * S3 + sp * S4);
    const R svc = cst<R>(d).svc, s3c = cst<R>(d).s3c, s3h = R(3) * cst<R>(d).s3f, s4 = cst<R>(d).s4;
    Q11 = me[5] + svc * (st.k11 - me[5]) + half * (R(1) + svc) * S5;
    Q21 = me[6] + s3c * (st.k21 - me[6]) + s3h * S6;
    Q12 = me[7] + s3c * (st.k12 - me[7]) + s3h * S7;
    Q22 = me[8] + (R(1) - s4) * (st.k22 - me[8]) + (R(1) - half * s4) * S8;
  }

  // scales of the stored planes
  constexpr R sF = std::is_same<typename P::F, _Float16>::value ? R(kF16Scale) : R(1);
  constexpr R sG = std::is_same<typename P::G, _Float16>::value ? R(kF16Scale) : R(1);

  // populations f* = M^-1 m* (deviations; M^-1 maps the rest moments to w_i)
  const R hF = half * sF, qF = quarter * sF;
  const R h20 = hF * (Q20 - Q22), h02 = hF * (Q02 - Q22);
  const R f1 = hF * (K10 - Q12) + h20;
  const R f3 = hF * (Q12 - K10) + h20;
  const R f2 = hF * (K01 - Q21) + h02;
  const R f4 = hF * (Q21 - K01) + h02;
  const R pa = qF * (Q22 + Q21), pb = qF * (Q11 + Q12);
  const R pc = qF * (Q22 - Q21), pd = qF * (Q11 - Q12);
  const R f5 = pa + pb;  // (k11 + k21 + k12 + k22)/4
  const R f6 = pa - pb;  // (-k11 + k21 - k12 + k22)/4
  const R f7 = pc + pd;  // (k11 - k21 - k12 + k22)/4
  const R f8 = pc - pd;  // (-k11 - k21 + k12 + k22)/4
  // rest population (row f0 of M^-1: k00 - k20 - k02 + k22; as deviations
  // the rest values cancel, and k00* = rho conserves mass)
  const R f0 = (dr - Q20 - Q02 + Q22) * sF;

  // D2Q5 (Eqs. 28-33, A2) in closed form, as deviations
  const R T = cst<R>(d).T0 + st.th;
  const R hvth = cst<R>(d).hv * st.th;
  const R zac = cst<R>(d).zac;
  const R q1 = zac * (st.n1 - ux * T);
  const R q2 = zac * (st.n2 - uy * T);
  R ax_, ay_;  // post-collision raw moments g1 + g3, g2 + g4 (deviations)
  if constexpr (!RAW) {
    const R e3t = cst<R>(d).zec * (ux2 * T - two * ux * st.n1 + st.n3 - hvth);
    const R e4t = cst<R>(d).znc * (uy2 * T - two * uy * st.n2 + st.n4 - hvth);
    ax_ = ux2 * T + q1 * two * ux + e3t + hvth;
    ay_ = uy2 * T + q2 * two * uy + e4t + hvth;
  } else {  // MRT: toward the raw equilibria of Eq. 33
    ax_ = ux2 * T + hvth + cst<R>(d).zec * (st.n3 - hvth - ux2 * T);
    ay_ = uy2 * T + hvth + cst<R>(d).znc * (st.n4 - hvth - uy2 * T);
  }
  const R bx_ = ux * T + q1, by_ = uy * T + q2;
  const R hG = half * sG;
  const R g1 = hG * (ax_ + bx_);
  const R g3 = hG * (ax_ - bx_);
  const R g2 = hG * (ay_ + by_);
  const R g4 = hG * (ay_ - by_);
  // rest population from heat conservation (equal to
  // (sigma - varpi) theta - |u|^2 T - 2 u.q - e3 - e4)
  R g0;
  if constexpr (kCompensatedRest<P>) {
    // g0 + rest_err = (sg + sg_lo) - ((g1 + g3) + (g2 + g4)) with only the
    // two pair sums rounded
    R e1, e2;
    const R gs = two_sum(g1 + g3, g2 + g4, e1);
    g0 = two_sum(st.sg, -gs, e2);
    rest_err = (e2 - e1) + st.sg_lo;
  } else {
    g0 = st.sg * sG - ((g1 + g3) + (g2 + g4));
  }

  out[0] = f0;
  out[1] = f1;
  out[2] = f2;
  out[3] = f3;
  out[4] = f4;
  out[5] = f5;
  out[6] = f6;
  out[7] = f7;
  out[8] = f8;
  out[9] = g0;
  out[10] = g1;
  out[11] = g2;
  out[12] = g3;
  out[13] = g4;
}

// Store post-collision deviations to the planes of `buf` at element offset
// idx, stochastically rounded with random words of (idx, seed); rest_err is
// the rounding error of the D2Q5 rest population (kCompensatedRest).
template <typename P, typename R = typename P::R>
__device__ __forceinline__ void store_planes(const CavDesc &d, const R out[kPlanes], R rest_err,
                                             char *__restrict__ buf, int idx, uint32_t seed) {
  const int plane = d.plane;
  typename P::F *of = const_cast<typename P::F *>(fplanes<P>(buf));
  typename P::G *og = const_cast<typename P::G *>(gplanes<P>(buf, plane));
  const uint32_t uidx = (uint32_t)idx;
  // random words for the stochastic rounding: two fields per word (the
  // compensated rest population, the only rounding of that policy, takes the
  // node's first word)
  uint32_t w = mix32((uint32_t)idx + seed);
  const uint32_t w0 = w;
  EncState e;
#pragma unroll
  for (int i = 0; i < kPlanes; ++i) {
    if (i < 9)
      stv(e, at(uniform_base(of + (size_t)i * plane), uidx), out[i], round_bits<R>(w, i));
    else if (i == 9 && kCompensatedRest<P>)
      stv(e, at(uniform_base(og), uidx), round_pair_sr(out[9], rest_err, w0 >> 16), 0u);
    else
      stv(e, at(uniform_base(og + (size_t)(i - 9) * plane), uidx), out[i],
          round_bits<R>(w, i));
    if (i & 1) w = next_bits<R>(w);
  }
}

// The values store_planes writes (same random words, same rounding) into the
// two-step kernel's LDS region at element c.
template <typename P, int TX, typename R = typename P::R>
__device__ __forceinline__ void store_region(const R out[kPlanes], R rest_err, char *lds, int c,
                                             int idx, uint32_t seed) {
  typename P::F *F = RegionPlanes<P, TX>::f(lds);
  typename P::G *G = RegionPlanes<P, TX>::g(lds);
  constexpr int N = Region<TX>::N;
  uint32_t w = mix32((uint32_t)idx + seed);
  const uint32_t w0 = w;
  EncState e;
#pragma unroll
  for (int i = 0; i < kPlanes; ++i) {
    const uint32_t r = round_bits<R>(w, i);
    if (i < 9)
      F[i * N + c] = enc(e, F, out[i], r);
    else if (i == 9 && kCompensatedRest<P>)
      G[c] = round_pair_sr(out[9], rest_err, w0 >> 16);
    else
      G[(i - 9) * N + c] = enc(e, G, out[i], r);
    if (i & 1) w = next_bits<R>(w);
  }
}

template <typename P, bool RAW, bool ROWS, typename R = typename P::R>
__device__ __forceinline__ void collide_store(const CavDesc &d, const NodeState<R> &st, bool wall,
                                              char *__restrict__ buf, int idx, uint32_t seed) {
  R out[kPlanes], rest_err = 0;
  collide<P, RAW, ROWS>(d, st, wall, out, rest_err);
  store_planes<P>(d, out, rest_err, buf, idx, seed);
}

// ------------------------------------------------------------ step kernel

// One time step of every tile in tiles[0 .. counts[0]).  parity selects the
// source buffer (0: A -> B, 1: B -> A).  write_snap records (u, v, theta) of
// the collision for the residual.  counts[2 + parity] holds the index of this
// step; the kernel passes it on in counts[3 - parity] for the next launch, so
// captured graphs need no baked-in step numbers.
template <typename P, bool RAW, bool ROWS>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(5))) step_kernel(const CavDesc *__restrict__ descs,
                                                   const Tile *__restrict__ tiles,
                                                   int32_t *__restrict__ counts, int parity,
                                                   int write_snap) {
  using R = typename P::R;
  const int ntiles = counts[0];
  const uint32_t step = (uint32_t)counts[2 + parity];
  if (blockIdx.x == 0 && threadIdx.x == 0) counts[3 - parity] = (int32_t)(step + 1);
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int cav = __builtin_amdgcn_readfirstlane(tiles[t].cav);
    if (cav < 0) continue;  // padding entry of the XCD-ordered list
    const int x0 = __builtin_amdgcn_readfirstlane(tiles[t].x0);
    const int y0 = __builtin_amdgcn_readfirstlane(tiles[t].y0);
    const CavDesc &d = descs[cav];
    const int lw = d.tw_log2;
    const int x = x0 + (int)(threadIdx.x & ((1u << lw) - 1u)), y = y0 + (int)(threadIdx.x >> lw);
    if (x < d.nx && y < d.ny) {
      const char *A = parity ? d.B : d.A;
      char *B = parity ? d.A : d.B;
      NodeState<R> st;
      const bool wall = node_state<P, ROWS>(d, GlobalSrc<P>{A}, x, y, st);
      const int idx = y * d.pitch + x;
      const uint32_t seed = mix32(step * 0x9E3779B9u + (uint32_t)cav * 0x85EBCA6Bu);
      collide_store<P, RAW, ROWS>(d, st, wall, B, idx, seed);
      if (write_snap) {
        d.snap[idx] = (float)st.ux;
        d.snap[(size_t)d.plane + idx] = (float)st.uy;
        d.snap[(size_t)2 * d.plane + idx] = (float)st.th;
      }
    }
  }
}

// ------------------------------------------------------- two-step kernel

// Two time steps of every tile of a two-step tile list (TX x kFusedY nodes,
// TX = 64 or 128, kThreads2<P, TX> threads) in one launch, any storage
// policy P.  Step one collides the tile
// and a one-node ring around it from the source buffer into LDS, in the
// storage types of P and with the values a stored step would hold (the same
// stochastic rounding); step two collides the tile again from LDS and stores
// it to the other buffer.  The populations cross HBM once per two node
// updates; each ring is recomputed by the neighbouring tiles.  The region is
// in unwrapped coordinates: the ring of a tile at a periodic side holds the
// wrapped neighbours, and ring nodes outside a walled side are neither
// computed nor read (boundary nodes gather inward).  *len holds the length
// of the tile list (the tiles of the active domains; the grid may be longer),
// counts[2 + parity] the index of the first step, and the kernel passes
// step + 2 on (the launches of the 64- and the 128-wide tiles of one pair of
// steps read and write the same values).  write_snap records (u, v, theta) of
// the second step.
template <typename P, int TX, bool RAW, bool ROWS>
__global__ void __launch_bounds__((kThreads2<P, TX>)) step2_kernel(const CavDesc *__restrict__ descs,
                                                       const Tile *__restrict__ tiles,
                                                       int32_t *__restrict__ counts,
                                                       const int32_t *__restrict__ len,
                                                       int parity, int write_snap) {
  using R = typename P::R;
  constexpr int kRegionW = Region<TX>::W, kRegion = Region<TX>::N;
  __shared__ __attribute__((aligned(16))) char lds[RegionPlanes<P, TX>::kBytes];
  const int ntiles = *len;  // the list of the active domains
  const uint32_t step = (uint32_t)counts[2 + parity];
  if (blockIdx.x == 0 && threadIdx.x == 0) counts[3 - parity] = (int32_t)(step + 2);
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int cav = __builtin_amdgcn_readfirstlane(tiles[t].cav);
    if (cav < 0) continue;  // padding entry of the XCD-ordered list
    const int x0 = __builtin_amdgcn_readfirstlane(tiles[t].x0);
    const int y0 = __builtin_amdgcn_readfirstlane(tiles[t].y0);
    const CavDesc &d = descs[cav];
    const char *A = parity ? d.B : d.A;
    char *B = parity ? d.A : d.B;
    const bool wrap_x = d.bc[0] == kPeriodic, wrap_y = d.bc[2] == kPeriodic;
    // Both steps of the tile.  EDGE = false: the tile's region holds no
    // boundary node and every pull stays inside the domain (no wrap, no
    // skipped ring node), so the per-node side tests are left out.  (A
    // lambda rather than a separate function: the compiler then keeps the
    // domain constants out of the scalar registers as in the plain loop.)
    auto tile = [&](auto edge_tag) {
      constexpr bool EDGE = decltype(edge_tag)::value;
      const uint32_t seed1 = mix32(step * 0x9E3779B9u + (uint32_t)cav * 0x85EBCA6Bu);
      for (int c = threadIdx.x; c < kRegion; c += blockDim.x) {
        int x = x0 - 1 + c % kRegionW, y = y0 - 1 + c / kRegionW;
        if constexpr (EDGE) {
          if (wrap_x) x = x < 0 ? x + d.nx : (x >= d.nx ? x - d.nx : x);
          if (wrap_y) y = y < 0 ? y + d.ny : (y >= d.ny ? y - d.ny : y);
          if (x < 0 || x >= d.nx || y < 0 || y >= d.ny) continue;
        }
        NodeState<R> st;
        const bool wall =
            node_state<P, ROWS, GlobalSrc<P, EDGE>, EDGE>(d, GlobalSrc<P, EDGE>{A}, x, y, st);
        R out[kPlanes], rest_err = 0;
        collide<P, RAW, ROWS>(d, st, wall, out, rest_err);
        store_region<P, TX>(out, rest_err, lds, c, y * d.pitch + x, seed1);
      }
      __syncthreads();
      const uint32_t seed2 = mix32((step + 1) * 0x9E3779B9u + (uint32_t)cav * 0x85EBCA6Bu);
      const LdsSrc<P, TX> src{lds, x0 - 1, y0 - 1};
      for (int q = threadIdx.x; q < TX * kFusedY; q += blockDim.x) {
        const int x = x0 + q % TX, y = y0 + q / TX;
        if constexpr (EDGE) {
          if (x >= d.nx || y >= d.ny) continue;
        }
        NodeState<R> st;
        const bool wall = node_state<P, ROWS, LdsSrc<P, TX>, EDGE>(d, src, x, y, st);
        const int idx = y * d.pitch + x;
        collide_store<P, RAW, ROWS>(d, st, wall, B, idx, seed2);
        if (write_snap) {
          d.snap[idx] = (float)st.ux;
          d.snap[(size_t)d.plane + idx] = (float)st.uy;
          d.snap[(size_t)2 * d.plane + idx] = (float)st.th;
        }
      }
    };
    // Interior tiles take the path without side tests in the wide kernel.
    // The narrow one serves contexts with small domains, whose tiles are
    // mostly edge tiles: there a second copy of the body costs more
    // (instruction cache, registers) than it saves.
    if constexpr (TX == kFusedXWide) {
      if (__builtin_amdgcn_readfirstlane(tiles[t].id))
        tile(std::true_type{});
      else
        tile(std::false_type{});
    } else {
      tile(std::true_type{});
    }
    __syncthreads();  // the next tile overwrites the region
  }
}

// ------------------------------------------------------------ init kernel

// Equilibrium population (deviation) of direction i for rho = 1 and u.
__device__ __forceinline__ double feq_dev_dir(int i, double ux, double uy, double ip) {
  double m[9];
  meq_dev(0.0, ux, uy, ip, m);
  // M^-1 rows (populations from raw moments)
  switch (i) {
    case 0: return m[0] - m[3] - m[4] + m[8];
    case 1: return 0.5 * (m[1] + m[3] - m[7] - m[8]);
    case 2: return 0.5 * (m[2] + m[4] - m[6] - m[8]);
    case 3: return 0.5 * (-m[1] + m[3] + m[7] - m[8]);
    case 4: return 0.5 * (-m[2] + m[4] + m[6] - m[8]);
    case 5: return 0.25 * (m[5] + m[6] + m[7] + m[8]);
    case 6: return 0.25 * (-m[5] + m[6] - m[7] + m[8]);
    case 7: return 0.25 * (m[5] - m[6] - m[7] + m[8]);
    default: return 0.25 * (-m[5] - m[6] + m[7] + m[8]);
  }
}

// g_i^eq(T, u) - g_i^eq(T0, 0) from Eq. 34.
__device__ __forceinline__ double geq_dev_dir(const CavDesc &d, int i, double ux, double uy,
                                              double th) {
  const double T = d.c.T0 + th;
  switch (i) {
    case 0: return d.c.sig_mv * th - (ux * ux + uy * uy) * T;
    case 1: return 0.5 * d.c.hv * th + 0.5 * (ux + ux * ux) * T;
    case 2: return 0.5 * d.c.hv * th + 0.5 * (uy + uy * uy) * T;
    case 3: return 0.5 * d.c.hv * th + 0.5 * (ux * ux - ux) * T;
    default: return 0.5 * d.c.hv * th + 0.5 * (uy * uy - uy) * T;
  }
}

// Fill the current buffer of one domain so that the next pull (streaming)
// delivers the equilibrium of the given fields at every node: element i of
// node x holds the equilibrium of node x + e_i (its own when x + e_i lies
// outside a non-periodic side; boundary nodes rebuild those entries anyway).
template <typename P>
__global__ void init_kernel(const CavDesc *__restrict__ descs, int cav, int parity,
                            const float *__restrict__ uvth, float th_uniform) {
  using F = typename P::F;
  using G = typename P::G;
  const CavDesc &d = descs[cav];
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= d.nx || y >= d.ny) return;
  const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  char *buf = parity ? d.B : d.A;
  F *A = const_cast<F *>(fplanes<P>(buf));
  G *Gp = const_cast<G *>(gplanes<P>(buf, d.plane));
  const size_t n = (size_t)d.nx * d.ny;
  const double scf = sizeof(F) == 2 ? (double)kF16Scale : 1.0;
  const double scg = sizeof(G) == 2 ? (double)kF16Scale : 1.0;
  for (int i = 0; i < 9; ++i) {
    int xs = x + ex[i], ys = y + ey[i];
    bool outside = false;
    if (xs < 0 || xs >= d.nx) {
      if (d.bc[0] == kPeriodic) xs = (xs + d.nx) % d.nx;
      else outside = true;
    }
    if (ys < 0 || ys >= d.ny) {
      if (d.bc[2] == kPeriodic) ys = (ys + d.ny) % d.ny;
      else outside = true;
    }
    if (outside) {
      xs = x;
      ys = y;
    }
    double ux = 0.0, uy = 0.0, th = th_uniform;
    if (uvth) {
      const size_t k = (size_t)ys * d.nx + xs;
      ux = uvth[k];
      uy = uvth[n + k];
      th = uvth[2 * n + k];
    }
    double phi, ip, cd, cf;
    medium_at(d, ys * d.pitch + xs, phi, ip, cd, cf);
    const int idx = y * d.pitch + x;
    A[(size_t)i * d.plane + idx] = (F)(scf * feq_dev_dir(i, ux, uy, ip));
    if (i < 5) Gp[(size_t)i * d.plane + idx] = (G)(scg * geq_dev_dir(d, i, ux, uy, th));
  }
}

// ------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum kRed doubles over a block in a fixed order; result valid in thread 0.
__device__ __forceinline__ void block_sum(double (&v)[kRed], double (*lds)[kRed]) {
  const int tid = threadIdx.x;
  const int nthreads = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63;
  for (int k = 0; k < kRed; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0)
    for (int k = 0; k < kRed; ++k) lds[wave][k] = v[k];
  __syncthreads();
  if (tid == 0) {
    const int nw = (nthreads + 63) >> 6;
    for (int k = 0; k < kRed; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += lds[w][k];
      v[k] = s;
    }
  }
}

// Residual partial sums of one tile per block.
template <typename P>
__global__ void __launch_bounds__(512) residual_kernel(const CavDesc *__restrict__ descs,
                                                       const Tile *__restrict__ tiles, int parity,
                                                       double *__restrict__ partials) {
  using R = typename P::R;
  __shared__ double lds[8][kRed];
  const int t = blockIdx.x;
  const int cav = __builtin_amdgcn_readfirstlane(tiles[t].cav);
  if (cav < 0) return;  // padding entry of an active list (uniform per block)
  const CavDesc &d = descs[cav];
  const int lw = d.tw_log2;
  const int x = tiles[t].x0 + (int)(threadIdx.x & ((1u << lw) - 1u));
  const int y = tiles[t].y0 + (int)(threadIdx.x >> lw);
  double v[kRed] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (x < d.nx && y < d.ny) {
    const char *A = parity ? d.B : d.A;
    NodeState<R> st;
    node_state<P, true>(d, GlobalSrc<P>{A}, x, y, st);
    const int idx = y * d.pitch + x;
    // the snapshot holds FP32 values: compare like with like
    const double ux = (double)(float)st.ux, uy = (double)(float)st.uy, th = (double)(float)st.th;
    const double du = ux - d.snap[idx];
    const double dv = uy - d.snap[(size_t)d.plane + idx];
    const double dth = th - d.snap[(size_t)2 * d.plane + idx];
    const double T = d.c.T0 + (double)st.th;
    v[0] = du * du + dv * dv;
    v[1] = (double)st.ux * (double)st.ux + (double)st.uy * (double)st.uy;
    v[2] = dth * dth;
    v[3] = T * T;
    v[4] = (double)st.dr;
    const bool bad = !isfinite((double)st.ux) || !isfinite((double)st.uy) ||
                     !isfinite((double)st.th) || !isfinite((double)st.rho);
    v[5] = bad ? 1.0 : 0.0;
    v[6] = 1.0;
  }
  block_sum(v, lds);
  const size_t slot = (size_t)tiles[t].id * kRed;
  if (threadIdx.x == 0)
    for (int k = 0; k < kRed; ++k) partials[slot + k] = v[k];
}

// Per-domain totals of the tile partial sums in two fixed-order passes
// (deterministic): block (g, cav) adds the partial sums of tiles
// [256 g, 256 g + 256) of the domain into gpart slot tile0 + g; one block per
// domain then adds its group sums.
constexpr int kGroup = 256;

__global__ void __launch_bounds__(256) residual_groups(const CavDesc *__restrict__ descs,
                                                       const double *__restrict__ partials,
                                                       double *__restrict__ gpart) {
  __shared__ double lds[4][kRed];
  const CavDesc &d = descs[blockIdx.y];
  const int g = blockIdx.x;
  if (g * kGroup >= d.ntiles) return;  // uniform per block
  double v[kRed] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int t = g * kGroup + threadIdx.x;
  if (t < d.ntiles)
    for (int k = 0; k < kRed; ++k) v[k] = partials[(size_t)(d.tile0 + t) * kRed + k];
  block_sum(v, lds);
  if (threadIdx.x == 0)
    for (int k = 0; k < kRed; ++k) gpart[(size_t)(d.tile0 + g) * kRed + k] = v[k];
}

__global__ void __launch_bounds__(256) residual_finalize(const CavDesc *__restrict__ descs,
                                                         const double *__restrict__ gpart,
                                                         double *__restrict__ results) {
  __shared__ double lds[4][kRed];
  const CavDesc &d = descs[blockIdx.x];
  const int ng = (d.ntiles + kGroup - 1) / kGroup;
  double v[kRed] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int g = threadIdx.x; g < ng; g += blockDim.x)
    for (int k = 0; k < kRed; ++k) v[k] += gpart[(size_t)(d.tile0 + g) * kRed + k];
  block_sum(v, lds);
  if (threadIdx.x == 0)
    for (int k = 0; k < kRed; ++k) results[(size_t)blockIdx.x * kRed + k] = v[k];
}

// Macroscopic fields of one domain into 4 dense planes: rho - 1, u, v, theta.
template <typename P>
__global__ void __launch_bounds__(512) macros_kernel(const CavDesc *__restrict__ descs,
                                                     const Tile *__restrict__ tiles, int tile0,
                                                     int parity, float *__restrict__ out) {
  using R = typename P::R;
  const int t = tile0 + blockIdx.x;
  const int cav = __builtin_amdgcn_readfirstlane(tiles[t].cav);
  const CavDesc &d = descs[cav];
  const int lw = d.tw_log2;
  const int x = tiles[t].x0 + (int)(threadIdx.x & ((1u << lw) - 1u));
  const int y = tiles[t].y0 + (int)(threadIdx.x >> lw);
  if (x >= d.nx || y >= d.ny) return;
  const char *A = parity ? d.B : d.A;
  NodeState<R> st;
  node_state<P, true>(d, GlobalSrc<P>{A}, x, y, st);
  const size_t n = (size_t)d.nx * d.ny, k = (size_t)y * d.nx + x;
  out[k] = (float)st.dr;
  out[n + k] = (float)st.ux;
  out[2 * n + k] = (float)st.uy;
  out[3 * n + k] = (float)st.th;
}

// Mean Nusselt number of one side per domain (one block per domain):
// Nu_j = -L dT/dn / dT with the one-sided derivative (-3 T0 + 4 T1 - T2)/2 taken
// from the wall inward, trapezoid mean over the wall nodes.
template <typename P>
__global__ void __launch_bounds__(256) nusselt_kernel(const CavDesc *__restrict__ descs, int cav0,
                                                      int side, int parity,
                                                      double *__restrict__ nu_part,
                                                      int max_chunks,
                                                      double *__restrict__ nu_local) {
  using R = typename P::R;
  __shared__ double lds[4][kRed];
  const int cav = cav0 + blockIdx.y;
  const CavDesc &d = descs[cav];
  const char *A = parity ? d.B : d.A;
  const bool along_y = side < 2;
  const int nw = along_y ? d.ny : d.nx;
  if ((int)blockIdx.x * 256 >= nw) return;  // uniform per block
  const double L = along_y ? d.nx - 1 : d.ny - 1;
  const double sign = (side == 0 || side == 2) ? 1.0 : -1.0;
  double v[kRed] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < nw) {
    double t[3];
    for (int k = 0; k < 3; ++k) {
      int x, y;
      if (along_y) {
        y = j;
        x = side == 0 ? k : d.nx - 1 - k;
      } else {
        x = j;
        y = side == 2 ? k : d.ny - 1 - k;
      }
      NodeState<R> st;
      node_state<P, true>(d, GlobalSrc<P>{A}, x, y, st);
      t[k] = (double)st.th;  // the gradient does not depend on the reference T0
    }
    const double nu = -L * sign * (-3.0 * t[0] + 4.0 * t[1] - t[2]) * 0.5 / d.c.dT;
    if (nu_local) nu_local[j] = nu;
    v[0] = (j == 0 || j == nw - 1) ? 0.5 * nu : nu;  // trapezoid weights
  }
  block_sum(v, lds);
  if (threadIdx.x == 0) nu_part[(size_t)cav * max_chunks + blockIdx.x] = v[0];
}

// Mean Nusselt number of each domain from its chunk sums (fixed order).
__global__ void __launch_bounds__(64) nusselt_finalize(const CavDesc *__restrict__ descs,
                                                       int cav0, int side,
                                                       const double *__restrict__ nu_part,
                                                       int max_chunks,
                                                       double *__restrict__ nu_mean) {
  const int cav = cav0 + blockIdx.x;
  const CavDesc &d = descs[cav];
  const int nw = side < 2 ? d.ny : d.nx;
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int c = 0; c * 256 < nw; ++c) s += nu_part[(size_t)cav * max_chunks + c];
  nu_mean[cav] = s / (nw - 1);
}

// --------------------------------------------------------------- launchers

static dim3 block_of(const LaunchShape &s) { return dim3(s.threads(), 1, 1); }

// Calls f(StoreX{}) for the storage kind of the context (0 FP32, 1 FP16,
// 2 FP16 flow + FP32 temperature).
template <typename Fn>
static void dispatch(int storage, Fn &&f) {
  if (storage == 0)
    f(StoreF32{});
  else if (storage == 1)
    f(StoreF16{});
  else if (storage == 2)
    f(StoreMix{});
  else
    f(StoreF32C{});
}

hipError_t launch_step(const CavDesc *descs, const Tile *tiles, int32_t *counts,
                       int32_t grid_tiles, int parity, int write_snap, int storage, int raw,
                       int rows, LaunchShape shape, hipStream_t s) {
  if (grid_tiles <= 0) return hipSuccess;
  const int blocks = shape.blocks > 0 && shape.blocks < grid_tiles ? shape.blocks : grid_tiles;
  const dim3 grid(blocks), block = block_of(shape);
  dispatch(storage, [&](auto p) {
    using P = decltype(p);
    if (raw && rows)
      hipLaunchKernelGGL((step_kernel<P, true, true>), grid, block, 0, s, descs, tiles, counts,
                         parity, write_snap);
    else if (raw)
      hipLaunchKernelGGL((step_kernel<P, true, false>), grid, block, 0, s, descs, tiles, counts,
                         parity, write_snap);
    else if (rows)
      hipLaunchKernelGGL((step_kernel<P, false, true>), grid, block, 0, s, descs, tiles, counts,
                         parity, write_snap);
    else
      hipLaunchKernelGGL((step_kernel<P, false, false>), grid, block, 0, s, descs, tiles,
                         counts, parity, write_snap);
  });
  return hipGetLastError();
}

namespace {
template <typename P, int TX>
void launch_step2_tx(const CavDesc *descs, const Tile *tiles, int32_t ntiles, int32_t *counts,
                     const int32_t *len, int parity, int write_snap, int raw, int rows,
                     hipStream_t s) {
  const dim3 grid(ntiles), block(kThreads2<P, TX>);
  if (raw && rows)
    hipLaunchKernelGGL((step2_kernel<P, TX, true, true>), grid, block, 0, s, descs, tiles, counts,
                       len, parity, write_snap);
  else if (raw)
    hipLaunchKernelGGL((step2_kernel<P, TX, true, false>), grid, block, 0, s, descs, tiles,
                       counts, len, parity, write_snap);
  else if (rows)
    hipLaunchKernelGGL((step2_kernel<P, TX, false, true>), grid, block, 0, s, descs, tiles,
                       counts, len, parity, write_snap);
  else
    hipLaunchKernelGGL((step2_kernel<P, TX, false, false>), grid, block, 0, s, descs, tiles,
                       counts, len, parity, write_snap);
}

template <typename P>
hipError_t launch_step2_p(const CavDesc *descs, const Tile *tiles, int32_t ntiles,
                          int32_t *counts, const int32_t *len, int parity, int write_snap,
                          int raw, int rows, int tile_x, hipStream_t s) {
  if (tile_x == kFusedXWide)
    launch_step2_tx<P, kFusedXWide>(descs, tiles, ntiles, counts, len, parity, write_snap, raw,
                                    rows, s);
  else if (tile_x == kFusedX)
    launch_step2_tx<P, kFusedX>(descs, tiles, ntiles, counts, len, parity, write_snap, raw, rows,
                                s);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
}  // namespace

hipError_t launch_step2(const CavDesc *descs, const Tile *tiles, int32_t ntiles, int32_t *counts,
                        const int32_t *len, int parity, int write_snap, int storage, int raw,
                        int rows, int tile_x, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (storage == 0)  // FP32 planes, FP64 arithmetic
    return launch_step2_p<StoreF32>(descs, tiles, ntiles, counts, len, parity, write_snap, raw,
                                    rows, tile_x, s);
  if (storage == 3)  // FP32 planes, FP32 arithmetic
    return launch_step2_p<StoreF32C>(descs, tiles, ntiles, counts, len, parity, write_snap, raw,
                                     rows, tile_x, s);
  if (storage == 1)  // FP16 planes
    return launch_step2_p<StoreF16>(descs, tiles, ntiles, counts, len, parity, write_snap, raw,
                                    rows, tile_x, s);
  if (storage == 2)  // FP16 flow, FP32 temperature planes
    return launch_step2_p<StoreMix>(descs, tiles, ntiles, counts, len, parity, write_snap, raw,
                                    rows, tile_x, s);
  return hipErrorInvalidValue;
}

hipError_t launch_init(const CavDesc *descs, int32_t cav, int nx, int ny, int parity,
                       const float *uvth, float th_uniform, int storage, hipStream_t s) {
  const dim3 blk(64, 4, 1), grd((nx + 63) / 64, (ny + 3) / 4, 1);
  dispatch(storage, [&](auto p) {
    using P = decltype(p);
    hipLaunchKernelGGL(init_kernel<P>, grd, blk, 0, s, descs, cav, parity, uvth, th_uniform);
  });
  return hipGetLastError();
}

hipError_t launch_residual(const CavDesc *descs, const Tile *tiles, int32_t ntiles, int parity,
                           double *partials, int storage, LaunchShape shape, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  dispatch(storage, [&](auto p) {
    using P = decltype(p);
    hipLaunchKernelGGL(residual_kernel<P>, dim3(ntiles), block_of(shape), 0, s, descs, tiles,
                       parity, partials);
  });
  return hipGetLastError();
}

hipError_t launch_residual_finalize(const CavDesc *descs, int32_t count, int32_t max_groups,
                                    const double *partials, double *gpart, double *results,
                                    hipStream_t s) {
  hipLaunchKernelGGL(residual_groups, dim3(max_groups, count), dim3(kGroup), 0, s, descs, partials,
                     gpart);
  hipLaunchKernelGGL(residual_finalize, dim3(count), dim3(256), 0, s, descs, gpart, results);
  return hipGetLastError();
}

hipError_t launch_macros(const CavDesc *descs, const Tile *tiles, int32_t tile0, int32_t ntiles,
                         int parity, float *out, int storage, LaunchShape shape, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  dispatch(storage, [&](auto p) {
    using P = decltype(p);
    hipLaunchKernelGGL(macros_kernel<P>, dim3(ntiles), block_of(shape), 0, s, descs, tiles, tile0,
                       parity, out);
  });
  return hipGetLastError();
}

hipError_t launch_nusselt(const CavDesc *descs, int32_t cav0, int32_t ncav, int32_t side,
                          int parity, double *nu_mean, double *nu_local, double *nu_part,
                          int32_t max_chunks, int storage, hipStream_t s) {
  dispatch(storage, [&](auto p) {
    using P = decltype(p);
    hipLaunchKernelGGL(nusselt_kernel<P>, dim3(max_chunks, ncav), dim3(256), 0, s, descs, cav0,
                       side, parity, nu_part, max_chunks, nu_local);
  });
  hipLaunchKernelGGL(nusselt_finalize, dim3(ncav), dim3(64), 0, s, descs, cav0, side, nu_part,
                     max_chunks, nu_mean);
  return hipGetLastError();
}

}  // namespace clb
