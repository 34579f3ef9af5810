// HIP kernels for gfx950: fused pull collide-stream step with the ELIBB
// boundary (Sec. II.A-E), initialisation / import, state export and FP64
// moments.
//
// One wavefront handles one segment of 64 consecutive x of a row (y, z); a block
// holds 4 segments, i.e. a whole 256-wide row for the 256^3 D3Q19 case.  Every
// population slot is read by exactly one lane (its consumer) and written by
// exactly one lane (its producer), so a step needs no synchronisation across
// waves.  Boundary work is wave-local: the wave stages its boundary nodes in
// LDS and rebuilds its cut links one link per lane.
#include <hip/hip_runtime.h>

#include "elibb.hpp"
#include "internal.hpp"
#include "lattice.hpp"
#include "storage.hpp"

#ifndef LBM_LATTICE
#error "kernels.hip is compiled once per lattice: -DLBM_LATTICE=D2Q9 | D3Q19 | D3Q27"
#endif

namespace lbm {

struct Coords {
  int x, y, z;
};

// Segment of the calling wave and the lane's coordinates.  Workgroups are dealt
// round-robin to the 8 XCDs; the logical block id makes XCD k walk the k-th
// contiguous eighth of the rows (the grid is padded to a multiple of 8).
struct SegInfo {
  uint32_t seg;      // wave-uniform
  uint32_t sx;       // wave-uniform segment index within the row
  uint32_t row;      // wave-uniform row y + ny z
  int lane;
  Coords c;          // c.y, c.z wave-uniform
};

__device__ __forceinline__ uint32_t fast_div(uint32_t n, const FastDiv& f) {
  return (uint32_t)(((uint64_t)__umulhi(n, f.m) + n) >> f.s);
}

__device__ __forceinline__ uint32_t logical_block(int remap) {
  const uint32_t b = blockIdx.x;
  if (!remap) return b;
  const uint32_t per = gridDim.x >> 3;
  return (b & 7u) * per + (b >> 3);
}

__device__ __forceinline__ SegInfo seg_info(const GridGeom& g, uint32_t block) {
  SegInfo s;
  s.lane = threadIdx.x & (SEG - 1);
  const uint32_t wave = block * WAVES_PER_BLOCK + __builtin_amdgcn_readfirstlane(threadIdx.x / SEG);
  s.seg = wave;
  const uint32_t row = __builtin_amdgcn_readfirstlane(fast_div(wave, g.div_nseg_x));
  const uint32_t sx = __builtin_amdgcn_readfirstlane(wave - row * (uint32_t)g.nseg_x);
  const uint32_t z = __builtin_amdgcn_readfirstlane(fast_div(row, g.div_ny));
  s.sx = sx;
  s.row = row;
  s.c.x = (int)sx * SEG + s.lane;
  s.c.y = (int)__builtin_amdgcn_readfirstlane(row - z * (uint32_t)g.ny);
  s.c.z = (int)z;
  return s;
}

__device__ __forceinline__ SegInfo seg_info(const GridGeom& g) { return seg_info(g, logical_block(g.xcd_remap)); }

// Direction tables for a direction index known only at run time (the link
// phase): velocity components packed two bits per direction, weights by shell.
template <class L, int AXIS>
constexpr uint64_t packed_c() {
  uint64_t v = 0;
  for (int i = 0; i < L::Q; ++i) v |= uint64_t((AXIS == 0 ? L::cx(i) : AXIS == 1 ? L::cy(i) : L::cz(i)) + 1) << (2 * i);
  return v;
}
template <class L, int AXIS>
__device__ __forceinline__ int dyn_c(int i) {
  constexpr uint64_t P = packed_c<L, AXIS>();
  return int((P >> (2 * i)) & 3ull) - 1;
}
template <class L, typename R>
__device__ __forceinline__ R dyn_w(int i) {
  if (L::Q == 27 && i >= 19) return R(L::w(19));
  return i == 0 ? R(L::w(0)) : (i <= 2 * L::D ? R(L::w(1)) : R(L::w(2 * L::D + 1)));
}
// opposite direction: axis pairs (1,2),(3,4),...; then groups of four sign pairs
template <class L>
__device__ __forceinline__ int dyn_opp(int i) {
  if (i == 0) return 0;
  if (i <= 2 * L::D) return (i & 1) ? i + 1 : i - 1;
  if (L::Q == 27 && i >= 19) return 45 - i;   // corners: every sign flips
  const int r = (i - 2 * L::D - 1) & 3;
  return i - r + (3 - r);
}
template <class L>
constexpr bool dyn_tables_ok() {
  for (int i = 0; i < L::Q; ++i) {
    const bool corner = L::Q == 27 && i >= 19;
    const int r = (i - 2 * L::D - 1) & 3;
    const int o = i == 0 ? 0 : (i <= 2 * L::D ? ((i & 1) ? i + 1 : i - 1) : (corner ? 45 - i : i - r + (3 - r)));
    if (o != L::opp(i)) return false;
    const double w = corner ? L::w(19) : (i == 0 ? L::w(0) : (i <= 2 * L::D ? L::w(1) : L::w(2 * L::D + 1)));
    if (w != L::w(i)) return false;
  }
  return true;
}
static_assert(dyn_tables_ok<D2Q9>() && dyn_tables_ok<D3Q19>() && dyn_tables_ok<D3Q27>(), "run-time direction tables");

// Moments of the shifted populations at one node.
template <typename R>
struct Moments {
  R drho, rho, ux, uy, uz, uu;
};

// c_i . v for a direction whose components are constants after unrolling,
// written as signed sums (products with 0 are not dropped by the compiler).
template <class L, typename R>
__device__ __forceinline__ R cdot(int i, R x, R y, R z) {
  R s = R(0);
  bool any = false;
  auto acc = [&](int c, R v) {
    if (c == 0) return;
    s = any ? (c > 0 ? s + v : s - v) : (c > 0 ? v : -v);
    any = true;
  };
  acc(L::cx(i), x);
  acc(L::cy(i), y);
  acc(L::cz(i), z);
  return s;
}

// Parameters of the collision models, which act on shifted populations with
// h^eq_i = f^eq_i - w_i = w_i [ (rho - 1) + rho (3 cu + 4.5 cu^2 - 1.5 uu) ]
// (eq. Eq2ndOrder, c_s^2 = 1/3) and Guo's source S_i = w_i [ 3 (c_i - u).F + 9 (c_i.u)(c_i.F) ]:
//   BGK (eq. LB-BGK)  h*_i = h_i - omega (h_i - h^eq_i) + (1 - omega/2) S_i
//   TRT (TRT models)  h*_i = h_i - omega+ (h+_i - h^eq+_i) - omega- (h-_i - h^eq-_i)
//                            + (1 - omega+/2) S+_i + (1 - omega-/2) S-_i
// where g+-_i = (g_i +- g_ibar)/2: h^eq+ = w [(rho - 1) + rho (4.5 cu^2 - 1.5 uu)],
// h^eq- = 3 w rho cu, S+ = w [9 cu cF - 3 u.F], S- = 3 w cF.  The updates are
// evaluated by Pairs (below); heq() is the equilibrium alone (link rebuild).
template <typename R, bool TRT>
struct Collider {
  R omega, kf, Fx, Fy, Fz;
  R omega_m;                     // TRT: omega-
  R src_eq, src_eq_m;            // 3 (1 - omega/2) / omega, and with omega- (Pairs)
  bool force;
  __device__ __forceinline__ R heq(R cx, R cy, R cz, R w, const Moments<R>& m) const {
    const R cu = cx * m.ux + cy * m.uy + cz * m.uz;
    return w * ((m.drho - R(1.5) * m.rho * m.uu) + m.rho * cu * (R(3) + R(4.5) * cu));
  }
};

// The BGK / TRT + Guo updates above with the work of a direction and its
// opposite shared.  The source enters through the equilibrium (omega h^eq'_i =
// omega h^eq_i + (1 - omega/2) S_i, per parity for TRT), and h^eq'_i splits into
// parts even and odd in c_i, h^eq'_i = E + O, h^eq'_ibar = E - O:
//   E = w [t + cu (4.5 rho cu + 9 s cF)],  O = w [3 rho cu + 3 s- cF],
//   t = (rho - 1) - 1.5 rho uu - 3 s u.F,  s = (1 - omega/2) / omega,
//   s- = (1 - omega-/2) / omega- (= s for BGK),
// with cu = c_i.u, cF = c_i.F for the member i of the pair with the smaller
// index (with F = 0 the source terms add exact zeros).  Then
//   BGK  h*_i = h_i + omega ([E + O] - h_i),   h*_ibar = h_ibar + omega ([E - O] - h_ibar),
//   TRT  h*_i = h_i - P - M,  h*_ibar = h_ibar - P + M,
//        P = omega (h+ - E),  M = omega- (h- - O),  h+- = (h_i +- h_ibar) / 2.
// Both keep the form h + correction: regrouped as (1 - omega) h + omega h^eq the
// BGK update biases the rounding of the momentum, which then builds up over
// steps in steady flow.  The node's own update and the link rebuild, which needs
// the bounced post-collision values again, both go through these helpers
// (explicit fused operations, no contraction), so that the two agree to the bit.
template <typename R>
struct Pairs {
  R om, omm, t, r45, r3, s3, s9, s3m;
  template <bool TRT>
  __device__ __forceinline__ Pairs(const Collider<R, TRT>& col, const Moments<R>& m) {
#pragma clang fp contract(off)
    om = col.omega;
    omm = col.omega_m;
    s3 = col.src_eq;                           // 3 s
    s9 = R(3) * col.src_eq;                    // 9 s
    s3m = TRT ? col.src_eq_m : col.src_eq;     // 3 s-
    const R uF = fma(m.uz, col.Fz, fma(m.uy, col.Fy, m.ux * col.Fx));
    t = fma(-s3, uF, fma(R(-1.5) * m.rho, m.uu, m.drho));
    r45 = R(4.5) * m.rho;
    r3 = R(3) * m.rho;
  }
  // E and O of a pair with weight w
  __device__ __forceinline__ void eo(R w, R cu, R cF, R& e, R& o) const {
#pragma clang fp contract(off)
    e = fma(cu, fma(w * r45, cu, (w * s9) * cF), w * t);
    o = fma(w * r3, cu, (w * s3m) * cF);
  }
  // BGK: post-collision value of a pair member from its pre-collision value
  __device__ __forceinline__ R value(R h, R e, R o, bool lower) const {
#pragma clang fp contract(off)
    return fma(om, lower ? e + (o - h) : e - (o + h), h);
  }
  // TRT: post-collision values of the lower member (h) and the upper one (hbar)
  __device__ __forceinline__ void values_trt(R h, R hbar, R e, R o, R& out, R& outbar) const {
#pragma clang fp contract(off)
    const R p = fma(R(0.5) * om, h + hbar, -(om * e));
    const R q = fma(R(0.5) * omm, h - hbar, -(omm * o));
    out = (h - p) - q;
    outbar = (hbar - p) + q;
  }
  // the rest population (even: relaxed with omega in both models)
  __device__ __forceinline__ R rest(R h, R w) const {
#pragma clang fp contract(off)
    return fma(om, w * t - h, h);
  }
  // post-collision values of direction i (a constant after unrolling) and of its opposite
  template <class L, bool TRT>
  __device__ __forceinline__ void pair(int i, R h, R hbar, const Moments<R>& m, const Collider<R, TRT>& col, R& out,
                                       R& outbar) const {
    R e, o;
    eo(R(L::w(i)), cdot<L, R>(i, m.ux, m.uy, m.uz), cdot<L, R>(i, col.Fx, col.Fy, col.Fz), e, o);
    if constexpr (TRT) {
      values_trt(h, hbar, e, o, out, outbar);
    } else {
      out = value(h, e, o, true);
      outbar = value(hbar, e, o, false);
    }
  }
};

// u.u with a fixed evaluation order (the node update and the link rebuild both use it)
template <typename R>
__device__ __forceinline__ R dot_uu(R ux, R uy, R uz) {
#pragma clang fp contract(off)
  return fma(uz, uz, fma(uy, uy, ux * ux));
}

// Non-equilibrium stress Pi_ab = sum_j c_ja c_jb (f_j - f^eq_j(rho, u)) over the
// lattice's D axes.  From shifted populations h_j = f_j - w_j:
//   Pi = sum_j c c h_j - (rho - 1) cs2 delta - rho u u
// (sum_j w_j c c = cs2 delta cancels against the equilibrium's rho cs2 delta).
template <typename R>
struct Stress {
  R xx, yy, zz, xy, xz, yz;
};

// Stress of boundary node t from its staged pre-collision populations.
template <class L, typename R>
__device__ __forceinline__ Stress<R> neq_stress(const R (*stage)[BLOCK], int t, const Moments<R>& m) {
  Stress<R> s{R(0), R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
  for (int j = 1; j < L::Q; ++j) {
    const R h = stage[j][t];
    if (L::cx(j)) s.xx += h;
    if (L::cy(j)) s.yy += h;
    if (L::cz(j)) s.zz += h;
    if (L::cx(j) && L::cy(j)) s.xy += R(L::cx(j) * L::cy(j)) * h;
    if (L::cx(j) && L::cz(j)) s.xz += R(L::cx(j) * L::cz(j)) * h;
    if (L::cy(j) && L::cz(j)) s.yz += R(L::cy(j) * L::cz(j)) * h;
  }
  const R d3 = m.drho * R(1.0 / 3.0);
  s.xx -= d3 + m.rho * m.ux * m.ux;
  s.yy -= d3 + m.rho * m.uy * m.uy;
  s.xy -= m.rho * m.ux * m.uy;
  if constexpr (L::D == 3) {
    s.zz -= d3 + m.rho * m.uz * m.uz;
    s.xz -= m.rho * m.ux * m.uz;
    s.yz -= m.rho * m.uy * m.uz;
  }
  return s;
}

// Stress after collision.  Pi is an even moment: BGK and TRT both relax it with
// omega (= omega+), and Guo's source adds (1 - omega/2) sum_j c c S_j =
// (1 - omega/2) (u F + F u).
template <class L, typename R, bool TRT>
__device__ __forceinline__ Stress<R> post_stress(const Stress<R>& s, const Collider<R, TRT>& col, const Moments<R>& m) {
  const R k = R(1) - col.omega;
  Stress<R> o{k * s.xx, k * s.yy, k * s.zz, k * s.xy, k * s.xz, k * s.yz};
  if (col.force) {
    o.xx += col.kf * R(2) * m.ux * col.Fx;
    o.yy += col.kf * R(2) * m.uy * col.Fy;
    o.xy += col.kf * (m.ux * col.Fy + m.uy * col.Fx);
    if constexpr (L::D == 3) {
      o.zz += col.kf * R(2) * m.uz * col.Fz;
      o.xz += col.kf * (m.ux * col.Fz + m.uz * col.Fx);
      o.yz += col.kf * (m.uy * col.Fz + m.uz * col.Fy);
    }
  }
  return o;
}

// Wall non-equilibrium of direction c from the Hermite expansion truncated at
// third order (eq. fi_neq), with the stress as second-order coefficient and the
// third-order one from the recursion (eq. malaspinas):
//   w [ H2:Pi / (2 cs2^2) + H3:(u Pi + u Pi + u Pi) / (6 cs2^3) ]
//   = w [ 4.5 (cPc - tr Pi / 3) + 13.5 ((c.u) cPc - (2 u.Pi.c + (c.u) tr Pi) / 3) ].
template <typename R>
__device__ __forceinline__ R regularized_neq(R cx, R cy, R cz, R w, const Stress<R>& s, R ux, R uy, R uz) {
  const R tr = s.xx + s.yy + s.zz;
  const R pcx = s.xx * cx + s.xy * cy + s.xz * cz;
  const R pcy = s.xy * cx + s.yy * cy + s.yz * cz;
  const R pcz = s.xz * cx + s.yz * cy + s.zz * cz;
  const R cpc = cx * pcx + cy * pcy + cz * pcz;
  const R upc = ux * pcx + uy * pcy + uz * pcz;
  const R cu = cx * ux + cy * uy + cz * uz;
  const R third = R(1.0 / 3.0);
  return w * (R(4.5) * (cpc - tr * third) + R(13.5) * (cu * cpc - third * (R(2) * upc + cu * tr)));
}

template <class L, typename R>
__device__ __forceinline__ Moments<R> moments(const R (&h)[L::Q], R Fx, R Fy, R Fz) {
  // over the pairs (i, ibar): the sum h_i + h_ibar enters the density, the
  // difference h_i - h_ibar the momentum along the nonzero components of c_i
  R drho = h[0], jx = R(0), jy = R(0), jz = R(0);
  bool ax = false, ay = false, az = false;
  auto acc = [](R& s, bool& any, int c, R v) {
    if (c == 0) return;
    s = any ? (c > 0 ? s + v : s - v) : (c > 0 ? v : -v);
    any = true;
  };
#pragma unroll
  for (int i = 1; i < L::Q; ++i) {
    if (i > L::opp(i)) continue;
    const R sum = h[i] + h[L::opp(i)], dif = h[i] - h[L::opp(i)];
    drho += sum;
    acc(jx, ax, L::cx(i), dif);
    acc(jy, ay, L::cy(i), dif);
    acc(jz, az, L::cz(i), dif);
  }
  Moments<R> m;
  m.drho = drho;
  m.rho = R(1) + drho;
  R inv;
  if constexpr (sizeof(R) == 4) {
    // hardware reciprocal (1 ulp) refined by one Newton step
    const R r0 = __builtin_amdgcn_rcpf(m.rho);
    inv = r0 + r0 * (R(1) - m.rho * r0);
  } else {
    inv = R(1) / m.rho;
  }
  m.ux = (jx + R(0.5) * Fx) * inv;
  m.uy = (jy + R(0.5) * Fy) * inv;
  m.uz = (jz + R(0.5) * Fz) * inv;
  m.uu = dot_uu(m.ux, m.uy, m.uz);
  return m;
}

// Source coordinate of a pull along one axis: coord - c, wrapped on a periodic
// axis, clamped onto the face layer at an outlet face, and otherwise left one
// step outside (the dense layout's halo; the compact layout never reads it:
// such pulls are cut links, patched from their link values).
__device__ __forceinline__ int axis_src(int coord, int c, int n, int periodic, int out_lo, int out_hi) {
  int v = coord - c;
  if (periodic) return v < 0 ? v + n : (v >= n ? v - n : v);
  if (v < 0 && out_lo) return 0;
  if (v >= n && out_hi) return n - 1;
  return v;
}

// Dense layout: element offsets of the pull sources, xs[1 + cx] + ys[1 + cy] + zs[1 + cz].
struct DenseIndex {
  uint32_t xs[3], ys[3], zs[3];
  uint32_t self;
  template <class L>
  __device__ __forceinline__ uint32_t src(int i) const {
    return xs[1 + L::cx(i)] + ys[1 + L::cy(i)] + zs[1 + L::cz(i)];
  }
};

// A lane past the row's end (x >= nx) takes the indices of the row's last node,
// so that every lane of a wave may pull (such a lane stores nothing).
__device__ __forceinline__ DenseIndex dense_index(const GridGeom& g, Coords c) {
  const uint32_t NX = (uint32_t)g.NX, NXY = (uint32_t)g.NX * (uint32_t)g.NY;
  const int o = g.outlet;
  const int x = c.x < g.nx ? c.x : g.nx - 1;
  DenseIndex p;
#pragma unroll
  for (int k = 0; k < 3; ++k) {   // k = 1 + c, the source of direction c is x - c
    p.xs[k] = (uint32_t)(axis_src(x, k - 1, g.nx, g.perx, o == 0, o == 1) + g.px);
    p.ys[k] = (uint32_t)(axis_src(c.y, k - 1, g.ny, g.pery, o == 2, o == 3) + g.py) * NX;
    p.zs[k] = (uint32_t)(axis_src(c.z, k - 1, g.nz, g.perz, o == 4, o == 5) + g.pz) * NXY;
  }
  p.self = p.xs[1] + p.ys[1] + p.zs[1];
  return p;
}

// Compact layout: slot of fluid node (x, row r) = slot0 of its segment + the
// number of fluid lanes below x (G = 64 guard slots in front, so that a
// segment whose fluid count before it is a multiple of the line size starts
// on a cache line).  For each source row (y - cy, z - cz) the lane keeps
// P = slot the node x would have in that row and B = whether (x, row) is
// fluid; then the source slot of direction i is P (cx = 0), P - 1 (cx = +1,
// node x - 1) or P + B (cx = -1, node x + 1), with the periodic wrap of the row
// ends handled by lo / hi.  The first segment of every source row comes from a
// host-built table (row_src), so a wave forms its nine source segments with
// one add each instead of wrapping and clamping coordinates.
template <class L>
struct CompactIndex {
  uint32_t P[3][3], B[3][3], lo[3][3], hi[3][3];
  bool xlo, xhi;
  uint32_t self;
  template <class LL>
  __device__ __forceinline__ uint32_t src(int i) const {
    const int a = 1 + LL::cy(i), b = 1 + LL::cz(i);
    if (LL::cx(i) == 0) return P[a][b];
    if (LL::cx(i) == 1) return xlo ? lo[a][b] : P[a][b] - 1u;
    return xhi ? hi[a][b] : P[a][b] + B[a][b];
  }
};

template <class L>
__device__ __forceinline__ CompactIndex<L> compact_index(const GridGeom& g, const LinkView& lk, const SegInfo& si) {
  constexpr int NR = L::D == 2 ? 3 : 9;
  CompactIndex<L> p;
  const uint32_t sx = si.sx;
  // only the first and the last segment of a row hold the x-edge lanes; their
  // pulls wrap (periodic x) or clamp onto the node itself (outlet, walls)
  const bool edge = sx == 0 || sx == (uint32_t)g.nseg_x - 1;
  const bool wrap = edge && g.perx;
  const int32_t* rs = lk.row_src + (size_t)si.row * NR;
  uint64_t fm[3][3];
  uint32_t f0[3][3], ed[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (L::D == 2 && b != 1) continue;
      const uint32_t s = (uint32_t)load_const(rs + (L::D == 2 ? a : 3 * a + b)) + sx;
      fm[a][b] = load_const(lk.seg_fluid + s);
      f0[a][b] = (uint32_t)load_const(lk.seg_fbase + s) + (uint32_t)g.guard;
      if (wrap) {
        // first segment: the row's last fluid node; last segment: its first
        const uint32_t s0 = s - sx;
        ed[a][b] = sx == 0 ? (uint32_t)load_const(lk.seg_fbase + s0 + (uint32_t)g.nseg_x) + (uint32_t)g.guard - 1u
                           : (uint32_t)load_const(lk.seg_fbase + s0) + (uint32_t)g.guard;
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (L::D == 2 && b != 1) continue;
      // number of fluid nodes of this segment below the lane (one mbcnt pair)
      const uint32_t below =
          __builtin_amdgcn_mbcnt_hi((uint32_t)(fm[a][b] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)fm[a][b], 0u));
      p.P[a][b] = f0[a][b] + below;
      p.B[a][b] = (uint32_t)((fm[a][b] >> si.lane) & 1ull);
      if (wrap) {
        p.lo[a][b] = ed[a][b];                                     // last fluid node of the row
        p.hi[a][b] = g.nseg_x == 1 ? f0[a][b] : ed[a][b];          // first fluid node of the row
      } else {
        p.lo[a][b] = p.P[a][b];
        p.hi[a][b] = p.P[a][b];
      }
    }
  }
  p.xlo = edge && si.c.x == 0;
  p.xhi = edge && si.c.x == g.nx - 1;
  p.self = p.P[1][1];
  return p;
}

template <class L, bool COMPACT>
struct IndexOf {
  using type = DenseIndex;
};
template <class L>
struct IndexOf<L, true> {
  using type = CompactIndex<L>;
};

template <class L, bool COMPACT>
__device__ __forceinline__ typename IndexOf<L, COMPACT>::type make_index(const GridGeom& g, const LinkView& lk,
                                                                         const SegInfo& si) {
  if constexpr (COMPACT) return compact_index<L>(g, lk, si);
  else return dense_index(g, si.c);
}

// Dense-layout storage index of x - c for run-time c (slot mode only).
__device__ __forceinline__ uint32_t src_index_dyn(const GridGeom& g, Coords c, int cx, int cy, int cz) {
  const int o = g.outlet;
  const int sx = axis_src(c.x, cx, g.nx, g.perx, o == 0, o == 1);
  const int sy = axis_src(c.y, cy, g.ny, g.pery, o == 2, o == 3);
  const int sz = axis_src(c.z, cz, g.nz, g.perz, o == 4, o == 5);
  return (uint32_t)(sx + g.px) + (uint32_t)g.NX * ((uint32_t)(sy + g.py) + (uint32_t)g.NY * (uint32_t)(sz + g.pz));
}

// A wave-uniform 64-bit value, pinned to scalar registers: an address formed
// as base + (this) + 32-bit lane offset then keeps its base in scalar registers
// instead of being folded into per-lane 64-bit arithmetic.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Integer mixing function ("lowbias32", C. Wellons' hash prospector, 2018):
// xorshift-multiply rounds with full avalanche; the random words of the
// stochastic rounding are this function of a slot index and the step count.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// A wave-uniform byte address (scalar registers) as a pointer into global
// memory: the accesses through it stay global memory instructions.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> global_at(uint64_t v) {
  return reinterpret_cast<gptr<T>>(v);
}

// Wave-local visibility of LDS writes made by other lanes of the same wave.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Replace the pulled values of the cut directions of the wave's boundary nodes
// by their link values (list mode).  Boundary lanes leave their patched
// populations in stage[0..Q-1][tid].  The first `npre` links of each lane come
// prefetched in (ldp, vp); the rest are read here.
template <class L, typename R, int NPRE>
__device__ __forceinline__ void patch_links(R (&h)[L::Q], R (*stage)[BLOCK], bool bnd, int tid, int wbase, int lb0,
                                            int lb1, int lane, const uint16_t* lld, const R* lv, const int (&ldp)[2],
                                            const R (&vp)[2]) {
  if (bnd) {
#pragma unroll
    for (int i = 0; i < L::Q; ++i) stage[i][tid] = h[i];
  }
  wave_lds_sync();
#pragma unroll
  for (int j = 0; j < NPRE; ++j) {
    const int k = lb0 + lane + j * SEG;
    if (k < lb1) stage[ldp[j] >> 8][wbase + (ldp[j] & (SEG - 1))] = vp[j];
  }
  for (int k = lb0 + lane + NPRE * SEG; k < lb1; k += SEG) {
    const int ld = lld[k];
    stage[ld >> 8][wbase + (ld & (SEG - 1))] = lv[k];
  }
  wave_lds_sync();
  if (bnd) {
#pragma unroll
    for (int i = 0; i < L::Q; ++i) h[i] = stage[i][tid];
  }
}

// ---------------------------------------------------------------------------
// Fused step.
//  1. every fluid lane pulls its Q shifted populations (h_i = f_i - w_i);
//     boundary lanes patch their cut directions from the link values (list mode);
//  2. moments, BGK (+ Guo), store the Q post-collision values at the node
//     (solid lanes of a non-empty segment store zeros in list mode so that
//     every touched cache line is written whole);
//  3. the wave rebuilds its cut links one per lane (eq. ELIBB-general with the
//     closed-form weights) from the staged data of its boundary nodes and
//     writes them to lv_out (list mode) or to the solid-side slot (slot mode);
// The zero-gradient outlet needs no work of its own: its pulls are clamped onto
// the face layer (see axis_src).
// ---------------------------------------------------------------------------
template <class L, int S, bool COMPACT, bool TRT, bool REG>
__device__ __forceinline__ void step_body(const StepParams& p, uint32_t block) {
  using St = Storage<S>;
  using T = typename St::T;
  using R = typename St::R;
  constexpr int NV = L::Q + 4;
  __shared__ R stage[NV][BLOCK];
  const GridGeom& g = p.g;
  const LinkView& lk = p.lk;
  // stochastic rounding: the domain's step count (this launch reads the
  // current parity's entry, block 0 advances the other one), hashed once
  uint32_t rstep = 0;
  if constexpr (St::stochastic) {
    const uint32_t t = load_const(p.rng_ctr + p.parity);
    if (block == 0 && threadIdx.x == 0) p.rng_ctr[1 - p.parity] = t + 1u;
    rstep = mix32(t ^ 0x5bd1e995u);
  }
  const SegInfo si = seg_info(g, block);
  if (si.seg >= g.nseg) return;
  const uint64_t fm = load_const(lk.seg_fluid + si.seg);
  if (fm == 0) return;
  const bool fluid = (fm >> si.lane) & 1ull;
  const bool inrow = si.c.x < g.nx;
  const Coords c = si.c;
  const T* __restrict__ src = static_cast<const T*>(p.src);
  T* __restrict__ dst = static_cast<T*>(p.dst);
  const size_t np = (size_t)g.npad;
  const int tid = threadIdx.x;
  const int wbase = tid & ~(SEG - 1);
  const bool list_mode = lk.lv_out != nullptr;

  // parameters: the doubles (FP64 kernels) or their FP32 roundings
  auto prm = [](double d, float f) -> R {
    if constexpr (sizeof(R) == 4) return f;
    else return R(d);
  };
  Collider<R, TRT> col;
  col.omega = prm(p.omega, p.omega_f);
  col.kf = R(1) - R(0.5) * col.omega;
  col.omega_m = prm(p.omega_minus, p.omega_minus_f);
  col.Fx = prm(p.force[0], p.force_f[0]);
  col.Fy = prm(p.force[1], p.force_f[1]);
  col.Fz = prm(p.force[2], p.force_f[2]);
  col.src_eq = prm(p.src_eq, p.src_eq_f);
  col.src_eq_m = prm(p.src_eq_minus, p.src_eq_minus_f);
  col.force = p.has_force != 0;

  // segments without boundary nodes have no links (and need not read seg_lbase)
  const uint64_t bmask = load_const(lk.seg_bnd + si.seg);
  int lb0 = 0, lb1 = 0;
  if (bmask) {
    lb0 = load_const(lk.seg_lbase + si.seg);
    lb1 = load_const(lk.seg_lbase + si.seg + 1);
  }
  const bool has_links = lb1 > lb0;
  const R* __restrict__ lq = static_cast<const R*>(lk.lq);
  const R* __restrict__ lg = static_cast<const R*>(lk.lg);
  const R* __restrict__ lvi = static_cast<const R*>(lk.lv_in);
  R* __restrict__ lvo = static_cast<R*>(lk.lv_out);
  const R* __restrict__ luv = static_cast<const R*>(lk.luv);
  // the first two links of each lane are fetched before the populations so that
  // their latency overlaps the pull
  int ldp[2] = {0, 0};
  R qp[2] = {R(1), R(1)}, gp[2] = {R(0), R(0)}, vp[2] = {R(0), R(0)};
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int k = lb0 + si.lane + j * SEG;
    if (k < lb1) {
      ldp[j] = lk.lld[k];
      qp[j] = lq[k];
      if (lg) gp[j] = lg[k];
      if (list_mode) vp[j] = lvi[k];
    }
  }

  const auto ix = make_index<L, COMPACT>(g, lk, si);
  // byte distance between direction arrays; the direction bases below are
  // advanced by it in scalar registers (a running sum, no multiplies)
  const uint64_t npb = (uint64_t)np * sizeof(T);
  // Every lane pulls, so that no branch and no zero fill are needed: in the
  // compact layout the slots formed for a lane that is not fluid (or lies past
  // the row's end) stay inside the population array (between the guard's last
  // slot and the last fluid slot + 1, which the array holds); in the dense
  // layout a solid lane reads its neighbours and a lane past the row's end
  // those of the row's last node.  Such lanes store nothing that is read (the
  // dense layout's list mode stores zeros from them).
  R h[L::Q];
  {
    uint64_t qb = uniform_u64(reinterpret_cast<uint64_t>(src));
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
      h[i] = St::template load<L>((const T*)(global_at<const T>(qb) + ix.template src<L>(i)), i);
      qb = uniform_u64(qb + npb);
    }
  }
  const bool bnd = fluid && ((bmask >> si.lane) & 1ull);
  if (has_links && list_mode) patch_links<L, R, 2>(h, stage, bnd, tid, wbase, lb0, lb1, si.lane, lk.lld, lvi, ldp, vp);

  Moments<R> m;
  m = moments<L, R>(h, col.Fx, col.Fy, col.Fz);
  // boundary nodes leave their moments (and, in slot mode, their pre-collision
  // populations) for the link phase
  if (bnd) {
    if (!list_mode) {
#pragma unroll
      for (int i = 0; i < L::Q; ++i) stage[i][tid] = h[i];
    }
    stage[L::Q + 0][tid] = m.drho;
    stage[L::Q + 1][tid] = m.ux;
    stage[L::Q + 2][tid] = m.uy;
    stage[L::Q + 3][tid] = m.uz;
  }
  // dense layout, list mode: solid lanes of a non-empty segment store zeros so
  // that the shared cache lines are written whole (nothing reads those slots);
  // the compact layout has no solid slots
  if (fluid || (!COMPACT && list_mode && inrow)) {
    // (every storing lane is fluid in the compact layout)
    const bool keep = COMPACT || fluid;
    // the slots of the storing lanes grow with the lane, so every address is
    // a wave-uniform base (scalar registers) plus a small 32-bit lane offset;
    // each pair is stored as soon as it is computed, so that the stores drain
    // while the rest of the collision runs
    const uint32_t self0 = __builtin_amdgcn_readfirstlane(ix.self);
    const uint32_t off = (ix.self - self0) * (uint32_t)sizeof(T);
    auto at = [&](int i) {
      return reinterpret_cast<T*>(reinterpret_cast<char*>(dst + uniform_u64(i * np + self0)) + off);
    };
    // stochastic rounding: one random word per node and step, offset per direction
    const uint32_t rnode = St::stochastic ? mix32(ix.self * 0x9e3779b1u + rstep) : 0u;
    auto put = [&](int i, R v) { store_rounded<S, L>(at(i), keep ? v : R(0), i, rnode + (uint32_t)i * 0x9e3779b9u); };
    const Pairs<R> pr(col, m);
    put(0, pr.rest(h[0], R(L::w(0))));
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
      if (i > L::opp(i)) continue;
      R v, vb;
      pr.template pair<L, TRT>(i, h[i], h[L::opp(i)], m, col, v, vb);
      put(i, v);
      put(L::opp(i), vb);
    }
  }

  if (has_links) {
    wave_lds_sync();
    const int xseg = c.x - si.lane;
    const R qc = prm(p.q_cut, p.q_cut_f);
    auto rebuild = [&](int k, int ld, R q, R gw) {
      const int nl = ld & (SEG - 1);
      const int i = ld >> 8;
      const int ib = dyn_opp<L>(i);
      const int t = wbase + nl;
      Moments<R> mb;
      mb.drho = stage[L::Q + 0][t];
      mb.rho = R(1) + mb.drho;
      mb.ux = stage[L::Q + 1][t];
      mb.uy = stage[L::Q + 2][t];
      mb.uz = stage[L::Q + 3][t];
      mb.uu = dot_uu(mb.ux, mb.uy, mb.uz);
      const R hb = stage[ib][t];
      const R hi = stage[i][t];
      const int icx = dyn_c<L, 0>(i), icy = dyn_c<L, 1>(i), icz = dyn_c<L, 2>(i);
      const R cx = R(icx), cy = R(icy), cz = R(icz);
      const R w = dyn_w<L, R>(i);
      const Coef<R> a = elibb_coefficients_fast<R>(p.variant, q, qc);
      // bounced direction: c_ibar = -c_i, w_ibar = w_i
      const R he_b = col.heq(-cx, -cy, -cz, w, mb);
      // post-collision values of ibar and i at node F, with the arithmetic of the
      // node's own update (Pairs) on the pair's member with the smaller index
      R hs_b, hs_i;
      {
        const Pairs<R> pr(col, mb);
        const bool low = i < ib;
        const R s = low ? R(1) : R(-1);
        const R cul = s * (cx * mb.ux + cy * mb.uy + cz * mb.uz);
        const R cFl = s * (cx * col.Fx + cy * col.Fy + cz * col.Fz);
        R e, o;
        pr.eo(w, cul, cFl, e, o);
        if constexpr (TRT) {
          R vl, vu;
          pr.values_trt(low ? hi : hb, low ? hb : hi, e, o, vl, vu);
          hs_i = low ? vl : vu;
          hs_b = low ? vu : vl;
        } else {
          hs_b = pr.value(hb, e, o, !low);
          hs_i = pr.value(hi, e, o, low);
        }
      }
      R n_pre, n_post;
      if constexpr (REG) {
        // regularised wall non-equilibrium (eq. fi_neq): the stress of node F at
        // t before and after collision, with u_w(t+1) and u_w(t) respectively
        const Stress<R> sp = neq_stress<L, R>(stage, t, mb);
        const Stress<R> sq = post_stress<L, R, TRT>(sp, col, mb);
        R u[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
        if (luv) {
#pragma unroll
          for (int a = 0; a < 6; ++a) u[a] = luv[k + a * lk.luv_stride];
        }
        n_pre = regularized_neq(cx, cy, cz, w, sp, u[3], u[4], u[5]);
        n_post = regularized_neq(cx, cy, cz, w, sq, u[0], u[1], u[2]);
      } else {
        n_pre = hb - he_b;               // bounced pre-collision non-equilibrium (eq. neqbb-s)
        n_post = hs_b - he_b;            // bounced post-collision non-equilibrium
      }
      R v = a.a4 * n_pre + a.a5 * n_post + a.a2 * hs_b + w * (mb.drho * (a.a4 + a.a5) + mb.rho * gw);
      v += a.a3 * hs_i;
      if (list_mode) {
        lvo[k] = v;
      } else {
        Coords cf = c;
        cf.x = xseg + nl;
        const uint32_t at = src_index_dyn(g, cf, icx, icy, icz);
        store_rounded<S, L>(dst + (size_t)i * np + at, v, i,
                            St::stochastic ? mix32((at + (uint32_t)i * (uint32_t)np) * 0x9e3779b1u + rstep) : 0u);
      }
    };
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int k = lb0 + si.lane + j * SEG;
      if (k < lb1) rebuild(k, ldp[j], qp[j], gp[j]);
    }
    for (int k = lb0 + si.lane + 2 * SEG; k < lb1; k += SEG) rebuild(k, lk.lld[k], lq[k], lg ? lg[k] : R(0));
  }
}

// Six waves per SIMD is what the LDS stage allows for the 32- and 16-bit forms
// (23.5 KB per workgroup); asking for it keeps the register allocator at or
// below 80 VGPRs (no spills), where left alone it takes 83 for the FP32
// compact kernels and drops them to five.
constexpr int step_waves_per_eu(int S) { return S == ST_F64 ? 1 : 6; }

template <class L, int S, bool COMPACT, bool TRT, bool REG>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(step_waves_per_eu(S)))) void step_kernel(
    StepParams p) {
  step_body<L, S, COMPACT, TRT, REG>(p, logical_block(p.g.xcd_remap));
}

// Several domains in one persistent launch.  Slot k of the tile table names a
// block of one domain (domain << TILE_SHIFT | block) or is empty; workgroup b
// walks the slots b, b + gridDim.x, ...  The host orders the table (see
// tile_table), so the grid size and the order are launch choices that leave
// every result unchanged.
// Entry of the step table with its pointers read through the constant address
// space (the host writes the table before the launch), so that the arrays they
// name are addressed with global memory instructions.
__device__ __forceinline__ StepParams table_entry(const StepParams* e) {
  StepParams p = *e;
  p.src = load_const(&e->src);
  p.dst = load_const(&e->dst);
  const LinkView* k = &e->lk;
  p.lk.seg_fluid = load_const(&k->seg_fluid);
  p.lk.seg_fbase = load_const(&k->seg_fbase);
  p.lk.row_src = load_const(&k->row_src);
  p.lk.seg_bnd = load_const(&k->seg_bnd);
  p.lk.seg_lbase = load_const(&k->seg_lbase);
  p.lk.lld = load_const(&k->lld);
  p.lk.lnode = load_const(&k->lnode);
  p.lk.lq = load_const(&k->lq);
  p.lk.lg = load_const(&k->lg);
  p.lk.lv_in = load_const(&k->lv_in);
  p.lk.lv_out = load_const(&k->lv_out);
  p.lk.luv = load_const(&k->luv);
  return p;
}

template <class L, int S, bool COMPACT, bool TRT, bool REG>
__global__ __launch_bounds__(BLOCK) void step_batch_kernel(const StepParams* __restrict__ tab,
                                                           const uint32_t* __restrict__ tiles, uint32_t nslots) {
  for (uint32_t k = blockIdx.x; k < nslots; k += gridDim.x) {
    const uint32_t t = __builtin_amdgcn_readfirstlane(tiles[k]);
    if (t != TILE_EMPTY) {
      const StepParams p = table_entry(tab + (t >> TILE_SHIFT));
      step_body<L, S, COMPACT, TRT, REG>(p, t & TILE_MASK);
    }
    wave_lds_sync();   // the next tile reuses the wave's LDS columns
  }
}

// Pre-collision shifted populations of one lane's node (pull + link patch).
// Every lane of the wave must call it (the patch is a wave-level exchange).
template <class L, int S, bool COMPACT>
__device__ __forceinline__ void gather_state(const GridGeom& g, const LinkView& lk, const void* srcv, const SegInfo& si,
                                             bool fluid, typename Storage<S>::R (&h)[L::Q],
                                             typename Storage<S>::R (*stage)[BLOCK]) {
  using St = Storage<S>;
  using T = typename St::T;
  using R = typename St::R;
  const T* src = static_cast<const T*>(srcv);
  const auto ix = make_index<L, COMPACT>(g, lk, si);
#pragma unroll
  for (int i = 0; i < L::Q; ++i) h[i] = R(0);
  if (fluid) {
#pragma unroll
    for (int i = 0; i < L::Q; ++i) h[i] = St::template load<L>(src + i * (size_t)g.npad + ix.template src<L>(i), i);
  }
  if (lk.lv_in) {
    const int lb0 = lk.seg_lbase[si.seg], lb1 = lk.seg_lbase[si.seg + 1];
    if (lb1 > lb0) {
      const bool bnd = fluid && ((lk.seg_bnd[si.seg] >> si.lane) & 1ull);
      const int ldp[2] = {0, 0};
      const R vp[2] = {R(0), R(0)};
      patch_links<L, R, 0>(h, stage, bnd, threadIdx.x, threadIdx.x & ~(SEG - 1), lb0, lb1, si.lane, lk.lld,
                           static_cast<const R*>(lk.lv_in), ldp, vp);
    }
  }
}

// ---------------------------------------------------------------------------
// Initialisation / import: write the pre-collision state into the pull slots
// (and, in list mode, the cut-link values with init_links_kernel).
// ---------------------------------------------------------------------------
template <class L>
__device__ __forceinline__ double init_value(const InitParams& p, int64_t n, int i) {
  if (p.f_in) return p.f_in[i * ((int64_t)p.g.nx * p.g.ny * p.g.nz) + n] - L::w(i);
  const double ux = p.u0[0], uy = p.u0[1], uz = p.u0[2];
  const double uu = ux * ux + uy * uy + uz * uz;
  const double cu = L::cx(i) * ux + L::cy(i) * uy + L::cz(i) * uz;
  return L::w(i) * ((p.rho0 - 1.0) + p.rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
}

template <class L, int S, bool COMPACT>
__global__ __launch_bounds__(BLOCK) void init_kernel(InitParams p) {
  using St = Storage<S>;
  using T = typename St::T;
  using R = typename St::R;
  const GridGeom& g = p.g;
  const LinkView& lk = p.lk;
  const SegInfo si = seg_info(g);
  if (si.seg >= g.nseg) return;
  const uint64_t fm = lk.seg_fluid[si.seg];
  // directions of this lane that are cut links (list mode): their slot is not
  // the node's to write (the value lives in the link arrays)
  uint32_t cut = 0u;
  if (lk.lv_out) {
    const int lb0 = lk.seg_lbase[si.seg], lb1 = lk.seg_lbase[si.seg + 1];
    for (int k = lb0; k < lb1; ++k) {
      const int ld = lk.lld[k];
      if ((ld & (SEG - 1)) == si.lane) cut |= 1u << (ld >> 8);
    }
  }
  const auto ix = make_index<L, COMPACT>(g, lk, si);
  if (!((fm >> si.lane) & 1ull)) return;
  const Coords c = si.c;
  T* dst = static_cast<T*>(p.dst);
  const int64_t n = c.x + (int64_t)g.nx * (c.y + (int64_t)g.ny * c.z);
  // outlet layer: an inward population shares its (clamped) source slot with the
  // upstream neighbour one layer in; that neighbour writes it if it is fluid
  bool skip_out = false;
  int oa = -1, osg = 0;
  if (g.outlet >= 0) {
    oa = g.outlet >> 1;
    osg = (g.outlet & 1) ? 1 : -1;
    const int coord = oa == 0 ? c.x : (oa == 1 ? c.y : c.z);
    const int na = oa == 0 ? g.nx : (oa == 1 ? g.ny : g.nz);
    if (coord == (osg > 0 ? na - 1 : 0) && na > 1) {
      Coords q = c;
      if (oa == 0) q.x -= osg;
      else if (oa == 1) q.y -= osg;
      else q.z -= osg;
      const uint32_t wq = (uint32_t)(q.x / SEG) + (uint32_t)g.nseg_x * ((uint32_t)q.y + (uint32_t)g.ny * (uint32_t)q.z);
      skip_out = (lk.seg_fluid[wq] >> (q.x % SEG)) & 1ull;
    } else {
      oa = -1;
    }
  }
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    if ((cut >> i) & 1u) continue;
    if (oa >= 0 && skip_out) {
      const int ca = oa == 0 ? L::cx(i) : (oa == 1 ? L::cy(i) : L::cz(i));
      if (ca == -osg) continue;
    }
    St::template store<L>(dst + i * (size_t)g.npad + ix.template src<L>(i), R(init_value<L>(p, n, i)), i);
  }
}

template <class L, int S>
__global__ __launch_bounds__(BLOCK) void init_links_kernel(InitParams p) {
  using R = typename Storage<S>::R;
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (k >= p.nlinks) return;
  const int i = p.lk.lld[k] >> 8;
  const int64_t n = p.lk.lnode[k];
  double v = 0.0;
#pragma unroll
  for (int j = 1; j < L::Q; ++j)
    if (j == i) v = init_value<L>(p, n, j);
  static_cast<R*>(p.lk.lv_out)[k] = R(v);
}

// ---------------------------------------------------------------------------
// Export of the pre-collision state f_i(x, t) to [Q][N] float64.
// ---------------------------------------------------------------------------
template <class L, int S, bool COMPACT>
__global__ __launch_bounds__(BLOCK) void export_kernel(ExportParams p) {
  using R = typename Storage<S>::R;
  __shared__ R stage[L::Q][BLOCK];
  const GridGeom& g = p.g;
  const SegInfo si = seg_info(g);
  if (si.seg >= g.nseg) return;
  const bool in = si.c.x < g.nx;
  const bool fluid = in && ((p.lk.seg_fluid[si.seg] >> si.lane) & 1ull);
  R h[L::Q];
  gather_state<L, S, COMPACT>(g, p.lk, p.src, si, fluid, h, stage);
  if (!in) return;
  const Coords c = si.c;
  const int64_t n = c.x + (int64_t)g.nx * (c.y + (int64_t)g.ny * c.z);
  const int64_t N = (int64_t)g.nx * g.ny * g.nz;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) p.f_out[i * N + n] = fluid ? double(h[i]) + L::w(i) : 0.0;
}

// ---------------------------------------------------------------------------
// FP64 moments and fixed-order block partial sums.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_sum_fixed(double (*sh)[BLOCK], double* v, int tid) {
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NPART; ++k) sh[k][tid] = v[k];
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if (tid < s) {
#pragma unroll
      for (int k = 0; k < NPART; ++k) sh[k][tid] += sh[k][tid + s];
    }
    __syncthreads();
  }
}

// Moments of every node and block partial sums of mass, momentum and (with a
// previous field) the residual.  Workgroup b walks the logical blocks b,
// b + gridDim.x, ... (one each when the grid covers the lattice), so the
// partials have one row per workgroup.
template <class L, int S, bool COMPACT>
__global__ __launch_bounds__(BLOCK) void macros_kernel(MacroParams p) {
  using R = typename Storage<S>::R;
  __shared__ double sh[NPART][BLOCK];
  __shared__ R stage[L::Q][BLOCK];
  const GridGeom& g = p.g;
  double v[NPART] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t b = blockIdx.x; b < p.nblocks; b += gridDim.x) {
    const SegInfo si = seg_info(g, (uint32_t)b);
    const bool seg_ok = si.seg < g.nseg;
    const bool in = seg_ok && si.c.x < g.nx;
    const bool fluid = in && ((p.lk.seg_fluid[si.seg] >> si.lane) & 1ull);
    R h[L::Q];
    if (seg_ok) gather_state<L, S, COMPACT>(g, p.lk, p.src, si, fluid, h, stage);
    if (in) {
      const Coords c = si.c;
      const int64_t n = c.x + (int64_t)g.nx * (c.y + (int64_t)g.ny * c.z);
      double rho = 0.0, ux = 0.0, uy = 0.0, uz = 0.0;
      if (fluid) {
        double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
          const double hi = double(h[i]);
          drho += hi;
          jx += L::cx(i) * hi;
          jy += L::cy(i) * hi;
          jz += L::cz(i) * hi;
        }
        rho = 1.0 + drho;
        ux = (jx + 0.5 * p.force[0]) / rho;
        uy = (jy + 0.5 * p.force[1]) / rho;
        uz = (jz + 0.5 * p.force[2]) / rho;
        v[0] += rho;
        v[1] += rho * ux;
        v[2] += rho * uy;
        v[3] += rho * uz;
        v[5] += ux * ux + uy * uy + (L::D == 3 ? uz * uz : 0.0);
        v[6] += (isfinite(rho) && isfinite(ux) && isfinite(uy) && isfinite(uz)) ? 0.0 : 1.0;
        if (p.uprev) {
          double* up = p.uprev + n * L::D;
          const double dx = ux - up[0], dy = uy - up[1], dz = L::D == 3 ? uz - up[2] : 0.0;
          v[4] += dx * dx + dy * dy + dz * dz;
          up[0] = ux;
          up[1] = uy;
          if (L::D == 3) up[2] = uz;
        }
      }
      if (p.rho) p.rho[n] = rho;
      if (p.u) {
        p.u[n * L::D + 0] = ux;
        p.u[n * L::D + 1] = uy;
        if (L::D == 3) p.u[n * L::D + 2] = uz;
      }
    }
    wave_lds_sync();   // the next block reuses the wave's LDS columns
  }
  block_sum_fixed(sh, v, threadIdx.x);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NPART; ++k) p.partials[blockIdx.x * NPART + k] = sh[k][0];
  }
}

#ifdef LBM_COMMON
__global__ __launch_bounds__(BLOCK) void reduce_kernel(const double* partials, int64_t nblocks, double* out) {
  __shared__ double sh[NPART][BLOCK];
  double v[NPART] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t b = threadIdx.x; b < nblocks; b += BLOCK) {
#pragma unroll
    for (int k = 0; k < NPART; ++k) v[k] += partials[b * NPART + k];
  }
  block_sum_fixed(sh, v, threadIdx.x);
  if (threadIdx.x < NPART) out[threadIdx.x] = sh[threadIdx.x][0];
}
#endif  // LBM_COMMON

// ---------------------------------------------------------------------------
// Momentum-exchange force and torque of the last step (Sec. II "Force
// computation", Galilean-invariant form): per cut link (x_F, i)
//   F = (c_ibar - u_w) f*_ibar(x_F, t-1) - (c_i - u_w) f_i(x_F, t),
//   T = r x F,  r = x_W - x_ref (minimum image), x_W = x_F - q c_i the wall point,
// with f*_ibar(x_F, t-1) the post-collision value the step left in x_F's own
// slot of direction ibar (no node pulls it: x_F - c_i is not fluid), and
// f_i(x_F, t) the link value it rebuilt.
// ---------------------------------------------------------------------------
template <class L, int S, bool COMPACT>
__global__ __launch_bounds__(BLOCK) void force_kernel(ForceParams p) {
  using St = Storage<S>;
  using T = typename St::T;
  using R = typename St::R;
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (k >= p.nl) return;
  const GridGeom& g = p.g;
  const int ld = p.lk.lld[k];
  const int i = ld >> 8;
  const int ib = dyn_opp<L>(i);
  const int64_t node = p.lk.lnode[k];
  const int64_t row = node / g.nx;
  const int x = (int)(node - row * g.nx);
  const int64_t y = row % g.ny, z = row / g.ny;
  int64_t slot;
  if constexpr (COMPACT) {
    const int64_t seg = row * g.nseg_x + x / SEG;
    const uint64_t below = p.lk.seg_fluid[seg] & ((1ull << (x % SEG)) - 1ull);
    slot = g.guard + (int64_t)p.lk.seg_fbase[seg] + __popcll(below);
  } else {
    slot = (x + g.px) + (int64_t)g.NX * ((y + g.py) + (int64_t)g.NY * (z + g.pz));
  }
  const double w = dyn_w<L, double>(i);
  const double fs = (double)St::template load<L>(static_cast<const T*>(p.pop) + (size_t)ib * g.npad + slot, ib) + w;
  const double fn = (double)static_cast<const R*>(p.lk.lv_in)[k] + w;
  const double c[3] = {(double)dyn_c<L, 0>(i), (double)dyn_c<L, 1>(i), (double)dyn_c<L, 2>(i)};
  double F[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double u = p.luw ? p.luw[3 * k + a] : 0.0;
    F[a] = (-c[a] - u) * fs - (c[a] - u) * fn;
  }
  // lever arm from the group's reference point to the wall point
  const double q = (double)static_cast<const R*>(p.lk.lq)[k];
  const int grp = p.group ? p.group[k] : 0;
  const double xw[3] = {x - q * c[0], (double)y - q * c[1], (double)z - q * c[2]};
  const int n3[3] = {g.nx, g.ny, g.nz}, per[3] = {g.perx, g.pery, g.perz};
  double r[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r[a] = xw[a] - (p.centre ? p.centre[3 * grp + a] : 0.0);
    if (per[a]) r[a] -= n3[a] * rint(r[a] / n3[a]);
  }
  if (L::D == 2) r[2] = 0.0;
  double* o = p.contrib + 6 * k;
  o[0] = F[0];
  o[1] = F[1];
  o[2] = F[2];
  o[3] = r[1] * F[2] - r[2] * F[1];
  o[4] = r[2] * F[0] - r[0] * F[2];
  o[5] = r[0] * F[1] - r[1] * F[0];
}

// Sum of the contributions (6 per link: force, torque) of the links of group
// blockIdx.x (all links when group is null), in a fixed order.  The link count
// is nl, or *nl_dev when that is given (counts held on the device).
#ifdef LBM_COMMON
__global__ __launch_bounds__(BLOCK) void group_sum_kernel(const double* contrib, const int32_t* group, int64_t nl,
                                                          const int32_t* nl_dev, double* out) {
  __shared__ double sh[NPART][BLOCK];
  double v[NPART] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int gid = blockIdx.x;
  const int64_t n = nl_dev ? (int64_t)*nl_dev : nl;
  for (int64_t k = threadIdx.x; k < n; k += BLOCK) {
    if (group && group[k] != gid) continue;
#pragma unroll
    for (int a = 0; a < 6; ++a) v[a] += contrib[6 * k + a];
  }
  block_sum_fixed(sh, v, threadIdx.x);
  if (threadIdx.x < 6) out[6 * gid + threadIdx.x] = sh[threadIdx.x][0];
}
#endif  // LBM_COMMON

// ---------------------------------------------------------------------------
// Launchers.  This file is compiled once per lattice (LBM_LATTICE names it);
// Launch<LBM_LATTICE> is instantiated here.  The build defining LBM_COMMON
// also holds the lattice-independent kernels and the lattice dispatch.
// ---------------------------------------------------------------------------
#define LBM_DISPATCH_L(KERNEL, LAT, storage, C, grid, stream, ...)                                             \
  do {                                                                                                         \
    switch (storage) {                                                                                         \
      case ST_F64: KERNEL<LAT, ST_F64, C><<<grid, BLOCK, 0, stream>>>(__VA_ARGS__); break;                     \
      case ST_F32: KERNEL<LAT, ST_F32, C><<<grid, BLOCK, 0, stream>>>(__VA_ARGS__); break;                     \
      case ST_F16S: KERNEL<LAT, ST_F16S, C><<<grid, BLOCK, 0, stream>>>(__VA_ARGS__); break;                   \
      default: KERNEL<LAT, ST_BF16S, C><<<grid, BLOCK, 0, stream>>>(__VA_ARGS__); break;                       \
    }                                                                                                          \
  } while (0)

// storage x layout
#define LBM_DISPATCH_SC(KERNEL, LAT, storage, compact, grid, stream, ...)                                      \
  do {                                                                                                         \
    if (compact) LBM_DISPATCH_L(KERNEL, LAT, storage, true, grid, stream, __VA_ARGS__);                        \
    else LBM_DISPATCH_L(KERNEL, LAT, storage, false, grid, stream, __VA_ARGS__);                               \
  } while (0)

// step kernels: storage x layout x collision x wall non-equilibrium estimator
#define LBM_STEP_L(KERNEL, LAT, storage, C, T, G, grid, stream, ...)                                           \
  do {                                                                                                         \
    switch (storage) {                                                                                         \
      case ST_F64: KERNEL<LAT, ST_F64, C, T, G><<<grid, BLOCK, 0, stream>>>(__VA_ARGS__); break;               \
      case ST_F32: KERNEL<LAT, ST_F32, C, T, G><<<grid, BLOCK, 0, stream>>>(__VA_ARGS__); break;               \
      case ST_F16S: KERNEL<LAT, ST_F16S, C, T, G><<<grid, BLOCK, 0, stream>>>(__VA_ARGS__); break;             \
      case ST_F16SR: KERNEL<LAT, ST_F16SR, C, T, G><<<grid, BLOCK, 0, stream>>>(__VA_ARGS__); break;           \
      case ST_BF16SR: KERNEL<LAT, ST_BF16SR, C, T, G><<<grid, BLOCK, 0, stream>>>(__VA_ARGS__); break;         \
      default: KERNEL<LAT, ST_BF16S, C, T, G><<<grid, BLOCK, 0, stream>>>(__VA_ARGS__); break;                 \
    }                                                                                                          \
  } while (0)

#define LBM_STEP_TG(KERNEL, LAT, storage, C, trt, reg, grid, stream, ...)                                      \
  do {                                                                                                         \
    if (trt) {                                                                                                 \
      if (reg) LBM_STEP_L(KERNEL, LAT, storage, C, true, true, grid, stream, __VA_ARGS__);                     \
      else LBM_STEP_L(KERNEL, LAT, storage, C, true, false, grid, stream, __VA_ARGS__);                        \
    } else {                                                                                                   \
      if (reg) LBM_STEP_L(KERNEL, LAT, storage, C, false, true, grid, stream, __VA_ARGS__);                    \
      else LBM_STEP_L(KERNEL, LAT, storage, C, false, false, grid, stream, __VA_ARGS__);                       \
    }                                                                                                          \
  } while (0)

#define LBM_STEP_SCT(KERNEL, LAT, storage, compact, trt, reg, grid, stream, ...)                               \
  do {                                                                                                         \
    if (compact) LBM_STEP_TG(KERNEL, LAT, storage, true, trt, reg, grid, stream, __VA_ARGS__);                 \
    else LBM_STEP_TG(KERNEL, LAT, storage, false, trt, reg, grid, stream, __VA_ARGS__);                        \
  } while (0)

template <class L>
hipError_t Launch<L>::step(int storage, const StepParams& p, hipStream_t s) {
  const dim3 grid((unsigned)grid_blocks(p.g));
  LBM_STEP_SCT(step_kernel, L, storage, p.g.compact, p.trt, p.wall_neq != 0, grid, s, p);
  return hipGetLastError();
}

template <class L>
hipError_t Launch<L>::step_batch(int storage, bool compact, bool trt, bool reg, const StepParams* tab,
                                 const uint32_t* tiles, uint32_t nslots, uint32_t grid, hipStream_t s) {
  LBM_STEP_SCT(step_batch_kernel, L, storage, compact, trt, reg, dim3(grid), s, tab, tiles, nslots);
  return hipGetLastError();
}

template <class L>
hipError_t Launch<L>::init(int storage, const InitParams& p, hipStream_t s) {
  LBM_DISPATCH_SC(init_kernel, L, storage, p.g.compact, dim3((unsigned)grid_blocks(p.g)), s, p);
  return hipGetLastError();
}

template <class L>
hipError_t Launch<L>::init_links(int storage, const InitParams& p, hipStream_t s) {
  const dim3 grid((unsigned)((p.nlinks + BLOCK - 1) / BLOCK));
  switch (storage) {
    case ST_F64: init_links_kernel<L, ST_F64><<<grid, BLOCK, 0, s>>>(p); break;
    case ST_F32: init_links_kernel<L, ST_F32><<<grid, BLOCK, 0, s>>>(p); break;
    case ST_F16S: init_links_kernel<L, ST_F16S><<<grid, BLOCK, 0, s>>>(p); break;
    default: init_links_kernel<L, ST_BF16S><<<grid, BLOCK, 0, s>>>(p); break;
  }
  return hipGetLastError();
}

template <class L>
hipError_t Launch<L>::export_state(int storage, const ExportParams& p, hipStream_t s) {
  LBM_DISPATCH_SC(export_kernel, L, storage, p.g.compact, dim3((unsigned)grid_blocks(p.g)), s, p);
  return hipGetLastError();
}

template <class L>
hipError_t Launch<L>::macros(int storage, const MacroParams& p, int64_t nblocks, hipStream_t s) {
  LBM_DISPATCH_SC(macros_kernel, L, storage, p.g.compact, dim3((unsigned)nblocks), s, p);
  return hipGetLastError();
}

template <class L>
hipError_t Launch<L>::force(int storage, const ForceParams& p, hipStream_t s) {
  const dim3 grid((unsigned)((p.nl + BLOCK - 1) / BLOCK));
  LBM_DISPATCH_SC(force_kernel, L, storage, p.g.compact, grid, s, p);
  return hipGetLastError();
}

template struct Launch<LBM_LATTICE>;

#ifdef LBM_COMMON
int64_t grid_blocks(const GridGeom& g) {
  const int64_t b = (g.nseg + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
  return (b + 7) / 8 * 8;   // multiple of the XCD count, see logical_block()
}

#define LBM_BY_LATTICE(lattice, CALL)                \
  switch (lattice) {                                 \
    case LBM_D2Q9: return Launch<D2Q9>::CALL;        \
    case LBM_D3Q19: return Launch<D3Q19>::CALL;      \
    default: return Launch<D3Q27>::CALL;             \
  }

hipError_t launch_step(int lattice, int storage, const StepParams& p, hipStream_t s) {
  LBM_BY_LATTICE(lattice, step(storage, p, s));
}

hipError_t launch_step_batch(int lattice, int storage, bool compact, bool trt, bool reg, const StepParams* tab,
                             const uint32_t* tiles, uint32_t nslots, uint32_t grid, hipStream_t s) {
  if (nslots == 0 || grid == 0) return hipSuccess;
  LBM_BY_LATTICE(lattice, step_batch(storage, compact, trt, reg, tab, tiles, nslots, grid, s));
}

hipError_t launch_init(int lattice, int storage, const InitParams& p, hipStream_t s) {
  LBM_BY_LATTICE(lattice, init(storage, p, s));
}

hipError_t launch_init_links(int lattice, int storage, const InitParams& p, hipStream_t s) {
  if (p.nlinks == 0 || p.lk.lv_out == nullptr) return hipSuccess;
  LBM_BY_LATTICE(lattice, init_links(storage, p, s));
}

hipError_t launch_export(int lattice, int storage, const ExportParams& p, hipStream_t s) {
  LBM_BY_LATTICE(lattice, export_state(storage, p, s));
}

hipError_t launch_macros(int lattice, int storage, const MacroParams& p, int64_t nblocks, hipStream_t s) {
  LBM_BY_LATTICE(lattice, macros(storage, p, nblocks, s));
}

hipError_t launch_force(int lattice, int storage, const ForceParams& p, int32_t n_groups, double* out, hipStream_t s) {
  if (p.nl > 0) {
    hipError_t e;
    switch (lattice) {
      case LBM_D2Q9: e = Launch<D2Q9>::force(storage, p, s); break;
      case LBM_D3Q19: e = Launch<D3Q19>::force(storage, p, s); break;
      default: e = Launch<D3Q27>::force(storage, p, s); break;
    }
    if (e != hipSuccess) return e;
  }
  group_sum_kernel<<<n_groups, BLOCK, 0, s>>>(p.contrib, p.group, p.nl, nullptr, out);
  return hipGetLastError();
}

hipError_t launch_group_sum(const double* contrib, const int32_t* group, int64_t nl, const int32_t* nl_dev,
                            int32_t n_groups, double* out, hipStream_t s) {
  group_sum_kernel<<<n_groups, BLOCK, 0, s>>>(contrib, group, nl, nl_dev, out);
  return hipGetLastError();
}

// Bandwidth calibration: `arrays` FP32 arrays of n elements (stride elements
// apart) copied from src to dst, one element of every array per lane, so a
// 64-lane wave reads and writes 64 consecutive elements of each array -- the
// step kernel's access pattern without its pulls and arithmetic.  Element e
// sits at shift + e: shift 0 puts every wave's run on 256 B boundaries, any
// other shift makes every run straddle one (the compact layout's runs start
// at arbitrary slots).
// With the array count known at compile time (the lattices' 9, 19 and 27) a
// lane issues all its loads before its first store, as the step kernel does.
template <int A>
__global__ __launch_bounds__(BLOCK) void stream_probe_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                             int64_t n, int64_t stride, int32_t arrays,
                                                             int32_t shift) {
  const int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (e >= n) return;
  if constexpr (A > 0) {
    float v[A];
#pragma unroll
    for (int a = 0; a < A; ++a) v[a] = src[a * stride + shift + e];
#pragma unroll
    for (int a = 0; a < A; ++a) dst[a * stride + shift + e] = v[a];
  } else {
    for (int a = 0; a < arrays; ++a) dst[a * stride + shift + e] = src[a * stride + shift + e];
  }
}

hipError_t launch_stream_probe(const float* src, float* dst, int64_t n, int64_t stride, int32_t arrays,
                               int32_t shift, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + BLOCK - 1) / BLOCK);
  switch (arrays) {
    case 9: stream_probe_kernel<9><<<grid, BLOCK, 0, s>>>(src, dst, n, stride, arrays, shift); break;
    case 19: stream_probe_kernel<19><<<grid, BLOCK, 0, s>>>(src, dst, n, stride, arrays, shift); break;
    case 27: stream_probe_kernel<27><<<grid, BLOCK, 0, s>>>(src, dst, n, stride, arrays, shift); break;
    default: stream_probe_kernel<0><<<grid, BLOCK, 0, s>>>(src, dst, n, stride, arrays, shift); break;
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int64_t nblocks, double* out, hipStream_t s) {
  reduce_kernel<<<1, BLOCK, 0, s>>>(partials, nblocks, out);
  return hipGetLastError();
}
#endif  // LBM_COMMON

}  // namespace lbm
