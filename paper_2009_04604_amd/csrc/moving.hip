// Device-side geometry of a moving rigid sphere (dense layout, slot mode): the
// fluid mask, the cut links (q from the exact ray-sphere intersection, wall
// velocity of the rigid-body motion, Sec. II.E moving boundaries) and the
// equilibrium refill of fresh nodes are rebuilt every step over the segments
// of the sphere's sweep region.
//
// Geometry arithmetic is done with explicitly rounded FP64 operations (no FMA
// contraction) so that classification and q reproduce the plain double
// precision definition bit for bit.
#include <hip/hip_runtime.h>

#include "elibb.hpp"
#include "internal.hpp"
#include "lattice.hpp"
#include "storage.hpp"

namespace lbm {
namespace {

struct Site {
  uint32_t seg;
  int lane, x, y, z;
};

__device__ __forceinline__ Site region_site(const MovingParams& p, int64_t wave) {
  Site s;
  s.seg = (uint32_t)p.reg_seg[wave];
  s.lane = threadIdx.x & 63;
  const GridGeom& g = p.g;
  const uint32_t row = s.seg / (uint32_t)g.nseg_x;
  const uint32_t sx = s.seg - row * (uint32_t)g.nseg_x;
  s.x = (int)sx * 64 + s.lane;
  s.y = (int)(row % (uint32_t)g.ny);
  s.z = (int)(row / (uint32_t)g.ny);
  return s;
}

// minimum image on a periodic axis: d - L rint(d / L) (round half to even).
// Within |d| < 0.49 L the quotient rounds to 0 and the result is d itself, so
// the division is only evaluated outside that band (same result either way).
__device__ __forceinline__ double min_image(double d, int L, int periodic) {
  if (!periodic) return d;
  const double Ld = (double)L;
  if (fabs(d) < 0.49 * Ld) return d;
  return __dsub_rn(d, __dmul_rn(Ld, rint(__ddiv_rn(d, Ld))));
}

// The spheres' kinematics K: the kernel argument's MovingKin (single-domain
// launches) or a row of the batch table read through the constant address space
// (KinTab: nothing writes it while a kernel runs, so its loads are scalar and
// need no reload after the kernel's own stores).
using KinTab = const __attribute__((address_space(4))) MovingKin;

// position relative to sphere s's centre (minimum image on periodic axes)
template <class K>
__device__ __forceinline__ void rel(const MovingParams& p, const K& k, int s, double x, double y, double z,
                                    double (&d)[3]) {
  d[0] = min_image(__dsub_rn(x, k.c[s][0]), p.g.nx, p.g.perx);
  d[1] = min_image(__dsub_rn(y, k.c[s][1]), p.g.ny, p.g.pery);
  d[2] = min_image(__dsub_rn(z, k.c[s][2]), p.g.nz, p.g.perz);
}

__device__ __forceinline__ double norm2(const double (&d)[3]) {
  return __dadd_rn(__dadd_rn(__dmul_rn(d[0], d[0]), __dmul_rn(d[1], d[1])), __dmul_rn(d[2], d[2]));
}

// solid (inside or on some sphere) at integer node coordinates
template <bool M, class K>
__device__ __forceinline__ bool solid_at(const MovingParams& p, const K& k, int x, int y, int z) {
  for (int s = 0; s < (M ? k.ns : 1); ++s) {
    double d[3];
    rel(p, k, s, (double)x, (double)y, (double)z, d);
    if (norm2(d) <= __dmul_rn(k.r[s], k.r[s])) return true;
  }
  return false;
}

__device__ __forceinline__ int wrap(int v, int n, int periodic) {
  if (!periodic) return v;
  return v < 0 ? v + n : (v >= n ? v - n : v);
}

// entering root lam of x_F - lam c with sphere s; `reach` tells whether it lies
// on the segment (0, 1] (a root within 1e-12 of the segment's ends counts)
template <class K>
__device__ __forceinline__ double crossing(const MovingParams& p, const K& k, int s, int x, int y, int z, int cx,
                                           int cy, int cz,
                                           bool& reach) {
  double d[3];
  rel(p, k, s, (double)x, (double)y, (double)z, d);
  const double c[3] = {(double)cx, (double)cy, (double)cz};
  const double A = __dadd_rn(__dadd_rn(__dmul_rn(c[0], c[0]), __dmul_rn(c[1], c[1])), __dmul_rn(c[2], c[2]));
  const double B = __dadd_rn(__dadd_rn(__dmul_rn(d[0], c[0]), __dmul_rn(d[1], c[1])), __dmul_rn(d[2], c[2]));
  const double C0 = __dsub_rn(norm2(d), __dmul_rn(k.r[s], k.r[s]));
  const double disc = __dsub_rn(__dmul_rn(B, B), __dmul_rn(A, C0));
  const double sq = disc >= 0.0 ? __dsqrt_rn(disc) : 0.0;
  const double lam = __ddiv_rn(__dsub_rn(B, sq), A);
  reach = disc >= 0.0 && lam > -1e-12 && lam <= 1.0 + 1e-12;
  return lam;
}

// first crossing lam in (0, 1] of a cut link over the spheres (the first
// sphere wins a tie; with one sphere, that sphere's root) and the sphere crossed
template <bool M, class K>
__device__ __forceinline__ double first_crossing(const MovingParams& p, const K& k, int x, int y, int z, int cx,
                                                 int cy, int cz,
                                                 int& owner) {
  // roots are compared after clamping onto the segment, as the host builder does
  bool reach;
  double best = fmin(fmax(crossing(p, k, 0, x, y, z, cx, cy, cz, reach), 1e-12), 1.0);
  bool found = reach;
  owner = 0;
  for (int s = 1; s < (M ? k.ns : 1); ++s) {
    const double lam = fmin(fmax(crossing(p, k, s, x, y, z, cx, cy, cz, reach), 1e-12), 1.0);
    if (reach && (!found || lam < best)) {
      best = lam;
      owner = s;
      found = true;
    }
  }
  return best;
}

// the sphere whose surface is nearest to (x, y, z) (the first one on a tie)
template <bool M, class K>
__device__ __forceinline__ int nearest_sphere(const MovingParams& p, const K& k, double x, double y, double z) {
  int best_s = 0;
  double best = 0.0;
  for (int s = 0; s < (M ? k.ns : 1); ++s) {
    double d[3];
    rel(p, k, s, x, y, z, d);
    const double gap = __dsub_rn(__dsqrt_rn(norm2(d)), k.r[s]);
    if (s == 0 || gap < best) {
      best = gap;
      best_s = s;
    }
  }
  return best_s;
}

// rigid-body velocity V + Omega x r, r the minimum image of x - centre(t)
__device__ __forceinline__ void body_velocity(const double (&Om)[3], const double (&V)[3], const double (&r)[3],
                                              double (&u)[3]) {
  u[0] = __dadd_rn(V[0], __dsub_rn(__dmul_rn(Om[1], r[2]), __dmul_rn(Om[2], r[1])));
  u[1] = __dadd_rn(V[1], __dsub_rn(__dmul_rn(Om[2], r[0]), __dmul_rn(Om[0], r[2])));
  u[2] = __dadd_rn(V[2], __dsub_rn(__dmul_rn(Om[0], r[1]), __dmul_rn(Om[1], r[0])));
}

// cut directions of the fluid node (x, y, z): source x - c_i inside the sphere
template <class L, bool M, class K>
__device__ __forceinline__ uint32_t cut_mask(const MovingParams& p, const K& k, int x, int y, int z) {
  const GridGeom& g = p.g;
  uint32_t m = 0u;
  for (int s = 0; s < (M ? k.ns : 1); ++s) {
    // a node farther than r + 2 from the centre has no neighbour (|c_i| <= sqrt 3) in the sphere
    double d[3];
    rel(p, k, s, (double)x, (double)y, (double)z, d);
    const double far = k.r[s] + 2.0;
    if (norm2(d) > far * far) continue;
    const double r2 = __dmul_rn(k.r[s], k.r[s]);
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
      const int sx = wrap(x - L::cx(i), g.nx, g.perx);
      const int sy = wrap(y - L::cy(i), g.ny, g.pery);
      const int sz = wrap(z - L::cz(i), g.nz, g.perz);
      double e[3];
      rel(p, k, s, (double)sx, (double)sy, (double)sz, e);
      if (norm2(e) <= r2) m |= 1u << i;
    }
  }
  return m;
}

template <class L, bool M, class K>
__device__ __forceinline__ void classify_body(const MovingParams& p, const K& k, int64_t wave) {
  const Site s = region_site(p, wave);
  const GridGeom& g = p.g;
  const bool in = s.x < g.nx;
  const bool fluid = in && !solid_at<M>(p, k, s.x, s.y, s.z);
  const uint64_t fm = __ballot(fluid);
  const uint32_t cm = fluid ? cut_mask<L, M, K>(p, k, s.x, s.y, s.z) : 0u;
  p.reg_cut[wave * 64 + s.lane] = cm;   // read back by fill in the same rebuild
  const int cnt = __popc(cm);
  const uint64_t bm = __ballot(cnt > 0);
  int tot = cnt;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off, 64);
  if (s.lane == 0) {
    p.seg_prev[s.seg] = p.seg_fluid[s.seg];
    p.seg_fluid[s.seg] = fm;
    p.seg_bnd[s.seg] = bm;
    p.reg_count[wave] = tot;
  }
}

// Link starts of the region segments: an exclusive prefix sum of the region
// counts (one workgroup of 1024: per-thread chunks, wave scans, wave offsets),
// written at seg_lbase[seg] and seg_lbase[seg + 1] of every region segment
// (neighbouring region segments write the same value at their shared entry),
// and the total at seg_lbase[nseg].
__device__ __forceinline__ void region_scan_body(const MovingParams& p) {
  __shared__ int32_t wsum[16];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t n = p.nreg;
  const int64_t chunk = (n + 1023) / 1024;
  const int64_t b = t * chunk, e = min(n, b + chunk);
  int32_t own = 0;
  for (int64_t k = b; k < e; ++k) own += p.reg_count[k];
  int32_t inc = own;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t v = __shfl_up(inc, off, 64);
    if (lane >= off) inc += v;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  if (w == 0) {
    const int32_t x = lane < 16 ? wsum[lane] : 0;
    int32_t xi = x;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      const int32_t v = __shfl_up(xi, off, 64);
      if (lane >= off) xi += v;
    }
    if (lane < 16) wsum[lane] = xi - x;
    if (lane == 15) p.seg_lbase[p.g.nseg] = xi;
  }
  __syncthreads();
  int32_t run = wsum[w] + inc - own;
  for (int64_t k = b; k < e; ++k) {
    const int32_t c = p.reg_count[k];
    const int32_t sg = p.reg_seg[k];
    p.seg_lbase[sg] = run;
    p.seg_lbase[sg + 1] = run + c;
    run += c;
  }
}

template <class L, typename R, bool M, class K>
__device__ __forceinline__ void fill_body(const MovingParams& p, const K& kn, int64_t wave) {
  if (p.reg_count[wave] == 0) return;   // wave-uniform: no cut link in this segment
  const Site s = region_site(p, wave);
  const uint32_t cm = p.reg_cut[wave * 64 + s.lane];   // classify's cut directions (0 off the fluid)
  // exclusive prefix of the lanes' link counts
  const int cnt = __popc(cm);
  int inc = cnt;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(inc, off, 64);
    if (s.lane >= off) inc += v;
  }
  int k = p.seg_lbase[s.seg] + inc - cnt;
  R* lq = static_cast<R*>(p.lq);
  R* lg = static_cast<R*>(p.lg);
  for (int i = 1; i < L::Q; ++i) {
    if (!((cm >> i) & 1u)) continue;
    const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
    int o;
    const double q = first_crossing<M>(p, kn, s.x, s.y, s.z, cx, cy, cz, o);
    // wall point and its rigid-body velocity at t and t+1 (of the sphere crossed)
    const double xw[3] = {__dsub_rn((double)s.x, __dmul_rn(q, (double)cx)), __dsub_rn((double)s.y, __dmul_rn(q, (double)cy)),
                          __dsub_rn((double)s.z, __dmul_rn(q, (double)cz))};
    double r[3];
    rel(p, kn, o, xw[0], xw[1], xw[2], r);
    double u0[3], u1[3];
    const double Om0[3] = {kn.Om[o][0], kn.Om[o][1], kn.Om[o][2]}, Om1[3] = {kn.Om1[o][0], kn.Om1[o][1], kn.Om1[o][2]};
    const double V0[3] = {kn.V[o][0], kn.V[o][1], kn.V[o][2]}, V1[3] = {kn.V1[o][0], kn.V1[o][1], kn.V1[o][2]};
    body_velocity(Om0, V0, r, u0);
    body_velocity(Om1, V1, r, u1);
    if (L::D == 2) u0[2] = u1[2] = 0.0;
    const double cu0 = cx * u0[0] + cy * u0[1] + cz * u0[2];
    const double cu1 = cx * u1[0] + cy * u1[1] + cz * u1[2];
    const double uu0 = u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2];
    const double uu1 = u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2];
    const Coef<R> a = elibb_coefficients<R>(p.variant, R(q), R(p.q_cut));
    const Coef<double> ad{a.a4, a.a5, a.a2, a.a3};
    p.lld[k] = (uint16_t)(s.lane | (i << 8));
    lq[k] = R(q);
    lg[k] = R(wall_term<double>(ad, cu0, uu0, cu1, uu1));
    if (p.luv) {
      R* uv = static_cast<R*>(p.luv);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        uv[k + a * p.luv_stride] = R(u0[a]);
        uv[k + (3 + a) * p.luv_stride] = R(u1[a]);
      }
    }
    ++k;
  }
}

// fresh nodes (solid at t-1, fluid at t): f = f^eq(rho_bar, u_body(x)), rho_bar the
// mean density of the neighbours that are fluid at t-1 and t (rho0 if none)
template <class L, int S, bool M, class K>
__device__ __forceinline__ void refill_body(const MovingParams& p, const K& kn, int64_t wave) {
  using St = Storage<S>;
  using T = typename St::T;
  using R = typename St::R;
  const Site s = region_site(p, wave);
  const GridGeom& g = p.g;
  const uint64_t fresh = p.seg_fluid[s.seg] & ~p.seg_prev[s.seg];
  if (!((fresh >> s.lane) & 1ull)) return;
  T* pop = static_cast<T*>(p.pop);
  const size_t np = (size_t)g.npad;
  auto slot = [&](int x, int y, int z) -> uint32_t {   // dense storage index (periodic box)
    return (uint32_t)(x + g.px) + (uint32_t)g.NX * ((uint32_t)(y + g.py) + (uint32_t)g.NY * (uint32_t)(z + g.pz));
  };
  double tot = 0.0;
  int cnt = 0;
#pragma unroll
  for (int j = 1; j < L::Q; ++j) {
    const int yx = wrap(s.x + L::cx(j), g.nx, g.perx);
    const int yy = wrap(s.y + L::cy(j), g.ny, g.pery);
    const int yz = wrap(s.z + L::cz(j), g.nz, g.perz);
    if (yx < 0 || yx >= g.nx || yy < 0 || yy >= g.ny || yz < 0 || yz >= g.nz) continue;
    const uint32_t ys = (uint32_t)(yx / 64) + (uint32_t)g.nseg_x * ((uint32_t)yy + (uint32_t)g.ny * (uint32_t)yz);
    const uint64_t bit = 1ull << (yx % 64);
    if (!(p.seg_fluid[ys] & bit) || !(p.seg_prev[ys] & bit)) continue;
    double rho = 1.0;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      const int sx = wrap(yx - L::cx(k), g.nx, g.perx);
      const int sy = wrap(yy - L::cy(k), g.ny, g.pery);
      const int sz = wrap(yz - L::cz(k), g.nz, g.perz);
      rho += (double)St::template load<L>(pop + k * np + slot(sx, sy, sz), k);
    }
    tot += rho;
    ++cnt;
  }
  const double rb = cnt > 0 ? tot / cnt : p.rho0;
  double r[3], u[3];
  const int o = nearest_sphere<M>(p, kn, (double)s.x, (double)s.y, (double)s.z);
  rel(p, kn, o, (double)s.x, (double)s.y, (double)s.z, r);
  const double Om0[3] = {kn.Om[o][0], kn.Om[o][1], kn.Om[o][2]}, V0[3] = {kn.V[o][0], kn.V[o][1], kn.V[o][2]};
  body_velocity(Om0, V0, r, u);
  if (L::D == 2) u[2] = 0.0;
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const double cu = L::cx(i) * u[0] + L::cy(i) * u[1] + L::cz(i) * u[2];
    const double h = L::w(i) * ((rb - 1.0) + rb * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    const int sx = wrap(s.x - L::cx(i), g.nx, g.perx);
    const int sy = wrap(s.y - L::cy(i), g.ny, g.pery);
    const int sz = wrap(s.z - L::cz(i), g.nz, g.perz);
    St::template store<L>(pop + i * np + slot(sx, sy, sz), R(h), i);
  }
}

// Momentum-exchange force and torque of the step that used geometry t (Sec. II
// "Force computation", Galilean-invariant form), per link of that geometry,
// evaluated after the step and before the links are rebuilt:
//   F = (c_ibar - u_w) f*_ibar(x_F, t) - (c_i - u_w) f_i(x_F, t+1),  T = r x F,
// r = x_W - x_c(t) (minimum image), u_w = V(t) + Omega x r; f*_ibar(x_F, t) is
// x_F's own post-collision slot (no node pulls it), f_i(x_F, t+1) the value the
// step stored in the solid-side slot x_F - c_i.  `pop` is the buffer the step
// wrote; out receives 6 doubles per link.
template <class L, int S>
__device__ __forceinline__ void force_body(const MovingParams& p, int64_t wave, double* out, int32_t* grp) {
  using St = Storage<S>;
  using T = typename St::T;
  using R = typename St::R;
  if (p.reg_count[wave] == 0) return;
  const Site s = region_site(p, wave);
  const GridGeom& g = p.g;
  const T* pop = static_cast<const T*>(p.pop);
  const size_t np = (size_t)g.npad;
  auto slot = [&](int x, int y, int z) -> size_t {
    return (size_t)(x + g.px) + (size_t)g.NX * ((size_t)(y + g.py) + (size_t)g.NY * (size_t)(z + g.pz));
  };
  const int lb0 = p.seg_lbase[s.seg], lb1 = p.seg_lbase[s.seg + 1];
  const R* lq = static_cast<const R*>(p.lq);
  for (int k = lb0 + s.lane; k < lb1; k += 64) {
    const int ld = p.lld[k];
    const int nl = ld & 63, i = ld >> 8;
    const int x = s.x - s.lane + nl;
    int cx = 0, cy = 0, cz = 0, ib = 0;
    double w = 0.0;
#pragma unroll
    for (int j = 1; j < L::Q; ++j)
      if (j == i) {
        cx = L::cx(j);
        cy = L::cy(j);
        cz = L::cz(j);
        ib = L::opp(j);
        w = L::w(j);
      }
    double fs = 0.0, fn = 0.0;
#pragma unroll
    for (int j = 1; j < L::Q; ++j) {
      if (j == ib) fs = (double)St::template load<L>(pop + j * np + slot(x, s.y, s.z), j) + w;
      if (j == i)
        fn = (double)St::template load<L>(pop + j * np + slot(wrap(x - cx, g.nx, g.perx), wrap(s.y - cy, g.ny, g.pery),
                                                               wrap(s.z - cz, g.nz, g.perz)), j) + w;
    }
    const double q = (double)lq[k];
    // the sphere the link crosses: the one holding its solid source node (the
    // spheres keep more than two nodes apart, so a link reaches one of them)
    int own = 0;
    for (int sp = 1; sp < p.k.ns; ++sp) {
      double e[3];
      rel(p, p.k, sp, (double)wrap(x - cx, g.nx, g.perx), (double)wrap(s.y - cy, g.ny, g.pery),
          (double)wrap(s.z - cz, g.nz, g.perz), e);
      if (norm2(e) <= __dmul_rn(p.k.r[sp], p.k.r[sp])) own = sp;
    }
    double r[3], u[3];
    rel(p, p.k, own, x - q * cx, s.y - q * cy, s.z - q * cz, r);
    const double Om0[3] = {p.k.Om[own][0], p.k.Om[own][1], p.k.Om[own][2]};
    const double V0[3] = {p.k.V[own][0], p.k.V[own][1], p.k.V[own][2]};
    body_velocity(Om0, V0, r, u);
    if (grp) grp[k] = own;
    if (L::D == 2) u[2] = r[2] = 0.0;
    const double c[3] = {(double)cx, (double)cy, (double)cz};
    double F[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) F[a] = (-c[a] - u[a]) * fs - (c[a] - u[a]) * fn;
    double* o = out + 6 * (int64_t)k;
    o[0] = F[0];
    o[1] = F[1];
    o[2] = F[2];
    o[3] = r[1] * F[2] - r[2] * F[1];
    o[4] = r[2] * F[0] - r[0] * F[2];
    o[5] = r[0] * F[1] - r[1] * F[0];
  }
}

// Single sphere: one wave per region segment.
template <class L, bool M>
__global__ __launch_bounds__(256) void classify_kernel(MovingParams p) {
  const int64_t wave = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (wave < p.nreg) classify_body<L, M>(p, p.k, wave);
}

__global__ __launch_bounds__(1024) void region_scan_kernel(MovingParams p) { region_scan_body(p); }

template <class L, typename R, bool M>
__global__ __launch_bounds__(256) void fill_kernel(MovingParams p) {
  const int64_t wave = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (wave < p.nreg) fill_body<L, R, M>(p, p.k, wave);
}

template <class L, int S, bool M>
__global__ __launch_bounds__(256) void refill_kernel(MovingParams p) {
  const int64_t wave = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (wave < p.nreg) refill_body<L, S, M>(p, p.k, wave);
}

template <class L, int S>
__global__ __launch_bounds__(256) void moving_force_kernel(MovingParams p, double* out, int32_t* grp) {
  const int64_t wave = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (wave < p.nreg) force_body<L, S>(p, wave, out, grp);
}

// Entry of the sphere table with its pointers read through the constant address
// space (the host writes the table; kernels only read it), so that the arrays
// they name are addressed with global memory instructions.
__device__ __forceinline__ MovingParams table_entry(const MovingParams* e) {
  MovingParams p = *e;
  p.reg_seg = load_const(&e->reg_seg);
  p.seg_fluid = load_const(&e->seg_fluid);
  p.seg_prev = load_const(&e->seg_prev);
  p.seg_bnd = load_const(&e->seg_bnd);
  p.reg_count = load_const(&e->reg_count);
  p.reg_cut = load_const(&e->reg_cut);
  p.seg_lbase = load_const(&e->seg_lbase);
  p.lld = load_const(&e->lld);
  p.lq = load_const(&e->lq);
  p.lg = load_const(&e->lg);
  p.luv = load_const(&e->luv);
  p.pop = load_const(&e->pop);
  return p;
}

// Batched spheres: the wave table names (sphere, region wave); the kinematics
// come from row *ctr of the table.
__device__ __forceinline__ bool batch_wave(const MovingBatch& b, MovingParams& p, KinTab*& kp, int64_t& wave) {
  const uint32_t gw = blockIdx.x * 4u + threadIdx.x / 64u;
  if (gw >= b.nwaves) return false;
  const uint32_t w = __builtin_amdgcn_readfirstlane(b.waves[gw]);
  p = table_entry(b.tab + (w >> TILE_SHIFT));
  // the kinematics stay in the table (read where used, not copied)
  kp = (KinTab*)(b.kin + (*b.ctr * b.nkin + p.kin_slot));
  wave = (int64_t)(w & TILE_MASK);
  return true;
}

template <class L, bool M>
__global__ __launch_bounds__(256) void classify_batch_kernel(MovingBatch b) {
  MovingParams p;
  KinTab* kp;
  int64_t wave;
  if (batch_wave(b, p, kp, wave)) classify_body<L, M>(p, *kp, wave);
}

__global__ __launch_bounds__(1024) void region_scan_batch_kernel(MovingBatch b) {
  region_scan_body(table_entry(b.tab + blockIdx.x));
}

template <class L, typename R, bool M>
__global__ __launch_bounds__(256) void fill_batch_kernel(MovingBatch b) {
  MovingParams p;
  KinTab* kp;
  int64_t wave;
  if (batch_wave(b, p, kp, wave)) fill_body<L, R, M>(p, *kp, wave);
}

template <class L, int S, bool M>
__global__ __launch_bounds__(256) void refill_batch_kernel(MovingBatch b) {
  MovingParams p;
  KinTab* kp;
  int64_t wave;
  if (batch_wave(b, p, kp, wave)) refill_body<L, S, M>(p, *kp, wave);
}

__global__ void advance_kernel(int64_t* ctr) {
  if (threadIdx.x == 0) ctr[0] = ctr[0] + 1;
}

}  // namespace

static inline dim3 region_grid(const MovingParams& p) { return dim3((unsigned)((p.nreg + 3) / 4)); }

// The kernels come in a one-sphere form (M = false: the sphere loops are a
// single iteration known at compile time, as fast as a kernel for one sphere)
// and a form for several spheres per domain.
template <bool M>
static void classify_launch(int lattice, const MovingParams& p, hipStream_t s) {
  if (lattice == LBM_D2Q9) classify_kernel<D2Q9, M><<<region_grid(p), 256, 0, s>>>(p);
  else if (lattice == LBM_D3Q19) classify_kernel<D3Q19, M><<<region_grid(p), 256, 0, s>>>(p);
  else classify_kernel<D3Q27, M><<<region_grid(p), 256, 0, s>>>(p);
}

hipError_t launch_moving_classify(int lattice, const MovingParams& p, hipStream_t s) {
  if (p.nreg == 0) return hipSuccess;
  if (p.k.ns > 1) classify_launch<true>(lattice, p, s);
  else classify_launch<false>(lattice, p, s);
  return hipGetLastError();
}

hipError_t launch_region_scan(const MovingParams& p, hipStream_t s) {
  region_scan_kernel<<<1, 1024, 0, s>>>(p);
  return hipGetLastError();
}

template <bool M>
static void fill_launch(int lattice, bool f64, const MovingParams& p, hipStream_t s) {
  if (lattice == LBM_D2Q9) {
    if (f64) fill_kernel<D2Q9, double, M><<<region_grid(p), 256, 0, s>>>(p);
    else fill_kernel<D2Q9, float, M><<<region_grid(p), 256, 0, s>>>(p);
  } else if (lattice == LBM_D3Q19) {
    if (f64) fill_kernel<D3Q19, double, M><<<region_grid(p), 256, 0, s>>>(p);
    else fill_kernel<D3Q19, float, M><<<region_grid(p), 256, 0, s>>>(p);
  } else {
    if (f64) fill_kernel<D3Q27, double, M><<<region_grid(p), 256, 0, s>>>(p);
    else fill_kernel<D3Q27, float, M><<<region_grid(p), 256, 0, s>>>(p);
  }
}

hipError_t launch_moving_fill(int lattice, int storage, const MovingParams& p, hipStream_t s) {
  if (p.nreg == 0) return hipSuccess;
  const bool f64 = storage == ST_F64;
  if (p.k.ns > 1) fill_launch<true>(lattice, f64, p, s);
  else fill_launch<false>(lattice, f64, p, s);
  return hipGetLastError();
}

template <bool M>
static void refill_launch(int lattice, int storage, const MovingParams& p, hipStream_t s) {
#define LBM_REFILL(LAT)                                                                     \
  switch (storage) {                                                                        \
    case ST_F64: refill_kernel<LAT, ST_F64, M><<<region_grid(p), 256, 0, s>>>(p); break;    \
    case ST_F32: refill_kernel<LAT, ST_F32, M><<<region_grid(p), 256, 0, s>>>(p); break;    \
    case ST_F16S: refill_kernel<LAT, ST_F16S, M><<<region_grid(p), 256, 0, s>>>(p); break;  \
    default: refill_kernel<LAT, ST_BF16S, M><<<region_grid(p), 256, 0, s>>>(p); break;      \
  }
  if (lattice == LBM_D2Q9) {
    LBM_REFILL(D2Q9)
  } else if (lattice == LBM_D3Q19) {
    LBM_REFILL(D3Q19)
  } else {
    LBM_REFILL(D3Q27)
  }
#undef LBM_REFILL
}

hipError_t launch_moving_refill(int lattice, int storage, const MovingParams& p, hipStream_t s) {
  if (p.nreg == 0) return hipSuccess;
  if (p.k.ns > 1) refill_launch<true>(lattice, storage, p, s);
  else refill_launch<false>(lattice, storage, p, s);
  return hipGetLastError();
}

hipError_t launch_moving_force(int lattice, int storage, const MovingParams& p, double* contrib, int32_t* grp,
                               double* out, hipStream_t s) {
  if (p.nreg > 0) {
#define LBM_MFORCE(LAT)                                                                            \
  switch (storage) {                                                                               \
    case ST_F64: moving_force_kernel<LAT, ST_F64><<<region_grid(p), 256, 0, s>>>(p, contrib, grp); break;\
    case ST_F32: moving_force_kernel<LAT, ST_F32><<<region_grid(p), 256, 0, s>>>(p, contrib, grp); break;\
    case ST_F16S: moving_force_kernel<LAT, ST_F16S><<<region_grid(p), 256, 0, s>>>(p, contrib, grp); break;\
    default: moving_force_kernel<LAT, ST_BF16S><<<region_grid(p), 256, 0, s>>>(p, contrib, grp); break;\
  }
    if (lattice == LBM_D2Q9) {
      LBM_MFORCE(D2Q9)
    } else if (lattice == LBM_D3Q19) {
      LBM_MFORCE(D3Q19)
    } else {
      LBM_MFORCE(D3Q27)
    }
#undef LBM_MFORCE
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return launch_group_sum(contrib, p.k.ns > 1 ? grp : nullptr, 0, p.seg_lbase + p.g.nseg, p.k.ns, out, s);
}

template <bool M>
static void moving_batch_launch(int lattice, int storage, const MovingBatch& b, hipStream_t s) {
  const dim3 grid((b.nwaves + 3) / 4);
  const bool f64 = storage == ST_F64;
#define LBM_MOVING_BATCH(LAT)                                                                  \
  classify_batch_kernel<LAT, M><<<grid, 256, 0, s>>>(b);                                       \
  region_scan_batch_kernel<<<b.nbox, 1024, 0, s>>>(b);                                         \
  if (f64) fill_batch_kernel<LAT, double, M><<<grid, 256, 0, s>>>(b);                          \
  else fill_batch_kernel<LAT, float, M><<<grid, 256, 0, s>>>(b);                               \
  switch (storage) {                                                                           \
    case ST_F64: refill_batch_kernel<LAT, ST_F64, M><<<grid, 256, 0, s>>>(b); break;           \
    case ST_F32: refill_batch_kernel<LAT, ST_F32, M><<<grid, 256, 0, s>>>(b); break;           \
    case ST_F16S: refill_batch_kernel<LAT, ST_F16S, M><<<grid, 256, 0, s>>>(b); break;         \
    default: refill_batch_kernel<LAT, ST_BF16S, M><<<grid, 256, 0, s>>>(b); break;             \
  }
  if (lattice == LBM_D2Q9) {
    LBM_MOVING_BATCH(D2Q9)
  } else if (lattice == LBM_D3Q19) {
    LBM_MOVING_BATCH(D3Q19)
  } else {
    LBM_MOVING_BATCH(D3Q27)
  }
#undef LBM_MOVING_BATCH
}

hipError_t launch_moving_batch(int lattice, int storage, const MovingBatch& b, hipStream_t s) {
  if (b.nbox == 0) return hipSuccess;
  if (b.multi) moving_batch_launch<true>(lattice, storage, b, s);
  else moving_batch_launch<false>(lattice, storage, b, s);
  return hipGetLastError();
}

hipError_t launch_advance(int64_t* ctr, hipStream_t s) {
  advance_kernel<<<1, 64, 0, s>>>(ctr);
  return hipGetLastError();
}

}  // namespace lbm
