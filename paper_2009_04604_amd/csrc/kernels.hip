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

namespace lbm {

struct Coords {
  int x, y, z;
};

// Segment of the calling wave and the lane's coordinates.  Workgroups are dealt
// round-robin to the 8 XCDs; the logical block id makes XCD k walk the k-th
// contiguous eighth of the rows (the grid is padded to a multiple of 8).
struct SegInfo {
  uint32_t seg;
  int lane;
  Coords c;
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

__device__ __forceinline__ SegInfo seg_info(const GridGeom& g) {
  SegInfo s;
  s.lane = threadIdx.x & (SEG - 1);
  const uint32_t wave = logical_block(g.xcd_remap) * WAVES_PER_BLOCK + __builtin_amdgcn_readfirstlane(threadIdx.x / SEG);
  s.seg = wave;
  const uint32_t row = fast_div(wave, g.div_nseg_x);
  const uint32_t sx = wave - row * (uint32_t)g.nseg_x;
  const uint32_t z = fast_div(row, g.div_ny);
  s.c.x = (int)sx * SEG + s.lane;
  s.c.y = (int)(row - z * (uint32_t)g.ny);
  s.c.z = (int)z;
  return s;
}

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
  return i == 0 ? R(L::w(0)) : (i <= 2 * L::D ? R(L::w(1)) : R(L::w(2 * L::D + 1)));
}
// opposite direction: axis pairs (1,2),(3,4),...; then groups of four sign pairs
template <class L>
__device__ __forceinline__ int dyn_opp(int i) {
  if (i == 0) return 0;
  if (i <= 2 * L::D) return (i & 1) ? i + 1 : i - 1;
  const int r = (i - 2 * L::D - 1) & 3;
  return i - r + (3 - r);
}
template <class L>
constexpr bool dyn_tables_ok() {
  for (int i = 0; i < L::Q; ++i) {
    const int r = (i - 2 * L::D - 1) & 3;
    const int o = i == 0 ? 0 : (i <= 2 * L::D ? ((i & 1) ? i + 1 : i - 1) : i - r + (3 - r));
    if (o != L::opp(i)) return false;
    const double w = i == 0 ? L::w(0) : (i <= 2 * L::D ? L::w(1) : L::w(2 * L::D + 1));
    if (w != L::w(i)) return false;
  }
  return true;
}
static_assert(dyn_tables_ok<D2Q9>() && dyn_tables_ok<D3Q19>(), "run-time direction tables");

// Moments of the shifted populations at one node.
template <typename R>
struct Moments {
  R drho, rho, ux, uy, uz, uu;
};

// Post-collision shifted population h*_i = h_i - omega (h_i - h^eq_i) + (1 - omega/2) S_i
// with h^eq_i = f^eq_i - w_i = w_i [ (rho - 1) + rho (3 cu + 4.5 cu^2 - 1.5 uu) ]
// (eq. LB-BGK, eq. Eq2ndOrder with c_s^2 = 1/3) and Guo's source term S_i.
template <typename R>
struct Collider {
  R omega, kf, Fx, Fy, Fz;
  bool force;
  __device__ __forceinline__ R heq(R cx, R cy, R cz, R w, const Moments<R>& m) const {
    const R cu = cx * m.ux + cy * m.uy + cz * m.uz;
    return w * ((m.drho - R(1.5) * m.rho * m.uu) + m.rho * cu * (R(3) + R(4.5) * cu));
  }
  __device__ __forceinline__ R post(R cx, R cy, R cz, R w, R h, const Moments<R>& m) const {
    const R cu = cx * m.ux + cy * m.uy + cz * m.uz;
    const R he = w * ((m.drho - R(1.5) * m.rho * m.uu) + m.rho * cu * (R(3) + R(4.5) * cu));
    R v = h + omega * (he - h);
    if (force) {
      const R cF = cx * Fx + cy * Fy + cz * Fz;
      const R uF = m.ux * Fx + m.uy * Fy + m.uz * Fz;
      v += (kf * w) * (R(3) * (cF - uF) + R(9) * cu * cF);
    }
    return v;
  }
};

template <class L, typename R>
__device__ __forceinline__ Moments<R> moments(const R (&h)[L::Q], R Fx, R Fy, R Fz) {
  R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    drho += h[i];
    if (L::cx(i)) jx += R(L::cx(i)) * h[i];
    if (L::cy(i)) jy += R(L::cy(i)) * h[i];
    if (L::cz(i)) jz += R(L::cz(i)) * h[i];
  }
  Moments<R> m;
  m.drho = drho;
  m.rho = R(1) + drho;
  const R inv = R(1) / m.rho;
  m.ux = (jx + R(0.5) * Fx) * inv;
  m.uy = (jy + R(0.5) * Fy) * inv;
  m.uz = (jz + R(0.5) * Fz) * inv;
  m.uu = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
  return m;
}

// Element offsets (within one direction array) of a node and of its pull
// sources: source of direction i = xs[1 + cx] + ys[1 + cy] + zs[1 + cz], with
// wrap on periodic axes and the halo layer beyond non-periodic faces.
struct PullIndex {
  uint32_t xs[3], ys[3], zs[3];
  uint32_t self;
};

__device__ __forceinline__ PullIndex pull_index(const GridGeom& g, Coords c) {
  const uint32_t NX = (uint32_t)g.NX, NXY = (uint32_t)g.NX * (uint32_t)g.NY;
  const int xm = (g.perx && c.x == 0) ? g.nx - 1 : c.x - 1;
  const int xp = (g.perx && c.x == g.nx - 1) ? 0 : c.x + 1;
  const int ym = (g.pery && c.y == 0) ? g.ny - 1 : c.y - 1;
  const int yp = (g.pery && c.y == g.ny - 1) ? 0 : c.y + 1;
  const int zm = (g.perz && c.z == 0) ? g.nz - 1 : c.z - 1;
  const int zp = (g.perz && c.z == g.nz - 1) ? 0 : c.z + 1;
  PullIndex p;
  // indexed by 1 + c: the source of direction c is x - c
  p.xs[0] = (uint32_t)(xp + g.px);
  p.xs[1] = (uint32_t)(c.x + g.px);
  p.xs[2] = (uint32_t)(xm + g.px);
  p.ys[0] = (uint32_t)(yp + g.py) * NX;
  p.ys[1] = (uint32_t)(c.y + g.py) * NX;
  p.ys[2] = (uint32_t)(ym + g.py) * NX;
  p.zs[0] = (uint32_t)(zp + g.pz) * NXY;
  p.zs[1] = (uint32_t)(c.z + g.pz) * NXY;
  p.zs[2] = (uint32_t)(zm + g.pz) * NXY;
  p.self = p.xs[1] + p.ys[1] + p.zs[1];
  return p;
}

template <class L>
__device__ __forceinline__ uint32_t src_of(const PullIndex& p, int i) {
  return p.xs[1 + L::cx(i)] + p.ys[1 + L::cy(i)] + p.zs[1 + L::cz(i)];
}

// Storage index of x - c for run-time c (element offset within one direction array).
__device__ __forceinline__ uint32_t src_index_dyn(const GridGeom& g, Coords c, int cx, int cy, int cz) {
  int sx = c.x - cx, sy = c.y - cy, sz = c.z - cz;
  sx = (g.perx && sx < 0) ? sx + g.nx : ((g.perx && sx >= g.nx) ? sx - g.nx : sx);
  sy = (g.pery && sy < 0) ? sy + g.ny : ((g.pery && sy >= g.ny) ? sy - g.ny : sy);
  sz = (g.perz && sz < 0) ? sz + g.nz : ((g.perz && sz >= g.nz) ? sz - g.nz : sz);
  return (uint32_t)(sx + g.px) + (uint32_t)g.NX * ((uint32_t)(sy + g.py) + (uint32_t)g.NY * (uint32_t)(sz + g.pz));
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
//  4. zero-gradient outlet copy on the outlet face layer.
// ---------------------------------------------------------------------------
template <class L, int S>
__global__ __launch_bounds__(BLOCK) void step_kernel(StepParams p) {
  using St = Storage<S>;
  using T = typename St::T;
  using R = typename St::R;
  constexpr int NV = L::Q + 4;
  __shared__ R stage[NV][BLOCK];
  const GridGeom& g = p.g;
  const LinkView& lk = p.lk;
  const SegInfo si = seg_info(g);
  if (si.seg >= g.nseg) return;
  const uint64_t fm = lk.seg_fluid[si.seg];
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

  Collider<R> col;
  col.omega = R(p.omega);
  col.kf = R(1) - R(0.5) * col.omega;
  col.Fx = R(p.force[0]);
  col.Fy = R(p.force[1]);
  col.Fz = R(p.force[2]);
  col.force = p.has_force != 0;

  const int lb0 = lk.seg_lbase[si.seg];
  const int lb1 = lk.seg_lbase[si.seg + 1];
  const bool has_links = lb1 > lb0;
  const R* __restrict__ lq = static_cast<const R*>(lk.lq);
  const R* __restrict__ lg = static_cast<const R*>(lk.lg);
  const R* __restrict__ lvi = static_cast<const R*>(lk.lv_in);
  R* __restrict__ lvo = static_cast<R*>(lk.lv_out);
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

  const PullIndex pi = pull_index(g, c);
  R h[L::Q];
  if (fluid) {
#pragma unroll
    for (int i = 0; i < L::Q; ++i) h[i] = St::template load<L>(src + i * np + src_of<L>(pi, i), i);
  }
  const bool bnd = fluid && ((lk.seg_bnd[si.seg] >> si.lane) & 1ull);
  if (has_links && list_mode) patch_links<L, R, 2>(h, stage, bnd, tid, wbase, lb0, lb1, si.lane, lk.lld, lvi, ldp, vp);

  Moments<R> m;
  if (!fluid) {
    // solid lane of a non-empty segment: zero populations, so that the shared
    // cache lines are written whole (list mode; nothing reads these slots)
#pragma unroll
    for (int i = 0; i < L::Q; ++i) h[i] = R(0);
  }
  m = moments<L, R>(h, col.Fx, col.Fy, col.Fz);
  if (fluid || (list_mode && inrow)) {
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
      const R v = col.post(R(L::cx(i)), R(L::cy(i)), R(L::cz(i)), R(L::w(i)), h[i], m);
      St::template store<L>(dst + i * np + pi.self, fluid ? v : R(0), i);
    }
  }
  if (fluid) {
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
  }

  if (has_links) {
    wave_lds_sync();
    const int xseg = c.x - si.lane;
    const R qc = R(p.q_cut);
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
      mb.uu = mb.ux * mb.ux + mb.uy * mb.uy + mb.uz * mb.uz;
      const R hb = stage[ib][t];
      const R hi = stage[i][t];
      const int icx = dyn_c<L, 0>(i), icy = dyn_c<L, 1>(i), icz = dyn_c<L, 2>(i);
      const R cx = R(icx), cy = R(icy), cz = R(icz);
      const R w = dyn_w<L, R>(i);
      const Coef<R> a = elibb_coefficients_fast<R>(p.variant, q, qc);
      // bounced direction: c_ibar = -c_i, w_ibar = w_i
      const R he_b = col.heq(-cx, -cy, -cz, w, mb);
      const R hs_b = col.post(-cx, -cy, -cz, w, hb, mb);
      const R n_pre = hb - he_b;         // bounced pre-collision non-equilibrium (eq. neqbb-s)
      const R n_post = hs_b - he_b;      // bounced post-collision non-equilibrium
      R v = a.a4 * n_pre + a.a5 * n_post + a.a2 * hs_b + w * (mb.drho * (a.a4 + a.a5) + mb.rho * gw);
      v += a.a3 * col.post(cx, cy, cz, w, hi, mb);
      if (list_mode) {
        lvo[k] = v;
      } else {
        Coords cf = c;
        cf.x = xseg + nl;
        St::template store<L>(dst + (size_t)i * np + src_index_dyn(g, cf, icx, icy, icz), v, i);
      }
    };
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int k = lb0 + si.lane + j * SEG;
      if (k < lb1) rebuild(k, ldp[j], qp[j], gp[j]);
    }
    for (int k = lb0 + si.lane + 2 * SEG; k < lb1; k += SEG) rebuild(k, lk.lld[k], lq[k], lg ? lg[k] : R(0));
  }

  // zero-gradient outlet: the face-layer node writes its post-collision values of
  // the inward directions into the halo slot beyond the face, which its
  // neighbour along the face pulls.
  if (fluid && p.outlet_face >= 0) {
    const int f = p.outlet_face, a = f >> 1;
    const int sgn = (f & 1) ? 1 : -1;
    const int coord = a == 0 ? c.x : (a == 1 ? c.y : c.z);
    const int n_a = a == 0 ? g.nx : (a == 1 ? g.ny : g.nz);
    if (coord == (sgn > 0 ? n_a - 1 : 0)) {
      Coords halo = c;
      if (a == 0) halo.x += sgn;
      else if (a == 1) halo.y += sgn;
      else halo.z += sgn;
      const uint32_t hidx = src_index_dyn(g, halo, 0, 0, 0);
#pragma unroll
      for (int i = 1; i < L::Q; ++i) {
        const int ca = a == 0 ? L::cx(i) : (a == 1 ? L::cy(i) : L::cz(i));
        if (ca == -sgn)
          St::template store<L>(dst + i * np + hidx, col.post(R(L::cx(i)), R(L::cy(i)), R(L::cz(i)), R(L::w(i)), h[i], m), i);
      }
    }
  }
}

// Pre-collision shifted populations of one lane's node (pull + link patch).
// Every lane of the wave must call it (the patch is a wave-level exchange).
template <class L, int S>
__device__ __forceinline__ void gather_state(const GridGeom& g, const LinkView& lk, const void* srcv, const SegInfo& si,
                                             bool fluid, typename Storage<S>::R (&h)[L::Q],
                                             typename Storage<S>::R (*stage)[BLOCK]) {
  using St = Storage<S>;
  using T = typename St::T;
  using R = typename St::R;
  const T* src = static_cast<const T*>(srcv);
  const PullIndex pi = pull_index(g, si.c);
#pragma unroll
  for (int i = 0; i < L::Q; ++i) h[i] = R(0);
  if (fluid) {
#pragma unroll
    for (int i = 0; i < L::Q; ++i) h[i] = St::template load<L>(src + i * (size_t)g.npad + src_of<L>(pi, i), i);
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

template <class L, int S>
__global__ __launch_bounds__(BLOCK) void init_kernel(InitParams p) {
  using St = Storage<S>;
  using T = typename St::T;
  using R = typename St::R;
  const GridGeom& g = p.g;
  const SegInfo si = seg_info(g);
  if (si.seg >= g.nseg) return;
  const uint64_t fm = p.lk.seg_fluid[si.seg];
  if (!((fm >> si.lane) & 1ull)) return;
  const Coords c = si.c;
  T* dst = static_cast<T*>(p.dst);
  const int64_t n = c.x + (int64_t)g.nx * (c.y + (int64_t)g.ny * c.z);
  const PullIndex pi = pull_index(g, c);
#pragma unroll
  for (int i = 0; i < L::Q; ++i)
    St::template store<L>(dst + i * (size_t)g.npad + src_of<L>(pi, i), R(init_value<L>(p, n, i)), i);
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
template <class L, int S>
__global__ __launch_bounds__(BLOCK) void export_kernel(ExportParams p) {
  using R = typename Storage<S>::R;
  __shared__ R stage[L::Q][BLOCK];
  const GridGeom& g = p.g;
  const SegInfo si = seg_info(g);
  if (si.seg >= g.nseg) return;
  const bool in = si.c.x < g.nx;
  const bool fluid = in && ((p.lk.seg_fluid[si.seg] >> si.lane) & 1ull);
  R h[L::Q];
  gather_state<L, S>(g, p.lk, p.src, si, fluid, h, stage);
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

template <class L, int S>
__global__ __launch_bounds__(BLOCK) void macros_kernel(MacroParams p) {
  using R = typename Storage<S>::R;
  __shared__ double sh[NPART][BLOCK];
  __shared__ R stage[L::Q][BLOCK];
  const GridGeom& g = p.g;
  const SegInfo si = seg_info(g);
  double v[NPART] = {0, 0, 0, 0, 0, 0, 0, 0};
  const bool seg_ok = si.seg < g.nseg;
  const bool in = seg_ok && si.c.x < g.nx;
  const bool fluid = in && ((p.lk.seg_fluid[si.seg] >> si.lane) & 1ull);
  R h[L::Q];
  if (seg_ok) gather_state<L, S>(g, p.lk, p.src, si, fluid, h, stage);
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
      const double* up = p.uprev + n * L::D;
      const double dx = ux - up[0], dy = uy - up[1], dz = L::D == 3 ? uz - up[2] : 0.0;
      v[0] = rho;
      v[1] = rho * ux;
      v[2] = rho * uy;
      v[3] = rho * uz;
      v[4] = dx * dx + dy * dy + dz * dz;
      v[5] = ux * ux + uy * uy + (L::D == 3 ? uz * uz : 0.0);
      v[6] = (isfinite(rho) && isfinite(ux) && isfinite(uy) && isfinite(uz)) ? 0.0 : 1.0;
      double* upw = p.uprev + n * L::D;
      upw[0] = ux;
      upw[1] = uy;
      if (L::D == 3) upw[2] = uz;
    }
    if (p.rho) p.rho[n] = rho;
    if (p.u) {
      p.u[n * L::D + 0] = ux;
      p.u[n * L::D + 1] = uy;
      if (L::D == 3) p.u[n * L::D + 2] = uz;
    }
  }
  block_sum_fixed(sh, v, threadIdx.x);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NPART; ++k) p.partials[blockIdx.x * NPART + k] = sh[k][0];
  }
}

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

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
int64_t grid_blocks(const GridGeom& g) {
  const int64_t b = (g.nseg + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
  return (b + 7) / 8 * 8;   // multiple of the XCD count, see logical_block()
}

#define LBM_DISPATCH(KERNEL, lattice, storage, grid, stream, params)                              \
  do {                                                                                            \
    if (lattice == LBM_D2Q9) {                                                                    \
      switch (storage) {                                                                          \
        case ST_F64: KERNEL<D2Q9, ST_F64><<<grid, BLOCK, 0, stream>>>(params); break;             \
        case ST_F32: KERNEL<D2Q9, ST_F32><<<grid, BLOCK, 0, stream>>>(params); break;             \
        case ST_F16S: KERNEL<D2Q9, ST_F16S><<<grid, BLOCK, 0, stream>>>(params); break;           \
        default: KERNEL<D2Q9, ST_BF16S><<<grid, BLOCK, 0, stream>>>(params); break;               \
      }                                                                                           \
    } else {                                                                                      \
      switch (storage) {                                                                          \
        case ST_F64: KERNEL<D3Q19, ST_F64><<<grid, BLOCK, 0, stream>>>(params); break;            \
        case ST_F32: KERNEL<D3Q19, ST_F32><<<grid, BLOCK, 0, stream>>>(params); break;            \
        case ST_F16S: KERNEL<D3Q19, ST_F16S><<<grid, BLOCK, 0, stream>>>(params); break;          \
        default: KERNEL<D3Q19, ST_BF16S><<<grid, BLOCK, 0, stream>>>(params); break;              \
      }                                                                                           \
    }                                                                                             \
  } while (0)

hipError_t launch_step(int lattice, int storage, const StepParams& p, hipStream_t s) {
  LBM_DISPATCH(step_kernel, lattice, storage, dim3((unsigned)grid_blocks(p.g)), s, p);
  return hipGetLastError();
}

hipError_t launch_init(int lattice, int storage, const InitParams& p, hipStream_t s) {
  LBM_DISPATCH(init_kernel, lattice, storage, dim3((unsigned)grid_blocks(p.g)), s, p);
  return hipGetLastError();
}

hipError_t launch_init_links(int lattice, int storage, const InitParams& p, hipStream_t s) {
  if (p.nlinks == 0 || p.lk.lv_out == nullptr) return hipSuccess;
  LBM_DISPATCH(init_links_kernel, lattice, storage, dim3((unsigned)((p.nlinks + BLOCK - 1) / BLOCK)), s, p);
  return hipGetLastError();
}

hipError_t launch_export(int lattice, int storage, const ExportParams& p, hipStream_t s) {
  LBM_DISPATCH(export_kernel, lattice, storage, dim3((unsigned)grid_blocks(p.g)), s, p);
  return hipGetLastError();
}

hipError_t launch_macros(int lattice, int storage, const MacroParams& p, int64_t nblocks, hipStream_t s) {
  LBM_DISPATCH(macros_kernel, lattice, storage, dim3((unsigned)nblocks), s, p);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int64_t nblocks, double* out, hipStream_t s) {
  reduce_kernel<<<1, BLOCK, 0, s>>>(partials, nblocks, out);
  return hipGetLastError();
}

}  // namespace lbm
