// HIP kernels for gfx950: fused pull collide-stream step with the ELIBB
// boundary (Sec. II.A-E), initialisation, state export and FP64 moments.
//
// One wavefront handles one segment of 64 consecutive x of a row (y, z); a block
// holds 4 segments, i.e. a whole 256-wide row for the 256^3 D3Q19 case.  Every
// population slot is read by exactly one lane (its consumer) and written by
// exactly one lane (its producer), so a step needs no synchronisation and no
// LDS: the work is Q coalesced loads + Q coalesced stores per fluid node, plus
// per cut link one q (and G) read and one store into the solid-side slot.
#include <hip/hip_runtime.h>

#include "elibb.hpp"
#include "internal.hpp"
#include "lattice.hpp"
#include "storage.hpp"

namespace lbm {

struct Coords {
  int x, y, z;
};

// Storage index of the pull source x - c_i (wrap on periodic axes; the halo
// layer of non-periodic axes absorbs the step outside the domain).
template <class L>
__device__ __forceinline__ int64_t src_index(const GridGeom& g, Coords c, int i) {
  int sx = c.x - L::cx(i), sy = c.y - L::cy(i), sz = c.z - L::cz(i);
  if (g.perx) sx = sx < 0 ? sx + g.nx : (sx >= g.nx ? sx - g.nx : sx);
  if (g.pery) sy = sy < 0 ? sy + g.ny : (sy >= g.ny ? sy - g.ny : sy);
  if (L::D == 3 && g.perz) sz = sz < 0 ? sz + g.nz : (sz >= g.nz ? sz - g.nz : sz);
  return (int64_t)(sx + g.px) + (int64_t)g.NX * ((int64_t)(sy + g.py) + (int64_t)g.NY * (sz + g.pz));
}

__device__ __forceinline__ int64_t self_index(const GridGeom& g, Coords c) {
  return (int64_t)(c.x + g.px) + (int64_t)g.NX * ((int64_t)(c.y + g.py) + (int64_t)g.NY * (c.z + g.pz));
}

// Segment of the calling wave and the lane's coordinates.
struct SegInfo {
  int64_t seg;
  int lane;
  Coords c;
};

__device__ __forceinline__ SegInfo seg_info(const GridGeom& g) {
  SegInfo s;
  s.lane = threadIdx.x & (SEG - 1);
  const int64_t wave = (int64_t)blockIdx.x * WAVES_PER_BLOCK + __builtin_amdgcn_readfirstlane(threadIdx.x / SEG);
  s.seg = wave;
  const int64_t row = wave / g.nseg_x;
  const int sx = (int)(wave - row * g.nseg_x);
  s.c.x = sx * SEG + s.lane;
  s.c.y = (int)(row % g.ny);
  s.c.z = (int)(row / g.ny);
  return s;
}

// Shifted equilibrium h^eq_i = f^eq_i - w_i = w_i [ (rho - 1) + rho (3 cu + 4.5 cu^2 - 1.5 uu) ]
// (eq. Eq2ndOrder with c_s^2 = 1/3); drho = rho - 1.
template <class L, typename R>
__device__ __forceinline__ R heq_dir(int i, R drho, R rho, R ux, R uy, R uz, R uu) {
  const R cu = R(L::cx(i)) * ux + R(L::cy(i)) * uy + R(L::cz(i)) * uz;
  return R(L::w(i)) * (drho + rho * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu));
}

// ---------------------------------------------------------------------------
// Fused step: pull, moments, BGK (+ Guo), store; then ELIBB for the node's cut
// links and the zero-gradient outlet copy.
// ---------------------------------------------------------------------------
template <class L, int S>
__global__ __launch_bounds__(BLOCK) void step_kernel(StepParams p) {
  using St = Storage<S>;
  using T = typename St::T;
  using R = typename St::R;
  const GridGeom& g = p.g;
  const SegInfo si = seg_info(g);
  if (si.seg >= g.nseg) return;
  const uint64_t fm = p.seg_fluid[si.seg];
  if (fm == 0) return;
  if (!((fm >> si.lane) & 1ull)) return;
  const Coords c = si.c;
  const T* __restrict__ src = static_cast<const T*>(p.src);
  T* __restrict__ dst = static_cast<T*>(p.dst);
  const int64_t np = g.npad;

  // shifted pre-collision populations h_i = f_i - w_i
  R h[L::Q];
#pragma unroll
  for (int i = 0; i < L::Q; ++i) h[i] = St::template load<L>(src + i * np + src_index<L>(g, c, i), i);

  R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    drho += h[i];
    if (L::cx(i)) jx += R(L::cx(i)) * h[i];
    if (L::cy(i)) jy += R(L::cy(i)) * h[i];
    if (L::cz(i)) jz += R(L::cz(i)) * h[i];
  }
  const R rho = R(1) + drho;
  const R Fx = R(p.force[0]), Fy = R(p.force[1]), Fz = R(p.force[2]);
  const R inv = R(1) / rho;
  const R ux = (jx + R(0.5) * Fx) * inv;
  const R uy = (jy + R(0.5) * Fy) * inv;
  const R uz = (jz + R(0.5) * Fz) * inv;
  const R uu = ux * ux + uy * uy + uz * uz;
  const R omega = R(p.omega);
  const R kf = R(1) - R(0.5) * omega;
  const R uF = ux * Fx + uy * Fy + uz * Fz;
  const bool force = p.has_force != 0;

  // post-collision h*_i: BGK (eq. LB-BGK) plus Guo's source term
  auto post = [&](int i) -> R {
    const R he = heq_dir<L, R>(i, drho, rho, ux, uy, uz, uu);
    R v = h[i] - omega * (h[i] - he);
    if (force) {
      const R cF = R(L::cx(i)) * Fx + R(L::cy(i)) * Fy + R(L::cz(i)) * Fz;
      const R cu = R(L::cx(i)) * ux + R(L::cy(i)) * uy + R(L::cz(i)) * uz;
      v += kf * R(L::w(i)) * (R(3) * (cF - uF) + R(9) * cu * cF);
    }
    return v;
  };

  const int64_t self = self_index(g, c);
#pragma unroll
  for (int i = 0; i < L::Q; ++i) St::template store<L>(dst + i * np + self, post(i), i);

  // ELIBB on the node's cut links (eq. ELIBB-general with the closed-form weights)
  const uint64_t bm = p.seg_bnd[si.seg];
  if ((bm >> si.lane) & 1ull) {
    const int b = p.seg_bbase[si.seg] + __popcll(bm & ((1ull << si.lane) - 1ull));
    const uint32_t mask = p.bmask[b];
    int li = p.blink[b];
    const R* __restrict__ lq = static_cast<const R*>(p.lq);
    const R* __restrict__ lg = static_cast<const R*>(p.lg);
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
      if ((mask >> i) & 1u) {
        const R q = lq[li];
        const Coef<R> a = elibb_coefficients<R>(p.variant, q, R(p.q_cut));
        const R gw = lg ? lg[li] : R(0);
        ++li;
        const int ib = L::opp(i);
        const R he_b = heq_dir<L, R>(ib, drho, rho, ux, uy, uz, uu);
        const R hs_b = post(ib);
        const R n_pre = h[ib] - he_b;        // bounced pre-collision non-equilibrium (eq. neqbb-s)
        const R n_post = hs_b - he_b;        // bounced post-collision non-equilibrium
        R v = a.a4 * n_pre + a.a5 * n_post + a.a2 * hs_b + R(L::w(i)) * (drho * (a.a4 + a.a5) + rho * gw);
        if (a.a3 != R(0)) v += a.a3 * post(i);
        St::template store<L>(dst + i * np + src_index<L>(g, c, i), v, i);
      }
    }
  }

  // zero-gradient outlet: the face-layer node writes its post-collision values of
  // the inward directions into the halo slot beyond the face, which its
  // neighbour along the face pulls.
  if (p.outlet_face >= 0) {
    const int f = p.outlet_face, a = f >> 1;
    const int sgn = (f & 1) ? 1 : -1;
    const int coord = a == 0 ? c.x : (a == 1 ? c.y : c.z);
    const int n_a = a == 0 ? g.nx : (a == 1 ? g.ny : g.nz);
    if (coord == (sgn > 0 ? n_a - 1 : 0)) {
      Coords halo = c;
      if (a == 0) halo.x += sgn;
      else if (a == 1) halo.y += sgn;
      else halo.z += sgn;
      const int64_t hidx = self_index(g, halo);
#pragma unroll
      for (int i = 1; i < L::Q; ++i) {
        const int ca = a == 0 ? L::cx(i) : (a == 1 ? L::cy(i) : L::cz(i));
        if (ca == -sgn) St::template store<L>(dst + i * np + hidx, post(i), i);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Initialisation / import: write the pre-collision state into the pull slots.
// ---------------------------------------------------------------------------
template <class L, int S>
__global__ __launch_bounds__(BLOCK) void init_kernel(InitParams p) {
  using St = Storage<S>;
  using T = typename St::T;
  using R = typename St::R;
  const GridGeom& g = p.g;
  const SegInfo si = seg_info(g);
  if (si.seg >= g.nseg) return;
  const uint64_t fm = p.seg_fluid[si.seg];
  if (!((fm >> si.lane) & 1ull)) return;
  const Coords c = si.c;
  T* dst = static_cast<T*>(p.dst);
  const int64_t n = c.x + (int64_t)g.nx * (c.y + (int64_t)g.ny * c.z);
  const int64_t N = (int64_t)g.nx * g.ny * g.nz;
  const double ux = p.u0[0], uy = p.u0[1], uz = p.u0[2];
  const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const double v = p.f_in ? p.f_in[i * N + n] - L::w(i) : heq_dir<L, double>(i, p.rho0 - 1.0, p.rho0, ux, uy, uz, uu);
    St::template store<L>(dst + i * g.npad + src_index<L>(g, c, i), R(v), i);
  }
}

// ---------------------------------------------------------------------------
// Export of the pre-collision state f_i(x, t) to [Q][N] float64.
// ---------------------------------------------------------------------------
template <class L, int S>
__global__ __launch_bounds__(BLOCK) void export_kernel(ExportParams p) {
  using St = Storage<S>;
  using T = typename St::T;
  const GridGeom& g = p.g;
  const SegInfo si = seg_info(g);
  if (si.seg >= g.nseg || si.c.x >= g.nx) return;
  const Coords c = si.c;
  const int64_t n = c.x + (int64_t)g.nx * (c.y + (int64_t)g.ny * c.z);
  const int64_t N = (int64_t)g.nx * g.ny * g.nz;
  const bool fluid = (p.seg_fluid[si.seg] >> si.lane) & 1ull;
  const T* src = static_cast<const T*>(p.src);
#pragma unroll
  for (int i = 0; i < L::Q; ++i)
    p.f_out[i * N + n] = fluid ? double(St::template load<L>(src + i * g.npad + src_index<L>(g, c, i), i)) + L::w(i) : 0.0;
}

// ---------------------------------------------------------------------------
// FP64 moments and fixed-order block partial sums.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_sum_fixed(double (*sh)[BLOCK], double* v, int tid) {
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
  using St = Storage<S>;
  using T = typename St::T;
  __shared__ double sh[NPART][BLOCK];
  const GridGeom& g = p.g;
  const SegInfo si = seg_info(g);
  double v[NPART] = {0, 0, 0, 0, 0, 0, 0, 0};
  const bool in = si.seg < g.nseg && si.c.x < g.nx;
  const bool fluid = in && ((p.seg_fluid[si.seg] >> si.lane) & 1ull);
  if (in) {
    const Coords c = si.c;
    const int64_t n = c.x + (int64_t)g.nx * (c.y + (int64_t)g.ny * c.z);
    double rho = 0.0, ux = 0.0, uy = 0.0, uz = 0.0;
    if (fluid) {
      const T* src = static_cast<const T*>(p.src);
      double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
      for (int i = 0; i < L::Q; ++i) {
        const double hi = double(St::template load<L>(src + i * g.npad + src_index<L>(g, c, i), i));
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
static inline dim3 grid_for(const GridGeom& g) {
  return dim3((unsigned)((g.nseg + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK));
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
  LBM_DISPATCH(step_kernel, lattice, storage, grid_for(p.g), s, p);
  return hipGetLastError();
}

hipError_t launch_init(int lattice, int storage, const InitParams& p, hipStream_t s) {
  LBM_DISPATCH(init_kernel, lattice, storage, grid_for(p.g), s, p);
  return hipGetLastError();
}

hipError_t launch_export(int lattice, int storage, const ExportParams& p, hipStream_t s) {
  LBM_DISPATCH(export_kernel, lattice, storage, grid_for(p.g), s, p);
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
