// C-ABI of liblbm: domain management, validation of the cut-link list, and the
// host side of the step / moments / state calls.  See include/lbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "elibb.hpp"
#include "error.hpp"
#include "internal.hpp"
#include "lattice.hpp"
#include "storage.hpp"

using namespace lbm;

namespace lbm {
thread_local std::string g_err;
std::atomic<uint64_t> g_uid{1};
uint64_t next_uid() { return g_uid.fetch_add(1); }
int set_error(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
void clear_error() { g_err.clear(); }
}  // namespace lbm

namespace {

int fail(int code, const std::string& msg) { return set_error(code, msg); }

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(LBM_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

struct Lat {
  int Q, D;
  int c[27][3];
  double w[27];
};

template <class L>
Lat make_lat() {
  Lat l{};
  l.Q = L::Q;
  l.D = L::D;
  for (int i = 0; i < L::Q; ++i) {
    l.c[i][0] = L::cx(i);
    l.c[i][1] = L::cy(i);
    l.c[i][2] = L::cz(i);
    l.w[i] = L::w(i);
  }
  return l;
}

const Lat& lat_of(int lattice) {
  static const Lat a = make_lat<D2Q9>(), b = make_lat<D3Q19>(), c = make_lat<D3Q27>();
  return lattice == LBM_D2Q9 ? a : (lattice == LBM_D3Q19 ? b : c);
}

template <typename P>
void dfree(P*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

template <typename P>
int dalloc(P*& p, size_t bytes) {
  void* q = nullptr;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE,
                                   std::string("hipMalloc: ") + hipGetErrorString(e));
  p = static_cast<P*>(q);
  return LBM_OK;
}

// The host planner's view of a domain's lattice and fluid mask.
HostGrid host_grid(const lbm_domain_s* d) {
  return make_host_grid(d->desc.lattice, d->g.nx, d->g.ny, d->g.nz, d->desc.periodic, d->desc.outlet_face,
                        d->mask.data());
}

// Device view of the links; lv_in / lv_out chosen by the caller.
LinkView link_view(const lbm_domain_s* d, const void* lv_in, void* lv_out) {
  LinkView lk{};
  lk.seg_fluid = d->seg_fluid;
  lk.seg_fbase = d->seg_fbase;
  lk.row_src = d->row_src;
  lk.seg_bnd = d->seg_bnd;
  lk.seg_lbase = d->seg_lbase;
  lk.lld = d->lld;
  lk.lnode = d->lnode;
  lk.lq = d->lq;
  lk.lg = d->lg;
  lk.lv_in = lv_in;
  lk.lv_out = lv_out;
  lk.luv = d->luv;
  lk.luv_stride = d->moving ? d->link_cap : d->nl;
  return lk;
}

}  // namespace

namespace lbm {

StepParams step_params(const lbm_domain_s* d, int cur) {
  StepParams p{};
  p.g = d->g;
  p.src = d->buf[cur];
  p.dst = d->buf[1 - cur];
  p.lk = link_view(d, d->lv[cur], d->lv[1 - cur]);
  p.omega = 1.0 / d->desc.tau;
  p.trt = d->desc.collision == LBM_TRT;
  // eq. magic-parameter: (1/omega+ - 1/2)(1/omega- - 1/2) = Lambda
  p.omega_minus = p.trt ? 1.0 / (d->desc.magic / (d->desc.tau - 0.5) + 0.5) : p.omega;
  for (int a = 0; a < 3; ++a) p.force[a] = d->desc.force[a];
  p.src_eq = 3.0 * (1.0 - 0.5 * p.omega) / p.omega;
  p.src_eq_minus = 3.0 * (1.0 - 0.5 * p.omega_minus) / p.omega_minus;
  p.has_force = (d->desc.force[0] != 0.0 || d->desc.force[1] != 0.0 || d->desc.force[2] != 0.0);
  p.variant = d->variant;
  p.q_cut = d->q_cut;
  p.outlet_face = d->desc.outlet_face;
  p.rng_ctr = d->rng_ctr;
  p.parity = cur;
  p.wall_neq = d->wall_neq;
  p.omega_f = (float)p.omega;
  p.omega_minus_f = (float)p.omega_minus;
  for (int a = 0; a < 3; ++a) p.force_f[a] = (float)p.force[a];
  p.src_eq_f = (float)p.src_eq;
  p.src_eq_minus_f = (float)p.src_eq_minus;
  p.q_cut_f = (float)p.q_cut;
  return p;
}

// Kinematics of the moving spheres for the geometry of time t: the sinusoid's
// centre x0 + A sin(2 pi t / T) e and velocity at t and t + 1 (one sphere), or
// the samples of prescribed paths; angular velocities at t and t + 1
// (constant unless sampled).
MovingKin moving_kin(const lbm_domain_s* d, int64_t t) {
  MovingKin k{};
  const int ns = d->mv_ns;
  k.ns = ns;
  for (int sp = 0; sp < ns; ++sp) k.r[sp] = d->mv_r[sp];
  for (int a = 0; a < 3; ++a) k.Om[0][a] = k.Om1[0][a] = d->mv_om[a];
  if (!d->path_c.empty()) {
    // sampled paths ([n][ns][3]): the geometry of time t needs x_c(t), V(t),
    // V(t+1) and, when sampled, Omega(t), Omega(t+1); a time past the path
    // (only in rows of a kinematics table that no step uses) takes its last
    // pair of samples
    const int64_t n = (int64_t)d->path_c.size() / (3 * ns);
    const int64_t tt = std::min<int64_t>(std::max<int64_t>(t, 0), n - 2);
    for (int sp = 0; sp < ns; ++sp) {
      const size_t o0 = 3 * ((size_t)tt * ns + sp), o1 = 3 * ((size_t)(tt + 1) * ns + sp);
      for (int a = 0; a < 3; ++a) {
        k.c[sp][a] = d->path_c[o0 + a];
        k.V[sp][a] = d->path_v[o0 + a];
        k.V1[sp][a] = d->path_v[o1 + a];
        if (!d->path_om.empty()) {
          k.Om[sp][a] = d->path_om[o0 + a];
          k.Om1[sp][a] = d->path_om[o1 + a];
        }
      }
      if (d->D == 2) k.c[sp][2] = k.V[sp][2] = k.V1[sp][2] = 0.0;
    }
    return k;
  }
  const double two_pi = 2.0 * M_PI;
  const double s = std::sin(two_pi * t / d->mv_period);
  const double c0 = std::cos(two_pi * t / d->mv_period), c1 = std::cos(two_pi * (t + 1) / d->mv_period);
  const double vamp = d->mv_amp * (two_pi / d->mv_period);
  for (int a = 0; a < 3; ++a) {
    k.c[0][a] = d->mv_x0[a] + d->mv_amp * s * d->mv_dir[a];
    k.V[0][a] = vamp * c0 * d->mv_dir[a];
    k.V1[0][a] = vamp * c1 * d->mv_dir[a];
  }
  if (d->D == 2) k.c[0][2] = k.V[0][2] = k.V1[0][2] = 0.0;
  return k;
}

// Steps a domain whose spheres follow sampled paths can still take: the
// geometry of time t uses the samples t and t+1.
int64_t path_steps_left(const lbm_domain_s* d) {
  if (d->path_c.empty()) return INT64_MAX;
  return (int64_t)d->path_c.size() / (3 * d->mv_ns) - 2 - d->steps;
}

// Static part of the moving-sphere rebuild; `cur` names the population buffer
// that holds the state the fresh nodes are refilled in.
MovingParams moving_params(const lbm_domain_s* d, int cur) {
  MovingParams mp{};
  mp.g = d->g;
  mp.variant = d->variant;
  mp.q_cut = d->q_cut;
  mp.reg_seg = d->reg_seg;
  mp.nreg = d->nreg;
  mp.seg_fluid = d->seg_fluid;
  mp.seg_prev = d->seg_prev;
  mp.seg_bnd = d->seg_bnd;
  mp.reg_count = d->reg_count;
  mp.reg_cut = d->reg_cut;
  mp.seg_lbase = d->seg_lbase;
  mp.lld = d->lld;
  mp.lq = d->lq;
  mp.lg = d->lg;
  mp.luv = d->luv;
  mp.luv_stride = d->link_cap;
  mp.pop = d->buf[cur];
  mp.rho0 = d->desc.rho0;
  return mp;
}

}  // namespace lbm

namespace {

// Export the current state to a device [Q][N] float64 buffer.
hipError_t export_state(lbm_domain_s* d, double* dev_f) {
  ExportParams p{};
  p.g = d->g;
  p.src = d->buf[d->cur];
  p.lk = link_view(d, d->lv[d->cur], nullptr);
  p.f_out = dev_f;
  return launch_export(d->desc.lattice, d->desc.storage, p, d->stream);
}

// Import a state from a device [Q][N] float64 buffer (null: the equilibrium of
// rho0, u0) into the pull slots and the current link values.
hipError_t import_state(lbm_domain_s* d, const double* dev_f) {
  InitParams ip{};
  ip.g = d->g;
  ip.dst = d->buf[d->cur];
  ip.lk = link_view(d, nullptr, d->lv[d->cur]);
  ip.nlinks = d->nl;
  ip.f_in = dev_f;
  ip.rho0 = d->desc.rho0;
  for (int a = 0; a < 3; ++a) ip.u0[a] = d->desc.u0[a];
  hipError_t e = launch_init(d->desc.lattice, d->desc.storage, ip, d->stream);
  if (e == hipSuccess) e = launch_init_links(d->desc.lattice, d->desc.storage, ip, d->stream);
  d->state_step = d->steps;
  return e;
}

// Geometry of the moving sphere at time t on the device (classify, link prefix,
// links, and with `refill` the fresh nodes of the current state).
hipError_t rebuild_moving(lbm_domain_s* d, int64_t t, bool refill) {
  MovingParams mp = moving_params(d, d->cur);
  mp.k = moving_kin(d, t);
  hipError_t e = launch_moving_classify(d->desc.lattice, mp, d->stream);
  if (e == hipSuccess) e = launch_region_scan(mp, d->stream);
  if (e == hipSuccess) e = launch_moving_fill(d->desc.lattice, d->desc.storage, mp, d->stream);
  if (e == hipSuccess && refill) e = launch_moving_refill(d->desc.lattice, d->desc.storage, mp, d->stream);
  return e;
}

void free_links(lbm_domain_s* d) {
  dfree(d->lld);
  dfree(d->lnode);
  dfree(d->lv[0]);
  dfree(d->lv[1]);
  dfree(d->lq);
  dfree(d->lg);
  dfree(d->luv);
  dfree(d->luw);
  dfree(d->lgrp);
  dfree(d->lforce);
  dfree(d->gforce);
  d->link_order.clear();
  d->n_groups = 1;
  d->nb = d->nl = 0;
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return lbm::g_err.c_str(); }

namespace {
// Elements per direction array: compact = the guard in front, the fluid nodes
// and one guard slot behind, rounded up to 64 elements; dense = the padded
// lattice.
int64_t population_stride(const lbm_domain_desc* d, const uint8_t* mask) {
  const int64_t NX = d->nx + ((d->periodic & 1) ? 0 : 2);
  const int64_t NY = d->ny + ((d->periodic & 2) ? 0 : 2);
  const int64_t NZ = d->lattice == LBM_D2Q9 ? 1 : d->nz + ((d->periodic & 4) ? 0 : 2);
  if (d->layout == LBM_LAYOUT_DENSE || !mask) return NX * NY * NZ;
  const int64_t N = (int64_t)d->nx * d->ny * d->nz;
  int64_t nf = 0;
  for (int64_t n = 0; n < N; ++n) nf += mask[n] ? 1 : 0;
  return (GUARD + nf + 1 + 63) / 64 * 64;
}
}  // namespace

size_t lbm_arena_bytes(const lbm_domain_desc* d, const uint8_t* fluid_mask) {
  if (!d || (d->lattice != LBM_D2Q9 && d->lattice != LBM_D3Q19 && d->lattice != LBM_D3Q27)) return 0;
  const int Q = d->lattice == LBM_D2Q9 ? 9 : (d->lattice == LBM_D3Q19 ? 19 : 27);
  const size_t one = (size_t)population_stride(d, fluid_mask) * Q * storage_bytes(d->storage);
  const size_t aligned = (one + 255) / 256 * 256;
  return 2 * aligned;
}

int lbm_init_domain(const lbm_domain_desc* desc, const uint8_t* fluid_mask, lbm_domain* out) {
  if (!desc || !fluid_mask || !out) return fail(LBM_EINVAL, "null argument");
  const lbm_domain_desc& d = *desc;
  if (d.lattice != LBM_D2Q9 && d.lattice != LBM_D3Q19 && d.lattice != LBM_D3Q27)
    return fail(LBM_EINVAL, "lattice must be LBM_D2Q9, LBM_D3Q19 or LBM_D3Q27");
  if (d.nx < 1 || d.ny < 1 || d.nz < 1) return fail(LBM_EINVAL, "nx, ny, nz must be >= 1");
  if (d.lattice == LBM_D2Q9 && d.nz != 1) return fail(LBM_EINVAL, "nz must be 1 for D2Q9");
  if (d.storage < LBM_F64 || d.storage > LBM_BF16_SHIFTED) return fail(LBM_EINVAL, "invalid storage");
  if (!(d.tau > 0.5) || !std::isfinite(d.tau)) return fail(LBM_EINVAL, "tau must be finite and > 0.5");
  if (!(d.rho0 > 0.0) || !std::isfinite(d.rho0)) return fail(LBM_EINVAL, "rho0 must be finite and > 0");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(d.force[a]) || !std::isfinite(d.u0[a])) return fail(LBM_EINVAL, "non-finite force or u0");
  if (d.lattice == LBM_D2Q9 && (d.force[2] != 0.0 || d.u0[2] != 0.0)) return fail(LBM_EINVAL, "z components must be 0 for D2Q9");
  int per = d.periodic;
  if (d.lattice == LBM_D2Q9) per |= 4;
  if (d.outlet_face < -1 || d.outlet_face > 5) return fail(LBM_EINVAL, "outlet_face out of range");
  if (d.outlet_face >= 0 && ((per >> (d.outlet_face >> 1)) & 1)) return fail(LBM_EINVAL, "outlet face lies on a periodic axis");
  const int64_t N = (int64_t)d.nx * d.ny * d.nz;
  if (d.layout != LBM_LAYOUT_COMPACT && d.layout != LBM_LAYOUT_DENSE) return fail(LBM_EINVAL, "invalid layout");
  if (d.collision != LBM_BGK && d.collision != LBM_TRT) return fail(LBM_EINVAL, "collision must be LBM_BGK or LBM_TRT");
  if (d.collision == LBM_TRT && !(d.magic > 0.0 && std::isfinite(d.magic)))
    return fail(LBM_EINVAL, "TRT magic parameter must be finite and > 0");
  if (d.rounding != LBM_ROUND_NEAREST && d.rounding != LBM_ROUND_STOCHASTIC)
    return fail(LBM_EINVAL, "rounding must be LBM_ROUND_NEAREST or LBM_ROUND_STOCHASTIC");
  if (d.rounding == LBM_ROUND_STOCHASTIC && d.storage != LBM_F16_SHIFTED && d.storage != LBM_BF16_SHIFTED)
    return fail(LBM_EINVAL, "stochastic rounding needs a 16-bit storage");
  // the kernels index populations and segments with 32-bit integers; checked
  // before any device call
  const int64_t npad = population_stride(desc, fluid_mask);
  const int64_t nseg = (int64_t)((d.nx + SEG - 1) / SEG) * d.ny * d.nz;
  if (npad >= ((int64_t)1 << 31) || nseg >= ((int64_t)1 << 31) / WAVES_PER_BLOCK)
    return fail(LBM_EINVAL, "lattice too large: more than 2^31 stored nodes");
  const size_t need = lbm_arena_bytes(desc, fluid_mask);
  if (d.arena && d.arena_bytes < need) return fail(LBM_EINVAL, "arena too small: need " + std::to_string(need) + " bytes");
  if (d.arena && ((uintptr_t)d.arena & 255)) return fail(LBM_EINVAL, "arena must be 256-byte aligned");

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(LBM_EDEVICE, "no HIP device");

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(LBM_EDEVICE, "no current HIP device");
  // per-device set-up of the no-allocation entry point's scratch address; a
  // failure only disables lbm_macros_noalloc (it reports the error)
  (void)noalloc_setup(dev);
  auto* dm = new lbm_domain_s();   // value-initialised: every pointer null, counters 0
  dm->desc = d;
  dm->device = dev;
  dm->desc.periodic = per;
  const Lat& L = lat_of(d.lattice);
  dm->Q = L.Q;
  dm->D = L.D;
  GridGeom& g = dm->g;
  g.nx = d.nx;
  g.ny = d.ny;
  g.nz = d.nz;
  g.perx = per & 1;
  g.pery = (per >> 1) & 1;
  g.perz = (per >> 2) & 1;
  g.px = g.perx ? 0 : 1;
  g.py = g.pery ? 0 : 1;
  g.pz = g.perz ? 0 : 1;
  g.NX = g.nx + 2 * g.px;
  g.NY = g.ny + 2 * g.py;
  g.NZ = g.nz + 2 * g.pz;
  g.nseg_x = (g.nx + SEG - 1) / SEG;
  g.nseg = (int64_t)g.nseg_x * g.ny * g.nz;
  g.guard = GUARD;
  g.div_nseg_x = make_fastdiv((uint32_t)g.nseg_x);
  g.div_ny = make_fastdiv((uint32_t)g.ny);
  g.xcd_remap = 0;
  g.compact = d.layout == LBM_LAYOUT_COMPACT;
  g.outlet = d.outlet_face;
  g.xcd_remap = g.compact ? 1 : 0;
  g.npad = npad;
  dm->N = N;
  dm->elem = storage_bytes(d.storage);
  dm->skind = d.rounding == LBM_ROUND_STOCHASTIC ? (d.storage == LBM_F16_SHIFTED ? ST_F16SR : ST_BF16SR) : d.storage;
  dm->stream = static_cast<hipStream_t>(d.stream);
  dm->variant = LBM_ELIBB_FQ;
  dm->q_cut = 0.01;
  dm->mask.assign(fluid_mask, fluid_mask + N);
  for (auto& v : dm->mask) v = v ? 1 : 0;
  dm->n_fluid = std::accumulate(dm->mask.begin(), dm->mask.end(), (int64_t)0);

  auto cleanup = [&](int code) {
    lbm_free_domain(dm);
    return code;
  };
  const size_t one = need / 2;
  if (d.arena) {
    dm->buf[0] = d.arena;
    dm->buf[1] = static_cast<char*>(d.arena) + one;
    dm->own_buf = false;
  } else {
    dm->own_buf = true;
    if (int e = dalloc(dm->buf[0], one)) return cleanup(e);
    if (int e = dalloc(dm->buf[1], one)) return cleanup(e);
  }
  hipError_t he = hipMemsetAsync(dm->buf[0], 0, one, dm->stream);
  if (he == hipSuccess) he = hipMemsetAsync(dm->buf[1], 0, one, dm->stream);
  if (he != hipSuccess) return cleanup(fail(LBM_EDEVICE, std::string("hipMemsetAsync: ") + hipGetErrorString(he)));

  // segment masks
  std::vector<uint64_t> sf;
  std::vector<int32_t> sfb;
  segment_index(host_grid(dm), sf, sfb);
  if (int e = dalloc(dm->seg_fbase, (g.nseg + 1) * 4)) return cleanup(e);
  if (int e = dalloc(dm->seg_fluid, g.nseg * 8)) return cleanup(e);
  if (int e = dalloc(dm->seg_bnd, g.nseg * 8)) return cleanup(e);
  if (int e = dalloc(dm->seg_lbase, (g.nseg + 1) * 4)) return cleanup(e);
  he = hipMemcpy(dm->seg_fluid, sf.data(), g.nseg * 8, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(dm->seg_fbase, sfb.data(), (g.nseg + 1) * 4, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemsetAsync(dm->seg_bnd, 0, g.nseg * 8, dm->stream);
  if (he == hipSuccess) he = hipMemsetAsync(dm->seg_lbase, 0, (g.nseg + 1) * 4, dm->stream);
  if (he != hipSuccess) return cleanup(fail(LBM_EDEVICE, std::string("upload: ") + hipGetErrorString(he)));
  if (g.compact) {
    std::vector<int32_t> rows;
    source_rows(host_grid(dm), rows);
    if (int e = dalloc(dm->row_src, rows.size() * 4)) return cleanup(e);
    he = hipMemcpy(dm->row_src, rows.data(), rows.size() * 4, hipMemcpyHostToDevice);
    if (he != hipSuccess) return cleanup(fail(LBM_EDEVICE, std::string("upload: ") + hipGetErrorString(he)));
  }

  // step count of the stochastic rounding, one entry per buffer parity
  if (int e = dalloc(dm->rng_ctr, 2 * sizeof(uint32_t))) return cleanup(e);
  he = hipMemsetAsync(dm->rng_ctr, 0, 2 * sizeof(uint32_t), dm->stream);
  if (he != hipSuccess) return cleanup(fail(LBM_EDEVICE, std::string("hipMemsetAsync: ") + hipGetErrorString(he)));

  // reductions and the velocity snapshot of the residual
  dm->red_blocks = grid_blocks(g);
  if (int e = dalloc(dm->partials, dm->red_blocks * NPART * 8)) return cleanup(e);
  if (int e = dalloc(dm->sums, NPART * 8)) return cleanup(e);
  dm->uprev = nullptr;   // the residual's snapshot is allocated by the first lbm_macros call

  dm->cur = 0;
  he = import_state(dm, nullptr);
  if (he != hipSuccess) return cleanup(fail(LBM_EDEVICE, std::string("init kernel: ") + hipGetErrorString(he)));
  dm->cur = 0;
  int bad_dir = 0;
  dm->links_ok = first_uncovered(host_grid(dm), {}, &bad_dir) < 0;
  dm->n_groups = 1;
  dm->uid = next_uid();
  *out = dm;
  clear_error();
  return LBM_OK;
}

int lbm_set_boundary_links(lbm_domain d, int64_t n_links, const int64_t* node, const int8_t* dir, const double* q,
                           const double* uw_t, const double* uw_t1, int32_t variant, double q_cutoff) {
  if (!d) return fail(LBM_EINVAL, "null domain");
  const bool f64 = d->desc.storage == LBM_F64;
  LinkPlan plan;
  if (int e = plan_links(host_grid(d), n_links, node, dir, q, uw_t, uw_t1, variant, q_cutoff, f64, plan)) return e;
  const GridGeom& g = d->g;
  const int64_t N = d->N;
  const bool moving = plan.moving;
  // the current state (pulled with the old links) survives the replacement; a
  // domain still in its initial state is simply initialised again
  const bool initial = d->steps == 0 && !d->state_set;
  double* fstate = nullptr;
  if (!initial) {
    if (int e = dalloc(fstate, (size_t)N * d->Q * 8)) return e;
    if (hipError_t he = export_state(d, fstate); he != hipSuccess) {
      (void)hipFree(fstate);
      return fail(LBM_EDEVICE, std::string("export: ") + hipGetErrorString(he));
    }
  }
  // upload (replace previous arrays)
  HIP_TRY(hipStreamSynchronize(d->stream));
  free_links(d);
  d->links_ok = false;
  const size_t rs = f64 ? 8 : 4;
  auto up = [&]() -> int {
    if (int e = dalloc(d->lld, plan.lld.size() * 2)) return e;
    if (int e = dalloc(d->lnode, plan.lnode.size() * 4)) return e;
    if (int e = dalloc(d->lq, plan.q.size() * rs)) return e;
    if (int e = dalloc(d->lv[0], plan.q.size() * rs)) return e;
    if (int e = dalloc(d->lv[1], plan.q.size() * rs)) return e;
    if (moving) {
      if (int e = dalloc(d->lg, plan.gw.size() * rs)) return e;
      if (int e = dalloc(d->luv, plan.uv.size() * rs)) return e;
    }
    HIP_TRY(hipMemcpy(d->lld, plan.lld.data(), plan.lld.size() * 2, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d->lnode, plan.lnode.data(), plan.lnode.size() * 4, hipMemcpyHostToDevice));
    auto upload_real = [&](void* dst, const std::vector<double>& v) -> hipError_t {
      if (f64) return hipMemcpy(dst, v.data(), v.size() * 8, hipMemcpyHostToDevice);
      std::vector<float> f(v.begin(), v.end());
      return hipMemcpy(dst, f.data(), f.size() * 4, hipMemcpyHostToDevice);
    };
    HIP_TRY(upload_real(d->lq, plan.q));
    if (moving) {
      HIP_TRY(upload_real(d->lg, plan.gw));
      // u_w(t) and u_w(t+1) of every stored link, [6][nl] (regularised wall non-equilibrium)
      HIP_TRY(upload_real(d->luv, plan.uv));
    }
    HIP_TRY(hipMemcpy(d->seg_bnd, plan.seg_bnd.data(), g.nseg * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d->seg_lbase, plan.seg_lbase.data(), (g.nseg + 1) * 4, hipMemcpyHostToDevice));
    // wall velocities at t, for the momentum-exchange force (only when a wall moves)
    if (plan.uw_any) {
      if (int e = dalloc(d->luw, plan.uw.size() * 8)) return e;
      HIP_TRY(hipMemcpy(d->luw, plan.uw.data(), plan.uw.size() * 8, hipMemcpyHostToDevice));
    }
    d->nb = plan.n_boundary;
    d->nl = n_links;
    HIP_TRY(import_state(d, fstate));
    HIP_TRY(hipStreamSynchronize(d->stream));
    return LBM_OK;
  };
  const int code = up();
  if (fstate) (void)hipFree(fstate);
  if (code != LBM_OK) return code;
  d->link_order = std::move(plan.order);
  d->links_step = d->steps;
  d->nl = n_links;
  d->variant = variant;
  d->q_cut = q_cutoff;
  d->links_ok = true;
  d->uid = next_uid();
  clear_error();
  return LBM_OK;
}

int lbm_set_wall_neq(lbm_domain d, int32_t mode) {
  if (!d) return fail(LBM_EINVAL, "null domain");
  if (mode != LBM_NEQ_BOUNCEBACK && mode != LBM_NEQ_REGULARIZED)
    return fail(LBM_EINVAL, "invalid wall non-equilibrium mode " + std::to_string(mode));
  if (d->moving) return fail(LBM_ESTATE, "choose the wall non-equilibrium before lbm_set_moving_sphere");
  if (mode != d->wall_neq) {
    d->wall_neq = mode;
    d->uid = next_uid();   // batches rebuild their tables
  }
  clear_error();
  return LBM_OK;
}

namespace {
// Common set-up of a moving sphere whose centre stays within [lo, hi] per axis:
// checks, the sweep region's segments, the link arrays, the geometry of time 0
// and the initial state.  The motion itself (sinusoid or sampled path) is set
// on the domain by the caller beforehand.
int install_moving(lbm_domain d, int ns, const double (*lo_c)[3], const double (*hi_c)[3], const double* radius,
                   const double omega[3], int32_t variant, double q_cutoff) {
  if (variant < LBM_ELIBB_FQ || variant > LBM_HWBB) return fail(LBM_EINVAL, "invalid variant");
  if (!(q_cutoff >= 0.0) || !std::isfinite(q_cutoff)) return fail(LBM_EINVAL, "q_cutoff must be finite and >= 0");
  if (d->g.compact) return fail(LBM_ESTATE, "a moving sphere needs the dense layout (desc.layout = LBM_LAYOUT_DENSE)");
  if (d->desc.outlet_face >= 0) return fail(LBM_ESTATE, "a moving sphere needs a domain without outlet");
  if (d->steps != 0 || d->moving || d->nl != 0) return fail(LBM_ESTATE, "set the moving sphere once, on a fresh domain without links");
  if (d->n_fluid != d->N) return fail(LBM_ESTATE, "the domain's initial mask must be all fluid");
  const GridGeom& g = d->g;
  if (!(g.perx && g.pery && g.perz)) return fail(LBM_ESTATE, "a moving sphere needs a fully periodic box");
  const int n3[3] = {g.nx, g.ny, d->D == 3 ? g.nz : 1 << 30};
  for (int sp = 0; sp < ns; ++sp)
    for (int a = 0; a < 3; ++a)
      if (2.0 * (radius[sp] + 0.5 * (hi_c[sp][a] - lo_c[sp][a]) + 2.0) >= n3[a])
        return fail(LBM_EINVAL, "each sphere and its sweep must fit in half the box on every axis");
  // the region: segments of the boxes swept by the spheres (plus two nodes)
  std::vector<char> in_seg(g.nseg, 0);
  const int n[3] = {g.nx, g.ny, g.nz}, per[3] = {g.perx, g.pery, g.perz};
  for (int sp = 0; sp < ns; ++sp) {
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = (int)std::floor(lo_c[sp][a] - radius[sp]) - 2;
      hi[a] = (int)std::ceil(hi_c[sp][a] + radius[sp]) + 2;
      if (d->D == 2 && a == 2) lo[a] = hi[a] = 0;
      if (hi[a] - lo[a] + 1 >= n[a]) {
        lo[a] = 0;
        hi[a] = n[a] - 1;
      } else if (!per[a]) {
        lo[a] = std::max(lo[a], 0);
        hi[a] = std::min(hi[a], n[a] - 1);
      }
    }
    for (int zz = lo[2]; zz <= hi[2]; ++zz)
      for (int yy = lo[1]; yy <= hi[1]; ++yy)
        for (int xx = lo[0]; xx <= hi[0]; xx += 1) {
          const int x = ((xx % n[0]) + n[0]) % n[0], y = ((yy % n[1]) + n[1]) % n[1], z = ((zz % n[2]) + n[2]) % n[2];
          in_seg[(x / SEG) + (int64_t)g.nseg_x * (y + (int64_t)g.ny * z)] = 1;
        }
  }
  std::vector<int32_t> reg;
  for (int64_t s2 = 0; s2 < g.nseg; ++s2)
    if (in_seg[s2]) reg.push_back((int32_t)s2);
  free_links(d);
  const size_t rs = d->desc.storage == LBM_F64 ? 8 : 4;
  d->nreg = (int64_t)reg.size();
  d->link_cap = d->nreg * SEG * (d->Q - 1);
  if (int e = dalloc(d->reg_seg, reg.size() * 4)) return e;
  if (int e = dalloc(d->seg_prev, g.nseg * 8)) return e;
  if (int e = dalloc(d->reg_count, reg.size() * 4)) return e;
  if (int e = dalloc(d->reg_cut, reg.size() * SEG * 4)) return e;
  if (int e = dalloc(d->lld, d->link_cap * 2)) return e;
  if (int e = dalloc(d->lq, d->link_cap * rs)) return e;
  if (int e = dalloc(d->lg, d->link_cap * rs)) return e;
  if (d->wall_neq == LBM_NEQ_REGULARIZED)
    if (int e = dalloc(d->luv, 6 * d->link_cap * rs)) return e;
  HIP_TRY(hipMemcpy(d->reg_seg, reg.data(), reg.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d->seg_prev, d->seg_fluid, g.nseg * 8, hipMemcpyDeviceToDevice));
  HIP_TRY(hipMemset(d->reg_count, 0, reg.size() * 4));
  for (int a = 0; a < 3; ++a) d->mv_om[a] = omega[a];
  d->mv_ns = ns;
  for (int sp = 0; sp < ns; ++sp) d->mv_r[sp] = radius[sp];
  d->variant = variant;
  d->q_cut = q_cutoff;
  d->moving = true;
  HIP_TRY(rebuild_moving(d, 0, false));
  HIP_TRY(import_state(d, nullptr));
  HIP_TRY(hipStreamSynchronize(d->stream));
  d->links_ok = true;
  d->uid = next_uid();
  clear_error();
  return LBM_OK;
}
}  // namespace

int lbm_set_moving_sphere(lbm_domain d, const double x0[3], double radius, double amplitude, double period,
                          const double direction[3], const double omega[3], int32_t variant, double q_cutoff) {
  if (!d || !x0 || !direction || !omega) return fail(LBM_EINVAL, "null argument");
  if (!(radius > 0.0) || !(period > 0.0) || !(amplitude >= 0.0)) return fail(LBM_EINVAL, "radius, period must be > 0, amplitude >= 0");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(x0[a]) || !std::isfinite(direction[a]) || !std::isfinite(omega[a])) return fail(LBM_EINVAL, "non-finite motion");
  if (d->moving) return fail(LBM_ESTATE, "set the moving sphere once, on a fresh domain without links");
  double lo_c[1][3], hi_c[1][3];
  for (int a = 0; a < 3; ++a) {
    const double ext = std::fabs(amplitude * direction[a]);
    lo_c[0][a] = x0[a] - ext;
    hi_c[0][a] = x0[a] + ext;
    d->mv_x0[a] = x0[a];
    d->mv_dir[a] = direction[a];
  }
  d->mv_amp = amplitude;
  d->mv_period = period;
  d->path_c.clear();
  d->path_v.clear();
  d->path_om.clear();
  return install_moving(d, 1, lo_c, hi_c, &radius, omega, variant, q_cutoff);
}

namespace {
// Spheres on sampled paths: centres and velocities per step ([n][ns][3]),
// angular velocity constant (omega, one sphere) or per step (omega_path,
// [n][ns][3]).
int set_moving_paths(lbm_domain d, int ns, const double* radius, const double* omega, const double* omega_path,
                     int64_t n_samples, const double* centre, const double* velocity, int32_t variant,
                     double q_cutoff) {
  if (ns < 1 || ns > MAX_SPHERES)
    return fail(LBM_EINVAL, "between 1 and " + std::to_string(MAX_SPHERES) + " spheres per domain");
  for (int sp = 0; sp < ns; ++sp)
    if (!(radius[sp] > 0.0) || !std::isfinite(radius[sp])) return fail(LBM_EINVAL, "radius must be finite and > 0");
  if (n_samples < 2) return fail(LBM_EINVAL, "a path needs at least 2 samples");
  if (omega)
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(omega[a])) return fail(LBM_EINVAL, "non-finite omega");
  const int64_t nv = 3 * n_samples * ns;
  for (int64_t k = 0; k < nv; ++k)
    if (!std::isfinite(centre[k]) || !std::isfinite(velocity[k]) || (omega_path && !std::isfinite(omega_path[k])))
      return fail(LBM_EINVAL, "non-finite path sample " + std::to_string(k / (3 * ns)));
  if (d->moving) return fail(LBM_ESTATE, "set the moving sphere once, on a fresh domain without links");
  // spheres keep apart: at every sample the surfaces are more than two nodes apart
  // (minimum image on the periodic axes)
  const int n3[3] = {d->g.nx, d->g.ny, d->g.nz};
  for (int64_t k = 0; k < n_samples; ++k)
    for (int a = 0; a < ns; ++a)
      for (int b = a + 1; b < ns; ++b) {
        double dd = 0.0;
        for (int x = 0; x < 3; ++x) {
          double v = centre[3 * (k * ns + a) + x] - centre[3 * (k * ns + b) + x];
          if (d->D == 2 && x == 2) v = 0.0;
          v -= n3[x] * std::nearbyint(v / n3[x]);
          dd += v * v;
        }
        if (!(std::sqrt(dd) > radius[a] + radius[b] + 2.0))
          return fail(LBM_EINVAL, "spheres " + std::to_string(a) + " and " + std::to_string(b) +
                                      " come within two nodes of each other at sample " + std::to_string(k));
      }
  double lo_c[MAX_SPHERES][3], hi_c[MAX_SPHERES][3];
  for (int sp = 0; sp < ns; ++sp)
    for (int a = 0; a < 3; ++a) {
      lo_c[sp][a] = hi_c[sp][a] = centre[3 * sp + a];
      for (int64_t k = 1; k < n_samples; ++k) {
        lo_c[sp][a] = std::min(lo_c[sp][a], centre[3 * (k * ns + sp) + a]);
        hi_c[sp][a] = std::max(hi_c[sp][a], centre[3 * (k * ns + sp) + a]);
      }
    }
  d->path_c.assign(centre, centre + nv);
  d->path_v.assign(velocity, velocity + nv);
  if (omega_path) d->path_om.assign(omega_path, omega_path + nv);
  else d->path_om.clear();
  d->mv_ns = ns;
  const double zero[3] = {0.0, 0.0, 0.0};
  const int e = install_moving(d, ns, lo_c, hi_c, radius, omega ? omega : zero, variant, q_cutoff);
  if (e != LBM_OK && !d->moving) {
    d->path_c.clear();
    d->path_v.clear();
    d->path_om.clear();
    d->mv_ns = 1;
  }
  return e;
}
}  // namespace

int lbm_set_moving_sphere_path(lbm_domain d, double radius, const double omega[3], int64_t n_samples,
                               const double* centre, const double* velocity, int32_t variant, double q_cutoff) {
  if (!d || !omega || !centre || !velocity) return fail(LBM_EINVAL, "null argument");
  return set_moving_paths(d, 1, &radius, omega, nullptr, n_samples, centre, velocity, variant, q_cutoff);
}

int lbm_set_moving_sphere_motion(lbm_domain d, double radius, int64_t n_samples, const double* centre,
                                 const double* velocity, const double* omega, int32_t variant, double q_cutoff) {
  if (!d || !omega || !centre || !velocity) return fail(LBM_EINVAL, "null argument");
  return set_moving_paths(d, 1, &radius, nullptr, omega, n_samples, centre, velocity, variant, q_cutoff);
}

int lbm_set_moving_spheres(lbm_domain d, int32_t n_spheres, const double* radius, int64_t n_samples,
                           const double* centre, const double* velocity, const double* omega, int32_t variant,
                           double q_cutoff) {
  if (!d || !radius || !omega || !centre || !velocity) return fail(LBM_EINVAL, "null argument");
  return set_moving_paths(d, n_spheres, radius, nullptr, omega, n_samples, centre, velocity, variant, q_cutoff);
}

int lbm_step(lbm_domain d, int32_t n_steps) {
  if (!d) return fail(LBM_EINVAL, "null domain");
  if (n_steps < 0) return fail(LBM_EINVAL, "n_steps < 0");
  if (!d->links_ok) return fail(LBM_ESTATE, "boundary links not set: some populations would be missing");
  if (n_steps > path_steps_left(d))
    return fail(LBM_ESTATE, "the sphere's path ends after " + std::to_string(path_steps_left(d)) + " more steps");
  for (int32_t s = 0; s < n_steps; ++s) {
    StepParams p = step_params(d, d->cur);
    hipError_t e = launch_step(d->desc.lattice, d->skind, p, d->stream);
    if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("step kernel: ") + hipGetErrorString(e));
    d->cur ^= 1;
    ++d->steps;
    if (d->moving) {
      if (d->track_force && s == n_steps - 1) {
        // force and torque on the links of the geometry this step used, before the rebuild
        MovingParams mp = moving_params(d, d->cur);
        mp.k = moving_kin(d, d->steps - 1);
        e = launch_moving_force(d->desc.lattice, d->desc.storage, mp, d->mforce, d->mgroup, d->mforce + 6 * d->link_cap,
                                d->stream);
        if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("moving force: ") + hipGetErrorString(e));
        d->force_step = d->steps;
      }
      e = rebuild_moving(d, d->steps, true);
      if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("moving geometry: ") + hipGetErrorString(e));
    }
  }
  return LBM_OK;
}

int lbm_macros(lbm_domain d, double* rho, double* u, double* sums) {
  if (!d) return fail(LBM_EINVAL, "null domain");
  const int64_t N = d->N;
  if (!d->uprev) {   // first call: the previous field is the initial one, u0 + F / (2 rho0) on fluid nodes
    if (int e = dalloc(d->uprev, N * d->D * 8)) return e;
    std::vector<double> up((size_t)N * d->D, 0.0);
    for (int64_t n = 0; n < N; ++n)
      if (d->mask[n])
        for (int a = 0; a < d->D; ++a) up[n * d->D + a] = d->desc.u0[a] + 0.5 * d->desc.force[a] / d->desc.rho0;
    HIP_TRY(hipMemcpyAsync(d->uprev, up.data(), up.size() * 8, hipMemcpyHostToDevice, d->stream));
    HIP_TRY(hipStreamSynchronize(d->stream));
  }
  if (rho && !d->rho_tmp)
    if (int e = dalloc(d->rho_tmp, N * 8)) return e;
  if (u && !d->u_tmp)
    if (int e = dalloc(d->u_tmp, N * d->D * 8)) return e;
  MacroParams p{};
  p.g = d->g;
  p.src = d->buf[d->cur];
  p.lk = link_view(d, d->lv[d->cur], nullptr);
  for (int a = 0; a < 3; ++a) p.force[a] = d->desc.force[a];
  p.rho = rho ? d->rho_tmp : nullptr;
  p.u = u ? d->u_tmp : nullptr;
  p.uprev = d->uprev;
  p.partials = d->partials;
  p.nblocks = d->red_blocks;
  HIP_TRY(launch_macros(d->desc.lattice, d->desc.storage, p, d->red_blocks, d->stream));
  HIP_TRY(launch_reduce(d->partials, d->red_blocks, d->sums, d->stream));
  double h[NPART];
  HIP_TRY(hipMemcpyAsync(h, d->sums, sizeof(h), hipMemcpyDeviceToHost, d->stream));
  if (rho) HIP_TRY(hipMemcpyAsync(rho, d->rho_tmp, N * 8, hipMemcpyDeviceToHost, d->stream));
  if (u) HIP_TRY(hipMemcpyAsync(u, d->u_tmp, N * d->D * 8, hipMemcpyDeviceToHost, d->stream));
  HIP_TRY(hipStreamSynchronize(d->stream));
  if (sums) {
    int k = 0;
    sums[k++] = h[0];
    sums[k++] = h[1];
    sums[k++] = h[2];
    if (d->D == 3) sums[k++] = h[3];
    sums[k++] = h[5] > 0.0 ? std::sqrt(h[4] / h[5]) : (h[4] > 0.0 ? INFINITY : 0.0);
  }
  if (h[6] > 0.0) return fail(LBM_EUNSTABLE, "non-finite density or velocity at " + std::to_string((int64_t)h[6]) + " nodes");
  clear_error();
  return LBM_OK;
}

int lbm_get_state(lbm_domain d, double* f) {
  if (!d || !f) return fail(LBM_EINVAL, "null argument");
  double* tmp = nullptr;
  const size_t bytes = (size_t)d->N * d->Q * 8;
  if (int e = dalloc(tmp, bytes)) return e;
  hipError_t e = export_state(d, tmp);
  if (e == hipSuccess) e = hipMemcpyAsync(f, tmp, bytes, hipMemcpyDeviceToHost, d->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(d->stream);
  (void)hipFree(tmp);
  if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("get_state: ") + hipGetErrorString(e));
  return LBM_OK;
}

int lbm_set_state(lbm_domain d, const double* f) {
  if (!d || !f) return fail(LBM_EINVAL, "null argument");
  double* tmp = nullptr;
  const size_t bytes = (size_t)d->N * d->Q * 8;
  if (int e = dalloc(tmp, bytes)) return e;
  hipError_t e = hipMemcpyAsync(tmp, f, bytes, hipMemcpyHostToDevice, d->stream);
  if (e == hipSuccess) e = import_state(d, tmp);
  d->state_set = true;
  if (e == hipSuccess) e = hipStreamSynchronize(d->stream);
  (void)hipFree(tmp);
  if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("set_state: ") + hipGetErrorString(e));
  return LBM_OK;
}

int lbm_set_link_groups(lbm_domain d, const int32_t* group, int32_t n_groups) {
  if (!d) return fail(LBM_EINVAL, "null domain");
  if (d->moving || !d->links_ok) return fail(LBM_ESTATE, "link groups need an installed static link list");
  if (n_groups < 1 || n_groups > 4096) return fail(LBM_EINVAL, "n_groups must lie in [1, 4096]");
  if (!group && n_groups != 1) return fail(LBM_EINVAL, "group ids are required for more than one group");
  std::vector<int32_t> sorted(d->nl, 0);
  if (group) {
    for (int64_t k = 0; k < d->nl; ++k) {
      const int32_t v = group[d->link_order[k]];
      if (v < 0 || v >= n_groups)
        return fail(LBM_EINVAL, "link " + std::to_string(d->link_order[k]) + ": group out of range");
      sorted[k] = v;
    }
  }
  HIP_TRY(hipStreamSynchronize(d->stream));
  dfree(d->lgrp);
  dfree(d->gforce);
  if (group && d->nl > 0) {
    if (int e = dalloc(d->lgrp, sorted.size() * 4)) return e;
    HIP_TRY(hipMemcpy(d->lgrp, sorted.data(), sorted.size() * 4, hipMemcpyHostToDevice));
  }
  d->n_groups = n_groups;
  clear_error();
  return LBM_OK;
}

}  // extern "C"

namespace {
// Force and torque per link group of the last step (static link lists).
int force_torque(lbm_domain d, const double* centres, double* force, double* torque) {
  if (d->moving) return fail(LBM_ESTATE, "the force of a moving sphere is not available (its links are rebuilt every step)");
  if (!d->links_ok) return fail(LBM_ESTATE, "boundary links not set");
  if (d->steps == d->links_step || d->steps == d->state_step)
    return fail(LBM_ESTATE, "no step taken since the links or the state were installed");
  if (centres)
    for (int k = 0; k < 3 * d->n_groups; ++k)
      if (!std::isfinite(centres[k])) return fail(LBM_EINVAL, "non-finite torque reference point");
  if (!d->lforce && d->nl > 0)
    if (int e = dalloc(d->lforce, (size_t)d->nl * 6 * 8)) return e;
  if (!d->gforce)
    if (int e = dalloc(d->gforce, (size_t)d->n_groups * 9 * 8)) return e;
  double* dcentre = nullptr;
  if (centres) {
    dcentre = d->gforce + 6 * d->n_groups;
    HIP_TRY(hipMemcpyAsync(dcentre, centres, (size_t)d->n_groups * 3 * 8, hipMemcpyHostToDevice, d->stream));
  }
  ForceParams p{};
  p.g = d->g;
  p.pop = d->buf[d->cur];
  p.lk = link_view(d, d->lv[d->cur], nullptr);
  p.luw = d->luw;
  p.group = d->lgrp;
  p.centre = dcentre;
  p.contrib = d->lforce;
  p.nl = d->nl;
  HIP_TRY(launch_force(d->desc.lattice, d->desc.storage, p, d->n_groups, d->gforce, d->stream));
  std::vector<double> h((size_t)d->n_groups * 6);
  HIP_TRY(hipMemcpyAsync(h.data(), d->gforce, h.size() * 8, hipMemcpyDeviceToHost, d->stream));
  HIP_TRY(hipStreamSynchronize(d->stream));
  for (int gi = 0; gi < d->n_groups; ++gi)
    for (int a = 0; a < 3; ++a) {
      if (force) force[3 * gi + a] = h[6 * gi + a];
      if (torque) torque[3 * gi + a] = h[6 * gi + 3 + a];
    }
  clear_error();
  return LBM_OK;
}
}  // namespace

extern "C" {

int lbm_momentum_exchange(lbm_domain d, double* force) {
  if (!d || !force) return fail(LBM_EINVAL, "null argument");
  return force_torque(d, nullptr, force, nullptr);
}

int lbm_force_torque(lbm_domain d, const double* centres, double* force, double* torque) {
  if (!d || !force || !torque) return fail(LBM_EINVAL, "null argument");
  return force_torque(d, centres, force, torque);
}

int lbm_set_force_tracking(lbm_domain d, int32_t on) {
  if (!d) return fail(LBM_EINVAL, "null domain");
  if (!d->moving) return fail(LBM_ESTATE, "force tracking is for moving spheres (static links: lbm_force_torque)");
  if (on != 0 && on != 1) return fail(LBM_EINVAL, "on must be 0 or 1");
  if (on && !d->mforce)
    if (int e = dalloc(d->mforce, ((size_t)d->link_cap + MAX_SPHERES) * 6 * 8)) return e;
  if (on && !d->mgroup)
    if (int e = dalloc(d->mgroup, (size_t)d->link_cap * 4)) return e;
  d->track_force = on != 0;
  d->force_step = -1;
  clear_error();
  return LBM_OK;
}

int lbm_moving_forces(lbm_domain d, int32_t n_spheres, double* force, double* torque) {
  if (!d || !force || !torque) return fail(LBM_EINVAL, "null argument");
  if (!d->moving || !d->track_force) return fail(LBM_ESTATE, "force tracking is not on (lbm_set_force_tracking)");
  if (n_spheres != d->mv_ns)
    return fail(LBM_EINVAL, "the domain has " + std::to_string(d->mv_ns) + " moving sphere(s)");
  if (d->force_step != d->steps)
    return fail(LBM_ESTATE, "the last step was not taken by lbm_step with tracking on (or none was taken)");
  double h[6 * MAX_SPHERES];
  HIP_TRY(hipMemcpyAsync(h, d->mforce + 6 * d->link_cap, 6 * n_spheres * sizeof(double), hipMemcpyDeviceToHost,
                         d->stream));
  HIP_TRY(hipStreamSynchronize(d->stream));
  for (int sp = 0; sp < n_spheres; ++sp)
    for (int a = 0; a < 3; ++a) {
      force[3 * sp + a] = h[6 * sp + a];
      torque[3 * sp + a] = h[6 * sp + 3 + a];
    }
  clear_error();
  return LBM_OK;
}

int lbm_moving_force(lbm_domain d, double* force, double* torque) {
  if (!d || !force || !torque) return fail(LBM_EINVAL, "null argument");
  if (d->moving && d->mv_ns != 1) return fail(LBM_EINVAL, "several moving spheres: lbm_moving_forces");
  return lbm_moving_forces(d, 1, force, torque);
}

int lbm_stream_probe(const float* src, float* dst, int64_t n, int64_t stride, int32_t arrays, int32_t shift,
                     void* stream) {
  if (!src || !dst) return fail(LBM_EINVAL, "null argument");
  if (n < 0 || arrays < 1 || shift < 0 || shift >= 64 || stride < n + shift || n >= ((int64_t)1 << 40))
    return fail(LBM_EINVAL, "need n >= 0, arrays >= 1, 0 <= shift < 64, stride >= n + shift");
  HIP_TRY(launch_stream_probe(src, dst, n, stride, arrays, shift, static_cast<hipStream_t>(stream)));
  clear_error();
  return LBM_OK;
}

int lbm_set_stream(lbm_domain d, void* stream) {
  if (!d) return fail(LBM_EINVAL, "null domain");
  d->stream = static_cast<hipStream_t>(stream);
  d->uid = next_uid();
  d->desc.stream = stream;
  return LBM_OK;
}

int lbm_set_launch_option(lbm_domain d, int32_t option, int32_t value) {
  if (!d) return fail(LBM_EINVAL, "null domain");
  if (option != LBM_OPT_XCD_REMAP || (value != 0 && value != 1)) return fail(LBM_EINVAL, "invalid launch option");
  d->g.xcd_remap = value;
  return LBM_OK;
}

int lbm_get_info(lbm_domain d, lbm_domain_info* info) {
  if (!d || !info) return fail(LBM_EINVAL, "null argument");
  info->n_nodes = d->N;
  info->n_fluid = d->n_fluid;
  info->n_boundary_nodes = d->nb;
  info->n_links = d->nl;
  if (d->moving) {   // the geometry of the current step lives on the device
    std::vector<uint64_t> sf(d->g.nseg), sb(d->g.nseg);
    int32_t nl = 0;
    HIP_TRY(hipStreamSynchronize(d->stream));
    HIP_TRY(hipMemcpy(sf.data(), d->seg_fluid, d->g.nseg * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(sb.data(), d->seg_bnd, d->g.nseg * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&nl, d->seg_lbase + d->g.nseg, 4, hipMemcpyDeviceToHost));
    info->n_fluid = info->n_boundary_nodes = 0;
    for (int64_t s2 = 0; s2 < d->g.nseg; ++s2) {
      info->n_fluid += __builtin_popcountll(sf[s2]);
      info->n_boundary_nodes += __builtin_popcountll(sb[s2]);
    }
    info->n_links = nl;
  }
  info->population_bytes = (int64_t)(2 * d->g.npad * d->Q * d->elem);
  const int64_t rs = d->desc.storage == LBM_F64 ? 8 : 4;
  // per link: ld, q, (Gw), two link values (list mode); per segment: masks and prefixes
  info->link_bytes = info->n_links * (2 + rs * (1 + (d->lg ? 1 : 0) + (d->lv[0] ? 2 : 0))) + d->g.nseg * 24;
  info->steps_done = d->steps;
  info->q = d->Q;
  info->storage = d->desc.storage;
  return LBM_OK;
}

int lbm_free_domain(lbm_domain d) {
  if (!d) return fail(LBM_EINVAL, "null domain");
  if (d->stream) (void)hipStreamSynchronize(d->stream);
  else (void)hipDeviceSynchronize();
  if (d->own_buf) {
    dfree(d->buf[0]);
    dfree(d->buf[1]);
  }
  dfree(d->seg_fluid);
  dfree(d->seg_bnd);
  dfree(d->seg_lbase);
  dfree(d->seg_fbase);
  dfree(d->rng_ctr);
  dfree(d->row_src);
  free_links(d);
  dfree(d->partials);
  dfree(d->sums);
  dfree(d->uprev);
  dfree(d->reg_seg);
  dfree(d->seg_prev);
  dfree(d->reg_count);
  dfree(d->reg_cut);
  dfree(d->mforce);   // sized once: the spheres are set once, before tracking
  dfree(d->mgroup);
  dfree(d->rho_tmp);
  dfree(d->u_tmp);
  delete d;
  return LBM_OK;
}

}  // extern "C"
