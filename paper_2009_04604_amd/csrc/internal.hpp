// Internal data structures shared by the host API and the kernels.
//
// Device data layout of one domain
// --------------------------------
// populations  two buffers, structure of arrays: Q direction arrays of
//              `stride` elements each, holding the shifted populations
//              h_i = f_i - w_i in the storage type.  Pull scheme: the value that
//              node x pulls in direction i lives in slot (x - c_i, i); after a
//              step slot (x, i) of a fluid node holds its post-collision h*_i.
//   compact    (static geometry) only fluid nodes are stored, in node order:
//              the slot of fluid node x is G + (number of fluid nodes before
//              x), found from the segment masks and their prefix counts
//              seg_fbase; the G = 64 slots in front and the tail are guards
//              (a segment whose fluid count before it is a multiple of 64
//              then starts on a cache line, as every segment of an all-fluid
//              row of 64 k nodes does).  Solid nodes cost neither memory nor
//              bandwidth.
//   dense      (moving geometry) [NZ][NY][NX] with NX = nx + 2 px etc.: one
//              halo layer on each non-periodic axis.
// outlet       a zero-gradient outlet face is a clamp of the pull source onto
//              the face layer: the outlet population reads the same slot as
//              its upstream neighbour (read-only sharing).
// source rows (compact layout) per row the first segment of each of its
//              pull-source rows (wrapped, clamped), so that a wave finds its
//              source segments without coordinate arithmetic.
// segments     one wave (64 lanes) handles 64 consecutive x of one row (y, z):
//              seg_fluid / seg_bnd are 64-bit lane masks of fluid and boundary
//              nodes; a segment with boundary nodes has its cut links in
//              links[seg_lbase[s] .. seg_lbase[s+1]) (nseg + 1 entries; entry
//              nseg is the link count).  Segments without boundary nodes never
//              read seg_lbase.
// links        ordered by (node, dir), so each segment's links are contiguous:
//              ld (uint16) = lane of the boundary node in its segment | dir << 8,
//              q and, when any wall moves, the wall term Gw (see elibb.hpp),
//              lnode the node index (used only outside the step).
// link values  with a static link list the rebuilt populations live in two
//              per-link arrays lv[2] (shifted, like the populations): step t
//              reads f_i(x_F, t) of every cut link from lv_in while pulling
//              and writes f_i(x_F, t+1) to lv_out, coalesced.  Without link
//              value arrays (moving geometry) the rebuilt value is stored in the
//              solid-side slot x_F - c_i that x_F pulls instead.
//              A wave stages its boundary nodes' populations and moments in LDS,
//              patches the cut directions, and rebuilds its links one per lane.
// block order  workgroups are dealt to the 8 XCDs round-robin; the kernels
//              remap the workgroup id so that each XCD walks a contiguous range
//              of rows (neighbouring rows share its L2).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "hostplan.hpp"
#include "lattice.hpp"

namespace lbm {
// Load through the constant address space, for data that no thread writes
// while the kernel runs (domain metadata, parameter tables written by the host).
// A wave-uniform address then becomes a scalar load, and a pointer loaded this
// way is taken for a global one: memory instructions through a pointer read from
// global memory would otherwise be flat ones (slower, and never scalar).
template <typename T>
__device__ __forceinline__ T load_const(const T* ptr) {
  return *(const __attribute__((address_space(4))) T*)ptr;
}
}  // namespace lbm

namespace lbm {

// Division by a run-time constant d < 2^31 for dividends n < 2^31:
// n / d = (umulhi(n, m) + n) >> s  (m, s chosen on the host).
struct FastDiv {
  uint32_t d, m, s;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f{d, 0u, 0u};
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  f.s = l;
  f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
  return f;
}

struct GridGeom {
  int32_t nx, ny, nz;            // domain size
  int32_t NX, NY, NZ;            // padded storage size
  int32_t px, py, pz;            // halo widths (0 or 1)
  int32_t perx, pery, perz;      // periodic flags
  int32_t nseg_x;                // segments per row
  int64_t nseg;                  // total segments (< 2^31)
  int32_t guard;                 // compact layout: slot of the first fluid node
  FastDiv div_nseg_x, div_ny;    // fast division by nseg_x and ny
  int32_t xcd_remap;             // 1: each XCD walks a contiguous eighth of the rows
  int32_t compact;               // 1: compact (fluid-only) layout
  int32_t outlet;                // outlet face or -1
  int64_t npad;                  // elements between direction arrays (stride)
};

struct LinkView {
  const uint64_t* seg_fluid;
  const int32_t* seg_fbase;      // [nseg + 1] fluid nodes before each segment
  const int32_t* row_src;        // compact layout: [rows][3 or 9] first segment of each pull-source row
  const uint64_t* seg_bnd;
  const int32_t* seg_lbase;      // [nseg + 1]
  const uint16_t* lld;           // link lane | dir << 8
  const int32_t* lnode;          // link node index
  const void* lq;                // link q (double for FP64 storage, float otherwise)
  const void* lg;                // link wall term Gw, or null when every wall rests
  const void* lv_in;             // link values at t (null: slot mode)
  void* lv_out;                  // link values at t+1
  const void* luv;               // [6][luv_stride] wall velocities u_w(t), u_w(t+1) per link
                                 // (regularised wall non-equilibrium with moving walls), or null
  int64_t luv_stride;
};

struct StepParams {
  GridGeom g;
  const void* src;
  void* dst;
  LinkView lk;
  double omega;                  // omega+ = 1/tau
  double omega_minus;            // TRT: omega-; BGK: omega
  int32_t trt;                   // 1: TRT collision
  double force[3];
  double src_eq;                 // 3 (1 - omega/2) / omega: Guo's source folded into the equilibrium
  double src_eq_minus;           // TRT: the same with omega- (odd part)
  int32_t has_force;
  int32_t variant;
  double q_cut;
  int32_t outlet_face;
  int32_t wall_neq;              // 0: bounced non-equilibrium (eq. neqbb-s); 1: regularised (eq. fi_neq);
                                 // selects the kernel variant (batches group by it)
  uint32_t* rng_ctr;             // stochastic rounding: the domain's step count, by buffer parity
                                 // ([parity] is read, block 0 writes [1 - parity] = [parity] + 1)
  int32_t parity;                // buffer holding the current state (the domain's cur)
  // omega, omega-, force, src_eq, src_eq_minus and q_cut rounded to FP32 on the
  // host (the FP32 and 16-bit kernels read these instead of converting the
  // doubles in every wave; the values are the same)
  float omega_f, omega_minus_f, force_f[3], src_eq_f, src_eq_minus_f, q_cut_f;
};

struct InitParams {
  GridGeom g;
  void* dst;
  LinkView lk;                   // lv_out receives the cut-link values (list mode)
  int64_t nlinks;
  const double* f_in;            // [Q][N] or null for the equilibrium (rho0, u0)
  double rho0, u0[3];
};

struct ExportParams {
  GridGeom g;
  const void* src;
  LinkView lk;                   // lv_in holds the cut-link values (list mode)
  double* f_out;                 // [Q][N]
};

struct MacroParams {
  GridGeom g;
  const void* src;
  LinkView lk;
  double force[3];
  double* rho;                   // [N] or null
  double* u;                     // [N*D] or null
  double* uprev;                 // [N*D] previous velocity (updated), or null: no residual
  double* partials;              // [gridDim.x][NPART]
  int64_t nblocks;               // logical blocks of the lattice (grid_blocks)
};
constexpr int NPART = 8;         // mass, mom x/y/z, |du|^2, |u|^2, non-finite count, pad

struct ForceParams {
  GridGeom g;
  const void* pop;               // current population buffer
  LinkView lk;                   // lv_in: the link values of the current time
  const double* luw;             // [3 nl] wall velocity per link, or null (walls at rest)
  const int32_t* group;          // [nl] group of each link, or null (one group)
  const double* centre;          // [3 n_groups] torque reference points, or null (origin)
  double* contrib;               // [6 nl] force and torque per link
  int64_t nl;
};

// Kinematics of a moving sphere for the geometry of time t.
// Spheres per domain in the moving rebuild.
constexpr int MAX_SPHERES = 4;

// Kinematics of a domain's spheres for the geometry of time t.
struct MovingKin {
  int32_t ns;                               // spheres in use (1 .. MAX_SPHERES)
  double r[MAX_SPHERES];                    // radii
  double c[MAX_SPHERES][3];                 // centres at t
  double V[MAX_SPHERES][3], V1[MAX_SPHERES][3];    // translational velocities at t and t+1
  double Om[MAX_SPHERES][3], Om1[MAX_SPHERES][3];  // angular velocities at t and t+1
};

// Moving spheres of one domain (dense layout, slot mode): the geometry of time t
// is rebuilt on the device over a fixed region of segments (the union of the
// spheres' sweep boxes).
struct MovingParams {
  GridGeom g;
  MovingKin k;                   // single-domain launches; batched launches read a table
  int32_t kin_slot;              // batched launches: column of this sphere in the table
  int32_t variant;
  double q_cut;
  const int32_t* reg_seg;        // region segments
  int64_t nreg;
  uint64_t* seg_fluid;           // fluid mask at t (written by classify)
  uint64_t* seg_prev;            // fluid mask at t-1 (written by classify)
  uint64_t* seg_bnd;
  int32_t* reg_count;            // cut links per region segment
  uint32_t* reg_cut;             // [nreg][64] cut directions of each region node (classify -> fill)
  int32_t* seg_lbase;            // link starts: written around the region segments
  uint16_t* lld;
  void* lq;
  void* lg;
  void* luv;                     // [6][luv_stride] wall velocities per link (regularised wall
                                 // non-equilibrium), or null
  int64_t luv_stride;            // link capacity
  void* pop;                     // current population buffer (refill)
  double rho0;
};

// Tile table of a batched step: domain << TILE_SHIFT | block of that domain.
constexpr uint32_t TILE_SHIFT = 22;
constexpr uint32_t TILE_MASK = (1u << TILE_SHIFT) - 1u;
constexpr uint32_t TILE_EMPTY = ~0u;

// Number of workgroups of the lattice kernels (a multiple of the 8 XCDs).
int64_t grid_blocks(const GridGeom& g);

// Per-lattice launchers (kernels.hip, compiled once per lattice and explicitly
// instantiated there); the entry points below dispatch on the lattice.
template <class L>
struct Launch {
  static hipError_t step(int storage, const StepParams& p, hipStream_t s);
  static hipError_t step_batch(int storage, bool compact, bool trt, bool reg, const StepParams* tab,
                               const uint32_t* tiles, uint32_t nslots, uint32_t grid, hipStream_t s);
  static hipError_t init(int storage, const InitParams& p, hipStream_t s);
  static hipError_t init_links(int storage, const InitParams& p, hipStream_t s);
  static hipError_t export_state(int storage, const ExportParams& p, hipStream_t s);
  static hipError_t macros(int storage, const MacroParams& p, int64_t nblocks, hipStream_t s);
  static hipError_t force(int storage, const ForceParams& p, hipStream_t s);
};
extern template struct Launch<D2Q9>;
extern template struct Launch<D3Q19>;
extern template struct Launch<D3Q27>;

// Launchers (kernels.hip); dispatch on lattice and storage.
hipError_t launch_step(int lattice, int storage, const StepParams& p, hipStream_t s);
hipError_t launch_init(int lattice, int storage, const InitParams& p, hipStream_t s);
hipError_t launch_init_links(int lattice, int storage, const InitParams& p, hipStream_t s);
hipError_t launch_export(int lattice, int storage, const ExportParams& p, hipStream_t s);
hipError_t launch_macros(int lattice, int storage, const MacroParams& p, int64_t nblocks, hipStream_t s);
hipError_t launch_reduce(const double* partials, int64_t nblocks, double* out, hipStream_t s);
hipError_t launch_force(int lattice, int storage, const ForceParams& p, int32_t n_groups, double* out,
                        hipStream_t s);
hipError_t launch_stream_probe(const float* src, float* dst, int64_t n, int64_t stride, int32_t arrays,
                               int32_t shift, hipStream_t s);
hipError_t launch_group_sum(const double* contrib, const int32_t* group, int64_t nl, const int32_t* nl_dev,
                            int32_t n_groups, double* out, hipStream_t s);
hipError_t launch_moving_classify(int lattice, const MovingParams& p, hipStream_t s);
// force and torque of the moving spheres over the links of the geometry the last
// step used (before the rebuild); contrib: [6 link_cap] scratch, grp: [link_cap]
// scratch (the sphere of each link), out: [ns][6]
hipError_t launch_moving_force(int lattice, int storage, const MovingParams& p, double* contrib, int32_t* grp,
                               double* out, hipStream_t s);
hipError_t launch_region_scan(const MovingParams& p, hipStream_t s);
hipError_t launch_moving_fill(int lattice, int storage, const MovingParams& p, hipStream_t s);
hipError_t launch_moving_refill(int lattice, int storage, const MovingParams& p, hipStream_t s);
hipError_t launch_step_batch(int lattice, int storage, bool compact, bool trt, bool reg, const StepParams* tab,
                             const uint32_t* tiles, uint32_t nslots, uint32_t grid, hipStream_t s);
// Batched moving-sphere rebuild (moving.hip).  tab: one MovingParams per sphere;
// waves: region waves as sphere << TILE_SHIFT | wave; kin: [step][nkin] table,
// row *ctr is the geometry time being built.
struct MovingBatch {
  const MovingParams* tab;
  int32_t nbox;
  int32_t multi;                 // 1: some box holds more than one sphere
  const uint32_t* waves;
  uint32_t nwaves;
  const MovingKin* kin;
  int32_t nkin;
  const int64_t* ctr;
};
hipError_t launch_moving_batch(int lattice, int storage, const MovingBatch& b, hipStream_t s);
hipError_t launch_advance(int64_t* ctr, hipStream_t s);
// Address of the no-allocation scratch array on a device, looked up once per
// device (noalloc.hip); called by lbm_init_domain with that device current.
hipError_t noalloc_setup(int device);

}  // namespace lbm

struct lbm_domain_s {
  lbm_domain_desc desc;
  int device;                    // HIP device current when the domain was created
  uint64_t uid;                  // unique per domain, renewed when its device layout changes
  int Q, D;
  lbm::GridGeom g;
  int64_t N;                     // nx * ny * nz
  size_t elem;                   // bytes per stored population value
  void* buf[2];
  int cur;                       // buffer holding the current state
  bool own_buf;
  hipStream_t stream;
  std::vector<uint8_t> mask;     // host copy of the fluid mask
  int64_t n_fluid;
  // segments
  uint64_t* seg_fluid;
  uint64_t* seg_bnd;
  int32_t* seg_lbase;
  int32_t* seg_fbase;
  int32_t* row_src;              // compact layout only (source_rows)
  // boundary nodes and links
  int64_t nb, nl;
  uint16_t* lld;
  int32_t* lnode;
  void* lq;
  void* lg;
  void* lv[2];                   // link values (list mode), lv[cur] is current
  bool links_ok;
  int32_t variant;
  double q_cut;
  int32_t wall_neq;              // LBM_NEQ_BOUNCEBACK or LBM_NEQ_REGULARIZED
  int32_t skind;                 // storage kind of the step kernels (ST_*; the stochastic kinds
                                 // for 16-bit storage with LBM_ROUND_STOCHASTIC)
  uint32_t* rng_ctr;             // [2] step count by buffer parity (stochastic rounding)
  void* luv;                     // [6][nl or link_cap] u_w(t), u_w(t+1) per link (moving walls), or null
  // reductions
  double* partials;
  double* sums;
  double* uprev;
  double* rho_tmp;
  double* u_tmp;
  int64_t red_blocks;
  int64_t steps;
  bool state_set;                // lbm_set_state was called (the state is not the initial one)
  int64_t state_step;            // steps when the state was last imported (set_state, links)
  // moving sphere (lbm_set_moving_sphere)
  bool moving;
  double mv_x0[3], mv_amp, mv_period, mv_dir[3], mv_om[3];
  int mv_ns = 1;                       // spheres (the sinusoid: one)
  double mv_r[lbm::MAX_SPHERES];       // radii
  std::vector<double> path_c, path_v;  // [n][ns][3] prescribed centres and velocities per step (empty: the sinusoid)
  std::vector<double> path_om;         // [n][ns][3] angular velocities per step (empty: constant mv_om)
  int32_t* reg_seg;
  int64_t nreg;
  uint64_t* seg_prev;
  int32_t* reg_count;
  uint32_t* reg_cut;
  int64_t link_cap;
  bool track_force;                  // lbm_set_force_tracking: force of the last step of each lbm_step call
  int64_t force_step;                // steps when that force was computed
  double* mforce;                    // [6 link_cap] per-link contributions, then [ns][6] the sums
  int32_t* mgroup;                   // [link_cap] the sphere of each link (several spheres)
  // momentum-exchange force (static link list)
  std::vector<int64_t> link_order;   // position in the caller's list of each stored link
  double* luw;                       // [3 nl] wall velocity at t, or null
  int32_t* lgrp;                     // [nl] group of each stored link, or null (one group)
  int32_t n_groups;
  double* lforce;                    // [6 nl] scratch: force and torque per link
  double* gforce;                    // [6 n_groups] sums, then [3 n_groups] torque reference points
  int64_t links_step;                // steps when the links were installed
};

namespace lbm {
// Kernel parameters of one domain (api.cpp), used by the single-domain calls
// and by the batched step.  `cur` names the buffer holding the current state.
StepParams step_params(const lbm_domain_s* d, int cur);
MovingParams moving_params(const lbm_domain_s* d, int cur);
MovingKin moving_kin(const lbm_domain_s* d, int64_t t);
// Steps left on a sphere's sampled path (INT64_MAX without one).
int64_t path_steps_left(const lbm_domain_s* d);
// Identity for caches of kernel parameters (a freed domain's address can be
// reused by a new one; links or a stream set anew also change the uid).
uint64_t next_uid();
}  // namespace lbm
