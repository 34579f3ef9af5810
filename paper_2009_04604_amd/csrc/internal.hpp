// Internal data structures shared by the host API and the kernels.
//
// Device data layout of one domain
// --------------------------------
// populations  two buffers, structure of arrays [Q][NZ][NY][NX] of the storage
//              type.  NX = nx + 2 px etc.: one halo layer (px = 1) on each
//              non-periodic axis, none on periodic ones.  Pull scheme: the value
//              that node x pulls in direction i lives in slot (x - c_i, i).
//              After a step, slot (x, i) of a fluid node x holds its post-
//              collision f*_i, and slot (x_F - c_i, i) of a cut link holds the
//              ELIBB value f_i(x_F, t+1) written by the boundary node itself.
// segments     one wave (64 lanes) handles 64 consecutive x of one row (y, z):
//              seg_fluid / seg_bnd are 64-bit lane masks of fluid and boundary
//              nodes, seg_bbase the index of the segment's first boundary node.
// boundary     per boundary node b (sorted by node index): bmask[b] bit i set iff
//              (node, i) is a cut link; blink[b] the index of its first link.
// links        per link, ordered by (node, dir): q and, when any wall moves, the
//              wall factor G (see elibb.hpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lbm.h"

namespace lbm {

constexpr int SEG = 64;          // lanes per segment (one wavefront)
constexpr int WAVES_PER_BLOCK = 4;
constexpr int BLOCK = SEG * WAVES_PER_BLOCK;

struct GridGeom {
  int32_t nx, ny, nz;            // domain size
  int32_t NX, NY, NZ;            // padded storage size
  int32_t px, py, pz;            // halo widths (0 or 1)
  int32_t perx, pery, perz;      // periodic flags
  int32_t nseg_x;                // segments per row
  int64_t nseg;                  // total segments
  int64_t npad;                  // NX * NY * NZ (stride between direction arrays)
};

struct StepParams {
  GridGeom g;
  const void* src;
  void* dst;
  const uint64_t* seg_fluid;
  const uint64_t* seg_bnd;
  const int32_t* seg_bbase;
  const uint32_t* bmask;
  const int32_t* blink;
  const void* lq;                // link q (double for FP64 storage, float otherwise)
  const void* lg;                // link wall factor G, or null when every wall rests
  double omega;
  double force[3];
  int32_t has_force;
  int32_t variant;
  double q_cut;
  int32_t outlet_face;
};

struct InitParams {
  GridGeom g;
  void* dst;
  const uint64_t* seg_fluid;
  const double* f_in;            // [Q][N] or null for the equilibrium (rho0, u0)
  double rho0, u0[3];
};

struct ExportParams {
  GridGeom g;
  const void* src;
  const uint64_t* seg_fluid;
  double* f_out;                 // [Q][N]
};

struct MacroParams {
  GridGeom g;
  const void* src;
  const uint64_t* seg_fluid;
  double force[3];
  double* rho;                   // [N] or null
  double* u;                     // [N*D] or null
  double* uprev;                 // [N*D] previous velocity (updated)
  double* partials;              // [nblocks][NPART]
};
constexpr int NPART = 8;         // mass, mom x/y/z, |du|^2, |u|^2, non-finite count, pad

// Launchers (kernels.hip); dispatch on lattice and storage.
hipError_t launch_step(int lattice, int storage, const StepParams& p, hipStream_t s);
hipError_t launch_init(int lattice, int storage, const InitParams& p, hipStream_t s);
hipError_t launch_export(int lattice, int storage, const ExportParams& p, hipStream_t s);
hipError_t launch_macros(int lattice, int storage, const MacroParams& p, int64_t nblocks, hipStream_t s);
hipError_t launch_reduce(const double* partials, int64_t nblocks, double* out, hipStream_t s);

}  // namespace lbm

struct lbm_domain_s {
  lbm_domain_desc desc;
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
  int32_t* seg_bbase;
  // boundary nodes and links
  int64_t nb, nl;
  uint32_t* bmask;
  int32_t* blink;
  void* lq;
  void* lg;
  bool links_ok;
  int32_t variant;
  double q_cut;
  // reductions
  double* partials;
  double* sums;
  double* uprev;
  double* rho_tmp;
  double* u_tmp;
  int64_t red_blocks;
  int64_t steps;
};
