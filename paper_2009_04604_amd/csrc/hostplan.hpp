// Host-side planning of a domain's storage and boundary links: plain C++ with
// no device calls, so that it also builds (and is tested) under the host
// sanitizers without a GPU.
//
//   segments   one 64-lane wave per 64 consecutive x of a row (y, z); the
//              fluid lane mask of every segment and its prefix count of fluid
//              nodes give the compact layout's slot of every fluid node.
//   links      validation of a caller's cut-link list against the fluid mask
//              and the domain's faces (Sec. II.B: a link joins a fluid node x_F
//              to a solid x_F - c_i, 0 < q <= 1), then the records the step
//              kernels read: links sorted by (node, dir), per segment a
//              boundary lane mask and the first link, and the moving-wall
//              term of each link (eq. ELIBB-general with the wall velocity).
#pragma once
#include <cstdint>
#include <vector>

namespace lbm {

constexpr int SEG = 64;          // lanes per segment (one wavefront)
constexpr int WAVES_PER_BLOCK = 4;
constexpr int BLOCK = SEG * WAVES_PER_BLOCK;
constexpr int GUARD = 64;        // compact layout: slots in front of the first fluid node

// The lattice extent as the host validation sees it.  mask: N bytes, 1 = fluid
// (owned by the caller, must outlive the view).  per: periodic flag per axis;
// outlet_face: -1 or the zero-gradient outlet face (2 axis + side).
struct HostGrid {
  int lattice;         // LBM_D2Q9, LBM_D3Q19 or LBM_D3Q27
  int n[3];
  int per[3];
  int outlet_face;
  const uint8_t* mask;
  int64_t N;
  int64_t nseg_x, nseg;
};

HostGrid make_host_grid(int lattice, int nx, int ny, int nz, int periodic, int outlet_face, const uint8_t* mask);

// Source x - c of a pull: false if it lies beyond a non-periodic face;
// otherwise s holds the wrapped coordinates.
bool pull_source(const HostGrid& g, const int c[3], int x, int y, int z, int s[3]);

// For a pull source beyond the outlet face: index of the node it is clamped
// onto if that node is fluid, else -1.
int64_t outlet_producer(const HostGrid& g, const int s[3]);

// First fluid node (and, in bad_dir, its direction) whose population is
// neither streamed from a fluid node, nor outlet-covered, nor linked
// (`linked`: per-node direction bit mask, or empty); -1 if there is none.
int64_t first_uncovered(const HostGrid& g, const std::vector<uint32_t>& linked, int* bad_dir);

// Fluid lane mask of every segment and the number of fluid nodes before it
// (nseg + 1 entries).
void segment_index(const HostGrid& g, std::vector<uint64_t>& fluid, std::vector<int32_t>& fbase);

// Compact layout: source rows of the pulls, per row r = y + ny z: entry k = 3 a + b (a, b in
// 0..2, D = 3; k = a for D = 2, b = 1) is the first segment of the row
// (y - (a - 1), z - (b - 1)) -- wrapped on periodic axes, clamped onto the
// outlet face, and otherwise clamped into the lattice (a row beyond a wall is
// only reached through cut links, whose pulled values are replaced).
int source_rows_per_row(int lattice);
void source_rows(const HostGrid& g, std::vector<int32_t>& row_src);

struct LinkPlan {
  std::vector<int64_t> order;    // caller's index of each stored link, sorted by (node, dir)
  std::vector<int32_t> lnode;    // node of each stored link
  std::vector<uint16_t> lld;     // lane in its segment | dir << 8
  std::vector<uint64_t> seg_bnd; // boundary lane mask per segment
  std::vector<int32_t> seg_lbase;// first link of each segment (nseg + 1 entries)
  int64_t n_boundary = 0;        // distinct boundary nodes
  std::vector<double> q;         // q of each stored link
  bool moving = false;           // some wall velocity is non-zero
  std::vector<double> gw;        // moving-wall term per stored link (moving only)
  std::vector<double> uv;        // [6][nl]: u_w(t), u_w(t+1) per stored link (moving only)
  bool uw_any = false;           // some u_w(t) is non-zero
  std::vector<double> uw;        // [nl][3] u_w(t) per stored link (uw_any only)
};

// Validate the caller's links (arrays as in lbm_set_boundary_links) and build
// the stored records.  `f64`: the moving-wall term is formed from the FP64
// weights, else from the FP32 ones the kernels use.  Returns LBM_OK, or
// LBM_EINVAL with the thread's error message naming the first bad link.
int plan_links(const HostGrid& g, int64_t n_links, const int64_t* node, const int8_t* dir, const double* q,
               const double* uw_t, const double* uw_t1, int variant, double q_cutoff, bool f64, LinkPlan& out);

}  // namespace lbm
