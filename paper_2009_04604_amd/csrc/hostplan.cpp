// Host-side planning of storage and boundary links (no device calls).
#include "hostplan.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>

#include "../../include/lbm.h"
#include "elibb.hpp"
#include "error.hpp"
#include "lattice.hpp"

namespace lbm {

namespace {

struct Dirs {
  int Q, D;
  int c[27][3];
};

template <class L>
Dirs make_dirs() {
  Dirs t{};
  t.Q = L::Q;
  t.D = L::D;
  for (int i = 0; i < L::Q; ++i) {
    t.c[i][0] = L::cx(i);
    t.c[i][1] = L::cy(i);
    t.c[i][2] = L::cz(i);
  }
  return t;
}

const Dirs& dirs_of(int lattice) {
  static const Dirs a = make_dirs<D2Q9>(), b = make_dirs<D3Q19>(), c = make_dirs<D3Q27>();
  return lattice == LBM_D2Q9 ? a : (lattice == LBM_D3Q19 ? b : c);
}

inline int64_t node_index(const HostGrid& g, const int p[3]) {
  return p[0] + (int64_t)g.n[0] * (p[1] + (int64_t)g.n[1] * p[2]);
}

}  // namespace

HostGrid make_host_grid(int lattice, int nx, int ny, int nz, int periodic, int outlet_face, const uint8_t* mask) {
  HostGrid g{};
  g.lattice = lattice;
  g.n[0] = nx;
  g.n[1] = ny;
  g.n[2] = nz;
  for (int a = 0; a < 3; ++a) g.per[a] = (periodic >> a) & 1;
  g.outlet_face = outlet_face;
  g.mask = mask;
  g.N = (int64_t)nx * ny * nz;
  g.nseg_x = (nx + SEG - 1) / SEG;
  g.nseg = g.nseg_x * ny * nz;
  return g;
}

bool pull_source(const HostGrid& g, const int c[3], int x, int y, int z, int s[3]) {
  const int p[3] = {x, y, z};
  bool inside = true;
  for (int a = 0; a < 3; ++a) {
    int v = p[a] - c[a];   // |c| <= 1: one wrap at most
    if (v < 0 || v >= g.n[a]) {
      if (g.per[a]) v += v < 0 ? g.n[a] : -g.n[a];
      else inside = false;
    }
    s[a] = v;
  }
  return inside;
}

int64_t outlet_producer(const HostGrid& g, const int s[3]) {
  const int f = g.outlet_face;
  if (f < 0) return -1;
  const int a = f >> 1;
  const bool beyond = (f & 1) ? s[a] >= g.n[a] : s[a] < 0;
  if (!beyond) return -1;
  int p[3] = {s[0], s[1], s[2]};
  p[a] = (f & 1) ? g.n[a] - 1 : 0;
  for (int b = 0; b < 3; ++b)
    if (p[b] < 0 || p[b] >= g.n[b]) return -1;
  const int64_t idx = node_index(g, p);
  return g.mask[idx] ? idx : -1;
}

int64_t first_uncovered(const HostGrid& g, const std::vector<uint32_t>& linked, int* bad_dir) {
  const Dirs& L = dirs_of(g.lattice);
  for (int z = 0; z < g.n[2]; ++z)
    for (int y = 0; y < g.n[1]; ++y)
      for (int x = 0; x < g.n[0]; ++x) {
        const int p[3] = {x, y, z};
        const int64_t n = node_index(g, p);
        if (!g.mask[n]) continue;
        for (int i = 1; i < L.Q; ++i) {
          int s[3];
          const bool inside = pull_source(g, L.c[i], x, y, z, s);
          if (inside && g.mask[node_index(g, s)]) continue;
          if (!linked.empty() && ((linked[n] >> i) & 1u)) continue;
          if (!inside && outlet_producer(g, s) >= 0) continue;
          *bad_dir = i;
          return n;
        }
      }
  return -1;
}

void segment_index(const HostGrid& g, std::vector<uint64_t>& fluid, std::vector<int32_t>& fbase) {
  fluid.assign(g.nseg, 0);
  for (int z = 0; z < g.n[2]; ++z)
    for (int y = 0; y < g.n[1]; ++y)
      for (int x = 0; x < g.n[0]; ++x) {
        const int p[3] = {x, y, z};
        if (g.mask[node_index(g, p)])
          fluid[(x / SEG) + g.nseg_x * (y + (int64_t)g.n[1] * z)] |= 1ull << (x % SEG);
      }
  fbase.assign(g.nseg + 1, 0);
  for (int64_t s = 0; s < g.nseg; ++s) fbase[s + 1] = fbase[s] + __builtin_popcountll(fluid[s]);
}

int source_rows_per_row(int lattice) { return lattice == LBM_D2Q9 ? 3 : 9; }

namespace {
// Source coordinate of a pull along one axis (coord - c), as the step kernels
// form it: wrapped, clamped onto an outlet face, else left outside.
int axis_source(int coord, int c, int n, int periodic, bool out_lo, bool out_hi) {
  const int v = coord - c;
  if (periodic) return v < 0 ? v + n : (v >= n ? v - n : v);
  if (v < 0 && out_lo) return 0;
  if (v >= n && out_hi) return n - 1;
  return v;
}
}  // namespace

void source_rows(const HostGrid& g, std::vector<int32_t>& row_src) {
  const int64_t nsx = g.nseg_x;
  const int64_t rows = (int64_t)g.n[1] * g.n[2];
  const int o = g.outlet_face;
  const bool d2 = g.lattice == LBM_D2Q9;
  const int nr = source_rows_per_row(g.lattice);
  row_src.assign(rows * nr, 0);
  for (int z = 0; z < g.n[2]; ++z)
    for (int y = 0; y < g.n[1]; ++y) {
      const int64_t r = y + (int64_t)g.n[1] * z;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          if (d2 && b != 1) continue;
          const int ys = axis_source(y, a - 1, g.n[1], g.per[1], o == 2, o == 3);
          const int zs = axis_source(z, b - 1, g.n[2], g.per[2], o == 4, o == 5);
          const int64_t yy = std::min(std::max(ys, 0), g.n[1] - 1), zz = std::min(std::max(zs, 0), g.n[2] - 1);
          row_src[r * nr + (d2 ? a : 3 * a + b)] = (int32_t)((yy + (int64_t)g.n[1] * zz) * nsx);
        }
    }
}

int plan_links(const HostGrid& g, int64_t n_links, const int64_t* node, const int8_t* dir, const double* q,
               const double* uw_t, const double* uw_t1, int variant, double q_cutoff, bool f64, LinkPlan& out) {
  out = LinkPlan{};
  if (n_links < 0) return set_error(LBM_EINVAL, "n_links < 0");
  if (n_links > 0 && (!node || !dir || !q)) return set_error(LBM_EINVAL, "node, dir and q are required");
  if (variant < LBM_ELIBB_FQ || variant > LBM_HWBB) return set_error(LBM_EINVAL, "invalid variant");
  if (!(q_cutoff >= 0.0) || !std::isfinite(q_cutoff)) return set_error(LBM_EINVAL, "q_cutoff must be finite and >= 0");
  if (n_links >= (int64_t)1 << 31) return set_error(LBM_EINVAL, "too many links");
  const Dirs& L = dirs_of(g.lattice);
  const int nx = g.n[0], ny = g.n[1];
  auto where = [&](int64_t k) {
    return "link " + std::to_string(k) + " (node " + std::to_string(node[k]) + ", dir " +
           std::to_string((int)dir[k]) + ")";
  };
  for (int64_t k = 0; k < n_links; ++k) {
    if (node[k] < 0 || node[k] >= g.N) return set_error(LBM_EINVAL, where(k) + ": node out of range");
    if (dir[k] < 1 || dir[k] >= L.Q) return set_error(LBM_EINVAL, where(k) + ": dir out of range");
    if (!(q[k] > 0.0 && q[k] <= 1.0)) return set_error(LBM_EINVAL, where(k) + ": q must lie in (0, 1]");
    for (int a = 0; a < 3; ++a) {
      if (uw_t && !std::isfinite(uw_t[3 * k + a])) return set_error(LBM_EINVAL, where(k) + ": non-finite uw_t");
      if (uw_t1 && !std::isfinite(uw_t1[3 * k + a])) return set_error(LBM_EINVAL, where(k) + ": non-finite uw_t1");
    }
    if (!g.mask[node[k]]) return set_error(LBM_EINVAL, where(k) + ": node is not fluid");
    const int64_t n = node[k];
    const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
    int s[3];
    const bool inside = pull_source(g, L.c[(int)dir[k]], x, y, z, s);
    if (inside && g.mask[node_index(g, s)])
      return set_error(LBM_EINVAL, where(k) + ": node - c_dir is a fluid node (not a cut link)");
    if (!inside && outlet_producer(g, s) >= 0)
      return set_error(LBM_EINVAL, where(k) + ": population is covered by the outlet");
  }
  std::vector<int64_t> order(n_links);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return node[a] != node[b] ? node[a] < node[b] : dir[a] < dir[b];
  });
  for (int64_t k = 1; k < n_links; ++k)
    if (node[order[k]] == node[order[k - 1]] && dir[order[k]] == dir[order[k - 1]])
      return set_error(LBM_EINVAL, where(order[k]) + ": duplicate link");

  std::vector<uint32_t> linked(g.N, 0u);
  for (int64_t k = 0; k < n_links; ++k) linked[node[k]] |= 1u << dir[k];
  int bad_dir = 0;
  const int64_t bad = first_uncovered(g, linked, &bad_dir);
  if (bad >= 0)
    return set_error(LBM_EINVAL, "population (node " + std::to_string(bad) + ", dir " + std::to_string(bad_dir) +
                                     ") is missing after streaming and not covered by a link");

  // segment masks and link records: links sorted by (node, dir) are contiguous
  // per segment; each carries its node's lane and its direction
  out.seg_bnd.assign(g.nseg, 0);
  out.seg_lbase.assign(g.nseg + 1, 0);
  out.lld.resize(n_links);
  out.lnode.resize(n_links);
  for (int64_t k = 0; k < n_links; ++k) {
    const int64_t n = node[order[k]];
    const int64_t row = n / nx;
    const int x = (int)(n - row * nx);
    const int64_t s = row * g.nseg_x + x / SEG;
    const int lane = x % SEG;
    if (!((out.seg_bnd[s] >> lane) & 1ull)) ++out.n_boundary;
    out.seg_bnd[s] |= 1ull << lane;
    out.seg_lbase[s + 1] += 1;
    out.lld[k] = (uint16_t)(lane | (int(dir[order[k]]) << 8));
    out.lnode[k] = (int32_t)n;
  }
  for (int64_t s = 0; s < g.nseg; ++s) out.seg_lbase[s + 1] += out.seg_lbase[s];

  for (int64_t k = 0; k < 3 * n_links && !out.moving; ++k)
    out.moving = (uw_t && uw_t[k] != 0.0) || (uw_t1 && uw_t1[k] != 0.0);
  for (int64_t k = 0; uw_t && k < 3 * n_links && !out.uw_any; ++k) out.uw_any = uw_t[k] != 0.0;
  out.q.resize(n_links);
  if (out.moving) {
    out.gw.resize(n_links);
    out.uv.assign(6 * (size_t)n_links, 0.0);
  }
  if (out.uw_any) out.uw.resize(3 * (size_t)n_links);
  for (int64_t k = 0; k < n_links; ++k) {
    const int64_t o = order[k];
    out.q[k] = q[o];
    if (out.uw_any)
      for (int a = 0; a < 3; ++a) out.uw[3 * k + a] = uw_t[3 * o + a];
    if (!out.moving) continue;
    const int i = dir[o];
    const double* u0 = uw_t ? uw_t + 3 * o : nullptr;
    const double* u1 = uw_t1 ? uw_t1 + 3 * o : u0;
    double cu0 = 0, uu0 = 0, cu1 = 0, uu1 = 0;
    for (int a = 0; a < L.D; ++a) {
      const double v0 = u0 ? u0[a] : 0.0, v1 = u1 ? u1[a] : 0.0;
      cu0 += L.c[i][a] * v0;
      uu0 += v0 * v0;
      cu1 += L.c[i][a] * v1;
      uu1 += v1 * v1;
      out.uv[a * n_links + k] = v0;
      out.uv[(3 + a) * n_links + k] = v1;
    }
    if (f64) {
      const Coef<double> c = elibb_coefficients<double>(variant, q[o], q_cutoff);
      out.gw[k] = wall_term<double>(c, cu0, uu0, cu1, uu1);
    } else {
      const Coef<float> c = elibb_coefficients<float>(variant, (float)q[o], (float)q_cutoff);
      const Coef<double> cd{c.a4, c.a5, c.a2, c.a3};
      out.gw[k] = wall_term<double>(cd, cu0, uu0, cu1, uu1);
    }
  }
  out.order = std::move(order);
  return LBM_OK;
}

}  // namespace lbm
