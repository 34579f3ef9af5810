// Host-only driver of the geometry builder and the link planner, built with
// g++ and the address / undefined-behaviour sanitizers (no GPU, no HIP).
//
// Reads commands from stdin, one per line (reals as C99 hex floats, so the
// values are exact):
//   geom LATTICE NX NY NZ PERIODIC OUTLET
//   sphere|cylinder CX CY CZ R INSIDE VX VY VZ OX OY OZ
//   spheres N            followed by N lines "CX CY CZ R"
//   face F Q UX UY UZ PROFILE
//   build PREFIX         build; write PREFIX.{mask,node,dir,q,uw,uw1,shape}
//   plan VARIANT QCUT F64  plan the built links, check the records, then check
//                        that every corrupted copy of the list is refused
//   bad                  invalid calls of the builder API (each must be refused)
//   end                  free the geometry
// Prints one line per command; any failed check prints "FAIL ..." and the
// program exits with status 1.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <iostream>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "../../paper_2009_04604_amd/csrc/error.hpp"
#include "../../paper_2009_04604_amd/csrc/hostplan.hpp"
#include "../../paper_2009_04604_amd/csrc/lattice.hpp"

namespace lbm {
thread_local std::string g_msg;
int set_error(int code, const std::string& msg) {
  g_msg = msg;
  return code;
}
void clear_error() { g_msg.clear(); }
}  // namespace lbm

namespace {

int g_failures = 0;

#define CHECK(cond, ...)                    \
  do {                                      \
    if (!(cond)) {                          \
      std::printf("FAIL %s: ", #cond);      \
      std::printf(__VA_ARGS__);             \
      std::printf("\n");                    \
      ++g_failures;                         \
    }                                       \
  } while (0)

double real(const std::string& s) { return std::strtod(s.c_str(), nullptr); }

struct Built {
  int lattice = 0, n[3] = {0, 0, 0}, periodic = 0, outlet = -1;
  std::vector<uint8_t> mask;
  std::vector<int64_t> node;
  std::vector<int8_t> dir;
  std::vector<double> q, uw, uw1;
};

template <typename T>
void dump(const std::string& path, const std::vector<T>& v) {
  FILE* f = std::fopen(path.c_str(), "wb");
  if (!f) {
    std::printf("FAIL cannot write %s\n", path.c_str());
    std::exit(1);
  }
  if (!v.empty()) std::fwrite(v.data(), sizeof(T), v.size(), f);
  std::fclose(f);
}

int lattice_q(int lattice) { return lattice == LBM_D2Q9 ? 9 : (lattice == LBM_D3Q19 ? 19 : 27); }

void direction(int lattice, int i, int c[3]) {
  if (lattice == LBM_D2Q9) {
    c[0] = D2Q9::cx(i), c[1] = D2Q9::cy(i), c[2] = D2Q9::cz(i);
  } else if (lattice == LBM_D3Q19) {
    c[0] = D3Q19::cx(i), c[1] = D3Q19::cy(i), c[2] = D3Q19::cz(i);
  } else {
    c[0] = D3Q27::cx(i), c[1] = D3Q27::cy(i), c[2] = D3Q27::cz(i);
  }
}

// Every stored record agrees with the caller's list it was planned from.
void check_plan(const lbm::HostGrid& g, const Built& b, const lbm::LinkPlan& p) {
  const int64_t nl = (int64_t)b.node.size();
  CHECK((int64_t)p.order.size() == nl, "order size");
  std::vector<int64_t> seen(p.order);
  std::sort(seen.begin(), seen.end());
  for (int64_t k = 0; k < nl; ++k) CHECK(seen[k] == k, "order is not a permutation at %lld", (long long)k);
  CHECK((int64_t)p.seg_lbase.size() == g.nseg + 1 && p.seg_lbase[g.nseg] == nl, "segment link counts");
  int64_t nb = 0;
  for (int64_t s = 0; s < g.nseg; ++s) {
    CHECK(p.seg_lbase[s] <= p.seg_lbase[s + 1], "seg_lbase not monotone at %lld", (long long)s);
    nb += __builtin_popcountll(p.seg_bnd[s]);
  }
  CHECK(nb == p.n_boundary, "boundary count %lld vs %lld", (long long)nb, (long long)p.n_boundary);
  for (int64_t k = 0; k < nl; ++k) {
    const int64_t o = p.order[k];
    const int64_t n = b.node[o];
    if (k > 0) {
      const int64_t po = p.order[k - 1];
      CHECK(b.node[po] < n || (b.node[po] == n && b.dir[po] < b.dir[o]), "links not sorted at %lld", (long long)k);
    }
    CHECK(p.lnode[k] == n, "lnode at %lld", (long long)k);
    const int64_t row = n / g.n[0];
    const int x = (int)(n - row * g.n[0]);
    const int64_t s = row * g.nseg_x + x / lbm::SEG;
    CHECK((p.lld[k] & 0xff) == x % lbm::SEG && (p.lld[k] >> 8) == b.dir[o], "lld at %lld", (long long)k);
    CHECK(p.seg_lbase[s] <= k && k < p.seg_lbase[s + 1], "link %lld outside its segment's range", (long long)k);
    CHECK((p.seg_bnd[s] >> (x % lbm::SEG)) & 1ull, "boundary bit of link %lld", (long long)k);
    CHECK(p.q[k] == b.q[o], "q at %lld", (long long)k);
    if (p.moving)
      for (int a = 0; a < 3; ++a) {
        if (a == 2 && b.lattice == LBM_D2Q9) continue;
        CHECK(p.uv[a * nl + k] == b.uw[3 * o + a] && p.uv[(3 + a) * nl + k] == b.uw1[3 * o + a], "uv at %lld",
              (long long)k);
      }
    if (p.uw_any)
      for (int a = 0; a < 3; ++a) CHECK(p.uw[3 * k + a] == b.uw[3 * o + a], "uw at %lld", (long long)k);
  }
}

// Expect plan_links to refuse the list with a message containing `what`.
void expect_refused(const lbm::HostGrid& g, const char* name, std::vector<int64_t> node, std::vector<int8_t> dir,
                    std::vector<double> q, std::vector<double> uw, std::vector<double> uw1, int variant, double qcut,
                    const char* what) {
  lbm::LinkPlan p;
  lbm::g_msg.clear();
  const int rc = lbm::plan_links(g, (int64_t)node.size(), node.data(), dir.data(), q.data(), uw.data(), uw1.data(),
                                 variant, qcut, true, p);
  CHECK(rc == LBM_EINVAL, "%s: accepted", name);
  CHECK(lbm::g_msg.find(what) != std::string::npos, "%s: message '%s' lacks '%s'", name, lbm::g_msg.c_str(), what);
}

void plan_case(const Built& b, int variant, double qcut, bool f64) {
  const int periodic = b.periodic | (b.lattice == LBM_D2Q9 ? 4 : 0);
  const lbm::HostGrid g =
      lbm::make_host_grid(b.lattice, b.n[0], b.n[1], b.n[2], periodic, b.outlet, b.mask.data());
  const int64_t nl = (int64_t)b.node.size();
  lbm::LinkPlan p;
  int rc = lbm::plan_links(g, nl, b.node.data(), b.dir.data(), b.q.data(), b.uw.data(), b.uw1.data(), variant,
                           qcut, f64, p);
  CHECK(rc == LBM_OK, "builder's links refused: %s", lbm::g_msg.c_str());
  if (rc != LBM_OK) return;
  check_plan(g, b, p);
  // the same list in another order gives the same records
  std::vector<int64_t> perm(nl);
  std::iota(perm.begin(), perm.end(), 0);
  std::shuffle(perm.begin(), perm.end(), std::mt19937_64(12345));
  Built s = b;
  for (int64_t k = 0; k < nl; ++k) {
    s.node[k] = b.node[perm[k]];
    s.dir[k] = b.dir[perm[k]];
    s.q[k] = b.q[perm[k]];
    for (int a = 0; a < 3; ++a) {
      s.uw[3 * k + a] = b.uw[3 * perm[k] + a];
      s.uw1[3 * k + a] = b.uw1[3 * perm[k] + a];
    }
  }
  lbm::LinkPlan ps;
  rc = lbm::plan_links(g, nl, s.node.data(), s.dir.data(), s.q.data(), s.uw.data(), s.uw1.data(), variant, qcut,
                       f64, ps);
  CHECK(rc == LBM_OK, "shuffled list refused");
  if (rc == LBM_OK) {
    check_plan(g, s, ps);
    CHECK(ps.lld == p.lld && ps.lnode == p.lnode && ps.seg_bnd == p.seg_bnd && ps.seg_lbase == p.seg_lbase &&
              ps.q == p.q && ps.gw == p.gw && ps.uv == p.uv,
          "records depend on the input order");
  }
  // corrupted copies
  const int Q = lattice_q(b.lattice);
  if (nl > 0) {
    auto n = b.node;
    auto d = b.dir;
    auto q = b.q;
    auto u = b.uw;
    auto u1 = b.uw1;
    n.push_back(n[0]);
    d.push_back(d[0]);
    q.push_back(q[0]);
    for (int a = 0; a < 3; ++a) {
      u.push_back(u[a]);
      u1.push_back(u1[a]);
    }
    expect_refused(g, "duplicate", n, d, q, u, u1, variant, qcut, "duplicate link");
    struct Mut {
      const char* name;
      int field;   // 0 node, 1 dir, 2 q, 3 uw
      double value;
      const char* what;
    } muts[] = {{"node -1", 0, -1, "node out of range"},
                {"node N", 0, (double)g.N, "node out of range"},
                {"dir 0", 1, 0, "dir out of range"},
                {"dir Q", 1, (double)Q, "dir out of range"},
                {"q 0", 2, 0.0, "q must lie in (0, 1]"},
                {"q > 1", 2, 1.5, "q must lie in (0, 1]"},
                {"q NaN", 2, std::nan(""), "q must lie in (0, 1]"},
                {"uw inf", 3, INFINITY, "non-finite uw_t"}};
    const int64_t k = nl / 2;
    for (const Mut& m : muts) {
      auto n2 = b.node;
      auto d2 = b.dir;
      auto q2 = b.q;
      auto u2 = b.uw;
      if (m.field == 0) n2[k] = (int64_t)m.value;
      if (m.field == 1) d2[k] = (int8_t)m.value;
      if (m.field == 2) q2[k] = m.value;
      if (m.field == 3) u2[3 * k] = m.value;
      expect_refused(g, m.name, n2, d2, q2, u2, b.uw1, variant, qcut, m.what);
    }
    // one link missing: its population is not covered
    auto n3 = b.node;
    auto d3 = b.dir;
    auto q3 = b.q;
    auto u3 = b.uw;
    auto v3 = b.uw1;
    n3.erase(n3.begin() + k);
    d3.erase(d3.begin() + k);
    q3.erase(q3.begin() + k);
    u3.erase(u3.begin() + 3 * k, u3.begin() + 3 * k + 3);
    v3.erase(v3.begin() + 3 * k, v3.begin() + 3 * k + 3);
    expect_refused(g, "missing link", n3, d3, q3, u3, v3, variant, qcut, "not covered by a link");
  }
  // a solid node, and a fluid node whose pull source against some direction is
  // a fluid node (so that direction is streamed, not a cut link)
  int64_t solid = -1, inner = -1;
  int inner_dir = 0;
  for (int64_t n = 0; n < g.N && (solid < 0 || inner < 0); ++n) {
    if (!b.mask[n]) {
      if (solid < 0) solid = n;
      continue;
    }
    if (inner >= 0) continue;
    const int x = (int)(n % b.n[0]), y = (int)((n / b.n[0]) % b.n[1]), z = (int)(n / ((int64_t)b.n[0] * b.n[1]));
    for (int i = 1; i < Q && inner < 0; ++i) {
      int c[3], s[3];
      direction(b.lattice, i, c);
      if (lbm::pull_source(g, c, x, y, z, s) && b.mask[s[0] + (int64_t)b.n[0] * (s[1] + (int64_t)b.n[1] * s[2])]) {
        inner = n;
        inner_dir = i;
      }
    }
  }
  auto with_extra = [&](int64_t node, int dir, const char* name, const char* what) {
    std::vector<int64_t> n = b.node;
    std::vector<int8_t> d = b.dir;
    std::vector<double> q = b.q, u = b.uw, u1 = b.uw1;
    n.push_back(node);
    d.push_back((int8_t)dir);
    q.push_back(0.5);
    for (int a = 0; a < 3; ++a) {
      u.push_back(0.0);
      u1.push_back(0.0);
    }
    expect_refused(g, name, n, d, q, u, u1, variant, qcut, what);
  };
  if (solid >= 0) with_extra(solid, 1, "solid node", "node is not fluid");
  if (inner >= 0) with_extra(inner, inner_dir, "streamed direction", "is a fluid node (not a cut link)");
  std::printf("plan ok links %lld boundary %lld moving %d\n", (long long)nl, (long long)p.n_boundary,
              (int)p.moving);
}

void bad_calls() {
  lbm_geometry g = nullptr;
  CHECK(lbm_geometry_create(7, 8, 8, 1, 7, -1, &g) == LBM_EINVAL, "bad lattice accepted");
  CHECK(lbm_geometry_create(LBM_D2Q9, 0, 8, 1, 7, -1, &g) == LBM_EINVAL, "nx 0 accepted");
  CHECK(lbm_geometry_create(LBM_D2Q9, 8, 8, 1, 7, -1, nullptr) == LBM_EINVAL, "null out accepted");
  CHECK(lbm_geometry_create(LBM_D2Q9, 8, 8, 1, 7, -1, &g) == LBM_OK, "valid create refused");
  const double c[3] = {4, 4, 0}, nanc[3] = {NAN, 4, 0};
  CHECK(lbm_geometry_add_sphere(g, c, -1.0, 1, nullptr, nullptr) == LBM_EINVAL, "negative radius accepted");
  CHECK(lbm_geometry_add_sphere(g, c, NAN, 1, nullptr, nullptr) == LBM_EINVAL, "NaN radius accepted");
  CHECK(lbm_geometry_add_sphere(g, nanc, 2.0, 1, nullptr, nullptr) == LBM_EINVAL, "NaN centre accepted");
  CHECK(lbm_geometry_add_cylinder(g, nullptr, 2.0, 1, nullptr, nullptr) == LBM_EINVAL, "null centre accepted");
  CHECK(lbm_geometry_add_spheres(g, -1, c, c) == LBM_EINVAL, "negative sphere count accepted");
  CHECK(lbm_geometry_add_face_wall(g, 0, 0.5, nullptr, 0) == LBM_EINVAL, "face wall on a periodic axis accepted");
  CHECK(lbm_geometry_add_face_wall(g, 9, 0.5, nullptr, 0) == LBM_EINVAL, "face 9 accepted");
  lbm_geometry h = nullptr;
  CHECK(lbm_geometry_create(LBM_D2Q9, 8, 8, 1, 1, -1, &h) == LBM_OK, "valid create refused");
  const double inf3[3] = {INFINITY, 0, 0};
  CHECK(lbm_geometry_add_face_wall(h, 2, 0.0, nullptr, 0) == LBM_EINVAL, "q_face 0 accepted");
  CHECK(lbm_geometry_add_face_wall(h, 2, 0.5, nullptr, 2) == LBM_EINVAL, "profile 2 accepted");
  CHECK(lbm_geometry_add_face_wall(h, 2, 0.5, inf3, 0) == LBM_EINVAL, "infinite wall velocity accepted");
  CHECK(lbm_geometry_add_face_wall(h, 2, 0.5, nullptr, 0) == LBM_OK, "valid face wall refused");
  CHECK(lbm_geometry_free(h) == LBM_OK, "free");
  int64_t nf = 0, nl = 0;
  CHECK(lbm_geometry_get(g, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) != LBM_OK, "get before build");
  CHECK(lbm_geometry_build(g, &nf, &nl) == LBM_OK, "empty build refused");
  CHECK(nf == 64 && nl == 0, "empty geometry: %lld fluid, %lld links", (long long)nf, (long long)nl);
  CHECK(lbm_geometry_free(g) == LBM_OK, "free");
  std::printf("bad ok\n");
}

// The compact layout's source-row table: for every fluid node and direction
// whose pull source is a fluid node (or the node an outlet face clamps it
// onto), the slot the step kernel forms from it (the source row's segment,
// its fluid lanes below, the row-end wrap) equals that node's slot counted
// directly.
void check_source_rows(const Built& b) {
  const int periodic = b.periodic | (b.lattice == LBM_D2Q9 ? 4 : 0);
  const lbm::HostGrid g =
      lbm::make_host_grid(b.lattice, b.n[0], b.n[1], b.n[2], periodic, b.outlet, b.mask.data());
  std::vector<uint64_t> fluid;
  std::vector<int32_t> fbase;
  lbm::segment_index(g, fluid, fbase);
  std::vector<int32_t> rows;
  lbm::source_rows(g, rows);
  const int nr = lbm::source_rows_per_row(b.lattice);
  CHECK((int64_t)rows.size() == (int64_t)g.n[1] * g.n[2] * nr, "table size");
  std::vector<int64_t> slot(g.N, -1);
  int64_t nf = 0;
  for (int64_t n = 0; n < g.N; ++n)
    if (b.mask[n]) slot[n] = lbm::GUARD + nf++;
  const int Q = lattice_q(b.lattice);
  const int64_t nsx = g.nseg_x;
  int64_t checked = 0;
  for (int z = 0; z < g.n[2]; ++z)
    for (int y = 0; y < g.n[1]; ++y)
      for (int x = 0; x < g.n[0]; ++x) {
        const int64_t n = x + (int64_t)g.n[0] * (y + (int64_t)g.n[1] * z);
        if (!b.mask[n]) continue;
        const int64_t r = y + (int64_t)g.n[1] * z, sx = x / lbm::SEG;
        const int lane = x % lbm::SEG;
        const bool edge = sx == 0 || sx == nsx - 1, wrap = edge && g.per[0];
        const bool xlo = edge && x == 0, xhi = edge && x == g.n[0] - 1;
        for (int i = 0; i < Q; ++i) {
          int c[3], s[3];
          direction(b.lattice, i, c);
          const bool inside = lbm::pull_source(g, c, x, y, z, s);
          int64_t src = -1;
          if (inside) {
            const int64_t m = s[0] + (int64_t)g.n[0] * (s[1] + (int64_t)g.n[1] * s[2]);
            if (b.mask[m]) src = m;
          } else {
            src = lbm::outlet_producer(g, s);
          }
          if (src < 0) continue;
          const int k = b.lattice == LBM_D2Q9 ? 1 + c[1] : 3 * (1 + c[1]) + (1 + c[2]);
          const int64_t seg = rows[r * nr + k] + sx;
          CHECK(seg >= 0 && seg < g.nseg, "source segment out of range");
          const uint64_t fm = fluid[seg];
          const int64_t f0 = fbase[seg] + lbm::GUARD, s0 = seg - sx;
          const int64_t edge = sx == 0 ? fbase[s0 + nsx] + lbm::GUARD - 1 : fbase[s0] + lbm::GUARD;
          const uint64_t below = lane ? (fm & ((1ull << lane) - 1)) : 0;
          const int64_t P = f0 + __builtin_popcountll(below);
          const int64_t B = (int64_t)((fm >> lane) & 1ull);
          const int64_t lo = wrap ? edge : P, hi = wrap ? (nsx == 1 ? f0 : edge) : P;
          const int64_t got = c[0] == 0 ? P : (c[0] == 1 ? (xlo ? lo : P - 1) : (xhi ? hi : P + B));
          CHECK(got == slot[src], "compact slot of node %lld dir %d: %lld, expected %lld", (long long)n, i,
                (long long)got, (long long)slot[src]);
          ++checked;
        }
      }
  // every lane of every segment (also lanes that are not fluid and lanes past
  // the row's end, which the compact step lets pull too) and every direction
  // (also cut links) reads inside the population array
  const int64_t npad = (lbm::GUARD + nf + 1 + 63) / 64 * 64;
  int64_t ranged = 0;
  for (int z = 0; z < g.n[2]; ++z)
    for (int y = 0; y < g.n[1]; ++y)
      for (int64_t sx = 0; sx < nsx; ++sx)
        for (int lane = 0; lane < lbm::SEG; ++lane) {
          const int64_t r = y + (int64_t)g.n[1] * z, x = sx * lbm::SEG + lane;
          const bool edge = sx == 0 || sx == nsx - 1, wrap = edge && g.per[0];
          const bool xlo = edge && x == 0, xhi = edge && x == g.n[0] - 1;
          for (int i = 0; i < Q; ++i) {
            int c[3];
            direction(b.lattice, i, c);
            const int k = b.lattice == LBM_D2Q9 ? 1 + c[1] : 3 * (1 + c[1]) + (1 + c[2]);
            const int64_t seg = rows[r * nr + k] + sx;
            CHECK(seg >= 0 && seg < g.nseg, "source segment out of range");
            const uint64_t fm = fluid[seg];
            const int64_t f0 = fbase[seg] + lbm::GUARD, s0 = seg - sx;
            const int64_t ed = sx == 0 ? fbase[s0 + nsx] + lbm::GUARD - 1 : fbase[s0] + lbm::GUARD;
            const uint64_t below = lane ? (fm & ((1ull << lane) - 1)) : 0;
            const int64_t P = f0 + __builtin_popcountll(below);
            const int64_t B = (int64_t)((fm >> lane) & 1ull);
            const int64_t lo = wrap ? ed : P, hi = wrap ? (nsx == 1 ? f0 : ed) : P;
            const int64_t got = c[0] == 0 ? P : (c[0] == 1 ? (xlo ? lo : P - 1) : (xhi ? hi : P + B));
            CHECK(got >= 0 && got < npad, "pull of lane %d segment %lld dir %d at slot %lld outside [0, %lld)", lane,
                  (long long)seg, i, (long long)got, (long long)npad);
            ++ranged;
          }
        }
  std::printf("source rows ok %lld in range %lld\n", (long long)checked, (long long)ranged);
}

}  // namespace

int main() {
  lbm_geometry g = nullptr;
  Built b;
  std::string cmd;
  while (std::cin >> cmd) {
    if (cmd == "geom") {
      std::cin >> b.lattice >> b.n[0] >> b.n[1] >> b.n[2] >> b.periodic >> b.outlet;
      const int rc = lbm_geometry_create(b.lattice, b.n[0], b.n[1], b.n[2], b.periodic, b.outlet, &g);
      CHECK(rc == LBM_OK, "create: %s", lbm::g_msg.c_str());
      std::printf("geom ok\n");
    } else if (cmd == "sphere" || cmd == "cylinder") {
      std::string t[11];
      int inside = 0;
      std::cin >> t[0] >> t[1] >> t[2] >> t[3] >> inside >> t[4] >> t[5] >> t[6] >> t[7] >> t[8] >> t[9];
      const double c[3] = {real(t[0]), real(t[1]), real(t[2])}, V[3] = {real(t[4]), real(t[5]), real(t[6])},
                   O[3] = {real(t[7]), real(t[8]), real(t[9])};
      const int rc = cmd == "sphere" ? lbm_geometry_add_sphere(g, c, real(t[3]), inside, V, O)
                                     : lbm_geometry_add_cylinder(g, c, real(t[3]), inside, V, O);
      CHECK(rc == LBM_OK, "%s: %s", cmd.c_str(), lbm::g_msg.c_str());
      std::printf("%s ok\n", cmd.c_str());
    } else if (cmd == "spheres") {
      int64_t n = 0;
      std::cin >> n;
      std::vector<double> c(3 * n), r(n);
      for (int64_t k = 0; k < n; ++k) {
        std::string t[4];
        std::cin >> t[0] >> t[1] >> t[2] >> t[3];
        for (int a = 0; a < 3; ++a) c[3 * k + a] = real(t[a]);
        r[k] = real(t[3]);
      }
      CHECK(lbm_geometry_add_spheres(g, n, c.data(), r.data()) == LBM_OK, "spheres: %s", lbm::g_msg.c_str());
      std::printf("spheres ok %lld\n", (long long)n);
    } else if (cmd == "face") {
      int f = 0, profile = 0;
      std::string t[4];
      std::cin >> f >> t[0] >> t[1] >> t[2] >> t[3] >> profile;
      const double u[3] = {real(t[1]), real(t[2]), real(t[3])};
      CHECK(lbm_geometry_add_face_wall(g, f, real(t[0]), u, profile) == LBM_OK, "face: %s", lbm::g_msg.c_str());
      std::printf("face ok\n");
    } else if (cmd == "build") {
      std::string prefix;
      std::cin >> prefix;
      int64_t nf = 0, nl = 0;
      const int rc = lbm_geometry_build(g, &nf, &nl);
      CHECK(rc == LBM_OK, "build: %s", lbm::g_msg.c_str());
      const int64_t N = (int64_t)b.n[0] * b.n[1] * b.n[2];
      b.mask.assign(N, 0);
      b.node.assign(nl, 0);
      b.dir.assign(nl, 0);
      b.q.assign(nl, 0);
      b.uw.assign(3 * nl, 0);
      b.uw1.assign(3 * nl, 0);
      std::vector<int32_t> shape(nl);
      CHECK(lbm_geometry_get(g, b.mask.data(), b.node.data(), b.dir.data(), b.q.data(), b.uw.data(), b.uw1.data()) ==
                LBM_OK,
            "get");
      CHECK(lbm_geometry_get_shapes(g, shape.data()) == LBM_OK, "shapes");
      dump(prefix + ".mask", b.mask);
      dump(prefix + ".node", b.node);
      dump(prefix + ".dir", b.dir);
      dump(prefix + ".q", b.q);
      dump(prefix + ".uw", b.uw);
      dump(prefix + ".uw1", b.uw1);
      dump(prefix + ".shape", shape);
      std::printf("built %lld %lld\n", (long long)nf, (long long)nl);
    } else if (cmd == "plan") {
      int variant = 0, f64 = 1;
      std::string qc;
      std::cin >> variant >> qc >> f64;
      plan_case(b, variant, real(qc), f64 != 0);
      check_source_rows(b);
    } else if (cmd == "bad") {
      bad_calls();
    } else if (cmd == "end") {
      CHECK(lbm_geometry_free(g) == LBM_OK, "free");
      g = nullptr;
      std::printf("end ok\n");
    } else {
      std::printf("FAIL unknown command %s\n", cmd.c_str());
      return 1;
    }
    std::fflush(stdout);
  }
  if (g) lbm_geometry_free(g);
  std::printf(g_failures ? "FAILURES %d\n" : "ALL OK\n", g_failures);
  return g_failures ? 1 : 0;
}
