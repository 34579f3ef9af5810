// Host geometry builder: fluid classification and cut links with exact wall
// intersections (Sec. II.B: q = |x_W - x_F| / |c_i|, the first wall crossing
// along the segment x_F -> x_F - c_i).
//
// Shapes: spheres / disks (solid inside or outside, rigid-body wall velocity),
// circular cylinders along z (the sphere's formulas in the xy-plane), plane
// walls parallel to non-periodic faces (constant or parabolic velocity).  Many
// solid-inside spheres are bucketed on a coarse grid so that a
// link is only tested against spheres that can reach it; candidates are always
// evaluated in insertion order, spheres before face walls, and the first
// strictly smaller crossing wins.
#include <algorithm>
#include <cmath>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/lbm.h"
#include "error.hpp"
#include "lattice.hpp"

namespace {

struct Sph {
  double c[3];
  double r;
  int inside;
  double V[3], Om[3];
  double ax[3];   // axes the distance is measured along: {1, 1, 1} sphere, {1, 1, 0} cylinder along z
};

struct Face {
  int face;
  double q;
  double uw[3];
  int profile;
};

}  // namespace

struct lbm_geometry_s {
  int lattice, Q, D;
  int n[3];
  int per[3];
  int outlet;
  std::vector<Sph> sph;
  std::vector<Face> faces;
  bool built = false;
  std::vector<uint8_t> mask;
  std::vector<int64_t> node;
  std::vector<int8_t> dir;
  std::vector<double> q, uw;
  std::vector<int32_t> shape;    // owner of each link: spheres in order of addition, then faces
  int c[27][3];
};

namespace {

constexpr double kLamMin = 1e-12;   // smallest q given to a node on the wall within rounding

int gfail(int code, const std::string& m) { return lbm::set_error(code, m); }

template <class L>
void fill_c(lbm_geometry_s* g) {
  g->Q = L::Q;
  g->D = L::D;
  for (int i = 0; i < L::Q; ++i) {
    g->c[i][0] = L::cx(i);
    g->c[i][1] = L::cy(i);
    g->c[i][2] = L::cz(i);
  }
}

// minimum image on periodic axes (round half to even, as nearbyint does)
inline double min_image(const lbm_geometry_s* g, int a, double d) {
  if (!g->per[a]) return d;
  const double L = g->n[a];
  return d - L * std::nearbyint(d / L);
}

inline bool solid_or_on(const lbm_geometry_s* g, const Sph& s, const double p[3]) {
  double r2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double d = min_image(g, a, p[a] - s.c[a]) * s.ax[a];
    r2 += d * d;
  }
  const double R2 = s.r * s.r;
  return s.inside ? r2 <= R2 : r2 >= R2;
}

// first crossing lam in (0, 1] of xf - lam c with the sphere surface, NaN if none
inline double sphere_crossing(const lbm_geometry_s* g, const Sph& s, const double xf[3], const double c0[3]) {
  double dd[3], c[3];
  for (int a = 0; a < 3; ++a) {
    dd[a] = min_image(g, a, xf[a] - s.c[a]) * s.ax[a];
    c[a] = c0[a] * s.ax[a];
  }
  const double A = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
  if (!(A > 0.0)) return NAN;   // along a cylinder's axis
  const double B = dd[0] * c[0] + dd[1] * c[1] + dd[2] * c[2];
  const double C0 = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2] - s.r * s.r;
  const double disc = B * B - A * C0;
  if (!(disc >= 0.0)) return NAN;
  const double sq = std::sqrt(disc);
  const double lam = s.inside ? (B - sq) / A : (B + sq) / A;
  // a fluid node on the surface to within rounding gives a root at lam ~ 0
  if (lam > -1e-12 && lam <= 1.0 + 1e-12) return std::min(std::max(lam, kLamMin), 1.0);
  return NAN;
}

inline double face_crossing(const lbm_geometry_s* g, const Face& f, const double xf[3], const double c[3]) {
  const int a = f.face >> 1;
  if (c[a] == 0.0) return NAN;
  const double plane = (f.face & 1) ? g->n[a] - 1 + f.q : -f.q;
  const double lam = (xf[a] - plane) / c[a];
  if (lam > 0.0 && lam <= 1.0 + 1e-12) return std::min(lam, 1.0);
  return NAN;
}

int add_round(lbm_geometry g, const double centre[3], double radius, int32_t solid_inside, const double V[3],
              const double Omega[3], bool cylinder) {
  if (!g || !centre) return gfail(LBM_EINVAL, "null argument");
  if (!(radius > 0.0) || !std::isfinite(radius)) return gfail(LBM_EINVAL, "radius must be finite and > 0");
  Sph s{};
  for (int a = 0; a < 3; ++a) {
    s.c[a] = (g->lattice == LBM_D2Q9 && a == 2) ? 0.0 : centre[a];
    s.V[a] = V ? V[a] : 0.0;
    s.Om[a] = Omega ? Omega[a] : 0.0;
    s.ax[a] = (cylinder && a == 2) ? 0.0 : 1.0;
    if (!std::isfinite(s.c[a]) || !std::isfinite(s.V[a]) || !std::isfinite(s.Om[a]))
      return gfail(LBM_EINVAL, "non-finite centre or motion");
  }
  s.r = radius;
  s.inside = solid_inside ? 1 : 0;
  g->sph.push_back(s);
  g->built = false;
  return LBM_OK;
}
}  // namespace

extern "C" {

int lbm_geometry_create(int32_t lattice, int32_t nx, int32_t ny, int32_t nz, int32_t periodic, int32_t outlet_face,
                        lbm_geometry* out) {
  if (!out) return gfail(LBM_EINVAL, "null output");
  if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19 && lattice != LBM_D3Q27) return gfail(LBM_EINVAL, "invalid lattice");
  if (nx < 1 || ny < 1 || nz < 1 || (lattice == LBM_D2Q9 && nz != 1)) return gfail(LBM_EINVAL, "invalid size");
  auto* g = new lbm_geometry_s();
  g->lattice = lattice;
  if (lattice == LBM_D2Q9) {
    fill_c<D2Q9>(g);
    periodic |= 4;
  } else if (lattice == LBM_D3Q19) {
    fill_c<D3Q19>(g);
  } else {
    fill_c<D3Q27>(g);
  }
  g->n[0] = nx;
  g->n[1] = ny;
  g->n[2] = nz;
  for (int a = 0; a < 3; ++a) g->per[a] = (periodic >> a) & 1;
  if (outlet_face < -1 || outlet_face > 5 || (outlet_face >= 0 && g->per[outlet_face >> 1])) {
    delete g;
    return gfail(LBM_EINVAL, "outlet face must lie on a non-periodic axis");
  }
  g->outlet = outlet_face;
  *out = g;
  return LBM_OK;
}


int lbm_geometry_add_sphere(lbm_geometry g, const double centre[3], double radius, int32_t solid_inside,
                            const double V[3], const double Omega[3]) {
  return add_round(g, centre, radius, solid_inside, V, Omega, false);
}

int lbm_geometry_add_cylinder(lbm_geometry g, const double centre[3], double radius, int32_t solid_inside,
                              const double V[3], const double Omega[3]) {
  return add_round(g, centre, radius, solid_inside, V, Omega, true);
}

int lbm_geometry_add_spheres(lbm_geometry g, int64_t n, const double* centres, const double* radii) {
  if (!g || (n > 0 && (!centres || !radii))) return gfail(LBM_EINVAL, "null argument");
  if (n < 0) return gfail(LBM_EINVAL, "n < 0");
  for (int64_t k = 0; k < n; ++k)
    if (int e = lbm_geometry_add_sphere(g, centres + 3 * k, radii[k], 1, nullptr, nullptr)) return e;
  return LBM_OK;
}

int lbm_geometry_add_face_wall(lbm_geometry g, int32_t face, double q_face, const double uw[3], int32_t profile) {
  if (!g) return gfail(LBM_EINVAL, "null geometry");
  if (face < 0 || face > 5 || g->per[face >> 1]) return gfail(LBM_EINVAL, "face must lie on a non-periodic axis");
  if (!(q_face > 0.0 && q_face <= 1.0)) return gfail(LBM_EINVAL, "q_face must lie in (0, 1]");
  if (profile != 0 && profile != 1) return gfail(LBM_EINVAL, "profile must be 0 or 1");
  for (int a = 0; uw && a < 3; ++a)
    if (!std::isfinite(uw[a])) return gfail(LBM_EINVAL, "non-finite wall velocity");
  Face f{};
  f.face = face;
  f.q = q_face;
  for (int a = 0; a < 3; ++a) f.uw[a] = uw ? uw[a] : 0.0;
  f.profile = profile;
  g->faces.push_back(f);
  g->built = false;
  return LBM_OK;
}

int lbm_geometry_build(lbm_geometry g, int64_t* n_fluid, int64_t* n_links) {
  if (!g) return gfail(LBM_EINVAL, "null geometry");
  const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
  const int64_t N = (int64_t)nx * ny * nz;
  g->mask.assign(N, 1);
  auto idx = [&](int x, int y, int z) { return x + (int64_t)nx * (y + (int64_t)ny * z); };

  // classification
  double rmax = 0.0;
  for (const Sph& s : g->sph) {
    if (!s.inside || s.ax[2] == 0.0) {   // outside shapes and cylinders: every node
      for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
          for (int x = 0; x < nx; ++x) {
            const double p[3] = {double(x), double(y), double(z)};
            if (solid_or_on(g, s, p)) g->mask[idx(x, y, z)] = 0;
          }
      continue;
    }
    rmax = std::max(rmax, s.r);
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      if (g->D == 2 && a == 2) {
        lo[a] = hi[a] = 0;
        continue;
      }
      lo[a] = (int)std::floor(s.c[a] - s.r) - 1;
      hi[a] = (int)std::ceil(s.c[a] + s.r) + 1;
      if (!g->per[a]) {
        lo[a] = std::max(lo[a], 0);
        hi[a] = std::min(hi[a], g->n[a] - 1);
      } else if (hi[a] - lo[a] + 1 > g->n[a]) {
        lo[a] = 0;
        hi[a] = g->n[a] - 1;
      }
    }
    for (int zz = lo[2]; zz <= hi[2]; ++zz)
      for (int yy = lo[1]; yy <= hi[1]; ++yy)
        for (int xx = lo[0]; xx <= hi[0]; ++xx) {
          const int x = ((xx % nx) + nx) % nx, y = ((yy % ny) + ny) % ny, z = ((zz % nz) + nz) % nz;
          const double p[3] = {double(x), double(y), double(z)};
          if (solid_or_on(g, s, p)) g->mask[idx(x, y, z)] = 0;
        }
  }

  // buckets of solid-inside spheres (cell size >= 2 rmax + 4): a link node can
  // only cross spheres registered in its own cell
  const double cell = std::max(8.0, 2.0 * rmax + 4.0);
  int nc[3];
  for (int a = 0; a < 3; ++a) nc[a] = std::max(1, (int)std::floor(g->n[a] / cell));
  auto cell_of = [&](int a, double v) {
    int k = (int)std::floor(v / (double(g->n[a]) / nc[a]));
    return std::min(std::max(k, 0), nc[a] - 1);
  };
  std::vector<std::vector<int>> bucket((size_t)nc[0] * nc[1] * nc[2]);
  std::vector<int> outside;
  for (int k = 0; k < (int)g->sph.size(); ++k) {
    const Sph& s = g->sph[k];
    if (!s.inside || s.ax[2] == 0.0) {   // candidates of every link
      outside.push_back(k);
      continue;
    }
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      const double w = double(g->n[a]) / nc[a];
      lo[a] = (int)std::floor((s.c[a] - s.r - 2.0) / w);
      hi[a] = (int)std::floor((s.c[a] + s.r + 2.0) / w);
      if (!g->per[a]) {
        lo[a] = std::max(lo[a], 0);
        hi[a] = std::min(hi[a], nc[a] - 1);
      } else if (hi[a] - lo[a] + 1 > nc[a]) {
        lo[a] = 0;
        hi[a] = nc[a] - 1;
      }
    }
    for (int cz = lo[2]; cz <= hi[2]; ++cz)
      for (int cy = lo[1]; cy <= hi[1]; ++cy)
        for (int cx = lo[0]; cx <= hi[0]; ++cx) {
          const int X = ((cx % nc[0]) + nc[0]) % nc[0], Y = ((cy % nc[1]) + nc[1]) % nc[1], Z = ((cz % nc[2]) + nc[2]) % nc[2];
          auto& b = bucket[X + (size_t)nc[0] * (Y + (size_t)nc[1] * Z)];
          if (b.empty() || b.back() != k) b.push_back(k);
        }
  }
  for (auto& b : bucket) {
    std::sort(b.begin(), b.end());
    b.erase(std::unique(b.begin(), b.end()), b.end());
  }

  g->node.clear();
  g->dir.clear();
  g->shape.clear();
  g->q.clear();
  g->uw.clear();
  std::vector<int> cand;
  int64_t nfl = 0;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int64_t n = idx(x, y, z);
        if (!g->mask[n]) continue;
        ++nfl;
        bool have_cand = false;
        for (int i = 1; i < g->Q; ++i) {
          const int* c = g->c[i];
          int s[3] = {x - c[0], y - c[1], z - c[2]};
          bool inside = true;
          for (int a = 0; a < 3; ++a) {   // |c| <= 1: one wrap at most
            if (s[a] < 0 || s[a] >= g->n[a]) {
              if (g->per[a]) s[a] += s[a] < 0 ? g->n[a] : -g->n[a];
              else inside = false;
            }
          }
          if (inside && g->mask[idx(s[0], s[1], s[2])]) continue;
          if (!inside && g->outlet >= 0) {
            const int a = g->outlet >> 1;
            const bool beyond = (g->outlet & 1) ? s[a] >= g->n[a] : s[a] < 0;
            if (beyond) {
              int p[3] = {s[0], s[1], s[2]};
              p[a] = (g->outlet & 1) ? g->n[a] - 1 : 0;
              bool ok = true;
              for (int b = 0; b < 3; ++b) ok = ok && p[b] >= 0 && p[b] < g->n[b];
              if (ok && g->mask[idx(p[0], p[1], p[2])]) continue;   // covered by the outlet
            }
          }
          // a cut link: first crossing over all shapes
          if (!have_cand) {
            cand.clear();
            const int X = cell_of(0, x), Y = cell_of(1, y), Z = cell_of(2, z);
            const auto& b = bucket[X + (size_t)nc[0] * (Y + (size_t)nc[1] * Z)];
            std::merge(b.begin(), b.end(), outside.begin(), outside.end(), std::back_inserter(cand));
            have_cand = true;
          }
          const double xf[3] = {double(x), double(y), double(z)};
          const double cc[3] = {double(c[0]), double(c[1]), double(c[2])};
          double best = INFINITY;
          int owner = -1;
          for (int k : cand) {
            const double lam = sphere_crossing(g, g->sph[k], xf, cc);
            if (lam < best) {
              best = lam;
              owner = k;
            }
          }
          for (int k = 0; k < (int)g->faces.size(); ++k) {
            const double lam = face_crossing(g, g->faces[k], xf, cc);
            if (lam < best) {
              best = lam;
              owner = (int)g->sph.size() + k;
            }
          }
          if (owner < 0)
            return gfail(LBM_EINVAL, "no wall crossing for link (node " + std::to_string(n) + ", dir " + std::to_string(i) + ")");
          const double xw[3] = {xf[0] - best * cc[0], xf[1] - best * cc[1], xf[2] - best * cc[2]};
          double u[3] = {0, 0, 0};
          if (owner < (int)g->sph.size()) {
            const Sph& s = g->sph[owner];
            double r[3];
            for (int a = 0; a < 3; ++a) r[a] = min_image(g, a, xw[a] - s.c[a]) * s.ax[a];
            u[0] = s.V[0] + (s.Om[1] * r[2] - s.Om[2] * r[1]);
            u[1] = s.V[1] + (s.Om[2] * r[0] - s.Om[0] * r[2]);
            u[2] = s.V[2] + (s.Om[0] * r[1] - s.Om[1] * r[0]);
          } else {
            const Face& f = g->faces[owner - g->sph.size()];
            double scale = 1.0;
            if (f.profile == 1) scale = 4.0 * (xw[1] + 0.5) * (ny - 0.5 - xw[1]) / (double(ny) * ny);
            for (int a = 0; a < 3; ++a) u[a] = f.uw[a] * scale;
          }
          if (g->D == 2) u[2] = 0.0;
          g->node.push_back(n);
          g->dir.push_back((int8_t)i);
          g->shape.push_back(owner);
          g->q.push_back(best);
          g->uw.insert(g->uw.end(), u, u + 3);
        }
      }
  g->built = true;
  if (n_fluid) *n_fluid = nfl;
  if (n_links) *n_links = (int64_t)g->node.size();
  return LBM_OK;
}

int lbm_geometry_get(lbm_geometry g, uint8_t* mask, int64_t* node, int8_t* dir, double* q, double* uw_t, double* uw_t1) {
  if (!g) return gfail(LBM_EINVAL, "null geometry");
  if (!g->built) return gfail(LBM_ESTATE, "geometry not built");
  if (mask) std::copy(g->mask.begin(), g->mask.end(), mask);
  if (node) std::copy(g->node.begin(), g->node.end(), node);
  if (dir) std::copy(g->dir.begin(), g->dir.end(), dir);
  if (q) std::copy(g->q.begin(), g->q.end(), q);
  if (uw_t) std::copy(g->uw.begin(), g->uw.end(), uw_t);
  if (uw_t1) std::copy(g->uw.begin(), g->uw.end(), uw_t1);
  return LBM_OK;
}

int lbm_geometry_get_shapes(lbm_geometry g, int32_t* shape) {
  if (!g) return gfail(LBM_EINVAL, "null geometry");
  if (!g->built) return gfail(LBM_ESTATE, "geometry not built");
  if (!shape && !g->shape.empty()) return gfail(LBM_EINVAL, "null shape array");
  std::copy(g->shape.begin(), g->shape.end(), shape);
  return LBM_OK;
}

int lbm_geometry_free(lbm_geometry g) {
  if (!g) return gfail(LBM_EINVAL, "null geometry");
  delete g;
  return LBM_OK;
}

}  // extern "C"
