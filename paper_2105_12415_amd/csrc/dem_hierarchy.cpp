// dem_build_hierarchy: offline construction of a particle's surrogate tree
// arrays with conservative epsilons (Section 4, surrogate tree definition and
// Definition "conservative"; Appendix B, Algorithm 7).  Host code, FP64.
//
// The tree topology (which coarse triangle stands in for which finer ones)
// comes from the caller, e.g. the nesting of a subdivided icosphere.  For
// each surrogate s the builder computes
//     eps(s) = eps0 + max over vertices v of fine descendants of dist(v, s),
// the smallest epsilon for which s's environment contains the eps0
// environment of every fine triangle under s: the distance to s is convex,
// so its maximum over a fine triangle is attained at one of the vertices.
// This holds per surrogate, independently of the epsilons of intermediate
// levels, so the cascade needs not be monotone (Section 4 corollary).
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <new>
#include <vector>

#include "dem.h"
#include "dem_geom.hpp"

namespace {

double point_tri_dist(const double* p, const double* a, const double* b, const double* c) {
  using dem::V3;
  V3<double> x{p[0], p[1], p[2]}, A{a[0], a[1], a[2]}, B{b[0], b[1], b[2]}, C{c[0], c[1], c[2]};
  V3<double> q;
  double w[3];
  double d2 = dem::point_tri(x, A, B - A, C - A, q, w);
  return std::sqrt(d2);
}

template <typename X>
X* alloc(size_t n) {
  return static_cast<X*>(std::calloc(n ? n : 1, sizeof(X)));
}

}  // namespace

extern "C" {

dem_status dem_build_hierarchy(const double* verts, int32_t n_verts, const int32_t* tris,
                               const int32_t* parent, const int32_t* level_sizes, int32_t n_levels,
                               double eps0, const dem_build_opts* opts, dem_hierarchy* out) {
  if (!out) return DEM_ERR_ARG;
  std::memset(out, 0, sizeof(*out));
  if (!verts || !tris || !level_sizes || n_verts <= 0 || n_levels < 1 || n_levels > DEM_MAX_LEVELS)
    return DEM_ERR_ARG;
  if (n_levels > 1 && !parent) return DEM_ERR_ARG;
  if (!(eps0 >= 0.0) || !std::isfinite(eps0)) return DEM_ERR_ARG;
  double coord_scale = opts ? opts->coord_scale : 0.0;
  double rel_slack = opts ? opts->rel_slack : 1e-6;
  if (!(coord_scale >= 0.0) || !(rel_slack >= 0.0)) return DEM_ERR_ARG;
  std::vector<int64_t> lb(n_levels + 1, 0);
  for (int l = 0; l < n_levels; ++l) {
    if (level_sizes[l] <= 0) return DEM_ERR_ARG;
    lb[l + 1] = lb[l] + level_sizes[l];
  }
  if (lb[n_levels] > std::numeric_limits<int32_t>::max()) return DEM_ERR_ARG;
  const int32_t n = (int32_t)lb[n_levels];
  for (int64_t i = 0; i < 3 * (int64_t)n; ++i)
    if (tris[i] < 0 || tris[i] >= n_verts) return DEM_ERR_ARG;
  double maxc = 0.0;
  for (int64_t i = 0; i < 3 * (int64_t)n_verts; ++i) {
    if (!std::isfinite(verts[i])) return DEM_ERR_ARG;
    maxc = std::fmax(maxc, std::fabs(verts[i]));
  }
  if (coord_scale == 0.0) coord_scale = maxc;

  // children ranges from the parent links: a surrogate of level l >= 1 hangs
  // below level l-1; a fine triangle (last level) below a surrogate of any
  // level (trees whose leaf sets sit at different depths)
  std::vector<int32_t> cb(n, 0), cc(n, 0);
  for (int l = 1; l < n_levels; ++l) {
    const int64_t lo = (l == n_levels - 1) ? 0 : lb[l - 1];
    int32_t prev = -1;
    for (int64_t t = lb[l]; t < lb[l + 1]; ++t) {
      int32_t p = parent[t];
      if (p < lo || p >= lb[l]) return DEM_ERR_NOT_CONSERVATIVE;
      if (p < prev) return DEM_ERR_NOT_CONSERVATIVE;  // children must be grouped by parent
      if (p != prev) {
        if (cc[p] != 0) return DEM_ERR_NOT_CONSERVATIVE;
        cb[p] = (int32_t)t;
      }
      cc[p]++;
      prev = p;
    }
  }
  for (int l = 0; l + 1 < n_levels; ++l)
    for (int64_t t = lb[l]; t < lb[l + 1]; ++t) {
      if (cc[t] == 0) return DEM_ERR_NOT_CONSERVATIVE;  // leaves only on the last level
      if (cc[t] > DEM_MAX_CHILDREN) return DEM_ERR_ARG;
    }

  // deviations: every fine vertex against every ancestor
  std::vector<double> dev(n, 0.0);
  for (int64_t f = lb[n_levels - 1]; f < n; ++f) {
    for (int32_t s = n_levels > 1 ? parent[f] : -1; s >= 0; s = (s >= lb[1] ? parent[s] : -1)) {
      const double* a = verts + 3 * (int64_t)tris[3 * (int64_t)s];
      const double* b = verts + 3 * (int64_t)tris[3 * (int64_t)s + 1];
      const double* c = verts + 3 * (int64_t)tris[3 * (int64_t)s + 2];
      for (int k = 0; k < 3; ++k) {
        const double* v = verts + 3 * (int64_t)tris[3 * f + k];
        double d = point_tri_dist(v, a, b, c);
        if (d > dev[s]) dev[s] = d;
      }
    }
  }

  out->n_tris = n;
  out->n_levels = n_levels;
  out->tri_verts = alloc<int32_t>(3 * (size_t)n);
  out->child_begin = alloc<int32_t>(n);
  out->child_count = alloc<int32_t>(n);
  out->level_begin = alloc<int32_t>(n_levels + 1);
  out->eps = alloc<double>(n);
  out->eps_f32 = alloc<float>(n);
  out->eps_f64 = alloc<double>(n);
  if (!out->tri_verts || !out->child_begin || !out->child_count || !out->level_begin || !out->eps ||
      !out->eps_f32 || !out->eps_f64) {
    dem_hierarchy_free(out);
    return DEM_ERR_OOM;
  }
  std::memcpy(out->tri_verts, tris, 3 * sizeof(int32_t) * (size_t)n);
  std::memcpy(out->child_begin, cb.data(), sizeof(int32_t) * (size_t)n);
  std::memcpy(out->child_count, cc.data(), sizeof(int32_t) * (size_t)n);
  for (int l = 0; l <= n_levels; ++l) out->level_begin[l] = (int32_t)lb[l];
  const double abs_slack = coord_scale * std::ldexp(1.0, -19);
  double max_dev = 0.0;
  for (int32_t t = 0; t < n; ++t) {
    bool fine = cc[t] == 0;
    double e = fine ? eps0 : eps0 + dev[t];
    out->eps[t] = e;
    double es = fine ? e : e * (1.0 + rel_slack) + abs_slack;
    out->eps_f64[t] = es;
    float f = (float)es;
    if ((double)f < es) f = std::nextafter(f, std::numeric_limits<float>::infinity());
    out->eps_f32[t] = f;
    if (!fine && dev[t] > max_dev) max_dev = dev[t];
  }
  out->root_begin = 0;
  out->root_count = (int32_t)(lb[1] - lb[0]);
  out->fine_begin = (int32_t)lb[n_levels - 1];
  out->fine_count = (int32_t)(lb[n_levels] - lb[n_levels - 1]);
  out->max_dev = max_dev;
  return DEM_OK;
}

void dem_hierarchy_free(dem_hierarchy* h) {
  if (!h) return;
  std::free(h->tri_verts);
  std::free(h->child_begin);
  std::free(h->child_count);
  std::free(h->level_begin);
  std::free(h->eps);
  std::free(h->eps_f32);
  std::free(h->eps_f64);
  std::memset(h, 0, sizeof(*h));
}

}  // extern "C"
