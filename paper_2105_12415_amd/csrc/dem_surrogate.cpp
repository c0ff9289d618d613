// dem_build_surrogate_tree: offline construction of a surrogate tree for a
// generic triangulated particle (Appendix B, Algorithm 7; surrogate triangles
// by the functional of Appendix A).  Host code, FP64.
//
// Top-down: the root surrogate stands for the whole mesh; a set with more
// than N_surrogate triangles is split into N_surrogate subsets by k-means on
// the triangle centroids, each subset gets its own surrogate, and so on; a
// set of at most N_surrogate triangles becomes the children of its
// surrogate.  Surrogates are numbered depth by depth (so the children of one
// surrogate are contiguous), the fine triangles follow, grouped by parent.
//
// The surrogate triangle x1, x2, x3 of a set T minimises
//   (1/b_s) sum_{x, t in T} |x - t|^b_s            (small: b_s high ~ max)
// + (a_a/2) |(x2 - x1) x (x3 - x1)|^-2             (not a point or a line)
// + (a_i/b_n) sum_{x, vertices v of T} max(0, (x - v).N)^b_n   (inside)
// with N the unit normal oriented like the set's area-weighted normal,
// starting from the triangle of T nearest the set's centre.  Coordinates are
// scaled by the set's radius, which makes the weights dimensionless.  The
// surrogate's epsilon is not chosen here: dem_build_hierarchy computes the
// smallest conservative one for whatever triangle this yields, so the fit
// only decides how well the surrogate prunes, never correctness.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "dem.h"
#include "dem_geom.hpp"

namespace {

using dem::V3;
using P3 = V3<double>;

P3 at(const double* v, int i) { return P3{v[3 * i], v[3 * i + 1], v[3 * i + 2]}; }
double norm(P3 a) { return std::sqrt(dem::dot(a, a)); }

struct Mesh {
  const double* v;
  const int32_t* t;
  P3 a(int f) const { return at(v, t[3 * f]); }
  P3 b(int f) const { return at(v, t[3 * f + 1]); }
  P3 c(int f) const { return at(v, t[3 * f + 2]); }
  P3 centroid(int f) const { return (1.0 / 3.0) * (a(f) + b(f) + c(f)); }
};

// k-means on triangle centroids: farthest-point initialisation (from the set's
// mean), Lloyd iterations, empty clusters refilled from the largest one.
std::vector<std::vector<int>> kmeans_split(const Mesh& m, const std::vector<int>& set, int k, int iters) {
  const int n = (int)set.size();
  std::vector<P3> c(n);
  P3 mean{0, 0, 0};
  for (int i = 0; i < n; ++i) {
    c[i] = m.centroid(set[i]);
    mean = mean + c[i];
  }
  mean = (1.0 / n) * mean;
  // farthest-point initialisation: the centroid farthest from the mean, then
  // repeatedly the one farthest from the centres chosen so far
  std::vector<P3> ctr;
  std::vector<double> dmin(n, INFINITY);
  int far = 0;
  double best = -1;
  for (int i = 0; i < n; ++i) {
    double d = dem::dot(c[i] - mean, c[i] - mean);
    if (d > best) { best = d; far = i; }
  }
  for (int j = 0; j < k; ++j) {
    ctr.push_back(c[far]);
    for (int i = 0; i < n; ++i) dmin[i] = std::min(dmin[i], dem::dot(c[i] - c[far], c[i] - c[far]));
    best = -1;
    for (int i = 0; i < n; ++i)
      if (dmin[i] > best) { best = dmin[i]; far = i; }
  }
  std::vector<int> lab(n, 0);
  for (int it = 0; it <= iters; ++it) {
    for (int i = 0; i < n; ++i) {
      double best = INFINITY;
      for (int j = 0; j < k; ++j) {
        double d = dem::dot(c[i] - ctr[j], c[i] - ctr[j]);
        if (d < best) { best = d; lab[i] = j; }
      }
    }
    // empty clusters take the farthest member of the largest cluster
    for (int j = 0; j < k; ++j) {
      std::vector<int> cnt(k, 0);
      for (int i = 0; i < n; ++i) cnt[lab[i]]++;
      if (cnt[j] > 0) continue;
      int big = (int)(std::max_element(cnt.begin(), cnt.end()) - cnt.begin());
      int far = -1;
      double best = -1;
      for (int i = 0; i < n; ++i)
        if (lab[i] == big) {
          double d = dem::dot(c[i] - ctr[big], c[i] - ctr[big]);
          if (d > best) { best = d; far = i; }
        }
      lab[far] = j;
      ctr[j] = c[far];
    }
    if (it == iters) break;
    std::vector<P3> acc(k, P3{0, 0, 0});
    std::vector<int> cnt(k, 0);
    for (int i = 0; i < n; ++i) {
      acc[lab[i]] = acc[lab[i]] + c[i];
      cnt[lab[i]]++;
    }
    for (int j = 0; j < k; ++j)
      if (cnt[j]) ctr[j] = (1.0 / cnt[j]) * acc[j];
  }
  std::vector<std::vector<int>> out(k);
  for (int i = 0; i < n; ++i) out[lab[i]].push_back(set[i]);
  out.erase(std::remove_if(out.begin(), out.end(), [](const std::vector<int>& s) { return s.empty(); }),
            out.end());
  return out;
}

struct Fit {
  const Mesh* m;
  const std::vector<int>* set;
  std::vector<P3> tv;  // the set's triangle vertices, scaled: 3 per triangle
  std::vector<P3> uv;  // the set's distinct vertices, scaled
  P3 nout;             // outer direction (area-weighted normal of the set)
  double bs, aa, ai, bn;

  // distance of point x to scaled triangle k, and its closest point
  double dist(P3 x, int k, P3& q) const {
    P3 a = tv[3 * k], e1 = tv[3 * k + 1] - a, e2 = tv[3 * k + 2] - a;
    double w[3];
    return std::sqrt(dem::point_tri(x, a, e1, e2, q, w));
  }
  P3 normal(const P3 x[3]) const {
    P3 n = dem::cross(x[1] - x[0], x[2] - x[0]);
    return dem::dot(n, nout) < 0 ? -1.0 * n : n;
  }
  double size_term(const P3 x[3], P3 g[3]) const {
    double f = 0;
    const int nt = (int)tv.size() / 3;
    for (int i = 0; i < 3; ++i) {
      g[i] = P3{0, 0, 0};
      for (int k = 0; k < nt; ++k) {
        P3 q;
        double d = dist(x[i], k, q);
        f += std::pow(d, bs) / bs;
        if (d > 0) g[i] = g[i] + (std::pow(d, bs - 1) / d) * (x[i] - q);  // d|x - t| / dx = (x - q)/d
      }
    }
    return f;
  }
  double other_terms(const P3 x[3]) const {
    P3 n = normal(x);
    double nn = dem::dot(n, n);
    if (!(nn > 0)) return INFINITY;
    double f = 0.5 * aa / nn;
    P3 un = (1.0 / std::sqrt(nn)) * n;
    for (int i = 0; i < 3; ++i)
      for (const P3& v : uv) {
        double h = dem::dot(x[i] - v, un);
        if (h > 0) f += ai * std::pow(h, bn) / bn;
      }
    return f;
  }
  double value(const P3 x[3]) const {
    P3 g[3];
    return size_term(x, g) + other_terms(x);
  }
};

// Minimise the surrogate functional by gradient descent with backtracking.
void fit_surrogate(Fit& F, P3 x[3], int iters) {
  double step = 0.05;
  double f = F.value(x);
  for (int it = 0; it < iters && step > 1e-9; ++it) {
    P3 g[3];
    F.size_term(x, g);
    // the remaining terms are cheap: central differences
    const double h = 1e-6;
    for (int i = 0; i < 3; ++i) {
      double* c = &x[i].x;
      double* gi = &g[i].x;
      for (int d = 0; d < 3; ++d) {
        double keep = c[d];
        c[d] = keep + h;
        double fp = F.other_terms(x);
        c[d] = keep - h;
        double fm = F.other_terms(x);
        c[d] = keep;
        gi[d] += (std::isfinite(fp) && std::isfinite(fm)) ? (fp - fm) / (2 * h) : 0.0;
      }
    }
    double gn = std::sqrt(dem::dot(g[0], g[0]) + dem::dot(g[1], g[1]) + dem::dot(g[2], g[2]));
    if (!(gn > 0) || !std::isfinite(gn)) break;
    for (;;) {
      P3 y[3];
      for (int i = 0; i < 3; ++i) y[i] = x[i] - (step / gn) * g[i];
      double fy = F.value(y);
      if (fy < f) {
        for (int i = 0; i < 3; ++i) x[i] = y[i];
        f = fy;
        step *= 1.5;
        break;
      }
      step *= 0.5;
      if (step < 1e-9) break;
    }
  }
}

// Surrogate triangle for a set of mesh triangles (original coordinates).
void make_surrogate(const Mesh& m, const std::vector<int>& set, const dem_tree_opts& o, P3 out[3]) {
  P3 c{0, 0, 0};
  int nv = 0;
  std::vector<int> vid;
  for (int f : set)
    for (int k = 0; k < 3; ++k) vid.push_back(m.t[3 * f + k]);
  std::sort(vid.begin(), vid.end());
  vid.erase(std::unique(vid.begin(), vid.end()), vid.end());
  for (int v : vid) { c = c + at(m.v, v); ++nv; }
  c = (1.0 / nv) * c;
  double r = 0;
  for (int v : vid) r = std::max(r, norm(at(m.v, v) - c));
  if (!(r > 0)) r = 1;
  const double s = 1.0 / r;
  Fit F;
  F.m = &m;
  F.set = &set;
  F.bs = o.beta_size;
  F.aa = o.alpha_area;
  F.ai = o.alpha_inside;
  F.bn = o.beta_normal;
  P3 nsum{0, 0, 0};
  for (int f : set) {
    P3 a = s * (m.a(f) - c), b = s * (m.b(f) - c), d = s * (m.c(f) - c);
    F.tv.push_back(a); F.tv.push_back(b); F.tv.push_back(d);
    nsum = nsum + dem::cross(b - a, d - a);
  }
  for (int v : vid) F.uv.push_back(s * (at(m.v, v) - c));
  F.nout = norm(nsum) > 0 ? nsum : P3{0, 0, 1};
  // start from the triangle of the set nearest the centre
  int start = set[0];
  double best = INFINITY;
  for (int f : set) {
    double d = norm(m.centroid(f) - c);
    if (d < best) { best = d; start = f; }
  }
  P3 x[3] = {s * (m.a(start) - c), s * (m.b(start) - c), s * (m.c(start) - c)};
  if (dem::dot(dem::cross(x[1] - x[0], x[2] - x[0]), F.nout) < 0) std::swap(x[1], x[2]);
  fit_surrogate(F, x, o.fit_iters);
  for (int i = 0; i < 3; ++i) out[i] = c + r * x[i];
}

template <typename X>
X* alloc(size_t n) {
  return static_cast<X*>(std::calloc(n ? n : 1, sizeof(X)));
}

}  // namespace

extern "C" {

void dem_default_tree_opts(dem_tree_opts* o) {
  if (!o) return;
  o->fanout = 8;
  o->kmeans_iters = 12;
  o->fit_iters = 60;
  o->beta_size = 8.0;
  o->alpha_area = 1e-3;
  o->alpha_inside = 1.0;
  o->beta_normal = 2.0;
}

dem_status dem_build_surrogate_tree(const double* verts, int32_t n_verts, const int32_t* tris,
                                    int32_t n_tris, const dem_tree_opts* opts, dem_surrogate_tree* out) {
  if (!out) return DEM_ERR_ARG;
  std::memset(out, 0, sizeof(*out));
  if (!verts || !tris || n_verts < 3 || n_tris < 1) return DEM_ERR_ARG;
  dem_tree_opts o;
  if (opts) o = *opts; else dem_default_tree_opts(&o);
  if (o.fanout < 2 || o.fanout > DEM_MAX_CHILDREN || o.kmeans_iters < 0 || o.fit_iters < 0 ||
      !(o.beta_size >= 2) || !(o.alpha_area > 0) || !(o.alpha_inside >= 0) || !(o.beta_normal >= 1))
    return DEM_ERR_ARG;
  for (int64_t i = 0; i < 3 * (int64_t)n_tris; ++i)
    if (tris[i] < 0 || tris[i] >= n_verts) return DEM_ERR_ARG;
  for (int64_t i = 0; i < 3 * (int64_t)n_verts; ++i)
    if (!std::isfinite(verts[i])) return DEM_ERR_ARG;
  const Mesh m{verts, tris};

  // breadth-first: surrogates depth by depth; leaf sets remember their parent
  struct Node { std::vector<int> set; int depth; };
  std::vector<Node> nodes;          // surrogate k stands for nodes[k].set
  std::vector<int> node_parent;
  std::vector<std::vector<int>> leaf_sets;  // fine children of surrogate k (empty if none)
  std::vector<int> all(n_tris);
  for (int i = 0; i < n_tris; ++i) all[i] = i;
  nodes.push_back({all, 0});
  node_parent.push_back(-1);
  for (size_t k = 0; k < nodes.size(); ++k) {
    leaf_sets.emplace_back();
    if ((int)nodes[k].set.size() <= o.fanout) {
      leaf_sets[k] = nodes[k].set;
      continue;
    }
    auto parts = kmeans_split(m, nodes[k].set, o.fanout, o.kmeans_iters);
    if (parts.size() < 2) {  // all centroids coincide: split by index
      parts.assign(o.fanout, {});
      for (size_t i = 0; i < nodes[k].set.size(); ++i) parts[i % o.fanout].push_back(nodes[k].set[i]);
    }
    for (auto& p : parts) {
      nodes.push_back({std::move(p), nodes[k].depth + 1});
      node_parent.push_back((int)k);
    }
  }
  const int n_sur = (int)nodes.size();
  const int n_depths = nodes.back().depth + 1;
  const int64_t total = (int64_t)n_sur + n_tris;
  const int64_t nv_out = (int64_t)n_verts + 3 * (int64_t)n_sur;
  if (total > 0x7fffffff || nv_out > 0x7fffffff) return DEM_ERR_ARG;

  out->n_verts = (int32_t)nv_out;
  out->n_tris = (int32_t)total;
  out->n_levels = n_depths + 1;
  out->verts = alloc<double>(3 * (size_t)nv_out);
  out->tris = alloc<int32_t>(3 * (size_t)total);
  out->parent = alloc<int32_t>((size_t)total);
  out->level_sizes = alloc<int32_t>((size_t)out->n_levels);
  out->fine_order = alloc<int32_t>((size_t)n_tris);
  if (!out->verts || !out->tris || !out->parent || !out->level_sizes || !out->fine_order) {
    dem_surrogate_tree_free(out);
    return DEM_ERR_OOM;
  }
  std::memcpy(out->verts, verts, 3 * sizeof(double) * (size_t)n_verts);
  for (int k = 0; k < n_sur; ++k) {
    P3 x[3];
    make_surrogate(m, nodes[k].set, o, x);
    for (int i = 0; i < 3; ++i) {
      const int64_t vi = (int64_t)n_verts + 3 * (int64_t)k + i;
      out->verts[3 * vi] = x[i].x;
      out->verts[3 * vi + 1] = x[i].y;
      out->verts[3 * vi + 2] = x[i].z;
      out->tris[3 * k + i] = (int32_t)vi;
    }
    out->parent[k] = node_parent[k];
    out->level_sizes[nodes[k].depth]++;
  }
  int64_t f = n_sur;
  for (int k = 0; k < n_sur; ++k)
    for (int t : leaf_sets[k]) {
      for (int i = 0; i < 3; ++i) out->tris[3 * f + i] = tris[3 * t + i];
      out->parent[f] = k;
      out->fine_order[f - n_sur] = t;
      ++f;
    }
  out->level_sizes[n_depths] = n_tris;
  return DEM_OK;
}

void dem_surrogate_tree_free(dem_surrogate_tree* t) {
  if (!t) return;
  std::free(t->verts);
  std::free(t->tris);
  std::free(t->parent);
  std::free(t->level_sizes);
  std::free(t->fine_order);
  std::memset(t, 0, sizeof(*t));
}

}  // extern "C"
