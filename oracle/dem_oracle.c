/*
 * FP64 CPU oracle for multiresolution triangle-mesh contact detection
 * (Noble & Weinzierl, "A multiresolution Discrete Element Method for
 * triangulated objects with implicit time stepping", arXiv 2105.12415).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously correct
 * reference that the GPU path is checked against.  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg load it; the product library
 * never links, includes or calls anything here, and shares no code with it.
 *
 * Everything is double precision, no fast-math, written from the definitions:
 *
 *  - tri_tri():   exact triangle-triangle distance by the comparison-based
 *                 method of Section 3 ("direct distance calculation"): six
 *                 edge-against-triangle intersection tests (intersecting
 *                 triangles have distance 0), otherwise the minimum of the six
 *                 point-to-triangle and nine edge-to-edge distances.  Each of
 *                 those sub-problems is a convex quadratic over a box or a
 *                 simplex and is solved as "unconstrained stationary point if
 *                 it is feasible, otherwise the minimum over the boundary".
 *  - contacts:    the contact set of Algorithm 2 with the contact predicate of
 *                 Section 2 (epsilon environments overlap <=> distance <=
 *                 eps_i + eps_j), over ALL fine triangle pairs of each
 *                 candidate particle pair.  The only shortcut is an exact
 *                 bounding-sphere rejection that cannot change the set.
 *  - energy/grad: E = k * sum (delta - d)^2 over contacts; the gradient by the
 *                 envelope theorem (d is a minimum over a fixed convex set).
 *  - surrogate_eps: the smallest epsilon that makes a surrogate triangle
 *                 conservative for its fine descendants (Definition
 *                 "conservative", Section 4; Algorithm 7 in Appendix B):
 *                 eps0 + max over fine descendant vertices of the distance to
 *                 the surrogate (the maximum of a convex function over a
 *                 triangle is attained at a vertex).
 *  - descent:     the pairwise multiresolution descent of Algorithm 5 driven
 *                 by EXACT distances, used to pin Lemma 1 (hierarchical ==
 *                 flat) and to count the pairs an exact descent must test.
 *
 * Parity pins for every function are in tests/test_oracle_*.py.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ----------------------------------------------------------------- vectors */
static void sub3(const double a[3], const double b[3], double r[3]) {
  r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2];
}
static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double a[3], const double b[3], double r[3]) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}
static void axpy3(const double a[3], double s, const double d[3], double r[3]) {
  r[0] = a[0] + s * d[0]; r[1] = a[1] + s * d[1]; r[2] = a[2] + s * d[2];
}
static double dist3(const double a[3], const double b[3]) {
  double d[3]; sub3(a, b, d); return sqrt(dot3(d, d));
}

/* -------------------------------------------------- point against segment */
/* Closest point of segment a + t (b - a), t in [0,1], to p. Returns t. */
static double point_segment(const double p[3], const double a[3], const double b[3], double q[3]) {
  double d[3], ap[3];
  sub3(b, a, d);
  sub3(p, a, ap);
  double dd = dot3(d, d);
  double t = 0.0;
  if (dd > 0.0) {
    t = dot3(ap, d) / dd;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
  }
  axpy3(a, t, d, q);
  return t;
}

/* A triangle is degenerate (a segment or a point: no interior) when the sine
 * of its angle at x0 is below 1e-12; FP64 rounding of the normal is ~1e-16. */
static int degenerate(double nn, double a, double c) { return !(nn > 1e-24 * a * c) || !(nn > 0.0); }

/* ------------------------------------------------- point against triangle */
/* Closest point q on triangle (x0,x1,x2) to p, with barycentric weights w.
 * Minimises |x0 + u e1 + v e2 - p|^2 over u,v >= 0, u + v <= 1.  The
 * unconstrained minimiser is the answer when feasible; otherwise the minimum
 * lies on the boundary, i.e. on one of the three edges.  The minimiser's
 * coordinates are ratios of signed areas (triple products with the normal
 * n = e1 x e2), which stay accurate for slivers; a degenerate triangle has
 * only its boundary.  Returns distance. */
static double point_triangle(const double p[3], const double x0[3], const double x1[3],
                             const double x2[3], double q[3], double w[3]) {
  double e1[3], e2[3], r[3], n[3], t1[3], t2[3];
  sub3(x1, x0, e1);
  sub3(x2, x0, e2);
  sub3(p, x0, r);
  cross3(e1, e2, n);
  double nn = dot3(n, n);
  if (!degenerate(nn, dot3(e1, e1), dot3(e2, e2))) {
    cross3(r, e2, t1);
    cross3(e1, r, t2);
    double u = dot3(n, t1) / nn;
    double v = dot3(n, t2) / nn;
    if (u >= 0.0 && v >= 0.0 && u + v <= 1.0) {
      q[0] = x0[0] + u * e1[0] + v * e2[0];
      q[1] = x0[1] + u * e1[1] + v * e2[1];
      q[2] = x0[2] + u * e1[2] + v * e2[2];
      w[0] = 1.0 - u - v; w[1] = u; w[2] = v;
      return dist3(p, q);
    }
  }
  /* boundary: edges x0-x1, x1-x2, x2-x0 */
  const double* E[3][2] = {{x0, x1}, {x1, x2}, {x2, x0}};
  double best = INFINITY;
  for (int k = 0; k < 3; ++k) {
    double qk[3];
    double t = point_segment(p, E[k][0], E[k][1], qk);
    double dk = dist3(p, qk);
    if (dk < best) {
      best = dk;
      q[0] = qk[0]; q[1] = qk[1]; q[2] = qk[2];
      w[0] = w[1] = w[2] = 0.0;
      w[k] += 1.0 - t;
      w[(k + 1) % 3] += t;
    }
  }
  return best;
}

/* -------------------------------------------------- segment against segment */
/* Closest points of p0 + s (p1 - p0) and q0 + t (q1 - q0), s,t in [0,1].
 * Unconstrained stationary point when it is inside the unit square and the
 * segments are not parallel; otherwise the minimum over the square's four
 * sides (each a point-against-segment problem). Returns distance. */
static double segment_segment(const double p0[3], const double p1[3], const double q0[3],
                              const double q1[3], double* s_out, double* t_out, double cp[3],
                              double cq[3]) {
  double d1[3], d2[3], r[3];
  sub3(p1, p0, d1);
  sub3(q1, q0, d2);
  sub3(p0, q0, r);
  double a = dot3(d1, d1), b = dot3(d1, d2), c = dot3(d2, d2);
  double e = dot3(d1, r), f = dot3(d2, r);
  double det = a * c - b * b;
  if (det > 1e-14 * a * c && det > 0.0) {
    /* s a - t b = -e ; s b - t c = -f */
    double s = (b * f - c * e) / det;
    double t = (a * f - b * e) / det;
    if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0) {
      axpy3(p0, s, d1, cp);
      axpy3(q0, t, d2, cq);
      *s_out = s; *t_out = t;
      return dist3(cp, cq);
    }
  }
  double best = INFINITY;
  double tmp[3];
  /* s = 0 and s = 1: endpoint of P against segment Q */
  for (int k = 0; k < 2; ++k) {
    const double* pe = k ? p1 : p0;
    double t = point_segment(pe, q0, q1, tmp);
    double dk = dist3(pe, tmp);
    if (dk < best) {
      best = dk;
      *s_out = (double)k; *t_out = t;
      cp[0] = pe[0]; cp[1] = pe[1]; cp[2] = pe[2];
      cq[0] = tmp[0]; cq[1] = tmp[1]; cq[2] = tmp[2];
    }
  }
  /* t = 0 and t = 1: endpoint of Q against segment P */
  for (int k = 0; k < 2; ++k) {
    const double* qe = k ? q1 : q0;
    double s = point_segment(qe, p0, p1, tmp);
    double dk = dist3(qe, tmp);
    if (dk < best) {
      best = dk;
      *s_out = s; *t_out = (double)k;
      cp[0] = tmp[0]; cp[1] = tmp[1]; cp[2] = tmp[2];
      cq[0] = qe[0]; cq[1] = qe[1]; cq[2] = qe[2];
    }
  }
  return best;
}

/* ----------------------------------------- segment piercing a triangle */
/* Does segment p0-p1 cross the plane of (x0,x1,x2) at a point inside the
 * triangle?  Coplanar segments are left to the distance tests (an in-plane
 * overlap makes a point-triangle or edge-edge distance zero).  On a hit,
 * x is the crossing point, s its parameter on the segment and w its
 * barycentric weights in the triangle. */
static int segment_pierces(const double p0[3], const double p1[3], const double x0[3],
                           const double x1[3], const double x2[3], double x[3], double* s,
                           double w[3]) {
  double e1[3], e2[3], n[3], r0[3], r1[3];
  sub3(x1, x0, e1);
  sub3(x2, x0, e2);
  cross3(e1, e2, n);
  double nn = dot3(n, n);
  /* a degenerate triangle has no interior to cross: touching it shows up as a
   * zero segment-segment or point distance */
  if (degenerate(nn, dot3(e1, e1), dot3(e2, e2))) return 0;
  sub3(p0, x0, r0);
  sub3(p1, x0, r1);
  double h0 = dot3(n, r0), h1 = dot3(n, r1);
  if (h0 == 0.0 && h1 == 0.0) return 0;
  if ((h0 > 0.0 && h1 > 0.0) || (h0 < 0.0 && h1 < 0.0)) return 0;
  double t = h0 / (h0 - h1);
  double d[3];
  sub3(p1, p0, d);
  axpy3(p0, t, d, x);
  /* barycentric coordinates of x in the triangle (x lies in its plane), as
   * ratios of signed areas */
  double r[3], t1[3], t2[3];
  sub3(x, x0, r);
  cross3(r, e2, t1);
  cross3(e1, r, t2);
  double u = dot3(n, t1) / nn;
  double v = dot3(n, t2) / nn;
  if (u >= 0.0 && v >= 0.0 && u + v <= 1.0) {
    w[0] = 1.0 - u - v; w[1] = u; w[2] = v;
    *s = t;
    return 1;
  }
  return 0;
}

/* -------------------------------------------------- triangle vs triangle */
/* Output record of one triangle-pair distance. */
typedef struct {
  double d;        /* exact distance */
  double p1[3];    /* closest point on A */
  double p2[3];    /* closest point on B */
  double w1[3];    /* barycentric weights of p1 in A */
  double w2[3];    /* barycentric weights of p2 in B */
  int feature;     /* 0..5 PT (A verts vs B, then B verts vs A), 6..14 SS, 15 intersect */
  int ambiguous;   /* another candidate within tolerance has different points */
} tt_result;

/* Relative distance tolerance under which two of the fifteen candidates
 * count as tied when flagging non-unique closest points (see tri_tri). */
static double g_ambiguity_rel = 1e-9;

void oracle_set_ambiguity_tol(double rel) { g_ambiguity_rel = rel; }

static void tri_tri(const double* A, const double* B, tt_result* res) {
  const double* a[3] = {A, A + 3, A + 6};
  const double* b[3] = {B, B + 3, B + 6};
  memset(res, 0, sizeof(*res));
  /* 1. edges of A piercing B, edges of B piercing A */
  for (int side = 0; side < 2; ++side) {
    const double** P = side ? b : a;
    const double** T = side ? a : b;
    for (int k = 0; k < 3; ++k) {
      double x[3], s, w[3];
      if (segment_pierces(P[k], P[(k + 1) % 3], T[0], T[1], T[2], x, &s, w)) {
        res->d = 0.0;
        res->feature = 15;
        double we[3] = {0.0, 0.0, 0.0};
        we[k] = 1.0 - s;
        we[(k + 1) % 3] = s;
        memcpy(res->p1, x, sizeof(x));
        memcpy(res->p2, x, sizeof(x));
        if (side == 0) {
          memcpy(res->w1, we, sizeof(we));
          memcpy(res->w2, w, sizeof(w));
        } else {
          memcpy(res->w1, w, sizeof(w));
          memcpy(res->w2, we, sizeof(we));
        }
        return;
      }
    }
  }
  /* 2. fifteen candidates: 6 point-triangle, 9 segment-segment */
  double cand_d[15], cand_p1[15][3], cand_p2[15][3], cand_w1[15][3], cand_w2[15][3];
  int n = 0;
  for (int k = 0; k < 3; ++k, ++n) { /* vertex k of A against B */
    double q[3], w[3];
    cand_d[n] = point_triangle(a[k], b[0], b[1], b[2], q, w);
    memcpy(cand_p1[n], a[k], 3 * sizeof(double));
    memcpy(cand_p2[n], q, sizeof(q));
    cand_w1[n][0] = cand_w1[n][1] = cand_w1[n][2] = 0.0;
    cand_w1[n][k] = 1.0;
    memcpy(cand_w2[n], w, sizeof(w));
  }
  for (int k = 0; k < 3; ++k, ++n) { /* vertex k of B against A */
    double q[3], w[3];
    cand_d[n] = point_triangle(b[k], a[0], a[1], a[2], q, w);
    memcpy(cand_p1[n], q, sizeof(q));
    memcpy(cand_p2[n], b[k], 3 * sizeof(double));
    memcpy(cand_w1[n], w, sizeof(w));
    cand_w2[n][0] = cand_w2[n][1] = cand_w2[n][2] = 0.0;
    cand_w2[n][k] = 1.0;
  }
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j, ++n) {
      double s, t, cp[3], cq[3];
      cand_d[n] = segment_segment(a[i], a[(i + 1) % 3], b[j], b[(j + 1) % 3], &s, &t, cp, cq);
      memcpy(cand_p1[n], cp, sizeof(cp));
      memcpy(cand_p2[n], cq, sizeof(cq));
      cand_w1[n][0] = cand_w1[n][1] = cand_w1[n][2] = 0.0;
      cand_w2[n][0] = cand_w2[n][1] = cand_w2[n][2] = 0.0;
      cand_w1[n][i] += 1.0 - s;
      cand_w1[n][(i + 1) % 3] += s;
      cand_w2[n][j] += 1.0 - t;
      cand_w2[n][(j + 1) % 3] += t;
    }
  }
  int best = 0;
  for (int k = 1; k < 15; ++k)
    if (cand_d[k] < cand_d[best]) best = k;
  res->d = cand_d[best];
  res->feature = best;
  memcpy(res->p1, cand_p1[best], 3 * sizeof(double));
  memcpy(res->p2, cand_p2[best], 3 * sizeof(double));
  memcpy(res->w1, cand_w1[best], 3 * sizeof(double));
  memcpy(res->w2, cand_w2[best], 3 * sizeof(double));
  /* non-unique closest points: a near-tie whose points differ */
  double scale = 0.0;
  for (int k = 0; k < 3; ++k) {
    scale = fmax(scale, dist3(a[k], a[(k + 1) % 3]));
    scale = fmax(scale, dist3(b[k], b[(k + 1) % 3]));
  }
  for (int k = 0; k < 15; ++k) {
    if (k == best) continue;
    if (cand_d[k] - cand_d[best] <= g_ambiguity_rel * scale) {
      double dp = dist3(cand_p1[k], cand_p1[best]) + dist3(cand_p2[k], cand_p2[best]);
      if (dp > 1e-6 * scale) res->ambiguous = 1;
    }
  }
}

/* Public: one pair. out = [d, p1(3), p2(3), w1(3), w2(3), feature, ambiguous] (15). */
void oracle_tri_tri(const double* A, const double* B, double* out) {
  tt_result r;
  tri_tri(A, B, &r);
  out[0] = r.d;
  memcpy(out + 1, r.p1, 3 * sizeof(double));
  memcpy(out + 4, r.p2, 3 * sizeof(double));
  memcpy(out + 7, r.w1, 3 * sizeof(double));
  memcpy(out + 10, r.w2, 3 * sizeof(double));
  out[13] = (double)r.feature;
  out[14] = (double)r.ambiguous;
}

/* Public: many pairs, n x 18 doubles in (A 9, B 9), n x 15 out; threaded. */
typedef struct {
  const double* in;
  double* out;
  int64_t n;
  int64_t next;
  pthread_mutex_t mu;
} batch_job;

static int64_t grab(int64_t* next, pthread_mutex_t* mu, int64_t chunk, int64_t n, int64_t* end) {
  pthread_mutex_lock(mu);
  int64_t b = *next;
  *next = b + chunk;
  pthread_mutex_unlock(mu);
  *end = b + chunk < n ? b + chunk : n;
  return b;
}

static void* batch_worker(void* arg) {
  batch_job* J = (batch_job*)arg;
  for (;;) {
    int64_t e;
    int64_t b = grab(&J->next, &J->mu, 4096, J->n, &e);
    if (b >= J->n) break;
    for (int64_t i = b; i < e; ++i) oracle_tri_tri(J->in + 18 * i, J->in + 18 * i + 9, J->out + 15 * i);
  }
  return NULL;
}

static int clamp_threads(int n_threads) {
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  return n_threads;
}

void oracle_tri_tri_batch(const double* in, int64_t n, double* out, int n_threads) {
  batch_job J = {in, out, n, 0};
  pthread_mutex_init(&J.mu, NULL);
  n_threads = clamp_threads(n_threads);
  pthread_t th[256];
  for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, batch_worker, &J);
  for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
  pthread_mutex_destroy(&J.mu);
}

/* Public: closest point of p on triangle X (9 doubles); out = [d, q(3), w(3)]. */
void oracle_point_triangle(const double* p, const double* X, double* out) {
  double q[3], w[3];
  out[0] = point_triangle(p, X, X + 3, X + 6, q, w);
  memcpy(out + 1, q, sizeof(q));
  memcpy(out + 4, w, sizeof(w));
}

/* Public: segment-segment; out = [d, s, t, cp(3), cq(3)]. */
void oracle_segment_segment(const double* P /*6*/, const double* Q /*6*/, double* out) {
  double s, t, cp[3], cq[3];
  out[0] = segment_segment(P, P + 3, Q, Q + 3, &s, &t, cp, cq);
  out[1] = s; out[2] = t;
  memcpy(out + 3, cp, sizeof(cp));
  memcpy(out + 6, cq, sizeof(cq));
}

/* --------------------------------------------------------- contact sets */
/* Scene in the oracle's own layout: verts [V][3] world coordinates,
 * fine triangles [T][3] global vertex ids, particle p owns triangles
 * [tri_begin[p], tri_begin[p] + tri_count[p]) and has epsilon eps[p]. */
typedef struct {
  const double* verts;
  const int32_t* tris;
  const int32_t* tri_begin;
  const int32_t* tri_count;
  const double* eps;
  const int32_t* pairs;
  int64_t n_pairs;
  double delta_override; /* NaN: eps_i + eps_j; else this threshold for every pair */
  int prereject;
  /* work distribution over (pair, row) units */
  int64_t* row_off; /* prefix over pairs of tri_count[pi] */
  int64_t n_rows;
  int64_t next;
  pthread_mutex_t mu;
  /* output, one growing buffer per thread */
  int n_threads;
  struct outbuf* bufs;
} contact_job;

typedef struct outbuf {
  int64_t n, cap;
  int32_t* pair;
  int32_t* ti;
  int32_t* tj;
  double* rec; /* 15 doubles per contact: as oracle_tri_tri */
  int64_t tested;
} outbuf;

static void outbuf_push(outbuf* o, int32_t pair, int32_t ti, int32_t tj, const tt_result* r) {
  if (o->n == o->cap) {
    int64_t nc = o->cap ? 2 * o->cap : 1024;
    o->pair = (int32_t*)realloc(o->pair, nc * sizeof(int32_t));
    o->ti = (int32_t*)realloc(o->ti, nc * sizeof(int32_t));
    o->tj = (int32_t*)realloc(o->tj, nc * sizeof(int32_t));
    o->rec = (double*)realloc(o->rec, nc * 15 * sizeof(double));
    o->cap = nc;
  }
  o->pair[o->n] = pair;
  o->ti[o->n] = ti;
  o->tj[o->n] = tj;
  double* q = o->rec + 15 * o->n;
  q[0] = r->d;
  memcpy(q + 1, r->p1, 3 * sizeof(double));
  memcpy(q + 4, r->p2, 3 * sizeof(double));
  memcpy(q + 7, r->w1, 3 * sizeof(double));
  memcpy(q + 10, r->w2, 3 * sizeof(double));
  q[13] = (double)r->feature;
  q[14] = (double)r->ambiguous;
  o->n++;
}

static void load_tri(const double* verts, const int32_t* tris, int64_t t, double X[9]) {
  for (int k = 0; k < 3; ++k) {
    const double* v = verts + 3 * (int64_t)tris[3 * t + k];
    X[3 * k] = v[0]; X[3 * k + 1] = v[1]; X[3 * k + 2] = v[2];
  }
}

/* Bounding sphere about the vertex mean; any point of the triangle lies
 * within r of c (the triangle is the convex hull of its vertices). */
static void bsphere(const double X[9], double c[3], double* r) {
  for (int q = 0; q < 3; ++q) c[q] = (X[q] + X[3 + q] + X[6 + q]) / 3.0;
  double m = 0.0;
  for (int k = 0; k < 3; ++k) m = fmax(m, dist3(X + 3 * k, c));
  *r = m;
}

static void* contact_worker(void* arg) {
  void** a = (void**)arg;
  contact_job* J = (contact_job*)a[0];
  outbuf* o = (outbuf*)a[1];
  for (;;) {
    int64_t e;
    int64_t b = grab(&J->next, &J->mu, 16, J->n_rows, &e);
    if (b >= J->n_rows) break;
    for (int64_t row = b; row < e; ++row) {
      /* find the pair owning this row (binary search in row_off) */
      int64_t lo = 0, hi = J->n_pairs - 1;
      while (lo < hi) {
        int64_t mid = (lo + hi + 1) / 2;
        if (J->row_off[mid] <= row) lo = mid; else hi = mid - 1;
      }
      int64_t pr = lo;
      int32_t pi = J->pairs[2 * pr], pj = J->pairs[2 * pr + 1];
      int64_t ti = J->tri_begin[pi] + (row - J->row_off[pr]);
      double delta = isnan(J->delta_override) ? J->eps[pi] + J->eps[pj] : J->delta_override;
      double A[9], ca[3], ra;
      load_tri(J->verts, J->tris, ti, A);
      bsphere(A, ca, &ra);
      for (int64_t k = 0; k < J->tri_count[pj]; ++k) {
        int64_t tj = J->tri_begin[pj] + k;
        double B[9];
        load_tri(J->verts, J->tris, tj, B);
        if (J->prereject && isfinite(delta)) {
          double cb[3], rb;
          bsphere(B, cb, &rb);
          double gap = dist3(ca, cb) - ra - rb;
          if (gap > delta + 1e-9 * (1.0 + fabs(delta) + ra + rb)) continue;
        }
        o->tested++;
        tt_result r;
        tri_tri(A, B, &r);
        if (r.d <= delta)
          outbuf_push(o, (int32_t)pr, (int32_t)(ti - J->tri_begin[pi]), (int32_t)k, &r);
      }
    }
  }
  return NULL;
}

/* Result of oracle_find_contacts, ordered by (pair, ti, tj); ti/tj are
 * particle-local fine triangle indices. Free with oracle_free_contacts. */
typedef struct {
  int64_t n;
  int32_t* pair;
  int32_t* ti;
  int32_t* tj;
  double* rec; /* n x 15: d, p1, p2, w1, w2, feature, ambiguous */
  int64_t tested; /* triangle pairs on which tri_tri ran */
} oracle_contacts;

static int cmp_key3(const void* x, const void* y) {
  const int64_t* a = (const int64_t*)x;
  const int64_t* b = (const int64_t*)y;
  for (int k = 0; k < 3; ++k) {
    if (a[k] < b[k]) return -1;
    if (a[k] > b[k]) return 1;
  }
  return 0;
}

int oracle_find_contacts(const double* verts, const int32_t* tris, const int32_t* tri_begin,
                         const int32_t* tri_count, const double* eps, const int32_t* pairs,
                         int64_t n_pairs, double delta_override, int prereject, int n_threads,
                         oracle_contacts* out) {
  memset(out, 0, sizeof(*out));
  if (n_pairs <= 0) return 0;
  n_threads = clamp_threads(n_threads);
  contact_job J;
  memset(&J, 0, sizeof(J));
  J.verts = verts; J.tris = tris; J.tri_begin = tri_begin; J.tri_count = tri_count;
  J.eps = eps; J.pairs = pairs; J.n_pairs = n_pairs; J.delta_override = delta_override;
  J.prereject = prereject;
  J.row_off = (int64_t*)malloc((n_pairs + 1) * sizeof(int64_t));
  J.row_off[0] = 0;
  for (int64_t p = 0; p < n_pairs; ++p) J.row_off[p + 1] = J.row_off[p] + tri_count[pairs[2 * p]];
  J.n_rows = J.row_off[n_pairs];
  pthread_mutex_init(&J.mu, NULL);
  outbuf* bufs = (outbuf*)calloc(n_threads, sizeof(outbuf));
  pthread_t th[256];
  void* args[256][2];
  for (int t = 0; t < n_threads; ++t) {
    args[t][0] = &J; args[t][1] = &bufs[t];
    pthread_create(&th[t], NULL, contact_worker, args[t]);
  }
  for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
  pthread_mutex_destroy(&J.mu);
  int64_t total = 0, tested = 0;
  for (int t = 0; t < n_threads; ++t) { total += bufs[t].n; tested += bufs[t].tested; }
  /* merge and order by (pair, ti, tj) */
  int64_t* key = (int64_t*)malloc((total ? total : 1) * 4 * sizeof(int64_t));
  int64_t m = 0;
  for (int t = 0; t < n_threads; ++t)
    for (int64_t i = 0; i < bufs[t].n; ++i, ++m) {
      key[4 * m] = bufs[t].pair[i]; key[4 * m + 1] = bufs[t].ti[i];
      key[4 * m + 2] = bufs[t].tj[i]; key[4 * m + 3] = ((int64_t)t << 40) | i;
    }
  qsort(key, total, 4 * sizeof(int64_t), cmp_key3);
  out->n = total;
  out->tested = tested;
  out->pair = (int32_t*)malloc((total ? total : 1) * sizeof(int32_t));
  out->ti = (int32_t*)malloc((total ? total : 1) * sizeof(int32_t));
  out->tj = (int32_t*)malloc((total ? total : 1) * sizeof(int32_t));
  out->rec = (double*)malloc((total ? total : 1) * 15 * sizeof(double));
  for (int64_t i = 0; i < total; ++i) {
    int t = (int)(key[4 * i + 3] >> 40);
    int64_t j = key[4 * i + 3] & ((1LL << 40) - 1);
    out->pair[i] = bufs[t].pair[j];
    out->ti[i] = bufs[t].ti[j];
    out->tj[i] = bufs[t].tj[j];
    memcpy(out->rec + 15 * i, bufs[t].rec + 15 * j, 15 * sizeof(double));
  }
  for (int t = 0; t < n_threads; ++t) {
    free(bufs[t].pair); free(bufs[t].ti); free(bufs[t].tj); free(bufs[t].rec);
  }
  free(bufs);
  free(key);
  free(J.row_off);
  return 0;
}

void oracle_free_contacts(oracle_contacts* c) {
  free(c->pair); free(c->ti); free(c->tj); free(c->rec);
  memset(c, 0, sizeof(*c));
}

/* ------------------------------------------------------ energy, gradient */
/* E = k * sum_c (delta_c - d_c)^2 over the given contacts (d <= delta).
 * dE/dx for a vertex of the first triangle = +2k (delta - d) w1 u and for one
 * of the second = -2k (delta - d) w2 u, with u = (p2 - p1) / d: moving a
 * vertex moves the closest point by its barycentric weight, and by the
 * envelope theorem only that motion changes d to first order.  d = 0
 * (intersecting triangles) stays 0 under small motions: no gradient.
 * tri_i / tri_j are global triangle ids into tris; grad is [V][3], added to. */
void oracle_energy_grad(const int32_t* tris, int64_t n, const int32_t* tri_i, const int32_t* tri_j,
                        const double* rec, const double* delta, double k, double* energy,
                        double* grad) {
  double E = 0.0;
  for (int64_t c = 0; c < n; ++c) {
    const double* q = rec + 15 * c;
    double d = q[0];
    double pen = delta[c] - d;
    if (pen < 0.0) continue;
    E += k * pen * pen;
    if (!(d > 0.0) || grad == NULL) continue;
    double u[3];
    sub3(q + 4, q + 1, u);
    for (int r = 0; r < 3; ++r) u[r] /= d;
    double g = 2.0 * k * pen;
    for (int v = 0; v < 3; ++v) {
      int64_t vi = tris[3 * (int64_t)tri_i[c] + v];
      int64_t vj = tris[3 * (int64_t)tri_j[c] + v];
      for (int r = 0; r < 3; ++r) {
        grad[3 * vi + r] += g * q[7 + v] * u[r];
        grad[3 * vj + r] -= g * q[10 + v] * u[r];
      }
    }
  }
  *energy = E;
}

/* ------------------------------------------------- surrogate epsilons */
/* Triangles of one particle, all levels: tris [T][3] (vertex ids into verts
 * [V][3]), parent[t] = index of the triangle it was split from (-1 at the
 * coarsest level), is_fine[t] = 1 for the particle triangulation.
 * eps_out[t] = eps0 for fine triangles, and for a surrogate s the smallest
 * epsilon for which s's environment contains every fine descendant's
 * eps0-environment: eps0 + max over fine descendant vertices v of dist(v, s). */
void oracle_surrogate_eps(const double* verts, const int32_t* tris, const int32_t* parent,
                          const uint8_t* is_fine, int64_t n_tris, double eps0, double* eps_out) {
  for (int64_t t = 0; t < n_tris; ++t) eps_out[t] = is_fine[t] ? eps0 : -INFINITY;
  for (int64_t f = 0; f < n_tris; ++f) {
    if (!is_fine[f]) continue;
    for (int64_t s = parent[f]; s >= 0; s = parent[s]) {
      double S[9];
      load_tri(verts, tris, s, S);
      for (int v = 0; v < 3; ++v) {
        double q[3], w[3];
        double dv = point_triangle(verts + 3 * (int64_t)tris[3 * f + v], S, S + 3, S + 6, q, w);
        if (eps0 + dv > eps_out[s]) eps_out[s] = eps0 + dv;
      }
    }
  }
}

/* ------------------------------------------- exact pairwise descent */
/* Pairwise form of Algorithm 5 with exact distances: starting from the root
 * pairs of each candidate particle pair, a triangle pair is tested (exact
 * distance vs eps_a + eps_b); a surviving pair whose members are both fine
 * is a contact, otherwise its non-fine side(s) unfold into their children.
 * Hierarchy in global numbering: child_begin/child_count per triangle
 * (count 0 = fine), root_begin/root_count per particle, eps per triangle.
 * Outputs: tests_per_depth[depth] counts (depth < 64), and the contact list
 * (global triangle ids, unordered) through the outbuf mechanism. */
typedef struct {
  const double* verts;
  const int32_t* tris;
  const int32_t* child_begin;
  const int32_t* child_count;
  const int32_t* root_begin;
  const int32_t* root_count;
  const double* eps;
  const int32_t* pairs;
  int64_t n_pairs;
  int64_t next;
  pthread_mutex_t mu;
} descent_job;

typedef struct {
  outbuf o;
  int64_t tests[64];
} descent_out;

static void descend(descent_job* J, descent_out* D, int32_t pr, int32_t a, int32_t b, int depth) {
  double A[9], B[9];
  load_tri(J->verts, J->tris, a, A);
  load_tri(J->verts, J->tris, b, B);
  tt_result r;
  tri_tri(A, B, &r);
  if (depth < 64) D->tests[depth]++;
  if (r.d > J->eps[a] + J->eps[b]) return;
  int fa = J->child_count[a] == 0, fb = J->child_count[b] == 0;
  if (fa && fb) {
    outbuf_push(&D->o, pr, a, b, &r);
    return;
  }
  int32_t ab = fa ? a : J->child_begin[a], an = fa ? 1 : J->child_count[a];
  int32_t bb = fb ? b : J->child_begin[b], bn = fb ? 1 : J->child_count[b];
  for (int32_t i = 0; i < an; ++i)
    for (int32_t j = 0; j < bn; ++j) descend(J, D, pr, ab + i, bb + j, depth + 1);
}

static void* descent_worker(void* arg) {
  void** a = (void**)arg;
  descent_job* J = (descent_job*)a[0];
  descent_out* D = (descent_out*)a[1];
  for (;;) {
    int64_t e;
    int64_t b = grab(&J->next, &J->mu, 1, J->n_pairs, &e);
    if (b >= J->n_pairs) break;
    int32_t pi = J->pairs[2 * b], pj = J->pairs[2 * b + 1];
    for (int32_t i = 0; i < J->root_count[pi]; ++i)
      for (int32_t j = 0; j < J->root_count[pj]; ++j)
        descend(J, D, (int32_t)b, J->root_begin[pi] + i, J->root_begin[pj] + j, 0);
  }
  return NULL;
}

int oracle_descent(const double* verts, const int32_t* tris, const int32_t* child_begin,
                   const int32_t* child_count, const int32_t* root_begin, const int32_t* root_count,
                   const double* eps, const int32_t* pairs, int64_t n_pairs, int n_threads,
                   int64_t* tests_per_depth, oracle_contacts* out) {
  memset(out, 0, sizeof(*out));
  for (int k = 0; k < 64; ++k) tests_per_depth[k] = 0;
  n_threads = clamp_threads(n_threads);
  descent_job J = {verts, tris, child_begin, child_count, root_begin, root_count, eps, pairs, n_pairs, 0};
  pthread_mutex_init(&J.mu, NULL);
  descent_out* outs = (descent_out*)calloc(n_threads, sizeof(descent_out));
  pthread_t th[256];
  void* args[256][2];
  for (int t = 0; t < n_threads; ++t) {
    args[t][0] = &J; args[t][1] = &outs[t];
    pthread_create(&th[t], NULL, descent_worker, args[t]);
  }
  for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
  pthread_mutex_destroy(&J.mu);
  int64_t total = 0;
  for (int t = 0; t < n_threads; ++t) {
    total += outs[t].o.n;
    for (int k = 0; k < 64; ++k) tests_per_depth[k] += outs[t].tests[k];
  }
  out->n = total;
  out->pair = (int32_t*)malloc((total ? total : 1) * sizeof(int32_t));
  out->ti = (int32_t*)malloc((total ? total : 1) * sizeof(int32_t));
  out->tj = (int32_t*)malloc((total ? total : 1) * sizeof(int32_t));
  out->rec = (double*)malloc((total ? total : 1) * 15 * sizeof(double));
  int64_t m = 0;
  for (int t = 0; t < n_threads; ++t) {
    for (int64_t i = 0; i < outs[t].o.n; ++i, ++m) {
      out->pair[m] = outs[t].o.pair[i];
      out->ti[m] = outs[t].o.ti[i];
      out->tj[m] = outs[t].o.tj[i];
      memcpy(out->rec + 15 * m, outs[t].o.rec + 15 * i, 15 * sizeof(double));
    }
    free(outs[t].o.pair); free(outs[t].o.ti); free(outs[t].o.tj); free(outs[t].o.rec);
  }
  free(outs);
  return 0;
}
