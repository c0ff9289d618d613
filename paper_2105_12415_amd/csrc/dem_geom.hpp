// Triangle geometry of the contact-detection path, for device and host.
//
// Two families of routines, both written for 64-lane SIMD execution (no
// data-dependent branches in the hot parts, selects instead):
//
//  * iterate_and_bound(): the paper's batched iterative closest-point solve
//    (Section 3, functional J and its modified Newton update; Algorithm 4
//    with a fixed iteration count) followed by a lower bound on the distance
//    obtained by projecting both triangles on the direction between the two
//    iterate points.  Any unit direction u gives
//        d(A,B) >= min_k u.b_k - max_k u.a_k,
//    so a pair whose bound exceeds its threshold is certainly not in contact
//    ("no contact" of the three-valued result) however far the iteration
//    got; a pair that is not pruned is "not terminated" unless the bound
//    also certifies the iterate's distance.
//
//  * exact_tri_tri(): the comparison-based distance (Section 3, direct
//    distance calculation): edge-against-triangle crossings give distance
//    0; otherwise the minimum of six point-to-triangle and nine
//    segment-to-segment distances.
//
// All positions are pair-local: triangle A is translated so that its first
// vertex is the origin, which keeps FP32 rounding proportional to the
// triangle sizes and their separation rather than to world coordinates.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>

#define DEM_HD __host__ __device__ __forceinline__

namespace dem {

// Type-exact math (float overloads on host and device).
DEM_HD float fm_(float a, float b, float c) { return fmaf(a, b, c); }
DEM_HD double fm_(double a, double b, double c) { return fma(a, b, c); }
DEM_HD float mn_(float a, float b) { return fminf(a, b); }
DEM_HD double mn_(double a, double b) { return fmin(a, b); }
DEM_HD float mx_(float a, float b) { return fmaxf(a, b); }
DEM_HD double mx_(double a, double b) { return fmax(a, b); }
DEM_HD float ab_(float a) { return fabsf(a); }
DEM_HD double ab_(double a) { return fabs(a); }
DEM_HD float sq_(float a) { return sqrtf(a); }
DEM_HD double sq_(double a) { return sqrt(a); }
// Half precision (the reduced-precision iteration): plain arithmetic in
// _Float16, fused multiply-add in one rounding.  NaN and infinity only ever
// reach the search direction, whose bound is formed in FP32 (see
// iterate_bound_mixed).
DEM_HD _Float16 fm_(_Float16 a, _Float16 b, _Float16 c) { return __builtin_fmaf16(a, b, c); }
DEM_HD _Float16 mn_(_Float16 a, _Float16 b) { return a < b ? a : b; }
DEM_HD _Float16 mx_(_Float16 a, _Float16 b) { return a > b ? a : b; }
DEM_HD _Float16 ab_(_Float16 a) { return a < _Float16(0) ? -a : a; }

template <typename T>
struct V3 {
  T x, y, z;
};

template <typename T>
DEM_HD V3<T> mk(T x, T y, T z) { return V3<T>{x, y, z}; }
template <typename T>
DEM_HD V3<T> operator+(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename T>
DEM_HD V3<T> operator-(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T>
DEM_HD V3<T> operator-(V3<T> a) { return {-a.x, -a.y, -a.z}; }
template <typename T>
DEM_HD V3<T> operator*(T s, V3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <typename T>
DEM_HD T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T>
DEM_HD V3<T> cross(V3<T> a, V3<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename T>
DEM_HD V3<T> fma3(T s, V3<T> d, V3<T> a) {  // a + s d
  return {fm_(s, d.x, a.x), fm_(s, d.y, a.y), fm_(s, d.z, a.z)};
}
template <typename T>
DEM_HD T clamp01(T v) { return mn_(mx_(v, T(0)), T(1)); }
template <typename T>
DEM_HD T sel(bool c, T a, T b) { return c ? a : b; }
template <typename T>
DEM_HD V3<T> sel(bool c, V3<T> a, V3<T> b) { return {c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z}; }
template <typename T>
DEM_HD T absmax3(V3<T> a) { return mx_(ab_(a.x), mx_(ab_(a.y), ab_(a.z))); }

DEM_HD float rsqrt_t(float v) { return 1.0f / sqrtf(v); }
DEM_HD double rsqrt_t(double v) { return 1.0 / sqrt(v); }

template <typename T>
struct Eps;
template <>
struct Eps<float> {
  static constexpr float u = 5.9604645e-8f;  // unit roundoff 2^-24
};
template <>
struct Eps<double> {
  static constexpr double u = 1.1102230246251565e-16;  // 2^-53
};

// Hardware reciprocal / reciprocal square root for FP32 on the device (1 ulp),
// used only where an approximate value is harmless: normalising the search
// direction (the bound's slack absorbs a 1-ulp length error) and projecting
// iterates into the triangle (only the direction depends on it).
DEM_HD float rcp_fast(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
DEM_HD double rcp_fast(double x) { return 1.0 / x; }
DEM_HD _Float16 rcp_fast(_Float16 x) { return _Float16(1) / x; }
DEM_HD float rsq_fast(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsqf(x);
#else
  return 1.0f / sqrtf(x);
#endif
}
DEM_HD double rsq_fast(double x) { return 1.0 / sqrt(x); }

// A triangle in "soup" form: first vertex, two edge vectors, epsilon, the
// negated damped Newton step lengths of its two barycentric parameters (ia,
// ib; see newton_steps), and a size bound (max|e1| + max|e2| over components)
// for the rounding slack.
template <typename T>
struct Tri {
  V3<T> v0, e1, e2;
  T eps, ia, ib, size;
};

// ------------------------------------------------------------------ iteration
struct IterParams {
  int n_iter;
  float nkappa;          // negated penalty half-step gain -alpha_it / (alpha_it + alpha_reg)
  int init_centroid;
};

DEM_HD float mn3_(float a, float b, float c) { return fminf(a, fminf(b, c)); }
DEM_HD double mn3_(double a, double b, double c) { return fmin(a, fmin(b, c)); }
DEM_HD _Float16 mn3_(_Float16 a, _Float16 b, _Float16 c) { return mn_(a, mn_(b, c)); }
DEM_HD float mx3_(float a, float b, float c) { return fmaxf(a, fmaxf(b, c)); }
DEM_HD double mx3_(double a, double b, double c) { return fmax(a, fmax(b, c)); }
DEM_HD _Float16 mx3_(_Float16 a, _Float16 b, _Float16 c) { return mx_(a, mx_(b, c)); }

// Stored step lengths of a triangle's two barycentric parameters in the
// damped diagonal-Newton update of the distance term (Section 3: Newton step
// with the diagonal of the Hessian, regularised by alpha_reg), negated so
// that every update of the iteration is an accumulating fused multiply-add:
//     x <- x + d_x (r . e_x),   d_x = -omega / (|e_x|^2 + alpha_reg),
// with alpha_reg = alpha_reg_rel (|e1|^2 + |e2|^2) / 2.  A parameter whose
// curvature is zero (an edge of zero length, no regularisation) keeps its
// value: step 0.
template <typename T>
DEM_HD void newton_steps(V3<T> e1, V3<T> e2, T areg_rel, T omega, T& d1, T& d2) {
  const T n1 = dot(e1, e1), n2 = dot(e2, e2);
  const T areg = areg_rel * T(0.5) * (n1 + n2);
  d1 = n1 + areg > T(0) ? -omega / (n1 + areg) : T(0);
  d2 = n2 + areg > T(0) ? -omega / (n2 + areg) : T(0);
}

// Half-step on the penalty part of J for one triangle's parameters: the
// quadratic exterior penalty alpha_it/2 sum max(0, g)^2 over the constraints
// g in {-a, -b, a + b - 1}, one Newton step with the curvature of one active
// constraint, alpha_it + alpha_reg, per coordinate (nk = -alpha_it /
// (alpha_it + alpha_reg)):
//     a <- a + nk (min(a, 0) + max(a + b - 1, 0)),  b likewise.
// Triangle B's parameters are kept negated, (c, d) = (-a2, -b2), so its
// constraints read c <= 0, d <= 0, c + d >= -1:
//     c <- c + nk (max(c, 0) + min(c + d + 1, 0)),  d likewise.
template <typename T>
DEM_HD void penalty_pos(T& a, T& b, T nk) {
  const T cs = mx_(a + b - T(1), T(0));
  const T ta = mn_(a, T(0)) + cs;
  const T tb = mn_(b, T(0)) + cs;
  a = fm_(nk, ta, a);
  b = fm_(nk, tb, b);
}
template <typename T>
DEM_HD void penalty_neg(T& c, T& d, T nk) {
  const T cs = mn_(c + d + T(1), T(0));
  const T tc = mx_(c, T(0)) + cs;
  const T td = mx_(d, T(0)) + cs;
  c = fm_(nk, tc, c);
  d = fm_(nk, td, d);
}

// N modified-Newton iterations on J (Section 3: a diagonal Newton step on the
// distance term, then a half-step on the constraint penalties; N fixed as in
// Algorithm 4) for triangles A, B in pair-local coordinates (A.v0 at the
// origin, B's first vertex at -D0).  Returns A's parameters (a1, b1) and B's
// negated, (c2, d2) = (-a2, -b2); the residual between the two points is
//     m = p_A - p_B = D0 + a1 e1A + b1 e2A + c2 e1B + d2 e2B.
template <typename T, int N>
DEM_HD void iterate_theta(const Tri<T>& A, const Tri<T>& B, V3<T> D0, const IterParams& ip, T& a1,
                          T& b1, T& c2, T& d2) {
  const T nk = T(ip.nkappa);
  V3<T> r;
  if (ip.init_centroid) {
    a1 = b1 = T(1) / T(3);
    c2 = d2 = -(T(1) / T(3));
    r = fma3(c2, B.e1 + B.e2, fma3(a1, A.e1 + A.e2, D0));
  } else {
    a1 = b1 = c2 = d2 = T(0);
    r = D0;
  }
#pragma unroll
  for (int it = 0; it < N; ++it) {
    if (it > 0) r = fma3(d2, B.e2, fma3(c2, B.e1, fma3(b1, A.e2, fma3(a1, A.e1, D0))));
    // gradient of 1/2 |r|^2 and the diagonal Newton step (A.ia ... B.ib hold
    // the negated step lengths)
    a1 = fm_(A.ia, dot(r, A.e1), a1);
    b1 = fm_(A.ib, dot(r, A.e2), b1);
    c2 = fm_(B.ia, dot(r, B.e1), c2);
    d2 = fm_(B.ib, dot(r, B.e2), d2);
    // constraint half-step
    penalty_pos(a1, b1, nk);
    penalty_neg(c2, d2, nk);
  }
}

// Lower bound on d(A, B) along the direction u = (p_B - p_A)/|p_B - p_A|
// between the iterate's points: any unit u gives
//     d(A, B) >= min_k u.w_k - max_k u.v_k
// (support of B minus support of A), which with m = p_A - p_B = -|m| u and
// A.v0 at the origin is
//     (m.D0 + min(0, m.e1A, m.e2A) - max(0, m.e1B, m.e2B)) / |m|.
// For m = 0 every product is 0 and so is the bound (nothing is pruned).
template <typename T>
DEM_HD T bound_along(const Tri<T>& A, const Tri<T>& B, V3<T> D0, T a1, T b1, T c2, T d2) {
  const V3<T> m = fma3(d2, B.e2, fma3(c2, B.e1, fma3(b1, A.e2, fma3(a1, A.e1, D0))));
  const T mm = dot(m, m);
  const T lo_a = mn3_(T(0), dot(m, A.e1), dot(m, A.e2));
  const T hi_b = mx3_(T(0), dot(m, B.e1), dot(m, B.e2));
  return (dot(m, D0) + lo_a - hi_b) * rsq_fast(mx_(mm, T(1e-30)));
}

// The iteration followed by the bound.  The final parameters are clamped to
// [0, 1] each (B's to [-1, 0]): the points then lie in the parallelograms
// spanned by the triangles' edges, which keeps the direction between them
// informative when the undamped Jacobi step has overshot (the bound itself
// holds for any direction).
template <typename T, int N>
DEM_HD T iterate_bound(const Tri<T>& A, const Tri<T>& B, V3<T> D0, const IterParams& ip) {
  T a1, b1, c2, d2;
  iterate_theta<T, N>(A, B, D0, ip, a1, b1, c2, d2);
  a1 = mn_(mx_(a1, T(0)), T(1));
  b1 = mn_(mx_(b1, T(0)), T(1));
  c2 = mx_(mn_(c2, T(0)), T(-1));
  d2 = mx_(mn_(d2, T(0)), T(-1));
  return bound_along(A, B, D0, a1, b1, c2, d2);
}

// Reduced-precision variant for FP32 scenes: the Newton iteration runs in
// half precision on the pair-local edges, offsets and step lengths; the
// bound along the resulting direction is formed in FP32.  The bound holds for
// any direction, so the half-precision rounding only changes how much is
// pruned, and the FP32 rounding slack (bound_slack) still covers the bound.
template <int N>
DEM_HD float iterate_bound_mixed(const Tri<float>& A, const Tri<float>& B, V3<float> D0, const IterParams& ip) {
  auto h3 = [](V3<float> v) { return V3<_Float16>{(_Float16)v.x, (_Float16)v.y, (_Float16)v.z}; };
  Tri<_Float16> Ah, Bh;
  Ah.e1 = h3(A.e1); Ah.e2 = h3(A.e2); Ah.ia = (_Float16)A.ia; Ah.ib = (_Float16)A.ib;
  Bh.e1 = h3(B.e1); Bh.e2 = h3(B.e2); Bh.ia = (_Float16)B.ia; Bh.ib = (_Float16)B.ib;
  _Float16 a1, b1, c2, d2;
  iterate_theta<_Float16, N>(Ah, Bh, h3(D0), ip, a1, b1, c2, d2);
  // back in FP32, clamped as in iterate_bound; a non-finite parameter
  // becomes 0 (a vertex; still a valid direction)
  auto fa = [](_Float16 v) { float x = (float)v; return x > 0.0f ? fminf(x, 1.0f) : 0.0f; };
  auto fb = [](_Float16 v) { float x = (float)v; return x < 0.0f ? fmaxf(x, -1.0f) : 0.0f; };
  return bound_along(A, B, D0, fa(a1), fa(b1), fb(c2), fb(d2));
}

// Rounding slack of the bound above: the computed bound of a pair at true
// distance d never exceeds d + slack (dot products of pair-local vectors in
// precision T, a 1-ulp direction length error, rounded soup edges).
template <typename T>
DEM_HD T bound_slack(const Tri<T>& A, const Tri<T>& B, V3<T> D0, T delta) {
  return T(64) * Eps<T>::u * (T(3) * (absmax3(D0) + A.size + B.size) + ab_(delta));
}

// Size bound stored with each soup triangle: max|e1| + max|e2| (components).
template <typename T>
DEM_HD T tri_size(V3<T> e1, V3<T> e2) { return absmax3(e1) + absmax3(e2); }

// ------------------------------------------------------------------ exact
// Barycentric weights of a point of a triangle in compact form (stored per
// contact for the adjoint): code 0 = an interior point, weights
// (1 - a - b, a, b); codes 1..4 = a point of the segment between two
// vertices with weight a at its second end: 1 = v0->v1, 2 = v1->v2,
// 3 = v2->v0, 4 = v0->v2 (a = 0 is the segment's first vertex).  Every
// producer of weights below forms them through bary_weights(), so a stored
// code reproduces its weights bit for bit.
template <typename T>
struct BaryCode {
  int code;
  T a, b;
};

template <typename T>
DEM_HD void bary_weights(int code, T a, T b, T w[3]) {
  const T c = T(1) - a;
  w[0] = code == 0 ? c - b : ((code == 1 || code == 4) ? c : (code == 3 ? a : T(0)));
  w[1] = (code == 0 || code == 1) ? a : (code == 2 ? c : T(0));
  w[2] = code == 0 ? b : ((code == 2 || code == 4) ? a : (code == 3 ? c : T(0)));
}

template <typename T>
DEM_HD void bary_weights(const BaryCode<T>& k, T w[3]) {
  bary_weights(k.code, k.a, k.b, w);
}

template <typename T>
struct Closest {
  T d2;         // squared distance
  V3<T> p, q;   // closest points on A and on B
  T wp[3], wq[3];
  int feature;  // 0-5 vertex-triangle, 6-14 edge-edge, 15 crossing
  BaryCode<T> cp, cq;  // wp = bary_weights(cp), wq = bary_weights(cq)
};

// Closest point of triangle (a, a+e1, a+e2) to x.  The projection onto the
// plane is written with the normal n = e1 x e2: the plane distance is
// (x-a).n/|n| and the barycentric coordinates are ratios of triple products,
// which keeps FP32 error proportional to the triangle size even for slivers
// (a Gram-matrix solve would lose the small angle to cancellation).  If the
// projection falls outside, the closest point lies on one of the edges, each
// a clamped 1-D projection.  Returns the squared distance.
template <typename T>
DEM_HD T point_tri(V3<T> x, V3<T> a, V3<T> e1, V3<T> e2, V3<T>& q, T w[3], BaryCode<T>& k) {
  V3<T> r = x - a;
  V3<T> n = cross(e1, e2);
  T nn = dot(n, n);
  T inn = nn > T(0) ? T(1) / nn : T(0);
  T s = dot(n, cross(r, e2)) * inn;
  T t = dot(n, cross(e1, r)) * inn;
  T hn = dot(r, n);
  bool inside = nn > T(0) && s >= T(0) && t >= T(0) && s + t <= T(1);
  T A11 = dot(e1, e1), A22 = dot(e2, e2);
  // edge 0: a -> a+e1 ; edge 1: a+e1 -> a+e2 ; edge 2: a -> a+e2
  T s0 = clamp01(A11 > T(0) ? dot(e1, r) / A11 : T(0));
  V3<T> q0 = fma3(s0, e1, a);
  V3<T> e3 = e2 - e1;
  T A33 = dot(e3, e3);
  T s1 = clamp01(A33 > T(0) ? dot(e3, r - e1) / A33 : T(0));
  V3<T> q1 = fma3(s1, e3, a + e1);
  T s2 = clamp01(A22 > T(0) ? dot(e2, r) / A22 : T(0));
  V3<T> q2 = fma3(s2, e2, a);
  V3<T> d0 = x - q0, d1 = x - q1, d2 = x - q2;
  T n0 = dot(d0, d0), n1 = dot(d1, d1), n2 = dot(d2, d2);
  // best edge (first minimum in edge order)
  T best = n0;
  V3<T> qb = q0;
  int code = 1;
  T ka = s0, kb = T(0);
  if (n1 < best) { best = n1; qb = q1; code = 2; ka = s1; }
  if (n2 < best) { best = n2; qb = q2; code = 4; ka = s2; }
  T din = hn * hn * inn;
  if (inside && din <= best) {
    best = din;
    qb = fma3(-hn * inn, n, x);
    code = 0; ka = s; kb = t;
  }
  q = qb;
  k.code = code; k.a = ka; k.b = kb;
  bary_weights(k, w);
  return best;
}

template <typename T>
DEM_HD T point_tri(V3<T> x, V3<T> a, V3<T> e1, V3<T> e2, V3<T>& q, T w[3]) {
  BaryCode<T> k;
  return point_tri(x, a, e1, e2, q, w, k);
}

// Closest points of segments p0 + s d1 and q0 + t d2, s, t in [0, 1]:
// s of the closest points of the two lines (clamped), t optimal for that s
// (clamped), then s re-optimised for a clamped t.  The line-line parameter
// comes from triple products with the common normal d1 x d2, which stays
// accurate in FP32 for nearly parallel segments.  The squared lengths of
// the two directions and their reciprocals are passed in (they are shared by
// the three edge pairs of each edge).  Returns the squared distance.
template <typename T>
DEM_HD T seg_seg_pre(V3<T> p0, V3<T> d1, T a, T ia, V3<T> q0, V3<T> d2, T e, T ie, T& s, T& t) {
  V3<T> r = p0 - q0;
  T f = dot(d2, r), c = dot(d1, r), b = dot(d1, d2);
  V3<T> n = cross(d1, d2);
  T nn = dot(n, n);
  bool skew = nn > T(64) * Eps<T>::u * Eps<T>::u * a * e && nn > T(0);
  T sl = clamp01(dot(cross(-r, d2), n) * rcp_fast(skew ? nn : T(1)));
  s = skew ? sl : T(0);
  t = (b * s + f) * ie;
  T s_lo = clamp01(-c * ia);
  T s_hi = clamp01((b - c) * ia);
  // a second segment of zero length is a point: t = 0 and s its projection
  bool lo = t < T(0) || !(e > T(0)), hi = t > T(1);
  s = lo ? s_lo : (hi ? s_hi : s);
  t = lo ? T(0) : (hi ? T(1) : t);
  V3<T> dd = fma3(s, d1, r) - t * d2;
  return dot(dd, dd);
}

template <typename T>
DEM_HD V3<T> pick3(int k, V3<T> x0, V3<T> x1, V3<T> x2) {
  return sel(k == 0, x0, sel(k == 1, x1, x2));
}
template <typename T>
DEM_HD T pick3(int k, T x0, T x1, T x2) {
  return k == 0 ? x0 : (k == 1 ? x1 : x2);
}

// Crossing tests of the three edges of triangle X (vertices x_k, edges
// x_k -> x_k+1, heights h_k of the vertices over Y's plane along n_Y) through
// triangle Y (vertices y_k, edges g_k): an edge whose end heights differ in
// sign meets the plane at one point, which must lie on the inner side of all
// three edges of Y (in-plane inward normals n_Y x g_k).  The first hit in
// edge order is kept.
template <typename T>
DEM_HD void crossings(const V3<T> (&X)[3], const V3<T> (&EX)[3], const T (&h)[3], const V3<T> (&Y)[3],
                      const V3<T> (&EY)[3], V3<T> nY, bool ok, bool& hit, V3<T>& xh) {
  const V3<T> m0 = cross(nY, EY[0]), m1 = cross(nY, EY[1]), m2 = cross(nY, EY[2]);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T h0 = h[k], h1 = h[(k + 1) % 3];
    const bool straddle = (h0 <= T(0) && h1 >= T(0)) || (h0 >= T(0) && h1 <= T(0));
    const bool flat = h0 == T(0) && h1 == T(0);
    const T den = h0 - h1;
    const T tt = den != T(0) ? h0 * rcp_fast(den) : T(0);
    const V3<T> x = fma3(tt, EX[k], X[k]);
    const bool inside = dot(m0, x - Y[0]) >= T(0) && dot(m1, x - Y[1]) >= T(0) && dot(m2, x - Y[2]) >= T(0);
    const bool c = ok && straddle && !flat && inside;
    xh = sel(c && !hit, x, xh);
    hit = hit || c;
  }
}

// Vertices of X against the interior of triangle Y = (y0, y0+g1, y0+g2):
// barycentric coordinates from the in-plane gradients (g2 x n)/|n|^2 and
// (n x g1)/|n|^2, squared distance h^2/|n|^2 from the heights.  A candidate
// replaces the best one only if strictly closer.
template <typename T>
DEM_HD void vertex_face(const V3<T> (&X)[3], const T (&h)[3], V3<T> y0, V3<T> g1, V3<T> g2, V3<T> nY,
                        T nn, int feat0, T& best, T& bs, T& bt, int& feat) {
  const T inn = nn > T(0) ? rcp_fast(nn) : T(0);
  const V3<T> gs = cross(g2, nY), gt = cross(nY, g1);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const V3<T> r = X[k] - y0;
    const T s = dot(r, gs) * inn, t = dot(r, gt) * inn;
    const T din = h[k] * h[k] * inn;
    const bool c = nn > T(0) && s >= T(0) && t >= T(0) && s + t <= T(1) && din < best;
    best = c ? din : best;
    bs = c ? s : bs;
    bt = c ? t : bt;
    feat = c ? feat0 + k : feat;
  }
}

// Exact distance between A = (a0, a0+e1, a0+e2) and B = (b0, b0+f1, b0+f2)
// by the comparison-based method (Section 3, direct distance calculation):
//  1. six edge-through-triangle crossing tests (a hit means distance 0);
//  2. otherwise the minimum over the six vertex-triangle and nine edge-edge
//     distances.  A vertex whose projection onto the other triangle's plane
//     falls outside that triangle has its closest point on one of that
//     triangle's edges, and the edge-edge distance of an edge through the
//     vertex is no larger, so only interior projections are candidates.
// Per-triangle quantities (normal, heights of each vertex over the other
// plane, edge reciprocals) are formed once; the search keeps (distance,
// feature, two parameters) and the closest points and weights are rebuilt
// for the winner only.
template <typename T>
DEM_HD void exact_tri_tri(V3<T> a0, V3<T> e1, V3<T> e2, V3<T> b0, V3<T> f1, V3<T> f2,
                          Closest<T>& out) {
  const V3<T> A[3] = {a0, a0 + e1, a0 + e2};
  const V3<T> B[3] = {b0, b0 + f1, b0 + f2};
  const V3<T> EA[3] = {e1, e2 - e1, -e2};  // edge k: vertex k -> vertex k+1
  const V3<T> EB[3] = {f1, f2 - f1, -f2};
  const V3<T> nA = cross(e1, e2), nB = cross(f1, f2);
  const T nnA = dot(nA, nA), nnB = dot(nB, nB);
  // heights of A's vertices over B's plane and of B's over A's (unnormalised)
  const T hA[3] = {dot(nB, A[0] - b0), dot(nB, A[1] - b0), dot(nB, A[2] - b0)};
  const T hB[3] = {dot(nA, B[0] - a0), dot(nA, B[1] - a0), dot(nA, B[2] - a0)};
  // 1. crossings
  bool hit = false;
  V3<T> xh = a0;
  crossings(A, EA, hA, B, EB, nB, nnB > T(0), hit, xh);
  crossings(B, EB, hB, A, EA, nA, nnA > T(0), hit, xh);
  // 2a. vertices against the interior of the other triangle
  T best = T(INFINITY), bs = T(0), bt = T(0);
  int feat = 0;
  vertex_face(A, hA, b0, f1, f2, nB, nnB, 0, best, bs, bt, feat);
  vertex_face(B, hB, a0, e1, e2, nA, nnA, 3, best, bs, bt, feat);
  // 2b. edges against edges
  // (the loop over A's edges stays rolled, its edge picked by selects, so
  // that only three edge pairs are in flight at once: register pressure)
#pragma unroll 1
  for (int i = 0; i < 3; ++i) {
    const V3<T> Ai = pick3(i, A[0], A[1], A[2]), EAi = pick3(i, EA[0], EA[1], EA[2]);
    const T aa = dot(EAi, EAi);
    const T ia = aa > T(0) ? rcp_fast(aa) : T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const T ee = dot(EB[j], EB[j]);
      const T ie = ee > T(0) ? rcp_fast(ee) : T(0);
      T s, t;
      const T d2 = seg_seg_pre(Ai, EAi, aa, ia, B[j], EB[j], ee, ie, s, t);
      const bool c = d2 < best;
      best = c ? d2 : best;
      bs = c ? s : bs;
      bt = c ? t : bt;
      feat = c ? 6 + 3 * i + j : feat;
    }
  }
  // closest points and weights of the winning feature
  V3<T> bp, bq;
  if (feat < 6) {
    const bool fromB = feat >= 3;
    const int k = fromB ? feat - 3 : feat;
    // (component-wise selects: a select of whole structs would be lowered
    // through private memory)
    // (normal and height recomputed: keeping them live through the
    // edge-edge search costs registers)
    const V3<T> x = sel(fromB, pick3(k, B[0], B[1], B[2]), pick3(k, A[0], A[1], A[2]));
    const V3<T> nY = sel(fromB, cross(e1, e2), cross(f1, f2));
    const T h = dot(nY, x - sel(fromB, a0, b0));
    const T nn = dot(nY, nY);
    // foot of the perpendicular along the normal (no cancellation in q - p)
    const V3<T> y = fma3(-h * rcp_fast(nn), nY, x);
    bp = sel(fromB, y, x);
    bq = sel(fromB, x, y);
    // the face side interior (bs, bt), the vertex side its vertex k
    out.cp.code = fromB ? 0 : 1 + k;
    out.cp.a = fromB ? bs : T(0);
    out.cp.b = fromB ? bt : T(0);
    out.cq.code = fromB ? 1 + k : 0;
    out.cq.a = fromB ? T(0) : bs;
    out.cq.b = fromB ? T(0) : bt;
  } else {
    const int i = (feat - 6) / 3, j = (feat - 6) - 3 * ((feat - 6) / 3);
    bp = fma3(bs, pick3(i, EA[0], EA[1], EA[2]), pick3(i, A[0], A[1], A[2]));
    bq = fma3(bt, pick3(j, EB[0], EB[1], EB[2]), pick3(j, B[0], B[1], B[2]));
    // edge k runs from vertex k to vertex k + 1 (mod 3): codes 1, 2, 3
    out.cp = BaryCode<T>{1 + i, bs, T(0)};
    out.cq = BaryCode<T>{1 + j, bt, T(0)};
  }
  if (hit) {
    best = T(0); bp = xh; bq = xh; feat = 15;
  }
  out.d2 = best;
  out.p = bp;
  out.q = bq;
  bary_weights(out.cp, out.wp);
  bary_weights(out.cq, out.wq);
  out.feature = feat;
}

// ------------------------------------------------------------------ certificate
// Certified hybrid result for a pair the bound did not prune (Algorithm 4's
// "found a contact point / no contact / not terminated", with the heuristic
// convergence test replaced by a proof): the iterate's point on A is snapped
// to the exact closest point on B, that one back onto A, and once more onto
// B (alternating projections converge to a closest pair of the two convex
// sets).  With U = |q - p| (an upper bound: both points are feasible) and
// the separation bound L* along u = (q - p)/U, the distance lies in
// [L*, U]; when U - L* <= tol, U is accepted as the distance.  Otherwise the
// pair is "not terminated" and needs the comparison-based fallback.
template <typename T, int N>
DEM_HD bool certify_pair(const Tri<T>& A, const Tri<T>& B, V3<T> D0, const IterParams& ip, T rel_tol,
                         T abs_tol, T& d, V3<T>& p, V3<T>& q, T wp[3], T wq[3], BaryCode<T>& kp,
                         BaryCode<T>& kq) {
  T a1, b1, nb1, nb2;  // B's negated parameters are not needed here
  iterate_theta<T, N>(A, B, D0, ip, a1, b1, nb1, nb2);
  const V3<T> z = {T(0), T(0), T(0)};
  const V3<T> b0 = -D0;
  V3<T> p1 = fma3(a1, A.e1, b1 * A.e2);
  V3<T> q1;
  point_tri(p1, b0, B.e1, B.e2, q1, wq, kq);
  point_tri(q1, z, A.e1, A.e2, p, wp, kp);
  T d2 = point_tri(p, b0, B.e1, B.e2, q, wq, kq);
  T U = sq_(d2);
  V3<T> w = q - p;
  V3<T> u = (U > T(0) ? T(1) / U : T(0)) * w;
  T hA = mx_(T(0), mx_(dot(u, A.e1), dot(u, A.e2)));
  T hB = mn_(T(0), mn_(dot(u, B.e1), dot(u, B.e2))) - dot(u, D0);
  T Ls = hB - hA;
  d = U;
  return U > abs_tol && (U - Ls) <= rel_tol * U + abs_tol;
}

template <typename T, int N>
DEM_HD bool certify_pair(const Tri<T>& A, const Tri<T>& B, V3<T> D0, const IterParams& ip, T rel_tol,
                         T abs_tol, T& d, V3<T>& p, V3<T>& q, T wp[3], T wq[3]) {
  BaryCode<T> kp, kq;
  return certify_pair<T, N>(A, B, D0, ip, rel_tol, abs_tol, d, p, q, wp, wq, kp, kq);
}

}  // namespace dem
