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
DEM_HD float rsq_fast(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsqf(x);
#else
  return 1.0f / sqrtf(x);
#endif
}
DEM_HD double rsq_fast(double x) { return 1.0 / sqrt(x); }

// A triangle in "soup" form: first vertex, two edge vectors, epsilon,
// diagonal of the regularised Hessian block (inverted) for its two
// barycentric parameters, and a size bound (max|e1| + max|e2| over
// components) for the rounding slack.
template <typename T>
struct Tri {
  V3<T> v0, e1, e2;
  T eps, ia, ib, size;
};

// ------------------------------------------------------------------ iteration
struct IterParams {
  int n_iter;
  float omega;
  float kappa1, kappa2;  // penalty half-step gains for 1 and 2 active constraints
  int init_centroid;
};

// One half-step on the penalty part of J for the parameters (a, b) of one
// triangle: quadratic exterior penalty alpha_it/2 * sum max(0, g)^2 over
// g in {-a, -b, a+b-1} (reading of the constraint terms), Hessian diagonal
// alpha_it * (#active constraints on the coordinate), regularised by
// alpha_reg.  With kappa_m = alpha_it / (m alpha_it + alpha_reg) the step is
// a scaled projection back onto the triangle.
template <typename T>
DEM_HD void penalty_half_step(T& a, T& b, T k1, T k2) {
  T ca = mx_(-a, T(0));
  T cb = mx_(-b, T(0));
  T cs = mx_(a + b - T(1), T(0));
  bool sa = cs > T(0);
  T ka = (ca > T(0) && sa) ? k2 : k1;
  T kb = (cb > T(0) && sa) ? k2 : k1;
  a += ka * (ca - cs);
  b += kb * (cb - cs);
}

// Point of the triangle for parameters (a, b) pulled into a, b >= 0 and
// rescaled onto a + b <= 1 (it only fixes the search direction).
template <typename T>
DEM_HD void to_simplex(T& a, T& b) {
  a = mx_(a, T(0));
  b = mx_(b, T(0));
  T inv = rcp_fast(mx_(a + b, T(1)));
  a *= inv;
  b *= inv;
}

// N modified-Newton iterations on J (Section 3: diagonal Newton step on the
// distance term, then a half-step on the constraint penalties; N fixed as
// in Algorithm 4) for triangles A, B in pair-local coordinates (A.v0 at the
// origin, B's first vertex at -D0).  Leaves the parameters projected into
// the two triangles.
template <typename T, int N>
DEM_HD void iterate_theta(const Tri<T>& A, const Tri<T>& B, V3<T> D0, const IterParams& ip, T& a1,
                          T& b1, T& a2, T& b2) {
  const T om = T(ip.omega), k1 = T(ip.kappa1), k2 = T(ip.kappa2);
  // damped inverse diagonal of the regularised Hessian, per parameter
  const T s1 = om * A.ia, s2 = om * A.ib, s3 = om * B.ia, s4 = om * B.ib;
  V3<T> r;  // residual t_A(a1,b1) - t_B(a2,b2)
  if (ip.init_centroid) {
    a1 = b1 = a2 = b2 = T(1) / T(3);
    r = fma3(a1, A.e1 + A.e2, fma3(-a2, B.e1 + B.e2, D0));
  } else {
    a1 = b1 = a2 = b2 = T(0);
    r = D0;
  }
#pragma unroll
  for (int it = 0; it < N; ++it) {
    if (it > 0) r = fma3(a1, A.e1, fma3(b1, A.e2, fma3(-a2, B.e1, fma3(-b2, B.e2, D0))));
    // gradient of 1/2 |r|^2 and the diagonal Newton step
    a1 -= s1 * dot(r, A.e1);
    b1 -= s2 * dot(r, A.e2);
    a2 += s3 * dot(r, B.e1);
    b2 += s4 * dot(r, B.e2);
    // constraint half-step
    penalty_half_step(a1, b1, k1, k2);
    penalty_half_step(a2, b2, k1, k2);
  }
  to_simplex(a1, b1);
  to_simplex(a2, b2);
}

// The iteration followed by the lower bound on the distance along the unit
// direction u between the two iterate points:
//     d(A, B) >= min_k u.b_k - max_k u.a_k.
// Returns the bound (-inf if the two points coincide: nothing is pruned).
template <typename T, int N>
DEM_HD T iterate_bound(const Tri<T>& A, const Tri<T>& B, V3<T> D0, const IterParams& ip) {
  T a1, b1, a2, b2;
  iterate_theta<T, N>(A, B, D0, ip, a1, b1, a2, b2);
  // w = p2 - p1 between the two (feasible) iterate points
  V3<T> w = fma3(a2, B.e1, fma3(b2, B.e2, fma3(-a1, A.e1, fma3(-b1, A.e2, -D0))));
  T ww = dot(w, w);
  V3<T> u = rsq_fast(mx_(ww, T(1e-30))) * w;
  // support of A along u (max) and of B along u (min)
  T hA = mx_(T(0), mx_(dot(u, A.e1), dot(u, A.e2)));
  T hB = mn_(T(0), mn_(dot(u, B.e1), dot(u, B.e2))) - dot(u, D0);
  return ww > T(0) ? hB - hA : -T(INFINITY);
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
template <typename T>
struct Closest {
  T d2;         // squared distance
  V3<T> p, q;   // closest points on A and on B
  T wp[3], wq[3];
  int feature;  // 0-5 vertex-triangle, 6-14 edge-edge, 15 crossing
};

// Closest point of triangle (a, a+e1, a+e2) to x.  The projection onto the
// plane is written with the normal n = e1 x e2: the plane distance is
// (x-a).n/|n| and the barycentric coordinates are ratios of triple products,
// which keeps FP32 error proportional to the triangle size even for slivers
// (a Gram-matrix solve would lose the small angle to cancellation).  If the
// projection falls outside, the closest point lies on one of the edges, each
// a clamped 1-D projection.  Returns the squared distance.
template <typename T>
DEM_HD T point_tri(V3<T> x, V3<T> a, V3<T> e1, V3<T> e2, V3<T>& q, T w[3]) {
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
  T wa = T(1) - s0, wb = s0, wc = T(0);
  if (n1 < best) { best = n1; qb = q1; wa = T(0); wb = T(1) - s1; wc = s1; }
  if (n2 < best) { best = n2; qb = q2; wa = T(1) - s2; wb = T(0); wc = s2; }
  T din = hn * hn * inn;
  if (inside && din <= best) {
    best = din;
    qb = fma3(-hn * inn, n, x);
    wa = T(1) - s - t; wb = s; wc = t;
  }
  q = qb;
  w[0] = wa; w[1] = wb; w[2] = wc;
  return best;
}

// Closest points of segments p0 + s d1 and q0 + t d2, s, t in [0, 1]:
// s of the closest points of the two lines (clamped), t optimal for that s
// (clamped), then s re-optimised for a clamped t.  The line-line parameter
// comes from triple products with the common normal d1 x d2, which stays
// accurate in FP32 for nearly parallel segments.  Squared distance.
template <typename T>
DEM_HD T seg_seg(V3<T> p0, V3<T> d1, V3<T> q0, V3<T> d2, T& s, T& t, V3<T>& cp, V3<T>& cq) {
  V3<T> r = p0 - q0;
  T a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r);
  T c = dot(d1, r), b = dot(d1, d2);
  V3<T> n = cross(d1, d2);
  T nn = dot(n, n);
  bool skew = nn > T(64) * Eps<T>::u * Eps<T>::u * a * e && nn > T(0);
  s = skew ? clamp01(dot(cross(-r, d2), n) / nn) : T(0);
  T ie = e > T(0) ? T(1) / e : T(0);
  T ia = a > T(0) ? T(1) / a : T(0);
  t = (b * s + f) * ie;
  T s_lo = clamp01(-c * ia);
  T s_hi = clamp01((b - c) * ia);
  bool lo = t < T(0), hi = t > T(1);
  s = lo ? s_lo : (hi ? s_hi : s);
  t = lo ? T(0) : (hi ? T(1) : t);
  cp = fma3(s, d1, p0);
  cq = fma3(t, d2, q0);
  V3<T> dd = cp - cq;
  return dot(dd, dd);
}

// Does segment p0 -> p0 + d cross the plane of triangle (a, a+e1, a+e2)
// inside the triangle?  Segments lying in the plane are left to the distance
// tests.  On a hit x is the crossing point.
template <typename T>
DEM_HD bool seg_crosses(V3<T> p0, V3<T> d, V3<T> a, V3<T> e1, V3<T> e2, V3<T>& x) {
  V3<T> n = cross(e1, e2);
  T h0 = dot(n, p0 - a);
  T h1 = dot(n, p0 + d - a);
  bool straddle = (h0 <= T(0) && h1 >= T(0)) || (h0 >= T(0) && h1 <= T(0));
  bool flat = (h0 == T(0) && h1 == T(0));
  T den = h0 - h1;
  T tt = den != T(0) ? h0 / den : T(0);
  x = fma3(tt, d, p0);
  // x inside: on the inner side of each edge (edge normals n x edge)
  V3<T> b = a + e1, c = a + e2;
  T s0 = dot(n, cross(e1, x - a));
  T s1 = dot(n, cross(c - b, x - b));
  T s2 = dot(n, cross(a - c, x - c));
  bool inside = s0 >= T(0) && s1 >= T(0) && s2 >= T(0);
  return straddle && !flat && inside && dot(n, n) > T(0);
}

// Exact distance between A = (a0, a0+e1, a0+e2) and B = (b0, b0+f1, b0+f2).
template <typename T>
DEM_HD void exact_tri_tri(V3<T> a0, V3<T> e1, V3<T> e2, V3<T> b0, V3<T> f1, V3<T> f2,
                          Closest<T>& out) {
  V3<T> A[3] = {a0, a0 + e1, a0 + e2};
  V3<T> B[3] = {b0, b0 + f1, b0 + f2};
  // crossings: edges of A through B, edges of B through A
  bool hit = false;
  V3<T> xh = a0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    V3<T> x;
    if (seg_crosses(A[k], A[(k + 1) % 3] - A[k], b0, f1, f2, x) && !hit) { hit = true; xh = x; }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    V3<T> x;
    if (seg_crosses(B[k], B[(k + 1) % 3] - B[k], a0, e1, e2, x) && !hit) { hit = true; xh = x; }
  }
  T best = T(INFINITY);
  V3<T> bp = a0, bq = b0;
  T wp0 = 1, wp1 = 0, wp2 = 0, wq0 = 1, wq1 = 0, wq2 = 0;
  int feat = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {  // vertex k of A against B
    V3<T> q;
    T w[3];
    T d2 = point_tri(A[k], b0, f1, f2, q, w);
    if (d2 < best) {
      best = d2; bp = A[k]; bq = q; feat = k;
      wp0 = T(k == 0); wp1 = T(k == 1); wp2 = T(k == 2);
      wq0 = w[0]; wq1 = w[1]; wq2 = w[2];
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {  // vertex k of B against A
    V3<T> q;
    T w[3];
    T d2 = point_tri(B[k], a0, e1, e2, q, w);
    if (d2 < best) {
      best = d2; bp = q; bq = B[k]; feat = 3 + k;
      wp0 = w[0]; wp1 = w[1]; wp2 = w[2];
      wq0 = T(k == 0); wq1 = T(k == 1); wq2 = T(k == 2);
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T s, t;
      V3<T> cp, cq;
      T d2 = seg_seg(A[i], A[(i + 1) % 3] - A[i], B[j], B[(j + 1) % 3] - B[j], s, t, cp, cq);
      if (d2 < best) {
        best = d2; bp = cp; bq = cq; feat = 6 + 3 * i + j;
        wp0 = (i == 0) ? T(1) - s : ((i == 2) ? s : T(0));
        wp1 = (i == 1) ? T(1) - s : ((i == 0) ? s : T(0));
        wp2 = (i == 2) ? T(1) - s : ((i == 1) ? s : T(0));
        wq0 = (j == 0) ? T(1) - t : ((j == 2) ? t : T(0));
        wq1 = (j == 1) ? T(1) - t : ((j == 0) ? t : T(0));
        wq2 = (j == 2) ? T(1) - t : ((j == 1) ? t : T(0));
      }
    }
  }
  if (hit) {
    best = T(0); bp = xh; bq = xh; feat = 15;
  }
  out.d2 = best;
  out.p = bp;
  out.q = bq;
  out.wp[0] = wp0; out.wp[1] = wp1; out.wp[2] = wp2;
  out.wq[0] = wq0; out.wq[1] = wq1; out.wq[2] = wq2;
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
                         T abs_tol, T& d, V3<T>& p, V3<T>& q, T wp[3], T wq[3]) {
  T a1, b1, a2, b2;
  iterate_theta<T, N>(A, B, D0, ip, a1, b1, a2, b2);
  const V3<T> z = {T(0), T(0), T(0)};
  const V3<T> b0 = -D0;
  V3<T> p1 = fma3(a1, A.e1, b1 * A.e2);
  V3<T> q1;
  point_tri(p1, b0, B.e1, B.e2, q1, wq);
  point_tri(q1, z, A.e1, A.e2, p, wp);
  T d2 = point_tri(p, b0, B.e1, B.e2, q, wq);
  T U = sq_(d2);
  V3<T> w = q - p;
  V3<T> u = (U > T(0) ? T(1) / U : T(0)) * w;
  T hA = mx_(T(0), mx_(dot(u, A.e1), dot(u, A.e2)));
  T hB = mn_(T(0), mn_(dot(u, B.e1), dot(u, B.e2))) - dot(u, D0);
  T Ls = hB - hA;
  d = U;
  return U > abs_tol && (U - Ls) <= rel_tol * U + abs_tol;
}

}  // namespace dem
