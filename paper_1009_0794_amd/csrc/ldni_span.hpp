// ldni_span.hpp -- the exact coverage predicate of one pixel centre and the
// conservative column span of a triangle on one pixel row.  Host and device
// code: the sampling kernels use both; the library's span self-test runs
// them on the host against every pixel of a triangle's rectangle.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ldni {

// Orientation of the ray with respect to the directed edge P->Q, both
// endpoints already translated into the ray frame.  The two products of
// float32 values are exact in float64, so the sign of the difference is
// exact.  A ray exactly on the edge line is decided as if displaced by
// (+eps, +eps^2): the edge below the ray (larger v) owns it, then the one to
// its left.
__host__ __device__ __forceinline__ int orient(float pu, float pv, float qu, float qv) {
  const double e = (double)pu * (double)qv - (double)pv * (double)qu;
  int s = (e > 0.0) - (e < 0.0);
  if (s == 0) s = (pv > qv) - (pv < qv);
  if (s == 0) s = (qu > pu) - (qu < pu);
  return s;
}

// Edge functions of a covered candidate (the depth needs them).
struct Edges {
  double ab, bc, ca;
};

// Exact coverage of the ray (ru, rv) by the triangle whose vertices are
// (au,av), (bu,bv), (cu,cv) (Definition 1 with the tie rule above): tav,
// tbv, tcv are the float32 v-translations of the row and dav, dbv, dcv the
// same values in float64.  Each edge function is one exact product plus one
// fused multiply-add: since both products of float32 values are exact in
// float64, the FMA returns the same correctly rounded difference as two
// products and a subtraction.  Hit iff all three signs agree and are not 0.
__host__ __device__ __forceinline__ bool covered(float au, float bu, float cu, float tav, float tbv, float tcv,
                                                 double dav, double dbv, double dcv, float ru, Edges& e) {
  const float tau = au - ru, tbu = bu - ru, tcu = cu - ru;
  const double dau = tau, dbu = tbu, dcu = tcu;
  e.ab = fma(dau, dbv, -(dav * dbu));
  e.bc = fma(dbu, dcv, -(dbv * dcu));
  e.ca = fma(dcu, dav, -(dcv * dau));
  const double mn = fmin(fmin(e.ab, e.bc), e.ca), mx = fmax(fmax(e.ab, e.bc), e.ca);
  if ((mn > 0.0) | (mx < 0.0)) return true;   // one strict sign
  if ((mn < 0.0) & (mx > 0.0)) return false;  // two strictly opposite signs: no tie can help
  const int s0 = orient(tau, tav, tbu, tbv);
  const int s1 = orient(tbu, tbv, tcu, tcv);
  const int s2 = orient(tcu, tcv, tau, tav);
  return (s0 != 0) & (s0 == s1) & (s1 == s2);
}

// ---------------------------------------------------------------------------
// Conservative span of a triangle on a pixel row
// ---------------------------------------------------------------------------
// On the row with centre v = cv, an edge X->Y of the real triangle (exact
// translations) has edge function E(c) = -dv (c - c*) in the pixel-centre
// coordinate c, with dv = Yv - Xv and c* = Xu + (cv - Xv) du/dv where the
// edge line meets the row.  Inside the triangle every E has the sign s of
// its signed area, so an edge with s*dv > 0 bounds c from above by c*, one
// with s*dv < 0 from below.  The exact predicate works on float32
// translations, which moves each E by at most tau = 2^-22 Wu Wv for pixel
// centres inside the triangle's rectangle (Wu, Wv its extents): a hit still
// has s*E >= -tau, so c* moves by at most tau / |dv| (the band below, taken
// eight times larger, in float32 with an approximate reciprocal).  When
// |area| is below 2^-16 Wu Wv the sign s itself is not trusted and the row
// is not clipped; an edge with |dv| below 2^-16 Wv (nearly parallel to the
// rows) or an inverse slope beyond 2^30 gives no bound.  The slope du/dv is
// formed in float32 with a reciprocal good to one ulp (relative error below
// 2^-21), so c* = fma(cv - Xv, g, Xu) is off by less than
// 2^-21 |c* - Xu| + 2^-24 |c*|.  Wherever such a bound can cut off a pixel of
// the rectangle, |c* - Xu| <= Wu + band and |c*| <= U + Wu (U the largest
// |u| of the vertices); the margin adds 2^-19 Wu + 2^-21 (U + Wu), twice
// that.  (A bound far outside the rectangle either does not bind or empties
// a row that holds no hit; its error, a tiny fraction of its distance, keeps
// it so.)
struct SpanPrep {
  // per edge X->Y (AB, BC, CA): X's u and v, du/dv, and what the edge adds
  // to its crossing c* for the row's lower bound (-margin, or -inf when it
  // is no lower bound) and for the upper bound (+margin, or +inf)
  float xu[3], xv[3], g[3], lo_add[3], hi_add[3];
  // Inner span: a pixel centre c with c >= c* + margin for every lower edge
  // and c <= c* - margin for every upper edge has s*E > tau on all three
  // edges, so every float32-translated edge function has the strict sign s:
  // a hit, with no tie involved.  Only when all three edges give a bound.
  bool inner;
};

__host__ __device__ __forceinline__ float approx_rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}

__host__ __device__ __forceinline__ SpanPrep span_prep(float au, float av, float bu, float bv, float cu,
                                                       float cv) {
  SpanPrep s;
  const float pu[3] = {au, bu, cu}, pv[3] = {av, bv, cv};
  const float wu = fmaxf(fmaxf(au, bu), cu) - fminf(fminf(au, bu), cu);
  const float wv = fmaxf(fmaxf(av, bv), cv) - fminf(fminf(av, bv), cv);
  // twice the signed area: products of float32 differences, exact in float64
  // up to the one rounding of each difference
  const double area2 = ((double)bu - (double)au) * ((double)cv - (double)av) -
                       ((double)bv - (double)av) * ((double)cu - (double)au);
  const float uabs = fmaxf(fmaxf(fabsf(au), fabsf(bu)), fabsf(cu));
  const bool clip = fabs(area2) > (double)wu * (double)wv * 0x1.0p-16 && wu > 0.0f && wv > 0.0f;
  const bool pos = area2 > 0.0;
  const float base = wu * 0x1.0p-19f + (uabs + wu) * 0x1.0p-21f;
  const float bandk = wu * wv * 0x1.0p-19f;
  const float wv16 = wv * 0x1.0p-16f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int k2 = k == 2 ? 0 : k + 1;
    const float du = pu[k2] - pu[k], dv = pv[k2] - pv[k];
    const float rinv = approx_rcp(dv);
    const float g = du * rinv;
    const bool use = clip && fabsf(dv) >= wv16 && fabsf(g) <= 1073741824.0f;
    const float m = base + bandk * fabsf(rinv);
    const bool upper = (dv > 0.0f) == pos;
    s.xu[k] = pu[k];
    s.xv[k] = pv[k];
    s.g[k] = use ? g : 0.0f;
    s.lo_add[k] = (use && !upper) ? -m : -INFINITY;
    s.hi_add[k] = (use && upper) ? m : INFINITY;
    s.inner = (k == 0 ? true : s.inner) && use;
  }
  return s;
}

// The u interval [lo, hi] of certain hits on the row (empty, lo > hi, when
// the entry has no inner span): each edge's bound moved inward by its margin.
__host__ __device__ __forceinline__ void span_inner(const SpanPrep& s, float rv, float& lo, float& hi) {
  if (!s.inner) {
    lo = INFINITY;
    hi = -INFINITY;
    return;
  }
  const float c0 = fmaf(rv - s.xv[0], s.g[0], s.xu[0]);
  const float c1 = fmaf(rv - s.xv[1], s.g[1], s.xu[1]);
  const float c2 = fmaf(rv - s.xv[2], s.g[2], s.xu[2]);
  // lo_add is -margin for a lower edge and -inf for an upper one: -lo_add is
  // +margin / +inf, and a lower bound must use +margin, an upper edge none
  const float l0 = s.lo_add[0] > -INFINITY ? c0 - s.lo_add[0] : -INFINITY;
  const float l1 = s.lo_add[1] > -INFINITY ? c1 - s.lo_add[1] : -INFINITY;
  const float l2 = s.lo_add[2] > -INFINITY ? c2 - s.lo_add[2] : -INFINITY;
  const float h0 = s.hi_add[0] < INFINITY ? c0 - s.hi_add[0] : INFINITY;
  const float h1 = s.hi_add[1] < INFINITY ? c1 - s.hi_add[1] : INFINITY;
  const float h2 = s.hi_add[2] < INFINITY ? c2 - s.hi_add[2] : INFINITY;
  lo = fmaxf(fmaxf(l0, l1), l2);
  hi = fminf(fminf(h0, h1), h2);
}

// The u interval [lo, hi] outside which no pixel centre of the row can be
// covered (lo = -inf / hi = +inf when unbounded).  Branch-free: an edge that
// gives no bound adds -inf (+inf) to its finite crossing.
__host__ __device__ __forceinline__ void span_bounds(const SpanPrep& s, float rv, float& lo, float& hi) {
  const float c0 = fmaf(rv - s.xv[0], s.g[0], s.xu[0]);
  const float c1 = fmaf(rv - s.xv[1], s.g[1], s.xu[1]);
  const float c2 = fmaf(rv - s.xv[2], s.g[2], s.xu[2]);
  lo = fmaxf(fmaxf(c0 + s.lo_add[0], c1 + s.lo_add[1]), c2 + s.lo_add[2]);
  hi = fminf(fminf(c0 + s.hi_add[0], c1 + s.hi_add[1]), c2 + s.hi_add[2]);
}

// Tile columns [x0, x0 + width) of the entry, clipped to the pixels whose
// centre lies in [lo, hi]: cu0 is the centre of tile column 0, inv_h the
// float32 reciprocal of the pixel width and slack (pixels) covers the
// float32 rounding of the centres and of this conversion.  Returns the first
// column and the count (0: none).
__host__ __device__ __forceinline__ int span_columns(float lo, float hi, float cu0, float inv_h, float slack,
                                                     int x0, int width, int& first) {
  float tl = (lo - cu0) * inv_h - slack;
  float th = (hi - cu0) * inv_h + slack;
  tl = fminf(fmaxf(tl, -2.0f), 1024.0f);
  th = fminf(fmaxf(th, -2.0f), 1024.0f);
  const int a = max((int)ceilf(tl), x0);
  const int b = min((int)floorf(th), x0 + width - 1);
  first = a;
  return b >= a ? b - a + 1 : 0;
}

// The tile columns [first, first + count) in [x0, x0 + width) whose centres
// lie inside [lo, hi] for certain: the conversion of span_columns rounded
// inward instead of outward.
__host__ __device__ __forceinline__ int inner_columns(float lo, float hi, float cu0, float inv_h, float slack,
                                                      int x0, int width, int& first) {
  float tl = (lo - cu0) * inv_h + slack;
  float th = (hi - cu0) * inv_h - slack;
  tl = fminf(fmaxf(tl, -2.0f), 1024.0f);
  th = fminf(fmaxf(th, -2.0f), 1024.0f);
  const int a = max((int)ceilf(tl), x0);
  const int b = min((int)floorf(th), x0 + width - 1);
  first = a;
  return b >= a ? b - a + 1 : 0;
}

}  // namespace ldni
