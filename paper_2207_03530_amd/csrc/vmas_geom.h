// Device geometry of the batched 2D physics step (VMAS, Sec. 3 "Core"):
// closest features between spheres, boxes and line segments (the x_ij of
// Eq. 2), the penalty magnitude of Eq. 2 and the pair force and torque arms
// of Eq. 3.
//
// Everything is templated on the scalar type S:
//   float -- the forward step;
//   D3    -- a forward-mode dual number carrying the derivatives with
//            respect to the (x, y, theta) of one entity, used by the adjoint.
// The value part of every D3 operation is the same FP32 operation as the
// float path (fused multiply-adds included), so both instantiations take the
// same branches and the same contact decisions.
#pragma once

#include <hip/hip_runtime.h>

#include "vmas_internal.h"

namespace vmas {

// ------------------------------------------------------------- test masks --

// Contact and broad-phase tests collect their results into per-lane bit masks:
// m * 2 + [hit] in one add with carry, the lane mask of the test as the
// carry in (the compiler otherwise builds each bit with a select and an or)
__device__ __forceinline__ uint32_t shift_in(uint32_t m, bool hit) {
  uint32_t r;
  uint64_t carry_out;
  asm("v_addc_co_u32_e64 %0, %1, %2, %2, %3"
      : "=v"(r), "=s"(carry_out)
      : "v"(m), "s"(__builtin_amdgcn_ballot_w64(hit)));
  return r;
}
// The n tests shifted in by shift_in (n in 0..32) as a mask with bit u set
// for the u-th test.
__device__ __forceinline__ uint32_t shifted_bits(uint32_t m, int n) {
  return n > 0 ? __builtin_bitreverse32(m << (32 - n)) : 0u;
}

// ------------------------------------------------------------ dual numbers --

struct D3 {
  float v, a, b, c;  // value and d/dx, d/dy, d/dtheta of the seeded entity
  __device__ __forceinline__ D3() {}
  __device__ __forceinline__ D3(float x) : v(x), a(0.0f), b(0.0f), c(0.0f) {}
  __device__ __forceinline__ D3(float x, float da, float db, float dc) : v(x), a(da), b(db), c(dc) {}
};
__device__ __forceinline__ D3 operator+(D3 p, D3 q) { return D3(p.v + q.v, p.a + q.a, p.b + q.b, p.c + q.c); }
__device__ __forceinline__ D3 operator-(D3 p, D3 q) { return D3(p.v - q.v, p.a - q.a, p.b - q.b, p.c - q.c); }
__device__ __forceinline__ D3 operator-(D3 p) { return D3(-p.v, -p.a, -p.b, -p.c); }
__device__ __forceinline__ D3 operator*(D3 p, D3 q) {
  return D3(p.v * q.v, p.a * q.v + p.v * q.a, p.b * q.v + p.v * q.b, p.c * q.v + p.v * q.c);
}
__device__ __forceinline__ D3 operator/(D3 p, D3 q) {
  const float r = 1.0f / q.v, v = p.v / q.v;
  return D3(v, (p.a - v * q.a) * r, (p.b - v * q.b) * r, (p.c - v * q.c) * r);
}

__device__ __forceinline__ float val(float x) { return x; }
__device__ __forceinline__ float val(D3 x) { return x.v; }

__device__ __forceinline__ float s_fma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ D3 s_fma(D3 p, D3 q, D3 r) {
  return D3(fmaf(p.v, q.v, r.v), p.a * q.v + p.v * q.a + r.a, p.b * q.v + p.v * q.b + r.b,
            p.c * q.v + p.v * q.c + r.c);
}
__device__ __forceinline__ float s_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ D3 s_sqrt(D3 p) {
  const float s = sqrtf(p.v), k = s > 0.0f ? 0.5f / s : 0.0f;
  return D3(s, p.a * k, p.b * k, p.c * k);
}
__device__ __forceinline__ float s_rsqrt(float x) { return __frsqrt_rn(x); }
__device__ __forceinline__ D3 s_rsqrt(D3 p) {
  const float r = __frsqrt_rn(p.v), k = -0.5f * r * r * r;
  return D3(r, p.a * k, p.b * k, p.c * k);
}
__device__ __forceinline__ float s_exp(float x) { return __expf(x); }
__device__ __forceinline__ D3 s_exp(D3 p) {
  const float e = __expf(p.v);
  return D3(e, p.a * e, p.b * e, p.c * e);
}
__device__ __forceinline__ float s_log(float x) { return __logf(x); }
__device__ __forceinline__ D3 s_log(D3 p) {
  const float l = __logf(p.v), k = 1.0f / p.v;
  return D3(l, p.a * k, p.b * k, p.c * k);
}
template <class S> __device__ __forceinline__ S s_abs(S x) { return val(x) < 0.0f ? -x : x; }
__device__ __forceinline__ float s_abs(float x) { return fabsf(x); }
template <class S> __device__ __forceinline__ S s_min(S x, S y) { return val(y) < val(x) ? y : x; }
template <class S> __device__ __forceinline__ S s_max(S x, S y) { return val(y) > val(x) ? y : x; }
__device__ __forceinline__ float s_min(float x, float y) { return fminf(x, y); }
__device__ __forceinline__ float s_max(float x, float y) { return fmaxf(x, y); }

// ---------------------------------------------------------------- vectors --

template <class S> struct V2T {
  S x, y;
};
template <class S> __device__ __forceinline__ V2T<S> vadd(V2T<S> a, V2T<S> b) { return {a.x + b.x, a.y + b.y}; }
template <class S> __device__ __forceinline__ V2T<S> vsub(V2T<S> a, V2T<S> b) { return {a.x - b.x, a.y - b.y}; }
template <class S> __device__ __forceinline__ V2T<S> vscl(V2T<S> a, S s) { return {a.x * s, a.y * s}; }
template <class S> __device__ __forceinline__ V2T<S> vneg(V2T<S> a) { return {-a.x, -a.y}; }
template <class S> __device__ __forceinline__ S vdot(V2T<S> a, V2T<S> b) { return s_fma(a.x, b.x, a.y * b.y); }
template <class S> __device__ __forceinline__ S vcross(V2T<S> a, V2T<S> b) {
  return s_fma(a.x, b.y, -(a.y * b.x));
}
// R(theta) v and R(theta)^T v with (cs, sn) = (cos, sin) theta.
template <class S> __device__ __forceinline__ V2T<S> vrot(S cs, S sn, V2T<S> v) {
  return {s_fma(cs, v.x, -(sn * v.y)), s_fma(sn, v.x, cs * v.y)};
}
template <class S> __device__ __forceinline__ V2T<S> vrot_t(S cs, S sn, V2T<S> v) {
  return {s_fma(cs, v.x, sn * v.y), s_fma(-sn, v.x, cs * v.y)};
}

// Value selects (component by component): a conditional between two
// aggregates would otherwise choose an address and keep both in scratch.
__device__ __forceinline__ float ssel(bool c, float a, float b) { return c ? a : b; }
__device__ __forceinline__ D3 ssel(bool c, D3 a, D3 b) {
  return D3(c ? a.v : b.v, c ? a.a : b.a, c ? a.b : b.b, c ? a.c : b.c);
}
template <class S> __device__ __forceinline__ V2T<S> vsel(bool c, V2T<S> a, V2T<S> b) {
  return {ssel(c, a.x, b.x), ssel(c, a.y, b.y)};
}

// Geometry of one entity for the narrow phase: pose and (constant) size.
template <class S> struct GeoT {
  V2T<S> c;
  S cs, sn;
  float d0, d1;
  int shape;
};

// Closest features of an ordered pair (lo, hi): signed distance between the
// cores, unit normal along which lo is pushed, contact points on lo and hi.
template <class S> struct HitT {
  S d;
  V2T<S> n, plo, phi;
};

template <class S> __device__ __forceinline__ void line_ends(const GeoT<S>& g, V2T<S>* a, V2T<S>* b) {
  const S h = S(0.5f * g.d0);
  const V2T<S> u = {g.cs * h, g.sn * h};
  *a = vsub(g.c, u);
  *b = vadd(g.c, u);
}

// Sphere centre c against a solid box: lo = sphere, hi = box. Inside, the
// nearest face (x on a tie) gives a negative distance.
template <class S> __device__ HitT<S> sphere_box(V2T<S> c, const GeoT<S>& bx) {
  const S hx = S(0.5f * bx.d0), hy = S(0.5f * bx.d1);
  const V2T<S> u = vrot_t(bx.cs, bx.sn, vsub(c, bx.c));
  V2T<S> nl, ql;
  HitT<S> h;
  const S ax = s_abs(u.x), ay = s_abs(u.y);
  if (val(ax) <= val(hx) && val(ay) <= val(hy)) {
    const S dx = hx - ax, dy = hy - ay;
    if (val(dx) <= val(dy)) {
      const float s = val(u.x) >= 0.0f ? 1.0f : -1.0f;
      h.d = -dx;
      nl = {S(s), S(0.0f)};
      ql = {S(s) * hx, u.y};
    } else {
      const float s = val(u.y) >= 0.0f ? 1.0f : -1.0f;
      h.d = -dy;
      nl = {S(0.0f), S(s)};
      ql = {u.x, S(s) * hy};
    }
  } else {
    ql = {s_min(s_max(u.x, -hx), hx), s_min(s_max(u.y, -hy), hy)};
    const V2T<S> w = vsub(u, ql);
    h.d = s_sqrt(vdot(w, w));
    nl = vscl(w, S(1.0f) / h.d);
  }
  h.n = vrot(bx.cs, bx.sn, nl);
  h.phi = vadd(bx.c, vrot(bx.cs, bx.sn, ql));
  h.plo = c;
  return h;
}

__device__ __forceinline__ int fsign(float x) { return (x > 0.0f) - (x < 0.0f); }

// Running minimum over vertex-versus-edge candidates (first strict minimum
// of the squared distance wins). A candidate is worked out in the frame of
// the edge p0 + s u, 0 <= s <= len (u unit): when the foot is interior the
// separation direction is the edge normal itself, so the normal stays exact
// to rounding of (cos, sin) however close the vertex is; only a foot at an
// end of the edge uses the (vertex - end) vector.
template <class S> struct ClosestT {
  float d2v;     // value of the running minimum of the squared distance
  S d2, d;
  V2T<S> e, q, dir;  // vertex, foot, unit direction from the foot to the vertex
  bool exact;        // dir already known (interior foot)
  bool of_lo;        // the vertex belongs to lo
};

template <class S>
__device__ __forceinline__ void consider(ClosestT<S>& b, V2T<S> e, V2T<S> p0, V2T<S> u, float len,
                                         bool of_lo) {
  const V2T<S> r = vsub(e, p0);
  const S st = vdot(r, u);
  const bool inner = val(st) > 0.0f && val(st) < len;
  // interior foot: offset along the left normal (-u.y, u.x)
  const S sn = vcross(u, r);
  const V2T<S> qi = {s_fma(u.x, st, p0.x), s_fma(u.y, st, p0.y)};
  // foot at an end of the edge
  const V2T<S> p1 = {s_fma(u.x, S(len), p0.x), s_fma(u.y, S(len), p0.y)};
  const V2T<S> qe = vsel(val(st) <= 0.0f, p0, p1);
  const V2T<S> we = vsub(e, qe);
  const S d2 = ssel(inner, sn * sn, vdot(we, we));
  // one update of every field (values, no field chosen by address), so the
  // running minimum stays in registers
  if (val(d2) < b.d2v) {
    b.d2v = val(d2);
    b.d2 = d2;
    b.d = ssel(inner, s_abs(sn), S(-1.0f));
    b.e = e;
    b.q = vsel(inner, qi, qe);
    b.dir = vsel(val(sn) >= 0.0f, V2T<S>{-u.y, u.x}, V2T<S>{u.y, -u.x});
    b.exact = inner;
    b.of_lo = of_lo;
  }
}

// fb_lo / fb_hi: the normal of lo used at zero distance when the vertex
// belongs to lo / to hi.
template <class S>
__device__ __forceinline__ HitT<S> finish_closest(const ClosestT<S>& b, V2T<S> fb_lo, V2T<S> fb_hi) {
  HitT<S> h;
  V2T<S> dir;
  if (b.exact) {
    h.d = b.d;
    dir = b.dir;
  } else {
    h.d = s_sqrt(b.d2);
    if (val(h.d) == 0.0f)
      dir = vsel(b.of_lo, fb_lo, vneg(fb_hi));
    else
      dir = vscl(vsub(b.e, b.q), S(1.0f) / h.d);
  }
  // vertex of lo, foot on hi: lo pushed from the foot to the vertex;
  // vertex of hi, foot on lo: lo pushed the other way
  h.n = vsel(b.of_lo, dir, vneg(dir));
  h.plo = vsel(b.of_lo, b.e, b.q);
  h.phi = vsel(b.of_lo, b.q, b.e);
  return h;
}

// Sphere centre c against a line segment: lo = sphere, hi = line.
template <class S> __device__ HitT<S> sphere_line(V2T<S> c, const GeoT<S>& l) {
  V2T<S> a, bb;
  line_ends(l, &a, &bb);
  ClosestT<S> b;
  b.d2v = INFINITY;
  consider(b, c, a, V2T<S>{l.cs, l.sn}, l.d0, true);
  return finish_closest(b, V2T<S>{-l.sn, l.cs}, V2T<S>{-l.sn, l.cs});
}

// Two segments: orientation-sign crossing test (collinear overlap counts as
// crossing); apart -> exact segment distance; crossing -> separating-axis
// depth of the endpoint nearest to the other supporting line.
// cutoff as for poly_poly: apart segments one of which lies wholly on one
// side of the other's line, farther than cutoff, are returned at +infinity.
template <class S>
__device__ HitT<S> line_line(const GeoT<S>& I, const GeoT<S>& J, float cutoff = INFINITY) {
  V2T<S> ai, bi, aj, bj;
  line_ends(I, &ai, &bi);
  line_ends(J, &aj, &bj);
  const V2T<S> ni = {-I.sn, I.cs}, nj = {-J.sn, J.cs};
  const V2T<S> ui = vsub(bi, ai), uj = vsub(bj, aj);
  // offsets of each segment's ends from the other's line, times its length
  const float c1 = val(vcross(ui, vsub(aj, ai))), c2 = val(vcross(ui, vsub(bj, ai)));
  const float c3 = val(vcross(uj, vsub(ai, aj))), c4 = val(vcross(uj, vsub(bi, aj)));
  const int o1 = fsign(c1), o2 = fsign(c2), o3 = fsign(c3), o4 = fsign(c4);
  bool crossing;
  if ((o1 | o2 | o3 | o4) == 0) {
    const float tu = val(vdot(ui, ui));
    const float ta = val(vdot(vsub(aj, ai), ui)), tb = val(vdot(vsub(bj, ai), ui));
    crossing = !(fmaxf(ta, tb) < 0.0f || fminf(ta, tb) > tu);
  } else {
    crossing = (o1 * o2 <= 0) && (o3 * o4 <= 0);
  }
  if (!crossing) {
    // The distance is at least the smaller offset of a segment lying on one
    // side of the other's line (the offsets carry the length |u| ~ d0; the
    // factor 1.001 covers the difference).
    if (cutoff >= 0.0f &&
        ((o1 == o2 && o1 != 0 && fminf(fabsf(c1), fabsf(c2)) > cutoff * I.d0 * 1.001f) ||
         (o3 == o4 && o3 != 0 && fminf(fabsf(c3), fabsf(c4)) > cutoff * J.d0 * 1.001f))) {
      HitT<S> far;
      far.d = S(INFINITY);
      far.n = far.plo = far.phi = V2T<S>{S(0.0f), S(0.0f)};
      return far;
    }
    ClosestT<S> b;
    b.d2v = INFINITY;
    const V2T<S> ti = {I.cs, I.sn}, tj = {J.cs, J.sn};
    consider(b, ai, aj, tj, J.d0, true);
    consider(b, bi, aj, tj, J.d0, true);
    consider(b, aj, ai, ti, I.d0, false);
    consider(b, bj, ai, ti, I.d0, false);
    return finish_closest(b, nj, vneg(ni));
  }
  // Endpoints in order ai, bi (against line J), aj, bj (against line I).
  HitT<S> h;
  float best = INFINITY;
  S bestS = S(0.0f);
  const V2T<S> ends[4] = {ai, bi, aj, bj};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const bool of_lo = k < 2;
    const V2T<S> base = of_lo ? aj : ai;
    const V2T<S> nrm = of_lo ? nj : ni;
    const S s = vdot(vsub(ends[k], base), nrm);
    const S dist = s_abs(s);
    if (val(dist) < best) {
      best = val(dist);
      bestS = dist;
      const V2T<S> push = val(s) > 0.0f ? vneg(nrm) : nrm;
      h.n = of_lo ? push : vneg(push);
      h.plo = ends[k];
      h.phi = ends[k];
    }
  }
  h.d = -bestS;
  return h;
}

// Convex polygon view of a box (NV = 4: 4 CCW vertices, 4 edges, 2 axes) or
// a line (NV = 2: 2 vertices, 1 edge, 1 axis); the counts are compile-time
// constants, so every loop below runs exactly over the real features.
template <class S> struct PolyT {
  V2T<S> v[4];
  V2T<S> ax[2];
  V2T<S> eu[4];  // unit direction of edge k (from v[k] to v[k+1])
  float el[4];   // its length
};
template <int NV> struct PolyN {
  static constexpr int nv = NV, ne = NV == 4 ? 4 : 1, na = NV == 4 ? 2 : 1;
};

template <int NV, class S> __device__ __forceinline__ void make_poly(const GeoT<S>& g, PolyT<S>& p) {
  if constexpr (NV == 4) {
    const S hx = S(0.5f * g.d0), hy = S(0.5f * g.d1);
    p.v[0] = vadd(g.c, vrot(g.cs, g.sn, V2T<S>{hx, hy}));
    p.v[1] = vadd(g.c, vrot(g.cs, g.sn, V2T<S>{-hx, hy}));
    p.v[2] = vadd(g.c, vrot(g.cs, g.sn, V2T<S>{-hx, -hy}));
    p.v[3] = vadd(g.c, vrot(g.cs, g.sn, V2T<S>{hx, -hy}));
    p.ax[0] = {g.cs, g.sn};
    p.ax[1] = {-g.sn, g.cs};
    p.eu[0] = {-g.cs, -g.sn};
    p.eu[1] = {g.sn, -g.cs};
    p.eu[2] = {g.cs, g.sn};
    p.eu[3] = {-g.sn, g.cs};
    p.el[0] = g.d0;
    p.el[1] = g.d1;
    p.el[2] = g.d0;
    p.el[3] = g.d1;
  } else {
    line_ends(g, &p.v[0], &p.v[1]);
    p.ax[0] = {-g.sn, g.cs};
    p.eu[0] = {g.cs, g.sn};
    p.el[0] = g.d0;
  }
}

template <int NV, class S>
__device__ __forceinline__ void project(const PolyT<S>& p, V2T<S> s, float* mn, float* mx) {
  float a = val(vdot(p.v[0], s)), b = a;
#pragma unroll
  for (int q = 1; q < NV; ++q) {
    const float t = val(vdot(p.v[q], s));
    a = fminf(a, t);
    b = fmaxf(b, t);
  }
  *mn = a;
  *mx = b;
}

// Projection extremes as S (only the winning axis needs derivatives).
template <int NV, class S> __device__ __forceinline__ S proj_min(const PolyT<S>& p, V2T<S> s) {
  S a = vdot(p.v[0], s);
#pragma unroll
  for (int q = 1; q < NV; ++q) a = s_min(a, vdot(p.v[q], s));
  return a;
}
template <int NV, class S> __device__ __forceinline__ S proj_max(const PolyT<S>& p, V2T<S> s) {
  S a = vdot(p.v[0], s);
#pragma unroll
  for (int q = 1; q < NV; ++q) a = s_max(a, vdot(p.v[q], s));
  return a;
}

// Axis k of the pair: lo's axes first, then hi's.
template <int NA, int NB, class S>
__device__ __forceinline__ V2T<S> pair_axis(const PolyT<S>& A, const PolyT<S>& B, int k) {
  constexpr int na = PolyN<NA>::na;
  return k < na ? A.ax[k] : B.ax[k - na];
}

// Line/box and box/box by the separating-axis test: apart -> exact distance
// between the convex sets (vertex against edge, lo's vertices first);
// overlapping -> smallest overlap over the axes (lo's first), contact point
// at the deepest vertex of the shape that does not own the winning axis.
// cutoff: when some axis separates the shapes by more than cutoff, the
// distance (which is at least that separation) is not worked out and d is
// returned as +infinity; callers that only test d <= d_min pass d_min plus
// a margin above the FP32 error of the separation and of the distance.
template <int NA, int NB, class S>
__device__ HitT<S> poly_poly(const GeoT<S>& I, const GeoT<S>& J, float cutoff) {
  using PA = PolyN<NA>;
  using PB = PolyN<NB>;
  constexpr int NAX = PA::na + PB::na;
  PolyT<S> A, B;
  make_poly<NA>(I, A);
  make_poly<NB>(J, B);
  bool separated = false;
  float best = INFINITY, gap = -INFINITY;
  int best_k = 0;
  bool best_plus = true;
#pragma unroll
  for (int k = 0; k < NAX; ++k) {
    const V2T<S> s = pair_axis<NA, NB>(A, B, k);
    float mina, maxa, minb, maxb;
    project<NA>(A, s, &mina, &maxa);
    project<NB>(B, s, &minb, &maxb);
    if (maxa < minb || maxb < mina) separated = true;
    gap = fmaxf(gap, fmaxf(minb - maxa, mina - maxb));
    const float op = maxb - mina, om = maxa - minb;
    const float ov = op <= om ? op : om;
    if (ov < best) {
      best = ov;
      best_k = k;
      best_plus = op <= om;
    }
  }
  if (separated) {
    if (gap > cutoff) {
      HitT<S> far;
      far.d = S(INFINITY);
      far.n = far.plo = far.phi = V2T<S>{S(0.0f), S(0.0f)};
      return far;
    }
    ClosestT<S> b;
    b.d2v = INFINITY;
#pragma unroll
    for (int q = 0; q < PA::nv; ++q) {
#pragma unroll
      for (int e = 0; e < PB::ne; ++e) consider(b, A.v[q], B.v[e], B.eu[e], B.el[e], true);
    }
#pragma unroll
    for (int q = 0; q < PB::nv; ++q) {
#pragma unroll
      for (int e = 0; e < PA::ne; ++e) consider(b, B.v[q], A.v[e], A.eu[e], A.el[e], false);
    }
    const V2T<S> fb = {S(1.0f), S(0.0f)};
    return finish_closest(b, fb, fb);
  }
  HitT<S> h;
  V2T<S> s = A.ax[0];
#pragma unroll
  for (int k = 1; k < NAX; ++k) {
    s = vsel(k == best_k, pair_axis<NA, NB>(A, B, k), s);
  }
  // overlap along the winning axis with derivatives
  h.d = best_plus ? -(proj_max<NB>(B, s) - proj_min<NA>(A, s))
                  : -(proj_max<NA>(A, s) - proj_min<NB>(B, s));
  h.n = vsel(best_plus, s, vneg(s));
  // axis of hi: deepest vertex of lo; axis of lo: deepest vertex of hi
  V2T<S> pa = A.v[0], pb = B.v[0];
  float ma = val(vdot(h.n, pa)), mb = val(vdot(h.n, pb));
#pragma unroll
  for (int q = 1; q < PA::nv; ++q) {
    const float t = val(vdot(h.n, A.v[q]));
    const bool lt = t < ma;
    ma = lt ? t : ma;
    pa = vsel(lt, A.v[q], pa);
  }
#pragma unroll
  for (int q = 1; q < PB::nv; ++q) {
    const float t = val(vdot(h.n, B.v[q]));
    const bool gt = t > mb;
    mb = gt ? t : mb;
    pb = vsel(gt, B.v[q], pb);
  }
  const V2T<S> p = vsel(best_k >= PA::na, pa, pb);
  h.plo = p;
  h.phi = p;
  return h;
}

// Narrow phase of a pair that is not sphere-sphere, canonical (lo, hi) order.
template <class S>
__device__ HitT<S> narrow(const GeoT<S>& lo, const GeoT<S>& hi, float cutoff = INFINITY) {
  if (lo.shape == SPHERE) return hi.shape == LINE ? sphere_line(lo.c, hi) : sphere_box(lo.c, hi);
  if (hi.shape == SPHERE) {
    const HitT<S> r = lo.shape == LINE ? sphere_line(hi.c, lo) : sphere_box(hi.c, lo);
    HitT<S> o;
    o.d = r.d;
    o.n = vneg(r.n);
    o.plo = r.phi;
    o.phi = r.plo;
    return o;
  }
  if (lo.shape == LINE && hi.shape == LINE) return line_line(lo, hi, cutoff);
  if (lo.shape == BOX && hi.shape == BOX) return poly_poly<4, 4>(lo, hi, cutoff);
  if (lo.shape == BOX) return poly_poly<4, 2>(lo, hi, cutoff);
  return poly_poly<2, 4>(lo, hi, cutoff);
}

// Cutoff for narrow() in a contact test against d_min: a separation beyond
// d_min by more than 1e-4 + 1e-5 (|coordinates| + sizes) cannot end in
// d <= d_min, the FP32 errors of the separation and of the exact distance
// being a few ulps of the coordinates.
__device__ __forceinline__ float contact_cutoff(const GeoT<float>& lo, const GeoT<float>& hi,
                                                float dmin) {
  const float scale = (fabsf(lo.c.x) + fabsf(lo.c.y) + lo.d0 + lo.d1) +
                      (fabsf(hi.c.x) + fabsf(hi.c.y) + hi.d0 + hi.d1);
  return dmin + (1e-4f + 1e-5f * scale);
}

// Magnitude of Eq. (2): c k log(1 + e^z), z = (d_min - d)/k, in the stable
// form max(z, 0) + log(1 + e^{-|z|}); the second term lies in (0, ln 2] and
// is evaluated with the hardware exp2/log2 (about 1 ulp each), an absolute
// error of a few 1e-8 against max(z, 0) >= 0.
// log(1 + e^-a) for a >= 0. The logarithm's argument lies in (1, 2], where
// the hardware base-2 logarithm needs no range or denormal handling.
__device__ __forceinline__ float softplus_tail(float a) {
  return __builtin_amdgcn_logf(1.0f + __expf(-a)) * 0.69314718f;
}
__device__ __forceinline__ D3 softplus_tail(D3 p) {
  const float e = __expf(-p.v);
  const float v = __builtin_amdgcn_logf(1.0f + e) * 0.69314718f;
  const float dv = -e / (1.0f + e);
  return D3(v, dv * p.a, dv * p.b, dv * p.c);
}

template <class S> __device__ __forceinline__ S contact_mag(S dmin, S d, const WorldK& w) {
  const S z = (dmin - d) * S(w.inv_k);
  return S(w.ck) * (s_max(z, S(0.0f)) + softplus_tail(s_abs(z)));
}

// Distance and unit normal along (dx, dy) from the squared length sq, with
// one reciprocal square root; coincident centres push the lower index +x.
template <class S>
__device__ __forceinline__ void sphere_normal(S dx, S dy, S sq, bool self_lo, S* d, V2T<S>* n) {
  if (val(sq) == 0.0f) {
    *d = S(0.0f);
    *n = self_lo ? V2T<S>{S(1.0f), S(0.0f)} : V2T<S>{S(-1.0f), S(0.0f)};
  } else {
    const S rs = s_rsqrt(sq);
    *d = sq * rs;
    *n = {dx * rs, dy * rs};
  }
}

// Contact predicate of Eq. (2) between two spheres, decided in FP32 on the
// squared lengths: fl(dx*dx + fl(dy*dy)) <= fl(d_min * d_min), one fused
// multiply-add.
__device__ __forceinline__ bool sphere_contact(float dx, float dy, float dmin, float* sq) {
  *sq = fmaf(dx, dx, __fmul_rn(dy, dy));
  return *sq <= __fmul_rn(dmin, dmin);
}

// Contact of the lane's entity (self, environment-local index a) with the
// partner in LDS slot q (local index b). Accumulates the lane's force and
// torque and reports the contact bit.
// OTHER >= 0 fixes the partner's shape at compile time (the caller knows it),
// which leaves only that shape's narrow-phase routines in the code.
template <bool SPH, int OTHER = -1>
__device__ __forceinline__ bool pair_force(const GeoT<float>& self, float rho_s, int a, const float4 P,
                                           const float4 S, int b, const WorldK& w, float& fx,
                                           float& fy, float& tq) {
  const float rho_o = S.z;
  const float dmin = (rho_s + rho_o) + w.min_dist;
  const int so = SPH ? SPHERE : (OTHER >= 0 ? OTHER : (__float_as_int(S.w) & 0xff));
  if (SPH || (self.shape == SPHERE && so == SPHERE)) {
    // Both spheres: x_ij joins the centres; decision on squared lengths.
    const float dx = self.c.x - P.x, dy = self.c.y - P.y;
    const float s = fmaf(dx, dx, __fmul_rn(dy, dy));
    if (!(s <= __fmul_rn(dmin, dmin))) return false;
    V2T<float> n;
    float d;
    sphere_normal(dx, dy, s, a < b, &d, &n);
    const float F = contact_mag(dmin, d, w);
    fx = fmaf(F, n.x, fx);
    fy = fmaf(F, n.y, fy);
    return true;
  }
  GeoT<float> o;
  o.c = V2T<float>{P.x, P.y};
  o.cs = P.z;
  o.sn = P.w;
  o.d0 = S.x;
  o.d1 = S.y;
  o.shape = so;
  const bool self_lo = a < b;
  // the pair in canonical order, chosen by value (one narrow-phase call)
  GeoT<float> lo, hi;
  lo.c.x = self_lo ? self.c.x : o.c.x;
  lo.c.y = self_lo ? self.c.y : o.c.y;
  lo.cs = self_lo ? self.cs : o.cs;
  lo.sn = self_lo ? self.sn : o.sn;
  lo.d0 = self_lo ? self.d0 : o.d0;
  lo.d1 = self_lo ? self.d1 : o.d1;
  lo.shape = self_lo ? self.shape : o.shape;
  hi.c.x = self_lo ? o.c.x : self.c.x;
  hi.c.y = self_lo ? o.c.y : self.c.y;
  hi.cs = self_lo ? o.cs : self.cs;
  hi.sn = self_lo ? o.sn : self.sn;
  hi.d0 = self_lo ? o.d0 : self.d0;
  hi.d1 = self_lo ? o.d1 : self.d1;
  hi.shape = self_lo ? o.shape : self.shape;
  const HitT<float> h = narrow(lo, hi, contact_cutoff(lo, hi, dmin));
  if (!(h.d <= dmin)) return false;
  const float F = contact_mag(dmin, h.d, w);
  const float sg = self_lo ? F : -F;
  const V2T<float> f = V2T<float>{sg * h.n.x, sg * h.n.y};
  const V2T<float> arm = vsub(self_lo ? h.plo : h.phi, self.c);
  fx += f.x;
  fy += f.y;
  tq += vcross(arm, f);
  return true;
}

// Whether a joint switches off the contact with local index b: excl holds up
// to 4 local indices below 255, one per byte, 0xff marking an unused byte (so
// local index 255 and above is never excluded).
__device__ __forceinline__ bool excluded(int excl, int b) {
  const unsigned u = (unsigned)excl;
  return ((unsigned)b < 255u) &
         (((u & 0xffu) == (unsigned)b) | (((u >> 8) & 0xffu) == (unsigned)b) |
          (((u >> 16) & 0xffu) == (unsigned)b) | ((u >> 24) == (unsigned)b));
}


// Joint between entities a and b (Eq. 1 force of a linear spring between the
// world anchor points P_a = x_a + R_a anchor_a and P_b): f_a = -k (l - rest)
// (P_a - P_b) / l, f_b = -f_a, torques from the anchor arms. Seen from the
// lane's entity ("self", which is a when is_a): its force, its torque and the
// other entity's torque. Returns false when the anchors coincide (no force).
template <class S>
__device__ __forceinline__ bool joint_eval(V2T<S> xs, S cs, S sn, V2T<S> xo, S co, S so, bool is_a,
                                           const JointK& J, float k, V2T<S>* f_self, S* tq_self,
                                           S* tq_other) {
  const V2T<S> xa = vsel(is_a, xs, xo), xb = vsel(is_a, xo, xs);
  const S ca = ssel(is_a, cs, co), sa = ssel(is_a, sn, so);
  const S cb = ssel(is_a, co, cs), sb = ssel(is_a, so, sn);
  const V2T<S> Pa = vadd(xa, vrot(ca, sa, V2T<S>{S(J.ax), S(J.ay)}));
  const V2T<S> Pb = vadd(xb, vrot(cb, sb, V2T<S>{S(J.bx), S(J.by)}));
  const V2T<S> dl = vsub(Pa, Pb);
  const S len = s_sqrt(vdot(dl, dl));
  if (val(len) == 0.0f) return false;
  const S mag = S(-k) * (len - S(J.rest)) / len;
  const V2T<S> fa = vscl(dl, mag);
  const V2T<S> fs = vsel(is_a, fa, vneg(fa));
  const V2T<S> arm_s = vsel(is_a, vsub(Pa, xa), vsub(Pb, xb));
  const V2T<S> arm_o = vsel(is_a, vsub(Pb, xb), vsub(Pa, xa));
  *f_self = fs;
  *tq_self = vcross(arm_s, fs);
  *tq_other = vcross(arm_o, vneg(fs));
  return true;
}

// Derivative form of one contact for the adjoint: the pair (self, other) is
// known to be in contact (decided by pair_force's FP32 rule); self carries
// the dual seeds. Outputs the force on self and both torques, with their
// derivatives with respect to self's (x, y, theta).
// SPH: both entities are spheres (sphere-only batches).
template <bool SPH = false>
__device__ __forceinline__ void pair_grad(const GeoT<D3>& self, float rho_s, bool self_lo,
                                          const GeoT<D3>& other, float rho_o, const WorldK& w,
                                          V2T<D3>* f_self, D3* tq_self, D3* tq_other) {
  const float dmin = (rho_s + rho_o) + w.min_dist;
  if (SPH || (self.shape == SPHERE && other.shape == SPHERE)) {
    const D3 dx = self.c.x - other.c.x, dy = self.c.y - other.c.y;
    const D3 sq = s_fma(dx, dx, dy * dy);
    V2T<D3> n;
    D3 d;
    sphere_normal(dx, dy, sq, self_lo, &d, &n);
    const D3 F = contact_mag(D3(dmin), d, w);
    *f_self = vscl(n, F);
    *tq_self = D3(0.0f);
    *tq_other = D3(0.0f);
    return;
  }
  // the pair in canonical order, chosen by value (one narrow-phase call)
  GeoT<D3> lo, hi;
  lo.c = vsel(self_lo, self.c, other.c);
  lo.cs = ssel(self_lo, self.cs, other.cs);
  lo.sn = ssel(self_lo, self.sn, other.sn);
  lo.d0 = self_lo ? self.d0 : other.d0;
  lo.d1 = self_lo ? self.d1 : other.d1;
  lo.shape = self_lo ? self.shape : other.shape;
  hi.c = vsel(self_lo, other.c, self.c);
  hi.cs = ssel(self_lo, other.cs, self.cs);
  hi.sn = ssel(self_lo, other.sn, self.sn);
  hi.d0 = self_lo ? other.d0 : self.d0;
  hi.d1 = self_lo ? other.d1 : self.d1;
  hi.shape = self_lo ? other.shape : self.shape;
  const HitT<D3> h = narrow(lo, hi);
  const D3 F = contact_mag(D3(dmin), h.d, w);
  const V2T<D3> flo = vscl(h.n, F);
  const V2T<D3> fs = vsel(self_lo, flo, vneg(flo));
  *f_self = fs;
  *tq_self = vcross(vsub(vsel(self_lo, h.plo, h.phi), self.c), fs);
  *tq_other = vcross(vsub(vsel(self_lo, h.phi, h.plo), other.c), vneg(fs));
}

}  // namespace vmas
