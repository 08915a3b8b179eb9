// HIP kernels (gfx950) of the batched 2D physics step of VMAS:
// Sec. 3 "Core", Eq. (1) forces and semi-implicit Euler, Eq. (2) penalty
// contact between the closest points of two shapes, Eq. (3) torque and the
// angular update.
//
// Mapping. A launch group (one workgroup) holds whole environments. Every
// entity of the group is staged in LDS (pose + static shape data); every
// entity that can move or rotate owns one lane and keeps its state in
// registers for all T steps of a rollout. A lane loops over the other
// entities of its environment (broadcast LDS reads: lanes of one environment
// read the same partner in the same iteration), evaluates each pair in the
// canonical (lower index, higher index) order and keeps its own side of the
// force, so the two lanes of a pair see exactly opposite forces and no
// cross-lane reduction (and no float atomic) is needed: results do not depend
// on how environments are packed into groups. Lanes are sorted by shape
// within a group so that a wavefront mostly runs one narrow-phase routine.
// Poses are double-buffered in LDS: one barrier per step.
//
// Arithmetic is FP32 and compiled without implicit contraction; every fused
// multiply-add is written out, so different kernels and plans agree bit for
// bit.

#include "vmas_internal.h"

namespace vmas {
namespace {

// ---------------------------------------------------------------- vectors --

struct V2 {
  float x, y;
};
__device__ __forceinline__ V2 vv(float x, float y) { return V2{x, y}; }
__device__ __forceinline__ V2 vadd(V2 a, V2 b) { return V2{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ V2 vsub(V2 a, V2 b) { return V2{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ V2 vscl(V2 a, float s) { return V2{a.x * s, a.y * s}; }
__device__ __forceinline__ V2 vneg(V2 a) { return V2{-a.x, -a.y}; }
__device__ __forceinline__ float vdot(V2 a, V2 b) { return fmaf(a.x, b.x, a.y * b.y); }
__device__ __forceinline__ float vcross(V2 a, V2 b) { return fmaf(a.x, b.y, -(a.y * b.x)); }
// R(theta) v and R(theta)^T v with (cs, sn) = (cos, sin) theta.
__device__ __forceinline__ V2 vrot(float cs, float sn, V2 v) {
  return V2{fmaf(cs, v.x, -(sn * v.y)), fmaf(sn, v.x, cs * v.y)};
}
__device__ __forceinline__ V2 vrot_t(float cs, float sn, V2 v) {
  return V2{fmaf(cs, v.x, sn * v.y), fmaf(-sn, v.x, cs * v.y)};
}

// Geometry of one entity for the narrow phase.
struct Geo {
  V2 c;
  float cs, sn;
  float d0, d1;
  int shape;
};

// Closest features of an ordered pair (lo, hi): signed distance between the
// cores, unit normal along which lo is pushed, contact points on lo and hi.
struct Hit {
  float d;
  V2 n, plo, phi;
};

__device__ __forceinline__ void line_ends(const Geo& g, V2* a, V2* b) {
  float h = 0.5f * g.d0;
  V2 u = V2{g.cs * h, g.sn * h};
  *a = vsub(g.c, u);
  *b = vadd(g.c, u);
}

// sphere centre c against a solid box: Hit with lo = sphere, hi = box.
__device__ Hit sphere_box(V2 c, const Geo& bx) {
  const float hx = 0.5f * bx.d0, hy = 0.5f * bx.d1;
  V2 u = vrot_t(bx.cs, bx.sn, vsub(c, bx.c));
  V2 nl, ql;
  Hit h;
  const float ax = fabsf(u.x), ay = fabsf(u.y);
  if (ax <= hx && ay <= hy) {
    const float dx = hx - ax, dy = hy - ay;
    if (dx <= dy) {
      const float s = u.x >= 0.0f ? 1.0f : -1.0f;
      h.d = -dx;
      nl = V2{s, 0.0f};
      ql = V2{s * hx, u.y};
    } else {
      const float s = u.y >= 0.0f ? 1.0f : -1.0f;
      h.d = -dy;
      nl = V2{0.0f, s};
      ql = V2{u.x, s * hy};
    }
  } else {
    ql = V2{fminf(fmaxf(u.x, -hx), hx), fminf(fmaxf(u.y, -hy), hy)};
    V2 w = vsub(u, ql);
    h.d = sqrtf(vdot(w, w));
    nl = vscl(w, 1.0f / h.d);
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
struct Closest {
  float d2, d;
  V2 e, q, dir;  // vertex, foot, unit direction from the foot to the vertex
  bool exact;    // dir already known (interior foot)
  bool of_lo;    // the vertex belongs to lo
};

__device__ __forceinline__ void consider(Closest& b, V2 e, V2 p0, V2 u, float len, bool of_lo) {
  const V2 r = vsub(e, p0);
  const float st = vdot(r, u);
  if (st > 0.0f && st < len) {
    const float sn = vcross(u, r);  // offset along the left normal (-u.y, u.x)
    const float d2 = sn * sn;
    if (d2 < b.d2) {
      b.d2 = d2;
      b.d = fabsf(sn);
      b.e = e;
      b.q = V2{fmaf(u.x, st, p0.x), fmaf(u.y, st, p0.y)};
      b.dir = sn >= 0.0f ? V2{-u.y, u.x} : V2{u.y, -u.x};
      b.exact = true;
      b.of_lo = of_lo;
    }
  } else {
    const V2 q = st <= 0.0f ? p0 : V2{fmaf(u.x, len, p0.x), fmaf(u.y, len, p0.y)};
    const V2 w = vsub(e, q);
    const float d2 = vdot(w, w);
    if (d2 < b.d2) {
      b.d2 = d2;
      b.d = -1.0f;
      b.e = e;
      b.q = q;
      b.exact = false;
      b.of_lo = of_lo;
    }
  }
}

// fb_lo / fb_hi: the normal of lo used at zero distance when the vertex
// belongs to lo / to hi.
__device__ __forceinline__ Hit finish_closest(const Closest& b, V2 fb_lo, V2 fb_hi) {
  Hit h;
  V2 dir;
  if (b.exact) {
    h.d = b.d;
    dir = b.dir;
  } else {
    h.d = sqrtf(b.d2);
    dir = h.d == 0.0f ? (b.of_lo ? fb_lo : vneg(fb_hi)) : vscl(vsub(b.e, b.q), 1.0f / h.d);
  }
  if (b.of_lo) {  // vertex of lo, foot on hi: lo pushed from the foot to the vertex
    h.n = dir;
    h.plo = b.e;
    h.phi = b.q;
  } else {        // vertex of hi, foot on lo: lo pushed the other way
    h.n = vneg(dir);
    h.plo = b.q;
    h.phi = b.e;
  }
  return h;
}

// sphere centre c against a line segment: Hit with lo = sphere, hi = line.
__device__ Hit sphere_line(V2 c, const Geo& l) {
  V2 a, bb;
  line_ends(l, &a, &bb);
  Closest b;
  b.d2 = INFINITY;
  consider(b, c, a, V2{l.cs, l.sn}, l.d0, true);
  return finish_closest(b, V2{-l.sn, l.cs}, V2{-l.sn, l.cs});
}

// Two segments: orientation-sign crossing test; apart -> exact distance,
// crossing -> separating-axis depth along a supporting-line normal.
__device__ Hit line_line(const Geo& I, const Geo& J) {
  V2 ai, bi, aj, bj;
  line_ends(I, &ai, &bi);
  line_ends(J, &aj, &bj);
  const V2 ni = V2{-I.sn, I.cs}, nj = V2{-J.sn, J.cs};
  const V2 ui = vsub(bi, ai), uj = vsub(bj, aj);
  const int o1 = fsign(vcross(ui, vsub(aj, ai)));
  const int o2 = fsign(vcross(ui, vsub(bj, ai)));
  const int o3 = fsign(vcross(uj, vsub(ai, aj)));
  const int o4 = fsign(vcross(uj, vsub(bi, aj)));
  bool crossing;
  if ((o1 | o2 | o3 | o4) == 0) {
    const float tu = vdot(ui, ui);
    const float ta = vdot(vsub(aj, ai), ui), tb = vdot(vsub(bj, ai), ui);
    crossing = !(fmaxf(ta, tb) < 0.0f || fminf(ta, tb) > tu);
  } else {
    crossing = (o1 * o2 <= 0) && (o3 * o4 <= 0);
  }
  if (!crossing) {
    Closest b;
    b.d2 = INFINITY;
    const V2 ti = V2{I.cs, I.sn}, tj = V2{J.cs, J.sn};
    consider(b, ai, aj, tj, J.d0, true);
    consider(b, bi, aj, tj, J.d0, true);
    consider(b, aj, ai, ti, I.d0, false);
    consider(b, bj, ai, ti, I.d0, false);
    return finish_closest(b, nj, vneg(ni));
  }
  // Endpoints in order ai, bi (against line J), aj, bj (against line I).
  Hit h;
  float best = INFINITY;
  V2 ends[4] = {ai, bi, aj, bj};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const bool of_lo = k < 2;
    const V2 base = of_lo ? aj : ai;
    const V2 nrm = of_lo ? nj : ni;
    const float s = vdot(vsub(ends[k], base), nrm);
    const float dist = fabsf(s);
    if (dist < best) {
      best = dist;
      const V2 push = s > 0.0f ? vneg(nrm) : nrm;
      h.n = of_lo ? push : vneg(push);
      h.plo = ends[k];
      h.phi = ends[k];
    }
  }
  h.d = -best;
  return h;
}

// Convex polygon view of a box (4 CCW vertices, 4 edges, 2 axes) or a line
// (2 vertices, 1 edge, 1 axis).
struct Poly {
  int nv, ne, na;
  V2 v[4];
  V2 ax[2];
  V2 eu[4];    // unit direction of edge k (from v[k] to v[k+1])
  float el[4]; // its length
};

__device__ __forceinline__ void make_poly(const Geo& g, Poly& p) {
  if (g.shape == BOX) {
    const float hx = 0.5f * g.d0, hy = 0.5f * g.d1;
    p.nv = 4;
    p.ne = 4;
    p.na = 2;
    p.v[0] = vadd(g.c, vrot(g.cs, g.sn, V2{hx, hy}));
    p.v[1] = vadd(g.c, vrot(g.cs, g.sn, V2{-hx, hy}));
    p.v[2] = vadd(g.c, vrot(g.cs, g.sn, V2{-hx, -hy}));
    p.v[3] = vadd(g.c, vrot(g.cs, g.sn, V2{hx, -hy}));
    p.ax[0] = V2{g.cs, g.sn};
    p.ax[1] = V2{-g.sn, g.cs};
    p.eu[0] = V2{-g.cs, -g.sn};
    p.eu[1] = V2{g.sn, -g.cs};
    p.eu[2] = V2{g.cs, g.sn};
    p.eu[3] = V2{-g.sn, g.cs};
    p.el[0] = g.d0;
    p.el[1] = g.d1;
    p.el[2] = g.d0;
    p.el[3] = g.d1;
  } else {
    p.nv = 2;
    p.ne = 1;
    p.na = 1;
    line_ends(g, &p.v[0], &p.v[1]);
    p.v[2] = p.v[1];
    p.v[3] = p.v[0];
    p.ax[0] = V2{-g.sn, g.cs};
    p.ax[1] = p.ax[0];
    p.eu[0] = V2{g.cs, g.sn};
    p.el[0] = g.d0;
    p.eu[1] = p.eu[2] = p.eu[3] = p.eu[0];
    p.el[1] = p.el[2] = p.el[3] = p.el[0];
  }
}

__device__ __forceinline__ void project(const Poly& p, V2 s, float* mn, float* mx) {
  float a = vdot(p.v[0], s), b = a;
#pragma unroll
  for (int q = 1; q < 4; ++q) {
    if (q < p.nv) {
      const float t = vdot(p.v[q], s);
      a = fminf(a, t);
      b = fmaxf(b, t);
    }
  }
  *mn = a;
  *mx = b;
}

// Line/box and box/box by the separating-axis test.
__device__ Hit poly_poly(const Geo& I, const Geo& J) {
  Poly A, B;
  make_poly(I, A);
  make_poly(J, B);
  bool separated = false;
  float best = INFINITY;
  int best_k = 0;
  V2 best_n = V2{1.0f, 0.0f};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k < A.na + B.na) {
      const V2 s = k < A.na ? A.ax[k] : B.ax[k - A.na];
      float mina, maxa, minb, maxb;
      project(A, s, &mina, &maxa);
      project(B, s, &minb, &maxb);
      if (maxa < minb || maxb < mina) separated = true;
      const float op = maxb - mina, om = maxa - minb;
      const float ov = op <= om ? op : om;
      if (ov < best) {
        best = ov;
        best_k = k;
        best_n = op <= om ? s : vneg(s);
      }
    }
  }
  if (separated) {
    Closest b;
    b.d2 = INFINITY;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q < A.nv) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (e < B.ne) consider(b, A.v[q], B.v[e], B.eu[e], B.el[e], true);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q < B.nv) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (e < A.ne) consider(b, B.v[q], A.v[e], A.eu[e], A.el[e], false);
      }
    }
    return finish_closest(b, V2{1.0f, 0.0f}, V2{1.0f, 0.0f});
  }
  Hit h;
  h.d = -best;
  h.n = best_n;
  V2 p;
  if (best_k >= A.na) {  // axis of hi: deepest vertex of lo
    p = A.v[0];
    float m = vdot(best_n, p);
#pragma unroll
    for (int q = 1; q < 4; ++q) {
      if (q < A.nv) {
        const float t = vdot(best_n, A.v[q]);
        if (t < m) {
          m = t;
          p = A.v[q];
        }
      }
    }
  } else {               // axis of lo: deepest vertex of hi
    p = B.v[0];
    float m = vdot(best_n, p);
#pragma unroll
    for (int q = 1; q < 4; ++q) {
      if (q < B.nv) {
        const float t = vdot(best_n, B.v[q]);
        if (t > m) {
          m = t;
          p = B.v[q];
        }
      }
    }
  }
  h.plo = p;
  h.phi = p;
  return h;
}

// Narrow phase of a non-sphere-sphere pair in canonical (lo, hi) order.
__device__ Hit narrow(const Geo& lo, const Geo& hi) {
  if (lo.shape == SPHERE) {
    return hi.shape == LINE ? sphere_line(lo.c, hi) : sphere_box(lo.c, hi);
  }
  if (hi.shape == SPHERE) {
    Hit r = lo.shape == LINE ? sphere_line(hi.c, lo) : sphere_box(hi.c, lo);
    Hit o;
    o.d = r.d;
    o.n = vneg(r.n);
    o.plo = r.phi;
    o.phi = r.plo;
    return o;
  }
  if (lo.shape == LINE && hi.shape == LINE) return line_line(lo, hi);
  return poly_poly(lo, hi);
}

// Magnitude of Eq. (2): c k log(1 + e^z), z = (d_min - d)/k, in the stable
// form max(z, 0) + log1p(e^{-|z|}).
__device__ __forceinline__ float contact_mag(float dmin, float d, const WorldK& w) {
  const float z = (dmin - d) * w.inv_k;
  return w.ck * (fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))));
}

// SplitMix64 (Steele, Lea, Flood 2014) finaliser.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ float draw_sym(uint64_t key, uint64_t idx) {
  const uint64_t z = mix64(key + (idx + 1ull) * 0x9E3779B97F4A7C15ull);
  const int k = (int)(z >> 40);
  return (float)(k - (1 << 23)) * (1.0f / 8388608.0f);
}

// Contact of the lane's entity (self, environment-local index a) with the
// partner in LDS slot q (local index b). Accumulates the lane's force and
// torque and reports the contact bit.
template <bool SPH>
__device__ __forceinline__ bool pair_force(const Geo& self, float rho_s, int a, const float4 P,
                                           const float4 S, int b, const WorldK& w, float& fx,
                                           float& fy, float& tq) {
  const float rho_o = S.z;
  const float dmin = (rho_s + rho_o) + w.min_dist;
  const int so = SPH ? SPHERE : (__float_as_int(S.w) & 0xff);
  if (SPH || (self.shape == SPHERE && so == SPHERE)) {
    // Both spheres: x_ij joins the centres; decision on squared lengths.
    const float dx = self.c.x - P.x, dy = self.c.y - P.y;
    const float s = __fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy));
    if (!(s <= __fmul_rn(dmin, dmin))) return false;
    const float d = sqrtf(s);
    V2 n;
    if (d == 0.0f) n = a < b ? V2{1.0f, 0.0f} : V2{-1.0f, 0.0f};
    else n = vscl(V2{dx, dy}, 1.0f / d);
    const float F = contact_mag(dmin, d, w);
    fx = fmaf(F, n.x, fx);
    fy = fmaf(F, n.y, fy);
    return true;
  }
  Geo o;
  o.c = V2{P.x, P.y};
  o.cs = P.z;
  o.sn = P.w;
  o.d0 = S.x;
  o.d1 = S.y;
  o.shape = so;
  const bool self_lo = a < b;
  const Hit h = self_lo ? narrow(self, o) : narrow(o, self);
  if (!(h.d <= dmin)) return false;
  const float F = contact_mag(dmin, h.d, w);
  const float sg = self_lo ? F : -F;
  const V2 f = V2{sg * h.n.x, sg * h.n.y};
  const V2 arm = vsub(self_lo ? h.plo : h.phi, self.c);
  fx += f.x;
  fy += f.y;
  tq += vcross(arm, f);
  return true;
}

__device__ __forceinline__ bool excluded(int excl, int b) {
  const unsigned u = (unsigned)excl;
  return ((u & 0xffu) == (unsigned)b) | (((u >> 8) & 0xffu) == (unsigned)b) |
         (((u >> 16) & 0xffu) == (unsigned)b) | ((u >> 24) == (unsigned)b);
}

// Persistent rollout: T steps of every environment of the group.
template <bool SPH, int MAXB>
__global__ void __launch_bounds__(MAXB) k_rollout(StepArgs a) {
  extern __shared__ float4 lds[];
  const int E = a.max_stage;
  float4* buf0 = lds;
  float4* buf1 = lds + E;
  float4* stat = lds + 2 * E;
  const int g = blockIdx.x, l = threadIdx.x, B = blockDim.x;
  const int N = a.w.N;
  const int s0 = a.stage_off[g], ns = a.stage_off[g + 1] - s0;
  for (int s = l; s < ns; s += B) {
    const int e = a.stage[s0 + s];
    float cs = 1.0f, sn = 0.0f;
    if (!SPH) sincosf(a.state[4 * N + e], &sn, &cs);
    const float4 P = make_float4(a.state[e], a.state[N + e], cs, sn);
    buf0[s] = P;
    buf1[s] = P;
    const EntParam p = a.ent[e];
    stat[s] = make_float4(p.d0, p.d1, p.rho, __int_as_float(p.sf));
  }
  const LaneRec r = a.lanes[(size_t)g * B + l];
  const bool act = r.ent >= 0;
  float x = 0, y = 0, vx = 0, vy = 0, th = 0, om = 0;
  EntParam p{};
  if (act) {
    const int e = r.ent;
    x = a.state[e];
    y = a.state[N + e];
    vx = a.state[2 * N + e];
    vy = a.state[3 * N + e];
    th = a.state[4 * N + e];
    om = a.state[5 * N + e];
    p = a.ent[e];
  }
  const int shape = p.sf & 0xff, fl = (p.sf >> 8) & 0xff;
  const bool movable = (fl & MOVABLE) != 0, rotatable = (fl & ROTATABLE) != 0;
  const bool collide = act && (fl & COLLIDABLE) != 0;
  const int myloc = r.slot - r.lo;
  const int nloc = r.hi - r.lo;
  const WorldK w = a.w;
  // Actions of step t0 + t (prefetched one step ahead).
  float2 an = make_float2(0.0f, 0.0f);
  const bool agent = act && r.agent >= 0;
  if (agent && a.T > 0) {
    if (a.actions) an = *reinterpret_cast<const float2*>(a.actions + 2 * (size_t)r.agent);
    else {
      const uint64_t base = ((uint64_t)a.t0 * (uint64_t)w.A + (uint64_t)r.agent) * 2ull;
      an = make_float2(draw_sym(a.key, base), draw_sym(a.key, base + 1));
    }
  }
  __syncthreads();
  for (int t = 0; t < a.T; ++t) {
    float4* cur = (t & 1) ? buf1 : buf0;
    float cs = 1.0f, sn = 0.0f;
    if (!SPH && act && shape != SPHERE) sincosf(th, &sn, &cs);
    if (t > 0) {
      if (act) cur[r.slot] = make_float4(x, y, cs, sn);
      __syncthreads();
    }
    float fx = an.x + p.mgx, fy = an.y + p.mgy, tq = 0.0f;
    if (agent && t + 1 < a.T) {
      if (a.actions)
        an = *reinterpret_cast<const float2*>(a.actions + 2 * ((size_t)(t + 1) * w.A + r.agent));
      else {
        const uint64_t base =
            ((uint64_t)(a.t0 + t + 1) * (uint64_t)w.A + (uint64_t)r.agent) * 2ull;
        an = make_float2(draw_sym(a.key, base), draw_sym(a.key, base + 1));
      }
    }
    const bool last = t == a.T - 1;
    uint8_t* mk = (last && a.mask) ? a.mask : nullptr;
    if (collide) {
      Geo self;
      self.c = V2{x, y};
      self.cs = cs;
      self.sn = sn;
      self.d0 = p.d0;
      self.d1 = p.d1;
      self.shape = SPH ? SPHERE : shape;
      for (int q = r.lo; q < r.hi; ++q) {
        if (q == r.slot) continue;
        const float4 S = stat[q];
        const int of = (__float_as_int(S.w) >> 8) & 0xff;
        if (!(of & COLLIDABLE)) continue;
        const int b = q - r.lo;
        if (!SPH && p.excl != -1 && excluded(p.excl, b)) continue;
        const float4 P = cur[q];
        const bool hit = pair_force<SPH>(self, p.rho, myloc, P, S, b, w, fx, fy, tq);
        if (mk && hit) {
          // The lower index writes the slot, or the higher one when the
          // lower entity has no lane (neither movable nor rotatable).
          const bool other_active = (of & (MOVABLE | ROTATABLE)) != 0;
          if (myloc < b || !other_active) {
            const int ia = min(myloc, b), ib = max(myloc, b);
            const int64_t idx = (int64_t)ia * nloc - (int64_t)ia * (ia + 1) / 2 + (ib - ia - 1);
            mk[a.pair_off[r.env] + idx] = 1;
          }
        }
      }
    }
    if (!SPH && act) {
      // Joints: spring between world anchors, evaluated in joint order.
      const int j0 = a.joff[r.ent], j1 = a.joff[r.ent + 1];
      for (int jj = j0; jj < j1; ++jj) {
        const JointK J = a.joints[a.jlist[jj]];
        const bool is_a = J.a == r.ent;
        const int other = is_a ? J.b : J.a;
        const float4 P = cur[r.lo + (other - r.first)];
        const V2 xa = is_a ? V2{x, y} : V2{P.x, P.y};
        const V2 xb = is_a ? V2{P.x, P.y} : V2{x, y};
        const float ca = is_a ? cs : P.z, sa = is_a ? sn : P.w;
        const float cb = is_a ? P.z : cs, sb = is_a ? P.w : sn;
        const V2 Pa = vadd(xa, vrot(ca, sa, V2{J.ax, J.ay}));
        const V2 Pb = vadd(xb, vrot(cb, sb, V2{J.bx, J.by}));
        const V2 dl = vsub(Pa, Pb);
        const float len = sqrtf(vdot(dl, dl));
        if (len == 0.0f) continue;
        const float mag = -w.joint_k * (len - J.rest) / len;
        const V2 f = is_a ? vscl(dl, mag) : vscl(dl, -mag);
        const V2 arm = is_a ? vsub(Pa, xa) : vsub(Pb, xb);
        fx += f.x;
        fy += f.y;
        tq += vcross(arm, f);
      }
    }
    if (last && a.forces && act) {
      a.forces[r.ent] = fx;
      a.forces[N + r.ent] = fy;
      a.forces[2 * N + r.ent] = tq;
    }
    // Eq. (1) and Eq. (3): semi-implicit Euler with damping.
    if (act && movable) {
      const float ax = fx * p.inv_m, ay = fy * p.inv_m;
      vx = fmaf(ax, w.dt, w.damp * vx);
      vy = fmaf(ay, w.dt, w.damp * vy);
      if (p.vmax > 0.0f) {
        const float sp = sqrtf(fmaf(vx, vx, vy * vy));
        if (sp > p.vmax) {
          const float s = p.vmax / sp;
          vx *= s;
          vy *= s;
        }
      }
      x = fmaf(vx, w.dt, x);
      y = fmaf(vy, w.dt, y);
    }
    if (act && rotatable) {
      om = fmaf(tq * p.inv_I, w.dt, w.damp * om);
      th = fmaf(om, w.dt, th);
    }
    if (a.traj && act) {
      float* o = a.traj + (size_t)(t + 1) * 6 * N;
      o[r.ent] = x;
      o[N + r.ent] = y;
      o[2 * N + r.ent] = vx;
      o[3 * N + r.ent] = vy;
      o[4 * N + r.ent] = th;
      o[5 * N + r.ent] = om;
    }
  }
  if (act && a.T > 0) {
    const int e = r.ent;
    a.state[e] = x;
    a.state[N + e] = y;
    a.state[2 * N + e] = vx;
    a.state[3 * N + e] = vy;
    a.state[4 * N + e] = th;
    a.state[5 * N + e] = om;
  }
}

__global__ void k_fill_u8(uint8_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_replicate(const float* __restrict__ src, float* __restrict__ dst, int64_t n,
                            int copies) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n * copies;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i % n];
}

int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_rollout(const StepArgs& a, int groups, int block, bool spheres_only,
                          hipStream_t s) {
  const size_t shm = (size_t)a.max_stage * 3 * sizeof(float4);
  if (block <= 256) {
    if (spheres_only)
      hipLaunchKernelGGL((k_rollout<true, 256>), dim3(groups), dim3(block), shm, s, a);
    else
      hipLaunchKernelGGL((k_rollout<false, 256>), dim3(groups), dim3(block), shm, s, a);
  } else {
    if (spheres_only)
      hipLaunchKernelGGL((k_rollout<true, 1024>), dim3(groups), dim3(block), shm, s, a);
    else
      hipLaunchKernelGGL((k_rollout<false, 1024>), dim3(groups), dim3(block), shm, s, a);
  }
  return hipGetLastError();
}

const void* rollout_kernel(bool spheres_only, int block) {
  if (block <= 256)
    return spheres_only ? (const void*)k_rollout<true, 256> : (const void*)k_rollout<false, 256>;
  return spheres_only ? (const void*)k_rollout<true, 1024> : (const void*)k_rollout<false, 1024>;
}

hipError_t launch_fill_u8(uint8_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_replicate(const float* src, float* dst, int64_t n, int copies, hipStream_t s) {
  if (n <= 0 || copies <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_replicate, dim3(grid_for(n * copies)), dim3(256), 0, s, src, dst, n,
                     copies);
  return hipGetLastError();
}

uint64_t action_key(uint64_t seed) {
  uint64_t z = seed + 3ull * 0x9E3779B97F4A7C15ull;  // stream 2: (stream + 1) * golden
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace vmas
