// Plain, slow, single-threaded FP64 CPU oracle of the batched 2D physics step
// of VMAS (Bettini, Kortvelesy, Blumenkamp, Prorok, "VMAS: A Vectorized
// Multi-Agent Simulator for Collective Robot Learning", 2022).
//
// TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU
// baseline of the benchmark load this library. It shares no code with the
// HIP path (no headers, no helpers, no tables); the only thing both sides
// consume is the seeded input generator, which holds none of the physics.
//
// What it computes, per environment, per step (Sec. 3 "Core"):
//   * Eq. (1): f_i = f^a_i + m_i g + sum_j f^e_ij, then semi-implicit Euler
//     with velocity damping (1 - zeta).
//   * Eq. (2): the penalty contact force c * k * log(1 + exp(-(|x_ij| - d_min)/k))
//     along the unit vector between the closest points of the two shapes,
//     applied when |x_ij| <= d_min.
//   * Eq. (3): torque from the contact point arm, then the same semi-implicit
//     Euler step on (theta, omega).
//   Points where the paper is silent are fixed as stated next to the code
//   (closest-point routines, signed distance for overlaps, joint model,
//   flag semantics, inertia defaults, max-speed clamp); each is a reading of
//   the paper, not something it prints.
//
// Everything is templated on the scalar type:
//   * double  -> the oracle proper;
//   * Dual    -> forward-mode tangents (exact JVP of the discrete step, used to
//                check the hand-written adjoint);
//   * float   -> the same definition evaluated in FP32, operation by
//                operation as written here. It is never the reference: the
//                parity tests use its distance from the FP64 result only to
//                size how far any FP32 evaluation of an environment's step can
//                be from the exact one (their conditioning allowance).
// Branches on the geometry are taken on values; a Dual carries the derivative
// of the branch that is taken.
//
// The contact decision of Eq. (2), |x_ij| <= d_min, is taken on the FP64
// signed distance of this file's own narrow phase against the FP64 sum
// d_min = rho_i + rho_j + min_dist. A GPU that decides in FP32 can disagree
// only for pairs whose distance lies within FP32 rounding of d_min; the tests
// count those as band cases. Parity unpinned: the values of c and k, the
// joint model and the tie-breaking order between equally close features are
// this implementation's reading, not fixed by the paper.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

// ---------------------------------------------------------------- scalars --

struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double x) : v(x), d(0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
inline bool operator==(Dual a, Dual b) { return a.v == b.v; }

inline double val(double x) { return x; }
inline double val(Dual x) { return x.v; }
inline double val(float x) { return x; }

inline double m_sqrt(double x) { return std::sqrt(x); }
inline Dual m_sqrt(Dual x) {
  double s = std::sqrt(x.v);
  return {s, s > 0 ? x.d / (2 * s) : 0.0};
}
inline double m_sin(double x) { return std::sin(x); }
inline Dual m_sin(Dual x) { return {std::sin(x.v), std::cos(x.v) * x.d}; }
inline double m_cos(double x) { return std::cos(x); }
inline Dual m_cos(Dual x) { return {std::cos(x.v), -std::sin(x.v) * x.d}; }
inline double m_exp(double x) { return std::exp(x); }
inline Dual m_exp(Dual x) {
  double e = std::exp(x.v);
  return {e, e * x.d};
}
inline double m_log1p(double x) { return std::log1p(x); }
inline Dual m_log1p(Dual x) { return {std::log1p(x.v), x.d / (1 + x.v)}; }
inline float m_sqrt(float x) { return std::sqrt(x); }
inline float m_sin(float x) { return std::sin(x); }
inline float m_cos(float x) { return std::cos(x); }
inline float m_exp(float x) { return std::exp(x); }
inline float m_log1p(float x) { return std::log1p(x); }
template <class T> inline T m_abs(T x) { return x < T(0) ? -x : x; }

// ------------------------------------------------------------ 2D vectors --

template <class T> struct V2 { T x, y; };
template <class T> inline V2<T> add(V2<T> a, V2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <class T> inline V2<T> sub(V2<T> a, V2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <class T> inline V2<T> mul(V2<T> a, T s) { return {a.x * s, a.y * s}; }
template <class T> inline V2<T> neg(V2<T> a) { return {-a.x, -a.y}; }
template <class T> inline T dot(V2<T> a, V2<T> b) { return a.x * b.x + a.y * b.y; }
// Signed scalar 2D cross product a_x b_y - a_y b_x: the torque of Eq. (3)
// read as a signed quantity (the norm printed there could never change sign).
template <class T> inline T cross(V2<T> a, V2<T> b) { return a.x * b.y - a.y * b.x; }
template <class T> inline T norm(V2<T> a) { return m_sqrt(dot(a, a)); }

enum { SPHERE = 0, BOX = 1, LINE = 2 };
enum { MOVABLE = 1, ROTATABLE = 2, COLLIDABLE = 4 };

// Pose of one entity plus its rotation R(theta) = [[c, -s], [s, c]].
template <class T> struct Pose {
  V2<T> c;
  T cs, sn;
};
template <class T> inline V2<T> rot(const Pose<T>& p, V2<T> v) {
  return {p.cs * v.x - p.sn * v.y, p.sn * v.x + p.cs * v.y};
}
template <class T> inline V2<T> rot_t(const Pose<T>& p, V2<T> v) {
  return {p.cs * v.x + p.sn * v.y, -p.sn * v.x + p.cs * v.y};
}

// Result of the narrow phase for the ordered pair (i, j): signed distance d
// between the cores (negative when they overlap), unit normal n along which i
// is pushed, and the contact points on i and on j that give the torque arms.
template <class T> struct Contact {
  T d;
  V2<T> n, pi, pj;
};

// Closest point to p on the segment [a, b] (clamped projection; a if a == b).
template <class T> V2<T> seg_closest(V2<T> p, V2<T> a, V2<T> b) {
  V2<T> ab = sub(b, a);
  T l2 = dot(ab, ab);
  if (l2 == T(0)) return a;
  T t = dot(sub(p, a), ab) / l2;
  if (t < T(0)) t = T(0);
  if (t > T(1)) t = T(1);
  return add(a, mul(ab, t));
}

// A line entity runs along its local x axis, centred on its position.
template <class T> void line_ends(const Pose<T>& p, T len, V2<T>* a, V2<T>* b) {
  V2<T> h = {p.cs * (len / T(2)), p.sn * (len / T(2))};
  *a = sub(p.c, h);
  *b = add(p.c, h);
}
// Left normal of a line entity, (-sin, cos).
template <class T> V2<T> line_normal(const Pose<T>& p) { return {-p.sn, p.cs}; }

// Box vertices, counter-clockwise from the (+x, +y) corner in the local frame.
template <class T> void box_verts(const Pose<T>& p, T lx, T ly, V2<T> v[4]) {
  T hx = lx / T(2), hy = ly / T(2);
  V2<T> loc[4] = {{hx, hy}, {-hx, hy}, {-hx, -hy}, {hx, -hy}};
  for (int k = 0; k < 4; ++k) v[k] = add(p.c, rot(p, loc[k]));
}

// -- sphere / sphere: the vector between the centres (MPE's form).
template <class T> Contact<T> sphere_sphere(V2<T> ci, V2<T> cj) {
  Contact<T> r;
  V2<T> dl = sub(ci, cj);
  r.d = norm(dl);
  if (r.d == T(0)) r.n = {T(1), T(0)};
  else r.n = {dl.x / r.d, dl.y / r.d};
  r.pi = ci;
  r.pj = cj;
  return r;
}

// -- sphere (i) / line (j): closest point on the segment.
template <class T> Contact<T> sphere_line(V2<T> c, const Pose<T>& pl, T len) {
  V2<T> a, b;
  line_ends(pl, len, &a, &b);
  V2<T> q = seg_closest(c, a, b);
  V2<T> dl = sub(c, q);
  Contact<T> r;
  r.d = norm(dl);
  if (r.d == T(0)) r.n = line_normal(pl);
  else r.n = {dl.x / r.d, dl.y / r.d};
  r.pi = c;
  r.pj = q;
  return r;
}

// -- sphere (i) / box (j): closest point on the solid rectangle; inside, the
//    nearest face (x face wins a tie) gives a negative distance.
template <class T> Contact<T> sphere_box(V2<T> c, const Pose<T>& pb, T lx, T ly) {
  T hx = lx / T(2), hy = ly / T(2);
  V2<T> u = rot_t(pb, sub(c, pb.c));
  V2<T> nl, ql;
  Contact<T> r;
  if (m_abs(u.x) <= hx && m_abs(u.y) <= hy) {
    T dx = hx - m_abs(u.x), dy = hy - m_abs(u.y);
    if (dx <= dy) {
      T s = u.x >= T(0) ? T(1) : T(-1);
      r.d = -dx;
      nl = {s, T(0)};
      ql = {s * hx, u.y};
    } else {
      T s = u.y >= T(0) ? T(1) : T(-1);
      r.d = -dy;
      nl = {T(0), s};
      ql = {u.x, s * hy};
    }
  } else {
    ql = u;
    if (ql.x < -hx) ql.x = -hx;
    if (ql.x > hx) ql.x = hx;
    if (ql.y < -hy) ql.y = -hy;
    if (ql.y > hy) ql.y = hy;
    V2<T> w = sub(u, ql);
    r.d = norm(w);
    nl = {w.x / r.d, w.y / r.d};
  }
  r.n = rot(pb, nl);
  r.pj = add(pb.c, rot(pb, ql));
  r.pi = c;
  return r;
}

template <class T> inline int sgn(T x) { return x > T(0) ? 1 : (x < T(0) ? -1 : 0); }

// Distance branch shared by the segment and polygon routines: the closest
// pair of features is a vertex of one shape against an edge of the other.
template <class T> struct Best {
  bool any = false;
  T d = T(0);
  V2<T> n, pi, pj;
  // Vertex e of i against its foot q on j: i is pushed from q towards e.
  void vert_i(V2<T> e, V2<T> q, V2<T> fallback) {
    T dd = norm(sub(e, q));
    if (!any || dd < d) {
      any = true;
      d = dd;
      pi = e;
      pj = q;
      if (dd == T(0)) n = fallback;
      else n = {(e.x - q.x) / dd, (e.y - q.y) / dd};
    }
  }
  // Vertex e of j against its foot q on i: i is pushed from e towards q.
  void vert_j(V2<T> e, V2<T> q, V2<T> fallback) {
    T dd = norm(sub(e, q));
    if (!any || dd < d) {
      any = true;
      d = dd;
      pi = q;
      pj = e;
      if (dd == T(0)) n = fallback;
      else n = {(q.x - e.x) / dd, (q.y - e.y) / dd};
    }
  }
};

// -- line (i) / line (j). Crossing is decided by the four orientation signs
//    (collinear overlap counts as crossing). Apart: exact segment-segment
//    distance from the four endpoint-to-segment distances, first strict
//    minimum in the order a_i, b_i, a_j, b_j. Crossing: the separating-axis
//    reading for two segments, d = -(smallest perpendicular distance of an
//    endpoint to the other segment's supporting line), pushing that endpoint
//    back across that line; both branches meet at d = 0 with the same normal.
template <class T> Contact<T> line_line(const Pose<T>& pi_, T li, const Pose<T>& pj_, T lj) {
  V2<T> ai, bi, aj, bj;
  line_ends(pi_, li, &ai, &bi);
  line_ends(pj_, lj, &aj, &bj);
  V2<T> ni = line_normal(pi_), nj = line_normal(pj_);
  int o1 = sgn(cross(sub(bi, ai), sub(aj, ai)));
  int o2 = sgn(cross(sub(bi, ai), sub(bj, ai)));
  int o3 = sgn(cross(sub(bj, aj), sub(ai, aj)));
  int o4 = sgn(cross(sub(bj, aj), sub(bi, aj)));
  bool crossing;
  if (o1 == 0 && o2 == 0 && o3 == 0 && o4 == 0) {
    V2<T> u = sub(bi, ai);
    T tu = dot(u, u);
    T ta = dot(sub(aj, ai), u), tb = dot(sub(bj, ai), u);
    T lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
    crossing = !(hi < T(0) || lo > tu);
  } else {
    crossing = (o1 * o2 <= 0) && (o3 * o4 <= 0);
  }
  Contact<T> r;
  if (!crossing) {
    Best<T> b;
    b.vert_i(ai, seg_closest(ai, aj, bj), nj);
    b.vert_i(bi, seg_closest(bi, aj, bj), nj);
    b.vert_j(aj, seg_closest(aj, ai, bi), neg(ni));
    b.vert_j(bj, seg_closest(bj, ai, bi), neg(ni));
    r.d = b.d;
    r.n = b.n;
    r.pi = b.pi;
    r.pj = b.pj;
    return r;
  }
  // Signed offsets of each endpoint from the other supporting line.
  V2<T> ends[4] = {ai, bi, aj, bj};
  bool first = true;
  T best = T(0);
  for (int k = 0; k < 4; ++k) {
    bool of_i = k < 2;
    V2<T> base = of_i ? aj : ai;
    V2<T> nrm = of_i ? nj : ni;
    T s = dot(sub(ends[k], base), nrm);
    T dist = m_abs(s);
    if (first || dist < best) {
      first = false;
      best = dist;
      // Direction in which the owner of the endpoint is pushed: from the
      // endpoint towards the other line; on the line, that line's normal.
      V2<T> push = s > T(0) ? neg(nrm) : (s < T(0) ? nrm : nrm);
      r.n = of_i ? push : neg(push);
      r.pi = ends[k];
      r.pj = ends[k];
    }
  }
  r.d = -best;
  return r;
}

// Convex polygon view of a box (4 CCW vertices, 4 edges, 2 axes) or a line
// (2 vertices, 1 edge, 1 axis: its normal).
template <class T> struct Poly {
  int nv, ne, na;
  V2<T> v[4];
  V2<T> ea[4], eb[4];
  V2<T> ax[2];
};
template <class T> Poly<T> make_poly(int shape, const Pose<T>& p, T d0, T d1) {
  Poly<T> q;
  if (shape == BOX) {
    box_verts(p, d0, d1, q.v);
    q.nv = 4;
    q.ne = 4;
    for (int k = 0; k < 4; ++k) {
      q.ea[k] = q.v[k];
      q.eb[k] = q.v[(k + 1) % 4];
    }
    q.na = 2;
    q.ax[0] = {p.cs, p.sn};
    q.ax[1] = {-p.sn, p.cs};
  } else {
    line_ends(p, d0, &q.v[0], &q.v[1]);
    q.nv = 2;
    q.ne = 1;
    q.ea[0] = q.v[0];
    q.eb[0] = q.v[1];
    q.na = 1;
    q.ax[0] = line_normal(p);
  }
  return q;
}

// -- line / box and box / box by the separating-axis test. Apart: exact
//    distance between the two convex sets (vertex of one against edge of the
//    other, i's vertices first). Overlapping: smallest overlap over the axes
//    (i's first, first strict minimum), contact point at the deepest vertex of
//    the shape that does not own the winning axis.
template <class T> Contact<T> poly_poly(const Poly<T>& A, const Poly<T>& B) {
  bool separated = false;
  for (int k = 0; k < A.na + B.na && !separated; ++k) {
    V2<T> s = k < A.na ? A.ax[k] : B.ax[k - A.na];
    T mina = dot(A.v[0], s), maxa = mina, minb = dot(B.v[0], s), maxb = minb;
    for (int q = 1; q < A.nv; ++q) {
      T t = dot(A.v[q], s);
      if (t < mina) mina = t;
      if (t > maxa) maxa = t;
    }
    for (int q = 1; q < B.nv; ++q) {
      T t = dot(B.v[q], s);
      if (t < minb) minb = t;
      if (t > maxb) maxb = t;
    }
    if (maxa < minb || maxb < mina) separated = true;
  }
  Contact<T> r;
  if (separated) {
    Best<T> b;
    V2<T> fb = {T(1), T(0)};
    for (int q = 0; q < A.nv; ++q)
      for (int e = 0; e < B.ne; ++e) b.vert_i(A.v[q], seg_closest(A.v[q], B.ea[e], B.eb[e]), fb);
    for (int q = 0; q < B.nv; ++q)
      for (int e = 0; e < A.ne; ++e) b.vert_j(B.v[q], seg_closest(B.v[q], A.ea[e], A.eb[e]), fb);
    r.d = b.d;
    r.n = b.n;
    r.pi = b.pi;
    r.pj = b.pj;
    return r;
  }
  bool first = true;
  T best = T(0);
  int best_k = 0;
  for (int k = 0; k < A.na + B.na; ++k) {
    V2<T> s = k < A.na ? A.ax[k] : B.ax[k - A.na];
    T mina = dot(A.v[0], s), maxa = mina, minb = dot(B.v[0], s), maxb = minb;
    for (int q = 1; q < A.nv; ++q) {
      T t = dot(A.v[q], s);
      if (t < mina) mina = t;
      if (t > maxa) maxa = t;
    }
    for (int q = 1; q < B.nv; ++q) {
      T t = dot(B.v[q], s);
      if (t < minb) minb = t;
      if (t > maxb) maxb = t;
    }
    T op = maxb - mina;  // translate i by +s
    T om = maxa - minb;  // translate i by -s
    T ov = op <= om ? op : om;
    if (first || ov < best) {
      first = false;
      best = ov;
      best_k = k;
      r.n = op <= om ? s : neg(s);
    }
  }
  r.d = -best;
  V2<T> p;
  if (best_k >= A.na) {  // axis of j: deepest vertex of i
    p = A.v[0];
    T m = dot(r.n, p);
    for (int q = 1; q < A.nv; ++q) {
      T t = dot(r.n, A.v[q]);
      if (t < m) {
        m = t;
        p = A.v[q];
      }
    }
  } else {  // axis of i: deepest vertex of j
    p = B.v[0];
    T m = dot(r.n, p);
    for (int q = 1; q < B.nv; ++q) {
      T t = dot(r.n, B.v[q]);
      if (t > m) {
        m = t;
        p = B.v[q];
      }
    }
  }
  r.pi = p;
  r.pj = p;
  return r;
}

// Narrow phase for the pair (i, j) in index order.
template <class T>
Contact<T> narrow(int si, T di0, T di1, const Pose<T>& pi, int sj, T dj0, T dj1, const Pose<T>& pj) {
  (void)di1;
  (void)dj1;
  if (si == SPHERE && sj == SPHERE) return sphere_sphere(pi.c, pj.c);
  if (si == SPHERE && sj == LINE) return sphere_line(pi.c, pj, dj0);
  if (si == SPHERE && sj == BOX) return sphere_box(pi.c, pj, dj0, dj1);
  if (sj == SPHERE) {  // swap roles, negate the normal
    Contact<T> r = si == LINE ? sphere_line(pj.c, pi, di0) : sphere_box(pj.c, pi, di0, di1);
    Contact<T> o;
    o.d = r.d;
    o.n = neg(r.n);
    o.pi = r.pj;
    o.pj = r.pi;
    return o;
  }
  if (si == LINE && sj == LINE) return line_line(pi, di0, pj, dj0);
  return poly_poly(make_poly(si, pi, di0, di1), make_poly(sj, pj, dj0, dj1));
}

// Stable log(1 + e^z) = max(z, 0) + log1p(e^{-|z|}), the k-scaled term of Eq. (2).
template <class T> T softplus(T z) {
  T a = m_abs(z);
  T m = z > T(0) ? z : T(0);
  return m + m_log1p(m_exp(-a));
}

}  // namespace

// ------------------------------------------------------------------ C API --

extern "C" {

// World description; all arrays are host memory owned by the caller.
// Entity e of environment b is global index env_offset[b] + e; the agents
// of b are its first n_agents[b] entities and their actions are rows
// agent_offset(b) + e of the [A][2] action array (environments in order).
typedef struct {
  int32_t n_envs;
  const int32_t* env_offset;  // [n_envs + 1]
  const int32_t* n_agents;    // [n_envs]
  const uint8_t* shape;       // [N] 0 sphere, 1 box, 2 line
  const double* dims;         // [N][2] sphere (r, -), box (lx, ly), line (L, -)
  const double* mass;         // [N]
  const double* inertia;      // [N] or NULL: <= 0 or NULL -> textbook default
  const double* max_speed;    // [N] or NULL: <= 0 -> no clamp
  const uint8_t* flags;       // [N] 1 movable, 2 rotatable, 4 collidable
  int32_t n_joints;
  const int32_t* joint_a;     // [J] global entity ids (same environment)
  const int32_t* joint_b;
  const double* anchor_a;     // [J][2] body-frame anchors
  const double* anchor_b;
  const double* rest;         // [J] rest lengths
  const uint8_t* joint_collide;  // [J] or NULL -> jointed pairs do not collide
  double dt, drag, gx, gy;    // delta t, zeta, g
  double c, k, min_dist;      // Eq. (2) intensity, softness, extra d_min
  double joint_k;             // joint stiffness
} oracle_world;

}  // extern "C"

namespace {

double default_inertia(int shape, double m, double d0, double d1) {
  if (shape == SPHERE) return m * d0 * d0 / 2;         // solid disc
  if (shape == BOX) return m * (d0 * d0 + d1 * d1) / 12;  // solid rectangle
  return m * d0 * d0 / 12;                               // thin rod
}

double inertia_of(const oracle_world* w, int i) {
  double I = w->inertia ? w->inertia[i] : 0.0;
  if (I > 0) return I;
  return default_inertia(w->shape[i], w->mass[i], w->dims[2 * i], w->dims[2 * i + 1]);
}

inline bool has_dof(uint8_t f) { return (f & (MOVABLE | ROTATABLE)) != 0; }

// Whether entities a and b (global ids) are joined by one of the joints in
// js[0..nj) whose flag disables their contact.
bool joint_excluded(const oracle_world* w, const int* js, int nj, int a, int b) {
  for (int t = 0; t < nj; ++t) {
    int q = js[t];
    int ja = w->joint_a[q], jb = w->joint_b[q];
    if ((ja == a && jb == b) || (ja == b && jb == a)) {
      if (!w->joint_collide || !w->joint_collide[q]) return true;
    }
  }
  return false;
}

// Pair eligibility: both collidable, at least one with a free degree of
// freedom, and not switched off by a joint.
bool pair_eligible(const oracle_world* w, const int* js, int nj, int a, int b) {
  uint8_t fa = w->flags[a], fb = w->flags[b];
  if (!(fa & COLLIDABLE) || !(fb & COLLIDABLE)) return false;
  if (!has_dof(fa) && !has_dof(fb)) return false;
  return !joint_excluded(w, js, nj, a, b);
}

// Environment that owns global entity i.
int env_of(const oracle_world* w, int i) {
  int lo = 0, hi = w->n_envs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) / 2;
    if (w->env_offset[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <class T> Pose<T> pose_of(const T* x, const T* y, const T* th, int i) {
  Pose<T> p;
  p.c = {x[i], y[i]};
  p.cs = m_cos(th[i]);
  p.sn = m_sin(th[i]);
  return p;
}

// One step of environments [e0, e1) in place. State is field-major [6][N]:
// x, y, vx, vy, theta, omega. mask (optional) gets one byte per pair slot,
// environments in order, pairs (a < b) in lexicographic order of the local
// indices; forces (optional) gets [3][N] = total force x, y and torque.
// World anchor points of joint q: P = x + R(theta) anchor for both ends.
template <class T>
void joint_points(const oracle_world* w, const T* X, const T* Y, const T* TH, int q, Pose<T>* pa,
                  Pose<T>* pb, V2<T>* Pa, V2<T>* Pb) {
  *pa = pose_of(X, Y, TH, w->joint_a[q]);
  *pb = pose_of(X, Y, TH, w->joint_b[q]);
  *Pa = add(pa->c, rot(*pa, V2<T>{T(w->anchor_a[2 * q]), T(w->anchor_a[2 * q + 1])}));
  *Pb = add(pb->c, rot(*pb, V2<T>{T(w->anchor_b[2 * q]), T(w->anchor_b[2 * q + 1])}));
}

template <class T>
void step_envs(const oracle_world* w, int e0, int e1, T* st, const T* act, uint8_t* mask,
               T* forces) {
  const int N = w->env_offset[w->n_envs];
  T *X = st, *Y = st + N, *VX = st + 2 * N, *VY = st + 3 * N, *TH = st + 4 * N, *OM = st + 5 * N;
  int64_t pair_base = 0, agent_base = 0;
  for (int b = 0; b < e0; ++b) {
    int64_t n = w->env_offset[b + 1] - w->env_offset[b];
    pair_base += n * (n - 1) / 2;
    agent_base += w->n_agents[b];
  }
  // Joints of each environment in the range, in joint order.
  std::vector<int> jcount(e1 - e0 + 1, 0), jlist;
  std::vector<int> jenv(w->n_joints);
  for (int q = 0; q < w->n_joints; ++q) {
    jenv[q] = env_of(w, w->joint_a[q]);
    if (jenv[q] >= e0 && jenv[q] < e1) jcount[jenv[q] - e0 + 1]++;
  }
  for (int b = 0; b < e1 - e0; ++b) jcount[b + 1] += jcount[b];
  jlist.resize(jcount[e1 - e0]);
  {
    std::vector<int> fill(jcount.begin(), jcount.end() - 1);
    for (int q = 0; q < w->n_joints; ++q)
      if (jenv[q] >= e0 && jenv[q] < e1) jlist[fill[jenv[q] - e0]++] = q;
  }
  std::vector<T> FX, FY, TQ;
  for (int b = e0; b < e1; ++b) {
    const int o = w->env_offset[b], n = w->env_offset[b + 1] - o;
    const int* js = jlist.data() + jcount[b - e0];
    const int nj = jcount[b - e0 + 1] - jcount[b - e0];
    FX.assign(n, T(0));
    FY.assign(n, T(0));
    TQ.assign(n, T(0));
    // Eq. (1): action force on agents, gravity m g on movable entities.
    for (int a = 0; a < n; ++a) {
      int i = o + a;
      if (a < w->n_agents[b]) {
        FX[a] = FX[a] + act[2 * (agent_base + a)];
        FY[a] = FY[a] + act[2 * (agent_base + a) + 1];
      }
      if (w->flags[i] & MOVABLE) {
        FX[a] = FX[a] + T(w->mass[i] * w->gx);
        FY[a] = FY[a] + T(w->mass[i] * w->gy);
      }
    }
    // Eq. (2) and the torque of Eq. (3), every pair once, lexicographic.
    int64_t slot = pair_base;
    for (int a = 0; a < n; ++a) {
      for (int c = a + 1; c < n; ++c, ++slot) {
        int i = o + a, j = o + c;
        if (mask) mask[slot] = 0;
        if (!pair_eligible(w, js, nj, i, j)) continue;
        Pose<T> pi = pose_of(X, Y, TH, i), pj = pose_of(X, Y, TH, j);
        Contact<T> r = narrow<T>(w->shape[i], T(w->dims[2 * i]), T(w->dims[2 * i + 1]), pi,
                                 w->shape[j], T(w->dims[2 * j]), T(w->dims[2 * j + 1]), pj);
        double ri = w->shape[i] == SPHERE ? w->dims[2 * i] : 0.0;
        double rj = w->shape[j] == SPHERE ? w->dims[2 * j] : 0.0;
        T dmin = T(ri + rj + w->min_dist);
        // Eq. (2): the force acts iff |x_ij| <= d_min (inclusive), decided on
        // the signed distance just computed.
        bool hit = val(r.d) <= val(dmin);
        if (mask) mask[slot] = hit ? 1 : 0;
        if (!hit) continue;
        T F = T(w->c * w->k) * softplus((dmin - r.d) / T(w->k));
        V2<T> f = mul(r.n, F);
        FX[a] = FX[a] + f.x;
        FY[a] = FY[a] + f.y;
        FX[c] = FX[c] - f.x;
        FY[c] = FY[c] - f.y;
        TQ[a] = TQ[a] + cross(sub(r.pi, pi.c), f);
        TQ[c] = TQ[c] + cross(sub(r.pj, pj.c), neg(f));
      }
    }
    // Joints: a linear spring between the two world anchor points.
    for (int t = 0; t < nj; ++t) {
      int q = js[t];
      int ia = w->joint_a[q], ib = w->joint_b[q];
      Pose<T> pa, pb;
      V2<T> Pa, Pb;
      joint_points(w, X, Y, TH, q, &pa, &pb, &Pa, &Pb);
      V2<T> dl = sub(Pa, Pb);
      T len = norm(dl);
      if (len == T(0)) continue;
      T mag = -T(w->joint_k) * (len - T(w->rest[q])) / len;
      V2<T> f = mul(dl, mag);
      int a = ia - o, c = ib - o;
      FX[a] = FX[a] + f.x;
      FY[a] = FY[a] + f.y;
      FX[c] = FX[c] - f.x;
      FY[c] = FY[c] - f.y;
      TQ[a] = TQ[a] + cross(sub(Pa, pa.c), f);
      TQ[c] = TQ[c] + cross(sub(Pb, pb.c), neg(f));
    }
    // Eq. (1) and Eq. (3): semi-implicit Euler with damping (1 - zeta).
    for (int a = 0; a < n; ++a) {
      int i = o + a;
      if (forces) {
        forces[i] = FX[a];
        forces[N + i] = FY[a];
        forces[2 * N + i] = TQ[a];
      }
      if (w->flags[i] & MOVABLE) {
        T damp = T(1.0 - w->drag);
        T vx = damp * VX[i] + FX[a] / T(w->mass[i]) * T(w->dt);
        T vy = damp * VY[i] + FY[a] / T(w->mass[i]) * T(w->dt);
        double vmax = w->max_speed ? w->max_speed[i] : 0.0;
        if (vmax > 0) {
          T sp = m_sqrt(vx * vx + vy * vy);
          if (sp > T(vmax)) {
            vx = vx * (T(vmax) / sp);
            vy = vy * (T(vmax) / sp);
          }
        }
        VX[i] = vx;
        VY[i] = vy;
        X[i] = X[i] + vx * T(w->dt);
        Y[i] = Y[i] + vy * T(w->dt);
      }
      if (w->flags[i] & ROTATABLE) {
        T damp = T(1.0 - w->drag);
        T om = damp * OM[i] + TQ[a] / T(inertia_of(w, i)) * T(w->dt);
        OM[i] = om;
        TH[i] = TH[i] + om * T(w->dt);
      }
    }
    pair_base += (int64_t)n * (n - 1) / 2;
    agent_base += w->n_agents[b];
  }
}

int64_t total_agents(const oracle_world* w) {
  int64_t A = 0;
  for (int b = 0; b < w->n_envs; ++b) A += w->n_agents[b];
  return A;
}

}  // namespace

extern "C" {

// One step of every environment, in place. Returns 0.
int oracle_step(const oracle_world* w, double* state, const double* actions, uint8_t* mask,
                double* forces) {
  step_envs<double>(w, 0, w->n_envs, state, actions, mask, forces);
  return 0;
}

// T steps of environments [e0, e1) (state and actions are the full arrays;
// actions [T][A][2]). traj (optional) receives [T+1][6][N] snapshots of the
// whole state array; mask_final (optional) the mask of the last step.
// Disjoint environment ranges may run concurrently from different threads.
int oracle_rollout_range(const oracle_world* w, int e0, int e1, double* state,
                         const double* actions, int T, double* traj, uint8_t* mask_final) {
  const int64_t N = w->env_offset[w->n_envs];
  const int64_t A = total_agents(w);
  if (traj) std::memcpy(traj, state, sizeof(double) * 6 * N);
  for (int t = 0; t < T; ++t) {
    step_envs<double>(w, e0, e1, state, actions + 2 * A * t, t == T - 1 ? mask_final : nullptr,
                      nullptr);
    if (traj) std::memcpy(traj + 6 * N * (t + 1), state, sizeof(double) * 6 * N);
  }
  return 0;
}

int oracle_rollout(const oracle_world* w, double* state, const double* actions, int T,
                   double* traj, uint8_t* mask_final) {
  return oracle_rollout_range(w, 0, w->n_envs, state, actions, T, traj, mask_final);
}

// Forward-mode tangent of a T-step rollout: given the tangent (dstate,
// dactions) of the inputs, returns the final state and its tangent, exactly
// for the discrete step (contact decisions held at their values).
int oracle_rollout_jvp(const oracle_world* w, double* state, double* dstate,
                       const double* actions, const double* dactions, int T) {
  const int64_t N = w->env_offset[w->n_envs];
  const int64_t A = total_agents(w);
  std::vector<Dual> s(6 * N), a(2 * A);
  for (int64_t q = 0; q < 6 * N; ++q) s[q] = Dual(state[q], dstate[q]);
  for (int t = 0; t < T; ++t) {
    for (int64_t q = 0; q < 2 * A; ++q)
      a[q] = Dual(actions[2 * A * t + q], dactions ? dactions[2 * A * t + q] : 0.0);
    step_envs<Dual>(w, 0, w->n_envs, s.data(), a.data(), nullptr, nullptr);
  }
  for (int64_t q = 0; q < 6 * N; ++q) {
    state[q] = s[q].v;
    dstate[q] = s[q].d;
  }
  return 0;
}

// The same step and rollout evaluated in FP32 (see the header: it only sizes
// the FP32 rounding allowance of the parity tests). state [6][N] float,
// actions [T][A][2] float, traj (optional) [T+1][6][N] float.
int oracle_rollout_fp32(const oracle_world* w, float* state, const float* actions, int T,
                        float* traj) {
  const int64_t N = w->env_offset[w->n_envs];
  const int64_t A = total_agents(w);
  if (traj) std::memcpy(traj, state, sizeof(float) * 6 * N);
  for (int t = 0; t < T; ++t) {
    step_envs<float>(w, 0, w->n_envs, state, actions + 2 * A * t, nullptr, nullptr);
    if (traj) std::memcpy(traj + 6 * N * (t + 1), state, sizeof(float) * 6 * N);
  }
  return 0;
}

// Length of every joint at `state` evaluated in FP32 by the step's own
// expression. A rest length taken from the initial state is computed by each
// side in its own arithmetic (the joints reading of Sec. 3 used here): the
// FP32 evaluation takes these, so a spring that starts at rest exerts exactly
// zero force in it too.
int oracle_joint_lengths_fp32(const oracle_world* w, const float* state, double* out) {
  const int64_t N = w->env_offset[w->n_envs];
  const float *X = state, *Y = state + N, *TH = state + 4 * N;
  for (int q = 0; q < w->n_joints; ++q) {
    Pose<float> pa, pb;
    V2<float> Pa, Pb;
    joint_points(w, X, Y, TH, q, &pa, &pb, &Pa, &Pb);
    out[q] = (double)norm(sub(Pa, Pb));
  }
  return 0;
}

// Narrow phase of one pair (i, j) in index order, for the pin tests.
// pose = (x, y, theta); out = (d, nx, ny, pix, piy, pjx, pjy).
int oracle_pair(int si, const double* di, const double* pose_i, int sj, const double* dj,
                const double* pose_j, double* out) {
  Pose<double> a, b;
  a.c = {pose_i[0], pose_i[1]};
  a.cs = std::cos(pose_i[2]);
  a.sn = std::sin(pose_i[2]);
  b.c = {pose_j[0], pose_j[1]};
  b.cs = std::cos(pose_j[2]);
  b.sn = std::sin(pose_j[2]);
  Contact<double> r = narrow<double>(si, di[0], di[1], a, sj, dj[0], dj[1], b);
  out[0] = r.d;
  out[1] = r.n.x;
  out[2] = r.n.y;
  out[3] = r.pi.x;
  out[4] = r.pi.y;
  out[5] = r.pj.x;
  out[6] = r.pj.y;
  return 0;
}

// Signed core distance d and d_min of every pair slot (same slot order as
// the mask; NaN for pairs that are not eligible), from the FP64 narrow phase.
int oracle_pair_distances(const oracle_world* w, const double* state, double* d_out,
                          double* dmin_out) {
  const int N = w->env_offset[w->n_envs];
  const double *X = state, *Y = state + N, *TH = state + 4 * N;
  std::vector<int> js;
  int64_t slot = 0;
  for (int b = 0; b < w->n_envs; ++b) {
    const int o = w->env_offset[b], n = w->env_offset[b + 1] - o;
    js.clear();
    for (int q = 0; q < w->n_joints; ++q)
      if (w->joint_a[q] >= o && w->joint_a[q] < o + n) js.push_back(q);
    for (int a = 0; a < n; ++a) {
      for (int c = a + 1; c < n; ++c, ++slot) {
        int i = o + a, j = o + c;
        if (!pair_eligible(w, js.data(), (int)js.size(), i, j)) {
          d_out[slot] = NAN;
          dmin_out[slot] = NAN;
          continue;
        }
        Pose<double> pi = pose_of(X, Y, TH, i), pj = pose_of(X, Y, TH, j);
        Contact<double> r = narrow<double>(w->shape[i], w->dims[2 * i], w->dims[2 * i + 1], pi,
                                           w->shape[j], w->dims[2 * j], w->dims[2 * j + 1], pj);
        double ri = w->shape[i] == SPHERE ? w->dims[2 * i] : 0.0;
        double rj = w->shape[j] == SPHERE ? w->dims[2 * j] : 0.0;
        d_out[slot] = r.d;
        dmin_out[slot] = ri + rj + w->min_dist;
      }
    }
  }
  return 0;
}

// Textbook moment of inertia used when none is given.
double oracle_default_inertia(int shape, double m, double d0, double d1) {
  return default_inertia(shape, m, d0, d1);
}

}  // extern "C"
