// Physics side of the learned contact surrogate: pair features, training
// targets from the exact step, and a step whose contact forces come from the
// MLP, with the exact Eq. (2) force as fallback for deep contacts.
//
// Features of the pair (i, j), i < j in an environment, in the pair frame
// e = (c_i - c_j) / |c_i - c_j| (e = +x for coincident centres), phi = the
// angle of e (12 values of O(1) scale, invariant under rigid motions):
//   g / Lk clamped to [-16, 16] and g / L, with g = |c_i - c_j| - R_i - R_j
//   the gap of the bounding circles (R: sphere r, box half diagonal, line
//   L/2), at two scales, cos and sin of
//   (theta_i - phi), cos and sin of (theta_j - phi) (1 and 0 for a sphere,
//   which has no orientation), dims_i / L, dims_j / L, shape code of i and
//   of j (sphere 0, box 0.5, line 1);
// L = 0.1, Lk = 0.001 (the scale of the contact margin k, over which
// Eq. (2) bends at onset). Target: the Eq. (2) force on i in the pair frame
// (along e, along the left normal of e) divided by c * Lf, Lf = 0.02 (zero
// when the pair is not in contact). The centre distance is not a feature: it
// is the gap plus the two bounding radii, which the sizes give.
// A pair is a candidate for the network when neither entity is a segment and
// their bounding circles (sphere r, box half diagonal) come within `band` of
// each other. A segment has no thickness, so the fallback rule (penetration
// beyond half the smaller size) has no meaning for it: pairs with a segment
// always take the exact narrow phase. The surrogate step compacts the
// candidates' features into consecutive rows (atomics per wavefront; the row
// order varies between runs, the per-row network output does not) so that
// the network runs on candidates only.

#include "vmas_geom.h"
#include "vmas_internal.h"

namespace vmas {
namespace {

constexpr float FEAT_L = 0.1f;   // length scale of the features
constexpr float FINE_L = 0.001f; // length scale of the fine gap feature
constexpr float FORCE_L = 0.02f; // force scale c * FORCE_L of the targets

__device__ __forceinline__ float bound_radius(int shape, float d0, float d1) {
  if (shape == SPHERE) return d0;
  if (shape == BOX) return 0.5f * sqrtf(d0 * d0 + d1 * d1);
  return 0.5f * d0;
}

// local pair index q of an environment of n entities -> (a, c), a < c
__device__ __forceinline__ void pair_of(int q, int n, int* a, int* c) {
  int aa = 0, base = 0;
  while (q >= base + (n - 1 - aa)) {
    base += n - 1 - aa;
    ++aa;
  }
  *a = aa;
  *c = aa + 1 + (q - base);
}

// Network candidate decision of the pair (lo, hi), lo the lower local
// index; eligibility (both collidable, not excluded) is the caller's. The
// feature kernels and the surrogate step call it with the same arguments in
// the same order, so they decide alike to the bit.
__device__ __forceinline__ bool net_candidate(float xlo, float ylo, float rlo, int slo, float xhi,
                                              float yhi, float rhi, int shi, float band) {
  if (slo == LINE || shi == LINE) return false;
  const float dx = xlo - xhi, dy = ylo - yhi;
  const float reach = (rlo + rhi) + band;
  return dx * dx + dy * dy <= reach * reach;
}

// The 12 features of the pair (i = lo, j = hi) into f.
__device__ __forceinline__ void write_features(float* f, float xi, float yi, float ci, float sni,
                                               float d0i, float d1i, int si, float xj, float yj,
                                               float cj, float snj, float d0j, float d1j, int sj) {
  const float dx = xi - xj, dy = yi - yj;
  const float dist = sqrtf(dx * dx + dy * dy);
  const float ex = dist > 0.0f ? dx / dist : 1.0f, ey = dist > 0.0f ? dy / dist : 0.0f;
  const float Ri = bound_radius(si, d0i, d1i), Rj = bound_radius(sj, d0j, d1j);
  const float gap = dist - (Ri + Rj);
  f[0] = fminf(fmaxf(gap / FINE_L, -16.0f), 16.0f);
  f[1] = gap / FEAT_L;
  // cos and sin of (theta - phi); a sphere has no orientation: (1, 0)
  f[2] = si == SPHERE ? 1.0f : fmaf(ci, ex, sni * ey);
  f[3] = si == SPHERE ? 0.0f : fmaf(sni, ex, -ci * ey);
  f[4] = sj == SPHERE ? 1.0f : fmaf(cj, ex, snj * ey);
  f[5] = sj == SPHERE ? 0.0f : fmaf(snj, ex, -cj * ey);
  f[6] = d0i / FEAT_L;
  f[7] = d1i / FEAT_L;
  f[8] = d0j / FEAT_L;
  f[9] = d1j / FEAT_L;
  f[10] = 0.5f * (float)si;  // SPHERE 0, BOX 1, LINE 2
  f[11] = 0.5f * (float)sj;
}

struct FeatArgs {
  const float* state;
  const EntParam* ent;
  const int32_t* env_off;   // [E + 1]
  const int64_t* pair_off;  // [E]
  const int64_t* slots;     // [m] pair slots, or NULL: every slot (m = P)
  int64_t m;
  float band;
  float* feat;              // [m][12]
  float* target;            // [m][2] or NULL
  uint8_t* flags;           // [m]: 1 candidate, 2 exact contact
  int n_envs;
  WorldK w;
};

__device__ int env_of_slot(const int64_t* pair_off, int E, int64_t p) {
  int lo = 0, hi = E - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pair_off[mid] <= p) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void k_pair_features(FeatArgs a) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.m) return;
  const int64_t p = a.slots ? a.slots[r] : r;
  const int N = a.w.N;
  // the last environment whose first slot is <= p (environments with fewer
  // than two entities own no slot and share their successor's offset)
  const int e = env_of_slot(a.pair_off, a.n_envs, p);
  const int o = a.env_off[e], n = a.env_off[e + 1] - o;
  int la, lc;
  pair_of((int)(p - a.pair_off[e]), n, &la, &lc);
  const int i = o + la, j = o + lc;
  const EntParam pi = a.ent[i], pj = a.ent[j];
  const int si = pi.sf & 0xff, sj = pj.sf & 0xff, fi = (pi.sf >> 8) & 0xff, fj = (pj.sf >> 8) & 0xff;
  const float xi = a.state[i], yi = a.state[N + i], ti = a.state[4 * N + i];
  const float xj = a.state[j], yj = a.state[N + j], tj = a.state[4 * N + j];
  float ci = 1.0f, sni = 0.0f, cj = 1.0f, snj = 0.0f;
  if (si != SPHERE) sincosf(ti, &sni, &ci);
  if (sj != SPHERE) sincosf(tj, &snj, &cj);
  const float Ri = bound_radius(si, pi.d0, pi.d1), Rj = bound_radius(sj, pj.d0, pj.d1);
  const bool eligible = (fi & COLLIDABLE) && (fj & COLLIDABLE) &&
                        ((fi | fj) & (MOVABLE | ROTATABLE)) && !excluded(pi.excl, lc) &&
                        !excluded(pj.excl, la);
  const bool cand = eligible && net_candidate(xi, yi, Ri, si, xj, yj, Rj, sj, a.band);
  write_features(a.feat + r * 12, xi, yi, ci, sni, pi.d0, pi.d1, si, xj, yj, cj, snj, pj.d0, pj.d1,
                 sj);
  const float dxe = xi - xj, dye = yi - yj;
  const float dist = sqrtf(dxe * dxe + dye * dye);
  const V2T<float> ex = dist > 0.0f ? V2T<float>{dxe / dist, dye / dist} : V2T<float>{1.0f, 0.0f};
  uint8_t fl = cand ? 1 : 0;
  float tx = 0.0f, ty = 0.0f;
  if (cand) {
    GeoT<float> gi;
    gi.c = {xi, yi};
    gi.cs = ci;
    gi.sn = sni;
    gi.d0 = pi.d0;
    gi.d1 = pi.d1;
    gi.shape = si;
    const float4 P = make_float4(xj, yj, cj, snj);
    const float4 S = make_float4(pj.d0, pj.d1, pj.rho, __int_as_float(pj.sf));
    float fx = 0.0f, fy = 0.0f, tq = 0.0f;
    if (pair_force<false>(gi, pi.rho, 0, P, S, 1, a.w, fx, fy, tq)) {
      fl |= 2;
      const float inv = 1.0f / (a.w.ck * a.w.inv_k * FORCE_L);  // 1 / (c Lf)
      tx = fmaf(fx, ex.x, fy * ex.y) * inv;         // along e
      ty = fmaf(fy, ex.x, -fx * ex.y) * inv;        // along the left normal of e
    }
  }
  a.flags[r] = fl;
  if (a.target) {
    a.target[r * 2] = tx;
    a.target[r * 2 + 1] = ty;
  }
}

struct CandArgs {
  StepArgs s;          // plan and state
  float band;
  float* feat;         // [P][12] candidate rows
  int32_t* slot_of;    // [rows] pair slot of each candidate row
  int32_t* count;      // number of candidate rows (starts at 0)
};

// The parameters of entity e: from its 16-byte SphRec where that describes
// it fully (a sphere-only batch with sph_only), else the 48-byte EntParam.
template <bool SPH>
__device__ __forceinline__ EntParam ent_of(const StepArgs& a, int e) {
  if (SPH && a.sph_only) {
    const SphRec q = a.sph[e];
    EntParam p{};
    p.d0 = q.rho;
    p.rho = q.rho;
    p.inv_m = q.inv_m;
    p.vmax = q.vmax;
    p.sf = q.sf;
    p.inv_I = 1.0f;  // never scales a nonzero torque here: 0 x 1/I = +0 either way
    p.excl = -1;
    return p;
  }
  return a.ent[e];
}

// Candidate features for the surrogate step, in consecutive rows: lane per
// entity that can move or rotate, poses staged in LDS as in the exact step.
// A pair is written by its lower entity, or by the higher one when the lower
// one has no lane. Rows: each lane counts its candidates, the workgroup
// scans the counts in LDS and takes its block of rows with one atomic, then
// every lane writes its candidates in partner order.
template <int MAXB, bool SPH>
__global__ void __launch_bounds__(MAXB) k_cand_features(CandArgs ca) {
  const StepArgs& a = ca.s;
  extern __shared__ float4 lds[];
  __shared__ int scan[MAXB / 64];  // wavefront totals
  __shared__ int gbase;
  const int E = a.max_stage;
  float4* pose = lds;
  float4* stat = lds + E;
  float* brad = reinterpret_cast<float*>(lds + 2 * E);  // bounding radius of each slot
  const int g = blockIdx.x, l = threadIdx.x, B = blockDim.x;
  const int N = a.w.N;
  const int s0 = a.stage_off[g], ns = a.stage_off[g + 1] - s0;
  for (int s = l; s < ns; s += B) {
    const int e = a.stage[s0 + s];
    const EntParam p = ent_of<SPH>(a, e);
    float cs = 1.0f, sn = 0.0f;
    if (uses_rotation(p.sf)) sincosf(a.state[4 * N + e], &sn, &cs);
    pose[s] = make_float4(a.state[e], a.state[N + e], cs, sn);
    stat[s] = make_float4(p.d0, p.d1, p.rho, __int_as_float(p.sf));
    brad[s] = bound_radius(p.sf & 0xff, p.d0, p.d1);
  }
  const LaneRec r = a.lanes[(size_t)g * B + l];
  __syncthreads();
  EntParam p{};
  p.excl = -1;
  if (r.ent >= 0) p = ent_of<SPH>(a, r.ent);
  const int shape = p.sf & 0xff;
  const bool live = r.ent >= 0 && ((p.sf >> 8) & COLLIDABLE);
  const float4 me = live ? pose[r.slot] : make_float4(0.0f, 0.0f, 1.0f, 0.0f);
  const float rme = bound_radius(shape, p.d0, p.d1);
  const int myloc = r.slot - r.lo, nloc = r.hi - r.lo;
  // whether partner slot q is a candidate written by this lane
  auto mine = [&](int q) {
    const int b = q - r.lo;
    if (b == myloc) return false;
    const float4 S = stat[q];
    const int so = __float_as_int(S.w) & 0xff, of = (__float_as_int(S.w) >> 8) & 0xff;
    if (!(myloc < b || !(of & (MOVABLE | ROTATABLE)))) return false;
    if (!(of & COLLIDABLE) || (p.excl != -1 && excluded(p.excl, b))) return false;
    const float4 P = pose[q];
    const float ro = brad[q];
    return myloc < b ? net_candidate(me.x, me.y, rme, shape, P.x, P.y, ro, so, ca.band)
                     : net_candidate(P.x, P.y, ro, so, me.x, me.y, rme, shape, ca.band);
  };
  // environments of at most 32 entities: one pass into a bit mask (bit b:
  // local partner b); larger ones test every partner again below
  const bool small = nloc <= 32;
  uint32_t cm = 0;
  int cnt = 0;
  if (live) {
    if (small) {
      for (int q = r.lo; q < r.hi; ++q) cm |= (mine(q) ? 1u : 0u) << (q - r.lo);
      cnt = __popc(cm);
    } else {
      for (int q = r.lo; q < r.hi; ++q) cnt += mine(q) ? 1 : 0;
    }
  }
  // exclusive prefix of the lane counts over the workgroup: within each
  // wavefront by shuffles, then the wavefront totals
  const int wl = l & 63, wv = l >> 6;
  int inc = cnt;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(inc, off, 64);
    if (wl >= off) inc += v;
  }
  if (wl == 63) scan[wv] = inc;  // wavefront totals
  __syncthreads();
  if (l == 0) {
    int total = 0;
    for (int k = 0; k < (B + 63) / 64; ++k) {
      const int t = scan[k];
      scan[k] = total;  // exclusive prefix of the wavefront totals
      total += t;
    }
    gbase = total > 0 ? atomicAdd(ca.count, total) : 0;
  }
  __syncthreads();
  if (!live || cnt == 0) return;
  int row = gbase + scan[wv] + inc - cnt;
  const int64_t poff = a.pair_off[r.env];
  for (int q = r.lo; q < r.hi; ++q) {
    if (small ? !((cm >> (q - r.lo)) & 1u) : !mine(q)) continue;
    const int b = q - r.lo;
    const float4 P = pose[q];
    const float4 S = stat[q];
    const int so = __float_as_int(S.w) & 0xff;
    const int ia = min(myloc, b), ib = max(myloc, b);
    const int64_t slot = poff + (int64_t)ia * nloc - (int64_t)ia * (ia + 1) / 2 + (ib - ia - 1);
    ca.slot_of[row] = (int32_t)slot;
    float* f = ca.feat + (int64_t)row * 12;
    if (myloc < b)
      write_features(f, me.x, me.y, me.z, me.w, p.d0, p.d1, shape, P.x, P.y, P.z, P.w, S.x, S.y, so);
    else
      write_features(f, P.x, P.y, P.z, P.w, S.x, S.y, so, me.x, me.y, me.z, me.w, p.d0, p.d1, shape);
    ++row;
  }
}

struct SurArgs {
  StepArgs s;             // plan, state, actions (T = 1), forces
  // [P][2] the network's output of each candidate pair at its pair slot
  // (force on lo in the pair frame / (c Lf)); read for candidates only
  const float* yhat;
  float band;             // candidate reach, as given to the feature kernel
  float fallback_frac;    // exact fallback when predicted penetration > frac * r
  int32_t* n_fallback;    // device counter, or NULL
};

// One step with surrogate contact forces (lane per entity that can move or
// rotate, poses staged in LDS as in the exact step). The network's force f is
// read through Eq. (2): where its penetration k log(expm1(|f| / (c k))) is
// beyond fallback_frac times the smaller half size, the exact pair force is
// used instead; otherwise f is replaced by the nearest force Eq. (2) can
// produce, 0 when |f| < F0 / 2 and at least F0 = c k ln 2 (the force at zero
// penetration) along f otherwise.
// SPH: every collidable or moving entity of the batch is a sphere (the
// sphere narrow phase alone is compiled in; the same arithmetic).
template <bool SPH>
__global__ void __launch_bounds__(256) k_step_surrogate(SurArgs sa) {
  const StepArgs& a = sa.s;
  extern __shared__ float4 lds[];
  const int E = a.max_stage;
  float4* pose = lds;
  float4* stat = lds + E;
  float* brad = reinterpret_cast<float*>(lds + 2 * E);  // bounding radius of each slot
  const int g = blockIdx.x, l = threadIdx.x, B = blockDim.x;
  const int N = a.w.N;
  const int s0 = a.stage_off[g], ns = a.stage_off[g + 1] - s0;
  for (int s = l; s < ns; s += B) {
    const int e = a.stage[s0 + s];
    const EntParam p = ent_of<SPH>(a, e);
    float cs = 1.0f, sn = 0.0f;
    if (uses_rotation(p.sf)) sincosf(a.state[4 * N + e], &sn, &cs);
    pose[s] = make_float4(a.state[e], a.state[N + e], cs, sn);
    stat[s] = make_float4(p.d0, p.d1, p.rho, __int_as_float(p.sf));
    brad[s] = bound_radius(p.sf & 0xff, p.d0, p.d1);
  }
  const LaneRec r = a.lanes[(size_t)g * B + l];
  const bool act = r.ent >= 0;
  __syncthreads();
  if (!act) return;
  const WorldK w = a.w;
  const int e = r.ent;
  float x = a.state[e], y = a.state[N + e], vx = a.state[2 * N + e], vy = a.state[3 * N + e];
  float th = a.state[4 * N + e], om = a.state[5 * N + e];
  const EntParam p = ent_of<SPH>(a, e);
  const int shape = SPH ? SPHERE : p.sf & 0xff, fl = (p.sf >> 8) & 0xff;
  float cs = 1.0f, sn = 0.0f;
  if (uses_rotation(p.sf)) sincosf(th, &sn, &cs);
  float fx = p.mgx, fy = p.mgy, tq = 0.0f;
  if (r.agent >= 0) {
    fx += a.actions[2 * (size_t)r.agent];
    fy += a.actions[2 * (size_t)r.agent + 1];
  }
  const int myloc = r.slot - r.lo, nloc = r.hi - r.lo;
  const float FS = w.ck * w.inv_k * FORCE_L;  // c Lf
  const float rme = bound_radius(shape, p.d0, p.d1);
  const float F0 = w.ck * 0.69314718f;  // Eq. (2) at zero penetration: c k ln 2
  int fallbacks = 0;
  if (fl & COLLIDABLE) {
    GeoT<float> self;
    self.c = {x, y};
    self.cs = cs;
    self.sn = sn;
    self.d0 = p.d0;
    self.d1 = p.d1;
    self.shape = shape;
    // partners class by class (spheres, boxes, segments), each in partner
    // order: the accumulation order of the exact step; classes absent from
    // the environment are skipped
    unsigned present = SPH ? 1u << SPHERE : 0u;
    if (!SPH)
      for (int q = r.lo; q < r.hi; ++q) present |= 1u << (__float_as_int(stat[q].w) & 0xff);
    for (int cls = 0; cls < (SPH ? 1 : 3); ++cls) {
      if (!(present & (1u << cls))) continue;
      for (int q = r.lo; q < r.hi; ++q) {
        if (q == r.slot) continue;
        const int b = q - r.lo;
        const float4 S = stat[q];
        const int so = SPH ? SPHERE : __float_as_int(S.w) & 0xff, of = (__float_as_int(S.w) >> 8) & 0xff;
        if (so != cls) continue;
        const float4 P = pose[q];
        if (!(of & COLLIDABLE) || (p.excl != -1 && excluded(p.excl, b))) continue;
        if (!SPH && (shape == LINE || so == LINE)) {
          // segments: exact narrow phase (same eligibility as the exact step)
          pair_force<false>(self, p.rho, myloc, P, S, b, w, fx, fy, tq);
          continue;
        }
        // the candidate decision of the feature kernel, repeated bit for bit
        const float ro = brad[q];
        const bool cand = myloc < b ? net_candidate(x, y, rme, shape, P.x, P.y, ro, so, sa.band)
                                    : net_candidate(P.x, P.y, ro, so, x, y, rme, shape, sa.band);
        if (!cand) continue;
        const int ia = min(myloc, b), ib = max(myloc, b);
        const int64_t slot = a.pair_off[r.env] + (int64_t)ia * nloc - (int64_t)ia * (ia + 1) / 2 + (ib - ia - 1);
        // surrogate force on lo, in the pair frame -> world
        const float hx = sa.yhat[2 * slot] * FS, hy = sa.yhat[2 * slot + 1] * FS;
        const float sgn = myloc < b ? 1.0f : -1.0f;  // e points from hi to lo
        const float ddx = sgn * (x - P.x), ddy = sgn * (y - P.y);
        const float dd = sqrtf(fmaf(ddx, ddx, ddy * ddy));
        const V2T<float> ex = dd > 0.0f ? V2T<float>{ddx / dd, ddy / dd} : V2T<float>{1.0f, 0.0f};
        const V2T<float> flo = {fmaf(hx, ex.x, -hy * ex.y), fmaf(hx, ex.y, hy * ex.x)};
        // predicted penetration from the inverse of Eq. (2): k log(expm1(|f| / (c k)))
        const float mag = sqrtf(flo.x * flo.x + flo.y * flo.y);
        const float pen = mag > 0.0f ? logf(expm1f(mag / w.ck)) / w.inv_k : -INFINITY;
        const float rr = fminf(shape == SPHERE ? p.d0 : 0.5f * fminf(p.d0, shape == BOX ? p.d1 : p.d0),
                               so == SPHERE ? S.x : 0.5f * fminf(S.x, so == BOX ? S.y : S.x));
        if (pen > sa.fallback_frac * rr) {
          ++fallbacks;
          pair_force<SPH>(self, p.rho, myloc, P, S, b, w, fx, fy, tq);
          continue;
        }
        // nearest force Eq. (2) can produce: 0, or at least the onset force
        // F0 = c k ln 2 (zero penetration), along the predicted direction
        if (!(mag >= 0.5f * F0)) continue;
        const float sc = mag < F0 ? F0 / mag : 1.0f;
        if (myloc < b) {
          fx = fmaf(sc, flo.x, fx);
          fy = fmaf(sc, flo.y, fy);
        } else {
          fx = fmaf(-sc, flo.x, fx);
          fy = fmaf(-sc, flo.y, fy);
        }
      }
    }
  }
  // joint springs are exact (they are not contacts)
  for (int jj = a.joff[e]; jj < a.joff[e + 1]; ++jj) {
    const JointK J = a.joints[a.jlist[jj]];
    const bool is_a = J.a == e;
    const float4 P = pose[r.lo + ((is_a ? J.b : J.a) - r.first)];
    V2T<float> f;
    float ts, to;
    if (joint_eval<float>(V2T<float>{x, y}, cs, sn, V2T<float>{P.x, P.y}, P.z, P.w, is_a, J,
                          w.joint_k, &f, &ts, &to)) {
      fx += f.x;
      fy += f.y;
      tq += ts;
    }
  }
  if (a.forces) {
    a.forces[e] = fx;
    a.forces[N + e] = fy;
    a.forces[2 * N + e] = tq;
  }
  if (fl & MOVABLE) {
    vx = fmaf(fx * p.inv_m, w.dt, w.damp * vx);
    vy = fmaf(fy * p.inv_m, w.dt, w.damp * vy);
    if (p.vmax > 0.0f) {
      const float sp = sqrtf(fmaf(vx, vx, vy * vy));
      if (sp > p.vmax) {
        vx *= p.vmax / sp;
        vy *= p.vmax / sp;
      }
    }
    x = fmaf(vx, w.dt, x);
    y = fmaf(vy, w.dt, y);
  }
  if (fl & ROTATABLE) {
    om = fmaf(tq * p.inv_I, w.dt, w.damp * om);
    th = fmaf(om, w.dt, th);
  }
  // all lanes have read the state they need before anyone writes (barrier
  // above); each lane writes only its own entity
  a.state[e] = x;
  a.state[N + e] = y;
  a.state[2 * N + e] = vx;
  a.state[3 * N + e] = vy;
  a.state[4 * N + e] = th;
  a.state[5 * N + e] = om;
  if (sa.n_fallback && fallbacks) atomicAdd(sa.n_fallback, fallbacks);
}

}  // namespace

hipError_t launch_pair_features(const float* state, const EntParam* ent, const int32_t* env_off,
                                const int64_t* pair_off, const int64_t* slots, int64_t m,
                                float band, float* feat, float* target, uint8_t* flags,
                                int n_envs, const WorldK& w, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  FeatArgs a{state, ent, env_off, pair_off, slots, m, band, feat, target, flags, n_envs, w};
  hipLaunchKernelGGL(k_pair_features, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_candidate_features(const StepArgs& a, int groups, int block, float band,
                                     float* feat, int32_t* slot_of, int32_t* count,
                                     bool spheres_only, hipStream_t s) {
  if (groups <= 0) return hipSuccess;
  CandArgs ca{a, band, feat, slot_of, count};
  const size_t shm = (size_t)a.max_stage * (2 * sizeof(float4) + sizeof(float));
  if (block > 256) {
    if (spheres_only)
      hipLaunchKernelGGL((k_cand_features<1024, true>), dim3(groups), dim3(block), shm, s, ca);
    else
      hipLaunchKernelGGL((k_cand_features<1024, false>), dim3(groups), dim3(block), shm, s, ca);
  } else {
    if (spheres_only)
      hipLaunchKernelGGL((k_cand_features<256, true>), dim3(groups), dim3(block), shm, s, ca);
    else
      hipLaunchKernelGGL((k_cand_features<256, false>), dim3(groups), dim3(block), shm, s, ca);
  }
  return hipGetLastError();
}

hipError_t launch_step_surrogate(const StepArgs& a, const float* yhat,
                                 float band, float frac, int32_t* n_fallback, int groups,
                                 int block, bool spheres_only, hipStream_t s) {
  SurArgs sa{a, yhat, band, frac, n_fallback};
  const size_t shm = (size_t)a.max_stage * (2 * sizeof(float4) + sizeof(float));
  if (spheres_only)
    hipLaunchKernelGGL(k_step_surrogate<true>, dim3(groups), dim3(block), shm, s, sa);
  else
    hipLaunchKernelGGL(k_step_surrogate<false>, dim3(groups), dim3(block), shm, s, sa);
  return hipGetLastError();
}

}  // namespace vmas
