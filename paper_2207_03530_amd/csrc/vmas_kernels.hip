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
// Poses are double-buffered in LDS: one barrier per step. The pair-queue
// variant (PQ) evaluates every pair that involves a box or a segment once:
// the lane that owns the pair (the lower index, or the one with a lane when
// the other has none) appends it to a per-class queue in LDS, all lanes of
// the group then work through the queues class by class (one narrow-phase
// routine per wavefront most of the time), and each entity adds its side of
// the results in the same class and partner order as the plain variant, bit
// for bit. A pair that finds its class queue full is evaluated by both of its
// lanes, as in the plain variant. Sphere batches have
// their own kernels (k_rollout_sph: centres only in LDS, hoisted contact
// distances; k_rollout_quad: environments of at most 4 movers on one lane
// quad, centres exchanged by DPP, no LDS).
//
// Arithmetic is FP32 and compiled without implicit contraction; every fused
// multiply-add is written out, so different kernels and plans agree bit for
// bit.

#include <type_traits>

#include "vmas_geom.h"
#include "vmas_internal.h"

namespace vmas {
namespace {

using V2 = V2T<float>;
using Geo = GeoT<float>;
using Hit = HitT<float>;

// SplitMix64 (Steele, Lea, Flood 2014) finaliser.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// Draw idx of the counter-based stream of a key: the finaliser of key +
// (idx + 1) golden, its top 24 bits mapped to [-1, 1).
constexpr uint64_t GOLDEN = 0x9E3779B97F4A7C15ull;
__device__ __forceinline__ float sym_of(uint64_t z) {
  const uint64_t m = mix64(z);
  const int k = (int)(m >> 40);
  return (float)(k - (1 << 23)) * (1.0f / 8388608.0f);
}
// The two action components of action row `row` at step t0 + t are draws
// 2 ((t0 + t) A + row) and that + 1, so their counters key + (idx + 1)
// golden are ctr0(row) + t step_ctr and that + golden (mod 2^64): a draw
// costs an addition instead of a 64-bit product.
__device__ __forceinline__ uint64_t ctr0(uint64_t key, int64_t t0, int64_t A, int64_t row) {
  return key + (((uint64_t)t0 * (uint64_t)A + (uint64_t)row) * 2ull + 1ull) * GOLDEN;
}
__device__ __forceinline__ uint64_t step_ctr(int64_t A) { return 2ull * (uint64_t)A * GOLDEN; }
__device__ __forceinline__ float2 draw_action(uint64_t z) {
  return make_float2(sym_of(z), sym_of(z + GOLDEN));
}

// Radius of the circle about an entity's centre that holds the whole shape
// (sphere r, box half diagonal, segment half length).
__device__ __forceinline__ float bounding_radius(int shape, float d0, float d1) {
  if (shape == SPHERE) return d0;
  if (shape == BOX) return 0.5f * sqrtf(d0 * d0 + d1 * d1);
  return 0.5f * d0;
}

// Pair classes of the queue (pairs with at least one box or segment).
constexpr int PQ_SB = 0, PQ_SL = 1, PQ_BB = 2, PQ_BL = 3, PQ_LL = 4, PQ_CLASSES = 5;
__device__ __forceinline__ int pair_class(int sa, int sb) {
  const int lo = min(sa, sb), hi = max(sa, sb);  // SPHERE < BOX < LINE
  if (lo == SPHERE) return hi == BOX ? PQ_SB : PQ_SL;
  if (lo == BOX) return hi == BOX ? PQ_BB : PQ_BL;
  return PQ_LL;
}

// narrow(lo, hi) for a pair of class C: the same routines in the same order,
// with the shape pair fixed at compile time up to which side is the sphere.
template <int C>
__device__ __forceinline__ Hit narrow_class(const Geo& lo, const Geo& hi, float cutoff) {
  if constexpr (C == PQ_SB || C == PQ_SL) {
    if (lo.shape == SPHERE) return C == PQ_SL ? sphere_line(lo.c, hi) : sphere_box(lo.c, hi);
    const Hit r = C == PQ_SL ? sphere_line(hi.c, lo) : sphere_box(hi.c, lo);
    Hit o;
    o.d = r.d;
    o.n = vneg(r.n);
    o.plo = r.phi;
    o.phi = r.plo;
    return o;
  } else if constexpr (C == PQ_LL) {
    return line_line(lo, hi, cutoff);
  } else if constexpr (C == PQ_BB) {
    return poly_poly<4, 4>(lo, hi, cutoff);
  } else {
    return lo.shape == BOX ? poly_poly<4, 2>(lo, hi, cutoff) : poly_poly<2, 4>(lo, hi, cutoff);
  }
}

__device__ __forceinline__ Geo staged_geo(const float4 P, const float4 S) {
  Geo g;
  g.c = V2{P.x, P.y};
  g.cs = P.z;
  g.sn = P.w;
  g.d0 = S.x;
  g.d1 = S.y;
  g.shape = __float_as_int(S.w) & 0xff;
  return g;
}

// One queued pair: contact test and force of Eq. (2) with the torques of
// Eq. (3) for both sides, as pair_force computes them for each side (the
// higher index receives the negated force). res = (f_lo, tq_lo, tq_hi).
template <int C>
__device__ __forceinline__ bool queued_pair(const float4* cur, const float4* stat, int qa, int qb,
                                            const WorldK& w, float4* res) {
  const float4 Sa = stat[qa], Sb = stat[qb];
  const Geo lo = staged_geo(cur[qa], Sa), hi = staged_geo(cur[qb], Sb);
  const float dmin = (Sa.z + Sb.z) + w.min_dist;
  const Hit h = narrow_class<C>(lo, hi, contact_cutoff(lo, hi, dmin));
  if (!(h.d <= dmin)) return false;
  const float F = contact_mag(dmin, h.d, w);
  const V2 flo = V2{F * h.n.x, F * h.n.y};
  const V2 fhi = V2{-F * h.n.x, -F * h.n.y};
  *res = make_float4(flo.x, flo.y, vcross(vsub(h.plo, lo.c), flo), vcross(vsub(h.phi, hi.c), fhi));
  return true;
}

// Persistent rollout: T steps of every environment of the group.// Persistent rollout: T steps of every environment of the group. A lane's
// contacts are accumulated partner class by partner class (spheres, boxes,
// segments), each class in partner order.
// Broad phase: a partner whose bounding circle stays farther than d_min plus
// a safety margin (1e-4 + 1e-5 (|x| + |y|), far above the FP32 error of the
// narrow-phase distance) from the lane's own cannot be in contact, so only
// the other partners run the narrow phase -- in partner order, with the
// same arithmetic, hence with the results of testing every partner.
// PQ: every environment has at most 32 entities; a.pq_cap[c] is the queue
// capacity of pair class c, a.pq_cap[PQ_CLASSES] their sum.
template <int MAXB, bool PQ>
__global__ void __launch_bounds__(MAXB) k_rollout(StepArgs a) {
  extern __shared__ float4 lds[];
  const int E = a.max_stage;
  float4* buf0 = lds;
  float4* buf1 = lds + E;
  float4* stat = lds + 2 * E;
  const int QT = PQ ? a.pq_cap[PQ_CLASSES] : 0;
  float4* qres = lds + 3 * E;                                // [QT] queued pair results
  float* brad = reinterpret_cast<float*>(lds + 3 * E + QT);  // bounding radius, NaN: not collidable
  uint32_t* hitw = reinterpret_cast<uint32_t*>(brad + E);    // [E] queued partners in contact
  uint32_t* selfw = hitw + E;                                // [E] partners the lane evaluates itself
  int* qcnt = reinterpret_cast<int*>(selfw + E);             // [8] queue fill per class
  int* qcap = qcnt + 8;                                      // [8] capacity per class
  int* qbase = qcnt + 16;                                    // [8] first entry of each class
  uint32_t* qent = reinterpret_cast<uint32_t*>(qcnt + 24);   // [QT] slot_lo | slot_hi << 11 | lo << 22 | hi << 27
  uint32_t* sphw = qent + QT;                                // [E] sphere partners to evaluate
  uint32_t* pairs = sphw + E;                                // [pq_max_pairs] the group's pairs
  uint16_t* qmap = reinterpret_cast<uint16_t*>(pairs + (PQ ? a.pq_max_pairs : 0));  // [E][32] queue entry of (entity, partner)
  const int g = blockIdx.x, l = threadIdx.x, B = blockDim.x;
  const int N = a.w.N;
  const int s0 = a.stage_off[g], ns = a.stage_off[g + 1] - s0;
  for (int s = l; s < ns; s += B) {
    const int e = a.stage[s0 + s];
    const EntParam p = a.ent[e];
    float cs = 1.0f, sn = 0.0f;
    if (uses_rotation(p.sf)) sincosf(a.state[4 * N + e], &sn, &cs);
    const float4 P = make_float4(a.state[e], a.state[N + e], cs, sn);
    buf0[s] = P;
    buf1[s] = P;
    stat[s] = make_float4(p.d0, p.d1, p.rho, __int_as_float(p.sf));
    brad[s] = ((p.sf >> 8) & COLLIDABLE) ? bounding_radius(p.sf & 0xff, p.d0, p.d1)
                                         : __int_as_float(0x7fc00000);
  }
  const int np0 = PQ ? a.pq_pair_off[g] : 0, npairs = PQ ? a.pq_pair_off[g + 1] - np0 : 0;
  for (int k = l; k < npairs; k += B) pairs[k] = a.pq_pairs[np0 + k];
  if (PQ && l == 0) {
    int acc = 0;
#pragma unroll
    for (int c = 0; c < PQ_CLASSES; ++c) {
      qcap[c] = a.pq_cap[c];
      qbase[c] = acc;
      acc += a.pq_cap[c];
    }
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
  const uint64_t z0 = ctr0(a.key, a.t0, w.A, agent ? r.agent : 0), zs = step_ctr(w.A);
  if (agent && a.T > 0) {
    if (a.actions) an = *reinterpret_cast<const float2*>(a.actions + 2 * (size_t)r.agent);
    else an = draw_action(z0);
  }
  __syncthreads();
  // shape classes of the first 32 partners (static for the whole rollout)
  uint32_t cls_sph0 = 0, cls_box0 = 0;
  for (int u = 0; u < min(32, nloc); ++u) {
    const int so = __float_as_int(stat[r.lo + u].w) & 0xff;
    cls_sph0 |= (so == SPHERE ? 1u : 0u) << u;
    cls_box0 |= (so == BOX ? 1u : 0u) << u;
  }
  // The lane's pairs of the broad phase (pair l + i B) and their summed
  // bounding radii never change: with at most PPL per lane they are kept in
  // registers (padding reads slot 0, its bit is masked off), so a step reads
  // only the two poses of each pair, all pairs of a block of 4 at once.
  constexpr int PPL = 16;
  const int npl = PQ ? (npairs + B - 1) / B : 0;  // the same for every lane
  const bool preg = PQ && npl <= PPL;
  uint32_t pw[PPL];
  float prad[PPL];
  uint32_t pvalid = 0;
#pragma unroll
  for (int i = 0; i < PPL; ++i) {
    const int k = l + i * B;
    const bool ok = preg && k < npairs;
    pw[i] = ok ? pairs[k] : 0u;
    prad[i] = ok ? brad[pw[i] & 0x7ff] + brad[(pw[i] >> 11) & 0x7ff] : 0.0f;
    pvalid |= (ok ? 1u : 0u) << i;
  }
  // Class of each of the lane's pairs (static): bit i of pm[c] is set when
  // pair l + i B belongs to queue class c, of pm_ss when it joins two
  // spheres.
  uint32_t pm[PQ_CLASSES] = {0u, 0u, 0u, 0u, 0u}, pm_ss = 0u;
  if (PQ) {
    for (int k = l, i = 0; k < npairs; k += B, ++i) {
      const uint32_t pe = pairs[k];
      const int sa = __float_as_int(stat[pe & 0x7ff].w) & 0xff;
      const int sb = __float_as_int(stat[(pe >> 11) & 0x7ff].w) & 0xff;
      const uint32_t bit = 1u << i;
      const int c = pair_class(sa, sb);
      const bool ss = sa == SPHERE && sb == SPHERE;
      pm_ss |= ss ? bit : 0u;
#pragma unroll
      for (int cc = 0; cc < PQ_CLASSES; ++cc) pm[cc] |= (!ss && c == cc) ? bit : 0u;
    }
  }
  // The lane's first two joints (static) in registers; further ones are
  // read from memory each step.
  int nj = 0, jslot[2] = {0, 0};
  bool jis_a[2] = {false, false};
  JointK jr[2] = {};
  const int j0 = act ? a.joff[r.ent] : 0;
  if (act) nj = a.joff[r.ent + 1] - j0;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    if (q < nj) {
      jr[q] = a.joints[a.jlist[j0 + q]];
      jis_a[q] = jr[q].a == r.ent;
      jslot[q] = r.lo + ((jis_a[q] ? jr[q].b : jr[q].a) - r.first);
    }
  }
  for (int t = 0; t < a.T; ++t) {
    float4* cur = (t & 1) ? buf1 : buf0;
    float cs = 1.0f, sn = 0.0f;
    if (act && uses_rotation(p.sf)) sincosf(th, &sn, &cs);
    if (PQ) {
      // A lane clears only its own words (another wavefront may still be
      // reading its own ones from the previous step); the words of slots
      // without a lane are written but never read.
      if (act) {
        if (t > 0) cur[r.slot] = make_float4(x, y, cs, sn);
        hitw[r.slot] = 0u;
        selfw[r.slot] = 0u;
        sphw[r.slot] = 0u;
      }
      if (l < 8) qcnt[l] = 0;
      __syncthreads();
    } else if (t > 0) {
      if (act) cur[r.slot] = make_float4(x, y, cs, sn);
      __syncthreads();
    }
    float fx = an.x + p.mgx, fy = an.y + p.mgy, tq = 0.0f;
    if (agent && t + 1 < a.T) {
      if (a.actions)
        an = *reinterpret_cast<const float2*>(a.actions + 2 * ((size_t)(t + 1) * w.A + r.agent));
      else
        an = draw_action(z0 + (uint64_t)(t + 1) * zs);
    }
    const bool last = t == a.T - 1;
    uint8_t* mk = (last && a.mask) ? a.mask : nullptr;
    if (PQ) {
      // Broad phase over the group's pairs, spread evenly over its lanes
      // (margin from the larger coordinates of the two): sphere pairs are
      // marked for both of their lanes, the others go to their class queue.
      // Tests first (no LDS atomic waits in between), then the candidates.
      uint32_t pc = 0;  // bit i: pair l + i B passed
      auto bp_test = [&](float2 Pa, float2 Pb, float rsum) {
        const float dx = Pa.x - Pb.x, dy = Pa.y - Pb.y;
        const float reach =
            w.min_dist + 1e-4f + 1e-5f * fmaxf(fabsf(Pa.x) + fabsf(Pa.y), fabsf(Pb.x) + fabsf(Pb.y));
        const float lim = rsum + reach;
        return dx * dx + dy * dy <= lim * lim;
      };
      if (preg) {
#pragma unroll
        for (int i0 = 0; i0 < PPL; i0 += 4) {
          if (i0 < npl) {
            float2 A[4], Bp[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              A[j] = *reinterpret_cast<const float2*>(cur + (pw[i0 + j] & 0x7ff));
              Bp[j] = *reinterpret_cast<const float2*>(cur + ((pw[i0 + j] >> 11) & 0x7ff));
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) pc = shift_in(pc, bp_test(A[j], Bp[j], prad[i0 + j]));
          }
        }
        pc = shifted_bits(pc, min(PPL, (npl + 3) & ~3)) & pvalid;
      } else {
        int i = 0;
        for (int k = l; k < npairs; k += B, ++i) {
          const uint32_t pe = pairs[k];
          const int qa = pe & 0x7ff, qb = (pe >> 11) & 0x7ff;
          const float4 Pa = cur[qa], Pb = cur[qb];
          pc = shift_in(pc, bp_test(make_float2(Pa.x, Pa.y), make_float2(Pb.x, Pb.y), brad[qa] + brad[qb]));
        }
        pc = shifted_bits(pc, i);
      }
      // Sphere pairs: a bit for each of the two lanes.
      for (uint32_t m = pc & pm_ss; m; m &= m - 1) {
        const uint32_t pe = pairs[l + __builtin_ctz(m) * B];
        atomicOr(&sphw[pe & 0x7ff], 1u << (pe >> 27));
        atomicOr(&sphw[(pe >> 11) & 0x7ff], 1u << ((pe >> 22) & 31));
      }
      // Other pairs, in bit order: the class comes from the lane's static
      // masks, so the reservation does not wait for the pair's word.
      for (uint32_t m = pc & ~pm_ss; m; m &= m - 1) {
        const uint32_t bit = m & (0u - m);
        const uint32_t pe = pairs[l + __builtin_ctz(m) * B];
        int c = 0;
#pragma unroll
        for (int cc = 1; cc < PQ_CLASSES; ++cc) c = (pm[cc] & bit) ? cc : c;
        const int kq = atomicAdd(&qcnt[c], 1);
        const int qa = pe & 0x7ff, qb = (pe >> 11) & 0x7ff;
        const int la = (pe >> 22) & 31, lb = pe >> 27;
        if (kq < qcap[c]) {
          const int e = qbase[c] + kq;
          qent[e] = pe;
          qmap[qa * 32 + lb] = (uint16_t)e;
          qmap[qb * 32 + la] = (uint16_t)e;
        } else {
          atomicOr(&selfw[qa], 1u << lb);
          atomicOr(&selfw[qb], 1u << la);
        }
      }
      lds_barrier();
      // Every lane of the group works through the queues, class by class;
      // each class starts at a multiple of 64 of the work index, so every
      // 64-wide chunk (one wavefront's share) holds a single class and a
      // wavefront runs one narrow-phase routine per chunk.
      int n_c[PQ_CLASSES], cstart[PQ_CLASSES + 1];
      cstart[0] = 0;
#pragma unroll
      for (int c = 0; c < PQ_CLASSES; ++c) {
        n_c[c] = min(qcnt[c], a.pq_cap[c]);
        cstart[c + 1] = cstart[c] + ((n_c[c] + 63) & ~63);
      }
      for (int i = l; i < cstart[PQ_CLASSES]; i += B) {
        int c = 0;
#pragma unroll
        for (int cc = 1; cc < PQ_CLASSES; ++cc) c += i >= cstart[cc] ? 1 : 0;
        c = __builtin_amdgcn_readfirstlane(c);  // the same on every lane of the wavefront
        const int k = i - cstart[c];
        if (k >= n_c[c]) continue;
        const int e = qbase[c] + k;
        const uint32_t ent = qent[e];
        const int qa = ent & 0x7ff, qb = (ent >> 11) & 0x7ff;
        const int la = (ent >> 22) & 31, lb = ent >> 27;
        float4 res;
        bool hit;
        switch (c) {
          case PQ_SB: hit = queued_pair<PQ_SB>(cur, stat, qa, qb, w, &res); break;
          case PQ_SL: hit = queued_pair<PQ_SL>(cur, stat, qa, qb, w, &res); break;
          case PQ_BB: hit = queued_pair<PQ_BB>(cur, stat, qa, qb, w, &res); break;
          case PQ_BL: hit = queued_pair<PQ_BL>(cur, stat, qa, qb, w, &res); break;
          default: hit = queued_pair<PQ_LL>(cur, stat, qa, qb, w, &res); break;
        }
        if (hit) {
          qres[e] = res;
          atomicOr(&hitw[qa], 1u << lb);
          atomicOr(&hitw[qb], 1u << la);
        }
      }
      lds_barrier();
      if (collide) {
        const uint32_t hits = hitw[r.slot], mine = selfw[r.slot];
        Geo self;
        self.c = V2{x, y};
        self.cs = cs;
        self.sn = sn;
        self.d0 = p.d0;
        self.d1 = p.d1;
        self.shape = shape;
        // partners class by class (sphere, box, segment), each in partner
        // order: queued results, or the lane's own evaluation
        auto run = [&](auto cls, uint32_t cm, bool direct) {
          constexpr int OTHER = decltype(cls)::value;
          while (cm) {
            const int u = __builtin_ctz(cm);
            cm &= cm - 1;
            const int q = r.lo + u;
            bool hit = true;
            if (direct || ((mine >> u) & 1u)) {
              if (p.excl != -1 && excluded(p.excl, u)) continue;
              hit = pair_force<false, OTHER>(self, p.rho, myloc, cur[q], stat[q], u, w, fx, fy, tq);
            } else {
              const float4 R = qres[qmap[r.slot * 32 + u]];
              const bool lo_side = myloc < u;
              fx += lo_side ? R.x : -R.x;
              fy += lo_side ? R.y : -R.y;
              tq += lo_side ? R.z : R.w;
            }
            if (mk && hit) {
              const int of = (__float_as_int(stat[q].w) >> 8) & 0xff;
              const bool other_active = (of & (MOVABLE | ROTATABLE)) != 0;
              if (myloc < u || !other_active) {
                const int ia = min(myloc, u), ib = max(myloc, u);
                const int64_t idx = (int64_t)ia * nloc - (int64_t)ia * (ia + 1) / 2 + (ib - ia - 1);
                mk[a.pair_off[r.env] + idx] = 1;
              }
            }
          }
        };
        const uint32_t mline = ~(cls_sph0 | cls_box0);
        if (shape == SPHERE)
          run(std::integral_constant<int, SPHERE>{}, sphw[r.slot] & cls_sph0, true);
        else
          run(std::integral_constant<int, SPHERE>{}, (hits | mine) & cls_sph0, false);
        run(std::integral_constant<int, BOX>{}, (hits | mine) & cls_box0, false);
        run(std::integral_constant<int, LINE>{}, (hits | mine) & mline, false);
      }
    } else if (collide) {
      Geo self;
      self.c = V2{x, y};
      self.cs = cs;
      self.sn = sn;
      self.d0 = p.d0;
      self.d1 = p.d1;
      self.shape = shape;
      const float rs = bounding_radius(self.shape, p.d0, p.d1);
      const float reach = w.min_dist + 1e-4f + 1e-5f * (fabsf(x) + fabsf(y));
      for (int base = 0; base < nloc; base += 32) {
        const int cnt = min(32, nloc - base);
        uint32_t cand = 0, msph = 0, mbox = 0;
        for (int u = 0; u < cnt; ++u) {
          const int q = r.lo + base + u;
          const float4 P = cur[q];
          const float dx = x - P.x, dy = y - P.y;
          const float lim = (rs + brad[q]) + reach;
          cand = shift_in(cand, dx * dx + dy * dy <= lim * lim);
        }
        cand = shifted_bits(cand, cnt);
        if (myloc >= base && myloc < base + 32) cand &= ~(1u << (myloc - base));
        if (base == 0) {
          msph = cls_sph0;
          mbox = cls_box0;
        } else {
          for (int u = 0; u < cnt; ++u) {
            const int so = __float_as_int(stat[r.lo + base + u].w) & 0xff;
            msph |= (so == SPHERE ? 1u : 0u) << u;
            mbox |= (so == BOX ? 1u : 0u) << u;
          }
        }
        // candidates class by class (sphere, box, line partners), each in
        // partner order: the lanes of a wavefront run one narrow-phase
        // routine at a time
        auto run = [&](auto cls, uint32_t cm) {
          constexpr int OTHER = decltype(cls)::value;
          while (cm) {
            const int u = __builtin_ctz(cm);
            cm &= cm - 1;
            const int q = r.lo + base + u;
            const int b = base + u;
            const float4 S = stat[q];
            const int of = (__float_as_int(S.w) >> 8) & 0xff;
            if (p.excl != -1 && excluded(p.excl, b)) continue;
            const float4 P = cur[q];
            const bool hit = pair_force<false, OTHER>(self, p.rho, myloc, P, S, b, w, fx, fy, tq);
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
        };
        run(std::integral_constant<int, SPHERE>{}, cand & msph);
        run(std::integral_constant<int, BOX>{}, cand & mbox);
        run(std::integral_constant<int, LINE>{}, cand & ~(msph | mbox));
      }
    }
    if (act && nj > 0) {
      // Joints: spring between world anchors, evaluated in joint order.
      auto joint = [&](const JointK& J, bool is_a, int q) {
        const float4 P = cur[q];
        V2 f;
        float ts, to;
        if (joint_eval<float>(V2{x, y}, cs, sn, V2{P.x, P.y}, P.z, P.w, is_a, J, w.joint_k, &f, &ts,
                              &to)) {
          fx += f.x;
          fy += f.y;
          tq += ts;
        }
      };
#pragma unroll
      for (int q = 0; q < 2; ++q)
        if (q < nj) joint(jr[q], jis_a[q], jslot[q]);
      for (int jj = j0 + 2; jj < j0 + nj; ++jj) {
        const JointK J = a.joints[a.jlist[jj]];
        const bool is_a = J.a == r.ent;
        joint(J, is_a, r.lo + ((is_a ? J.b : J.a) - r.first));
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
      float* o = a.traj + (size_t)(t + 1) * (a.traj_xy ? 2 : 6) * N;
      o[r.ent] = x;
      o[N + r.ent] = y;
      if (!a.traj_xy) {
        o[2 * N + r.ent] = vx;
        o[3 * N + r.ent] = vy;
        o[4 * N + r.ent] = th;
        o[5 * N + r.ent] = om;
      }
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

// Sphere-only batches (every collidable or moving entity is a sphere): the
// pair force acts along the line of centres and never makes a torque, so the
// per-step LDS exchange is the centre (x, y) alone; radius and flags are
// staged once. The actions of KCH steps are loaded per chunk into registers
// one chunk ahead, which hides the HBM latency behind KCH steps of work (the
// per-step barrier waits for LDS traffic only, so the loads stay in flight);
// the chunk loop is unrolled so every action register is addressed
// statically.
//
// NB in 4..32: every environment of the plan has at most NB entities. A lane's
// partners are the NB - 1 slots of its environment other than its own (slot
// u' + [u' >= own slot] for partner u'), fixed for the whole rollout, so their
// LDS addresses and squared contact distances fl((r_i + r_j [+ d_min])^2) are
// computed once into registers, -1 for partners past the environment (they
// read neighbours or padding). The per-step test of a partner is then the
// FP32 rule fl(dx^2 + fl(dy^2)) <= dmin2 (one fused multiply-add). NB = 64:
// blocks of 8 slots unrolled, the contact distance from the staged radius,
// a 64-bit hit mask. NB = 0: any size, 32 partners per pass. MD: the world has a nonzero minimum
// distance. The arithmetic of a contact is the same, operation for operation,
// in every variant and as the sphere path of k_rollout (pair_force on two spheres).
#ifndef VMAS_KCH
#define VMAS_KCH 8
#endif
constexpr int KCH = VMAS_KCH;

template <int MAXB, int NB, bool MD, bool OUT>
__global__ void __launch_bounds__(MAXB) k_rollout_sph(StepArgs a) {
  extern __shared__ float2 lds2[];
  const int E = a.max_stage + NB;  // slots per array, padding included
  float2* pos0 = lds2;
  float2* pos1 = lds2 + E;
  float2* stat = lds2 + 2 * E;     // (radius or NaN if not collidable, flags)
  const int g = blockIdx.x, l = threadIdx.x, B = blockDim.x;
  const int N = a.w.N;
  const int s0 = a.stage_off[g], ns = a.stage_off[g + 1] - s0;
  const float qnan = __int_as_float(0x7fc00000);
  for (int s = l; s < ns + NB; s += B) {
    float2 P = make_float2(0.0f, 0.0f), S = make_float2(qnan, 0.0f);  // padding
    if (s < ns) {
      const int e = a.stage[s0 + s];
      const int sf = a.ent[e].sf;
      P = make_float2(a.state[e], a.state[N + e]);
      S = make_float2(((sf >> 8) & COLLIDABLE) ? a.ent[e].rho : qnan, __int_as_float(sf));
    }
    pos0[s] = P;
    pos1[s] = P;
    stat[s] = S;
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
  const int fl = (p.sf >> 8) & 0xff;
  const bool movable = act && (fl & MOVABLE) != 0, rotatable = act && (fl & ROTATABLE) != 0;
  const bool collide = act && (fl & COLLIDABLE) != 0;
  const bool agent = act && r.agent >= 0;
  const int myloc = r.slot - r.lo, nloc = r.hi - r.lo;
  const int gmaxn = a.grp_maxn[g];
  const WorldK w = a.w;
  const int T = a.T;
  const size_t A = (size_t)w.A;
  const bool drawn = a.actions == nullptr;  // uniform
  const float2* ap = reinterpret_cast<const float2*>(a.actions) + (agent ? r.agent : 0);
  const uint64_t z0 = ctr0(a.key, a.t0, w.A, agent ? r.agent : 0), zs = step_ctr(w.A);
  float2 cur[KCH], nxt[KCH];
  auto load_chunk = [&](float2* dst, int c) {
#pragma unroll
    for (int k = 0; k < KCH; ++k) dst[k] = make_float2(0.0f, 0.0f);
    if (!drawn) {
#pragma unroll
      for (int k = 0; k < KCH; ++k)
        if (agent && c + k < T) dst[k] = ap[(size_t)(c + k) * A];
    } else {
#pragma unroll
      for (int k = 0; k < KCH; ++k)
        if (agent && c + k < T) dst[k] = draw_action(z0 + (uint64_t)(c + k) * zs);
    }
  };
  load_chunk(cur, 0);
  wait_global_loads();
  __syncthreads();
  // partner u' sits in slot u' + [u' >= own slot]; its squared contact
  // distance (-1: never in contact)
  constexpr bool HOIST = NB > 0 && NB <= 32;
  constexpr int NP = HOIST ? NB - 1 : 1;
  int sl[NP];
  float dm2[NP], pdm[NP];  // squared contact distance, contact distance
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    sl[u] = u + (u >= myloc ? 1 : 0);
    dm2[u] = -1.0f;
    pdm[u] = 0.0f;
    if (HOIST && collide && sl[u] < nloc) {
      float dmin = p.rho + stat[r.lo + sl[u]].x;
      if (MD) dmin += w.min_dist;
      dm2[u] = __fmul_rn(dmin, dmin);
      pdm[u] = dmin;
    }
  }
  // NB == 64: slots u < nloc other than the lane's own
  const uint64_t valid64 = (nloc >= 64 ? ~0ull : ((1ull << nloc) - 1ull)) & ~(1ull << (myloc & 63));
  // NB == 64, equal radii: when every partner of every lane of the
  // wavefront is collidable with the lane's own radius, each partner's
  // contact distance is the lane's fl((r + r [+ d_min])^2) -- the value the
  // per-partner sum gives -- and the partners' records need not be read
  bool eq_r = true;
  if (NB == 64 && collide)
    for (int u = 0; u < nloc; ++u) eq_r &= u == myloc || stat[r.lo + u].x == p.rho;
  const bool uni = NB == 64 && __builtin_amdgcn_ballot_w64(collide && !eq_r) == 0;
  float dm2u;
  {
    float dmin = p.rho + p.rho;
    if (MD) dmin += w.min_dist;
    dm2u = __fmul_rn(dmin, dmin);
  }
  for (int c = 0; c < T; c += KCH) {
    if (c + KCH < T) load_chunk(nxt, c + KCH);
#pragma unroll
    for (int k = 0; k < KCH; ++k) {
      const int t = c + k;
      if (t < T) {  // uniform over the block
        float2* cb = (t & 1) ? pos1 : pos0;
        if (t > 0) {
          if (act) cb[r.slot] = make_float2(x, y);
          lds_barrier();
        }
        float fx = cur[k].x + p.mgx, fy = cur[k].y + p.mgy;
        uint8_t* mk = (OUT && t == T - 1 && a.mask) ? a.mask : nullptr;
        // contact force of partner slot q (in contact), and its mask entry
        auto contact = [&](int q) {
          const float2 P = cb[q];
          const float2 S = stat[q];
          float dmin = p.rho + S.x;
          if (MD) dmin += w.min_dist;
          const float dx = x - P.x, dy = y - P.y;
          const float sq = fmaf(dx, dx, __fmul_rn(dy, dy));
          // sphere_normal without a branch: the same values, selected
          const float rs = __frsqrt_rn(sq);
          const bool coincide = sq == 0.0f;
          const float d = coincide ? 0.0f : sq * rs;
          const V2 n = {coincide ? (r.slot < q ? 1.0f : -1.0f) : dx * rs, coincide ? 0.0f : dy * rs};
          const float F = contact_mag(dmin, d, w);
          fx = fmaf(F, n.x, fx);
          fy = fmaf(F, n.y, fy);
          if (mk) {
            const int of = __float_as_int(S.y) >> 8;
            const int b = q - r.lo;
            if (myloc < b || (of & (MOVABLE | ROTATABLE)) == 0) {
              const int ia = min(myloc, b), ib = max(myloc, b);
              const int64_t idx = (int64_t)ia * nloc - (int64_t)ia * (ia + 1) / 2 + (ib - ia - 1);
              mk[a.pair_off[r.env] + idx] = 1;
            }
          }
        };
        if (collide) {
          if constexpr (NB == 64) {
            // up to 64 slots, 8 per block (uniform guard), own slot and
            // slots past the environment masked out once per rollout; the
            // contact distance comes from the staged radius
            const float2* pb = ((k & 1) ? pos1 : pos0) + r.lo;  // KCH is even
            const float2* sb = stat + r.lo;
            // each test shifted into the low end of a 32-bit word (one
            // add with carry), the first partner ending in the top bit;
            // reversed into bit u = partner u below
            uint32_t mlo = 0u, mhi = 0u;
            if (uni) {
#pragma unroll
              for (int blk = 0; blk < 64; blk += 8) {
                if (blk < gmaxn) {
                  float2 P[8];
#pragma unroll
                  for (int v = 0; v < 8; ++v) P[v] = pb[blk + v];
                  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                  for (int v = 0; v < 8; ++v) {
                    const float dx = x - P[v].x, dy = y - P[v].y;
                    const bool hit = fmaf(dx, dx, __fmul_rn(dy, dy)) <= dm2u;
                    if (blk < 32) mlo = shift_in(mlo, hit);
                    else mhi = shift_in(mhi, hit);
                  }
                }
              }
            } else {
#pragma unroll
              for (int blk = 0; blk < 64; blk += 8) {
                if (blk < gmaxn) {
                  // the block's reads in flight before its tests
                  float2 P[8], S[8];
#pragma unroll
                  for (int v = 0; v < 8; ++v) {
                    P[v] = pb[blk + v];
                    S[v] = sb[blk + v];
                  }
                  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                  for (int v = 0; v < 8; ++v) {
                    float dmin = p.rho + S[v].x;
                    if (MD) dmin += w.min_dist;
                    const float dx = x - P[v].x, dy = y - P[v].y;
                    const bool hit = fmaf(dx, dx, __fmul_rn(dy, dy)) <= __fmul_rn(dmin, dmin);
                    if (blk < 32) mlo = shift_in(mlo, hit);
                    else mhi = shift_in(mhi, hit);
                  }
                }
              }
            }
            // blocks past the group's largest environment were not tested
            const int nt = min(64, (gmaxn + 7) & ~7);
            uint64_t hits = ((uint64_t)shifted_bits(mhi, nt - min(32, nt)) << 32) |
                            shifted_bits(mlo, min(32, nt));
            hits &= valid64;
            while (hits) {
              const int u = __builtin_ctzll(hits);
              hits &= hits - 1;
              contact(r.lo + u);
            }
          } else if constexpr (NB > 0) {
            // Pass 1: the test of every partner into a bit mask (partner u'
            // -> bit u'). Pass 2: forces for the set bits only, first
            // partner first, so a wavefront runs the force code as often as
            // its busiest lane has contacts.
            const float2* pb = ((k & 1) ? pos1 : pos0) + r.lo;  // KCH is even
            if constexpr (NP <= 8) {
              // one block: the offsets stay in registers, and a contact
              // picks its partner's values by selects instead of reading
              // the partner from LDS again
              if (0 < gmaxn - 1) {  // uniform over the block
                float2 P[NP];
#pragma unroll
                for (int v = 0; v < NP; ++v) P[v] = pb[sl[v]];
                __builtin_amdgcn_sched_barrier(0);
                float pdx[NP], pdy[NP], psq[NP];
                uint32_t hits = 0;
#pragma unroll
                for (int v = 0; v < NP; ++v) {
                  pdx[v] = x - P[v].x;
                  pdy[v] = y - P[v].y;
                  psq[v] = fmaf(pdx[v], pdx[v], __fmul_rn(pdy[v], pdy[v]));
                  hits = shift_in(hits, psq[v] <= dm2[v]);
                }
                hits = shifted_bits(hits, NP);
                while (hits) {
                  const int u = __builtin_ctz(hits);
                  hits &= hits - 1;
                  float dx = pdx[0], dy = pdy[0], sq = psq[0], dmin = pdm[0];
                  int b = sl[0];
#pragma unroll
                  for (int v = 1; v < NP; ++v) {
                    const bool m = u == v;
                    dx = m ? pdx[v] : dx;
                    dy = m ? pdy[v] : dy;
                    sq = m ? psq[v] : sq;
                    dmin = m ? pdm[v] : dmin;
                    b = m ? sl[v] : b;
                  }
                  const float rs = __frsqrt_rn(sq);
                  const bool coincide = sq == 0.0f;
                  const float d = coincide ? 0.0f : sq * rs;
                  const V2 n = {coincide ? (myloc < b ? 1.0f : -1.0f) : dx * rs, coincide ? 0.0f : dy * rs};
                  const float F = contact_mag(dmin, d, w);
                  fx = fmaf(F, n.x, fx);
                  fy = fmaf(F, n.y, fy);
                  if (mk) {
                    const int of = __float_as_int(stat[r.lo + b].y) >> 8;
                    if (myloc < b || (of & (MOVABLE | ROTATABLE)) == 0) {
                      const int ia = min(myloc, b), ib = max(myloc, b);
                      const int64_t idx = (int64_t)ia * nloc - (int64_t)ia * (ia + 1) / 2 + (ib - ia - 1);
                      mk[a.pair_off[r.env] + idx] = 1;
                    }
                  }
                }
              }
            } else {
            uint32_t hits = 0;
#pragma unroll
            for (int blk = 0; blk < NP; blk += 8) {
              if (blk < gmaxn - 1) {  // uniform over the block
                // all reads of the block in flight before the tests (the
                // scheduler otherwise holds one back behind the others)
                float2 P[8];
#pragma unroll
                for (int v = 0; v < 8 && blk + v < NP; ++v) P[v] = pb[sl[blk + v]];
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int v = 0; v < 8 && blk + v < NP; ++v) {
                  const float dx = x - P[v].x, dy = y - P[v].y;
                  hits = shift_in(hits, fmaf(dx, dx, __fmul_rn(dy, dy)) <= dm2[blk + v]);
                }
              }
            }
            hits = shifted_bits(hits, gmaxn > 1 ? min(NP, (gmaxn - 1 + 7) & ~7) : 0);
            while (hits) {
              const int u = __builtin_ctz(hits);
              hits &= hits - 1;
              contact(r.lo + u + (u >= myloc ? 1 : 0));
            }
            }
          } else {
            // any size: 32 partners per pass, tested into a bit mask, then the
            // force code for the set bits; the trip count is the largest
            // environment of the group (uniform over the workgroup), an index
            // past the lane's own environment is clamped to a valid slot and
            // masked out
            for (int base = 0; base < gmaxn; base += 32) {
              const int cnt = min(32, gmaxn - base);
              uint32_t hits = 0;
              for (int u = 0; u < cnt; ++u) {
                const int q = min(r.lo + base + u, r.hi - 1);
                const float2 P = cb[q];
                float dmin = p.rho + stat[q].x;
                if (MD) dmin += w.min_dist;
                const float dx = x - P.x, dy = y - P.y;
                const bool hit = (fmaf(dx, dx, __fmul_rn(dy, dy)) <= __fmul_rn(dmin, dmin)) &
                                 (base + u < nloc);
                hits = shift_in(hits, hit);
              }
              hits = shifted_bits(hits, cnt);
              if (myloc >= base && myloc < base + 32) hits &= ~(1u << (myloc - base));
              while (hits) {
                const int u = __builtin_ctz(hits);
                hits &= hits - 1;
                contact(r.lo + base + u);
              }
            }
          }
        }
        if (OUT && t == T - 1 && a.forces && act) {
          a.forces[r.ent] = fx;
          a.forces[N + r.ent] = fy;
          a.forces[2 * N + r.ent] = 0.0f;
        }
        if (movable) {
          const float ax = fx * p.inv_m, ay = fy * p.inv_m;
          vx = fmaf(ax, w.dt, w.damp * vx);
          vy = fmaf(ay, w.dt, w.damp * vy);
          if (p.vmax > 0.0f) {
            const float sp = sqrtf(fmaf(vx, vx, vy * vy));
            if (sp > p.vmax) {
              const float sc = p.vmax / sp;
              vx *= sc;
              vy *= sc;
            }
          }
          x = fmaf(vx, w.dt, x);
          y = fmaf(vy, w.dt, y);
        }
        if (rotatable) {
          om = fmaf(0.0f * p.inv_I, w.dt, w.damp * om);
          th = fmaf(om, w.dt, th);
        }
        if (OUT && a.traj && act) {
          float* o = a.traj + (size_t)(t + 1) * (a.traj_xy ? 2 : 6) * N;
          o[r.ent] = x;
          o[N + r.ent] = y;
          if (!a.traj_xy) {
            o[2 * N + r.ent] = vx;
            o[3 * N + r.ent] = vy;
            o[4 * N + r.ent] = th;
            o[5 * N + r.ent] = om;
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < KCH; ++k) cur[k] = nxt[k];
  }
  if (act && T > 0) {
    const int e = r.ent;
    a.state[e] = x;
    a.state[N + e] = y;
    a.state[2 * N + e] = vx;
    a.state[3 * N + e] = vy;
    a.state[4 * N + e] = th;
    a.state[5 * N + e] = om;
  }
}

// Quad schedule for sphere-only batches whose environments have at most 4
// entities that move or rotate and at most 4 static collidable entities
// (e.g. 4 agents and 2 landmarks): the movers of an environment sit on one
// aligned quad of lanes and read each other's centres with DPP quad
// permutations, so a step needs no LDS traffic and no barrier. Static
// entities never move; their centres, like every contact distance, are
// loaded into registers once. Contacts are visited in partner order (local
// index) with the arithmetic of the other sphere kernels, so results are
// bitwise those of every other schedule.
template <int CTRL>
__device__ __forceinline__ float quad_perm(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}

template <bool MD, int NS, bool OUT>
__global__ void __launch_bounds__(256) k_rollout_quad(StepArgs a) {
  const int gl = blockIdx.x * blockDim.x + threadIdx.x;
  const int qi = gl >> 2, qp = gl & 3;
  const bool in = qi < (a.env_list ? a.n_list : a.n_envs);
  const int env = in ? (a.env_list ? a.env_list[qi] : qi) : 0;
  const int N = a.w.N;
  // the environment record as one 16-byte word, unpacked with shifts (no
  // per-lane array, which the compiler would place in LDS)
  int4 qw = make_int4(0, 0, -1, -1);
  int o = 0, n = 0;
  if (in) {
    qw = reinterpret_cast<const int4*>(a.quad)[env];
    o = a.env_off[env];
    n = a.env_off[env + 1] - o;
  }
  auto lane_loc = [&](int u) { return (int)(int8_t)((uint32_t)qw.z >> (8 * u)); };
  auto stat_loc = [&](int u) { return (int)(int8_t)((uint32_t)qw.w >> (8 * u)); };
  const int myloc = lane_loc(qp);
  const bool act = myloc >= 0;
  const int e = o + myloc;
  float x = 0, y = 0, vx = 0, vy = 0, th = 0, om = 0;
  EntParam p{};
  if (act) {
    x = a.state[e];
    y = a.state[N + e];
    vx = a.state[2 * N + e];
    vy = a.state[3 * N + e];
    th = a.state[4 * N + e];
    om = a.state[5 * N + e];
    p = a.ent[e];
  }
  const int fl = (p.sf >> 8) & 0xff;
  const bool movable = act && (fl & MOVABLE) != 0, rotatable = act && (fl & ROTATABLE) != 0;
  const bool collide = act && (fl & COLLIDABLE) != 0;
  const bool agent = act && myloc < qw.y;
  const WorldK w = a.w;
  // partners: quad lanes qp ^ 1, qp ^ 2, qp ^ 3, then NS static entities
  // (NS: the most any environment of the batch has); bit (1 << local index)
  // of each, its radius, flags and contact distance squared (-1: never in
  // contact)
  constexpr int NP = 3 + NS;
  uint32_t bit[NP];
  float rad[NP], dm2[NP], sx[NS > 0 ? NS : 1], sy[NS > 0 ? NS : 1];
  int pfl[NP];
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    const int loc = u < 3 ? lane_loc(qp ^ (u + 1)) : stat_loc(u - 3);
    bit[u] = loc >= 0 ? 1u << loc : 0u;
    rad[u] = 0.0f;
    pfl[u] = 0;
    dm2[u] = -1.0f;
    if (u >= 3) {
      sx[u - 3] = 0.0f;
      sy[u - 3] = 0.0f;
    }
    if (loc >= 0) {
      const EntParam q = a.ent[o + loc];
      rad[u] = q.rho;
      pfl[u] = (q.sf >> 8) & 0xff;
      if (u >= 3) {
        sx[u - 3] = a.state[o + loc];
        sy[u - 3] = a.state[N + o + loc];
      }
      if (collide && (pfl[u] & COLLIDABLE)) {
        float dmin = p.rho + q.rho;
        if (MD) dmin += w.min_dist;
        dm2[u] = __fmul_rn(dmin, dmin);
      }
    }
  }
  const int T = a.T;
  const size_t A = (size_t)w.A;
  const int arow = agent ? qw.x + myloc : 0;
  const bool drawn = a.actions == nullptr;  // uniform
  const float2* ap = reinterpret_cast<const float2*>(a.actions) + arow;
  const uint64_t z0 = ctr0(a.key, a.t0, w.A, arow), zs = step_ctr(w.A);
  float2 cur[KCH], nxt[KCH];
  auto load_chunk = [&](float2* dst, int c) {
#pragma unroll
    for (int k = 0; k < KCH; ++k) dst[k] = make_float2(0.0f, 0.0f);
    if (!drawn) {
#pragma unroll
      for (int k = 0; k < KCH; ++k)
        if (agent && c + k < T) dst[k] = ap[(size_t)(c + k) * A];
    } else {
#pragma unroll
      for (int k = 0; k < KCH; ++k)
        if (agent && c + k < T) dst[k] = draw_action(z0 + (uint64_t)(c + k) * zs);
    }
  };
  load_chunk(cur, 0);
  wait_global_loads();
  for (int c = 0; c < T; c += KCH) {
    if (c + KCH < T) load_chunk(nxt, c + KCH);
#pragma unroll
    for (int k = 0; k < KCH; ++k) {
      const int t = c + k;
      if (t < T) {  // uniform
        // centres of the quad partners (every lane takes part)
        float px[NP], py[NP];
        px[0] = quad_perm<0xB1>(x);  // lane ^ 1
        py[0] = quad_perm<0xB1>(y);
        px[1] = quad_perm<0x4E>(x);  // lane ^ 2
        py[1] = quad_perm<0x4E>(y);
        px[2] = quad_perm<0x1B>(x);  // lane ^ 3
        py[2] = quad_perm<0x1B>(y);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          px[3 + s] = sx[s];
          py[3 + s] = sy[s];
        }
        float fx = cur[k].x + p.mgx, fy = cur[k].y + p.mgy;
        uint8_t* mk = (OUT && t == T - 1 && a.mask) ? a.mask : nullptr;
        if (collide) {
          uint32_t hits = 0;
#pragma unroll
          for (int u = 0; u < NP; ++u) {
            const float dx = x - px[u], dy = y - py[u];
            const bool hit = fmaf(dx, dx, __fmul_rn(dy, dy)) <= dm2[u];
            hits |= hit ? bit[u] : 0u;
          }
          while (hits) {  // partner order: lowest local index first
            const uint32_t b1 = hits & (0u - hits);
            hits ^= b1;
            const int ploc = __builtin_ctz(b1);
            float PX = 0.0f, PY = 0.0f, PR = 0.0f;
            int PF = 0;
#pragma unroll
            for (int u = 0; u < NP; ++u) {
              if (bit[u] == b1) {
                PX = px[u];
                PY = py[u];
                PR = rad[u];
                PF = pfl[u];
              }
            }
            float dmin = p.rho + PR;
            if (MD) dmin += w.min_dist;
            const float dx = x - PX, dy = y - PY;
            const float sq = fmaf(dx, dx, __fmul_rn(dy, dy));
            V2 nrm;
            float d;
            sphere_normal(dx, dy, sq, myloc < ploc, &d, &nrm);
            const float F = contact_mag(dmin, d, w);
            fx = fmaf(F, nrm.x, fx);
            fy = fmaf(F, nrm.y, fy);
            if (mk && (myloc < ploc || (PF & (MOVABLE | ROTATABLE)) == 0)) {
              const int ia = min(myloc, ploc), ib = max(myloc, ploc);
              const int64_t idx = (int64_t)ia * n - (int64_t)ia * (ia + 1) / 2 + (ib - ia - 1);
              mk[a.pair_off[env] + idx] = 1;
            }
          }
        }
        if (OUT && t == T - 1 && a.forces && act) {
          a.forces[e] = fx;
          a.forces[N + e] = fy;
          a.forces[2 * N + e] = 0.0f;
        }
        if (movable) {
          const float ax = fx * p.inv_m, ay = fy * p.inv_m;
          vx = fmaf(ax, w.dt, w.damp * vx);
          vy = fmaf(ay, w.dt, w.damp * vy);
          if (p.vmax > 0.0f) {
            const float sp = sqrtf(fmaf(vx, vx, vy * vy));
            if (sp > p.vmax) {
              const float sc = p.vmax / sp;
              vx *= sc;
              vy *= sc;
            }
          }
          x = fmaf(vx, w.dt, x);
          y = fmaf(vy, w.dt, y);
        }
        if (rotatable) {
          om = fmaf(0.0f * p.inv_I, w.dt, w.damp * om);
          th = fmaf(om, w.dt, th);
        }
        if (OUT && a.traj && act) {
          float* out = a.traj + (size_t)(t + 1) * (a.traj_xy ? 2 : 6) * N;
          out[e] = x;
          out[N + e] = y;
          if (!a.traj_xy) {
            out[2 * N + e] = vx;
            out[3 * N + e] = vy;
            out[4 * N + e] = th;
            out[5 * N + e] = om;
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < KCH; ++k) cur[k] = nxt[k];
  }
  if (act && T > 0) {
    a.state[e] = x;
    a.state[N + e] = y;
    a.state[2 * N + e] = vx;
    a.state[3 * N + e] = vy;
    a.state[4 * N + e] = th;
    a.state[5 * N + e] = om;
  }
}

// Quad schedule with ordered partners, for sphere batches whose every
// environment puts its (at most 4) movers first -- local indices 0 .. m-1 on
// quad lanes 0 .. m-1 -- and its (at most NS) static collidable entities
// after them (e.g. 4 agents and 2 landmarks). Partner slot k of quad lane q
// is mover k + [k >= q], read with a quad permutation that serves slot k in
// local-index order on every lane, and static s comes after all movers, so
// the slots are in local-index order: contacts are added in the order every
// other schedule uses, and a partner's values are never selected at run
// time. Per step a lane tests its NS + 3 partners (the partner's centre is
// used once, in the difference, where the compiler folds the permutation
// into the subtraction), and a wavefront runs the contact code of slot k
// only when some lane hit partner k (about a quarter of the wavefront-steps
// of the 30,000-environment workload have a contact at all). The angular
// update of a sphere is the identity while omega is +0 (no torque on a
// sphere), so it is skipped for a wavefront whose angular velocities are
// all +0 and whose angles hold no -0. Results are bitwise those of the other
// sphere schedules.
template <int CTRL>
__device__ __forceinline__ float quad_src(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}

template <bool MD, int NS, bool OUT>
__global__ void __launch_bounds__(64) k_rollout_quad_ord(StepArgs a) {
  const int gl = blockIdx.x * blockDim.x + threadIdx.x;
  const int qi = gl >> 2, qp = gl & 3;
  const bool in = qi < (a.env_list ? a.n_list : a.n_envs);
  const int N = a.w.N;
  // Set-up in two rounds of independent loads (every load issued
  // unconditionally from a valid index, the value selected afterwards): the
  // environment's record and offsets, then the lane's own state and
  // parameters and the static partners' centres, radii and flags. The
  // movers' radii and flags come from their own lanes (quad permutations).
  // The environment record is read as one 16-byte word and unpacked with
  // shifts (no per-lane array, which the compiler would place in LDS).
  const int envc = in ? (a.env_list ? a.env_list[qi] : qi) : 0;
  const int env = envc;
  const int4 qw = reinterpret_cast<const int4*>(a.quad)[envc];
  const int o = a.env_off[envc], n = a.env_off[envc + 1] - o;
  const int agent_row = qw.x, n_agents = in ? qw.y : 0;
  // local index of the mover on quad lane u (-1: idle) / of static u (-1: none)
  auto lane_loc = [&](int u) { return in ? (int)(int8_t)((uint32_t)qw.z >> (8 * u)) : -1; };
  auto stat_loc = [&](int u) { return in ? (int)(int8_t)((uint32_t)qw.w >> (8 * u)) : -1; };
  const bool act = lane_loc(qp) >= 0;  // lane qp holds local entity qp
  const int T = a.T;
  const size_t A = (size_t)a.w.A;
  const bool agent = act && qp < n_agents;
  const int arow = agent ? agent_row + qp : 0;  // a lane without an action reads row 0
  const bool drawn = a.actions == nullptr;  // uniform
  const float2* ap = reinterpret_cast<const float2*>(a.actions) + arow;
  const uint64_t z0 = ctr0(a.key, a.t0, a.w.A, arow), zs = step_ctr(a.w.A);
  // Actions of KCH steps per chunk, two chunks in flight (ping-pong, no
  // register copies); rows past the rollout are clamped to its last row
  // (read, never used), so every load is unconditional. The first chunk is
  // requested here, with the lane's own state, before anything waits.
  auto load_chunk = [&](float2* dst, int c) {
    if (!drawn) {
      if (A > 0) {
#pragma unroll
        for (int k = 0; k < KCH; ++k) dst[k] = ap[(size_t)min(c + k, T - 1) * A];
      }
    } else {
#pragma unroll
      for (int k = 0; k < KCH; ++k) dst[k] = draw_action(z0 + (uint64_t)min(c + k, T - 1) * zs);
    }
  };
  float2 bufA[KCH];
#pragma unroll
  for (int k = 0; k < KCH; ++k) bufA[k] = make_float2(0.0f, 0.0f);
  if (T > 0) load_chunk(bufA, 0);
  const int e = o + qp;
  const int ec = act ? e : min(o, N - 1);  // a valid index for the loads
  float x = a.state[ec], y = a.state[N + ec], vx = a.state[2 * N + ec],
        vy = a.state[3 * N + ec], th = a.state[4 * N + ec], om = a.state[5 * N + ec];
  // the lane's parameters from its 16-byte record; gravity and 1/I from
  // the full record only where the batch has them (uniform)
  const SphRec ps = a.sph[ec];
  EntParam p{};
  p.rho = ps.rho;
  p.inv_m = ps.inv_m;
  p.vmax = ps.vmax;
  p.sf = ps.sf;
  p.inv_I = 1.0f;  // 0 x 1/I is +0 for every finite 1/I >= 0
  if (!a.sph_only) {
    const EntParam& q = a.ent[ec];
    p.mgx = q.mgx;
    p.mgy = q.mgy;
    p.inv_I = q.inv_I;
  }
  float srad[NS > 0 ? NS : 1], sx[NS > 0 ? NS : 1], sy[NS > 0 ? NS : 1];
  int sfl[NS > 0 ? NS : 1], sloc[NS > 0 ? NS : 1];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    sloc[s] = stat_loc(s);
    const int es = min(o + (sloc[s] >= 0 ? sloc[s] : 0), N - 1);
    const SphRec rs = a.sph[es];
    const float r = rs.rho;
    const int sfv = rs.sf;
    const float cx = a.state[es], cy = a.state[N + es];
    srad[s] = r;
    sfl[s] = sloc[s] >= 0 ? (sfv >> 8) & 0xff : 0;
    sx[s] = cx;
    sy[s] = cy;
  }
  if (!act) {
    x = y = vx = vy = th = om = 0.0f;
    p = EntParam{};
  }
  const int fl = (p.sf >> 8) & 0xff;
  const bool movable = act && (fl & MOVABLE) != 0, rotatable = act && (fl & ROTATABLE) != 0;
  const bool collide = act && (fl & COLLIDABLE) != 0;
  const WorldK w = a.w;
  // slots 0..2: movers k + [k >= qp] (their radius and whether they collide
  // from their lanes); slots 3..: statics. Contact distance squared (-1:
  // never in contact), contact distance, local index.
  constexpr int NP = 3 + NS;
  float prad[3];
  int pcol[3];
  prad[0] = quad_src<0x01>(p.rho);
  prad[1] = quad_src<0x5A>(p.rho);
  prad[2] = quad_src<0xBF>(p.rho);
  {
    const float c = collide ? 1.0f : 0.0f;
    pcol[0] = quad_src<0x01>(c) != 0.0f;
    pcol[1] = quad_src<0x5A>(c) != 0.0f;
    pcol[2] = quad_src<0xBF>(c) != 0.0f;
  }
  float dm2[NP], pdm[NP];
  int ploc[NP];
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    int loc;
    bool pc;
    float pr;
    if (u < 3) {
      loc = u + (u >= qp ? 1 : 0);
      pc = loc < 4 && lane_loc(loc) >= 0 && pcol[u];
      pr = prad[u];
    } else {
      loc = sloc[u - 3];
      pc = loc >= 0 && (sfl[u - 3] & COLLIDABLE);
      pr = srad[u - 3];
    }
    ploc[u] = loc < 0 ? 255 : loc;
    float dmin = p.rho + pr;
    if (MD) dmin += w.min_dist;
    const bool ok = collide && pc;
    dm2[u] = ok ? __fmul_rn(dmin, dmin) : -1.0f;
    pdm[u] = ok ? dmin : 0.0f;
  }
  // angles and angular velocities change only while some omega is not +0
  // or some angle is -0 (see above); otherwise the update is the identity
  const bool spin = __builtin_amdgcn_ballot_w64(rotatable && (__float_as_uint(om) != 0u ||
                                                              __float_as_uint(th) == 0x80000000u)) != 0;
  // a mover that is not an agent takes no action (zero force); otherwise
  // every lane's action row is read as is
  const bool mute = __builtin_amdgcn_ballot_w64(act && !agent) != 0;
  // unit masses: f / m is f itself (x * 1 is exact), so the multiply goes
  const bool unit = __builtin_amdgcn_ballot_w64(movable && p.inv_m != 1.0f) == 0;
  auto run = [&](auto spin_tag, auto mute_tag, auto unit_tag) {
    constexpr bool SPIN = decltype(spin_tag)::value, MUTE = decltype(mute_tag)::value;
    constexpr bool UNIT = decltype(unit_tag)::value;
    // one step with the actions f of step t
    auto step = [&](float2 f, int t) {
      if (MUTE && !agent) f = make_float2(0.0f, 0.0f);
      float dx[NP], dy[NP], sq[NP];
      bool hit[NP];
      // movers in local order: lane q takes slot k from lane k + [k >= q]
      dx[0] = x - quad_src<0x01>(x);  // quad_perm [1, 0, 0, 0]
      dy[0] = y - quad_src<0x01>(y);
      dx[1] = x - quad_src<0x5A>(x);  // quad_perm [2, 2, 1, 1]
      dy[1] = y - quad_src<0x5A>(y);
      dx[2] = x - quad_src<0xBF>(x);  // quad_perm [3, 3, 3, 2]
      dy[2] = y - quad_src<0xBF>(y);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        dx[3 + s] = x - sx[s];
        dy[3 + s] = y - sy[s];
      }
      bool any = false;
#pragma unroll
      for (int u = 0; u < NP; ++u) {
        sq[u] = fmaf(dx[u], dx[u], __fmul_rn(dy[u], dy[u]));
        hit[u] = sq[u] <= dm2[u];
        any |= hit[u];
      }
      float fx = f.x + p.mgx, fy = f.y + p.mgy;
      uint8_t* mk = (OUT && t == T - 1 && a.mask) ? a.mask : nullptr;
      if (__builtin_amdgcn_ballot_w64(any) != 0) {
#pragma unroll
        for (int u = 0; u < NP; ++u) {
          if (hit[u]) {  // partner order: lowest local index first
            const float rs = __frsqrt_rn(sq[u]);
            float d = sq[u] * rs, nx = dx[u] * rs, ny = dy[u] * rs;
            if (__builtin_amdgcn_ballot_w64(sq[u] == 0.0f) != 0) {  // coincident centres (rare)
              const bool self_lo = u >= 3 || u >= qp;
              if (sq[u] == 0.0f) {
                d = 0.0f;
                nx = self_lo ? 1.0f : -1.0f;
                ny = 0.0f;
              }
            }
            const float F = contact_mag(pdm[u], d, w);
            fx = fmaf(F, nx, fx);
            fy = fmaf(F, ny, fy);
            if (mk) {
              const int pl = ploc[u];
              const int pf = u >= 3 ? sfl[u - 3] : fl;
              if (qp < pl || (pf & (MOVABLE | ROTATABLE)) == 0) {
                const int ia = min(qp, pl), ib = max(qp, pl);
                const int64_t idx = (int64_t)ia * n - (int64_t)ia * (ia + 1) / 2 + (ib - ia - 1);
                mk[a.pair_off[env] + idx] = 1;
              }
            }
          }
        }
      }
      if (OUT && t == T - 1 && a.forces && act) {
        a.forces[e] = fx;
        a.forces[N + e] = fy;
        a.forces[2 * N + e] = 0.0f;
      }
      if (movable) {
        const float ax = UNIT ? fx : fx * p.inv_m, ay = UNIT ? fy : fy * p.inv_m;
        vx = fmaf(ax, w.dt, w.damp * vx);
        vy = fmaf(ay, w.dt, w.damp * vy);
        if (p.vmax > 0.0f) {
          const float sp = sqrtf(fmaf(vx, vx, vy * vy));
          if (sp > p.vmax) {
            const float sc = p.vmax / sp;
            vx *= sc;
            vy *= sc;
          }
        }
        x = fmaf(vx, w.dt, x);
        y = fmaf(vy, w.dt, y);
      }
      if (SPIN && rotatable) {
        om = fmaf(0.0f * p.inv_I, w.dt, w.damp * om);
        th = fmaf(om, w.dt, th);
      }
      if (OUT && a.traj && act) {
        float* out = a.traj + (size_t)(t + 1) * (a.traj_xy ? 2 : 6) * N;
        out[e] = x;
        out[N + e] = y;
        if (!a.traj_xy) {
          out[2 * N + e] = vx;
          out[3 * N + e] = vy;
          out[4 * N + e] = th;
          out[5 * N + e] = om;
        }
      }
    };
    float2 bufB[KCH];
#pragma unroll
    for (int k = 0; k < KCH; ++k) bufB[k] = make_float2(0.0f, 0.0f);
    for (int c = 0; c < T; c += 2 * KCH) {
      load_chunk(bufB, c + KCH);
#pragma unroll
      for (int k = 0; k < KCH; ++k)
        if (c + k < T) step(bufA[k], c + k);  // uniform
      if (c + KCH >= T) break;
      load_chunk(bufA, c + 2 * KCH);
#pragma unroll
      for (int k = 0; k < KCH; ++k)
        if (c + KCH + k < T) step(bufB[k], c + KCH + k);
    }
  };
  if (T > 0) {
    // the wavefront-uniform special cases, each its own instance of the loop
    // (the general instance is correct for every wavefront: with spin set the
    // angular update of a wavefront at rest is the identity, with mute set an
    // agent keeps its action, a mass of 1 divides exactly); launches with
    // outputs take the general instance only
    using Y = std::true_type;
    using Nn = std::false_type;
    if (OUT) {
      run(Y{}, Y{}, Nn{});
    } else if (spin || mute) {
      if (spin && mute) run(Y{}, Y{}, Nn{});
      else if (spin) run(Y{}, Nn{}, Nn{});
      else run(Nn{}, Y{}, Nn{});
    } else {
      if (unit) run(Nn{}, Nn{}, Y{});
      else run(Nn{}, Nn{}, Nn{});
    }
  }
  if (act && T > 0) {
    a.state[e] = x;
    a.state[N + e] = y;
    a.state[2 * N + e] = vx;
    a.state[3 * N + e] = vy;
    a.state[4 * N + e] = th;
    a.state[5 * N + e] = om;
  }
}

// Partner-slot bound of the sphere kernel for a plan whose largest
// environment has max_n entities (0: the any-size loop).
int sph_nb(int max_n) {
  for (int nb : {4, 6, 8, 16, 32, 64})
    if (max_n <= nb) return nb;
  return 0;
}

template <int MAXB, int NB>
const void* sph_pick(bool md, bool out) {
  if (md)
    return out ? (const void*)k_rollout_sph<MAXB, NB, true, true>
               : (const void*)k_rollout_sph<MAXB, NB, true, false>;
  return out ? (const void*)k_rollout_sph<MAXB, NB, false, true>
             : (const void*)k_rollout_sph<MAXB, NB, false, false>;
}

const void* sph_kernel256(int nb, bool md, bool out) {
  switch (nb) {
    case 4: return sph_pick<256, 4>(md, out);
    case 6: return sph_pick<256, 6>(md, out);
    case 8: return sph_pick<256, 8>(md, out);
    case 16: return sph_pick<256, 16>(md, out);
    case 32: return sph_pick<256, 32>(md, out);
    case 64: return sph_pick<256, 64>(md, out);
    default: return sph_pick<256, 0>(md, out);
  }
}

template <int NS>
const void* quad_ord_pick(bool md, bool out) {
  if (md)
    return out ? (const void*)k_rollout_quad_ord<true, NS, true>
               : (const void*)k_rollout_quad_ord<true, NS, false>;
  return out ? (const void*)k_rollout_quad_ord<false, NS, true>
             : (const void*)k_rollout_quad_ord<false, NS, false>;
}

template <int NS>
const void* quad_pick(bool md, bool out) {
  if (md)
    return out ? (const void*)k_rollout_quad<true, NS, true>
               : (const void*)k_rollout_quad<true, NS, false>;
  return out ? (const void*)k_rollout_quad<false, NS, true>
             : (const void*)k_rollout_quad<false, NS, false>;
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

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
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

// Debug check of a state [6][N]: an entity holding a NaN or an infinity marks
// its environment (env_off: [n_envs + 1] CSR, found by bisection); the first
// mark of an environment adds one to both counters (cnt[0]: newly marked
// since the last report, cnt[1]: all marked).
__global__ void k_check_nonfinite(const float* __restrict__ state, int N,
                                  const int32_t* __restrict__ env_off, int n_envs,
                                  uint32_t* env_bad, uint32_t* cnt) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    bool ok = true;
#pragma unroll
    for (int f = 0; f < 6; ++f) ok &= isfinite(state[(size_t)f * N + i]);
    if (ok) continue;
    int lo = 0, hi = n_envs - 1;  // the environment b with env_off[b] <= i < env_off[b + 1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (env_off[mid] <= i) lo = mid;
      else hi = mid - 1;
    }
    if (atomicExch(&env_bad[lo], 1u) == 0u) {
      atomicAdd(&cnt[0], 1u);
      atomicAdd(&cnt[1], 1u);
    }
  }
}

// Rest length of joint q from the anchors in state0, with joint_eval's
// arithmetic (the rotation of an entity as the step kernels stage it).
__global__ void k_joint_rest(const float* __restrict__ st, int N, const EntParam* __restrict__ ent,
                             JointK* joints, const uint8_t* __restrict__ from_state, int J) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= J || !from_state[q]) return;
  JointK jk = joints[q];
  float ca = 1.0f, sa = 0.0f, cb = 1.0f, sb = 0.0f;
  if (uses_rotation(ent[jk.a].sf)) sincosf(st[4 * N + jk.a], &sa, &ca);
  if (uses_rotation(ent[jk.b].sf)) sincosf(st[4 * N + jk.b], &sb, &cb);
  const V2 xa = {st[jk.a], st[N + jk.a]}, xb = {st[jk.b], st[N + jk.b]};
  const V2 Pa = vadd(xa, vrot(ca, sa, V2{jk.ax, jk.ay}));
  const V2 Pb = vadd(xb, vrot(cb, sb, V2{jk.bx, jk.by}));
  const V2 dl = vsub(Pa, Pb);
  joints[q].rest = s_sqrt(vdot(dl, dl));
}

int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

// Padding slots of the sphere kernel chosen for a launch shape.
int sph_pad(int block, int max_n) { return block <= 256 ? sph_nb(max_n) : 0; }

const void* rollout_kernel(bool spheres_only, bool quad, bool pq, int block, int max_n,
                           float min_dist, bool out, bool quad_ordered) {
  const bool md = min_dist != 0.0f;
  // quad: max_n carries the most static collidable entities of an environment
  if (quad && quad_ordered)
    return max_n == 0 ? quad_ord_pick<0>(md, out)
                      : (max_n <= 2 ? quad_ord_pick<2>(md, out) : quad_ord_pick<4>(md, out));
  if (quad) return max_n <= 2 ? quad_pick<2>(md, out) : quad_pick<4>(md, out);
  if (spheres_only)
    return block > 256 ? sph_pick<1024, 0>(md, out) : sph_kernel256(sph_pad(block, max_n), md, out);
  if (pq) return block <= 256 ? (const void*)k_rollout<256, true> : (const void*)k_rollout<1024, true>;
  return block <= 256 ? (const void*)k_rollout<256, false> : (const void*)k_rollout<1024, false>;
}

size_t rollout_lds_bytes(int max_stage, bool spheres_only, bool quad, int pq_total, int pq_pairs,
                         int block, int max_n) {
  if (quad) return 0;
  if (!spheres_only && pq_total > 0)
    return (size_t)(3 * max_stage + pq_total) * sizeof(float4) +
           (size_t)max_stage * (4 * sizeof(uint32_t) + 32 * sizeof(uint16_t)) + 24 * sizeof(int) +
           (size_t)(pq_total + pq_pairs) * sizeof(uint32_t);
  if (!spheres_only) return (size_t)max_stage * (3 * sizeof(float4) + sizeof(float));
  return (size_t)(max_stage + sph_pad(block, max_n)) * 3 * sizeof(float2);
}

hipError_t launch_rollout(const StepArgs& a, int groups, int block, bool spheres_only,
                          hipStream_t s) {
  const bool quad = a.quad != nullptr;
  const bool out = a.traj || a.mask || a.forces;
  const int pq_total = a.pq_cap[PQ_CLASSES];
  const void* f = rollout_kernel(spheres_only, quad, pq_total > 0, block, a.max_n, a.w.min_dist, out,
                                 a.quad_ordered != 0);
  const size_t shm =
      rollout_lds_bytes(a.max_stage, spheres_only, quad, pq_total, a.pq_max_pairs, block, a.max_n);
  StepArgs args = a;
  void* kargs[1] = {&args};
  return hipLaunchKernel(f, dim3(groups), dim3(block), kargs, shm, s);
}

hipError_t launch_joint_rest(const float* state0, int N, const EntParam* ent, JointK* joints,
                             const uint8_t* from_state, int J, hipStream_t s) {
  if (J <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_joint_rest, dim3((J + 255) / 256), dim3(256), 0, s, state0, N, ent, joints,
                     from_state, J);
  return hipGetLastError();
}

hipError_t launch_check_nonfinite(const float* state, int N, const int32_t* env_off, int n_envs,
                                  uint32_t* env_bad, uint32_t* cnt, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_nonfinite, dim3(grid_for(N)), dim3(256), 0, s, state, N, env_off,
                     n_envs, env_bad, cnt);
  return hipGetLastError();
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

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
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
