// Adjoint (reverse-mode derivative) of one step of the batched 2D physics
// step of VMAS (Sec. 3 "Core": Eq. 1 forces and semi-implicit Euler with
// damping, Eq. 2 contact force, Eq. 3 torque and angular update).
//
// Given the state s_t, the actions a_t and dL/ds_{t+1}, every lane (one per
// entity of its group, static entities included) computes dL/ds_t for its
// entity and dL/da_t for its agent:
//   1. reverse of the integration (x' = x + v' dt, v' = clamp(v^),
//      v^ = (1 - zeta) v + f/m dt, and the same for theta, omega) gives the
//      adjoints of the total force and torque on the entity, which are
//      shared through LDS;
//   2. every contact and joint the entity takes part in is re-evaluated with
//      dual numbers seeded on the entity's own (x, y, theta): the force on
//      it and the two torques, with their derivatives, are contracted with
//      the force/torque adjoints of both entities of the pair.
// Contact decisions and closest-feature branches are those of the forward
// step (same FP32 values), i.e. the derivative of the piecewise-smooth map
// on the piece the forward pass is on.
//
// One launch runs T reverse steps (t = T-1 .. 0) of a segment whose states
// and actions are stored one step after the other: every entity has a lane,
// which carries its entity's gradient from step to step in registers; T = 1
// is the single-step adjoint.

#include "vmas_geom.h"
#include "vmas_internal.h"

namespace vmas {
namespace {

// Radius of the circle about an entity's centre that holds its shape.
__device__ __forceinline__ float circle_radius(int shape, float d0, float d1) {
  if (shape == SPHERE) return d0;
  if (shape == BOX) return 0.5f * sqrtf(d0 * d0 + d1 * d1);
  return 0.5f * d0;
}

// SPH: sphere-only batch (only the sphere pair code is compiled in); held to
// 128 VGPRs, four wavefronts per SIMD (a few bytes of spills: faster than
// three wavefronts without).
template <int MAXB, bool SPH>
__global__ void __launch_bounds__(MAXB, SPH ? 4 : 1) k_step_backward(BackArgs a) {
  extern __shared__ float4 lds[];
  const int E = a.max_stage;
  float4* pose = lds;          // x, y, cos, sin
  float4* stat = lds + E;      // d0, d1, rho, shape | flags << 8
  float4* adj = lds + 2 * E;   // adjoint of force x, y and torque
  float* brad = reinterpret_cast<float*>(lds + 3 * E);  // bounding radius of each slot
  const int g = blockIdx.x, l = threadIdx.x, B = blockDim.x;
  const int N = a.w.N;
  const int s0 = a.stage_off[g], ns = a.stage_off[g + 1] - s0;
  for (int s = l; s < ns; s += B) {
    const EntParam p = a.ent[a.stage[s0 + s]];
    stat[s] = make_float4(p.d0, p.d1, p.rho, __int_as_float(p.sf));
    brad[s] = circle_radius(p.sf & 0xff, p.d0, p.d1);
  }
  const LaneRec r = a.lanes[(size_t)g * B + l];
  const bool act = r.ent >= 0;
  const WorldK w = a.w;
  EntParam p{};
  float gx = 0, gy = 0, gvx = 0, gvy = 0, gth = 0, gom = 0;
  if (act) {
    const int e = r.ent;
    p = a.ent[e];
    gx = a.gnext[e];
    gy = a.gnext[N + e];
    gvx = a.gnext[2 * N + e];
    gvy = a.gnext[3 * N + e];
    gth = a.gnext[4 * N + e];
    gom = a.gnext[5 * N + e];
  }
  const int shape = p.sf & 0xff, fl = (p.sf >> 8) & 0xff;
  const bool movable = act && (fl & MOVABLE), rotatable = act && (fl & ROTATABLE);
  const bool collide = act && (fl & COLLIDABLE);
  const bool agent = act && r.agent >= 0;
  const int myloc = r.slot - r.lo;
  const float rs = circle_radius(shape, p.d0, p.d1);
  // Bounding circles farther apart than d_min plus a margin far above the
  // FP32 error of the narrow-phase distance cannot be in contact: such
  // partners skip pair_force, which would find no contact (sphere batches
  // test every partner, their test being as cheap as this one).
  auto apart = [&](float x, float y, int q, const float4 P) {
    if (SPH) return false;
    const float reach = w.min_dist + 1e-4f + 1e-5f * (fabsf(x) + fabsf(y));
    const float lim = (rs + brad[q]) + reach;
    const float dx = x - P.x, dy = y - P.y;
    return !(dx * dx + dy * dy <= lim * lim);
  };
  // Sphere batches: the entity of the lane's first staging slot and its
  // joint range are kept in registers, and the state of step t is loaded
  // while step t + 1 is worked on (the barriers wait for LDS traffic only,
  // so the loads stay in flight): the first staging slot's centre and the
  // lane's own centre, and its velocity only under a speed cap (the
  // clamp's adjoint is the one use of it; a sphere's angle and omega enter
  // nothing, omega's step being linear in damping and torque). Without
  // speed caps the states may be positions only (stride 2 N). The general kernel,
  // at the edge of its register budget, loads its state at the top of each
  // step.
  const int e_st = SPH && l < ns ? a.stage[s0 + l] : 0;
  const int jlo = SPH && act ? a.joff[r.ent] : 0, jhi = SPH && act ? a.joff[r.ent + 1] : 0;
  float px = 0, py = 0, sx = 0, sy = 0, svx = 0, svy = 0;
  auto fetch = [&](int t) {
    const float* st = a.state + (size_t)t * a.stride;
    if (l < ns) {
      px = st[e_st];
      py = st[N + e_st];
    }
    if (act) {
      const int e = r.ent;
      sx = st[e];
      sy = st[N + e];
      if (p.vmax > 0.0f) {
        svx = st[2 * N + e];
        svy = st[3 * N + e];
      }
    }
  };
  if (SPH && a.T > 0) fetch(a.T - 1);
  bool uni = false;  // sphere batches: the equal-radius test (set at the first step)
  float dm2u = 0.0f;
  {
    const float dmu = (p.rho + p.rho) + w.min_dist;
    dm2u = __fmul_rn(dmu, dmu);
  }
  for (int t = a.T - 1; t >= 0; --t) {
    const float* state = a.state + (size_t)t * a.stride;
    const float* actions = a.actions ? a.actions + (size_t)t * 2 * w.A : nullptr;
    float* gact = a.gact ? a.gact + (size_t)t * 2 * w.A : nullptr;
    lds_barrier();  // the previous step's readers of pose and adj are done
    if (SPH && t == a.T - 1) {
      // Equal radii (static, once the records are staged): when every
      // partner of every lane of the wavefront collides, moves and has the
      // lane's own radius, each contact distance is the lane's
      // (r + r) + d_min -- the value the per-partner sum gives.
      bool eq = true;
      if (collide)
        for (int q = r.lo; q < r.hi; ++q) {
          const float4 S = stat[q];
          const int of = (__float_as_int(S.w) >> 8) & 0xff;
          eq &= q == r.slot ||
                (S.z == p.rho && (of & COLLIDABLE) && (of & (MOVABLE | ROTATABLE)));
        }
      uni = __builtin_amdgcn_ballot_w64(collide && !eq) == 0;
    }
    float x = 0, y = 0, vx = 0, vy = 0, th = 0;
    if constexpr (SPH) {
      // a sphere's orientation enters no sphere pair
      if (l < ns) pose[l] = make_float4(px, py, 1.0f, 0.0f);
      for (int s = l + B; s < ns; s += B) {
        const int e = a.stage[s0 + s];
        pose[s] = make_float4(state[e], state[N + e], 1.0f, 0.0f);
      }
      x = sx;
      y = sy;
      vx = svx;
      vy = svy;
      if (t > 0) fetch(t - 1);
    } else {
      for (int s = l; s < ns; s += B) {
        const int e = a.stage[s0 + s];
        float cs = 1.0f, sn = 0.0f;
        sincosf(state[4 * N + e], &sn, &cs);
        pose[s] = make_float4(state[e], state[N + e], cs, sn);
      }
      if (act) {
        const int e = r.ent;
        x = state[e];
        y = state[N + e];
        vx = state[2 * N + e];
        vy = state[3 * N + e];
        th = state[4 * N + e];
      }
    }
    float cs = 1.0f, sn = 0.0f;
    if (!SPH && act) sincosf(th, &sn, &cs);
    lds_barrier();

    // 1. Reverse of the integration.
    float Fbx = 0.0f, Fby = 0.0f, Tb = 0.0f;
    float ox = gx, oy = gy, ovx = gvx, ovy = gvy, oth = gth, oom = gom;
    if (movable) {
      // v' = clamp(v^), x' = x + v' dt
      const float vtx = fmaf(gx, w.dt, gvx), vty = fmaf(gy, w.dt, gvy);
      float hx = vtx, hy = vty;  // adjoint of v^
      if (p.vmax > 0.0f) {
        // forward force, exactly as the step computed it (for the clamp)
        const float2 an = agent ? *reinterpret_cast<const float2*>(actions + 2 * (size_t)r.agent)
                                : make_float2(0.0f, 0.0f);
        float fx = an.x + p.mgx, fy = an.y + p.mgy, tq = 0.0f;
        if (collide) {
          GeoT<float> self;
          self.c = V2T<float>{x, y};
          self.cs = cs;
          self.sn = sn;
          self.d0 = p.d0;
          self.d1 = p.d1;
          self.shape = shape;
          for (int q = r.lo; q < r.hi; ++q) {
            if (q == r.slot) continue;
            const float4 S = stat[q];
            const int of = (__float_as_int(S.w) >> 8) & 0xff;
            if (!(of & COLLIDABLE)) continue;
            if (p.excl != -1 && excluded(p.excl, q - r.lo)) continue;
            if (apart(x, y, q, pose[q])) continue;
            pair_force<SPH>(self, p.rho, myloc, pose[q], S, q - r.lo, w, fx, fy, tq);
          }
        }
        for (int jj = SPH ? jlo : a.joff[r.ent]; jj < (SPH ? jhi : a.joff[r.ent + 1]); ++jj) {
          const JointK J = a.joints[a.jlist[jj]];
          const bool is_a = J.a == r.ent;
          const float4 P = pose[r.lo + ((is_a ? J.b : J.a) - r.first)];
          V2T<float> f;
          float ts, to;
          if (joint_eval<float>(V2T<float>{x, y}, cs, sn, V2T<float>{P.x, P.y}, P.z, P.w, is_a, J,
                                w.joint_k, &f, &ts, &to)) {
            fx += f.x;
            fy += f.y;
          }
        }
        const float ux = fmaf(fx * p.inv_m, w.dt, w.damp * vx);
        const float uy = fmaf(fy * p.inv_m, w.dt, w.damp * vy);
        const float sp = sqrtf(fmaf(ux, ux, uy * uy));
        if (sp > p.vmax) {
          // v' = v^ vmax / |v^|: Jacobian (vmax/|v^|) (I - n n^T), symmetric
          const float k = p.vmax / sp, nx = ux / sp, ny = uy / sp;
          const float dot = nx * vtx + ny * vty;
          hx = k * (vtx - nx * dot);
          hy = k * (vty - ny * dot);
        }
      }
      ovx = w.damp * hx;
      ovy = w.damp * hy;
      Fbx = hx * p.inv_m * w.dt;
      Fby = hy * p.inv_m * w.dt;
    }
    if (rotatable) {
      const float wt = fmaf(gth, w.dt, gom);
      oom = w.damp * wt;
      Tb = wt * p.inv_I * w.dt;
    }
    if (act) adj[r.slot] = make_float4(Fbx, Fby, Tb, 0.0f);
    lds_barrier();

    // 2. Pose adjoint through the contacts and joints of the entity.
    if (act) {
      GeoT<D3> self;
      self.c = V2T<D3>{D3(x, 1.0f, 0.0f, 0.0f), D3(y, 0.0f, 1.0f, 0.0f)};
      self.cs = D3(cs, 0.0f, 0.0f, -sn);
      self.sn = D3(sn, 0.0f, 0.0f, cs);
      self.d0 = p.d0;
      self.d1 = p.d1;
      self.shape = shape;
      const bool self_dof = (fl & (MOVABLE | ROTATABLE)) != 0;
      auto contract = [&](const V2T<D3>& f, D3 ts, D3 to, float4 A_self, float4 A_other) {
        const float ax = A_self.x - A_other.x, ay = A_self.y - A_other.y;
        ox += f.x.a * ax + f.y.a * ay + ts.a * A_self.z + to.a * A_other.z;
        oy += f.x.b * ax + f.y.b * ay + ts.b * A_self.z + to.b * A_other.z;
        oth += f.x.c * ax + f.y.c * ay + ts.c * A_self.z + to.c * A_other.z;
      };
      const float4 A_self = adj[r.slot];
      if (SPH && collide) {
        // spheres: the forward's FP32 test of every partner, 8 partners'
        // reads in flight at a time, into a mask of up to 64 partners; then
        // the contacts in partner order (no joints in a sphere batch)
        for (int q0 = r.lo; q0 < r.hi; q0 += 64) {
          const int cnt = min(64, r.hi - q0);
          uint32_t mlo = 0u, mhi = 0u;  // shift_in masks of partners 0..31, 32..63
          if (uni) {
            // every partner collides and moves with the lane's own radius:
            // the partners' positions are all the test reads
            for (int b0 = 0; b0 < cnt; b0 += 8) {
              float2 P[8];
#pragma unroll
              for (int v = 0; v < 8; ++v)
                P[v] = *reinterpret_cast<const float2*>(&pose[min(q0 + b0 + v, r.hi - 1)].x);
#pragma unroll
              for (int v = 0; v < 8; ++v) {
                const int q = q0 + b0 + v;
                const float dx = x - P[v].x, dy = y - P[v].y;
                const bool hit = fmaf(dx, dx, __fmul_rn(dy, dy)) <= dm2u;
                if (b0 < 32) mlo = shift_in(mlo, q < r.hi && q != r.slot && hit);
                else mhi = shift_in(mhi, q < r.hi && q != r.slot && hit);
              }
            }
          } else
          for (int b0 = 0; b0 < cnt; b0 += 8) {
            float4 P[8], S[8];
#pragma unroll
            for (int v = 0; v < 8; ++v) {
              const int q = min(q0 + b0 + v, r.hi - 1);
              P[v] = pose[q];
              S[v] = stat[q];
            }
#pragma unroll
            for (int v = 0; v < 8; ++v) {
              const int q = q0 + b0 + v;
              const int of = (__float_as_int(S[v].w) >> 8) & 0xff;
              const bool elig = q < r.hi && q != r.slot && (of & COLLIDABLE) &&
                                (self_dof || (of & (MOVABLE | ROTATABLE)));
              const float dmin = (p.rho + S[v].z) + w.min_dist;
              const float dx = x - P[v].x, dy = y - P[v].y;
              const bool hit = fmaf(dx, dx, __fmul_rn(dy, dy)) <= __fmul_rn(dmin, dmin);
              if (b0 < 32) mlo = shift_in(mlo, elig && hit);
              else mhi = shift_in(mhi, elig && hit);
            }
          }
          const int nt = min(64, (cnt + 7) & ~7);
          uint64_t hits = ((uint64_t)shifted_bits(mhi, nt - min(32, nt)) << 32) |
                          shifted_bits(mlo, min(32, nt));
          while (hits) {
            const int q = q0 + __builtin_ctzll(hits);
            hits &= hits - 1;
            const float4 P = pose[q];
            const float4 S = stat[q];
            GeoT<D3> other;
            other.c = V2T<D3>{D3(P.x), D3(P.y)};
            other.cs = D3(P.z);
            other.sn = D3(P.w);
            other.d0 = S.x;
            other.d1 = S.y;
            other.shape = SPHERE;
            V2T<D3> f;
            D3 ts, to;
            pair_grad<SPH>(self, p.rho, myloc < q - r.lo, other, S.z, w, &f, &ts, &to);
            contract(f, ts, to, A_self, adj[q]);
          }
        }
      } else if (collide) {
        GeoT<float> selff;
        selff.c = V2T<float>{x, y};
        selff.cs = cs;
        selff.sn = sn;
        selff.d0 = p.d0;
        selff.d1 = p.d1;
        selff.shape = shape;
        for (int q = r.lo; q < r.hi; ++q) {
          if (q == r.slot) continue;
          const float4 S = stat[q];
          const int of = (__float_as_int(S.w) >> 8) & 0xff;
          if (!(of & COLLIDABLE)) continue;
          if (!self_dof && !(of & (MOVABLE | ROTATABLE))) continue;
          if (p.excl != -1 && excluded(p.excl, q - r.lo)) continue;
          const float4 P = pose[q];
          if (apart(x, y, q, P)) continue;
          float fx = 0.0f, fy = 0.0f, tq = 0.0f;
          if (!pair_force<SPH>(selff, p.rho, myloc, P, S, q - r.lo, w, fx, fy, tq)) continue;
          GeoT<D3> other;
          other.c = V2T<D3>{D3(P.x), D3(P.y)};
          other.cs = D3(P.z);
          other.sn = D3(P.w);
          other.d0 = S.x;
          other.d1 = S.y;
          other.shape = __float_as_int(S.w) & 0xff;
          V2T<D3> f;
          D3 ts, to;
          pair_grad<SPH>(self, p.rho, myloc < q - r.lo, other, S.z, w, &f, &ts, &to);
          contract(f, ts, to, A_self, adj[q]);
        }
      }
      for (int jj = SPH ? jlo : a.joff[r.ent]; jj < (SPH ? jhi : a.joff[r.ent + 1]); ++jj) {
        const JointK J = a.joints[a.jlist[jj]];
        const bool is_a = J.a == r.ent;
        const int q = r.lo + ((is_a ? J.b : J.a) - r.first);
        const float4 P = pose[q];
        V2T<D3> f;
        D3 ts, to;
        if (joint_eval<D3>(self.c, self.cs, self.sn, V2T<D3>{D3(P.x), D3(P.y)}, D3(P.z), D3(P.w),
                           is_a, J, w.joint_k, &f, &ts, &to))
          contract(f, ts, to, A_self, adj[q]);
      }
      if (agent && gact) {
        gact[2 * (size_t)r.agent] = Fbx;
        gact[2 * (size_t)r.agent + 1] = Fby;
      }
    }
    gx = ox;
    gy = oy;
    gvx = ovx;
    gvy = ovy;
    gth = oth;
    gom = oom;
  }
  if (act) {
    const int e = r.ent;
    a.gstate[e] = gx;
    a.gstate[N + e] = gy;
    a.gstate[2 * N + e] = gvx;
    a.gstate[3 * N + e] = gvy;
    a.gstate[4 * N + e] = gth;
    a.gstate[5 * N + e] = gom;
  }
}

}  // namespace

hipError_t launch_backward(const BackArgs& a, int groups, int block, bool spheres_only,
                           hipStream_t s) {
  const size_t shm = (size_t)a.max_stage * (3 * sizeof(float4) + sizeof(float));
  if (block <= 256) {
    if (spheres_only)
      hipLaunchKernelGGL((k_step_backward<256, true>), dim3(groups), dim3(block), shm, s, a);
    else
      hipLaunchKernelGGL((k_step_backward<256, false>), dim3(groups), dim3(block), shm, s, a);
  } else {
    if (spheres_only)
      hipLaunchKernelGGL((k_step_backward<1024, true>), dim3(groups), dim3(block), shm, s, a);
    else
      hipLaunchKernelGGL((k_step_backward<1024, false>), dim3(groups), dim3(block), shm, s, a);
  }
  return hipGetLastError();
}

}  // namespace vmas
