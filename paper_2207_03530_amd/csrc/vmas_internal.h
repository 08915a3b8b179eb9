// Internal declarations shared by the host runtime and the HIP kernels of
// the batched 2D physics step (VMAS, Sec. 3 "Core", Eq. 1-3). Not part of the
// public boundary (include/vmas.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vmas.h"

namespace vmas {

enum : int { SPHERE = 0, BOX = 1, LINE = 2 };
enum : int { MOVABLE = 1, ROTATABLE = 2, COLLIDABLE = 4 };
// EntParam.sf bit: the entity's orientation enters the geometry of a step
// (boxes and segments always; a sphere only when a joint anchors it off its
// centre). Entities without it use the identity rotation, which no routine
// that reads them can tell from their own.
enum : int { SF_ROTATES = 1 << 16 };
__host__ __device__ inline bool uses_rotation(int sf) { return (sf & SF_ROTATES) != 0; }

// Static per-entity parameters, one 48-byte record per entity.
struct EntParam {
  float d0, d1;        // sphere (r, 0), box (lx, ly), line (L, 0)
  float inv_m, inv_I;  // 1/m, 1/I
  float vmax;          // <= 0: no speed cap
  float rho;           // radius added to d_min: r for spheres, 0 otherwise
  float mgx, mgy;      // gravity force m g (0 unless movable)
  int32_t sf;          // shape | flags << 8 | SF_ROTATES
  int32_t excl;        // up to 4 environment-local partner indices (one byte
                       // each, 0xff = none) whose contact a joint switches off
  int32_t pad[2];
};

// The fields of EntParam that the quad schedules read, in one 16-byte
// record per entity (a third of EntParam's bytes).
struct alignas(16) SphRec {
  float rho;     // radius added to d_min
  float inv_m;   // 1/m
  float vmax;    // <= 0: no speed cap
  int32_t sf;    // shape | flags << 8 | SF_ROTATES
};

// One lane of a launch group: the entity it integrates and where it sits.
struct LaneRec {
  int32_t ent;    // global entity id, -1 = idle lane
  int32_t slot;   // LDS slot of the entity inside the group
  int32_t lo;     // LDS slot of the first entity of its environment
  int32_t hi;     // one past the last
  int32_t agent;  // action row, -1 = not an agent
  int32_t env;    // environment id
  int32_t first;  // global id of the first entity of its environment
  int32_t pad;
};

// A joint: linear spring between body-frame anchors of entities a and b.
struct JointK {
  int32_t a, b;
  float ax, ay, bx, by;
  float rest;
  float pad;
};

// World constants folded for the kernels.
struct WorldK {
  float dt, damp;      // delta t, 1 - zeta
  float gx, gy;        // g
  float ck, inv_k;     // c * k, 1 / k
  float min_dist;
  float joint_k;
  int32_t A;           // total agents (row stride of one action step)
  int32_t N;           // total entities
  int32_t pad[2];
};

// One environment of the quad schedule (sphere-only batches whose
// environments have at most 4 entities that move or rotate and at most 4
// static collidable ones): its movers sit on one aligned quad of lanes.
struct QuadEnv {
  int32_t agent_row;    // action row of the environment's first agent
  int32_t n_agents;     // agents are local entities 0 .. n_agents - 1
  int8_t lane_loc[4];   // local index of the entity on quad lane q, -1: idle lane
  int8_t stat_loc[4];   // local index of the s-th static collidable entity, -1: none
};

// Arguments of the step / rollout kernels.
struct StepArgs {
  float* state;            // [6][N]
  const float* actions;    // [T][A][2] or NULL (drawn in kernel)
  uint64_t key;            // SplitMix64 key of the action stream
  int32_t t0, T;
  float* traj;             // [T+1][6][N] or NULL
  uint8_t* mask;           // [P] or NULL (last step)
  float* forces;           // [3][N] or NULL (last step)
  const EntParam* ent;     // [N]
  const LaneRec* lanes;    // [groups * block]
  const int32_t* stage_off;  // [groups + 1]
  const int32_t* stage;      // staged global entity ids
  const int32_t* joff;       // [N + 1] per-entity joint lists
  const int32_t* jlist;
  const JointK* joints;
  const int64_t* pair_off;   // [n_envs] first mask slot of each environment
  const int32_t* grp_maxn;   // [groups] size of the largest environment of each group
  int32_t max_stage;         // LDS slots per group
  int32_t max_n;             // size of the largest environment of the plan
  const QuadEnv* quad;       // [n_envs] quad schedule, or NULL
  const int32_t* env_off;    // [n_envs + 1] first entity of each environment
  int32_t n_envs;
  int32_t quad_ordered;      // quad schedule whose movers are local 0..m-1 on lanes 0..m-1
  // pair-queue plans (batches with boxes or segments, environments of at
  // most 32 entities): queue capacity per pair class (sphere-box,
  // sphere-segment, box-box, box-segment, segment-segment) and their sum;
  // all 0 for the other plans
  int32_t pq_cap[6];
  // eligible pairs of each group (collidable, one side with a lane, not
  // switched off by a joint), packed slot_lo | slot_hi << 11 | lo << 22 |
  // hi << 27, groups back to back
  const uint32_t* pq_pairs;
  const int32_t* pq_pair_off;  // [groups + 1]
  int32_t pq_max_pairs;        // most pairs of one group (at most 32 x block)
  int32_t n_list;              // quad schedules: environments in env_list
  const int32_t* env_list;     // quad schedules on a subset of the environments
                               // ([n_list] environment ids), or NULL: all
  const SphRec* sph;           // [N] compact records of EntParam's fields
  int32_t sph_only;            // 1: no joints, and every entity has zero gravity
                               // force (+0) and a finite 1/I >= 0: a sphere is then
                               // fully described by its SphRec (d0 = rho, d1 = 0,
                               // no joint exclusions, m g = 0; 0 x 1/I = +0)
  int32_t traj_xy;             // 1: the trajectory holds positions only, compact:
                               // [T+1][2][N] (x, y of every slot)
  WorldK w;
};

// Waits until this wavefront's global loads have returned (s_waitcnt
// vmcnt(0), the other counters untouched). Placed after the first action
// chunk is loaded, it keeps that load from being outstanding at the top of
// the step loop, where the compiler would otherwise wait for every load in
// flight -- the next chunk's prefetch included -- at the start of each chunk.
__device__ __forceinline__ void wait_global_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Workgroup barrier for LDS traffic only: waits for this wavefront's LDS
// operations, then meets the other wavefronts. Unlike __syncthreads() it does
// not wait for outstanding global loads (prefetched actions stay in flight).
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Arguments of the adjoint kernel (one step backwards).
struct BackArgs {
  const float* state;      // [T][6][N] states t0 .. t0 + T - 1 (sphere batches
                           // without speed caps: [T][2][N] positions suffice)
  int64_t stride;          // floats from one step's state to the next (6 N or 2 N)
  const float* actions;    // [T][A][2] actions of the same steps
  const float* gnext;      // [6][N] dL/ds_{t0+T}
  float* gstate;           // [6][N] dL/ds_t0
  float* gact;             // [T][A][2] or NULL
  const EntParam* ent;
  const LaneRec* lanes;
  const int32_t* stage_off;
  const int32_t* stage;
  const int32_t* joff;
  const int32_t* jlist;
  const JointK* joints;
  int32_t max_stage;
  int32_t T;               // reverse steps of the launch (>= 1)
  WorldK w;
};

// Host-side launchers (vmas_kernels.hip).
hipError_t launch_rollout(const StepArgs& a, int groups, int block, bool spheres_only,
                          hipStream_t s);
hipError_t launch_backward(const BackArgs& a, int groups, int block, bool spheres_only,
                           hipStream_t s);
// Device function of the rollout kernel launched by launch_rollout (for
// explicit graph construction) and its dynamic LDS size.
const void* rollout_kernel(bool spheres_only, bool quad, bool pq, int block, int max_n,
                           float min_dist, bool out, bool quad_ordered = false);
size_t rollout_lds_bytes(int max_stage, bool spheres_only, bool quad, int pq_total, int pq_pairs,
                         int block, int max_n);
// Rest lengths of the joints marked in from_state ([J], 1 = take the anchor
// distance in state0), evaluated with the step's own FP32 arithmetic, so
// such a joint exerts exactly no force in state0. Writes joints[q].rest.
hipError_t launch_joint_rest(const float* state0, int N, const EntParam* ent, JointK* joints,
                             const uint8_t* from_state, int J, hipStream_t s);
hipError_t launch_check_nonfinite(const float* state, int N, const int32_t* env_off, int n_envs,
                                  uint32_t* env_bad, uint32_t* cnt, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, int64_t n, hipStream_t s);
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_replicate(const float* src, float* dst, int64_t n, int copies, hipStream_t s);
hipError_t launch_axpy_zero(float* p, int64_t n, hipStream_t s);

hipError_t launch_pair_features(const float* state, const EntParam* ent, const int32_t* env_off,
                                const int64_t* pair_off, const int64_t* slots, int64_t m,
                                float band, float* feat, float* target, uint8_t* flags,
                                int n_envs, const WorldK& w, hipStream_t s);
// out_idx: row r of the output goes to Y[out_idx[r]] (NULL: to Y[r])
vmas_status mlp_forward_counted(vmas_mlp* m, const float* X, int64_t max_n, const int32_t* d_n,
                                const int32_t* out_idx, float* Y, hipStream_t s);
hipError_t launch_candidate_features(const StepArgs& a, int groups, int block, float band,
                                     float* feat, int32_t* slot_of, int32_t* count,
                                     bool spheres_only, hipStream_t s);
hipError_t launch_step_surrogate(const StepArgs& a, const float* yhat_slot,
                                 float band, float frac, int32_t* n_fallback, int groups,
                                 int block, bool spheres_only, hipStream_t s);

// Host-side SplitMix64 key of (seed, stream): mix64(seed + (stream + 1) * golden).
uint64_t action_key(uint64_t seed);

}  // namespace vmas
