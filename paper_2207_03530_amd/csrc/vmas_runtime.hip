// Host runtime of the C boundary (include/vmas.h): argument validation,
// device copies of the static batch description, launch plans, the cached
// rollout graph, the autotuner and the checkpointed adjoint driver.
//
// Launch plans. A plan packs whole environments into workgroups of `block`
// lanes: every entity that can move or rotate gets a lane, every entity of
// the group is staged in LDS. Plans differ in the block size and in whether
// environments are packed in their natural order or sorted by size (which
// keeps the lanes of one wavefront on environments of similar size when
// sizes are uneven); sphere batches whose environments have at most 4 movers
// also get the quad plan (one lane quad per environment), and batches with
// boxes or segments (environments of at most 32 entities) the pair-queue
// plans (a static list of each workgroup's pairs; every pair tested and
// evaluated once). The per-lane arithmetic does not depend on the packing, so
// every plan returns the same bits; the autotuner picks the fastest on the
// caller's workload. Two more plans are not schedules: the adjoint plan (every
// entity has a lane) and the 1024-lane plan of the surrogate's candidate
// kernel.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "vmas.h"
#include "vmas_internal.h"

using namespace vmas;

namespace {

thread_local std::string g_err;

vmas_status fail(vmas_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(VMAS_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

struct Plan {
  std::string name;
  int block = 64;
  bool sorted = false;
  bool all_lanes = false;  // every entity gets a lane (adjoint plans)
  bool valid = false;
  int groups = 0;
  int max_stage = 0;
  int max_n = 0;  // largest environment of the plan
  bool quad = false;          // quad schedule (d_quad), no lane records
  bool quad_ordered = false;  // quad schedule with movers at local 0..m-1 (ordered partners)
  bool pq = false;            // pair-queue variant of the entity-lane kernel
  int32_t pq_cap[6] = {0, 0, 0, 0, 0, 0};  // queue capacity per pair class, then the sum
  uint32_t* d_pq_pairs = nullptr;   // eligible pairs of each group
  int32_t* d_pq_pair_off = nullptr;
  int pq_max_pairs = 0;
  QuadEnv* d_quad = nullptr;
  int32_t* d_env_list = nullptr;  // quad plans on a subset of the environments
  int n_list = 0;
  bool composite = false;  // size-bucketed plan: the chosen part of every bucket, launched at once
  LaneRec* d_lanes = nullptr;
  int32_t* d_stage_off = nullptr;
  int32_t* d_stage = nullptr;
  int32_t* d_maxn = nullptr;  // largest environment of each group
};

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace

namespace vmas {
vmas_status set_error(vmas_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}
}  // namespace vmas

// One bucket of environment sizes of a size-bucketed plan: its candidate
// plans (each over the bucket's environments only) and the chosen one.
struct Bucket {
  int lo = 0, hi = 0;  // environment sizes lo .. hi
  std::vector<Plan> cands;
  int choice = 0;
};

struct vmas_batch {
  int device = 0;
  int n_envs = 0, N = 0, A = 0, J = 0, max_env = 0;
  int64_t P = 0;
  bool spheres_only = true;
  bool all_move = true;  // every entity moves or turns: every plan gives each a lane
  bool any_vmax = false;  // some entity has a speed cap
  WorldK w{};
  EntParam* d_ent = nullptr;
  SphRec* d_sph = nullptr;
  bool sph_only = false;
  int32_t* d_joff = nullptr;
  int32_t* d_jlist = nullptr;
  JointK* d_joints = nullptr;
  int64_t* d_pair_off = nullptr;
  int32_t* d_env_off = nullptr;
  // surrogate workspace: features [P][12], MLP outputs [P][2], flags [P]
  float* d_feat = nullptr;
  float* d_yhat = nullptr;
  int32_t* d_rows = nullptr;   // [P] pair slot of each candidate row, then [1] the count
  std::vector<Plan> plans;
  int cur = 0;
  int lane_plan = 0;  // entity-lane plan of the surrogate kernels: the largest block up to 256
  Plan back;  // adjoint plan: every entity has a lane
  Plan cand;  // 1024-lane plan of the surrogate's candidate kernel (fewer workgroups
              // take rows from the one shared counter)
  // checkpoint workspace of the adjoint driver and the autotuner scratch
  float* d_ws = nullptr;
  size_t ws_floats = 0;
  // cached rollout graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int graph_T = -1, graph_plan = -1;
  int graph_gen = -1, plan_gen = 0;  // plan_gen changes with a bucketed plan's choices
  bool graph_drawn = false;
  // size-bucketed plan (sphere batches of uneven sizes): buckets, and the
  // side streams and events on which its parts run at the same time
  std::vector<Bucket> buckets;
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> side_done;
  hipEvent_t fork = nullptr;
  std::vector<hipGraphNode_t> gnodes;  // graph nodes of a composite plan
  std::string tune_key;                // autotune cache key
  bool tune_cached = false;            // the last autotune came from the cache
  // debug check of the state after every step call (VMAS_DEBUG_NONFINITE)
  bool debug_nonfinite = false;
  uint32_t* d_bad = nullptr;      // [n_envs] 1: the environment reached a non-finite state
  uint32_t* d_bad_cnt = nullptr;  // [2] marked since the last report, marked in all
};

namespace {

void free_plan(Plan& p) {
  if (p.d_lanes) (void)hipFree(p.d_lanes);
  if (p.d_stage_off) (void)hipFree(p.d_stage_off);
  if (p.d_stage) (void)hipFree(p.d_stage);
  if (p.d_maxn) (void)hipFree(p.d_maxn);
  if (p.d_quad) (void)hipFree(p.d_quad);
  if (p.d_pq_pairs) (void)hipFree(p.d_pq_pairs);
  if (p.d_pq_pair_off) (void)hipFree(p.d_pq_pair_off);
  if (p.d_env_list) (void)hipFree(p.d_env_list);
  p.d_env_list = nullptr;
  p.d_pq_pairs = nullptr;
  p.d_pq_pair_off = nullptr;
  p.d_quad = nullptr;
  p.d_maxn = nullptr;
  p.d_lanes = nullptr;
  p.d_stage_off = nullptr;
  p.d_stage = nullptr;
}

void free_batch(vmas_batch* b) {
  if (!b) return;
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto& p : b->plans) free_plan(p);
  for (auto& bk : b->buckets)
    for (auto& p : bk.cands) free_plan(p);
  for (hipStream_t st : b->side) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : b->side_done) (void)hipEventDestroy(ev);
  if (b->fork) (void)hipEventDestroy(b->fork);
  free_plan(b->back);
  free_plan(b->cand);
  if (b->d_ent) (void)hipFree(b->d_ent);
  if (b->d_sph) (void)hipFree(b->d_sph);
  if (b->d_joff) (void)hipFree(b->d_joff);
  if (b->d_jlist) (void)hipFree(b->d_jlist);
  if (b->d_joints) (void)hipFree(b->d_joints);
  if (b->d_pair_off) (void)hipFree(b->d_pair_off);
  if (b->d_env_off) (void)hipFree(b->d_env_off);
  if (b->d_feat) (void)hipFree(b->d_feat);
  if (b->d_yhat) (void)hipFree(b->d_yhat);
  if (b->d_rows) (void)hipFree(b->d_rows);
  if (b->d_ws) (void)hipFree(b->d_ws);
  if (b->d_bad) (void)hipFree(b->d_bad);
  if (b->d_bad_cnt) (void)hipFree(b->d_bad_cnt);
  delete b;
}

template <class T> vmas_status upload(T** dst, const T* src, size_t n) {
  *dst = nullptr;
  if (n == 0) return VMAS_OK;
  hipError_t e = hipMalloc((void**)dst, n * sizeof(T));
  if (e != hipSuccess) {
    *dst = nullptr;
    return fail(e == hipErrorOutOfMemory ? VMAS_ERR_OUT_OF_MEMORY : VMAS_ERR_DEVICE,
                "hipMalloc(%zu bytes) failed: %s", n * sizeof(T), hipGetErrorString(e));
  }
  e = hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(VMAS_ERR_DEVICE, "hipMemcpy failed: %s", hipGetErrorString(e));
  return VMAS_OK;
}

inline bool finite(float x) { return std::isfinite(x); }

double default_inertia(int shape, double m, double d0, double d1) {
  if (shape == SPHERE) return m * d0 * d0 / 2.0;
  if (shape == BOX) return m * (d0 * d0 + d1 * d1) / 12.0;
  return m * d0 * d0 / 12.0;
}

// Host description after validation.
struct HostDesc {
  std::vector<int32_t> off, nag;
  std::vector<int64_t> agent_off;  // first action row of each environment
  std::vector<int> env_of;
};

vmas_status validate(const vmas_world_params* pr, const vmas_batch_desc* d, HostDesc& h) {
  if (!pr || !d) return fail(VMAS_ERR_INVALID_ARGUMENT, "params and desc must not be NULL");
  if (!(finite(pr->dt) && pr->dt > 0))
    return fail(VMAS_ERR_INVALID_ARGUMENT, "dt must be finite and > 0");
  if (!(finite(pr->drag) && pr->drag >= 0 && pr->drag <= 1))
    return fail(VMAS_ERR_INVALID_ARGUMENT, "drag must be in [0, 1]");
  if (!(finite(pr->gravity[0]) && finite(pr->gravity[1])))
    return fail(VMAS_ERR_INVALID_ARGUMENT, "gravity must be finite");
  if (!(finite(pr->contact_force) && pr->contact_force >= 0))
    return fail(VMAS_ERR_INVALID_ARGUMENT, "contact_force must be finite and >= 0");
  if (!(finite(pr->contact_margin) && pr->contact_margin > 0))
    return fail(VMAS_ERR_INVALID_ARGUMENT, "contact_margin must be finite and > 0");
  if (!(finite(pr->min_dist) && pr->min_dist >= 0))
    return fail(VMAS_ERR_INVALID_ARGUMENT, "min_dist must be finite and >= 0");
  if (!(finite(pr->joint_stiffness) && pr->joint_stiffness >= 0))
    return fail(VMAS_ERR_INVALID_ARGUMENT, "joint_stiffness must be finite and >= 0");
  if (pr->flags & ~(uint32_t)VMAS_DEBUG_NONFINITE)
    return fail(VMAS_ERR_INVALID_ARGUMENT, "params.flags has unknown bits (0x%x)", pr->flags);
  if (d->n_envs < 1) return fail(VMAS_ERR_INVALID_ARGUMENT, "n_envs must be >= 1");
  const int E = d->n_envs;
  h.off.assign(E + 1, 0);
  if (d->env_offset) {
    if (d->env_offset[0] != 0) return fail(VMAS_ERR_INVALID_ARGUMENT, "env_offset[0] must be 0");
    for (int b = 0; b < E; ++b) {
      if (d->env_offset[b + 1] < d->env_offset[b])
        return fail(VMAS_ERR_INVALID_ARGUMENT, "env_offset must be non-decreasing (env %d)", b);
      h.off[b + 1] = d->env_offset[b + 1];
    }
  } else {
    if (d->n_per_env < 0) return fail(VMAS_ERR_INVALID_ARGUMENT, "n_per_env must be >= 0");
    if ((int64_t)d->n_per_env * E > INT32_MAX)
      return fail(VMAS_ERR_INVALID_ARGUMENT, "too many entities");
    for (int b = 0; b <= E; ++b) h.off[b] = b * d->n_per_env;
  }
  const int N = h.off[E];
  if (N < 1) return fail(VMAS_ERR_INVALID_ARGUMENT, "the batch has no entity");
  if (!d->n_agents || !d->shape || !d->dims || !d->mass || !d->flags)
    return fail(VMAS_ERR_INVALID_ARGUMENT, "n_agents, shape, dims, mass and flags are required");
  h.nag.assign(d->n_agents, d->n_agents + E);
  int64_t A = 0;
  for (int b = 0; b < E; ++b) {
    const int n = h.off[b + 1] - h.off[b];
    if (h.nag[b] < 0 || h.nag[b] > n)
      return fail(VMAS_ERR_INVALID_ARGUMENT, "n_agents[%d] = %d outside [0, %d]", b, h.nag[b], n);
    A += h.nag[b];
  }
  if (A * 2 > INT32_MAX) return fail(VMAS_ERR_INVALID_ARGUMENT, "too many agents");
  h.agent_off.assign(E, 0);
  for (int b = 1; b < E; ++b) h.agent_off[b] = h.agent_off[b - 1] + h.nag[b - 1];
  for (int i = 0; i < N; ++i) {
    const int s = d->shape[i];
    if (s != SPHERE && s != BOX && s != LINE)
      return fail(VMAS_ERR_INVALID_ARGUMENT, "shape[%d] = %d is not a vmas_shape", i, s);
    if (d->flags[i] & ~7) return fail(VMAS_ERR_INVALID_ARGUMENT, "flags[%d] has unknown bits", i);
    const float d0 = d->dims[2 * i], d1 = d->dims[2 * i + 1];
    if (!(finite(d0) && d0 > 0)) return fail(VMAS_ERR_INVALID_ARGUMENT, "dims[%d][0] must be > 0", i);
    if (s == BOX && !(finite(d1) && d1 > 0))
      return fail(VMAS_ERR_INVALID_ARGUMENT, "dims[%d][1] of a box must be > 0", i);
    const bool dof = (d->flags[i] & (MOVABLE | ROTATABLE)) != 0;
    if (dof && !(finite(d->mass[i]) && d->mass[i] > 0))
      return fail(VMAS_ERR_INVALID_ARGUMENT, "mass[%d] must be > 0 for a movable or rotatable entity", i);
    if (d->inertia && !finite(d->inertia[i]))
      return fail(VMAS_ERR_INVALID_ARGUMENT, "inertia[%d] must be finite", i);
    if (d->max_speed && !finite(d->max_speed[i]))
      return fail(VMAS_ERR_INVALID_ARGUMENT, "max_speed[%d] must be finite", i);
  }
  if (d->n_joints < 0) return fail(VMAS_ERR_INVALID_ARGUMENT, "n_joints must be >= 0");
  h.env_of.assign(N, 0);
  for (int b = 0; b < E; ++b)
    for (int i = h.off[b]; i < h.off[b + 1]; ++i) h.env_of[i] = b;
  if (d->n_joints > 0) {
    if (!d->joint_a || !d->joint_b || !d->joint_anchor_a || !d->joint_anchor_b || !d->joint_rest)
      return fail(VMAS_ERR_INVALID_ARGUMENT, "joint arrays are required when n_joints > 0");
    for (int q = 0; q < d->n_joints; ++q) {
      const int a = d->joint_a[q], c = d->joint_b[q];
      if (a < 0 || a >= N || c < 0 || c >= N || a == c)
        return fail(VMAS_ERR_INVALID_ARGUMENT, "joint %d has bad entity ids (%d, %d)", q, a, c);
      if (h.env_of[a] != h.env_of[c])
        return fail(VMAS_ERR_INVALID_ARGUMENT, "joint %d links two environments", q);
      for (int k = 0; k < 2; ++k)
        if (!finite(d->joint_anchor_a[2 * q + k]) || !finite(d->joint_anchor_b[2 * q + k]))
          return fail(VMAS_ERR_INVALID_ARGUMENT, "joint %d anchors must be finite", q);
      if (!finite(d->joint_rest[q]))
        return fail(VMAS_ERR_INVALID_ARGUMENT, "joint %d rest length must be finite", q);
      if (d->joint_rest[q] < 0 && !d->init_state)
        return fail(VMAS_ERR_INVALID_ARGUMENT,
                    "joint %d has rest < 0 (from the initial state) but init_state is NULL", q);
    }
  }
  return VMAS_OK;
}

// Builds one launch plan on the host and uploads it.
// Queue capacity per pair class of the pair-queue plans: the most eligible
// pairs of the class in one group, at most PQ_CAP_PER_ENV per environment of
// the group and PQ_CAP_MAX in all (pairs beyond a full queue are evaluated by
// both of their lanes, so the capacity trades LDS, hence resident
// workgroups, against that slower path).
constexpr int PQ_CAP_PER_ENV = 32;
constexpr int PQ_CAP_MAX = 256;
constexpr size_t PQ_LDS_MAX = 80 * 1024;

int pq_pair_class(int sa, int sb) {
  const int lo = std::min(sa, sb), hi = std::max(sa, sb);
  if (lo == SPHERE) return hi == BOX ? 0 : 1;
  if (lo == BOX) return hi == BOX ? 2 : 3;
  return 4;
}

// Host twin of the kernels' excluded(): local indices are stored below 255,
// a 0xff byte is unused.
bool excludes(int32_t excl, int loc) {
  if (excl == -1 || loc < 0 || loc >= 255) return false;
  for (int k = 0; k < 4; ++k)
    if ((((uint32_t)excl >> (8 * k)) & 0xffu) == (uint32_t)loc) return true;
  return false;
}

// pq_ent: entity table of a pair-queue plan (NULL for the other plans).
vmas_status build_plan(vmas_batch* b, const HostDesc& h, const std::vector<uint8_t>& shape,
                       const std::vector<uint8_t>& flags, int block, bool sorted, Plan& p,
                       bool all_lanes = false, const std::vector<EntParam>* pq_ent = nullptr,
                       const std::vector<char>* subset = nullptr, int lane_cap = 0) {
  p.block = block;
  p.sorted = sorted;
  p.all_lanes = all_lanes;
  p.pq = pq_ent != nullptr;
  p.name = std::string(all_lanes ? "adjoint-lane/" : (p.pq ? "pair-queue/" : "entity-lane/")) +
           std::to_string(block) + (sorted ? "/size-sorted" : "/natural") +
           (lane_cap > 0 ? "/even" : "");
  const int fill = lane_cap > 0 ? std::min(lane_cap, block) : block;
  const int E = b->n_envs;
  auto has_lane = [&](int i) { return all_lanes || (flags[i] & (MOVABLE | ROTATABLE)) != 0; };
  std::vector<int> active(E, 0);
  for (int e = 0; e < E; ++e)
    for (int i = h.off[e]; i < h.off[e + 1]; ++i) active[e] += has_lane(i);
  std::vector<int> order;
  for (int e = 0; e < E; ++e)
    if (active[e] > 0 && (all_lanes ? h.off[e + 1] > h.off[e] : true) && (!subset || (*subset)[e]))
      order.push_back(e);
  if (sorted)
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return (h.off[x + 1] - h.off[x]) > (h.off[y + 1] - h.off[y]);
    });
  const int stage_cap = std::min(1260, std::max(4 * block, b->max_env));  // 52 B of LDS per slot
  std::vector<std::vector<int>> groups;
  int lanes = 0, staged = 0;
  for (int e : order) {
    const int n = h.off[e + 1] - h.off[e];
    if (active[e] > block || n > stage_cap) {
      p.valid = false;
      return VMAS_OK;
    }
    if (groups.empty() || lanes + active[e] > fill || staged + n > stage_cap) {
      groups.emplace_back();
      lanes = 0;
      staged = 0;
    }
    groups.back().push_back(e);
    lanes += active[e];
    staged += n;
  }
  const int G = (int)groups.size();
  std::vector<LaneRec> lane((size_t)std::max(G, 1) * block);
  std::vector<int32_t> stage_off(G + 1, 0), stage, maxn(std::max(G, 1), 0);
  int max_stage = 1;
  for (int g = 0; g < G; ++g) {
    std::vector<LaneRec> recs;
    int slot = 0;
    for (int e : groups[g]) {
      const int lo = slot, n = h.off[e + 1] - h.off[e];
      maxn[g] = std::max(maxn[g], n);
      const int agent_row = (int)h.agent_off[e];
      for (int i = h.off[e]; i < h.off[e + 1]; ++i, ++slot) {
        stage.push_back(i);
        if (has_lane(i)) {
          LaneRec r;
          r.ent = i;
          r.slot = slot;
          r.lo = lo;
          r.hi = lo + n;
          const int loc = i - h.off[e];
          r.agent = loc < h.nag[e] ? agent_row + loc : -1;
          r.env = e;
          r.first = h.off[e];
          r.pad = 0;
          recs.push_back(r);
        }
      }
    }
    // shape-coherent lanes: spheres, then boxes, then lines
    std::stable_sort(recs.begin(), recs.end(),
                     [&](const LaneRec& x, const LaneRec& y) { return shape[x.ent] < shape[y.ent]; });
    for (int l = 0; l < block; ++l) {
      LaneRec r{};
      r.ent = -1;
      if (l < (int)recs.size()) r = recs[l];
      lane[(size_t)g * block + l] = r;
    }
    stage_off[g + 1] = (int32_t)stage.size();
    max_stage = std::max(max_stage, slot);
  }
  p.groups = G;
  p.max_stage = max_stage;
  p.max_n = 0;
  for (int32_t m : maxn) p.max_n = std::max(p.max_n, (int)m);
  if (p.pq) {
    // environments of at most 32 entities; capacities from the eligible
    // pairs (both collidable, one with a lane, no joint exclusion, not
    // sphere-sphere) of each group
    if (p.max_n > 32) {
      p.valid = false;
      return VMAS_OK;
    }
    const std::vector<EntParam>& ent = *pq_ent;
    int cap[5] = {0, 0, 0, 0, 0};
    std::vector<uint32_t> pairs;
    std::vector<int32_t> pair_off(G + 1, 0);
    for (int g = 0; g < G; ++g) {
      int cnt[5] = {0, 0, 0, 0, 0};
      int slot = 0;  // LDS slot of the environment's first entity
      for (int e : groups[g]) {
        const int n = h.off[e + 1] - h.off[e];
        for (int i = h.off[e]; i < h.off[e + 1]; ++i)
          for (int j = i + 1; j < h.off[e + 1]; ++j) {
            if (!(flags[i] & COLLIDABLE) || !(flags[j] & COLLIDABLE)) continue;
            if (!(flags[i] & (MOVABLE | ROTATABLE)) && !(flags[j] & (MOVABLE | ROTATABLE))) continue;
            const int li = i - h.off[e], lj = j - h.off[e];
            if (excludes(ent[i].excl, lj)) continue;
            pairs.push_back((uint32_t)(slot + li) | ((uint32_t)(slot + lj) << 11) |
                            ((uint32_t)li << 22) | ((uint32_t)lj << 27));
            if (shape[i] == SPHERE && shape[j] == SPHERE) continue;
            ++cnt[pq_pair_class(shape[i], shape[j])];
          }
        slot += n;
      }
      pair_off[g + 1] = (int32_t)pairs.size();
      p.pq_max_pairs = std::max(p.pq_max_pairs, pair_off[g + 1] - pair_off[g]);
      const int lim = std::min(PQ_CAP_MAX, PQ_CAP_PER_ENV * (int)groups[g].size());
      for (int c = 0; c < 5; ++c) cap[c] = std::max(cap[c], std::min(cnt[c], lim));
    }
    int total = 0;
    for (int c = 0; c < 5; ++c) {
      p.pq_cap[c] = cap[c];
      total += cap[c];
    }
    p.pq_cap[5] = total;
    // a lane tests at most 32 pairs per step (one bit each)
    if (total == 0 || p.pq_max_pairs > 32 * block ||
        rollout_lds_bytes(p.max_stage, false, false, total, p.pq_max_pairs, block, p.max_n) >
            PQ_LDS_MAX) {
      p.valid = false;
      return VMAS_OK;
    }
    vmas_status s;
    if ((s = upload(&p.d_pq_pairs, pairs.data(), std::max<size_t>(pairs.size(), 1))) != VMAS_OK)
      return s;
    if ((s = upload(&p.d_pq_pair_off, pair_off.data(), pair_off.size())) != VMAS_OK) return s;
  }
  vmas_status s;
  if ((s = upload(&p.d_lanes, lane.data(), lane.size())) != VMAS_OK) return s;
  if ((s = upload(&p.d_stage_off, stage_off.data(), stage_off.size())) != VMAS_OK) return s;
  if ((s = upload(&p.d_stage, stage.data(), std::max<size_t>(stage.size(), 1))) != VMAS_OK) return s;
  if ((s = upload(&p.d_maxn, maxn.data(), maxn.size())) != VMAS_OK) return s;
  p.valid = true;
  return VMAS_OK;
}

// Builds the quad schedule (sphere-only batches; every environment has at
// most 4 entities that move or rotate, at most 4 static collidable ones and
// at most 32 entities); p.valid stays false when the batch does not qualify.
vmas_status build_quad_plan(vmas_batch* b, const HostDesc& h, const std::vector<uint8_t>& flags,
                            Plan& p, bool ordered = false, const std::vector<char>* subset = nullptr) {
  p.name = ordered ? "quad-ordered/64" : "quad/256";
  p.block = ordered ? 64 : 256;
  p.quad = true;
  p.quad_ordered = ordered;
  p.valid = false;
  if (!b->spheres_only) return VMAS_OK;
  const int E = b->n_envs;
  std::vector<QuadEnv> q(std::max(E, 1));
  for (auto& r : q) {
    r.agent_row = 0;
    r.n_agents = 0;
    for (int u = 0; u < 4; ++u) r.lane_loc[u] = r.stat_loc[u] = -1;
  }
  std::vector<int32_t> list;
  int max_static = 0;
  for (int e = 0; e < E; ++e) {
    if (subset && !(*subset)[e]) continue;
    list.push_back(e);
    const int o = h.off[e], n = h.off[e + 1] - o;
    if (n > 32) return VMAS_OK;
    QuadEnv& r = q[e];
    r.agent_row = (int32_t)h.agent_off[e];
    r.n_agents = h.nag[e];
    for (int u = 0; u < 4; ++u) r.lane_loc[u] = r.stat_loc[u] = -1;
    int nl = 0, nsx = 0;
    for (int i = 0; i < n; ++i) {
      const uint8_t f = flags[o + i];
      if (f & (MOVABLE | ROTATABLE)) {
        if (nl == 4) return VMAS_OK;
        if (ordered && i != nl) return VMAS_OK;  // movers must be local 0 .. m-1
        r.lane_loc[nl++] = (int8_t)i;
      } else if (f & COLLIDABLE) {
        if (nsx == 4) return VMAS_OK;
        r.stat_loc[nsx++] = (int8_t)i;
      }
    }
    max_static = std::max(max_static, nsx);
  }
  if ((int64_t)E * 4 > INT32_MAX - 256) return VMAS_OK;
  vmas_status s = upload(&p.d_quad, q.data(), q.size());
  if (s != VMAS_OK) return s;
  const int n_quads = subset ? (int)list.size() : E;
  if (subset) {
    if ((s = upload(&p.d_env_list, list.data(), std::max<size_t>(list.size(), 1))) != VMAS_OK)
      return s;
    p.n_list = (int)list.size();
  }
  p.groups = (int)(((int64_t)n_quads * 4 + p.block - 1) / p.block);
  p.max_n = max_static;  // the quad kernels size their static slots by it
  p.valid = n_quads > 0;
  return VMAS_OK;
}

// Environment-size buckets of the size-bucketed plan.
constexpr int BUCKET_HI[] = {4, 8, 16, 32, 64, 1 << 30};

// Builds the buckets and their candidate plans (sphere-only batches whose
// environment sizes span at least two buckets): per bucket the size-sorted
// entity-lane plans of 64, 128 and 256 lanes and, where every environment of
// the bucket fits it, the ordered quad plan, each over the bucket's
// environments only. The first valid candidate is the initial choice.
vmas_status build_buckets(vmas_batch* b, const HostDesc& h, const std::vector<uint8_t>& shape,
                          const std::vector<uint8_t>& flags) {
  if (!b->spheres_only || b->n_envs < 32) return VMAS_OK;
  const int E = b->n_envs;
  std::vector<int> bucket_of(E, -1), count(6, 0);
  for (int e = 0; e < E; ++e) {
    const int n = h.off[e + 1] - h.off[e];
    int k = 0;
    while (n > BUCKET_HI[k]) ++k;
    bucket_of[e] = k;
    if (n > 0) ++count[k];
  }
  int used = 0;
  for (int k = 0; k < 6; ++k) used += count[k] > 0;
  if (used < 2) return VMAS_OK;
  for (int k = 0; k < 6; ++k) {
    if (count[k] == 0) continue;
    std::vector<char> subset(E, 0);
    for (int e = 0; e < E; ++e) subset[e] = bucket_of[e] == k;
    Bucket bk;
    bk.lo = k == 0 ? 1 : BUCKET_HI[k - 1] + 1;
    bk.hi = BUCKET_HI[k];
    vmas_status s;
    {
      Plan p;
      if ((s = build_quad_plan(b, h, flags, p, true, &subset)) != VMAS_OK) {
        free_plan(p);
        return s;
      }
      if (p.valid) bk.cands.push_back(p);
      else free_plan(p);
    }
    for (int block : {64, 128, 256}) {
      Plan p;
      if ((s = build_plan(b, h, shape, flags, block, true, p, false, nullptr, &subset)) != VMAS_OK) {
        free_plan(p);
        return s;
      }
      if (p.valid) bk.cands.push_back(p);
      else free_plan(p);
    }
    if (bk.cands.empty()) {  // a bucket no candidate fits: no bucketed plan
      for (auto& bb : b->buckets)
        for (auto& p : bb.cands) free_plan(p);
      b->buckets.clear();
      return VMAS_OK;
    }
    b->buckets.push_back(std::move(bk));
  }
  for (size_t k = 0; k < b->buckets.size(); ++k) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    b->side.push_back(st);
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    b->side_done.push_back(ev);
  }
  HIPCHK(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
  return VMAS_OK;
}

// Name of the size-bucketed plan from its current choices.
std::string bucketed_name(const vmas_batch* b) {
  std::string n = "bucketed";
  for (const auto& bk : b->buckets)
    n += "/" + std::to_string(bk.lo) + "-" + (bk.hi >= (1 << 30) ? std::string("") :
                                                 std::to_string(bk.hi)) + ":" +
         bk.cands[bk.choice].name;
  return n;
}

StepArgs make_args(vmas_batch* b, const Plan& p) {
  StepArgs a{};
  a.ent = b->d_ent;
  a.sph = b->d_sph;
  a.sph_only = b->sph_only ? 1 : 0;
  a.lanes = p.d_lanes;
  a.stage_off = p.d_stage_off;
  a.stage = p.d_stage;
  a.joff = b->d_joff;
  a.jlist = b->d_jlist;
  a.joints = b->d_joints;
  a.pair_off = b->d_pair_off;
  a.grp_maxn = p.d_maxn;
  a.max_stage = p.max_stage;
  a.max_n = p.max_n;
  a.quad = p.quad ? p.d_quad : nullptr;
  a.quad_ordered = p.quad_ordered ? 1 : 0;
  a.env_list = p.d_env_list;
  a.n_list = p.n_list;
  a.env_off = b->d_env_off;
  a.n_envs = b->n_envs;
  for (int c = 0; c < 6; ++c) a.pq_cap[c] = p.pq ? p.pq_cap[c] : 0;
  a.pq_pairs = p.pq ? p.d_pq_pairs : nullptr;
  a.pq_pair_off = p.pq ? p.d_pq_pair_off : nullptr;
  a.pq_max_pairs = p.pq ? p.pq_max_pairs : 0;
  a.w = b->w;
  return a;
}

vmas_status check_batch(const vmas_batch* b) {
  if (!b) return fail(VMAS_ERR_INVALID_ARGUMENT, "batch is NULL");
  return VMAS_OK;
}

// VMAS_DEBUG_NONFINITE: environments marked by the check after an earlier
// call are reported (once) by the next call on the handle. Synchronises s.
vmas_status report_nonfinite(vmas_batch* b, hipStream_t s) {
  if (!b->debug_nonfinite) return VMAS_OK;
  uint32_t c[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(c, b->d_bad_cnt, sizeof(c), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (c[0] == 0) return VMAS_OK;
  HIPCHK(launch_fill_i32((int32_t*)b->d_bad_cnt, 1, 0, s));
  return fail(VMAS_ERR_NONFINITE,
              "%u environment(s) reached a non-finite state since the last report (%u in all; "
              "vmas_nonfinite_envs lists them); no work was enqueued by this call",
              c[0], c[1]);
}

// VMAS_DEBUG_NONFINITE: marks the environments of `state` that hold a NaN or
// an infinity (enqueued on s after the step work).
vmas_status check_nonfinite(vmas_batch* b, const float* state, hipStream_t s) {
  if (!b->debug_nonfinite) return VMAS_OK;
  HIPCHK(launch_check_nonfinite(state, b->N, b->d_env_off, b->n_envs, b->d_bad, b->d_bad_cnt, s));
  return VMAS_OK;
}

// The call's own arguments (buffers, actions, steps) carried over to the
// arguments of another plan.
StepArgs with_call(vmas_batch* b, const Plan& p, const StepArgs& call) {
  StepArgs a = make_args(b, p);
  a.state = call.state;
  a.actions = call.actions;
  a.key = call.key;
  a.t0 = call.t0;
  a.T = call.T;
  a.traj = call.traj;
  a.traj_xy = call.traj_xy;
  a.mask = call.mask;
  a.forces = call.forces;
  return a;
}

// Size-bucketed plan: the chosen part of every bucket on its own side
// stream, all forked from and joined back into s (the parts touch disjoint
// environments, so they run at the same time).
vmas_status launch_composite(vmas_batch* b, const StepArgs& call, hipStream_t s) {
  HIPCHK(hipEventRecord(b->fork, s));
  for (size_t k = 0; k < b->buckets.size(); ++k) {
    const Plan& part = b->buckets[k].cands[b->buckets[k].choice];
    if (part.groups == 0) continue;
    const StepArgs pa = with_call(b, part, call);
    HIPCHK(hipStreamWaitEvent(b->side[k], b->fork, 0));
    hipError_t e = launch_rollout(pa, part.groups, part.block, b->spheres_only, b->side[k]);
    if (e != hipSuccess) return fail(VMAS_ERR_DEVICE, "rollout launch failed: %s", hipGetErrorString(e));
    HIPCHK(hipEventRecord(b->side_done[k], b->side[k]));
    HIPCHK(hipStreamWaitEvent(s, b->side_done[k], 0));
  }
  return VMAS_OK;
}

vmas_status launch_plan(vmas_batch* b, StepArgs a, hipStream_t s) {
  const Plan& p = b->plans[b->cur];
  if (p.composite) return launch_composite(b, a, s);
  if (p.groups == 0) return VMAS_OK;
  hipError_t e = launch_rollout(a, p.groups, p.block, b->spheres_only, s);
  if (e != hipSuccess) return fail(VMAS_ERR_DEVICE, "rollout launch failed: %s", hipGetErrorString(e));
  return VMAS_OK;
}

}  // namespace

extern "C" {

const char* vmas_last_error(void) { return g_err.c_str(); }

vmas_status vmas_create_batch(const vmas_world_params* params, const vmas_batch_desc* desc,
                              int device, vmas_batch** out) {
  g_err.clear();
  if (!out) return fail(VMAS_ERR_INVALID_ARGUMENT, "out must not be NULL");
  *out = nullptr;
  HostDesc h;
  vmas_status st = validate(params, desc, h);
  if (st != VMAS_OK) return st;
  const int E = desc->n_envs, N = h.off[E];
  // Host-side tables.
  std::vector<uint8_t> shape(desc->shape, desc->shape + N), flags(desc->flags, desc->flags + N);
  std::vector<EntParam> ent(N);
  bool spheres_only = true;
  int max_env = 0;
  for (int e = 0; e < E; ++e) max_env = std::max(max_env, h.off[e + 1] - h.off[e]);
  for (int i = 0; i < N; ++i) {
    EntParam& p = ent[i];
    const int s = shape[i], f = flags[i];
    p.d0 = desc->dims[2 * i];
    p.d1 = s == BOX ? desc->dims[2 * i + 1] : 0.0f;
    const float m = desc->mass[i];
    const bool mov = f & MOVABLE, rot = f & ROTATABLE;
    p.inv_m = mov ? 1.0f / m : 0.0f;
    double I = desc->inertia ? desc->inertia[i] : 0.0;
    if (!(I > 0)) I = default_inertia(s, m, p.d0, p.d1);
    p.inv_I = rot ? (float)(1.0 / I) : 0.0f;
    p.vmax = desc->max_speed ? desc->max_speed[i] : 0.0f;
    p.rho = s == SPHERE ? p.d0 : 0.0f;
    p.mgx = mov ? m * params->gravity[0] : 0.0f;
    p.mgy = mov ? m * params->gravity[1] : 0.0f;
    p.sf = s | (f << 8) | (s != SPHERE ? SF_ROTATES : 0);
    p.excl = -1;
    p.pad[0] = p.pad[1] = 0;
    if (s != SPHERE && (f & COLLIDABLE)) spheres_only = false;
    if (s != SPHERE && (f & (MOVABLE | ROTATABLE))) spheres_only = false;
  }
  // Joints: per-entity lists, contact exclusions, rest lengths.
  const int J = desc->n_joints;
  std::vector<JointK> joints(J);
  std::vector<uint8_t> rest_from_state(J, 0);
  std::vector<int32_t> joff(N + 1, 0), jlist;
  std::vector<std::vector<int>> per(N);
  for (int q = 0; q < J; ++q) {
    JointK& k = joints[q];
    k.a = desc->joint_a[q];
    k.b = desc->joint_b[q];
    k.ax = desc->joint_anchor_a[2 * q];
    k.ay = desc->joint_anchor_a[2 * q + 1];
    k.bx = desc->joint_anchor_b[2 * q];
    k.by = desc->joint_anchor_b[2 * q + 1];
    k.pad = 0;
    // an anchor off a sphere's centre makes the sphere's orientation part
    // of the geometry
    if (shape[k.a] == SPHERE && (k.ax != 0.0f || k.ay != 0.0f)) ent[k.a].sf |= SF_ROTATES;
    if (shape[k.b] == SPHERE && (k.bx != 0.0f || k.by != 0.0f)) ent[k.b].sf |= SF_ROTATES;
    float rest = desc->joint_rest[q];
    if (rest < 0) {
      // replaced on the device by the same distance in the step's own FP32
      // arithmetic (launch_joint_rest), so the spring is exactly at rest there
      rest_from_state[q] = 1;
      const float* s0 = desc->init_state;
      double Pa[2], Pb[2];
      const int ids[2] = {k.a, k.b};
      const float anc[2][2] = {{k.ax, k.ay}, {k.bx, k.by}};
      double* P[2] = {Pa, Pb};
      for (int u = 0; u < 2; ++u) {
        const int e = ids[u];
        const double th = s0[4 * (size_t)N + e], c = std::cos(th), s = std::sin(th);
        P[u][0] = s0[e] + c * anc[u][0] - s * anc[u][1];
        P[u][1] = s0[(size_t)N + e] + s * anc[u][0] + c * anc[u][1];
      }
      rest = (float)std::hypot(Pa[0] - Pb[0], Pa[1] - Pb[1]);
    }
    k.rest = rest;
    spheres_only = false;
    per[k.a].push_back(q);
    per[k.b].push_back(q);
    const bool collide = desc->joint_collide && desc->joint_collide[q];
    if (!collide) {
      for (int u = 0; u < 2; ++u) {
        const int me = u ? k.b : k.a, other = u ? k.a : k.b;
        const int loc = other - h.off[h.env_of[other]];
        if (loc > 254) {
          return fail(VMAS_ERR_UNSUPPORTED,
                      "joint %d: a non-colliding jointed entity must have a local index < 255", q);
        }
        uint32_t ex = (uint32_t)ent[me].excl;
        int k2 = 0;
        while (k2 < 4 && ((ex >> (8 * k2)) & 0xffu) != 0xffu) ++k2;
        if (k2 == 4)
          return fail(VMAS_ERR_UNSUPPORTED,
                      "entity %d has more than 4 non-colliding joint partners", me);
        ex = (ex & ~(0xffu << (8 * k2))) | ((uint32_t)loc << (8 * k2));
        ent[me].excl = (int32_t)ex;
      }
    }
  }
  for (int i = 0; i < N; ++i) {
    joff[i + 1] = joff[i] + (int)per[i].size();
    for (int q : per[i]) jlist.push_back(q);
  }
  std::vector<int64_t> pair_off(E, 0);
  int64_t P = 0;
  for (int e = 0; e < E; ++e) {
    pair_off[e] = P;
    const int64_t n = h.off[e + 1] - h.off[e];
    P += n * (n - 1) / 2;
  }
  int64_t A = 0;
  for (int e = 0; e < E; ++e) A += h.nag[e];

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(VMAS_ERR_DEVICE, "no HIP device is available");
  if (device < 0 || device >= ndev)
    return fail(VMAS_ERR_INVALID_ARGUMENT, "device %d outside [0, %d)", device, ndev);
  DeviceGuard guard(device);
  if (!guard.ok) return fail(VMAS_ERR_DEVICE, "hipSetDevice(%d) failed", device);

  vmas_batch* b = new vmas_batch();
  b->device = device;
  b->n_envs = E;
  b->N = N;
  b->A = (int)A;
  b->J = J;
  b->P = P;
  b->max_env = max_env;
  b->spheres_only = spheres_only;
  for (int i = 0; i < N; ++i) {
    if (!(desc->flags[i] & (MOVABLE | ROTATABLE))) b->all_move = false;
    if (ent[i].vmax > 0.0f) b->any_vmax = true;
  }
  b->w.dt = params->dt;
  b->w.damp = 1.0f - params->drag;
  b->w.gx = params->gravity[0];
  b->w.gy = params->gravity[1];
  b->w.ck = params->contact_force * params->contact_margin;
  b->w.inv_k = 1.0f / params->contact_margin;
  b->w.min_dist = params->min_dist;
  b->w.joint_k = params->joint_stiffness;
  b->w.A = (int)A;
  b->w.N = N;
  std::vector<SphRec> sph(ent.size());
  b->sph_only = J == 0;  // joints bring exclusions and anchor torques
  for (size_t i = 0; i < ent.size(); ++i) {
    sph[i] = SphRec{ent[i].rho, ent[i].inv_m, ent[i].vmax, ent[i].sf};
    uint32_t gx, gy, ii;
    std::memcpy(&gx, &ent[i].mgx, 4);
    std::memcpy(&gy, &ent[i].mgy, 4);
    std::memcpy(&ii, &ent[i].inv_I, 4);
    if (gx != 0u || gy != 0u || (ii >> 31) != 0u || !std::isfinite(ent[i].inv_I))
      b->sph_only = false;
  }
  vmas_status s;
  if ((s = upload(&b->d_ent, ent.data(), ent.size())) != VMAS_OK ||
      (s = upload(&b->d_sph, sph.data(), std::max<size_t>(sph.size(), 1))) != VMAS_OK ||
      (s = upload(&b->d_joff, joff.data(), joff.size())) != VMAS_OK ||
      (s = upload(&b->d_jlist, jlist.data(), jlist.size())) != VMAS_OK ||
      (s = upload(&b->d_joints, joints.data(), joints.size())) != VMAS_OK ||
      (s = upload(&b->d_pair_off, pair_off.data(), pair_off.size())) != VMAS_OK ||
      (s = upload(&b->d_env_off, h.off.data(), h.off.size())) != VMAS_OK) {
    free_batch(b);
    return s;
  }
  if (std::any_of(rest_from_state.begin(), rest_from_state.end(), [](uint8_t v) { return v != 0; })) {
    // rest lengths taken from the initial state: the anchor distance in the
    // step kernels' FP32 arithmetic
    float* d_s0 = nullptr;
    uint8_t* d_from = nullptr;
    if ((s = upload(&d_s0, desc->init_state, 6 * (size_t)N)) != VMAS_OK ||
        (s = upload(&d_from, rest_from_state.data(), rest_from_state.size())) != VMAS_OK) {
      if (d_s0) (void)hipFree(d_s0);
      if (d_from) (void)hipFree(d_from);
      free_batch(b);
      return s;
    }
    hipError_t e = launch_joint_rest(d_s0, N, b->d_ent, b->d_joints, d_from, J, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    (void)hipFree(d_s0);
    (void)hipFree(d_from);
    if (e != hipSuccess) {
      free_batch(b);
      return fail(VMAS_ERR_DEVICE, "joint rest lengths: %s", hipGetErrorString(e));
    }
  }
  if (params->flags & VMAS_DEBUG_NONFINITE) {
    b->debug_nonfinite = true;
    const std::vector<uint32_t> zeros(E, 0u);
    const uint32_t zc[2] = {0u, 0u};
    if ((s = upload(&b->d_bad, zeros.data(), zeros.size())) != VMAS_OK ||
        (s = upload(&b->d_bad_cnt, zc, 2)) != VMAS_OK) {
      free_batch(b);
      return s;
    }
  }
  const int blocks[3] = {64, 128, 256};
  int first_valid = -1;
  for (int sorted = 0; sorted < 2; ++sorted) {
    for (int bi = 0; bi < 3; ++bi) {
      Plan p;
      if ((s = build_plan(b, h, shape, flags, blocks[bi], sorted != 0, p)) != VMAS_OK) {
        free_plan(p);
        free_batch(b);
        return s;
      }
      b->plans.push_back(p);
      if (p.valid && first_valid < 0) first_valid = (int)b->plans.size() - 1;
    }
  }
  if (first_valid < 0) {
    // environments too large for 256 lanes: one bigger block
    int need = 64;
    for (int e = 0; e < E; ++e) {
      int act = 0;
      for (int i = h.off[e]; i < h.off[e + 1]; ++i) act += (flags[i] & (MOVABLE | ROTATABLE)) != 0;
      while (need < act) need *= 2;
    }
    if (need > 1024) {
      free_batch(b);
      return fail(VMAS_ERR_UNSUPPORTED, "an environment has more than 1024 entities that move or rotate");
    }
    Plan p;
    if ((s = build_plan(b, h, shape, flags, need, false, p)) != VMAS_OK) {
      free_plan(p);
      free_batch(b);
      return s;
    }
    b->plans.push_back(p);
    if (p.valid) first_valid = (int)b->plans.size() - 1;
  }
  if (first_valid < 0) {
    free_batch(b);
    return fail(VMAS_ERR_UNSUPPORTED, "an environment is too large to stage in LDS");
  }
  b->cur = first_valid;
  // the surrogate's candidate kernel takes one atomic per workgroup: prefer
  // the largest workgroups (fewest atomics on one counter)
  b->lane_plan = first_valid;
  for (int q = 0; q < (int)b->plans.size(); ++q)
    if (b->plans[q].valid && !b->plans[q].quad && !b->plans[q].pq && b->plans[q].block <= 256 &&
        b->plans[q].block > b->plans[b->lane_plan].block)
      b->lane_plan = q;
  if (!spheres_only && max_env <= 32) {
    // pair-queue plans: every pair with a box or a segment evaluated once
    for (int sorted = 0; sorted < 2; ++sorted) {
      for (int bi = 0; bi < 3; ++bi) {
        Plan p;
        if ((s = build_plan(b, h, shape, flags, blocks[bi], sorted != 0, p, false, &ent)) !=
            VMAS_OK) {
          free_plan(p);
          free_batch(b);
          return s;
        }
        if (p.valid)
          b->plans.push_back(p);
        else
          free_plan(p);
      }
    }
    // The same plans with the lanes spread evenly over the compute units: a
    // whole number of workgroups per CU, each filled to an equal share of
    // the lanes (whole environments), so that no CU runs more environments
    // than another (4,096 environments of 28 movers: 512 groups of 8 instead
    // of 456 of 9, two per CU).
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
      n_cu = 0;
    int64_t L = 0;
    for (int i = 0; i < N; ++i) L += (flags[i] & (MOVABLE | ROTATABLE)) != 0;
    for (int bi = 1; bi < 3 && n_cu > 0 && L > 0; ++bi) {
      const int64_t per = (int64_t)n_cu * blocks[bi];
      const int64_t G = ((L + per - 1) / per) * n_cu;
      const int cap = (int)((L + G - 1) / G);
      if (cap > blocks[bi] - max_env) continue;  // what the plain packing gives
      Plan p;
      if ((s = build_plan(b, h, shape, flags, blocks[bi], false, p, false, &ent, nullptr, cap)) !=
          VMAS_OK) {
        free_plan(p);
        free_batch(b);
        return s;
      }
      if (p.valid)
        b->plans.push_back(p);
      else
        free_plan(p);
    }
  }
  for (int ordered = 0; ordered < 2; ++ordered) {
    Plan p;
    if ((s = build_quad_plan(b, h, flags, p, ordered != 0)) != VMAS_OK) {
      free_plan(p);
      free_batch(b);
      return s;
    }
    b->plans.push_back(p);
  }
  if ((s = build_buckets(b, h, shape, flags)) != VMAS_OK) {
    free_batch(b);
    return s;
  }
  if (!b->buckets.empty()) {
    Plan p;
    p.composite = true;
    p.valid = true;
    p.name = bucketed_name(b);
    b->plans.push_back(p);
  }
  {
    // autotune cache key: device architecture and the histogram of
    // (size, movers, static collidables) over the environments
    hipDeviceProp_t prop{};
    std::string arch = hipGetDeviceProperties(&prop, device) == hipSuccess ? prop.gcnArchName : "?";
    std::map<std::tuple<int, int, int>, int> hist;
    for (int e = 0; e < E; ++e) {
      int mv = 0, st = 0;
      for (int i = h.off[e]; i < h.off[e + 1]; ++i) {
        if (flags[i] & (MOVABLE | ROTATABLE)) ++mv;
        else if (flags[i] & COLLIDABLE) ++st;
      }
      ++hist[std::make_tuple(h.off[e + 1] - h.off[e], mv, st)];
    }
    std::string key = arch + (spheres_only ? "|spheres" : "|shapes") + "|J" + std::to_string(J) +
                      "|md" + std::to_string(params->min_dist != 0.0f);
    for (const auto& kv : hist)
      key += "|" + std::to_string(std::get<0>(kv.first)) + "," + std::to_string(std::get<1>(kv.first)) +
             "," + std::to_string(std::get<2>(kv.first)) + "x" + std::to_string(kv.second);
    b->tune_key = key;
  }
  if (P > 0 && (s = build_plan(b, h, shape, flags, 1024, false, b->cand)) != VMAS_OK) {
    free_batch(b);
    return s;
  }
  {
    // The adjoint plan: every entity has a lane; environments in size order.
    // Sphere batches (four reverse-step wavefronts per SIMD) pack them into
    // 256-lane workgroups, the fewest wavefronts (uneven16384: 9,092 against
    // 11,134 for 64 lanes in natural order; 1.14 against 1.32 ms per 50-step
    // adjoint); the general reverse step (two per SIMD) keeps workgroups of
    // the smallest power of two that holds the largest environment, at
    // least 64 lanes.
    int need = spheres_only ? 256 : 64;
    for (int e = 0; e < E; ++e)
      while (need < h.off[e + 1] - h.off[e] && need < 1024) need *= 2;
    if ((s = build_plan(b, h, shape, flags, need, true, b->back, true)) != VMAS_OK) {
      free_batch(b);
      return s;
    }
  }
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_batch(b);
    return fail(VMAS_ERR_DEVICE, "hipDeviceSynchronize failed: %s", hipGetErrorString(e));
  }
  *out = b;
  return VMAS_OK;
}

vmas_status vmas_destroy_batch(vmas_batch* batch) {
  g_err.clear();
  if (!batch) return VMAS_OK;
  DeviceGuard guard(batch->device);
  free_batch(batch);
  return VMAS_OK;
}

vmas_status vmas_batch_get_info(const vmas_batch* b, vmas_batch_info* info) {
  g_err.clear();
  if (!b || !info) return fail(VMAS_ERR_INVALID_ARGUMENT, "batch and info must not be NULL");
  info->n_envs = b->n_envs;
  info->n_entities = b->N;
  info->n_agents = b->A;
  info->n_joints = b->J;
  info->n_pair_slots = b->P;
  info->schedule = b->cur;
  info->n_schedules = (int32_t)b->plans.size();
  info->max_env_size = b->max_env;
  info->tune_cached = b->tune_cached ? 1 : 0;
  return VMAS_OK;
}

const char* vmas_schedule_name(const vmas_batch* b, int32_t schedule) {
  if (!b || schedule < 0 || schedule >= (int)b->plans.size()) return "";
  return b->plans[schedule].valid ? b->plans[schedule].name.c_str() : "";
}

vmas_status vmas_set_schedule(vmas_batch* b, int32_t schedule) {
  g_err.clear();
  if (check_batch(b) != VMAS_OK) return VMAS_ERR_INVALID_ARGUMENT;
  if (schedule < 0 || schedule >= (int)b->plans.size() || !b->plans[schedule].valid)
    return fail(VMAS_ERR_INVALID_ARGUMENT, "schedule %d is not a valid plan", schedule);
  b->cur = schedule;
  return VMAS_OK;
}

vmas_status vmas_step(vmas_batch* b, float* state, const float* actions, uint8_t* mask,
                      float* forces, void* stream) {
  g_err.clear();
  if (check_batch(b) != VMAS_OK) return VMAS_ERR_INVALID_ARGUMENT;
  if (!state) return fail(VMAS_ERR_INVALID_ARGUMENT, "state must not be NULL");
  if (!actions && b->A > 0) return fail(VMAS_ERR_INVALID_ARGUMENT, "actions must not be NULL");
  DeviceGuard guard(b->device);
  hipStream_t s = (hipStream_t)stream;
  vmas_status st = report_nonfinite(b, s);
  if (st != VMAS_OK) return st;
  if (mask) HIPCHK(launch_fill_u8(mask, b->P, s));
  if (forces) HIPCHK(launch_fill_f32(forces, 3 * (int64_t)b->N, 0.0f, s));
  StepArgs a = make_args(b, b->plans[b->cur]);
  a.state = state;
  a.actions = actions;
  a.key = 0;
  a.t0 = 0;
  a.T = 1;
  a.traj = nullptr;
  a.mask = mask;
  a.forces = forces;
  if ((st = launch_plan(b, a, s)) != VMAS_OK) return st;
  return check_nonfinite(b, state, s);
}

}  // extern "C"

namespace {

// vmas_rollout without the debug report and check (also the forward replays
// of the adjoint driver and the autotuner's trials, on library workspaces).
// traj_xy: the trajectory gets positions only (every entity must have a lane)
vmas_status rollout_impl(vmas_batch* b, float* state, const float* actions, uint64_t seed,
                         int32_t t0, int32_t T, float* traj, uint8_t* final_mask, hipStream_t s,
                         bool traj_xy = false) {
  if (!state) return fail(VMAS_ERR_INVALID_ARGUMENT, "state must not be NULL");
  if (T < 0) return fail(VMAS_ERR_INVALID_ARGUMENT, "T must be >= 0");
  if (t0 < 0) return fail(VMAS_ERR_INVALID_ARGUMENT, "t0 must be >= 0");
  if ((int64_t)T * b->A * 2 > ((int64_t)1 << 40))
    return fail(VMAS_ERR_INVALID_ARGUMENT, "T * A too large");
  // trajectory slot 0 is the start state; the kernels write slots 1..T of
  // every entity with a lane, so only entities without one (neither
  // movable nor rotatable) need their state copied into every slot
  if (traj_xy && !b->all_move) return fail(VMAS_ERR_INVALID_ARGUMENT, "positions-only trajectory");
  if (traj)
    HIPCHK(launch_replicate(state, traj, (traj_xy ? 2 : 6) * (int64_t)b->N, b->all_move ? 1 : T + 1, s));
  if (T == 0) return VMAS_OK;
  if (final_mask) HIPCHK(launch_fill_u8(final_mask, b->P, s));
  StepArgs a = make_args(b, b->plans[b->cur]);
  a.state = state;
  a.actions = actions;
  a.key = action_key(seed);
  a.t0 = t0;
  a.T = T;
  a.traj = traj;
  a.traj_xy = traj && traj_xy ? 1 : 0;
  a.mask = final_mask;
  a.forces = nullptr;
  return launch_plan(b, a, s);
}

}  // namespace

extern "C" {

vmas_status vmas_rollout(vmas_batch* b, float* state, const float* actions, uint64_t seed,
                         int32_t t0, int32_t T, float* traj, uint8_t* final_mask, void* stream) {
  g_err.clear();
  if (check_batch(b) != VMAS_OK) return VMAS_ERR_INVALID_ARGUMENT;
  if (!state) return fail(VMAS_ERR_INVALID_ARGUMENT, "state must not be NULL");
  if (T < 0 || t0 < 0) return fail(VMAS_ERR_INVALID_ARGUMENT, "T and t0 must be >= 0");
  if ((int64_t)T * b->A * 2 > ((int64_t)1 << 40))
    return fail(VMAS_ERR_INVALID_ARGUMENT, "T * A too large");
  DeviceGuard guard(b->device);
  hipStream_t s = (hipStream_t)stream;
  vmas_status st = report_nonfinite(b, s);
  if (st != VMAS_OK) return st;
  if ((st = rollout_impl(b, state, actions, seed, t0, T, traj, final_mask, s)) != VMAS_OK)
    return st;
  return T > 0 ? check_nonfinite(b, state, s) : VMAS_OK;
}

vmas_status vmas_rollout_graph(vmas_batch* b, float* state, const float* actions, uint64_t seed,
                               int32_t t0, int32_t T, float* traj, uint8_t* final_mask,
                               void* stream) {
  g_err.clear();
  if (check_batch(b) != VMAS_OK) return VMAS_ERR_INVALID_ARGUMENT;
  if (traj || final_mask || T <= 0)  // only the plain state-in/state-out rollout is cached
    return vmas_rollout(b, state, actions, seed, t0, T, traj, final_mask, stream);
  if (!state) return fail(VMAS_ERR_INVALID_ARGUMENT, "state must not be NULL");
  if (t0 < 0) return fail(VMAS_ERR_INVALID_ARGUMENT, "t0 must be >= 0");
  DeviceGuard guard(b->device);
  hipStream_t s = (hipStream_t)stream;
  vmas_status st0 = report_nonfinite(b, s);
  if (st0 != VMAS_OK) return st0;
  const Plan& p = b->plans[b->cur];
  // the plan's launches: the plan itself, or the chosen part of every
  // bucket of a size-bucketed plan (independent graph nodes, which may run
  // at the same time)
  std::vector<const Plan*> parts;
  if (p.composite) {
    for (const auto& bk : b->buckets)
      if (bk.cands[bk.choice].groups > 0) parts.push_back(&bk.cands[bk.choice]);
  } else if (p.groups > 0) {
    parts.push_back(&p);
  }
  if (parts.empty()) return VMAS_OK;
  StepArgs call{};
  call.state = state;
  call.actions = actions;
  call.key = action_key(seed);
  call.t0 = t0;
  call.T = T;
  const bool drawn = actions == nullptr;
  std::vector<StepArgs> args(parts.size());
  std::vector<void*> argp(parts.size());
  std::vector<hipKernelNodeParams> kps(parts.size());
  for (size_t k = 0; k < parts.size(); ++k) {
    const Plan& q = *parts[k];
    args[k] = with_call(b, q, call);
    argp[k] = &args[k];
    hipKernelNodeParams& kp = kps[k];
    kp = hipKernelNodeParams{};
    kp.func = const_cast<void*>(rollout_kernel(b->spheres_only, q.quad, q.pq, q.block, q.max_n,
                                               b->w.min_dist, false, q.quad_ordered));
    kp.gridDim = dim3(q.groups);
    kp.blockDim = dim3(q.block);
    kp.sharedMemBytes = (unsigned)rollout_lds_bytes(q.max_stage, b->spheres_only, q.quad,
                                                    q.pq ? q.pq_cap[5] : 0, q.pq_max_pairs, q.block,
                                                    q.max_n);
    kp.kernelParams = &argp[k];
    kp.extra = nullptr;
  }
  if (!b->gexec || b->graph_T != T || b->graph_plan != b->cur || b->graph_drawn != drawn ||
      b->graph_gen != b->plan_gen) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->gnodes.clear();
    // The graph holds the rollout kernel nodes, without dependencies; it is
    // built explicitly (no stream capture), so any stream, the default one
    // included, works.
    HIPCHK(hipGraphCreate(&b->graph, 0));
    for (size_t k = 0; k < parts.size(); ++k) {
      hipGraphNode_t node = nullptr;
      HIPCHK(hipGraphAddKernelNode(&node, b->graph, nullptr, 0, &kps[k]));
      b->gnodes.push_back(node);
    }
    HIPCHK(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
    b->graph_T = T;
    b->graph_plan = b->cur;
    b->graph_drawn = drawn;
    b->graph_gen = b->plan_gen;
  } else {
    for (size_t k = 0; k < parts.size(); ++k)
      HIPCHK(hipGraphExecKernelNodeSetParams(b->gexec, b->gnodes[k], &kps[k]));
  }
  HIPCHK(hipGraphLaunch(b->gexec, s));
  return check_nonfinite(b, state, s);
}

}  // extern "C"

namespace {

// Autotune choices cached across handles in this process, keyed by device
// architecture and the batch's histogram of environment shapes (plus the
// rollout length bucket): the plan id and the part chosen for every size
// bucket. With VMAS_AUTOTUNE_CACHE set, the cache is also read from and
// appended to that file (one line per key: key, plan id, part choices).
struct TuneChoice {
  int plan = 0;
  std::vector<int> parts;
};
std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune;
bool g_tune_loaded = false;

void tune_load_file() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("VMAS_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[16384];
  while (std::fgets(line, sizeof(line), f)) {
    char* tab1 = std::strchr(line, '\t');
    if (!tab1) continue;
    *tab1 = 0;
    char* tab2 = std::strchr(tab1 + 1, '\t');
    TuneChoice c;
    c.plan = std::atoi(tab1 + 1);
    if (tab2)
      for (char* q = tab2 + 1; *q && *q != '\n';) {
        c.parts.push_back((int)std::strtol(q, &q, 10));
        if (*q == ',') ++q;
      }
    g_tune[line] = c;
  }
  std::fclose(f);
}

void tune_store(const std::string& key, const TuneChoice& c) {
  g_tune[key] = c;
  const char* path = std::getenv("VMAS_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s\t%d\t", key.c_str(), c.plan);
  for (size_t k = 0; k < c.parts.size(); ++k) std::fprintf(f, k ? ",%d" : "%d", c.parts[k]);
  std::fprintf(f, "\n");
  std::fclose(f);
}

std::string tune_key_T(const vmas_batch* b, int T) {
  int tb = 1;
  while (tb < T && tb < 1024) tb *= 2;  // rollout length bucket
  return b->tune_key + "|T" + std::to_string(tb);
}

void set_bucket_choice(vmas_batch* b, const std::vector<int>& parts) {
  for (size_t k = 0; k < b->buckets.size() && k < parts.size(); ++k)
    if (parts[k] >= 0 && parts[k] < (int)b->buckets[k].cands.size()) b->buckets[k].choice = parts[k];
  for (auto& p : b->plans)
    if (p.composite) p.name = bucketed_name(b);
  ++b->plan_gen;
}

}  // namespace

extern "C" {

vmas_status vmas_autotune(vmas_batch* b, const float* state, const float* actions, int32_t T,
                          void* stream, int32_t* chosen) {
  g_err.clear();
  if (check_batch(b) != VMAS_OK) return VMAS_ERR_INVALID_ARGUMENT;
  if (!state || T < 1) return fail(VMAS_ERR_INVALID_ARGUMENT, "state must be given and T >= 1");
  DeviceGuard guard(b->device);
  hipStream_t s = (hipStream_t)stream;
  const int nplans = (int)b->plans.size();
  const std::string key = tune_key_T(b, T);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_load_file();
    auto it = g_tune.find(key);
    if (it != g_tune.end() && it->second.plan >= 0 && it->second.plan < nplans &&
        b->plans[it->second.plan].valid && it->second.parts.size() == b->buckets.size()) {
      set_bucket_choice(b, it->second.parts);
      b->cur = it->second.plan;
      b->tune_cached = true;
      if (chosen) *chosen = b->cur;
      return VMAS_OK;
    }
  }
  b->tune_cached = false;
  const size_t n = 6 * (size_t)b->N;
  float* scratch = nullptr;
  HIPCHK(hipMalloc((void**)&scratch, n * sizeof(float)));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int prev = b->cur;
  std::vector<float> ms_min(nplans, INFINITY);
  vmas_status st = VMAS_OK;
  auto trial = [&](int q, float* ms_out) {
    b->cur = q;
    if (hipMemcpyAsync(scratch, state, n * sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess)
      return fail(VMAS_ERR_DEVICE, "autotune copy failed");
    (void)hipEventRecord(e0, s);
    vmas_status r = rollout_impl(b, scratch, actions, 12345u, 0, T, nullptr, nullptr, s);
    (void)hipEventRecord(e1, s);
    if (r != VMAS_OK) return r;
    if (hipEventSynchronize(e1) != hipSuccess) return fail(VMAS_ERR_DEVICE, "autotune sync failed");
    (void)hipEventElapsedTime(ms_out, e0, e1);
    return VMAS_OK;
  };
  // one candidate part of size bucket k alone (its environments only)
  auto trial_part = [&](size_t k, int c, float* ms_out) {
    const Plan& part = b->buckets[k].cands[c];
    if (hipMemcpyAsync(scratch, state, n * sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess)
      return fail(VMAS_ERR_DEVICE, "autotune copy failed");
    StepArgs call{};
    call.state = scratch;
    call.actions = actions;
    call.key = action_key(12345u);
    call.T = T;
    const StepArgs pa = with_call(b, part, call);
    (void)hipEventRecord(e0, s);
    hipError_t e = launch_rollout(pa, part.groups, part.block, b->spheres_only, s);
    (void)hipEventRecord(e1, s);
    if (e != hipSuccess) return fail(VMAS_ERR_DEVICE, "autotune launch failed: %s", hipGetErrorString(e));
    if (hipEventSynchronize(e1) != hipSuccess) return fail(VMAS_ERR_DEVICE, "autotune sync failed");
    (void)hipEventElapsedTime(ms_out, e0, e1);
    return VMAS_OK;
  };
  // Warm-up (clocks and code objects settle): about 20 ms of the first plan.
  {
    float ms = 0, spent = 0;
    for (int rep = 0; rep < 200 && spent < 20.0f && st == VMAS_OK; ++rep) {
      st = trial(prev, &ms);
      spent += ms;
    }
  }
  // Size buckets first: every candidate part of a bucket timed on the
  // bucket alone, two rounds of two runs; the fastest run decides.
  std::vector<int> parts(b->buckets.size(), 0);
  for (size_t k = 0; k < b->buckets.size() && st == VMAS_OK; ++k) {
    const int nc = (int)b->buckets[k].cands.size();
    std::vector<float> best(nc, INFINITY);
    for (int round = 0; round < 2 && st == VMAS_OK && nc > 1; ++round)
      for (int c = 0; c < nc && st == VMAS_OK; ++c)
        for (int rep = 0; rep < 2 && st == VMAS_OK; ++rep) {
          float ms = 0;
          st = trial_part(k, c, &ms);
          if (st == VMAS_OK && ms < best[c]) best[c] = ms;
        }
    for (int c = 1; c < nc; ++c)
      if (best[c] < 0.97f * best[parts[k]]) parts[k] = c;
  }
  if (st == VMAS_OK && !b->buckets.empty()) set_bucket_choice(b, parts);
  // Three rounds over all plans, two timed runs each: the fastest run of a
  // plan over the rounds is its time.
  for (int round = 0; round < 3 && st == VMAS_OK; ++round) {
    for (int q = 0; q < nplans && st == VMAS_OK; ++q) {
      if (!b->plans[q].valid) continue;
      for (int rep = 0; rep < 2 && st == VMAS_OK; ++rep) {
        float ms = 0;
        st = trial(q, &ms);
        if (st == VMAS_OK && ms < ms_min[q]) ms_min[q] = ms;
      }
    }
  }
  // a later schedule must be clearly faster (3 %) to replace the current
  // choice, which keeps the choice stable where schedules are within noise
  int best = -1;
  for (int q = 0; q < nplans && st == VMAS_OK; ++q) {
    if (!b->plans[q].valid) continue;
    if (best < 0 || ms_min[q] < 0.97f * ms_min[best]) best = q;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(scratch);
  if (st != VMAS_OK) {
    b->cur = prev;
    return st;
  }
  b->cur = best;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    TuneChoice c;
    c.plan = best;
    c.parts = parts;
    tune_store(key, c);
  }
  if (chosen) *chosen = best;
  return VMAS_OK;
}

// T reverse steps in one launch: states [T][6][N] (t0 .. t0 + T - 1), their
// actions [T][A][2], dL/ds_{t0+T} -> dL/ds_t0 and dL/da of every step.
// states: T states, `stride` floats apart (6 N; 2 N for positions only,
// which the sphere reverse step accepts when no entity has a speed cap).
static vmas_status adjoint_segment(vmas_batch* b, const float* states, int64_t stride,
                                   const float* actions, int T, const float* gnext, float* gstate,
                                   float* gact, hipStream_t s) {
  // Entities without a lane in no group (environments of size 0) keep a zero gradient.
  BackArgs a{};
  a.state = states;
  a.stride = stride;
  a.actions = actions;
  a.gnext = gnext;
  a.gstate = gstate;
  a.gact = gact;
  a.ent = b->d_ent;
  a.lanes = b->back.d_lanes;
  a.stage_off = b->back.d_stage_off;
  a.stage = b->back.d_stage;
  a.joff = b->d_joff;
  a.jlist = b->d_jlist;
  a.joints = b->d_joints;
  a.max_stage = b->back.max_stage;
  a.T = T;
  a.w = b->w;
  if (b->back.groups == 0) return VMAS_OK;
  hipError_t e = launch_backward(a, b->back.groups, b->back.block, b->spheres_only, s);
  if (e != hipSuccess) return fail(VMAS_ERR_DEVICE, "adjoint launch failed: %s", hipGetErrorString(e));
  return VMAS_OK;
}

vmas_status vmas_step_backward(vmas_batch* b, const float* state_t, const float* actions_t,
                               const float* grad_state_next, float* grad_state_t,
                               float* grad_actions_t, void* stream) {
  g_err.clear();
  if (check_batch(b) != VMAS_OK) return VMAS_ERR_INVALID_ARGUMENT;
  if (!state_t || !grad_state_next || !grad_state_t)
    return fail(VMAS_ERR_INVALID_ARGUMENT, "state_t, grad_state_next and grad_state_t are required");
  if (!actions_t && b->A > 0) return fail(VMAS_ERR_INVALID_ARGUMENT, "actions_t must not be NULL");
  if (grad_state_t == grad_state_next || grad_state_t == state_t)
    return fail(VMAS_ERR_INVALID_ARGUMENT, "grad_state_t must not alias its inputs");
  if (!b->back.valid)
    return fail(VMAS_ERR_UNSUPPORTED, "an environment is too large for the adjoint plan");
  DeviceGuard guard(b->device);
  vmas_status st = report_nonfinite(b, (hipStream_t)stream);
  if (st != VMAS_OK) return st;
  return adjoint_segment(b, state_t, 6 * (int64_t)b->N, actions_t, 1, grad_state_next, grad_state_t,
                         grad_actions_t,
                         (hipStream_t)stream);
}

}  // extern "C"

namespace {

// Arguments of a rollout adjoint, checked on the host; sets the workspace
// size in floats.
vmas_status backward_args(vmas_batch* b, const float* state0, const float* actions, int32_t T,
                          int32_t ckpt_every, const float* grad_state_T, size_t* need) {
  if (check_batch(b) != VMAS_OK) return VMAS_ERR_INVALID_ARGUMENT;
  if (!state0 || !grad_state_T) return fail(VMAS_ERR_INVALID_ARGUMENT, "state0 and grad_state_T are required");
  if (T < 1) return fail(VMAS_ERR_INVALID_ARGUMENT, "T must be >= 1");
  if (ckpt_every < 1) return fail(VMAS_ERR_INVALID_ARGUMENT, "ckpt_every must be >= 1");
  if (!actions && b->A > 0) return fail(VMAS_ERR_INVALID_ARGUMENT, "actions must not be NULL");
  if (!b->back.valid)
    return fail(VMAS_ERR_UNSUPPORTED, "an environment is too large for the adjoint plan");
  const int k = std::min(ckpt_every, T);
  const int nseg = (T + k - 1) / k;
  // nseg checkpoints, k + 1 states of the segment being replayed, two
  // gradient buffers
  *need = 6 * (size_t)b->N * ((size_t)nseg + (size_t)k + 1 + 2);
  return VMAS_OK;
}

// The checkpointed adjoint on a workspace of backward_args' size.
vmas_status backward_on(vmas_batch* b, float* ws, const float* state0, const float* actions,
                        int32_t T, int32_t ckpt_every, const float* grad_state_T,
                        float* grad_state0, float* grad_actions, hipStream_t s) {
  const int k = std::min(ckpt_every, T);
  const int nseg = (T + k - 1) / k;
  const size_t S6 = 6 * (size_t)b->N, S2 = 2 * (size_t)b->N;
  const size_t A2 = 2 * (size_t)b->A;
  auto act_at = [&](int t) { return actions ? actions + A2 * (size_t)t : nullptr; };
  // the workspace: room for nseg + k + 1 states, then two gradient buffers
  const size_t room = S6 * ((size_t)nseg + k + 1);
  float* g0 = ws + room;
  float* g1 = g0 + S6;
  auto gact_at = [&](int t) { return grad_actions ? grad_actions + A2 * (size_t)t : nullptr; };
  // The sphere reverse step reads only the positions of a step's state when
  // no entity has a speed cap (the clamp's adjoint needs the velocities).
  const bool xy = b->spheres_only && b->all_move && !b->any_vmax;
  if (!xy) {
    // checkpoints at t = 0, k, 2k, ..., then each segment replayed from its
    // checkpoint (full states) and stepped back through in one launch
    float* ckpt = ws;
    float* seg = ckpt + S6 * nseg;
    HIPCHK(hipMemcpyAsync(ckpt, state0, S6 * sizeof(float), hipMemcpyDeviceToDevice, s));
    for (int q = 1; q < nseg; ++q) {
      HIPCHK(hipMemcpyAsync(ckpt + S6 * q, ckpt + S6 * (q - 1), S6 * sizeof(float),
                            hipMemcpyDeviceToDevice, s));
      vmas_status st = rollout_impl(b, ckpt + S6 * q, act_at((q - 1) * k), 0, 0, k, nullptr, nullptr, s);
      if (st != VMAS_OK) return st;
    }
    HIPCHK(hipMemcpyAsync(g0, grad_state_T, S6 * sizeof(float), hipMemcpyDeviceToDevice, s));
    for (int q = nseg - 1; q >= 0; --q) {
      const int t0 = q * k, len = std::min(k, T - t0);
      // seg[0 .. len]: states t0 .. t0 + len (the rollout writes them as a
      // trajectory; g1 is the rolled state's scratch, overwritten below)
      HIPCHK(hipMemcpyAsync(g1, ckpt + S6 * q, S6 * sizeof(float), hipMemcpyDeviceToDevice, s));
      vmas_status st = rollout_impl(b, g1, act_at(t0), 0, 0, len, seg, nullptr, s);
      if (st != VMAS_OK) return st;
      st = adjoint_segment(b, seg, (int64_t)S6, act_at(t0), len, g0, g1, gact_at(t0), s);
      if (st != VMAS_OK) return st;
      std::swap(g0, g1);
    }
  } else {
    // Positions are 2 N floats a step, so the same room holds more than
    // checkpoints. A window of the last segments w .. nseg-1 gets the
    // positions of all its steps from one forward launch, and its reverse
    // steps run in one launch; segments 0 .. w-1 are replayed from their
    // checkpoints (0 is state0 itself, 1 .. w-1 are stored) into the first
    // k + 1 slots of the window, free by then. w is the first segment for
    // which the stored checkpoints and the window fit (w = nseg: no window,
    // every segment replayed).
    int w = nseg;
    for (int q = 0; q <= nseg; ++q) {
      const size_t ck = S6 * (size_t)std::max(std::min(q, nseg) - 1, 0);
      const size_t slots = q == nseg ? (size_t)k + 1
                                     : (q == 0 ? (size_t)T + 1
                                               : std::max((size_t)k + 1, (size_t)T - (size_t)q * k + 1));
      if (ck + S2 * slots <= room) {
        w = q;
        break;
      }
    }
    float* ckpt = ws;  // the state at j k (j = 1 .. w-1) at ckpt + S6 (j - 1)
    float* win = ckpt + S6 * (size_t)std::max(w - 1, 0);
    auto ck = [&](int j) -> const float* { return j == 0 ? state0 : ckpt + S6 * (size_t)(j - 1); };
    for (int j = 1; j < w; ++j) {
      HIPCHK(hipMemcpyAsync(ckpt + S6 * (j - 1), ck(j - 1), S6 * sizeof(float), hipMemcpyDeviceToDevice, s));
      vmas_status st = rollout_impl(b, ckpt + S6 * (j - 1), act_at((j - 1) * k), 0, 0, k, nullptr, nullptr, s);
      if (st != VMAS_OK) return st;
    }
    HIPCHK(hipMemcpyAsync(g0, grad_state_T, S6 * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (w < nseg) {
      // the state at w k in g1 (free until the reverse steps), then the
      // window's forward launch and its reverse steps
      HIPCHK(hipMemcpyAsync(g1, ck(std::max(w - 1, 0)), S6 * sizeof(float), hipMemcpyDeviceToDevice, s));
      if (w > 0) {
        vmas_status st = rollout_impl(b, g1, act_at((w - 1) * k), 0, 0, k, nullptr, nullptr, s);
        if (st != VMAS_OK) return st;
      }
      vmas_status st = rollout_impl(b, g1, act_at(w * k), 0, 0, T - w * k, win, nullptr, s, true);
      if (st != VMAS_OK) return st;
      st = adjoint_segment(b, win, (int64_t)S2, act_at(w * k), T - w * k, g0, g1, gact_at(w * k), s);
      if (st != VMAS_OK) return st;
      std::swap(g0, g1);
    }
    for (int q = std::min(w, nseg) - 1; q >= 0; --q) {
      const int t0 = q * k, len = std::min(k, T - t0);
      HIPCHK(hipMemcpyAsync(g1, ck(q), S6 * sizeof(float), hipMemcpyDeviceToDevice, s));
      vmas_status st = rollout_impl(b, g1, act_at(t0), 0, 0, len, win, nullptr, s, true);
      if (st != VMAS_OK) return st;
      st = adjoint_segment(b, win, (int64_t)S2, act_at(t0), len, g0, g1, gact_at(t0), s);
      if (st != VMAS_OK) return st;
      std::swap(g0, g1);
    }
  }
  if (grad_state0)
    HIPCHK(hipMemcpyAsync(grad_state0, g0, S6 * sizeof(float), hipMemcpyDeviceToDevice, s));
  return VMAS_OK;
}

// Fixed scratch of the allocation-free adjoint: SCRATCH_FLOATS floats in a
// file-scope device array (each device the library runs on holds its own
// copy until the process ends). Host code never passes the array's name to
// a kernel or a copy: it takes the device address from hipGetSymbolAddress,
// once per device (with that device current), and uses that.
constexpr size_t SCRATCH_FLOATS = (size_t)16 << 20;  // 64 MiB
__device__ __align__(256) float scratch[SCRATCH_FLOATS];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[MAX_DEVICES] = {};

vmas_status scratch_of(int device, float** out) {
  if (device < 0 || device >= MAX_DEVICES)
    return fail(VMAS_ERR_UNSUPPORTED, "device %d: static scratch supports devices 0..%d", device,
                MAX_DEVICES - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(VMAS_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[device];
  return VMAS_OK;
}

}  // namespace

extern "C" {

vmas_status vmas_rollout_backward(vmas_batch* b, const float* state0, const float* actions,
                                  int32_t T, int32_t ckpt_every, const float* grad_state_T,
                                  float* grad_state0, float* grad_actions, void* stream) {
  g_err.clear();
  size_t need = 0;
  vmas_status st0 = backward_args(b, state0, actions, T, ckpt_every, grad_state_T, &need);
  if (st0 != VMAS_OK) return st0;
  DeviceGuard guard(b->device);
  hipStream_t s = (hipStream_t)stream;
  if ((st0 = report_nonfinite(b, s)) != VMAS_OK) return st0;
  if (b->ws_floats < need) {
    if (b->d_ws) (void)hipFree(b->d_ws);
    b->d_ws = nullptr;
    b->ws_floats = 0;
    hipError_t e = hipMalloc((void**)&b->d_ws, need * sizeof(float));
    if (e != hipSuccess)
      return fail(VMAS_ERR_OUT_OF_MEMORY, "checkpoint workspace (%zu bytes): %s", need * sizeof(float),
                  hipGetErrorString(e));
    b->ws_floats = need;
  }
  return backward_on(b, b->d_ws, state0, actions, T, ckpt_every, grad_state_T, grad_state0,
                     grad_actions, s);
}

vmas_status vmas_rollout_backward_noalloc(vmas_batch* b, const float* state0, const float* actions,
                                          int32_t T, int32_t ckpt_every, const float* grad_state_T,
                                          float* grad_state0, float* grad_actions, void* stream) {
  g_err.clear();
  size_t need = 0;
  vmas_status st = backward_args(b, state0, actions, T, ckpt_every, grad_state_T, &need);
  if (st != VMAS_OK) return st;
  if (need > SCRATCH_FLOATS)
    return fail(VMAS_ERR_INVALID_ARGUMENT,
                "the checkpoint workspace of %zu bytes exceeds the static scratch of %zu bytes "
                "(6 N (ceil(T / k) + k + 3) floats must fit)",
                need * sizeof(float), SCRATCH_FLOATS * sizeof(float));
  DeviceGuard guard(b->device);
  hipStream_t s = (hipStream_t)stream;
  if ((st = report_nonfinite(b, s)) != VMAS_OK) return st;
  float* ws = nullptr;
  if ((st = scratch_of(b->device, &ws)) != VMAS_OK) return st;
  return backward_on(b, ws, state0, actions, T, ckpt_every, grad_state_T, grad_state0,
                     grad_actions, s);
}

vmas_status vmas_pair_features(vmas_batch* b, const float* state, float band,
                               const int64_t* slots, int64_t m, float* features, float* targets,
                               uint8_t* flags, void* stream) {
  g_err.clear();
  if (check_batch(b) != VMAS_OK) return VMAS_ERR_INVALID_ARGUMENT;
  if (!state || !features || !flags)
    return fail(VMAS_ERR_INVALID_ARGUMENT, "state, features and flags are required");
  if (!(std::isfinite(band) && band >= 0)) return fail(VMAS_ERR_INVALID_ARGUMENT, "band must be >= 0");
  if (!slots && m != b->P)
    return fail(VMAS_ERR_INVALID_ARGUMENT, "without a slot list m must be the number of pair slots");
  if (m < 0) return fail(VMAS_ERR_INVALID_ARGUMENT, "m must be >= 0");
  DeviceGuard guard(b->device);
  HIPCHK(launch_pair_features(state, b->d_ent, b->d_env_off, b->d_pair_off, slots, m, band,
                              features, targets, flags, b->n_envs, b->w, (hipStream_t)stream));
  return VMAS_OK;
}

vmas_status vmas_step_surrogate(vmas_batch* b, vmas_mlp* mlp, float* state, const float* actions,
                                float band, float fallback_frac, float* forces,
                                int32_t* n_fallback, void* stream) {
  g_err.clear();
  if (check_batch(b) != VMAS_OK) return VMAS_ERR_INVALID_ARGUMENT;
  if (!mlp || !state) return fail(VMAS_ERR_INVALID_ARGUMENT, "mlp and state are required");
  if (!actions && b->A > 0) return fail(VMAS_ERR_INVALID_ARGUMENT, "actions must not be NULL");
  if (!(std::isfinite(band) && band >= 0 && std::isfinite(fallback_frac)))
    return fail(VMAS_ERR_INVALID_ARGUMENT, "band must be >= 0 and fallback_frac finite");
  if (b->P >= INT32_MAX)
    return fail(VMAS_ERR_INVALID_ARGUMENT, "surrogate step supports fewer than 2^31 pair slots");
  DeviceGuard guard(b->device);
  hipStream_t s = (hipStream_t)stream;
  vmas_status st0 = report_nonfinite(b, s);
  if (st0 != VMAS_OK) return st0;
  if (!b->d_feat && b->P > 0) {
    hipError_t e;
    if ((e = hipMalloc((void**)&b->d_feat, (size_t)b->P * 12 * sizeof(float))) != hipSuccess ||
        (e = hipMalloc((void**)&b->d_yhat, (size_t)b->P * 2 * sizeof(float))) != hipSuccess ||
        (e = hipMalloc((void**)&b->d_rows, (size_t)(b->P + 1) * sizeof(int32_t))) != hipSuccess)
      return fail(VMAS_ERR_OUT_OF_MEMORY, "surrogate workspace: %s", hipGetErrorString(e));
  }
  if (forces) HIPCHK(launch_fill_f32(forces, 3 * (int64_t)b->N, 0.0f, s));
  const Plan& p = b->plans[b->lane_plan];  // lane records are needed
  if (p.groups == 0) return VMAS_OK;
  if (p.block > 256)
    return fail(VMAS_ERR_UNSUPPORTED, "surrogate step: environments with more than 256 movers");
  StepArgs a = make_args(b, p);
  a.state = state;
  a.actions = actions;
  a.T = 1;
  a.forces = forces;
  if (b->P > 0) {
    // candidates' features into consecutive rows, the network on those rows only
    int32_t* count = b->d_rows + b->P;
    HIPCHK(launch_fill_i32(count, 1, 0, s));
    if (b->cand.valid) {
      StepArgs ac = make_args(b, b->cand);
      ac.state = state;
      HIPCHK(launch_candidate_features(ac, b->cand.groups, b->cand.block, band, b->d_feat, b->d_rows,
                                       count, b->spheres_only, s));
    } else {
      HIPCHK(launch_candidate_features(a, p.groups, p.block, band, b->d_feat, b->d_rows, count,
                                       b->spheres_only, s));
    }
    // outputs scattered to the candidates' pair slots
    vmas_status st = mlp_forward_counted(mlp, b->d_feat, b->P, count, b->d_rows, b->d_yhat, s);
    if (st != VMAS_OK) return st;
  }
  HIPCHK(launch_step_surrogate(a, b->d_yhat, band, fallback_frac, n_fallback, p.groups, p.block,
                               b->spheres_only, s));
  return check_nonfinite(b, state, s);
}

vmas_status vmas_nonfinite_envs(vmas_batch* b, uint8_t* marks, int32_t* count, int32_t clear,
                                void* stream) {
  g_err.clear();
  if (check_batch(b) != VMAS_OK) return VMAS_ERR_INVALID_ARGUMENT;
  if (!b->debug_nonfinite)
    return fail(VMAS_ERR_INVALID_ARGUMENT, "the batch was created without VMAS_DEBUG_NONFINITE");
  DeviceGuard guard(b->device);
  hipStream_t s = (hipStream_t)stream;
  std::vector<uint32_t> m(b->n_envs);
  uint32_t c[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(m.data(), b->d_bad, m.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(c, b->d_bad_cnt, sizeof(c), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (marks)
    for (int e = 0; e < b->n_envs; ++e) marks[e] = m[e] ? 1 : 0;
  if (count) *count = (int32_t)c[1];
  if (clear) {
    HIPCHK(launch_fill_i32((int32_t*)b->d_bad, b->n_envs, 0, s));
    HIPCHK(launch_fill_i32((int32_t*)b->d_bad_cnt, 2, 0, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  return VMAS_OK;
}

}  // extern "C"
