// Batched forms: many environments (lattices of different sizes, each with
// its own body) advanced together.
//
// Every phase of a step becomes one work list over all environments: item i
// of a phase belongs to the environment whose prefix range holds it. Static
// item counts (markers, tiles, collide blocks) come with host-computed
// prefixes; the active-tile counts are only known on the device, so the
// macro and spreading phases build their prefix in LDS from the counters.
// Two drivers use the same phase functions:
//   kb_* kernels     one launch per phase (a step = 6+ launches; the collide
//                    one launch per collide kind present, each specialised),
//                    suitable for capture into a graph of many steps; they
//                    also take 2-byte storage and the implicit correction;
//   kb_persistent    one launch for all steps: each workgroup loops over the
//                    phases, separated by a device-wide barrier. The grid is
//                    sized to be co-resident; the barrier's wait is bounded
//                    (a timeout sets a status bit and every workgroup exits).
//                    F32 storage and direct forcing only.
// UNI = true: every environment is of collide kind 0 (open x faces, no
// rotation, periodic y and z, BGK, F32), so the per-environment branches on
// those flags compile away. The interpolation branches on rotation only, so
// the per-phase driver takes its UNI template whenever no frame rotates.
#pragma once

#include "ib.hpp"

namespace lbmib {

constexpr int kMaxEnvs = WG;  // one thread per environment in the LDS prefix scan

struct BatchArgs {
  const EnvView *envs;  // [nenv]
  int nenv;
  const int *pre;       // [PRE_ROWS][nenv + 1] exclusive item prefixes (rows named by PRE_*)
  const int *corder;    // [nenv] environment at each position of the collide prefix (grouped by kind)
  int tot[4];
  int mdf;              // direct-forcing passes
  unsigned *bar;        // grid barrier: [0] arrivals, [1] generation
  int *status;          // bit 0: barrier timeout
};

// Rows of BatchArgs::pre: per-environment exclusive item prefixes (row 4 holds
// the collide order, corder); PRE_CG counts conjugate-gradient items.
enum { PRE_SKIN = 0, PRE_ACTIVE = 1, PRE_INTERP = 2, PRE_COLLIDE = 3, PRE_CG = 5, PRE_ROWS = 6 };

// Largest e with pre[e] <= item (pre non-decreasing, pre[nenv] > item).
__device__ inline int find_env(const int *pre, int nenv, int item) {
  int lo = 0, hi = nenv;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= item)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Exclusive prefix over environments of (active tiles x mult), in LDS.
// Returns the total. Every thread of the workgroup must call it.
__device__ inline int dynamic_prefix(const BatchArgs &b, int mult, int *s_pre, int tid) {
  int v = 0;
  if (tid < b.nenv) v = n_active_of(b.envs[tid]) * mult;
  s_pre[tid + 1] = v;
  if (tid == 0) s_pre[0] = 0;
  __syncthreads();
  for (int off = 1; off < WG; off <<= 1) {
    const int add = tid >= off ? s_pre[tid + 1 - off] : 0;
    __syncthreads();
    s_pre[tid + 1] += add;
    __syncthreads();
  }
  return s_pre[b.nenv];
}

__device__ inline FrameF env_frame(const EnvView &e, int s) { return frame_from(e.frames + (size_t)18 * s); }
__device__ inline int env_cur(const EnvView &e, int s) { return e.cur0 ^ (s & 1); }

// collide_cell for any environment of one collision kind: boundary kind and
// frame chosen at run time.
template <bool TRT>
__device__ inline void collide_any_t(const EnvView &e, const FrameF &fr, int cur, int lb, int tx, int ty) {
  if (!(e.g.yper && e.g.zper)) {
    if (e.g.xper)
      e.rot ? collide_cell<StoreF32, true, true, true, TRT>(e, fr, cur, lb, tx, ty)
            : collide_cell<StoreF32, true, false, true, TRT>(e, fr, cur, lb, tx, ty);
    else
      e.rot ? collide_cell<StoreF32, false, true, true, TRT>(e, fr, cur, lb, tx, ty)
            : collide_cell<StoreF32, false, false, true, TRT>(e, fr, cur, lb, tx, ty);
  } else if (e.g.xper) {
    e.rot ? collide_cell<StoreF32, true, true, false, TRT>(e, fr, cur, lb, tx, ty)
          : collide_cell<StoreF32, true, false, false, TRT>(e, fr, cur, lb, tx, ty);
  } else {
    e.rot ? collide_cell<StoreF32, false, true, false, TRT>(e, fr, cur, lb, tx, ty)
          : collide_cell<StoreF32, false, false, false, TRT>(e, fr, cur, lb, tx, ty);
  }
}

// Any environment: boundary kind, rotation and collision (BGK or TRT) from
// its view, each uniform over a workgroup.
__device__ inline void collide_any(const EnvView &e, const FrameF &fr, int cur, int lb, int tx, int ty) {
  if (e.two_rate)
    collide_any_t<true>(e, fr, cur, lb, tx, ty);
  else
    collide_any_t<false>(e, fr, cur, lb, tx, ty);
}

// Collide kind of an environment: bit 0 periodic x, bit 1 rotating frame,
// bit 2 an open y or z face, bit 3 TRT; bits 4-5 the population format
// (Store*::kind). Kind 0 (open x, no rotation, periodic y and z, BGK, F32)
// is the common case.
enum { kCollideKinds = 48 };
__host__ __device__ inline int collide_kind(const EnvView &e) {
  return (e.g.xper ? 1 : 0) | (e.rot ? 2 : 0) | (e.g.yper && e.g.zper ? 0 : 4) | (e.two_rate ? 8 : 0) |
         (e.storage << 4);
}

template <int SK> struct StoreOf { using type = StoreF32; };
template <> struct StoreOf<1> { using type = StoreF16; };
template <> struct StoreOf<2> { using type = StoreBF16; };

// K >= 0: the environment is of kind K (one specialised collide, registers
// of that variant only); K < 0: any F32 kind, chosen at run time.
template <int K>
__device__ inline void collide_item(const EnvView &e, const FrameF &fr, int cur, int lb, int tx, int ty) {
  if constexpr (K < 0)
    collide_any(e, fr, cur, lb, tx, ty);
  else
    collide_cell<typename StoreOf<(K >> 4)>::type, (K & 1) != 0, (K & 2) != 0, (K & 4) != 0, (K & 8) != 0>(
        e, fr, cur, lb, tx, ty);
}

// ------------------------------------------------------------ phase bodies --
__device__ inline void phase_skin(const BatchArgs &b, int s, int item, int tid) {
  const int ei = find_env(b.pre + PRE_SKIN * (b.nenv + 1), b.nenv, item);
  const EnvView &e = b.envs[ei];
  skin_item(e, e.poses + (size_t)s * e.nbones * 24, item - b.pre[PRE_SKIN * (b.nenv + 1) + ei], tid);
}

__device__ inline void phase_active(const BatchArgs &b, int item, int tid) {
  const int ei = find_env(b.pre + PRE_ACTIVE * (b.nenv + 1), b.nenv, item);
  active_item(b.envs[ei], item - b.pre[PRE_ACTIVE * (b.nenv + 1) + ei], tid);
}

template <class S, bool UNI>
__device__ inline void macro_rot(const EnvView &e, const FrameF &fr, int cur, int slot, int tid) {
  if (!UNI && e.rot)
    macro_item<S, true>(e, fr, cur, slot, tid);
  else
    macro_item<S, false>(e, fr, cur, slot, tid);
}

// ANYS: environments may store 2-byte populations (per-phase driver); the
// persistent kernel takes F32 only.
template <bool UNI, bool ANYS = false>
__device__ inline void phase_macro(const BatchArgs &b, int s, int item, const int *s_pre, int tid) {
  const int ei = find_env(s_pre, b.nenv, item);
  const EnvView &e = b.envs[ei];
  const FrameF fr = env_frame(e, s);
  const int cur = env_cur(e, s), slot = item - s_pre[ei];
  if (!UNI && ANYS && e.storage == StoreF16::kind)
    macro_rot<StoreF16, UNI>(e, fr, cur, slot, tid);
  else if (!UNI && ANYS && e.storage == StoreBF16::kind)
    macro_rot<StoreBF16, UNI>(e, fr, cur, slot, tid);
  else
    macro_rot<StoreF32, UNI>(e, fr, cur, slot, tid);
}

template <bool UNI>
__device__ inline void phase_interp(const BatchArgs &b, int s, int pass, int item, int tid) {
  const int ei = find_env(b.pre + PRE_INTERP * (b.nenv + 1), b.nenv, item);
  const EnvView &e = b.envs[ei];
  const FrameF fr = env_frame(e, s);
  const int local = item - b.pre[PRE_INTERP * (b.nenv + 1) + ei];
  float *part = (e.wrench != nullptr && pass == b.mdf - 1) ? e.partials : nullptr;
  if (!UNI && e.rot) {
    if (pass > 0)
      interp_item<true, true>(e, fr, local, tid, part);
    else
      interp_item<true, false>(e, fr, local, tid, part);
  } else {
    if (pass > 0)
      interp_item<false, true>(e, fr, local, tid, part);
    else
      interp_item<false, false>(e, fr, local, tid, part);
  }
}

// final: the step's last spreading pass; its first item per environment also
// sums the wrench partials.
__device__ inline void phase_spread(const BatchArgs &b, int s, bool final_pass, int item, const int *s_pre,
                                    int tid) {
  const int ei = find_env(s_pre, b.nenv, item);
  const EnvView &e = b.envs[ei];
  const int local = item - s_pre[ei];
  if (final_pass && local == 0 && e.wrench != nullptr)
    wrench_sum(e.partials, interp_items(e.n), e.wrench + (size_t)8 * s, tid);
  spread_item(e, local, tid);
}

// Collide item -> (environment, logical block); 512 threads as e.bx x e.by.
// Collide items are numbered over the environments in kind order (corder).
template <int K>
__device__ inline void phase_collide(const BatchArgs &b, int s, int item, int tid) {
  const int *pre = b.pre + PRE_COLLIDE * (b.nenv + 1);
  const int pos = find_env(pre, b.nenv, item);
  const EnvView &e = b.envs[b.corder[pos]];
  const FrameF fr = env_frame(e, s);
  const int lb = item - pre[pos];
  const int cur = env_cur(e, s);
  const int tx = tid % e.bx, ty = tid / e.bx;
  collide_item<K>(e, fr, cur, lb, tx, ty);
}

// Collide items [i0, i1) in order, looking the environment up once per run
// of items that belong to it (a persistent workgroup walks a contiguous range).
template <bool UNI>
__device__ inline void collide_range(const BatchArgs &b, int s, int i0, int i1, int tid) {
  const int *pre = b.pre + PRE_COLLIDE * (b.nenv + 1);
  int item = i0;
  while (item < i1) {
    const int pos = find_env(pre, b.nenv, item);
    const EnvView &e = b.envs[b.corder[pos]];
    const FrameF fr = env_frame(e, s);
    const int cur = env_cur(e, s);
    const int lo = pre[pos], hi = min(pre[pos + 1], i1);
    const int tx = tid % e.bx, ty = tid / e.bx;
    for (; item < hi; ++item) collide_item<UNI ? 0 : -1>(e, fr, cur, item - lo, tx, ty);
  }
}

// ------------------------------------- implicit velocity correction, batched --
// Each environment's conjugate gradients, as in the single-lattice kernels:
// every environment counts the last-arrival of its own items (its own
// counters), so one launch covers the items of all environments. The batch
// runs them when every environment uses LBM_IB_IMPLICIT (per-phase driver).
__global__ void __launch_bounds__(kCgWG) kb_cg_init(BatchArgs b, int s) {
  const int *pre = b.pre + PRE_CG * (b.nenv + 1);
  const int ei = find_env(pre, b.nenv, blockIdx.x);
  const EnvView &e = b.envs[ei];
  const FrameF fr = env_frame(e, s);
  if (e.rot)
    cg_init_item<true>(e, fr, blockIdx.x - pre[ei]);
  else
    cg_init_item<false>(e, fr, blockIdx.x - pre[ei]);
}

// Spreading of CG step j's search direction into each environment's gcg.
__global__ void __launch_bounds__(WG) kb_spread_cg(BatchArgs b, int j) {
  __shared__ int s_pre[kMaxEnvs + 1];
  const int tot = dynamic_prefix(b, kSpreadSplit, s_pre, threadIdx.x);
  for (int item = blockIdx.x; item < tot; item += gridDim.x) {
    const int ei = find_env(s_pre, b.nenv, item);
    const EnvView &e = b.envs[ei];
    spread_item<true>(e, item - s_pre[ei], threadIdx.x, e.gcg, cg_scal(e, 1, j), j == 0);
  }
}

// Grid: the total of PRE_INTERP (each environment's interpolation items).
__global__ void __launch_bounds__(WG) kb_cg_apply(BatchArgs b, int j) {
  const int *pre = b.pre + PRE_INTERP * (b.nenv + 1);
  const int ei = find_env(pre, b.nenv, blockIdx.x);
  cg_apply_item(b.envs[ei], blockIdx.x - pre[ei], threadIdx.x, j);
}

// Grid: the total of PRE_CG.
__global__ void __launch_bounds__(kCgWG) kb_cg_update(BatchArgs b, int s, int j, int last) {
  const int *pre = b.pre + PRE_CG * (b.nenv + 1);
  const int ei = find_env(pre, b.nenv, blockIdx.x);
  const EnvView &e = b.envs[ei];
  cg_update_item(e, env_frame(e, s), blockIdx.x - pre[ei], j, last != 0);
}

// Clears gcg of every active tile before the next CG step's spreading.
__global__ void __launch_bounds__(WG) kb_cg_clear(BatchArgs b) {
  __shared__ int s_pre[kMaxEnvs + 1];
  const int tot = dynamic_prefix(b, 1, s_pre, threadIdx.x);
  for (int item = blockIdx.x; item < tot; item += gridDim.x) {
    const int ei = find_env(s_pre, b.nenv, item);
    unsigned long long *gq = b.envs[ei].gcg + (size_t)(item - s_pre[ei]) * 1536;
    for (int q = threadIdx.x; q < 1536; q += WG) gq[q] = 0ull;
  }
}

// ------------------------------------------------------ per-phase kernels --
__global__ void __launch_bounds__(WG) kb_skin(BatchArgs b, int s) { phase_skin(b, s, blockIdx.x, threadIdx.x); }

__global__ void __launch_bounds__(WG) kb_active(BatchArgs b) { phase_active(b, blockIdx.x, threadIdx.x); }

template <bool UNI>
__global__ void __launch_bounds__(WG) kb_macro(BatchArgs b, int s) {
  __shared__ int s_pre[kMaxEnvs + 1];
  const int tot = dynamic_prefix(b, 1, s_pre, threadIdx.x);
  for (int item = blockIdx.x; item < tot; item += gridDim.x) phase_macro<UNI, true>(b, s, item, s_pre, threadIdx.x);
}

template <bool UNI>
__global__ void __launch_bounds__(WG) kb_interp(BatchArgs b, int s, int pass) {
  phase_interp<UNI>(b, s, pass, blockIdx.x, threadIdx.x);
}

__global__ void __launch_bounds__(WG) kb_spread(BatchArgs b, int s, int final_pass) {
  __shared__ int s_pre[kMaxEnvs + 1];
  const int tot = dynamic_prefix(b, kSpreadSplit, s_pre, threadIdx.x);
  for (int item = blockIdx.x; item < tot; item += gridDim.x)
    phase_spread(b, s, final_pass != 0, item, s_pre, threadIdx.x);
}

// Collide items item0 .. item0 + gridDim.x - 1, all of environments of kind
// K, one per workgroup in launch order (the same mapping as the
// single-lattice collide). One launch per kind present.
template <int K>
__global__ void __launch_bounds__(WG) kb_collide(BatchArgs b, int s, int item0) {
  const int item = item0 + blockIdx.x;
  if (item < b.tot[PRE_COLLIDE]) phase_collide<K>(b, s, item, threadIdx.x);
}

// --------------------------------------------------------- grid barrier ----
constexpr long kBarrierSpins = 1L << 25;  // ~1 s of waiting: a longer wait is a failure

// Device-wide barrier for a co-resident grid. Release: each workgroup's
// writes are made visible at device scope before it arrives; acquire: after
// the generation changes. Returns false (in every thread) after a timeout.
__device__ inline bool grid_sync(const BatchArgs &b) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    __threadfence();
    const unsigned gen = __hip_atomic_load(&b.bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned arrived = __hip_atomic_fetch_add(&b.bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == gridDim.x - 1) {
      __hip_atomic_store(&b.bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&b.bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long spins = 0;
      while (__hip_atomic_load(&b.bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kBarrierSpins) {
          ok = 0;
          break;
        }
      }
    }
    if (!ok) atomicOr(b.status, 1);
    if (__hip_atomic_load(b.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1) ok = 0;
    __threadfence();
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// All steps of all environments in one launch (grid: co-resident, multiple of
// 8). The launch bound asks for at least 4 waves per SIMD (at most 128 VGPRs),
// so that two 512-thread workgroups share a CU; the collide phase gives each
// workgroup a contiguous range of items.
template <bool UNI>
__global__ void __launch_bounds__(WG, 4) kb_persistent(BatchArgs b, int nsteps) {
  __shared__ int s_pre[kMaxEnvs + 1];
  const int tid = threadIdx.x;
  for (int s = 0; s < nsteps; ++s) {
    for (int item = blockIdx.x; item < b.tot[PRE_SKIN]; item += gridDim.x) phase_skin(b, s, item, tid);
    if (!grid_sync(b)) return;
    for (int item = blockIdx.x; item < b.tot[PRE_ACTIVE]; item += gridDim.x) phase_active(b, item, tid);
    if (!grid_sync(b)) return;
    int tot = dynamic_prefix(b, 1, s_pre, tid);
    for (int item = blockIdx.x; item < tot; item += gridDim.x) phase_macro<UNI>(b, s, item, s_pre, tid);
    if (!grid_sync(b)) return;
    tot = dynamic_prefix(b, kSpreadSplit, s_pre, tid);
    for (int pass = 0; pass < b.mdf; ++pass) {
      if (pass > 0) {
        for (int item = blockIdx.x; item < tot; item += gridDim.x) phase_spread(b, s, false, item, s_pre, tid);
        if (!grid_sync(b)) return;
      }
      for (int item = blockIdx.x; item < b.tot[PRE_INTERP]; item += gridDim.x)
        phase_interp<UNI>(b, s, pass, item, tid);
      if (!grid_sync(b)) return;
    }
    for (int item = blockIdx.x; item < tot; item += gridDim.x) phase_spread(b, s, true, item, s_pre, tid);
    if (!grid_sync(b)) return;
    {
      const int total = b.tot[PRE_COLLIDE];
      const int per = (total + (int)gridDim.x - 1) / (int)gridDim.x;
      const int i0 = min(total, (int)blockIdx.x * per);
      collide_range<UNI>(b, s, i0, min(total, i0 + per), tid);
    }
    if (!grid_sync(b)) return;
  }
}

}  // namespace lbmib
