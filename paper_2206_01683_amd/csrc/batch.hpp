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
  unsigned *bar;        // grid barrier words and the collide work queue (BAR_*, kBarWords)
};

// Barrier words, each on its own 128-byte line (indices into BatchArgs::bar):
// the top arrival count, the generation, the collide work queue, the status
// word, then one arrival count per group of kBarGroup workgroups.
constexpr int kBarLine = 32;
enum : int {
  BAR_TOP = 0,
  BAR_GEN = kBarLine,
  BAR_QUEUE = 2 * kBarLine,
  BAR_STATUS = 3 * kBarLine,
  BAR_GROUPS = 4 * kBarLine
};
constexpr int kBarGroup = 32;      // workgroups per first-level arrival count
constexpr int kBarMaxGroups = 64;  // so at most 2048 workgroups
constexpr int kBarWords = BAR_GROUPS + kBarMaxGroups * kBarLine;

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
// Returns the total. Every thread of the workgroup must call it. Up to 64
// environments the first wave scans them with lane shuffles (one barrier);
// more take the workgroup-wide scan.
__device__ inline int dynamic_prefix(const BatchArgs &b, int mult, int *s_pre, int tid) {
  int v = 0;
  if (tid < b.nenv) v = n_active_of(b.envs[tid]) * mult;
  if (b.nenv <= 64) {
    if (tid < 64) {
      const int lane = tid;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int up = __builtin_amdgcn_ds_bpermute((lane >= off ? lane - off : lane) << 2, v);
        if (lane >= off) v += up;
      }
      s_pre[tid + 1] = v;
      if (tid == 0) s_pre[0] = 0;
    }
    __syncthreads();
    return s_pre[b.nenv];
  }
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

// Step s's frame of environment e. The values are uniform over the
// workgroup: moving them to scalar registers keeps 18 vector registers free
// for the collide.
__device__ inline float uniform_f(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ inline FrameF env_frame(const EnvView &e, int s) {
  FrameF f = frame_from((const gmem<double> *)e.frames + (size_t)18 * s);
  for (int a = 0; a < 3; ++a) {
    f.acc[a] = uniform_f(f.acc[a]);
    f.omg[a] = uniform_f(f.omg[a]);
    f.alp[a] = uniform_f(f.alp[a]);
    f.org[a] = uniform_f(f.org[a]);
    f.ulo[a] = uniform_f(f.ulo[a]);
    f.uhi[a] = uniform_f(f.uhi[a]);
  }
  return f;
}
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
  spread_item<kBatchSpreadSplit>(e, local, tid);
}

// Collide item -> (environment, logical block); 512 threads as e.bx x e.by.
// Collide items are numbered over the environments in kind order (corder).
template <int K>
__device__ inline void phase_collide(const BatchArgs &b, const EnvView *__restrict__ envs, const int *__restrict__ pre0,
                                     const int *__restrict__ corder, int s, int item, int tid) {
  const int *pre = pre0 + PRE_COLLIDE * (b.nenv + 1);
  const int pos = find_env(pre, b.nenv, item);
  const EnvView &e = envs[corder[pos]];
  const FrameF fr = env_frame(e, s);
  const int lb = item - pre[pos];
  const int cur = env_cur(e, s);
  const int tx = tid % e.bx, ty = tid / e.bx;
  collide_item<K>(e, fr, cur, lb, tx, ty);
}

// Collide items handed out in launch order by a device-wide ticket counter
// (bar[BAR_QUEUE], cleared at every grid barrier), so that the resident workgroups
// sweep a compact, moving window of the lattices as the hardware's dispatch
// of a per-phase launch does (workgroups that each walked a contiguous range
// of their own streamed from hundreds of distant regions at once). Each
// workgroup fetches its next ticket while the current item runs.
template <bool UNI>
__device__ inline void collide_queue(const BatchArgs &b, int s, int tid) {
  __shared__ int s_ticket[2];
  const int total = b.tot[PRE_COLLIDE];
  const int *pre = b.pre + PRE_COLLIDE * (b.nenv + 1);
  if (tid == 0) s_ticket[0] = (int)atomicAdd(&b.bar[BAR_QUEUE], 1u);
  __syncthreads();
  for (int k = 0;; k ^= 1) {
    const int item = s_ticket[k];
    if (item >= total) break;  // the same value in every thread
    if (tid == 0) s_ticket[k ^ 1] = (int)atomicAdd(&b.bar[BAR_QUEUE], 1u);
    const int pos = find_env(pre, b.nenv, item);
    const EnvView &e = b.envs[b.corder[pos]];
    const int tx = tid % e.bx, ty = tid / e.bx;
    collide_item<UNI ? 0 : -1>(e, env_frame(e, s), env_cur(e, s), item - pre[pos], tx, ty);
    __syncthreads();  // the next ticket is visible; this one was read by every thread
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
  const int tot = dynamic_prefix(b, kBatchSpreadSplit, s_pre, threadIdx.x);
  for (int item = blockIdx.x; item < tot; item += gridDim.x) {
    const int ei = find_env(s_pre, b.nenv, item);
    const EnvView &e = b.envs[ei];
    spread_item<true, kBatchSpreadSplit>(e, item - s_pre[ei], threadIdx.x, e.gcg, cg_scal(e, 1, j), j == 0);
  }
}

// Grid: the total of PRE_INTERP (each environment's interpolation items).
__global__ void __launch_bounds__(WG) kb_cg_apply(BatchArgs b, int j) {
  const int *pre = b.pre + PRE_INTERP * (b.nenv + 1);
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const int ei = find_env(pre, b.nenv, item);
  cg_apply_item(b.envs[ei], item - pre[ei], threadIdx.x, j);
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
  const XcdWalk w = xcd_walk(dynamic_prefix(b, 1, s_pre, threadIdx.x));
  for (int item = w.first; item < w.end; item += w.step) phase_macro<UNI, true>(b, s, item, s_pre, threadIdx.x);
}

template <bool UNI>
__global__ void __launch_bounds__(WG) kb_interp(BatchArgs b, int s, int pass) {
  // grid = every environment's interpolation items; each XCD takes consecutive
  // items (the markers of a few environments), so its L2 holds their band macros
  phase_interp<UNI>(b, s, pass, xcd_item(blockIdx.x, gridDim.x), threadIdx.x);
}

__global__ void __launch_bounds__(WG) kb_spread(BatchArgs b, int s, int final_pass) {
  __shared__ int s_pre[kMaxEnvs + 1];
  const int tot = dynamic_prefix(b, kBatchSpreadSplit, s_pre, threadIdx.x);
  for (int item = blockIdx.x; item < tot; item += gridDim.x)
    phase_spread(b, s, final_pass != 0, item, s_pre, threadIdx.x);
}

// Collide items item0 .. item0 + gridDim.x - 1, all of environments of kind
// K, one per workgroup in launch order (the same mapping as the
// single-lattice collide). One launch per kind present.
template <int K>
__global__ void __launch_bounds__(WG) kb_collide(BatchArgs b, const EnvView *__restrict__ envs,
                                                 const int *__restrict__ pre, const int *__restrict__ corder, int s,
                                                 int item0) {
  const int item = item0 + blockIdx.x;
  if (item < b.tot[PRE_COLLIDE]) phase_collide<K>(b, envs, pre, corder, s, item, threadIdx.x);
}

// --------------------------------------------------------- grid barrier ----
constexpr long kBarrierSpins = 1L << 24;  // ~1 s of waiting: a longer wait is a failure

// Device-wide barrier for a co-resident grid, in two levels: a workgroup
// arrives on its group's count; the last of a group arrives on the top count;
// the last of those clears the work queue and advances the generation, which
// the others wait for. Spreading the arrivals over lines cuts the chain of
// serialized device-scope atomics from one per workgroup to about
// kBarGroup + groups.
// Memory ordering: each arrival is an acquire-release read-modify-write at
// device scope (it writes this workgroup's L2 lines back before it counts),
// and a waiter polls the generation with relaxed loads and acquires once when
// it changes. An acquiring poll would invalidate its XCD's L2 on every
// iteration, under the feet of the workgroups still busy in the phase.
// Returns false (in every thread) after a timeout.
__device__ inline bool grid_sync(const BatchArgs &b) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned gen = __hip_atomic_load(&b.bar[BAR_GEN], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned nwg = gridDim.x;
    const unsigned grp = blockIdx.x / kBarGroup;
    const unsigned ngrp = (nwg + kBarGroup - 1) / kBarGroup;
    const unsigned in_grp = min((unsigned)kBarGroup, nwg - grp * kBarGroup);
    unsigned *gc = &b.bar[BAR_GROUPS + grp * kBarLine];
    bool last = false;
    if (__hip_atomic_fetch_add(gc, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == in_grp - 1) {
      __hip_atomic_store(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = __hip_atomic_fetch_add(&b.bar[BAR_TOP], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == ngrp - 1;
    }
    if (last) {
      __hip_atomic_store(&b.bar[BAR_TOP], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&b.bar[BAR_QUEUE], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // empty work queue
      __hip_atomic_fetch_add(&b.bar[BAR_GEN], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long spins = 0;
      while (__hip_atomic_load(&b.bar[BAR_GEN], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > kBarrierSpins) {
          ok = 0;
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    int *status = reinterpret_cast<int *>(&b.bar[BAR_STATUS]);
    if (!ok) atomicOr(status, 1);
    if (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1) ok = 0;
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// Thread index for one phase of the persistent kernel. It passes through an
// empty asm so that the index arithmetic of each phase stays inside that
// phase: hoisted out of the step loop, every phase's per-thread addresses
// would stay live across all the others and spill.
__device__ inline int phase_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}
// The workgroup index and grid size likewise (scalar registers).
__device__ inline int phase_blk() {
  int t = blockIdx.x;
  asm volatile("" : "+s"(t));
  return t;
}
__device__ inline int phase_grid() {
  int t = gridDim.x;
  asm volatile("" : "+s"(t));
  return t;
}

// All steps of all environments in one launch (grid: co-resident, multiple of
// 8). The launch bound asks for at least 6 waves per SIMD (at most 80 VGPRs):
// three 512-thread workgroups per CU. The collide phase takes its items from
// a work queue in launch order.
template <bool UNI>
__global__ void __launch_bounds__(WG, 6) kb_persistent(BatchArgs b, int nsteps) {
  __shared__ int s_pre[kMaxEnvs + 1];
  for (int s = 0; s < nsteps; ++s) {
    {
      const int tid = phase_tid(), blk = phase_blk(), grid = phase_grid();
      for (int item = blk; item < b.tot[PRE_SKIN]; item += grid) phase_skin(b, s, item, tid);
    }
    if (!grid_sync(b)) return;
    {
      const int tid = phase_tid(), blk = phase_blk(), grid = phase_grid();
      for (int item = blk; item < b.tot[PRE_ACTIVE]; item += grid) phase_active(b, item, tid);
    }
    if (!grid_sync(b)) return;
    {
      const int tid = phase_tid(), blk = phase_blk(), grid = phase_grid();
      const int tot = dynamic_prefix(b, 1, s_pre, tid);
      const XcdWalk w = xcd_walk(tot, blk, grid);
      for (int item = w.first; item < w.end; item += w.step) phase_macro<UNI>(b, s, item, s_pre, tid);
    }
    if (!grid_sync(b)) return;
    int tot;
    {
      const int tid = phase_tid();
      tot = dynamic_prefix(b, kBatchSpreadSplit, s_pre, tid);
    }
    for (int pass = 0; pass < b.mdf; ++pass) {
      if (pass > 0) {
        const int tid = phase_tid(), blk = phase_blk(), grid = phase_grid();
        for (int item = blk; item < tot; item += grid) phase_spread(b, s, false, item, s_pre, tid);
        if (!grid_sync(b)) return;
      }
      {
        const int tid = phase_tid(), blk = phase_blk(), grid = phase_grid();
        for (int item = blk; item < b.tot[PRE_INTERP]; item += grid)
          phase_interp<UNI>(b, s, pass, item, tid);
      }
      if (!grid_sync(b)) return;
    }
    {
      const int tid = phase_tid(), blk = phase_blk(), grid = phase_grid();
      for (int item = blk; item < tot; item += grid) phase_spread(b, s, true, item, s_pre, tid);
    }
    if (!grid_sync(b)) return;
    {
      collide_queue<UNI>(b, s, phase_tid());
    }
    if (!grid_sync(b)) return;
  }
}

}  // namespace lbmib
