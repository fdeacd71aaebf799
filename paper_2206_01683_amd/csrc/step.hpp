// One lattice step with the immersed-boundary phases running beside the
// collide in a single launch. This step's markers were skinned and their
// tiles binned into this step's tile map before the launch (by the previous
// step's launch, or by launches of their own for the first step of a call).
//
// Workgroups [0, nib) run the immersed-boundary chain, with barriers among
// themselves: band macros, interpolation with direct forcing (and its
// multi-direct passes), spreading into the fixed-point force; then they count
// themselves done, skin the next step's markers and bin its tiles into the
// other tile map (the two maps alternate between steps). The other workgroups
// are the collide blocks, in launch order as in k_collide. A block none of
// whose cells lies in an active tile needs no immersed force and collides at
// once; a block with band cells waits for the chain first. Active tiles fill
// a fraction of a percent of the lattice, so nearly all of the collide's
// 216 B per cell stream while the latency-bound chain runs, instead of after
// it, and a step is one launch.
//
// Correctness does not depend on timing: the chain reads the source buffer
// (cur) and writes its own band arrays, the next step's marker data and the
// other tile map, none of which the collide reads; the collide writes the
// other population buffer, reads this step's tile map (complete before the
// launch) and reads the immersed force only after the done count, by an
// acquire. The done count grows over the launches of a call (the host passes
// each launch's target). The chain's workgroups are the lowest-numbered, so
// they are resident before any collide block can wait for them. The
// arithmetic is the same inline code as the separate kernels', so results
// agree bit for bit.
#pragma once

#include "ib.hpp"

namespace lbmib {

// Barrier among the nib chain workgroups (co-resident: dispatched first).
// Arrival is an acquire-release read-modify-write at device scope; waiters
// poll with relaxed loads and acquire once.
__device__ inline void chain_sync(unsigned *sched, int nib) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned gen = __hip_atomic_load(&sched[SCHED_GEN], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__hip_atomic_fetch_add(&sched[SCHED_ARRIVE], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
        (unsigned)nib - 1) {
      __hip_atomic_store(&sched[SCHED_ARRIVE], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&sched[SCHED_GEN], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      while (__hip_atomic_load(&sched[SCHED_GEN], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen)
        __builtin_amdgcn_s_sleep(2);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  __syncthreads();
}

// The chain of workgroup blk of nib: the same phases and order as the
// separate launches of step_one (macro; per pass: spread of the force so far
// after the first, interpolation; final spread with the wrench sum), then,
// when next_pose is not null, the next step's skinning and binning into
// next_slots.
template <class S, bool ROT>
__device__ inline void ib_chain(const EnvView &e, const FrameF &fr, int cur, int blk, int nib, int passes,
                                float *wrench, const float *next_pose, int *next_slots, int tid) {
  unsigned *sched = e.sched;
  const int na = n_active_of(e);
  for (int slot = blk; slot < na; slot += nib) macro_item<S, ROT>(e, fr, cur, slot, tid);
  chain_sync(sched, nib);
  const int nspread = na * kSpreadSplit, ninterp = interp_items(e.n);
  for (int it = 0; it < passes; ++it) {
    if (it > 0) {
      for (int item = blk; item < nspread; item += nib) spread_item(e, item, tid);
      chain_sync(sched, nib);
    }
    float *part = (wrench != nullptr && it == passes - 1) ? e.partials : nullptr;
    for (int item = blk; item < ninterp; item += nib) {
      if (it > 0)
        interp_item<ROT, true>(e, fr, item, tid, part);
      else
        interp_item<ROT, false>(e, fr, item, tid, part);
    }
    chain_sync(sched, nib);
  }
  if (blk == 0 && wrench != nullptr) wrench_sum(e.partials, ninterp, wrench, tid);
  for (int item = blk; item < nspread; item += nib) spread_item(e, item, tid);
  __syncthreads();
  if (tid == 0) __hip_atomic_fetch_add(&sched[SCHED_DONE], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  if (next_pose == nullptr) return;
  // the next step, once every chain workgroup has finished spreading (which
  // reads this step's marker data, chunk boxes and active list)
  chain_sync(sched, nib);
  for (int item = blk; item < skin_items(e.n); item += nib) skin_item(e, next_pose, item, tid);
  chain_sync(sched, nib);
  for (int item = blk; item < active_items(e); item += nib) active_item(e, item, tid, false, next_slots);
}

// Grid: nib + e.nblocks workgroups of WG threads; the collide shape of e is
// linear (e.by == 0, e.bx == WG) or 2-D with e.bx * e.by == WG. e.tile_slot:
// this step's tile map; done_target: the done count once this launch's chain
// has finished its spreading.
template <class S, bool XPER, bool ROT, bool YZ, bool TRT>
__global__ void __launch_bounds__(WG) k_step_overlap(EnvView e, FrameF fr, int cur, int nib, int passes,
                                                      float *wrench, const float *next_pose, int *next_slots,
                                                      unsigned done_target) {
  const int tid = threadIdx.x;
  if ((int)blockIdx.x < nib) {
    ib_chain<S, ROT>(e, fr, cur, blockIdx.x, nib, passes, wrench, next_pose, next_slots, tid);
    return;
  }
  const int lb = (int)blockIdx.x - nib;
  if (lb >= e.nblocks) return;
  const int tx = e.by == 0 ? tid : tid % e.bx, ty = e.by == 0 ? 0 : tid / e.bx;
  CellAt c;
  float f[Q];
  const bool have = collide_load<S, XPER, YZ>(e, cur, lb, tx, ty, c, f);
  // a band cell reads the immersed force at its source node (xs, ys, zs)
  int band = 0;
  if (have) {
    const int ys = YZ ? c.ys : c.y, zs = YZ ? c.zs : c.z;
    band = e.tile_slot[(c.xs >> 3) + e.g.tnx * ((ys >> 3) + e.g.tny * (zs >> 3))] >= 0;
  }
  if (__syncthreads_or(band)) {
    if (tid == 0) {
      while (__hip_atomic_load(&e.sched[SCHED_DONE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < done_target)
        __builtin_amdgcn_s_sleep(2);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
  }
  if (have) collide_finish<S, XPER, ROT, YZ, TRT>(e, fr, cur, c, f);
}

}  // namespace lbmib
