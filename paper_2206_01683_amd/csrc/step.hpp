// One lattice step with the immersed-boundary phases running beside the
// collide in a single launch. This step's markers were skinned and their
// tiles binned into this step's tile map before the launch (by the previous
// step's launch, or by launches of their own for the first step of a call).
//
// Workgroups [0, nib) run the immersed-boundary chain, with barriers among
// themselves: band macros, interpolation with direct forcing (and its
// multi-direct passes), spreading into the fixed-point force, then the
// collide of the band cells (those whose source node lies in an active tile,
// the only cells with an immersed force); then they skin the next step's
// markers and bin its tiles into the other tile map (the two maps alternate
// between steps). The other workgroups are the collide blocks, in launch
// order as in k_collide: each collides its cells outside the band at once and
// leaves the band cells to the chain. Active tiles fill a fraction of a
// percent of the lattice, so nearly all of the collide's 216 B per cell
// stream while the latency-bound chain runs, no collide block waits for it,
// and a step is one launch.
//
// Correctness does not depend on timing: the chain reads the source buffer
// (cur) and writes its own band arrays, the band cells of the other buffer,
// the next step's marker data and the other tile map; the collide blocks read
// the source buffer and this step's tile map (complete before the launch) and
// write the other buffer outside the band. The two never touch the same
// words. The arithmetic is the same inline code as the separate kernels', so
// results agree bit for bit.
#pragma once

#include "ib.hpp"

namespace lbmib {

// Polls of a chain barrier before a waiter gives up (well over a second):
// the host keeps the chain within what the device holds at once, so only a
// device shared with work that never yields its slots can reach it.
constexpr long kChainSpins = 1L << 22;

// Barrier among the nib chain workgroups (co-resident: dispatched first).
// Arrival is an acquire-release read-modify-write at device scope; waiters
// poll with relaxed loads and acquire once. A waiter that gives up raises
// the schedule guard and goes on (its results are then void), so that the
// launch always ends.
__device__ inline void chain_sync(unsigned *sched, int nib, int *guard) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned gen = __hip_atomic_load(&sched[SCHED_GEN], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__hip_atomic_fetch_add(&sched[SCHED_ARRIVE], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
        (unsigned)nib - 1) {
      __hip_atomic_store(&sched[SCHED_ARRIVE], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&sched[SCHED_GEN], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long spins = 0;
      while (__hip_atomic_load(&sched[SCHED_GEN], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > kChainSpins) {
          atomicOr(guard, (int)GUARD_SCHEDULE);
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  __syncthreads();
}

// The band cells of active slot `slot`: the cells whose source node lies in
// its tile, that is the tile's own cells, and on an open face whose last tile
// is one node wide (a dimension of 8k + 1) also the face nodes beyond it
// (the source node of a face node is its inward neighbour). A cell of the
// box whose source lies in another tile is that tile's.
template <class S, bool XPER, bool ROT, bool YZ, bool TRT>
__device__ inline void band_collide_item(const EnvView &e, const FrameF &fr, int cur, int slot, int tid) {
  const GridArgs &g = e.g;
  const int t = ((const gmem<int> *)e.active)[slot];
  const int tx = t % g.tnx, rest = t / g.tnx, ty = rest % g.tny, tz = rest / g.tny;
  const int x0 = tx << 3, y0 = ty << 3, z0 = tz << 3;
  int x1 = min(x0 + 8, g.nx), y1 = min(y0 + 8, g.ny), z1 = min(z0 + 8, g.nz);
  if (!XPER && x1 == g.nx - 1) ++x1;
  if (YZ && !g.yper && y1 == g.ny - 1) ++y1;
  if (YZ && !g.zper && z1 == g.nz - 1) ++z1;
  const int ex = x1 - x0, ey = y1 - y0, cnt = ex * ey * (z1 - z0);
  for (int lc = tid; lc < cnt; lc += WG) {
    const int x = x0 + lc % ex, r = lc / ex, y = y0 + r % ey, z = z0 + r / ey;
    const CellAt c = cell_at<XPER, YZ>(g, x, y, z);
    if (((c.xs >> 3) != tx) | ((c.ys >> 3) != ty) | ((c.zs >> 3) != tz)) continue;
    float f[Q];
    collide_pull<S, XPER, YZ>(e, cur, c, f);
    collide_finish<S, XPER, ROT, YZ, TRT>(e, fr, cur, c, f);
  }
}

// The chain of workgroup blk of nib: the same phases and order as the
// separate launches of step_one (macro; per pass: spread of the force so far
// after the first, interpolation; final spread with the wrench sum), the
// collide of the band cells, then, when next_pose is not null, the next
// step's skinning and binning into next_slots.
template <class S, bool XPER, bool ROT, bool YZ, bool TRT>
__device__ inline void ib_chain(const EnvView &e, const FrameF &fr, int cur, int blk, int nib, int passes,
                                float *wrench, const float *next_pose, int *next_slots, int tid) {
  unsigned *sched = e.sched;
  const int na = n_active_of(e);
  for (int slot = blk; slot < na; slot += nib) macro_item<S, ROT>(e, fr, cur, slot, tid);
  chain_sync(sched, nib, e.guard);
  const int nspread = na * kSpreadSplit, ninterp = interp_items(e.n);
  for (int it = 0; it < passes; ++it) {
    if (it > 0) {
      for (int item = blk; item < nspread; item += nib) spread_item(e, item, tid);
      chain_sync(sched, nib, e.guard);
    }
    float *part = (wrench != nullptr && it == passes - 1) ? e.partials : nullptr;
    for (int item = blk; item < ninterp; item += nib) {
      if (it > 0)
        interp_item<ROT, true>(e, fr, item, tid, part);
      else
        interp_item<ROT, false>(e, fr, item, tid, part);
    }
    chain_sync(sched, nib, e.guard);
  }
  if (blk == 0 && wrench != nullptr) wrench_sum(e.partials, ninterp, wrench, tid);
  for (int item = blk; item < nspread; item += nib) spread_item(e, item, tid);
  chain_sync(sched, nib, e.guard);
  for (int slot = blk; slot < na; slot += nib) band_collide_item<S, XPER, ROT, YZ, TRT>(e, fr, cur, slot, tid);
  if (next_pose == nullptr) return;
  // The next step's skinning needs no barrier after the band collide: it
  // writes the marker data, chunk boxes and tile flags, which only the
  // phases before the last barrier read, and the active count (na was read
  // at the start). The binning rewrites the active list the band collide
  // reads, so it waits for every workgroup.
  for (int item = blk; item < skin_items(e.n); item += nib) skin_item(e, next_pose, item, tid);
  chain_sync(sched, nib, e.guard);
  for (int item = blk; item < active_items(e); item += nib) active_item(e, item, tid, false, next_slots);
}

// Grid: nib + e.nblocks workgroups of WG threads; the collide shape of e is
// linear (e.by == 0, e.bx == WG) or 2-D with e.bx * e.by == WG. e.tile_slot:
// this step's tile map.
template <class S, bool XPER, bool ROT, bool YZ, bool TRT>
__global__ void __launch_bounds__(WG) k_step_overlap(EnvView e, FrameF fr, int cur, int nib, int passes,
                                                      float *wrench, const float *next_pose, int *next_slots) {
  const int tid = threadIdx.x;
  if ((int)blockIdx.x < nib) {
    ib_chain<S, XPER, ROT, YZ, TRT>(e, fr, cur, blockIdx.x, nib, passes, wrench, next_pose, next_slots, tid);
    return;
  }
  const int lb = (int)blockIdx.x - nib;
  if (lb >= e.nblocks) return;
  const int tx = e.by == 0 ? tid : tid % e.bx, ty = e.by == 0 ? 0 : tid / e.bx;
  int x, y, z;
  if (!cell_of(e, lb, tx, ty, x, y, z)) return;
  const CellAt c = cell_at<XPER, YZ>(e.g, x, y, z);
  // a band cell (source node in an active tile) is the chain's
  if (((const gmem<int> *)e.tile_slot)[(c.xs >> 3) + e.g.tnx * ((c.ys >> 3) + e.g.tny * (c.zs >> 3))] >= 0) return;
  float f[Q];
  collide_pull<S, XPER, YZ>(e, cur, c, f);
  collide_finish<S, XPER, ROT, YZ, TRT>(e, fr, cur, c, f);
}

}  // namespace lbmib
