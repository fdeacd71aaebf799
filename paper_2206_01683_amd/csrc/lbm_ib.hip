// Host side of the C interface declared in include/lbm_ib.h: argument
// validation, workspace layout, kernel dispatch on the caller's stream.
//
// The library allocates no device memory: the caller hands in two population
// buffers and one workspace, sized by lbm_population_bytes and
// lbm_workspace_bytes. The context itself is a small host object.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "../../include/lbm_ib.h"
#include "adjoint.hpp"
#include "batch.hpp"
#include "step.hpp"
#include "swimmer.hpp"

using namespace lbmib;

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Workspace layout (all offsets 256-byte aligned).
struct Layout {
  size_t sched;             // scheduling words of the overlapped step
  int tnx, tny, tnz, ntiles, cap, maxm;
  size_t guard, counters, tile_flag, tile_slot, tile_slot2, active, mbase, chunk_box, partials, macro, gbuf, rec, mstate;
  size_t gbar, adjfix, mbar, pbar, facebuf;
  size_t gcg, cg, cgpart;  // implicit velocity correction only
  size_t nrm;              // slip walls only
  size_t total;
};

bool params_ok(const lbm_params *p) {
  if (!p) return false;
  if (p->nx < 4 || p->ny < 4 || p->nz < 4) return false;
  if ((int64_t)p->nx * p->ny * p->nz > (int64_t)1 << 31) return false;
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return false;
  const int32_t faces[3][2] = {{p->bc_lo, p->bc_hi}, {p->bc_y[0], p->bc_y[1]}, {p->bc_z[0], p->bc_z[1]}};
  for (int a = 0; a < 3; ++a) {
    if (faces[a][0] < 0 || faces[a][0] > 2 || faces[a][1] < 0 || faces[a][1] > 2) return false;
    if ((faces[a][0] == LBM_BC_PERIODIC) != (faces[a][1] == LBM_BC_PERIODIC)) return false;
  }
  if (p->storage < LBM_STORE_F32 || p->storage > LBM_STORE_BF16) return false;
  if (p->max_markers < 0 || p->max_markers > (1 << 24)) return false;
  if (p->max_bones < 1 || p->mdf_iters < 1 || p->mdf_iters > 16) return false;
  if (p->max_active_tiles < 0) return false;
  if (p->block_x < 0 || p->block_y < -1 || p->block_x > 512 || p->block_x * p->block_y > 512) return false;
  if (p->block_x > 0 && p->block_x % 64 != 0) return false;
  if (p->block_y == -1 && p->block_x == 0) return false;
  if (!(p->ib_alpha > 0.0) || !std::isfinite(p->ib_alpha)) return false;
  if (p->ib_scheme != LBM_IB_DIRECT && p->ib_scheme != LBM_IB_IMPLICIT) return false;
  if (p->collision != LBM_COLLIDE_BGK && p->collision != LBM_COLLIDE_TRT) return false;
  if (p->collision == LBM_COLLIDE_TRT && !(p->trt_lambda > 0.0 && std::isfinite(p->trt_lambda))) return false;
  if (p->wall_mode != LBM_WALL_NO_SLIP && p->wall_mode != LBM_WALL_SLIP) return false;
  if (p->layout != LBM_LAYOUT_AUTO && p->layout != LBM_LAYOUT_PLANES && p->layout != LBM_LAYOUT_ROWS) return false;
  if (p->ib_workgroups < -1 || p->ib_workgroups > 1024) return false;
  return true;
}

size_t elem_bytes(int storage) { return storage == LBM_STORE_F32 ? 4 : 2; }

// Population plane stride: 256-element aligned plus 192 elements, so the 27
// plane bases do not all fall on the same large power-of-two boundary (+192
// measured about 1% faster on the collide than +64, +128 or +448, and +64
// about 1% faster than none).
uint32_t plane_elems(const lbm_params *p) {
  size_t n = (size_t)p->nx * p->ny * p->nz;
  return (uint32_t)(align_up(n, 256) + 192);
}

// Row layout ([nz][ny][27][nx]) for these parameters, else planes.
bool rows_layout(const lbm_params *p) {
  return p->layout == LBM_LAYOUT_ROWS || (p->layout == LBM_LAYOUT_AUTO && p->nx % 32 == 0);
}

// Population and row strides (elements) of the stored layout.
void pop_strides(const lbm_params *p, uint32_t &ps, uint32_t &rs) {
  if (rows_layout(p)) {
    ps = (uint32_t)p->nx;
    rs = 27u * (uint32_t)p->nx;
  } else {
    ps = plane_elems(p);
    rs = (uint32_t)p->nx;
  }
}

Layout layout(const lbm_params *p) {
  Layout L{};
  L.tnx = (p->nx + 7) / 8;
  L.tny = (p->ny + 7) / 8;
  L.tnz = (p->nz + 7) / 8;
  L.ntiles = L.tnx * L.tny * L.tnz;
  L.maxm = std::max(p->max_markers, 1);
  int cap = p->max_active_tiles > 0 ? p->max_active_tiles : L.ntiles;
  cap = std::min(cap, L.ntiles);
  if (p->max_markers == 0) cap = 1;
  L.cap = std::max(cap, 1);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.guard = take(64);
  L.counters = take(64);
  L.sched = take(sizeof(unsigned) * SCHED_WORDS);
  L.tile_flag = take(sizeof(int) * L.ntiles);
  L.tile_slot = take(sizeof(int) * L.ntiles);
  L.tile_slot2 = take(sizeof(int) * L.ntiles);  // the one-launch step's second tile map
  L.active = take(sizeof(int) * L.cap);
  L.mbase = take(sizeof(short4) * (size_t)L.maxm);
  L.chunk_box = take(sizeof(int4) * (size_t)((L.maxm + 63) / 64 + 8));
  L.partials = take(sizeof(float) * 8 * (size_t)interp_items(L.maxm));
  L.macro = take(sizeof(float) * 4 * 512 * (size_t)L.cap);
  L.gbuf = take(sizeof(unsigned long long) * 3 * 512 * (size_t)L.cap);
  L.rec = take(sizeof(float) * REC * (size_t)L.maxm);
  L.mstate = take(sizeof(float) * 4 * (size_t)L.maxm);
  L.gbar = L.adjfix = L.mbar = L.pbar = L.facebuf = 0;
  if (p->with_adjoint) {
    L.gbar = take(sizeof(float) * 3 * 512 * (size_t)L.cap);
    L.adjfix = take(sizeof(unsigned long long) * 4 * 512 * (size_t)L.cap);
    L.mbar = take(sizeof(float) * 6 * (size_t)L.maxm);
    L.pbar = take(sizeof(float) * 24 * kPoseSplit * (size_t)p->max_bones);
    L.facebuf = take(sizeof(float) * 2 * 4 * (size_t)p->ny * p->nz);
  }
  L.nrm = p->wall_mode == LBM_WALL_SLIP ? take(sizeof(float) * 3 * (size_t)L.maxm) : 0;
  L.gcg = L.cg = L.cgpart = 0;
  if (p->ib_scheme == LBM_IB_IMPLICIT) {
    L.gcg = take(sizeof(unsigned long long) * 3 * 512 * (size_t)L.cap);
    L.cg = take(sizeof(float) * 12 * (size_t)L.maxm);
    L.cgpart = take(sizeof(float) * cg_part_floats(L.maxm));
  }
  L.total = o;
  return L;
}

__global__ void k_fill_int(int *p, int v, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

}  // namespace

struct lbm_ctx {
  lbm_params p;
  Layout L;
  void *f[2];
  int cur;  // buffer holding the latest post-collision state
  char *ws;
  hipStream_t stream;
  int64_t steps;
  uint32_t plane;
  uint32_t ps, rs;  // population and row strides of the stored layout
  bool slots_dirty;
  bool is_static;  // created by lbm_init_static: workspace in `scratch`, not freed by lbm_destroy
  int bx, by;
  // measurement hook: up to 3 events per timed step (start, after IB, after
  // collide); prof_chained[s]: step s of a one-launch run records only its
  // end, and starts at the previous step's end (no IB before its launch)
  bool prof;
  std::vector<hipEvent_t> ev;
  std::vector<unsigned char> prof_chained;
  int prof_used;
};

static constexpr int kProfSteps = 4096;

namespace {

template <class T>
T *wsp(lbm_ctx *c, size_t off) {
  return reinterpret_cast<T *>(c->ws + off);
}

GridArgs grid_args(const lbm_ctx *c) {
  GridArgs g;
  g.nx = c->p.nx;
  g.ny = c->p.ny;
  g.nz = c->p.nz;
  g.plane = c->plane;
  g.ps = c->ps;
  g.rs = c->rs;
  g.xper = c->p.bc_lo == LBM_BC_PERIODIC;
  g.bc_lo = c->p.bc_lo;
  g.bc_hi = c->p.bc_hi;
  g.tnx = c->L.tnx;
  g.tny = c->L.tny;
  g.yper = c->p.bc_y[0] == LBM_BC_PERIODIC;
  g.zper = c->p.bc_z[0] == LBM_BC_PERIODIC;
  for (int q = 0; q < 2; ++q) {
    g.bc_y[q] = c->p.bc_y[q];
    g.bc_z[q] = c->p.bc_z[q];
  }
  return g;
}

FrameF frame_f(const lbm_frame *fr) {
  FrameF f{};
  if (!fr) return f;
  for (int a = 0; a < 3; ++a) {
    f.acc[a] = (float)fr->acc[a];
    f.omg[a] = (float)fr->omega[a];
    f.alp[a] = (float)fr->alpha[a];
    f.org[a] = (float)fr->origin[a];
    f.ulo[a] = (float)fr->u_lo[a];
    f.uhi[a] = (float)fr->u_hi[a];
  }
  return f;
}

bool rotating(const lbm_frame *fr) {
  if (!fr) return false;
  for (int a = 0; a < 3; ++a)
    if (fr->omega[a] != 0.0 || fr->alpha[a] != 0.0) return true;
  return false;
}

bool frame_ok(const lbm_frame *fr) {
  const double *d = &fr->acc[0];
  for (int q = 0; q < 18; ++q)
    if (!std::isfinite(d[q])) return false;
  return true;
}

lbm_status launched() { return hipGetLastError() == hipSuccess ? LBM_OK : LBM_ERR_DEVICE; }

// Thread block of the collide launches: bx x by, or bx x 1 for the linear shape.
dim3 collide_block(const lbm_ctx *c) { return dim3(c->bx, c->by > 0 ? c->by : 1); }

// Device view of a context; the immersed-boundary fields describe `m` (may be
// null: no body this step).
EnvView env_view(lbm_ctx *c, const lbm_markers *m) {
  EnvView e{};
  e.g = grid_args(c);
  const double tau = c->p.tau;
  e.inv_tau = (float)(1.0 / tau);
  e.omt = (float)(1.0 - 1.0 / tau);
  e.pref = (float)(1.0 - 0.5 / tau);
  e.two_rate = c->p.collision == LBM_COLLIDE_TRT ? 1 : 0;
  e.storage = c->p.storage == LBM_STORE_F16 ? StoreF16::kind
              : c->p.storage == LBM_STORE_BF16 ? StoreBF16::kind
                                               : StoreF32::kind;
  if (e.two_rate) {
    const double wp = 1.0 / tau, wm = 1.0 / (0.5 + c->p.trt_lambda / (tau - 0.5));
    e.trt = TrtRates{(float)wp, (float)wm, (float)(1.0 - 0.5 * wp), (float)(1.0 - 0.5 * wm),
                     (float)(1.0 - 0.5 * (wp + wm)), (float)(0.5 * (wm - wp))};
  }
  e.bx = c->bx;
  e.by = c->by;
  if (c->by == 0) {  // linear shape: bx consecutive cells per block
    e.gx = e.gy = 0;
    e.nblocks = (int)(((size_t)c->p.nx * c->p.ny * c->p.nz + c->bx - 1) / c->bx);
  } else {
    e.gx = (c->p.nx + c->bx - 1) / c->bx;
    e.gy = (c->p.ny + c->by - 1) / c->by;
    e.nblocks = e.gx * e.gy * c->p.nz;
  }
  e.f[0] = c->f[0];
  e.f[1] = c->f[1];
  e.ib = (m && m->n > 0) ? 1 : 0;
  e.cap = c->L.cap;
  e.ntiles = c->L.ntiles;
  e.alpha2 = (float)(2.0 * c->p.ib_alpha);
  if (e.ib) {
    e.n = m->n;
    e.nbones = m->nbones;
    e.xrest = m->xrest;
    e.weight = m->weight;
    e.dv = m->dv;
    e.bone = m->bone;
    e.X = m->X;
    e.U = m->U;
    e.F = m->F;
    if (c->p.wall_mode == LBM_WALL_SLIP) {
      e.slip = 1;
      e.nrest = m->nrest;
      e.Nrm = wsp<float>(c, c->L.nrm);
    }
  }
  e.tile_flag = wsp<int>(c, c->L.tile_flag);
  e.tile_slot = wsp<int>(c, c->L.tile_slot);
  e.active = wsp<int>(c, c->L.active);
  e.counters = wsp<int>(c, c->L.counters);
  e.guard = wsp<int>(c, c->L.guard);
  e.sched = wsp<unsigned>(c, c->L.sched);
  e.mbase = wsp<short4>(c, c->L.mbase);
  e.chunk_box = wsp<int4>(c, c->L.chunk_box);
  e.partials = wsp<float>(c, c->L.partials);
  e.macro = wsp<float4>(c, c->L.macro);
  e.gfix = wsp<unsigned long long>(c, c->L.gbuf);
  e.rec = wsp<float>(c, c->L.rec);
  e.mstate = wsp<float>(c, c->L.mstate);
  if (c->p.ib_scheme == LBM_IB_IMPLICIT) {
    e.gcg = wsp<unsigned long long>(c, c->L.gcg);
    e.cg = wsp<float>(c, c->L.cg);
    e.cgpart = wsp<float>(c, c->L.cgpart);
  }
  e.cur0 = c->cur;
  return e;
}

// -------------------------------------------------------------- dispatch --
template <class S, bool TRT>
void collide_kernels(const EnvView &e, const FrameF &fr, int cur, int grid, dim3 blk, size_t lds, hipStream_t s,
                     bool xper, bool rot, bool yz) {
  if (yz) {  // open y or z faces
    if (xper && rot)
      k_collide<S, true, true, true, TRT><<<grid, blk, lds, s>>>(e, fr, cur);
    else if (xper)
      k_collide<S, true, false, true, TRT><<<grid, blk, lds, s>>>(e, fr, cur);
    else if (rot)
      k_collide<S, false, true, true, TRT><<<grid, blk, lds, s>>>(e, fr, cur);
    else
      k_collide<S, false, false, true, TRT><<<grid, blk, lds, s>>>(e, fr, cur);
  } else if (xper && rot) {
    k_collide<S, true, true, false, TRT><<<grid, blk, lds, s>>>(e, fr, cur);
  } else if (xper) {
    k_collide<S, true, false, false, TRT><<<grid, blk, lds, s>>>(e, fr, cur);
  } else if (rot) {
    k_collide<S, false, true, false, TRT><<<grid, blk, lds, s>>>(e, fr, cur);
  } else {
    k_collide<S, false, false, false, TRT><<<grid, blk, lds, s>>>(e, fr, cur);
  }
}

// LDS a collide launch reserves (and never uses) so that about twelve waves,
// three per SIMD, share a compute unit: each lane issues its 27 loads at
// once, so few waves keep enough bytes in flight, and the F32 collide streams
// faster so than at the eight waves per SIMD its registers allow (fish,
// 384x192x192, 256-cell blocks: 508 us with three blocks per compute unit,
// against 538 at four, 534 at two and 527-532 uncapped). The size sits
// between the bounds for per_cu and per_cu + 1 blocks, in whole KiB. The
// 2-byte forms move half the bytes per load and run best at full occupancy
// (256 us, 258-260 us capped).
template <class S>
size_t collide_lds(dim3 blk) {
  if (S::kind != StoreF32::kind) return 0;
  constexpr int kLdsPerCu = 160 * 1024, kWavesPerCu = 12;
  const int waves = (int)((blk.x * blk.y + 63) / 64);
  const int per_cu = std::max(1, (kWavesPerCu + waves / 2) / waves);
  return (size_t)(2 * kLdsPerCu / (2 * per_cu + 1)) & ~(size_t)1023;
}

template <class S>
lbm_status launch_collide(lbm_ctx *c, const EnvView &e, const FrameF &fr, bool rot) {
  const int grid = e.nblocks;
  const dim3 blk = collide_block(c);
  const size_t lds = collide_lds<S>(blk);
  const bool yz = !(e.g.yper && e.g.zper), xper = e.g.xper != 0;
  if (c->p.collision == LBM_COLLIDE_TRT)
    collide_kernels<S, true>(e, fr, c->cur, grid, blk, lds, c->stream, xper, rot, yz);
  else
    collide_kernels<S, false>(e, fr, c->cur, grid, blk, lds, c->stream, xper, rot, yz);
  return launched();
}

// Workgroups of `kernel` (WG threads) that the current device holds at once,
// or 0 if the runtime cannot tell.
template <class K>
int coresident_workgroups(K kernel) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, WG, 0) != hipSuccess)
    return 0;
  return per_cu * cus;
}

// The chain's barrier needs all its workgroups resident together: nib is
// held to what the device holds at once of this kernel (queried once per
// form; the results do not depend on nib).
template <class S, bool TRT>
lbm_status step_overlap_kernels(const EnvView &e, const FrameF &fr, int cur, int nib, int passes, float *wrench,
                                const float *next_pose, int *next_slots, hipStream_t s, bool xper, bool rot,
                                bool yz) {
#define LBM_STEP_OVERLAP(XP, RT, YZ_)                                                                           \
  do {                                                                                                          \
    static const int cap = coresident_workgroups(k_step_overlap<S, XP, RT, YZ_, TRT>);                          \
    const int n = std::min(nib, cap);                                                                           \
    if (n < 1) return LBM_ERR_DEVICE;                                                                           \
    k_step_overlap<S, XP, RT, YZ_, TRT><<<n + e.nblocks, WG, 0, s>>>(e, fr, cur, n, passes, wrench, next_pose,  \
                                                                    next_slots);                                \
  } while (0)
  if (yz) {  // open y or z faces
    if (xper && rot)
      LBM_STEP_OVERLAP(true, true, true);
    else if (xper)
      LBM_STEP_OVERLAP(true, false, true);
    else if (rot)
      LBM_STEP_OVERLAP(false, true, true);
    else
      LBM_STEP_OVERLAP(false, false, true);
  } else if (xper && rot) {
    LBM_STEP_OVERLAP(true, true, false);
  } else if (xper) {
    LBM_STEP_OVERLAP(true, false, false);
  } else if (rot) {
    LBM_STEP_OVERLAP(false, true, false);
  } else {
    LBM_STEP_OVERLAP(false, false, false);
  }
#undef LBM_STEP_OVERLAP
  return launched();
}

// Whether the immersed-boundary chain runs beside the collide, one launch per
// step: on request only (ib_workgroups > 0 chain workgroups, direct forcing).
// Under the collide's load the chain's dependent accesses slow several-fold,
// so it pays only where the collide is long enough to hide it. On the
// 384x192x192 fish at F32 with 24-40 chain workgroups a step takes
// 0.532-0.543 ms against 0.570 ms in separate launches (fewer than 20 and the
// chain outlasts the collide; more take slots from it); with 2-byte storage
// (the collide takes 255 us, the chain longer), four forcing passes, or
// lattices small for their markers (the 150x50x100 two-fish domain, the
// 128x64x64 fin) it loses.
bool overlap_chain(const lbm_ctx *c) { return c->p.ib_scheme == LBM_IB_DIRECT && c->p.ib_workgroups > 0; }

// The band macros, interpolation and spreading beside the collide, and the
// next step's skinning and binning (next_pose != null) into next_slots, in one
// launch (k_step_overlap) with e0.tile_slot this step's tile map; the collide
// blocks take 512 cells each (the context's 2-D shape if it has 512 cells,
// else 512 consecutive cells).
template <class S>
lbm_status launch_step_overlap(lbm_ctx *c, const EnvView &e0, const FrameF &fr, bool rot, float *wrench,
                               const float *next_pose, int *next_slots) {
  EnvView e = e0;
  if (!(c->by > 0 && c->bx * c->by == WG)) {
    e.bx = WG;
    e.by = 0;
    e.gx = e.gy = 0;
    e.nblocks = (int)(((size_t)c->p.nx * c->p.ny * c->p.nz + WG - 1) / WG);
  }
  const int nib = c->p.ib_workgroups;
  const bool yz = !(e.g.yper && e.g.zper), xper = e.g.xper != 0;
  if (c->p.collision == LBM_COLLIDE_TRT)
    return step_overlap_kernels<S, true>(e, fr, c->cur, nib, c->p.mdf_iters, wrench, next_pose, next_slots,
                                         c->stream, xper, rot, yz);
  return step_overlap_kernels<S, false>(e, fr, c->cur, nib, c->p.mdf_iters, wrench, next_pose, next_slots, c->stream,
                                        xper, rot, yz);
}

template <class S>
lbm_status launch_macro(lbm_ctx *c, const EnvView &e, const FrameF &fr, bool rot) {
  const int grid = std::min(c->L.cap, 2048);
  if (rot)
    k_macro<S, true><<<grid, WG, 0, c->stream>>>(e, fr, c->cur);
  else
    k_macro<S, false><<<grid, WG, 0, c->stream>>>(e, fr, c->cur);
  return launched();
}

// wrench != nullptr: also sum the interpolation kernel's wrench partials.
lbm_status launch_spread(lbm_ctx *c, const EnvView &e, float *wrench) {
  const int grid = std::min(c->L.cap * kSpreadSplit, 2048);
  k_spread<<<grid, WG, 0, c->stream>>>(e, wrench);
  return launched();
}

lbm_status launch_interp(lbm_ctx *c, const EnvView &e, const FrameF &fr, bool rot, bool mdf, bool want_wrench) {
  const int grid = interp_items(e.n);
  float *part = want_wrench ? e.partials : nullptr;
  if (rot && mdf)
    k_interp<true, true><<<grid, WG, 0, c->stream>>>(e, fr, part);
  else if (rot)
    k_interp<true, false><<<grid, WG, 0, c->stream>>>(e, fr, part);
  else if (mdf)
    k_interp<false, true><<<grid, WG, 0, c->stream>>>(e, fr, part);
  else
    k_interp<false, false><<<grid, WG, 0, c->stream>>>(e, fr, part);
  return launched();
}

// Conjugate-gradient steps of the implicit velocity correction (after the
// first interpolation pass; the final spread into gfix follows).
lbm_status launch_implicit(lbm_ctx *c, const EnvView &e, const FrameF &fr, bool rot) {
  lbm_status st;
  const int items = cg_items(e.n);
  if (rot)
    k_cg_init<true><<<items, kCgWG, 0, c->stream>>>(e, fr);
  else
    k_cg_init<false><<<items, kCgWG, 0, c->stream>>>(e, fr);
  if ((st = launched()) != LBM_OK) return st;
  const int spread_grid = std::min(c->L.cap * kSpreadSplit, 2048);
  const int clear_grid = std::max(items, std::min((int)(((size_t)c->L.cap * 1536 + 4 * kCgWG - 1) / (4 * kCgWG)), 1024));
  const int steps = c->p.mdf_iters;
  for (int j = 0; j < steps; ++j) {
    const bool last = j == steps - 1;
    k_spread_cg<<<spread_grid, WG, 0, c->stream>>>(e, j);
    if ((st = launched()) != LBM_OK) return st;
    k_cg_apply<<<interp_items(e.n), WG, 0, c->stream>>>(e, j);
    if ((st = launched()) != LBM_OK) return st;
    k_cg_update<<<last ? items : clear_grid, kCgWG, 0, c->stream>>>(e, fr, j, last ? 1 : 0);
    if ((st = launched()) != LBM_OK) return st;
  }
  return LBM_OK;
}

void prof_mark(lbm_ctx *c, int which) {
  if (c->prof && c->prof_used < kProfSteps) (void)hipEventRecord(c->ev[3 * c->prof_used + which], c->stream);
}

// Ends a timed step. chained: only its end event was recorded (see prof_chained).
void prof_step(lbm_ctx *c, bool chained) {
  if (!c->prof || c->prof_used >= kProfSteps) return;
  c->prof_chained[c->prof_used] = chained ? 1 : 0;
  c->prof_used++;
}

template <class S>
lbm_status step_one(lbm_ctx *c, const lbm_markers *m, const float *pose, const lbm_frame *frame, float *wrench) {
  const FrameF fr = frame_f(frame);
  const bool rot = rotating(frame);
  const EnvView e = env_view(c, m);
  lbm_status st;
  prof_mark(c, 0);
  if (e.ib) {
    k_skin_mark<<<skin_items(e.n), WG, 0, c->stream>>>(e, pose);
    if ((st = launched()) != LBM_OK) return st;
    k_active<<<(e.ntiles + WG - 1) / WG, WG, 0, c->stream>>>(e);
    if ((st = launched()) != LBM_OK) return st;
    c->slots_dirty = true;
    if ((st = launch_macro<S>(c, e, fr, rot)) != LBM_OK) return st;
    const int passes = c->p.mdf_iters;
    if (c->p.ib_scheme == LBM_IB_IMPLICIT) {
      if ((st = launch_interp(c, e, fr, rot, false, false)) != LBM_OK) return st;
      if ((st = launch_implicit(c, e, fr, rot)) != LBM_OK) return st;
    } else {
      for (int it = 0; it < passes; ++it) {
        if (it > 0 && (st = launch_spread(c, e, nullptr)) != LBM_OK) return st;
        if ((st = launch_interp(c, e, fr, rot, it > 0, wrench != nullptr && it == passes - 1)) != LBM_OK) return st;
      }
    }
    if ((st = launch_spread(c, e, wrench)) != LBM_OK) return st;
  } else if (c->slots_dirty) {
    // no body this step: clear the active-tile map so no stale force is read
    k_fill_int<<<256, 256, 0, c->stream>>>(wsp<int>(c, c->L.tile_slot), -1, c->L.ntiles);
    if ((st = launched()) != LBM_OK) return st;
    c->slots_dirty = false;
  }
  prof_mark(c, 1);
  if ((st = launch_collide<S>(c, e, fr, rot)) != LBM_OK) return st;
  prof_mark(c, 2);
  prof_step(c, false);
  if (!e.ib && wrench) {
    k_fill_int<<<1, 64, 0, c->stream>>>(reinterpret_cast<int *>(wrench), 0, 8);
    if ((st = launched()) != LBM_OK) return st;
  }
  c->cur ^= 1;
  c->steps += 1;
  return LBM_OK;
}

// nsteps steps with the immersed-boundary chain beside the collide
// (overlap_chain): the first step's skinning and binning in launches of their
// own, then one launch per step, each skinning and binning the next step. The
// tile maps alternate between steps, starting so that the last step uses the
// context's own map (L.tile_slot), which the other paths read.
template <class S>
lbm_status step_fused(lbm_ctx *c, const lbm_markers *m, const float *poses, const lbm_frame *frames, int nsteps,
                      float *wrench) {
  if (nsteps == 0) return LBM_OK;
  EnvView e = env_view(c, m);
  int *maps[2] = {wsp<int>(c, c->L.tile_slot), wsp<int>(c, c->L.tile_slot2)};
  const int first = (nsteps - 1) & 1;
  const size_t pose_stride = (size_t)m->nbones * 24;
  lbm_status st;
  prof_mark(c, 0);
  e.tile_slot = maps[first];
  k_skin_mark<<<skin_items(e.n), WG, 0, c->stream>>>(e, poses);
  if ((st = launched()) != LBM_OK) return st;
  k_active<<<(e.ntiles + WG - 1) / WG, WG, 0, c->stream>>>(e);  // also zeroes the barrier count
  if ((st = launched()) != LBM_OK) return st;
  c->slots_dirty = true;
  for (int s = 0; s < nsteps; ++s) {
    // one event per step after the first (each launch directly follows the
    // previous one, whose end event is its start): event packets between
    // launches cost the step a few microseconds each
    const bool chained = s > 0 && c->prof_used > 0;
    if (!chained) prof_mark(c, 1);
    e.tile_slot = maps[(first + s) & 1];
    const float *next_pose = s + 1 < nsteps ? poses + (size_t)(s + 1) * pose_stride : nullptr;
    st = launch_step_overlap<S>(c, e, frame_f(&frames[s]), rotating(&frames[s]),
                                wrench ? wrench + (size_t)s * 8 : nullptr, next_pose, maps[(first + s + 1) & 1]);
    if (st != LBM_OK) return st;
    prof_mark(c, 2);
    prof_step(c, chained);
    c->cur ^= 1;
    c->steps += 1;
  }
  return LBM_OK;
}

template <class S>
lbm_status init_eq(lbm_ctx *c, const float *rho0, const float *u0) {
  GridArgs g = grid_args(c);
  dim3 grid((c->p.nx + 63) / 64, c->p.ny, c->p.nz);
  k_init_equilibrium<S><<<grid, 64, 0, c->stream>>>(rho0, u0, static_cast<typename S::T *>(c->f[c->cur]), g);
  return launched();
}

template <class S>
lbm_status load_canon(lbm_ctx *c, const float *f) {
  GridArgs g = grid_args(c);
  dim3 grid((c->p.nx + 63) / 64, c->p.ny, c->p.nz);
  k_load_canonical<S><<<grid, 64, 0, c->stream>>>(f, static_cast<typename S::T *>(c->f[c->cur]), g);
  return launched();
}

template <class S>
lbm_status read_canon(lbm_ctx *c, float *f) {
  GridArgs g = grid_args(c);
  dim3 grid((c->p.nx + 63) / 64, c->p.ny, c->p.nz);
  k_read_canonical<S><<<grid, 64, 0, c->stream>>>(static_cast<const typename S::T *>(c->f[c->cur]), f, g);
  return launched();
}

template <class S>
lbm_status macros(lbm_ctx *c, const lbm_frame *frame, float *rho, float *u) {
  GridArgs g = grid_args(c);
  dim3 grid((c->p.nx + 63) / 64, c->p.ny, c->p.nz);
  const auto *src = static_cast<const typename S::T *>(c->f[c->cur]);
  if (rotating(frame))
    k_macros<S, true><<<grid, 64, 0, c->stream>>>(src, g, frame_f(frame), rho, u);
  else
    k_macros<S, false><<<grid, 64, 0, c->stream>>>(src, g, frame_f(frame), rho, u);
  return launched();
}

#define LBM_BY_STORAGE(c, FN, ...)                                    \
  ((c)->p.storage == LBM_STORE_F32   ? FN<StoreF32>(c, __VA_ARGS__)  \
   : (c)->p.storage == LBM_STORE_F16 ? FN<StoreF16>(c, __VA_ARGS__)  \
                                     : FN<StoreBF16>(c, __VA_ARGS__))

bool markers_ok(const lbm_ctx *c, const lbm_markers *m) {
  if (!m) return true;
  if (m->n < 0) return false;
  if (m->n == 0) return true;
  if (!m->xrest || !m->bone || !m->weight || !m->dv || !m->X || !m->U || !m->F) return false;
  if (c->p.wall_mode == LBM_WALL_SLIP && !m->nrest) return false;
  if (m->nbones < 1 || m->nbones > c->p.max_bones) return false;
  return true;
}

// Fill a context for parameters p (already validated) bound to the caller's
// population buffers and to workspace ws, and queue the initial state.
lbm_status setup_ctx(lbm_ctx *c, const lbm_params *p, void *f_a, void *f_b, char *ws, const float *rho0,
                     const float *u0, void *hip_stream) {
  c->p = *p;
  c->L = layout(p);
  c->f[0] = f_a;
  c->f[1] = f_b;
  c->cur = 0;
  c->ws = ws;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->steps = 0;
  c->plane = plane_elems(p);
  pop_strides(p, c->ps, c->rs);
  c->slots_dirty = false;
  c->is_static = false;
  c->prof = false;
  c->prof_used = 0;
  // collide block: bx x by cells (by = 0: bx consecutive cells of the
  // x-fastest order). Default: 256 consecutive cells with the row layout;
  // with planes a 64-multiple along x covering as much of a row as fits.
  int bx = p->block_x, by = p->block_y;
  if (bx == 0 && by == 0 && rows_layout(p)) {
    bx = 256;
  } else if (by == -1) {
    by = 0;
  } else {
    if (bx == 0) bx = p->nx >= 128 ? 128 : 64;
    if (by == 0) by = std::max(1, 512 / bx);
  }
  c->bx = bx;
  c->by = by;
  // every workspace field that must start cleared, by kernels (no memset
  // nodes, so the sequence can sit in a captured graph)
  k_fill_int<<<256, 256, 0, c->stream>>>(wsp<int>(c, c->L.tile_flag), 0, c->L.ntiles);
  k_fill_int<<<256, 256, 0, c->stream>>>(wsp<int>(c, c->L.tile_slot2), -1, c->L.ntiles);
  k_fill_int<<<256, 256, 0, c->stream>>>(wsp<int>(c, c->L.tile_slot), -1, c->L.ntiles);
  k_fill_int<<<1, 64, 0, c->stream>>>(wsp<int>(c, c->L.guard), 0, 16);
  k_fill_int<<<1, 64, 0, c->stream>>>(wsp<int>(c, c->L.counters), 0, 16);
  lbm_status st = launched();
  if (st != LBM_OK) return st;
  return LBM_BY_STORAGE(c, init_eq, rho0, u0);
}

// Workspace of the contexts lbm_init_static creates: one array per device
// (each GPU the library runs on holds its own copy until the process ends),
// shared by every such context on that device. Host code reaches it only
// through the address hipGetSymbolAddress returns for the current device;
// the array's name in host code is not a device address.
constexpr size_t kStaticWorkspaceBytes = LBM_STATIC_WORKSPACE_BYTES;
constexpr int kMaxStaticDevices = 64;
__device__ __align__(256) char scratch[kStaticWorkspaceBytes];

char *g_scratch_ptr[kMaxStaticDevices];
lbm_ctx g_static_ctx[kMaxStaticDevices];
std::mutex g_scratch_mu;

// Device address of `scratch` on device dev (the current device), looked up
// once per device; null if the runtime cannot resolve it.
char *static_workspace(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    if (reinterpret_cast<uintptr_t>(ptr) % 256 != 0) return nullptr;
    g_scratch_ptr[dev] = static_cast<char *>(ptr);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

size_t lbm_population_bytes(const lbm_params *p) {
  if (!params_ok(p)) return 0;
  return (size_t)27 * plane_elems(p) * elem_bytes(p->storage);
}

size_t lbm_workspace_bytes(const lbm_params *p) {
  if (!params_ok(p)) return 0;
  return layout(p).total;
}

lbm_status lbm_population_strides(const lbm_params *p, int64_t *strides) {
  if (!params_ok(p) || !strides) return LBM_ERR_ARG;
  uint32_t ps, rs;
  pop_strides(p, ps, rs);
  strides[0] = ps;
  strides[1] = rs;
  strides[2] = rows_layout(p) ? 1 : 0;
  return LBM_OK;
}

lbm_status lbm_init(lbm_ctx **out, const lbm_params *p, void *f_a, void *f_b, void *workspace, const float *rho0,
                    const float *u0, void *hip_stream) {
  if (!out || !params_ok(p) || !f_a || !f_b || !workspace || f_a == f_b) return LBM_ERR_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return LBM_ERR_ARG;
  *out = nullptr;
  lbm_ctx *c = new (std::nothrow) lbm_ctx;
  if (!c) return LBM_ERR_ARG;
  const lbm_status st = setup_ctx(c, p, f_a, f_b, static_cast<char *>(workspace), rho0, u0, hip_stream);
  if (st != LBM_OK) {
    delete c;
    return st;
  }
  *out = c;
  return LBM_OK;
}

lbm_status lbm_init_static(lbm_ctx **out, const lbm_params *p, void *f_a, void *f_b, const float *rho0,
                           const float *u0, void *hip_stream) {
  if (!out || !params_ok(p) || !f_a || !f_b || f_a == f_b) return LBM_ERR_ARG;
  *out = nullptr;
  if (layout(p).total > kStaticWorkspaceBytes) return LBM_ERR_CAPACITY;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LBM_ERR_DEVICE;
  if (dev < 0 || dev >= kMaxStaticDevices) return LBM_ERR_UNSUPPORTED;
  char *ws = static_workspace(dev);
  if (!ws) return LBM_ERR_DEVICE;
  lbm_ctx *c = &g_static_ctx[dev];
  const lbm_status st = setup_ctx(c, p, f_a, f_b, ws, rho0, u0, hip_stream);
  c->is_static = true;
  if (st != LBM_OK) return st;
  *out = c;
  return LBM_OK;
}

lbm_status lbm_load_populations(lbm_ctx *c, const float *f) {
  if (!c || !f) return LBM_ERR_ARG;
  c->steps = 0;
  return LBM_BY_STORAGE(c, load_canon, f);
}

lbm_status lbm_read_populations(lbm_ctx *c, float *f) {
  if (!c || !f) return LBM_ERR_ARG;
  return LBM_BY_STORAGE(c, read_canon, f);
}

lbm_status lbm_macros(lbm_ctx *c, const lbm_frame *frame, float *rho, float *u) {
  if (!c || (!rho && !u)) return LBM_ERR_ARG;
  if (frame && !frame_ok(frame)) return LBM_ERR_ARG;
  return LBM_BY_STORAGE(c, macros, frame, rho, u);
}

lbm_status lbm_ib_step(lbm_ctx *c, const lbm_markers *m, const float *poses, const lbm_frame *frames,
                       int32_t nsteps, float *wrench) {
  if (!c || nsteps < 0 || (nsteps > 0 && !frames)) return LBM_ERR_ARG;
  if (!markers_ok(c, m)) return LBM_ERR_ARG;
  const bool ib = m && m->n > 0;
  if (ib && m->n > c->p.max_markers) return LBM_ERR_CAPACITY;
  if (ib && !poses) return LBM_ERR_ARG;
  for (int s = 0; s < nsteps; ++s)
    if (!frame_ok(&frames[s])) return LBM_ERR_ARG;
  // the implicit correction on a slip wall needs a frame that does not rotate
  if (ib && c->p.wall_mode == LBM_WALL_SLIP && c->p.ib_scheme == LBM_IB_IMPLICIT)
    for (int s = 0; s < nsteps; ++s)
      if (rotating(&frames[s])) return LBM_ERR_UNSUPPORTED;
  if (ib && overlap_chain(c)) return LBM_BY_STORAGE(c, step_fused, m, poses, frames, nsteps, wrench);
  for (int s = 0; s < nsteps; ++s) {
    const float *pose = ib ? poses + (size_t)s * m->nbones * 24 : nullptr;
    float *w = wrench ? wrench + (size_t)s * 8 : nullptr;
    lbm_status st = LBM_BY_STORAGE(c, step_one, m, pose, &frames[s], w);
    if (st != LBM_OK) return st;
  }
  return LBM_OK;
}

lbm_status lbm_state_save(lbm_ctx *c, void *dst) {
  if (!c || !dst) return LBM_ERR_ARG;
  const size_t bytes = (size_t)27 * c->plane * elem_bytes(c->p.storage);
  return hipMemcpyAsync(dst, c->f[c->cur], bytes, hipMemcpyDeviceToDevice, c->stream) == hipSuccess ? LBM_OK
                                                                                                  : LBM_ERR_DEVICE;
}

lbm_status lbm_state_restore(lbm_ctx *c, const void *src, int64_t step) {
  if (!c || !src || step < 0) return LBM_ERR_ARG;
  const size_t bytes = (size_t)27 * c->plane * elem_bytes(c->p.storage);
  if (hipMemcpyAsync(c->f[c->cur], src, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return LBM_ERR_DEVICE;
  c->steps = step;
  return LBM_OK;
}

lbm_status lbm_bind_populations(lbm_ctx *c, void *f_cur, void *f_next) {
  if (!c || !f_cur || !f_next || f_cur == f_next) return LBM_ERR_ARG;
  c->f[0] = f_cur;
  c->f[1] = f_next;
  c->cur = 0;
  return LBM_OK;
}

}  // extern "C"

namespace {

// Checks shared by the adjoint entry points; LBM_OK when the request is valid.
// need_pose_bar false: a forward-only request (lbm_adjoint_record).
lbm_status adjoint_request_ok(const lbm_ctx *c, const lbm_markers *m, const float *pose, const double *w,
                              float *pose_bar, bool need_pose_bar = true) {
  if (!markers_ok(c, m)) return LBM_ERR_ARG;
  const bool ib = m && m->n > 0;
  if (ib && (!pose || (need_pose_bar && !pose_bar))) return LBM_ERR_ARG;
  if (ib && m->n > c->p.max_markers) return LBM_ERR_CAPACITY;
  for (int q = 0; q < 4; ++q)
    if (!std::isfinite(w[q])) return LBM_ERR_ARG;
  if (c->p.storage != LBM_STORE_F32 || c->p.mdf_iters != 1 || c->p.ib_scheme != LBM_IB_DIRECT ||
      c->p.collision != LBM_COLLIDE_BGK || c->p.wall_mode != LBM_WALL_NO_SLIP || !c->p.with_adjoint)
    return LBM_ERR_UNSUPPORTED;
  if (c->p.bc_y[0] != LBM_BC_PERIODIC || c->p.bc_z[0] != LBM_BC_PERIODIC) return LBM_ERR_UNSUPPORTED;
  return LBM_OK;
}

// Forward immersed-boundary phases of one step (one direct-forcing pass), from
// the state in e.f[0], into the IB arrays e points at.
// wrench != null: also the step's wrench row, as lbm_ib_step writes it.
lbm_status ib_forward(lbm_ctx *c, const EnvView &e, const FrameF &fr, const float *pose, float *wrench = nullptr) {
  k_skin_mark<<<skin_items(e.n), WG, 0, c->stream>>>(e, pose);
  k_active<<<(e.ntiles + WG - 1) / WG, WG, 0, c->stream>>>(e);
  k_macro<StoreF32, false><<<std::min(c->L.cap, 2048), WG, 0, c->stream>>>(e, fr, 0);
  k_interp<false, false><<<interp_items(e.n), WG, 0, c->stream>>>(e, fr, wrench ? e.partials : nullptr);
  k_spread<<<std::min(c->L.cap * kSpreadSplit, 2048), WG, 0, c->stream>>>(e, wrench);
  return launched();
}

// The adjoint passes of one step whose forward IB data e points at (state in
// e.f[0]): lam_next -> lam_prev, pose_bar += the step's pose adjoint.
// mbar: where the marker adjoints go (null: the workspace's); pose_bar null:
// the pose reduction is left to the caller (a segment does it once).
lbm_status adjoint_passes(lbm_ctx *c, const EnvView &e, const FrameF &fr, const double *w, const float *lam_next,
                          float *lam_prev, float *pose_bar, float *mbar = nullptr) {
  AdjArgs A{};
  for (int a = 0; a < 3; ++a) {
    A.wF[a] = (float)w[a];
    A.a0[a] = -fr.acc[a];
    A.bc_u_lo[a] = fr.ulo[a];
    A.bc_u_hi[a] = fr.uhi[a];
  }
  A.wP = (float)w[3];
  A.lam_next = lam_next;
  A.lam_prev = lam_prev;
  A.gbar = wsp<float>(c, c->L.gbar);
  A.adjfix = wsp<unsigned long long>(c, c->L.adjfix);
  A.mbar = mbar ? mbar : wsp<float>(c, c->L.mbar);
  A.facebuf = wsp<float>(c, c->L.facebuf);
  lbm_status st;
  const int face_blocks = e.g.xper ? 0 : (2 * c->p.ny * c->p.nz + kFacePerBlock - 1) / kFacePerBlock;
  const int gbar_blocks = e.ib ? std::min(c->L.cap, 2048) : 0;
  if (face_blocks + gbar_blocks > 0) {
    k_adj_gbar<<<face_blocks + gbar_blocks, WG, 0, c->stream>>>(e, A, face_blocks);
    if ((st = launched()) != LBM_OK) return st;
  }
  if (e.ib) {
    k_adj_markers<<<wave_items(e.n), WG, 0, c->stream>>>(e, A);
    k_adj_spread<<<std::min(c->L.cap * kSpreadSplit, 2048), WG, 0, c->stream>>>(e, A);
    if ((st = launched()) != LBM_OK) return st;
  }
  const int grid = e.nblocks;
  const dim3 blk = collide_block(c);
  if (e.g.xper)
    k_adj_collide<true><<<grid, blk, 0, c->stream>>>(e, A);
  else
    k_adj_collide<false><<<grid, blk, 0, c->stream>>>(e, A);
  if ((st = launched()) != LBM_OK) return st;
  if (e.ib && pose_bar) {
    float *pbar = wsp<float>(c, c->L.pbar);
    k_adj_pose_part<<<dim3(e.nbones, kPoseSplit, 1), 256, 0, c->stream>>>(e, A.mbar, 0, pbar, 0);
    k_adj_pose_sum<<<dim3(e.nbones, 1), 64, 0, c->stream>>>(pbar, 0, pose_bar, e.nbones);
    if ((st = launched()) != LBM_OK) return st;
  }
  return LBM_OK;
}

// One slot of the adjoint IB ring: the forward IB data of one step.
struct RingSlot {
  size_t X, U, F, rec, mstate, mbase, chunk_box, tile_slot, active, counters, macro, gfix, mbar, pbar, total;
};

RingSlot ring_slot(const lbm_params *p) {
  const Layout L = layout(p);
  RingSlot r{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  const size_t n = (size_t)L.maxm;
  r.X = take(sizeof(float) * 3 * n);
  r.U = take(sizeof(float) * 3 * n);
  r.F = take(sizeof(float) * 3 * n);
  r.rec = take(sizeof(float) * REC * n);
  r.mstate = take(sizeof(float) * 4 * n);
  r.mbase = take(sizeof(short4) * n);
  r.chunk_box = take(sizeof(int4) * ((n + 63) / 64 + 8));
  r.tile_slot = take(sizeof(int) * (size_t)L.ntiles);
  r.active = take(sizeof(int) * (size_t)L.cap);
  r.counters = take(64);
  r.macro = take(sizeof(float) * 4 * 512 * (size_t)L.cap);
  r.gfix = take(sizeof(unsigned long long) * 3 * 512 * (size_t)L.cap);
  r.mbar = take(sizeof(float) * 6 * n);
  r.pbar = take(sizeof(float) * 24 * kPoseSplit * (size_t)p->max_bones);
  r.total = o;
  return r;
}

// e with its per-step IB arrays in ring slot `base`.
void point_at_slot(EnvView &e, const RingSlot &r, char *base) {
  e.X = reinterpret_cast<float *>(base + r.X);
  e.U = reinterpret_cast<float *>(base + r.U);
  e.F = reinterpret_cast<float *>(base + r.F);
  e.rec = reinterpret_cast<float *>(base + r.rec);
  e.mstate = reinterpret_cast<float *>(base + r.mstate);
  e.mbase = reinterpret_cast<short4 *>(base + r.mbase);
  e.chunk_box = reinterpret_cast<int4 *>(base + r.chunk_box);
  e.tile_slot = reinterpret_cast<int *>(base + r.tile_slot);
  e.active = reinterpret_cast<int *>(base + r.active);
  e.counters = reinterpret_cast<int *>(base + r.counters);
  e.macro = reinterpret_cast<float4 *>(base + r.macro);
  e.gfix = reinterpret_cast<unsigned long long *>(base + r.gfix);
}

}  // namespace

extern "C" {

lbm_status lbm_adjoint_step(lbm_ctx *c, const void *state, const lbm_markers *m, const float *pose,
                            const lbm_frame *frame, const double *w, const void *lam_next, void *lam_prev,
                            float *pose_bar) {
  if (!c || !state || !frame || !w || !lam_next || !lam_prev || lam_next == lam_prev) return LBM_ERR_ARG;
  if (!frame_ok(frame)) return LBM_ERR_ARG;
  lbm_status st = adjoint_request_ok(c, m, pose, w, pose_bar);
  if (st != LBM_OK) return st;
  if (rotating(frame)) return LBM_ERR_UNSUPPORTED;
  EnvView e = env_view(c, m);
  e.f[0] = const_cast<void *>(state);
  e.f[1] = nullptr;
  const FrameF fr = frame_f(frame);
  if (e.ib) {
    if ((st = ib_forward(c, e, fr, pose)) != LBM_OK) return st;
    c->slots_dirty = true;
  }
  return adjoint_passes(c, e, fr, w, static_cast<const float *>(lam_next), static_cast<float *>(lam_prev),
                        pose_bar);
}

size_t lbm_adjoint_ring_bytes(const lbm_params *p, int32_t nseg) {
  if (!params_ok(p) || nseg < 1) return 0;
  return ring_slot(p).total * (size_t)nseg;
}

}  // extern "C"

namespace {

// Arguments shared by the segment entry points. ring: nring entries, the
// last one may be null when last_optional.
lbm_status segment_args_ok(lbm_ctx *c, const void *ckpt, void *const *ring, int32_t nseg, int32_t nring,
                           bool last_optional, const lbm_frame *frames, const void *lam, const void *lam_tmp,
                           const void *ib_ring) {
  if (!c || !ckpt || nseg < 1 || !frames || !ib_ring) return LBM_ERR_ARG;
  if (reinterpret_cast<uintptr_t>(ib_ring) % 256 != 0) return LBM_ERR_ARG;
  if (nring > 0 && !ring) return LBM_ERR_ARG;
  for (int t = 0; t < nring; ++t) {
    if (!ring[t]) {
      if (last_optional && t == nring - 1) continue;
      return LBM_ERR_ARG;
    }
    if (ring[t] == ckpt || (lam && ring[t] == lam) || (lam_tmp && ring[t] == lam_tmp)) return LBM_ERR_ARG;
    for (int u = 0; u < t; ++u)
      if (ring[u] == ring[t]) return LBM_ERR_ARG;
  }
  for (int t = 0; t < nseg; ++t) {
    if (!frame_ok(&frames[t])) return LBM_ERR_ARG;
    if (rotating(&frames[t])) return LBM_ERR_UNSUPPORTED;
  }
  return LBM_OK;
}

// Forward over a segment from ckpt: state t+1 into ring[t] (skipped where
// t + 1 == nseg and ring has no such entry), each step's IB data in its slot
// of ib_ring, wrench rows if wrench != null.
lbm_status segment_record(lbm_ctx *c, const void *ckpt, void *const *ring, int32_t nseg, int32_t nring,
                          const lbm_markers *m, const float *poses, const lbm_frame *frames, void *ib_ring,
                          float *wrench) {
  const RingSlot rs = ring_slot(&c->p);
  char *rbase = static_cast<char *>(ib_ring);
  const size_t pstride = m && m->n > 0 ? (size_t)m->nbones * 24 : 0;
  lbm_status st;
  for (int t = 0; t < nseg; ++t) {
    EnvView e = env_view(c, m);
    e.f[0] = t == 0 ? const_cast<void *>(ckpt) : ring[t - 1];
    e.f[1] = t < nring ? ring[t] : nullptr;
    point_at_slot(e, rs, rbase + rs.total * (size_t)t);
    const FrameF fr = frame_f(&frames[t]);
    float *wr = wrench ? wrench + 8 * (size_t)t : nullptr;
    if (e.ib && (st = ib_forward(c, e, fr, poses + pstride * t, wr)) != LBM_OK) return st;
    if (!e.ib && wr) {
      k_fill_int<<<1, 64, 0, c->stream>>>(reinterpret_cast<int *>(wr), 0, 8);
      if ((st = launched()) != LBM_OK) return st;
    }
    if (e.f[1]) {
      const int grid = e.nblocks;
      const dim3 blk = collide_block(c);
      if (e.g.xper)
        k_collide<StoreF32, true, false><<<grid, blk, 0, c->stream>>>(e, fr, 0);
      else
        k_collide<StoreF32, false, false><<<grid, blk, 0, c->stream>>>(e, fr, 0);
      if ((st = launched()) != LBM_OK) return st;
    }
  }
  return LBM_OK;
}

// Reverse passes over a recorded segment; the result lands in `lam` (an odd
// count starts from a copy).
lbm_status segment_sweep(lbm_ctx *c, const void *ckpt, void *const *ring, int32_t nseg, const lbm_markers *m,
                         const lbm_frame *frames, const double *w, void *lam, void *lam_tmp, float *pose_bar,
                         void *ib_ring) {
  const RingSlot rs = ring_slot(&c->p);
  char *rbase = static_cast<char *>(ib_ring);
  lbm_status st;
  auto state_of = [&](int t) -> void * { return t == 0 ? const_cast<void *>(ckpt) : ring[t - 1]; };
  const size_t lam_bytes = (size_t)27 * c->plane * sizeof(float);
  float *next = static_cast<float *>(lam), *prev = static_cast<float *>(lam_tmp);
  if (nseg & 1) {
    if (hipMemcpyAsync(lam_tmp, lam, lam_bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
      return LBM_ERR_DEVICE;
    std::swap(next, prev);
  }
  for (int t = nseg - 1; t >= 0; --t) {
    EnvView e = env_view(c, m);
    e.f[0] = state_of(t);
    e.f[1] = nullptr;
    char *slot = rbase + rs.total * (size_t)t;
    point_at_slot(e, rs, slot);
    const FrameF fr = frame_f(&frames[t]);
    // marker adjoints stay in the step's slot; the pose sums run once below
    if ((st = adjoint_passes(c, e, fr, w, next, prev, nullptr, reinterpret_cast<float *>(slot + rs.mbar))) !=
        LBM_OK)
      return st;
    std::swap(next, prev);
  }
  if (m && m->n > 0) {
    const EnvView e = env_view(c, m);
    const size_t fstride = rs.total / sizeof(float);
    k_adj_pose_part<<<dim3(m->nbones, kPoseSplit, nseg), 256, 0, c->stream>>>(
        e, reinterpret_cast<float *>(rbase + rs.mbar), fstride, reinterpret_cast<float *>(rbase + rs.pbar), fstride);
    k_adj_pose_sum<<<dim3(m->nbones, nseg), 64, 0, c->stream>>>(reinterpret_cast<float *>(rbase + rs.pbar), fstride,
                                                                 pose_bar, m->nbones);
    if ((st = launched()) != LBM_OK) return st;
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_adjoint_segment(lbm_ctx *c, const void *ckpt, void *const *ring, int32_t nseg, const lbm_markers *m,
                               const float *poses, const lbm_frame *frames, const double *w, void *lam,
                               void *lam_tmp, float *pose_bar, void *ib_ring) {
  if (!w || !lam || !lam_tmp || lam == lam_tmp) return LBM_ERR_ARG;
  lbm_status st = segment_args_ok(c, ckpt, ring, nseg, nseg - 1, false, frames, lam, lam_tmp, ib_ring);
  if (st != LBM_OK) return st;
  if ((st = adjoint_request_ok(c, m, poses, w, pose_bar)) != LBM_OK) return st;
  if ((st = segment_record(c, ckpt, ring, nseg, nseg - 1, m, poses, frames, ib_ring, nullptr)) != LBM_OK) return st;
  return segment_sweep(c, ckpt, ring, nseg, m, frames, w, lam, lam_tmp, pose_bar, ib_ring);
}

lbm_status lbm_adjoint_record(lbm_ctx *c, const void *ckpt, void *const *ring, int32_t nseg, const lbm_markers *m,
                              const float *poses, const lbm_frame *frames, void *ib_ring, float *wrench) {
  lbm_status st = segment_args_ok(c, ckpt, ring, nseg, nseg, true, frames, nullptr, nullptr, ib_ring);
  if (st != LBM_OK) return st;
  static const double kNoWeights[4] = {0.0, 0.0, 0.0, 0.0};
  if ((st = adjoint_request_ok(c, m, poses, kNoWeights, nullptr, false)) != LBM_OK) return st;
  return segment_record(c, ckpt, ring, nseg, nseg, m, poses, frames, ib_ring, wrench);
}

lbm_status lbm_adjoint_sweep(lbm_ctx *c, const void *ckpt, void *const *ring, int32_t nseg, const lbm_markers *m,
                             const float *poses, const lbm_frame *frames, const double *w, void *lam, void *lam_tmp,
                             float *pose_bar, void *ib_ring) {
  if (!w || !lam || !lam_tmp || lam == lam_tmp) return LBM_ERR_ARG;
  lbm_status st = segment_args_ok(c, ckpt, ring, nseg, nseg - 1, false, frames, lam, lam_tmp, ib_ring);
  if (st != LBM_OK) return st;
  if ((st = adjoint_request_ok(c, m, poses, w, pose_bar)) != LBM_OK) return st;
  return segment_sweep(c, ckpt, ring, nseg, m, frames, w, lam, lam_tmp, pose_bar, ib_ring);
}

lbm_status lbm_swimmer_init(const lbm_swimmer *s, lbm_swimmer_state *st, const double *vel0, double heading,
                            const double *psi, const double *psidot) {
  if (!swimmer_ok(s) || !st || !psi || !psidot || !std::isfinite(heading)) return LBM_ERR_ARG;
  ChainShape c;
  if (!chain_shape(s, psi, psidot, c)) return LBM_ERR_ARG;
  for (int q = 0; q < 2; ++q) {
    st->vel[q] = vel0 ? vel0[q] : 0.0;
    st->acc[q] = 0.0;
    st->pos[q] = 0.0;
  }
  st->heading = heading;
  st->spin = 0.0;
  st->spin_prev = 0.0;
  st->ang_mom = c.Ls;
  st->inertia = c.Ic;
  return LBM_OK;
}

lbm_status lbm_swimmer_prepare(const lbm_swimmer *s, const lbm_swimmer_state *st, const double *psi,
                               const double *psidot, float *poses, lbm_frame *frame) {
  if (!swimmer_ok(s) || !st || !psi || !psidot || !poses || !frame) return LBM_ERR_ARG;
  ChainShape c;
  if (!chain_shape(s, psi, psidot, c)) return LBM_ERR_ARG;
  const double th = st->heading, w = st->spin;
  const double ct = std::cos(th), sn = std::sin(th);
  for (int j = 0; j < s->nbones; ++j) {
    // joint j relative to the mass centre: position and velocity in the frame
    const double dx = c.J[j][0] - c.rc[0], dy = c.J[j][1] - c.rc[1];
    const double vx = c.Jd[j][0] - c.rcd[0], vy = c.Jd[j][1] - c.rcd[1];
    const double Rdx = ct * dx - sn * dy, Rdy = sn * dx + ct * dy;
    const double P[3] = {s->origin[0] + Rdx, s->origin[1] + Rdy, s->origin[2]};
    const double Pd[3] = {-w * Rdy + ct * vx - sn * vy, w * Rdx + sn * vx + ct * vy, 0.0};
    const double al = th + psi[j], ca = std::cos(al), sa = std::sin(al), rate = w + psidot[j];
    const double R[9] = {ca, -sa, 0.0, sa, ca, 0.0, 0.0, 0.0, 1.0};
    const double Rd[9] = {-rate * sa, -rate * ca, 0.0, rate * ca, -rate * sa, 0.0, 0.0, 0.0, 0.0};
    const double *Jr = s->joints_rest + 3 * j;
    float *o = poses + 24 * j;
    for (int r = 0; r < 3; ++r) {
      double t = P[r], td = Pd[r];
      for (int k = 0; k < 3; ++k) {
        o[3 * r + k] = (float)R[3 * r + k];
        o[12 + 3 * r + k] = (float)Rd[3 * r + k];
        t -= R[3 * r + k] * Jr[k];
        td -= Rd[3 * r + k] * Jr[k];
      }
      o[9 + r] = (float)t;
      o[21 + r] = (float)td;
    }
  }
  for (int q = 0; q < 3; ++q) {
    frame->acc[q] = q < 2 ? st->acc[q] : 0.0;
    frame->omega[q] = 0.0;
    frame->alpha[q] = 0.0;
    frame->origin[q] = s->origin[q];
    frame->u_lo[q] = q < 2 ? -st->vel[q] : 0.0;
    frame->u_hi[q] = frame->u_lo[q];
  }
  return LBM_OK;
}

lbm_status lbm_swimmer_advance(const lbm_swimmer *s, lbm_swimmer_state *st, const float *wrench,
                               const double *psi_next, const double *psidot_next) {
  if (!swimmer_ok(s) || !st || !wrench || !psi_next || !psidot_next) return LBM_ERR_ARG;
  for (int q = 0; q < 8; ++q)
    if (!std::isfinite(wrench[q])) return LBM_ERR_ARG;
  ChainShape c;
  if (!chain_shape(s, psi_next, psidot_next, c)) return LBM_ERR_ARG;
  const double M = chain_mass(s), r = s->fluid_ratio, k = s->added_mass;
  for (int q = 0; q < 2; ++q) {
    const double a = st->acc[q];
    st->vel[q] += a;
    st->pos[q] += st->vel[q];
    st->acc[q] = ((double)wrench[q] / M + (r + k) * a) / (1.0 + k);
  }
  if (s->free_yaw) {
    const double dspin = st->spin - st->spin_prev, Ik = k * c.Ic;
    const double rhs = st->ang_mom + (double)wrench[5] + (r * st->inertia + Ik) * dspin - c.Ls + Ik * st->spin;
    st->spin_prev = st->spin;
    st->spin = rhs / (c.Ic + Ik);
    st->ang_mom = c.Ic * st->spin + c.Ls;
    st->heading += st->spin;
  } else {  // heading held: a holding torque absorbs the rest
    st->spin_prev = st->spin = 0.0;
    st->ang_mom = c.Ls;
  }
  st->inertia = c.Ic;
  return LBM_OK;
}

lbm_status lbm_body_forces(lbm_ctx *c, const lbm_markers *m, const double *center, float *out) {
  if (!c || !m || !center || !out || !markers_ok(c, m) || m->n <= 0) return LBM_ERR_ARG;
  k_wrench<<<1 + m->nbones, 1024, 0, c->stream>>>(m->X, m->U, m->F, m->dv, m->bone, m->weight, m->n,
                                                   (float)center[0], (float)center[1], (float)center[2], out);
  return launched();
}

lbm_status lbm_check(lbm_ctx *c) {
  if (!c) return LBM_ERR_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LBM_ERR_DEVICE;
  int guard = 0;
  if (hipMemcpy(&guard, wsp<int>(c, c->L.guard), sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return LBM_ERR_DEVICE;
  k_fill_int<<<1, 64, 0, c->stream>>>(wsp<int>(c, c->L.guard), 0, 1);
  if (launched() != LBM_OK || hipStreamSynchronize(c->stream) != hipSuccess) return LBM_ERR_DEVICE;
  if (guard & GUARD_UNSTABLE) return LBM_ERR_UNSTABLE;
  if (guard & GUARD_MARKER_RANGE) return LBM_ERR_MARKER_RANGE;
  if (guard & GUARD_CAPACITY) return LBM_ERR_CAPACITY;
  if (guard & GUARD_BONE) return LBM_ERR_ARG;
  if (guard & GUARD_SCHEDULE) return LBM_ERR_DEVICE;
  return LBM_OK;
}

lbm_status lbm_profile_enable(lbm_ctx *c, int enable) {
  if (!c) return LBM_ERR_ARG;
  if (enable && c->ev.empty()) {
    c->ev.resize(3 * kProfSteps);
    c->prof_chained.assign(kProfSteps, 0);
    for (auto &e : c->ev)
      if (hipEventCreate(&e) != hipSuccess) return LBM_ERR_DEVICE;
  }
  c->prof = enable != 0;
  return LBM_OK;
}

lbm_status lbm_profile_collect(lbm_ctx *c, double *ib_ms, double *collide_ms, int64_t *steps) {
  if (!c) return LBM_ERR_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LBM_ERR_DEVICE;
  double a = 0.0, b = 0.0;
  for (int s = 0; s < c->prof_used; ++s) {
    float t0 = 0.f, t1 = 0.f;
    if (c->prof_chained[s]) {  // from the previous step's end
      if (hipEventElapsedTime(&t1, c->ev[3 * (s - 1) + 2], c->ev[3 * s + 2]) != hipSuccess) return LBM_ERR_DEVICE;
    } else {
      if (hipEventElapsedTime(&t0, c->ev[3 * s], c->ev[3 * s + 1]) != hipSuccess) return LBM_ERR_DEVICE;
      if (hipEventElapsedTime(&t1, c->ev[3 * s + 1], c->ev[3 * s + 2]) != hipSuccess) return LBM_ERR_DEVICE;
    }
    a += t0;
    b += t1;
  }
  if (ib_ms) *ib_ms = a;
  if (collide_ms) *collide_ms = b;
  if (steps) *steps = c->prof_used;
  c->prof_used = 0;
  return LBM_OK;
}

lbm_status lbm_set_stream(lbm_ctx *c, void *hip_stream) {
  if (!c) return LBM_ERR_ARG;
  c->stream = static_cast<hipStream_t>(hip_stream);
  return LBM_OK;
}

int64_t lbm_step_count(const lbm_ctx *c) { return c ? c->steps : -1; }

const char *lbm_strerror(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_ERR_ARG: return "invalid argument";
    case LBM_ERR_DEVICE: return "HIP runtime or kernel launch failure";
    case LBM_ERR_UNSTABLE: return "unstable state: non-finite value or |u| >= 0.4";
    case LBM_ERR_MARKER_RANGE: return "marker within 2 cells (3 on the high side) of an open face";
    case LBM_ERR_CAPACITY: return "capacity exceeded (markers or active tiles)";
    case LBM_ERR_UNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

void lbm_destroy(lbm_ctx *c) {
  if (!c) return;
  if (c->is_static) {  // a per-device slot: keep it (and its events) for the next lbm_init_static
    c->prof = false;
    return;
  }
  for (auto &e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"

// ------------------------------------------------------------------ batch --
struct lbm_batch {
  int nenv;
  std::vector<lbm_env> envs;
  std::vector<EnvView> views;  // host copy of the uploaded descriptors
  std::vector<int> pre;        // [PRE_ROWS][nenv + 1]: item prefixes, collide order (row 4), CG items (PRE_CG)
  int kind_lo[kCollideKinds];  // collide items of kind k: [kind_lo[k], kind_lo[k] + kind_n[k])
  int kind_n[kCollideKinds];
  EnvView *d_envs;
  int *d_pre;
  unsigned *d_bar;
  int *d_status;
  int tot[4];
  int mdf;
  hipStream_t stream;
  int persistent_grid[2];  // [uniform]
  bool uniform;            // every environment of collide kind 0 (open x, non-rotating, periodic y/z, BGK, F32)
  bool two_byte;           // some environment stores 2-byte populations (per-phase driver only)
  bool implicit;           // every environment uses the implicit correction (per-phase driver only)
  bool still;              // no environment's frame rotates (the interpolation's only per-kind branch)
  int tot_cg;              // conjugate-gradient items over all environments
  bool dirty;
  hipGraph_t graph;
  hipGraphExec_t exec;
  int graph_nsteps, graph_mode;
  // Concurrent groups of the per-phase driver (empty: one group). Each group
  // is a batch of its own over a subset of the environments, run on its own
  // stream between a fork and a join event on this batch's stream.
  std::vector<lbm_batch *> sub;
  std::vector<hipEvent_t> sub_ev;  // [0] fork, [1 + g] join of group g
};

namespace {

size_t batch_layout(int nenv, size_t *o_envs, size_t *o_pre, size_t *o_bar) {
  size_t o = 0;
  *o_envs = o;
  o = align_up(o + sizeof(EnvView) * (size_t)nenv, 256);
  *o_pre = o;
  o = align_up(o + sizeof(int) * PRE_ROWS * (size_t)(nenv + 1), 256);
  *o_bar = o;
  o = align_up(o + sizeof(unsigned) * kBarWords, 256);
  return o;
}

bool env_ok(const lbm_env &v) {
  const lbm_ctx *c = v.ctx;
  if (!c || !(c->bx * c->by == WG || (c->bx == WG && c->by == 0))) return false;
  if (v.m.n < 1 || v.m.n > c->p.max_markers || !markers_ok(c, &v.m)) return false;
  if (!v.poses || !v.frames) return false;
  return true;
}

void batch_views(lbm_batch *b) {
  for (int e = 0; e < b->nenv; ++e) {
    lbm_ctx *c = b->envs[e].ctx;
    EnvView v = env_view(c, &b->envs[e].m);
    v.poses = b->envs[e].poses;
    v.frames = reinterpret_cast<const double *>(b->envs[e].frames);
    v.wrench = b->envs[e].wrench;
    v.rot = b->envs[e].rotating ? 1 : 0;
    v.cur0 = c->cur;
    b->views[e] = v;
  }
  const int stride = b->nenv + 1;
  for (int q = 0; q < 4; ++q) b->pre[q * stride] = 0;
  b->pre[PRE_CG * stride] = 0;
  for (int e = 0; e < b->nenv; ++e) {
    const EnvView &v = b->views[e];
    b->pre[0 * stride + e + 1] = b->pre[0 * stride + e] + skin_items(v.n);
    b->pre[1 * stride + e + 1] = b->pre[1 * stride + e] + (v.ntiles + WG - 1) / WG;
    b->pre[2 * stride + e + 1] = b->pre[2 * stride + e] + interp_items(v.n);
    b->pre[PRE_CG * stride + e + 1] = b->pre[PRE_CG * stride + e] + cg_items(v.n);
  }
  b->tot_cg = b->pre[PRE_CG * stride + b->nenv];
  // collide items: environments grouped by collide kind, each group one launch
  int *corder = &b->pre[4 * stride];
  int pos = 0;
  for (int k = 0; k < kCollideKinds; ++k) {
    b->kind_lo[k] = b->pre[3 * stride + pos];
    for (int e = 0; e < b->nenv; ++e) {
      if (collide_kind(b->views[e]) != k) continue;
      corder[pos] = e;
      b->pre[3 * stride + pos + 1] = b->pre[3 * stride + pos] + b->views[e].nblocks;
      ++pos;
    }
    b->kind_n[k] = b->pre[3 * stride + pos] - b->kind_lo[k];
  }
  corder[b->nenv] = 0;
  for (int q = 0; q < 4; ++q) b->tot[q] = b->pre[q * stride + b->nenv];
}

lbm_status batch_upload(lbm_batch *b) {
  batch_views(b);
  if (hipMemcpyAsync(b->d_envs, b->views.data(), sizeof(EnvView) * b->nenv, hipMemcpyHostToDevice, b->stream) !=
          hipSuccess ||
      hipMemcpyAsync(b->d_pre, b->pre.data(), sizeof(int) * b->pre.size(), hipMemcpyHostToDevice, b->stream) !=
          hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return LBM_ERR_DEVICE;
  b->dirty = false;
  return LBM_OK;
}

BatchArgs batch_args(const lbm_batch *b) {
  BatchArgs a;
  a.envs = b->d_envs;
  a.nenv = b->nenv;
  a.pre = b->d_pre;
  a.corder = b->d_pre + 4 * (b->nenv + 1);
  for (int q = 0; q < 4; ++q) a.tot[q] = b->tot[q];
  a.mdf = b->mdf;
  a.bar = b->d_bar;
  return a;
}

template <int K>
void launch_kb_collide(const BatchArgs &a, int s, int item0, int n, hipStream_t st) {
  kb_collide<K><<<n, WG, 0, st>>>(a, a.envs, a.pre, a.corder, s, item0);
}

template <int... K>
constexpr std::array<void (*)(const BatchArgs &, int, int, int, hipStream_t), sizeof...(K)> kb_collide_table(
    std::integer_sequence<int, K...>) {
  return {&launch_kb_collide<K>...};
}

// One collide launch per kind present, each kernel specialised to its kind.
void batch_collide(const lbm_batch *b, const BatchArgs &a, int s) {
  static constexpr auto table = kb_collide_table(std::make_integer_sequence<int, kCollideKinds>{});
  for (int k = 0; k < kCollideKinds; ++k)
    if (b->kind_n[k] > 0) table[k](a, s, b->kind_lo[k], b->kind_n[k], b->stream);
}

template <bool UNI>
lbm_status batch_enqueue_t(lbm_batch *b, int nsteps, int mode) {
  const BatchArgs a = batch_args(b);
  if (mode == LBM_BATCH_PERSISTENT) {
    kb_persistent<UNI><<<b->persistent_grid[UNI ? 1 : 0], WG, 0, b->stream>>>(a, nsteps);
    return launched();
  }
  int cap_items = 0;
  for (int e = 0; e < b->nenv; ++e) cap_items += b->views[e].cap;
  const int gdyn = std::max(8, std::min(cap_items * kSpreadSplit, 4096));
  // interpolation branches per environment only on rotation
  auto interp = [&](const BatchArgs &args, int s, int pass) {
    if (UNI || b->still)
      kb_interp<true><<<b->tot[PRE_INTERP], WG, 0, b->stream>>>(args, s, pass);
    else
      kb_interp<false><<<b->tot[PRE_INTERP], WG, 0, b->stream>>>(args, s, pass);
  };
  for (int s = 0; s < nsteps; ++s) {
    kb_skin<<<b->tot[PRE_SKIN], WG, 0, b->stream>>>(a, s);
    kb_active<<<b->tot[PRE_ACTIVE], WG, 0, b->stream>>>(a);
    kb_macro<UNI><<<gdyn, WG, 0, b->stream>>>(a, s);
    if (b->implicit) {  // mdf = conjugate-gradient steps
      interp(a, s, 0);
      kb_cg_init<<<b->tot_cg, kCgWG, 0, b->stream>>>(a, s);
      for (int j = 0; j < b->mdf; ++j) {
        const bool last = j == b->mdf - 1;
        kb_spread_cg<<<gdyn, WG, 0, b->stream>>>(a, j);
        kb_cg_apply<<<b->tot[PRE_INTERP], WG, 0, b->stream>>>(a, j);
        kb_cg_update<<<b->tot_cg, kCgWG, 0, b->stream>>>(a, s, j, last ? 1 : 0);
        if (!last) kb_cg_clear<<<gdyn, WG, 0, b->stream>>>(a);
      }
    } else {
      for (int pass = 0; pass < b->mdf; ++pass) {
        if (pass > 0) kb_spread<<<gdyn, WG, 0, b->stream>>>(a, s, 0);
        interp(a, s, pass);
      }
    }
    kb_spread<<<gdyn, WG, 0, b->stream>>>(a, s, 1);
    batch_collide(b, a, s);
    lbm_status st = launched();
    if (st != LBM_OK) return st;
  }
  return LBM_OK;
}

lbm_status batch_enqueue(lbm_batch *b, int nsteps, int mode) {
  return b->uniform ? batch_enqueue_t<true>(b, nsteps, mode) : batch_enqueue_t<false>(b, nsteps, mode);
}

void batch_drop_graph(lbm_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_nsteps = -1;
}

void batch_drop_groups(lbm_batch *b);

// Cell-balanced split of the environments into ngroups groups: largest
// lattice first, each to the group with the fewest cells so far (ties to the
// lower group); within a group the environments keep the batch's order.
std::vector<std::vector<int>> batch_partition(const lbm_batch *b, int ngroups) {
  std::vector<int> order(b->nenv);
  for (int e = 0; e < b->nenv; ++e) order[e] = e;
  auto cells = [&](int e) {
    const lbm_params &q = b->envs[e].ctx->p;
    return (int64_t)q.nx * q.ny * q.nz;
  };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cells(x) > cells(y); });
  std::vector<int64_t> load(ngroups, 0);
  std::vector<int> owner(b->nenv, 0);
  for (int e : order) {
    int g = 0;
    for (int h = 1; h < ngroups; ++h)
      if (load[h] < load[g]) g = h;
    owner[e] = g;
    load[g] += cells(e);
  }
  std::vector<std::vector<int>> groups(ngroups);
  for (int e = 0; e < b->nenv; ++e) groups[owner[e]].push_back(e);
  return groups;
}

void batch_drop_groups(lbm_batch *b) {
  for (lbm_batch *s : b->sub) {
    (void)hipStreamSynchronize(s->stream);
    lbm_batch_destroy(s);
  }
  for (hipEvent_t ev : b->sub_ev)
    if (ev) (void)hipEventDestroy(ev);
  b->sub.clear();
  b->sub_ev.clear();
}

}  // namespace

extern "C" {

size_t lbm_batch_bytes(int32_t nenv) {
  if (nenv < 1 || nenv > kMaxEnvs) return 0;
  size_t a, p, q;
  return batch_layout(nenv, &a, &p, &q);
}

lbm_status lbm_batch_create(lbm_batch **out, const lbm_env *envs, int32_t nenv, void *dev, void *hip_stream) {
  if (!out || !envs || nenv < 1 || nenv > kMaxEnvs || !dev) return LBM_ERR_ARG;
  if (reinterpret_cast<uintptr_t>(dev) % 256 != 0) return LBM_ERR_ARG;
  *out = nullptr;
  for (int e = 0; e < nenv; ++e) {
    if (!env_ok(envs[e])) return LBM_ERR_ARG;
    if (envs[e].ctx->p.mdf_iters != envs[0].ctx->p.mdf_iters) return LBM_ERR_ARG;
    if (envs[e].ctx->p.ib_scheme != envs[0].ctx->p.ib_scheme) return LBM_ERR_UNSUPPORTED;
    // as lbm_ib_step: the slip-wall correction's system is unsymmetric in a rotating frame
    if (envs[e].ctx->p.ib_scheme == LBM_IB_IMPLICIT && envs[e].ctx->p.wall_mode == LBM_WALL_SLIP &&
        envs[e].rotating)
      return LBM_ERR_UNSUPPORTED;
    for (int f = 0; f < e; ++f)
      if (envs[f].ctx == envs[e].ctx) return LBM_ERR_ARG;
  }
  lbm_batch *b = new (std::nothrow) lbm_batch;
  if (!b) return LBM_ERR_ARG;
  b->nenv = nenv;
  b->envs.assign(envs, envs + nenv);
  b->views.resize(nenv);
  b->pre.assign(PRE_ROWS * (size_t)(nenv + 1), 0);
  size_t o_envs, o_pre, o_bar;
  batch_layout(nenv, &o_envs, &o_pre, &o_bar);
  char *base = static_cast<char *>(dev);
  b->d_envs = reinterpret_cast<EnvView *>(base + o_envs);
  b->d_pre = reinterpret_cast<int *>(base + o_pre);
  b->d_bar = reinterpret_cast<unsigned *>(base + o_bar);
  b->d_status = reinterpret_cast<int *>(b->d_bar + BAR_STATUS);
  b->mdf = envs[0].ctx->p.mdf_iters;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->graph = nullptr;
  b->exec = nullptr;
  b->graph_nsteps = -1;
  b->graph_mode = -1;
  b->uniform = true;
  b->two_byte = false;
  b->implicit = envs[0].ctx->p.ib_scheme == LBM_IB_IMPLICIT;
  b->still = true;
  for (int e = 0; e < nenv; ++e) {
    const lbm_params &q = envs[e].ctx->p;
    if (envs[e].rotating || q.bc_lo == LBM_BC_PERIODIC || q.bc_y[0] != LBM_BC_PERIODIC ||
        q.bc_z[0] != LBM_BC_PERIODIC || q.collision != LBM_COLLIDE_BGK || q.storage != LBM_STORE_F32)
      b->uniform = false;
    if (q.storage != LBM_STORE_F32) b->two_byte = true;
    if (envs[e].rotating) b->still = false;
  }
  int dev_id = 0, cus = 0, per_cu[2] = {0, 0};
  if (hipGetDevice(&dev_id) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu[0], kb_persistent<false>, WG, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu[1], kb_persistent<true>, WG, 0) != hipSuccess ||
      per_cu[0] < 1 || per_cu[1] < 1) {
    delete b;
    return LBM_ERR_DEVICE;
  }
  for (int u = 0; u < 2; ++u)
    b->persistent_grid[u] = std::min(kBarGroup * kBarMaxGroups, std::max(8, (per_cu[u] * cus) / 8 * 8));
  k_fill_int<<<8, 256, 0, b->stream>>>(reinterpret_cast<int *>(b->d_bar), 0, kBarWords);
  lbm_status st = launched();
  if (st == LBM_OK) st = batch_upload(b);
  if (st != LBM_OK) {
    delete b;
    return st;
  }
  *out = b;
  return LBM_OK;
}

lbm_status lbm_batch_run(lbm_batch *b, int32_t nsteps, int32_t mode, int32_t graph) {
  if (!b || nsteps < 0 || (mode != LBM_BATCH_PHASES && mode != LBM_BATCH_PERSISTENT)) return LBM_ERR_ARG;
  if (graph && (nsteps % 2 != 0 || b->stream == nullptr)) return LBM_ERR_ARG;
  if (mode == LBM_BATCH_PERSISTENT && (b->two_byte || b->implicit)) return LBM_ERR_UNSUPPORTED;
  if (nsteps == 0) return LBM_OK;
  lbm_status st;
  if (mode == LBM_BATCH_PHASES && !b->sub.empty()) {
    // groups run concurrently, each on its own stream, after the work already
    // queued on this batch's stream; this stream then waits for all of them
    if (hipEventRecord(b->sub_ev[0], b->stream) != hipSuccess) return LBM_ERR_DEVICE;
    for (size_t g = 0; g < b->sub.size(); ++g) {
      lbm_batch *s = b->sub[g];
      if (hipStreamWaitEvent(s->stream, b->sub_ev[0], 0) != hipSuccess) return LBM_ERR_DEVICE;
      if ((st = lbm_batch_run(s, nsteps, mode, graph)) != LBM_OK) return st;
      if (hipEventRecord(b->sub_ev[1 + g], s->stream) != hipSuccess ||
          hipStreamWaitEvent(b->stream, b->sub_ev[1 + g], 0) != hipSuccess)
        return LBM_ERR_DEVICE;
    }
    return LBM_OK;
  }
  for (int e = 0; e < b->nenv; ++e)
    if (b->views[e].cur0 != b->envs[e].ctx->cur) b->dirty = true;
  if (b->dirty) {
    batch_drop_graph(b);
    if ((st = batch_upload(b)) != LBM_OK) return st;
  }
  if (graph) {
    if (!b->exec || b->graph_nsteps != nsteps || b->graph_mode != mode) {
      batch_drop_graph(b);
      if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return LBM_ERR_DEVICE;
      st = batch_enqueue(b, nsteps, mode);
      hipGraph_t g = nullptr;
      const hipError_t ce = hipStreamEndCapture(b->stream, &g);
      if (st != LBM_OK || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return LBM_ERR_DEVICE;
      }
      b->graph = g;
      if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        batch_drop_graph(b);
        return LBM_ERR_DEVICE;
      }
      b->graph_nsteps = nsteps;
      b->graph_mode = mode;
    }
    if (hipGraphLaunch(b->exec, b->stream) != hipSuccess) return LBM_ERR_DEVICE;
  } else if ((st = batch_enqueue(b, nsteps, mode)) != LBM_OK) {
    return st;
  }
  for (int e = 0; e < b->nenv; ++e) {
    lbm_ctx *c = b->envs[e].ctx;
    c->cur ^= (nsteps & 1);
    c->steps += nsteps;
    c->slots_dirty = true;
  }
  return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch *b, int32_t reps, int32_t *shapes_out) {
  if (!b || reps < 1) return LBM_ERR_ARG;
  static const int cand[5][2] = {{64, 8}, {128, 4}, {256, 2}, {512, 1}, {512, 0}};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return LBM_ERR_DEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return LBM_ERR_DEVICE;
  }
  lbm_status st = LBM_OK;
  for (int e = 0; e < b->nenv && st == LBM_OK; ++e) {
    lbm_ctx *c = b->envs[e].ctx;
    hipStream_t keep = c->stream;
    c->stream = b->stream;
    float best = 1e30f;
    int bi = 1;
    for (int q = 0; q < 5 && st == LBM_OK; ++q) {
      if (cand[q][1] > 0 && cand[q][0] > (int)align_up((size_t)c->p.nx, 64) && q > 0) continue;
      c->bx = cand[q][0];
      c->by = cand[q][1];
      const EnvView v = env_view(c, nullptr);
      // the collide reads f[cur] and writes f[cur ^ 1] (scratch until the next
      // step), so timing it leaves the state unchanged
      st = LBM_BY_STORAGE(c, launch_collide, v, FrameF{}, false);
      if (st != LBM_OK || hipEventRecord(e0, b->stream) != hipSuccess) break;
      for (int r = 0; r < reps && st == LBM_OK; ++r) st = LBM_BY_STORAGE(c, launch_collide, v, FrameF{}, false);
      float ms = 0.f;
      if (st != LBM_OK || hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = LBM_ERR_DEVICE;
        break;
      }
      if (ms < best) {
        best = ms;
        bi = q;
      }
    }
    c->bx = cand[bi][0];
    c->by = cand[bi][1];
    c->stream = keep;
    if (shapes_out) {
      shapes_out[2 * e] = c->bx;
      shapes_out[2 * e + 1] = c->by;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->dirty = true;
  for (lbm_batch *s : b->sub) s->dirty = true;
  return st;
}

lbm_status lbm_batch_set_shapes(lbm_batch *b, const int32_t *shapes) {
  if (!b || !shapes) return LBM_ERR_ARG;
  for (int e = 0; e < b->nenv; ++e) {
    const int bx = shapes[2 * e], by = shapes[2 * e + 1];
    if (!(bx == WG && by == 0) && (bx < 64 || bx % 64 != 0 || bx * by != WG)) return LBM_ERR_ARG;
  }
  for (int e = 0; e < b->nenv; ++e) {
    b->envs[e].ctx->bx = shapes[2 * e];
    b->envs[e].ctx->by = shapes[2 * e + 1];
  }
  b->dirty = true;
  for (lbm_batch *s : b->sub) s->dirty = true;
  return LBM_OK;
}

lbm_status lbm_batch_check(lbm_batch *b) {
  if (!b) return LBM_ERR_ARG;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return LBM_ERR_DEVICE;
  int status = 0;
  if (hipMemcpy(&status, b->d_status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return LBM_ERR_DEVICE;
  if (status & 1) {
    // a barrier timed out: the run stopped early and the barrier counters are
    // stale; reset them (and the flag) so the next run starts clean
    k_fill_int<<<8, 256, 0, b->stream>>>(reinterpret_cast<int *>(b->d_bar), 0, kBarWords);
    if (launched() != LBM_OK || hipStreamSynchronize(b->stream) != hipSuccess) return LBM_ERR_DEVICE;
    return LBM_ERR_DEVICE;
  }
  for (int e = 0; e < b->nenv; ++e) {
    lbm_ctx *c = b->envs[e].ctx;
    hipStream_t keep = c->stream;
    c->stream = b->stream;
    const lbm_status st = lbm_check(c);
    c->stream = keep;
    if (st != LBM_OK) return st;
  }
  return LBM_OK;
}

size_t lbm_batch_group_bytes(int32_t nenv, int32_t ngroups) {
  if (nenv < 1 || nenv > kMaxEnvs || ngroups < 2 || ngroups > LBM_BATCH_MAX_GROUPS || ngroups > nenv) return 0;
  // every group holds at most nenv - ngroups + 1 environments
  return (size_t)ngroups * lbm_batch_bytes(nenv - ngroups + 1);
}

lbm_status lbm_batch_set_groups(lbm_batch *b, int32_t ngroups, void *const *streams, void *dev) {
  if (!b || ngroups < 1 || ngroups > LBM_BATCH_MAX_GROUPS || ngroups > b->nenv) return LBM_ERR_ARG;
  if (ngroups == 1) {
    batch_drop_groups(b);
    return LBM_OK;
  }
  if (!streams || !dev || reinterpret_cast<uintptr_t>(dev) % 256 != 0) return LBM_ERR_ARG;
  for (int g = 0; g < ngroups; ++g) {
    if (!streams[g]) return LBM_ERR_ARG;
    for (int h = 0; h < g; ++h)
      if (streams[h] == streams[g]) return LBM_ERR_ARG;
  }
  // the work queued on the groups' old streams and tables ends before they change
  if (hipStreamSynchronize(b->stream) != hipSuccess) return LBM_ERR_DEVICE;
  batch_drop_groups(b);
  const std::vector<std::vector<int>> groups = batch_partition(b, ngroups);
  const size_t slice = lbm_batch_bytes(b->nenv - ngroups + 1);
  lbm_status st = LBM_OK;
  b->sub_ev.assign(ngroups + 1, nullptr);
  for (int k = 0; k <= ngroups && st == LBM_OK; ++k)
    if (hipEventCreateWithFlags(&b->sub_ev[k], hipEventDisableTiming) != hipSuccess) st = LBM_ERR_DEVICE;
  for (int g = 0; g < ngroups && st == LBM_OK; ++g) {
    std::vector<lbm_env> part;
    for (int e : groups[g]) part.push_back(b->envs[e]);
    lbm_batch *s = nullptr;
    st = lbm_batch_create(&s, part.data(), (int32_t)part.size(), static_cast<char *>(dev) + g * slice,
                          streams[g]);
    if (st == LBM_OK) b->sub.push_back(s);
  }
  if (st != LBM_OK) batch_drop_groups(b);
  return st;
}

void lbm_batch_destroy(lbm_batch *b) {
  if (!b) return;
  batch_drop_groups(b);
  batch_drop_graph(b);
  delete b;
}

}  // extern "C"
