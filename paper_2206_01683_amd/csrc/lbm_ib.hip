// Host side of the C interface declared in include/lbm_ib.h: argument
// validation, workspace layout, kernel dispatch on the caller's stream.
//
// The library allocates no device memory: the caller hands in two population
// buffers and one workspace, sized by lbm_population_bytes and
// lbm_workspace_bytes. The context itself is a small host object.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/lbm_ib.h"
#include "ib.hpp"

using namespace lbmib;

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Workspace layout (all offsets 256-byte aligned).
struct Layout {
  int tnx, tny, tnz, ntiles, cap, maxm;
  size_t guard, counters, tile_flag, tile_slot, active, mbase, chunk_box, partials, macro, gbuf, rec, mstate, total;
};

bool params_ok(const lbm_params *p) {
  if (!p) return false;
  if (p->nx < 4 || p->ny < 4 || p->nz < 4) return false;
  if ((int64_t)p->nx * p->ny * p->nz > (int64_t)1 << 31) return false;
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return false;
  const bool lo_per = p->bc_lo == LBM_BC_PERIODIC, hi_per = p->bc_hi == LBM_BC_PERIODIC;
  if (lo_per != hi_per) return false;
  if (p->bc_lo < 0 || p->bc_lo > 2 || p->bc_hi < 0 || p->bc_hi > 2) return false;
  if (p->storage < LBM_STORE_F32 || p->storage > LBM_STORE_BF16) return false;
  if (p->max_markers < 0 || p->max_markers > (1 << 24)) return false;
  if (p->max_bones < 1 || p->mdf_iters < 1 || p->mdf_iters > 16) return false;
  if (p->max_active_tiles < 0) return false;
  if (p->block_x < 0 || p->block_y < 0 || p->block_x * p->block_y > 512) return false;
  if (p->block_x > 0 && p->block_x % 64 != 0) return false;
  if (!(p->ib_alpha > 0.0) || !std::isfinite(p->ib_alpha)) return false;
  return true;
}

size_t elem_bytes(int storage) { return storage == LBM_STORE_F32 ? 4 : 2; }

// Population plane stride: 256-element aligned plus 64 elements, so the 27
// plane bases do not all fall on the same large power-of-two boundary.
uint32_t plane_elems(const lbm_params *p) {
  size_t n = (size_t)p->nx * p->ny * p->nz;
  return (uint32_t)(align_up(n, 256) + 64);
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
  L.tile_flag = take(sizeof(int) * L.ntiles);
  L.tile_slot = take(sizeof(int) * L.ntiles);
  L.active = take(sizeof(int) * L.cap);
  L.mbase = take(sizeof(short4) * (size_t)L.maxm);
  L.chunk_box = take(sizeof(int4) * (size_t)((L.maxm + 63) / 64 + 8));
  L.partials = take(sizeof(float) * 8 * (size_t)interp_items(L.maxm));
  L.macro = take(sizeof(float) * 4 * 512 * (size_t)L.cap);
  L.gbuf = take(sizeof(unsigned long long) * 3 * 512 * (size_t)L.cap);
  L.rec = take(sizeof(float) * REC * (size_t)L.maxm);
  L.mstate = take(sizeof(float) * 4 * (size_t)L.maxm);
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
  bool slots_dirty;
  int bx, by;
  // measurement hook: 3 events per timed step (start, after IB, after collide)
  bool prof;
  std::vector<hipEvent_t> ev;
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
  g.xper = c->p.bc_lo == LBM_BC_PERIODIC;
  g.bc_lo = c->p.bc_lo;
  g.bc_hi = c->p.bc_hi;
  g.tnx = c->L.tnx;
  g.tny = c->L.tny;
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

// Device view of a context; the immersed-boundary fields describe `m` (may be
// null: no body this step).
EnvView env_view(lbm_ctx *c, const lbm_markers *m) {
  EnvView e{};
  e.g = grid_args(c);
  const double tau = c->p.tau;
  e.inv_tau = (float)(1.0 / tau);
  e.omt = (float)(1.0 - 1.0 / tau);
  e.pref = (float)(1.0 - 0.5 / tau);
  e.bx = c->bx;
  e.by = c->by;
  e.gx = (c->p.nx + c->bx - 1) / c->bx;
  e.gy = (c->p.ny + c->by - 1) / c->by;
  e.nblocks = e.gx * e.gy * c->p.nz;
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
  }
  e.tile_flag = wsp<int>(c, c->L.tile_flag);
  e.tile_slot = wsp<int>(c, c->L.tile_slot);
  e.active = wsp<int>(c, c->L.active);
  e.counters = wsp<int>(c, c->L.counters);
  e.guard = wsp<int>(c, c->L.guard);
  e.mbase = wsp<short4>(c, c->L.mbase);
  e.chunk_box = wsp<int4>(c, c->L.chunk_box);
  e.partials = wsp<float>(c, c->L.partials);
  e.macro = wsp<float4>(c, c->L.macro);
  e.gfix = wsp<unsigned long long>(c, c->L.gbuf);
  e.rec = wsp<float>(c, c->L.rec);
  e.mstate = wsp<float>(c, c->L.mstate);
  e.cur0 = c->cur;
  return e;
}

// -------------------------------------------------------------- dispatch --
template <class S>
lbm_status launch_collide(lbm_ctx *c, const EnvView &e, const FrameF &fr, bool rot) {
  const int grid = ((e.nblocks + 7) / 8) * 8;
  dim3 blk(c->bx, c->by);
  const bool xper = e.g.xper;
  if (xper && rot)
    k_collide<S, true, true><<<grid, blk, 0, c->stream>>>(e, fr, c->cur);
  else if (xper)
    k_collide<S, true, false><<<grid, blk, 0, c->stream>>>(e, fr, c->cur);
  else if (rot)
    k_collide<S, false, true><<<grid, blk, 0, c->stream>>>(e, fr, c->cur);
  else
    k_collide<S, false, false><<<grid, blk, 0, c->stream>>>(e, fr, c->cur);
  return launched();
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

void prof_mark(lbm_ctx *c, int which) {
  if (c->prof && c->prof_used < kProfSteps) (void)hipEventRecord(c->ev[3 * c->prof_used + which], c->stream);
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
    for (int it = 0; it < passes; ++it) {
      if (it > 0 && (st = launch_spread(c, e, nullptr)) != LBM_OK) return st;
      if ((st = launch_interp(c, e, fr, rot, it > 0, wrench != nullptr && it == passes - 1)) != LBM_OK) return st;
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
  if (c->prof && c->prof_used < kProfSteps) c->prof_used++;
  if (!e.ib && wrench) {
    k_fill_int<<<1, 64, 0, c->stream>>>(reinterpret_cast<int *>(wrench), 0, 8);
    if ((st = launched()) != LBM_OK) return st;
  }
  c->cur ^= 1;
  c->steps += 1;
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
  if (m->nbones < 1 || m->nbones > c->p.max_bones) return false;
  return true;
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

lbm_status lbm_init(lbm_ctx **out, const lbm_params *p, void *f_a, void *f_b, void *workspace, const float *rho0,
                    const float *u0, void *hip_stream) {
  if (!out || !params_ok(p) || !f_a || !f_b || !workspace || f_a == f_b) return LBM_ERR_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return LBM_ERR_ARG;
  *out = nullptr;
  lbm_ctx *c = new (std::nothrow) lbm_ctx;
  if (!c) return LBM_ERR_ARG;
  c->p = *p;
  c->L = layout(p);
  c->f[0] = f_a;
  c->f[1] = f_b;
  c->cur = 0;
  c->ws = static_cast<char *>(workspace);
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->steps = 0;
  c->plane = plane_elems(p);
  c->slots_dirty = false;
  c->prof = false;
  c->prof_used = 0;
  // collide block: 64-multiple along x covering as much of a row as fits
  int bx = p->block_x, by = p->block_y;
  if (bx == 0) bx = p->nx >= 128 ? 128 : 64;
  if (by == 0) by = std::max(1, 512 / bx);
  c->bx = bx;
  c->by = by;
  lbm_status st;
  k_fill_int<<<256, 256, 0, c->stream>>>(wsp<int>(c, c->L.tile_flag), 0, c->L.ntiles);
  k_fill_int<<<256, 256, 0, c->stream>>>(wsp<int>(c, c->L.tile_slot), -1, c->L.ntiles);
  k_fill_int<<<1, 64, 0, c->stream>>>(wsp<int>(c, c->L.guard), 0, 16);
  k_fill_int<<<1, 64, 0, c->stream>>>(wsp<int>(c, c->L.counters), 0, 16);
  if ((st = launched()) != LBM_OK || (st = LBM_BY_STORAGE(c, init_eq, rho0, u0)) != LBM_OK) {
    delete c;
    return st;
  }
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
  for (int s = 0; s < nsteps; ++s) {
    const float *pose = ib ? poses + (size_t)s * m->nbones * 24 : nullptr;
    float *w = wrench ? wrench + (size_t)s * 8 : nullptr;
    lbm_status st = LBM_BY_STORAGE(c, step_one, m, pose, &frames[s], w);
    if (st != LBM_OK) return st;
  }
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
  return LBM_OK;
}

lbm_status lbm_profile_enable(lbm_ctx *c, int enable) {
  if (!c) return LBM_ERR_ARG;
  if (enable && c->ev.empty()) {
    c->ev.resize(3 * kProfSteps);
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
    if (hipEventElapsedTime(&t0, c->ev[3 * s], c->ev[3 * s + 1]) != hipSuccess) return LBM_ERR_DEVICE;
    if (hipEventElapsedTime(&t1, c->ev[3 * s + 1], c->ev[3 * s + 2]) != hipSuccess) return LBM_ERR_DEVICE;
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
  for (auto &e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"
