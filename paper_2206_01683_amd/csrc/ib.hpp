// Immersed-boundary phases of one step: skinning, tile binning, interpolation
// with direct forcing, gather-form spreading and the body wrench.
//
// The immersed force lives only in "active" 8x8x8 tiles: tiles that some
// marker's 4x4x4 Peskin stencil touches. Each step rebuilds the active set.
// Every phase is a device function of (environment, work item) run by one
// 512-thread workgroup, so the same code serves the single-lattice kernels,
// the batched per-phase kernels and the persistent batched kernel:
//   skin_item     512 markers: linear blend skinning, wrap/range guard, flag
//                 the tiles each stencil touches (plain stores), per-wave
//                 chunk boxes (tile range of 64 consecutive markers)
//   active_item   512 tiles: compact the flags into slots and an active list
//   macro_item    one active tile: density and unforced velocity of its 512
//                 cells; clears the tile's fixed-point force
//   interp_item   32 markers, 16 lanes each, one lane per x-row of 4
//                 stencil nodes: row sums, then 16-lane sums -> U*_k, rho_k,
//                 direct forcing F_k, marker record, wrench partials
//   spread_item   (active tile, part): the markers whose stencils touch the
//                 tile add their stencil nodes into an LDS tile in 64-bit fixed
//                 point (order-independent, so deterministic), merged into the
//                 tile's fixed-point force with one atomic per nonzero cell
//   wrench_sum    adds the wrench partials in a fixed order
#pragma once

#include "fluid.hpp"

namespace lbmib {

constexpr int WG = 512;              // threads per workgroup in every IB phase
constexpr int REC = 20;              // floats per marker record: w[12], base[3], pad, fdv[3], pad
constexpr int kSpreadSplit = 4;      // spreading work items per active tile (single lattice)
constexpr int kBatchSpreadSplit = 2; // the same in the batched forms, whose many tiles need less splitting
constexpr int kWavePer = WG / 64;    // markers per item of the one-wave-per-marker kernels (adjoint)
constexpr int kInterpMk = WG / 16;   // markers per interpolation (and CG apply) item, 16 lanes each

// Scheduling words of the overlapped step (step.hpp), each on its own
// 128-byte line, in the workspace (EnvView::sched): the chain's barrier
// arrival count and generation. k_active clears the arrival count.
constexpr int kSchedLine = 32;
enum : int { SCHED_ARRIVE = 0, SCHED_GEN = kSchedLine, SCHED_WORDS = 2 * kSchedLine };

__device__ inline int stencil_base(float X) { return (int)floorf(X) - 1; }

// Tiles of the nodes base..base+3 along one axis (wrapped when periodic),
// one per node; first[s] is false when node s's tile repeats an earlier
// node's. Fixed-size and fully unrolled, so everything stays in registers.
__device__ inline void axis_node_tiles(int base, int n, bool per, int t[4], bool first[4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    int j = base + s;
    if (per) j = wrap_idx(j, n);
    t[s] = j >> 3;
    first[s] = true;
#pragma unroll
    for (int q = 0; q < s; ++q) first[s] = first[s] && t[q] != t[s];
  }
}

__device__ inline bool axis_touches(int base, int n, bool per, int tile) {
  bool hit = false;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    int j = base + s;
    if (per) j = wrap_idx(j, n);
    hit |= (j >> 3) == tile;
  }
  return hit;
}

// Value of lane (this lane ^ o) of the wave (ds_bpermute). The lane id
// passes through an empty asm so that its arithmetic is redone where it is
// used: in the persistent kernel, hoisting it out of the step loop would hold
// one register per offset across every phase.
__device__ inline int xor_lane_addr(int o) {
  int lane = __lane_id();
  asm volatile("" : "+v"(lane));
  return (lane ^ o) << 2;
}
__device__ inline int shfl_xor_i(int v, int o) { return __builtin_amdgcn_ds_bpermute(xor_lane_addr(o), v); }
__device__ inline float shfl_xor_f(float v, int o) { return __int_as_float(shfl_xor_i(__float_as_int(v), o)); }

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += shfl_xor_f(v, o);
  return v;
}

__device__ inline bool box_hits(int packed, int t) { return t >= (packed & 0xFFFF) && t <= (packed >> 16); }

// --------------------------------------------------------------- skinning --
// Markers 512*item .. 512*item+511 with bone poses `pose` of this step.
// Linear blend skinning X = sum_b w_b (R_b xrest + t_b), U = sum_b w_b
// (dR_b xrest + dt_b). Periodic axes: X wrapped into [0, n). Open x: markers
// must satisfy 2 <= X < nx - 3 so the stencil stays on nodes 1 .. nx-2; others
// raise the range guard and are clamped so that every access stays in bounds.
// Item 0 also clears the active-tile counter of this step. (Always inlined:
// called as a function, its call would hold the persistent kernel's registers
// across it and push that kernel past its budget.)
__device__ __attribute__((always_inline)) inline void skin_item(const EnvView &e, const float *__restrict__ pose,
                                                                int item, int tid) {
  const int k = item * WG + tid;
  const int n = e.n;
  if (k == 0) {
    e.counters[0] = 0;  // active tiles of this step
    e.counters[1] = 0;  // arrival count of the implicit correction's reductions
  }
  const int tns[3] = {e.g.tnx, e.g.tny, (e.g.nz + 7) >> 3};
  const int dims[3] = {e.g.nx, e.g.ny, e.g.nz};
  int lo[3] = {1 << 20, 1 << 20, 1 << 20}, hi[3] = {-1, -1, -1};
  // the environment's arrays through global pointers (see gmem)
  const gmem<float> *xrest = (const gmem<float> *)e.xrest, *nrest = (const gmem<float> *)e.nrest;
  const gmem<float> *weight = (const gmem<float> *)e.weight, *gpose = (const gmem<float> *)pose;
  const gmem<int> *bone = (const gmem<int> *)e.bone;
  gmem<float> *X = (gmem<float> *)e.X, *U = (gmem<float> *)e.U;
  gmem<int> *tile_flag = (gmem<int> *)e.tile_flag;
  if (k < n) {
    const float r0 = xrest[k], r1 = xrest[n + k], r2 = xrest[2 * n + k];
    float p[3] = {0.f, 0.f, 0.f}, v[3] = {0.f, 0.f, 0.f}, nv[3] = {0.f, 0.f, 0.f};
    float n0 = 0.f, n1 = 0.f, n2 = 0.f;
    if (e.slip) {
      n0 = nrest[k];
      n1 = nrest[n + k];
      n2 = nrest[2 * n + k];
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      int b = bone[j * n + k];
      float w = weight[j * n + k];
      if ((unsigned)b >= (unsigned)e.nbones) {
        atomicOr(e.guard, (int)GUARD_BONE);
        b = 0;
        w = 0.f;
      }
      const gmem<float> *P = gpose + 24 * b;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        p[r] += w * (P[3 * r] * r0 + P[3 * r + 1] * r1 + P[3 * r + 2] * r2 + P[9 + r]);
        v[r] += w * (P[12 + 3 * r] * r0 + P[12 + 3 * r + 1] * r1 + P[12 + 3 * r + 2] * r2 + P[21 + r]);
        nv[r] += w * (P[3 * r] * n0 + P[3 * r + 1] * n1 + P[3 * r + 2] * n2);
      }
      // one bone's 24 pose values live at a time: keeps the phase within the
      // register budget of the kernels it is inlined into
      __builtin_amdgcn_sched_barrier(0);
    }
    if (e.slip) {  // the rest normal turned by the blended rotations, unit length
      const float il = rsqrtf(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
#pragma unroll
      for (int r = 0; r < 3; ++r) ((gmem<float> *)e.Nrm)[r * n + k] = nv[r] * il;
    }
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const float nn = (float)dims[ax];
      const bool per = ax == 0 ? e.g.xper != 0 : (ax == 1 ? e.g.yper != 0 : e.g.zper != 0);
      if (per) {
        float q = p[ax] - nn * floorf(p[ax] / nn);
        if (!(q >= 0.f && q < nn)) q = 0.f;
        p[ax] = q;
      } else if (!(p[ax] >= 2.0f && p[ax] < nn - 3.0f)) {
        atomicOr(e.guard, (int)GUARD_MARKER_RANGE);
        p[ax] = (p[ax] >= 2.0f) ? nn - 3.5f : 2.0f;
      }
      X[ax * n + k] = p[ax];
      U[ax * n + k] = v[ax];
    }
    const int bs[3] = {stencil_base(p[0]), stencil_base(p[1]), stencil_base(p[2])};
    gmem<short> *mb = (gmem<short> *)e.mbase + 4 * (size_t)k;
    mb[0] = (short)bs[0];
    mb[1] = (short)bs[1];
    mb[2] = (short)bs[2];
    mb[3] = 0;
    int tx[4], ty[4], tz[4];
    bool fx[4], fy[4], fz[4];
    axis_node_tiles(bs[0], e.g.nx, e.g.xper, tx, fx);
    axis_node_tiles(bs[1], e.g.ny, e.g.yper, ty, fy);
    axis_node_tiles(bs[2], e.g.nz, e.g.zper, tz, fz);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int l = 0; l < 4; ++l)
          if (fz[i] && fy[j] && fx[l]) tile_flag[tx[l] + e.g.tnx * (ty[j] + e.g.tny * tz[i])] = 1;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      if (bs[ax] < 0 || bs[ax] + 3 >= dims[ax]) {  // wrapping stencil: whole axis
        lo[ax] = 0;
        hi[ax] = tns[ax] - 1;
      } else {
        lo[ax] = bs[ax] >> 3;
        hi[ax] = (bs[ax] + 3) >> 3;
      }
    }
  }
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      lo[ax] = min(lo[ax], shfl_xor_i(lo[ax], o));
      hi[ax] = max(hi[ax], shfl_xor_i(hi[ax], o));
    }
  }
  if ((tid & 63) == 0 && k < n) {
    gmem<int> *cb = (gmem<int> *)e.chunk_box + 4 * (size_t)(k >> 6);
    cb[0] = lo[0] | (hi[0] << 16);
    cb[1] = lo[1] | (hi[1] << 16);
    cb[2] = lo[2] | (hi[2] << 16);
    cb[3] = 0;
  }
}

__device__ __host__ inline int skin_items(int n) { return (n + WG - 1) / WG; }

// ---------------------------------------------------------- active tiles --
// Tiles 512*item .. 512*item+511: slots in workgroup order from one atomic per
// workgroup. Slot numbering only decides storage locations, never results.
// Clears the flags for the next step. slots: the tile map to write (null:
// e.tile_slot). reset_sched: item 0 also clears the overlapped step's barrier
// count (not when the overlapped step itself bins the next step's tiles).
__device__ inline void active_item(const EnvView &e, int item, int tid, bool reset_sched = true,
                                   int *slots = nullptr) {
  __shared__ int s_w[WG / 64];
  __shared__ int s_base;
  const int lane = tid & 63, wv = tid >> 6;
  const int t = item * WG + tid;
  if (item == 0 && tid == 0 && e.sched != nullptr && reset_sched) {
    e.sched[SCHED_ARRIVE] = 0u;
  }
  int *tile_slot = slots != nullptr ? slots : e.tile_slot;
  int f = 0;
  if (t < e.ntiles) {
    f = e.tile_flag[t] != 0;
    e.tile_flag[t] = 0;
  }
  const unsigned long long bal = __ballot(f);
  if (lane == 0) s_w[wv] = __popcll(bal);
  __syncthreads();
  if (tid == 0) {
    int tot = 0;
    for (int q = 0; q < WG / 64; ++q) tot += s_w[q];
    s_base = tot ? atomicAdd(&e.counters[0], tot) : 0;
  }
  __syncthreads();
  int pre = s_base;
  for (int q = 0; q < wv; ++q) pre += s_w[q];
  pre += __popcll(bal & ((1ull << lane) - 1ull));
  if (t < e.ntiles) {
    if (f && pre < e.cap) {
      tile_slot[t] = pre;
      e.active[pre] = t;
    } else {
      tile_slot[t] = -1;
      if (f) atomicOr(e.guard, (int)GUARD_CAPACITY);
    }
  }
  __syncthreads();  // s_w / s_base are reused by the next item
}

__device__ inline int active_items(const EnvView &e) { return (e.ntiles + WG - 1) / WG; }
__device__ inline int n_active_of(const EnvView &e) { return min(e.counters[0], e.cap); }

// XCD-contiguous walk over work items 0 .. tot-1. The dispatcher hands
// workgroup b to XCD b % kXcds, and each XCD has its own L2; an active tile's
// x-rows are 8 cells (32 bytes at F32) of 128-byte lines that it shares with
// its x-neighbours, which hold the next slots. Giving each XCD one contiguous
// range of items makes those neighbours meet in one L2 instead of fetching
// each line once per XCD. Every item is visited exactly once for any grid;
// workgroups past the last multiple of kXcds take no items.
constexpr int kXcds = 8;
struct XcdWalk {
  int first, end, step;
};
__device__ inline XcdWalk xcd_walk(int tot, int blk, int grid) {
  const int per = grid / kXcds;
  if (per == 0) return {blk, tot, grid};  // small grid: plain stride
  const int x = blk % kXcds, r = blk / kXcds;
  if (r >= per) return {0, 0, 1};
  const int chunk = (tot + kXcds - 1) / kXcds;
  const int lo = x * chunk, hi = min(tot, lo + chunk);
  return {lo + r, hi, per};
}
__device__ inline XcdWalk xcd_walk(int tot) { return xcd_walk(tot, (int)blockIdx.x, (int)gridDim.x); }

// Item of workgroup blk in a grid of exactly `grid` workgroups, one item each,
// XCD-contiguous: with grid = 8q + m, XCD x (workgroups x, x + 8, ...) takes
// the q + (x < m) consecutive items from x q + min(x, m) on. A bijection of
// 0 .. grid-1, so every item runs once.
__device__ inline int xcd_item(int blk, int grid) {
  const int q = grid / kXcds, m = grid % kXcds, x = blk % kXcds;
  return x * q + min(x, m) + blk / kXcds;
}

// ----------------------------------------------------------- band macros --
// Density and unforced velocity u* (frame force, no IB force) of every cell
// of active tile `slot`; also clears the tile's fixed-point immersed force.
template <class S, bool ROT>
__device__ inline void macro_item(const EnvView &e, const FrameF &fr, int cur, int slot, int tid) {
  using T = typename S::T;
  const gmem<T> *__restrict__ src = (const gmem<T> *)e.f[cur];
  const GridArgs &g = e.g;
  const int t = ((const gmem<int> *)e.active)[slot];
  const int tx = t % g.tnx, ty = (t / g.tnx) % g.tny, tz = t / (g.tnx * g.tny);
  const int x = tx * 8 + (tid & 7), y = ty * 8 + ((tid >> 3) & 7), z = tz * 8 + (tid >> 6);
  float4 out = make_float4(1.f, 0.f, 0.f, 0.f);
  if (x < g.nx && y < g.ny && z < g.nz && (g.xper || (x > 0 && x < g.nx - 1))) {
    const int xm = g.xper ? wrap_idx(x - 1, g.nx) : x - 1;
    const int xp = g.xper ? wrap_idx(x + 1, g.nx) : x + 1;
    float f[Q];  // deviations h_i = f_i - w_i
    pull27<S, true>(src, g, xm, x, xp, wrap_idx(y - 1, g.ny), y, wrap_idx(y + 1, g.ny),
                    wrap_idx(z - 1, g.nz), z, wrap_idx(z + 1, g.nz), f);
    float drho, mx, my, mz;
    moments(f, drho, mx, my, mz);
    const float rho = 1.0f + drho;
    float ax, ay, az;
    frame_a0<ROT>(fr, (float)x, (float)y, (float)z, ax, ay, az);
    float ux, uy, uz;
    const float ir = 1.0f / rho;
    solve_coriolis<ROT>(fr, mx * ir + 0.5f * ax, my * ir + 0.5f * ay, mz * ir + 0.5f * az, ux, uy, uz);
    out = make_float4(rho, ux, uy, uz);
  }
  ((gmem<vfloat4> *)e.macro)[(size_t)slot * 512 + tid] = vfloat4{out.x, out.y, out.z, out.w};
  gmem<unsigned long long> *gp = (gmem<unsigned long long> *)e.gfix + (size_t)slot * 1536;
  gp[tid] = 0ull;
  gp[512 + tid] = 0ull;
  gp[1024 + tid] = 0ull;
  if (e.gcg != nullptr) {  // implicit correction: its search-direction force starts at zero too
    gmem<unsigned long long> *gq = (gmem<unsigned long long> *)e.gcg + (size_t)slot * 1536;
    gq[tid] = 0ull;
    gq[512 + tid] = 0ull;
    gq[1024 + tid] = 0ull;
  }
}

// --------------------------------------------------------- interpolation --
// Markers 32*item .. 32*item+31, four per wave, 16 lanes each. Lane
// sub = lane & 15 of a marker's group holds the x-row of stencil nodes
// (0..3, sub & 3, sub >> 2): it issues the row's four gathers together, sums
// the row, and a 16-lane butterfly (every lane of the group ends with the
// same bits) completes the 64-node sums. Node weight delta = wx (wy wz),
// the product the spreading uses.
// pass 0: U*_k = sum u* delta, rho_k = sum rho delta, F_k = 2 alpha rho_k (U_k - U*_k).
// pass p > 0 (multi-direct forcing): the interpolated velocity includes the
// current immersed force, u = u* + (I + [omega]x)^-1 g / (2 rho), and
// F_k += 2 alpha rho_k (U_k - U_k^interp).
// The record carries this pass's F increment times dV (spreading adds each
// pass into the step's force). With partials != nullptr: the fluid's force,
// torque about the frame origin and power, summed per item into
// partials[item][8].
__device__ inline float group16_sum(float v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v += shfl_xor_f(v, o);
  return v;
}

// Stencil geometry of marker position X for row lane sub: the base node per
// axis, the four x weights, the row's y and z weights, and per x node of the
// row its tile index and its cell index within the tile.
struct StencilRow {
  int base[3];
  float wx[4], wy, wz;
  int tile[4], lc[4];
};

__device__ inline StencilRow stencil_row(const GridArgs &g, const float X[3], int sub) {
  StencilRow r;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) r.base[ax] = stencil_base(X[ax]);
  const int jy = r.base[1] + (sub & 3), jz = r.base[2] + (sub >> 2);
#pragma unroll
  for (int i = 0; i < 4; ++i) r.wx[i] = peskin4(X[0] - (float)(r.base[0] + i));
  r.wy = peskin4(X[1] - (float)jy);
  r.wz = peskin4(X[2] - (float)jz);
  const int yn = wrap_idx(jy, g.ny), zn = wrap_idx(jz, g.nz);
  const int trow = g.tnx * ((yn >> 3) + g.tny * (zn >> 3));
  const int lrow = ((yn & 7) << 3) | ((zn & 7) << 6);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int xn = g.xper ? wrap_idx(r.base[0] + i, g.nx) : r.base[0] + i;
    r.tile[i] = (xn >> 3) + trow;
    r.lc[i] = (xn & 7) | lrow;
  }
  return r;
}

template <bool ROT, bool MDF>
__device__ inline void interp_item(const EnvView &e, const FrameF &fr, int item, int tid, float *partials) {
  // multiply-adds fuse only within one expression, never across statements,
  // so every kernel that inlines this item rounds its outputs identically
#pragma clang fp contract(on)
  __shared__ float s_part[kInterpMk][8];
  const int sub = tid & 15, mk = tid >> 4;
  const int k = item * kInterpMk + mk;
  const int n = e.n;
  const GridArgs &g = e.g;
  const bool live = k < n;
  // the environment's arrays through global pointers (see gmem)
  const gmem<float> *X = (const gmem<float> *)e.X, *U = (const gmem<float> *)e.U;
  const gmem<int> *tile_slot = (const gmem<int> *)e.tile_slot;
  const gmem<vfloat4> *macro = (const gmem<vfloat4> *)e.macro;
  gmem<float> *F = (gmem<float> *)e.F, *mstate = (gmem<float> *)e.mstate;
  float part[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float Xk[3] = {0.f, 0.f, 0.f}, Uk[3] = {0.f, 0.f, 0.f}, dvk = 0.f;
  StencilRow st{};
  float sr = 0.f, sx = 0.f, sy = 0.f, sz = 0.f;
  if (live) {
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      Xk[ax] = X[ax * n + k];
      // loaded now, used after the stencil gather: off the dependent chain
      Uk[ax] = U[ax * n + k];
    }
    dvk = ((const gmem<float> *)e.dv)[k];
    st = stencil_row(g, Xk, sub);
    int sl[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) sl[i] = tile_slot[st.tile[i]];
    float4 m[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      m[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (sl[i] >= 0) {
        const vfloat4 v = macro[(size_t)sl[i] * 512 + st.lc[i]];
        m[i] = make_float4(v.x, v.y, v.z, v.w);
      } else
        atomicOr(e.guard, (int)GUARD_CAPACITY);
    }
    if (MDF) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (sl[i] < 0) continue;
        const gmem<unsigned long long> *gp = (const gmem<unsigned long long> *)e.gfix + (size_t)sl[i] * 1536;
        const float h = 0.5f / m[i].x;
        float dx, dy, dz;
        solve_coriolis<ROT>(fr, from_fix(gp[st.lc[i]]) * h, from_fix(gp[512 + st.lc[i]]) * h,
                            from_fix(gp[1024 + st.lc[i]]) * h, dx, dy, dz);
        m[i].y += dx;
        m[i].z += dy;
        m[i].w += dz;
      }
    }
    const float wyz = st.wy * st.wz;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float d = st.wx[i] * wyz;
      sr += m[i].x * d;
      sx += m[i].y * d;
      sy += m[i].z * d;
      sz += m[i].w * d;
    }
  }
  // every lane takes part (a group of 16 is all live or all not)
  sr = group16_sum(sr);
  sx = group16_sum(sx);
  sy = group16_sum(sy);
  sz = group16_sum(sz);
  if (live) {
    gmem<float> *r = (gmem<float> *)e.rec + (size_t)k * REC;
    if (sub == 0) *(gmem<vfloat4> *)r = vfloat4{st.wx[0], st.wx[1], st.wx[2], st.wx[3]};
    if (sub < 4) r[4 + sub] = st.wy;                // row (sy, 0)
    if ((sub & 3) == 0) r[8 + (sub >> 2)] = st.wz;  // row (0, sz)
    if (sub == 0) {
      float rk;
      float Fk[3], inc[3];
      const float Ui[3] = {sx, sy, sz};
      // velocity to correct: U - U^interp, or on a slip wall its normal part
      float dU[3] = {Uk[0] - Ui[0], Uk[1] - Ui[1], Uk[2] - Ui[2]};
      if (e.slip) {
        const float nk[3] = {e.Nrm[k], e.Nrm[n + k], e.Nrm[2 * n + k]};
        const float dn = dU[0] * nk[0] + dU[1] * nk[1] + dU[2] * nk[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) dU[c] = dn * nk[c];
      }
      if (!MDF) {
        rk = sr;
        mstate[k] = rk;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          mstate[(c + 1) * (size_t)n + k] = Ui[c];
          inc[c] = e.alpha2 * rk * dU[c];
          Fk[c] = inc[c];
        }
      } else {
        rk = mstate[k];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          inc[c] = e.alpha2 * rk * dU[c];
          Fk[c] = F[c * n + k] + inc[c];
        }
      }
      float fd[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        F[c * n + k] = Fk[c];
        fd[c] = Fk[c] * dvk;
        r[16 + c] = inc[c] * dvk;
        r[12 + c] = __int_as_float(st.base[c]);
      }
      // fluid on body: -F dV; torque (X - x0) x (-F dV); power F.U dV
      const float rx = Xk[0] - fr.org[0], ry = Xk[1] - fr.org[1], rz = Xk[2] - fr.org[2];
      part[0] = -fd[0];
      part[1] = -fd[1];
      part[2] = -fd[2];
      part[3] = -(ry * fd[2] - rz * fd[1]);
      part[4] = -(rz * fd[0] - rx * fd[2]);
      part[5] = -(rx * fd[1] - ry * fd[0]);
      part[6] = fd[0] * Uk[0] + fd[1] * Uk[1] + fd[2] * Uk[2];
    }
  }
  if (partials == nullptr) return;  // uniform over the workgroup
  if (sub == 0)
    for (int q = 0; q < 7; ++q) s_part[mk][q] = part[q];
  __syncthreads();
  if (tid < 8) {
    float sum = 0.f;
    if (tid < 7)
      for (int q = 0; q < kInterpMk; ++q) sum += s_part[q][tid];
    partials[(size_t)item * 8 + tid] = sum;
  }
  __syncthreads();
}

__device__ __host__ inline int interp_items(int n) { return (n + kInterpMk - 1) / kInterpMk; }
__device__ __host__ inline int wave_items(int n) { return (n + kWavePer - 1) / kWavePer; }

// Wrench of the step: the interpolation partials summed in item order.
__device__ inline void wrench_sum(const float *__restrict__ partials, int nparts, float *__restrict__ wrench, int tid) {
  __shared__ float s_red[WG];
  const int col = tid & 7, row0 = tid >> 3;
  float acc = 0.f;
  if (col < 7)
    for (int b = row0; b < nparts; b += WG / 8) acc += partials[(size_t)b * 8 + col];
  s_red[tid] = acc;
  __syncthreads();
  if (tid < 8) {
    float sum = 0.f;
    for (int r2 = 0; r2 < WG / 8; ++r2) sum += s_red[r2 * 8 + tid];
    wrench[tid] = tid < 7 ? sum : 0.f;
  }
  __syncthreads();
}

// --------------------------------------------------------------- spreading --
// Work item (active tile `slot`, part): g(x) = sum_k F_k dV_k delta(x - X_k)
// over the tile's 512 cells. Wave w of part p owns marker chunks
// c = 8 p + w (mod 8 kSpreadSplit), 64 markers each. It loads 64 of its chunk
// boxes at once and keeps the chunks whose box meets the tile; in each such
// chunk every lane tests its own marker and, on a hit, walks that marker's
// 4x4x4 stencil, adding the nodes inside the tile into the LDS tile with
// 64-bit LDS atomics (2^-40 fixed point). The workgroup then adds its nonzero
// cells into the tile's fixed-point force, one global atomic per cell and
// component. Integer sums make the result independent of every order.
__device__ inline void cg_direction(const EnvView &e, int k, const float *beta, bool first, float p[3]);

// CG = true: the spread values are the search direction of the implicit
// correction's conjugate-gradient step (cg_direction with beta, first), not
// the record's.
template <bool CG, int SPLIT = kSpreadSplit>
__device__ inline void spread_item(const EnvView &e, int item, int tid, unsigned long long *target,
                                   const float *beta = nullptr, bool first = true) {
  __shared__ unsigned long long s_acc[3][512];
  const int lane = tid & 63, wv = tid >> 6;
  const GridArgs &g = e.g;
  const int n = e.n;
  const int nchunks = (n + 63) >> 6;
  const int slot = item / SPLIT, part = item % SPLIT;
  const int t = ((const gmem<int> *)e.active)[slot];
  const int tx = t % g.tnx, ty = (t / g.tnx) % g.tny, tz = t / (g.tnx * g.tny);
  for (int q = tid; q < 3 * 512; q += WG) (&s_acc[0][0])[q] = 0ull;
  __syncthreads();
  const int stride = (WG / 64) * SPLIT;
  const int c_first = part * (WG / 64) + wv;
  for (int it = 0; c_first + stride * 64 * it < nchunks; ++it) {
    const int cl = c_first + stride * (lane + 64 * it);  // chunk examined by this lane
    bool pass = false;
    if (cl < nchunks) {
      const gmem<int> *bp = (const gmem<int> *)e.chunk_box + 4 * (size_t)cl;
      const int4 box = make_int4(bp[0], bp[1], bp[2], bp[3]);
      pass = box_hits(box.x, tx) && box_hits(box.y, ty) && box_hits(box.z, tz);
    }
    unsigned long long cbal = __ballot(pass);
    while (cbal) {
      const int jc = __ffsll((long long)cbal) - 1;
      cbal &= cbal - 1ull;
      const int k = (c_first + stride * (jc + 64 * it)) * 64 + lane;
      bool hit = false;
      if (k < n) {
        const gmem<short> *mb = (const gmem<short> *)e.mbase + 4 * (size_t)k;
        const short4 b = make_short4(mb[0], mb[1], mb[2], mb[3]);
        hit = axis_touches(b.x, g.nx, g.xper, tx) && axis_touches(b.y, g.ny, true, ty) &&
              axis_touches(b.z, g.nz, true, tz);
      }
      if (hit) {
        float r[20];
        const gmem<vfloat4> *rp = (const gmem<vfloat4> *)e.rec + (size_t)k * (REC / 4);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const vfloat4 v = rp[q];
          r[4 * q] = v.x;
          r[4 * q + 1] = v.y;
          r[4 * q + 2] = v.z;
          r[4 * q + 3] = v.w;
        }
        if (CG) {
          cg_direction(e, k, beta, first, &r[16]);
          if (e.slip) {  // the search direction is a normal force p n
            const float p0 = r[16];
            r[16] = p0 * e.Nrm[k];
            r[17] = p0 * e.Nrm[n + k];
            r[18] = p0 * e.Nrm[2 * (size_t)n + k];
          }
        }
        const int bx = __float_as_int(r[12]), by = __float_as_int(r[13]), bz = __float_as_int(r[14]);
        int lx[4], ly[4], lz[4];  // local index part per stencil node, -1 outside the tile
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int jx = bx + q, jy = wrap_idx(by + q, g.ny), jz = wrap_idx(bz + q, g.nz);
          if (g.xper) jx = wrap_idx(jx, g.nx);
          lx[q] = (jx >> 3) == tx ? (jx & 7) : -1;
          ly[q] = (jy >> 3) == ty ? ((jy & 7) << 3) : -1;
          lz[q] = (jz >> 3) == tz ? ((jz & 7) << 6) : -1;
        }
#pragma unroll
        for (int qz = 0; qz < 4; ++qz) {
          if (lz[qz] < 0) continue;
#pragma unroll
          for (int qy = 0; qy < 4; ++qy) {
            if (ly[qy] < 0) continue;
            const float wyz = r[4 + qy] * r[8 + qz];
#pragma unroll
            for (int qx = 0; qx < 4; ++qx) {
              if (lx[qx] < 0) continue;
              const float d = r[qx] * wyz;
              const int lc = lx[qx] | ly[qy] | lz[qz];
              atomicAdd(&s_acc[0][lc], to_fix(r[16] * d));
              atomicAdd(&s_acc[1][lc], to_fix(r[17] * d));
              atomicAdd(&s_acc[2][lc], to_fix(r[18] * d));
            }
          }
        }
      }
    }
  }
  __syncthreads();
  gmem<unsigned long long> *gp = (gmem<unsigned long long> *)target + (size_t)slot * 1536;
  for (int q = tid; q < 3 * 512; q += WG) {
    const unsigned long long v = (&s_acc[0][0])[q];
    if (v != 0ull) __hip_atomic_fetch_add(&gp[q], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

template <int SPLIT = kSpreadSplit>
__device__ inline void spread_item(const EnvView &e, int item, int tid) {
  spread_item<false, SPLIT>(e, item, tid, e.gfix);
}

// ----------------------------------------------- single-lattice launches --
__global__ void __launch_bounds__(WG) k_skin_mark(EnvView e, const float *pose) {
  skin_item(e, pose, blockIdx.x, threadIdx.x);
}

__global__ void __launch_bounds__(WG) k_active(EnvView e) { active_item(e, blockIdx.x, threadIdx.x); }

template <class S, bool ROT>
__global__ void __launch_bounds__(WG) k_macro(EnvView e, FrameF fr, int cur) {
  const XcdWalk w = xcd_walk(n_active_of(e));
  for (int slot = w.first; slot < w.end; slot += w.step) macro_item<S, ROT>(e, fr, cur, slot, threadIdx.x);
}

// Grid: exactly interp_items(n) workgroups. The markers of one XCD are
// consecutive, so its L2 holds the band macros of their stretch of body.
template <bool ROT, bool MDF>
__global__ void __launch_bounds__(WG) k_interp(EnvView e, FrameF fr, float *partials) {
  interp_item<ROT, MDF>(e, fr, xcd_item(blockIdx.x, gridDim.x), threadIdx.x, partials);
}

// wrench != nullptr: workgroup 0 first sums the interpolation partials.
__global__ void __launch_bounds__(WG) k_spread(EnvView e, float *wrench) {
  if (blockIdx.x == 0 && wrench != nullptr) wrench_sum(e.partials, interp_items(e.n), wrench, threadIdx.x);
  const int items = n_active_of(e) * kSpreadSplit;
  for (int item = blockIdx.x; item < items; item += gridDim.x) spread_item(e, item, threadIdx.x);
}

// ------------------------------------------- implicit velocity correction --
// The marker forces G_k = F_k dV_k solve S G = (I + [omega]x)(U - U*) with
// S = interp . 1/(2 rho) . spread (the implicit immersed boundary of Wu and
// Shu, cited in the paper's Introduction): interpolating u* + M spread(G) /
// (2 rho) then gives U at every marker, M = (I + [omega]x)^-1 the Coriolis
// solve of the fluid velocity. M is the same at every node, so S acts on each
// component alone and is symmetric positive semidefinite; conjugate
// gradients with the diagonal preconditioner 2 rho_k (S's diagonal is
// (3/8)^3 / (2 rho) for a uniform density) take mdf_iters steps from G = 0.
// The spread and the interpolation of S use the weights of the marker record,
// so the discrete S is exactly symmetric up to float rounding. On a slip wall
// the unknown is one normal force gamma_k n_k per marker: the vectors keep it
// in component 0 (the others stay zero, and their guarded alpha and beta
// vanish), the spread takes p n and the apply the normal part of S p n,
// (N^T S N) gamma = N^T (U - U*); the frame must not rotate.
//
// Per step, after the first interpolation pass (rho_k, U*_k, record):
//   cg_init_item     r = (I + [omega]x)(U - U*), G = 0; rz_0 = r.z, z = 2 rho_k r
//   step j = 0, 1, ...:
//     spread (CG)    p_j = z_j + beta_j p_{j-1} (p_0 = z_0) computed per
//                    marker hit, spread into gcg
//     cg_apply_item  q = S p_j from gcg; stores p_j and q; p.q rows
//     cg_update_item alpha_j = rz_j / p_j.q; G += alpha_j p_j; r -= alpha_j q;
//                    rz_{j+1};
//                    beta_{j+1} = rz_{j+1} / rz_j; clears gcg; on the last
//                    step F = G / dV, the record carries G, wrench partials
//   then the ordinary spread of the record into gfix.
// Each dot product is a sum of per-workgroup partial rows added in row order:
// p.q by every update workgroup; r.z by the init or update workgroup that
// arrives last (cg_last_arrival), which stores rz and beta for the kernels
// that follow. Every workgroup uses the same values, and the step is
// deterministic.
constexpr int kCgWG = 256;     // markers per init and update workgroup
constexpr int kCgMaxSteps = 16;
__device__ __host__ inline int cg_items(int n) { return (n + kCgWG - 1) / kCgWG; }
// Partial rows and scalars, 4 floats each: p.q rows (one per apply
// workgroup), r.z rows (one per init/update workgroup), then rz_j and beta_j
// for j = 0 .. kCgMaxSteps.
__device__ __host__ inline size_t cg_part_floats(int n) {
  return 4 * ((size_t)interp_items(n) + (size_t)cg_items(n) + 2 * (kCgMaxSteps + 1));
}
__device__ inline float *cg_pq(const EnvView &e) { return e.cgpart; }
__device__ inline float *cg_rzp(const EnvView &e) { return e.cgpart + 4 * (size_t)interp_items(e.n); }
__device__ inline float *cg_scal(const EnvView &e, int which, int j) {  // which: 0 rz, 1 beta
  return cg_rzp(e) + 4 * (size_t)cg_items(e.n) + 4 * (size_t)(which * (kCgMaxSteps + 1) + j);
}

// Sums of parts[j][0..2] over j < m in row order, by the whole workgroup (a
// multiple of 64 threads, at most 1024). Ends with a barrier.
__device__ inline void cg_sum3(const float *__restrict__ parts, int m, float out[3]) {
  __shared__ float s[3][16];
  const int tid = threadIdx.x, nt = blockDim.x;
  float a[3] = {0.f, 0.f, 0.f};
  for (int j = tid; j < m; j += nt)
#pragma unroll
    for (int c = 0; c < 3; ++c) a[c] += parts[4 * (size_t)j + c];
#pragma unroll
  for (int c = 0; c < 3; ++c) a[c] = wave_sum(a[c]);
  if ((tid & 63) == 0)
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c][tid >> 6] = a[c];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float t = 0.f;
    for (int w = 0; w < (nt >> 6); ++w) t += s[c][w];
    out[c] = t;
  }
  __syncthreads();
}

// Workgroup sums of v[0..2] written to part[0..2] by thread 0. Ends with a
// barrier.
__device__ inline void cg_part3(const float v[3], float *__restrict__ part) {
  __shared__ float s[3][16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float w[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) w[c] = wave_sum(v[c]);
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c][wv] = w[c];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float t = 0.f;
      for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += s[c][q];
      part[c] = t;
    }
  __syncthreads();
}

// Called by every thread of each of `count` workgroups after thread 0 has
// written the workgroup's partial row: true in the workgroup that arrives
// last, which then sees every row. That workgroup resets the counter for the
// next kernel.
__device__ inline bool cg_last_arrival(int *counter, int count) {
  __shared__ int s_last;
  if (threadIdx.x == 0) {
    __threadfence();  // the row, visible device-wide before the arrival
    const int prev = atomicAdd(counter, 1);
    s_last = prev == count - 1 ? 1 : 0;
    if (s_last) atomicExch(counter, 0);
  }
  __syncthreads();
  const bool last = s_last != 0;
  if (last) __threadfence();
  return last;
}

// Search direction of marker k: p = z + beta p_prev, z = 2 rho_k r (p = z on
// the first step).
__device__ inline void cg_direction(const EnvView &e, int k, const float *beta, bool first, float p[3]) {
  const int n = e.n;
  const float p2 = 2.0f * e.mstate[k];
  const float *r = e.cg + 3 * (size_t)n, *pp = e.cg + 6 * (size_t)n;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float z = p2 * r[c * n + k];
    p[c] = first ? z : z + beta[c] * pp[c * n + k];
  }
}

template <bool ROT>
__device__ inline void cg_init_item(const EnvView &e, const FrameF &fr, int item) {
  const int n = e.n, k = item * kCgWG + (int)threadIdx.x;
  float rz[3] = {0.f, 0.f, 0.f};
  if (k < n) {
    float R[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) R[c] = e.U[c * n + k] - e.mstate[(c + 1) * (size_t)n + k];
    float r[3] = {R[0], R[1], R[2]};
    if (ROT) {
      float wx, wy, wz;
      cross3(fr.omg, R[0], R[1], R[2], wx, wy, wz);
      r[0] += wx;
      r[1] += wy;
      r[2] += wz;
    }
    if (e.slip) {  // one unknown per marker, the normal force: r = n.(U - U*) in component 0
      r[0] = e.Nrm[k] * R[0] + e.Nrm[n + k] * R[1] + e.Nrm[2 * (size_t)n + k] * R[2];
      r[1] = r[2] = 0.f;
    }
    const float p2 = 2.0f * e.mstate[k];
    float *G = e.cg, *rr = e.cg + 3 * (size_t)n;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      G[c * n + k] = 0.f;
      rr[c * n + k] = r[c];
      rz[c] = r[c] * (p2 * r[c]);
    }
  }
  cg_part3(rz, cg_rzp(e) + 4 * (size_t)item);
  if (cg_last_arrival(e.counters + 1, cg_items(n))) {
    float t[3];
    cg_sum3(cg_rzp(e), cg_items(n), t);
    if (threadIdx.x < 3) cg_scal(e, 0, 0)[threadIdx.x] = t[threadIdx.x];
  }
}

// Markers 32*item .. 32*item+31, 16 lanes each, lane = x-row of stencil
// nodes (as interp_item): q_k = sum_x delta(x - X_k) gcg(x) / (2 rho(x)) with
// gcg the spread of step j's search direction, which is stored here. The
// weights are the record's, multiplied as the spreading multiplies them, so
// the discrete S is symmetric.
__device__ inline void cg_apply_item(const EnvView &e, int item, int tid, int j) {
#pragma clang fp contract(on)  // as interp_item
  __shared__ float s_pq[kInterpMk][3];
  const int sub = tid & 15, mk = tid >> 4;
  const int k = item * kInterpMk + mk;
  const int n = e.n;
  const GridArgs &g = e.g;
  const bool live = k < n;
  float pq[3] = {0.f, 0.f, 0.f};
  float v[3] = {0.f, 0.f, 0.f};
  if (live) {
    const float *r = e.rec + (size_t)k * REC;
    const int jy = __float_as_int(r[13]) + (sub & 3), jz = __float_as_int(r[14]) + (sub >> 2);
    const int bx = __float_as_int(r[12]);
    const float wyz = r[4 + (sub & 3)] * r[8 + (sub >> 2)];
    const int yn = wrap_idx(jy, g.ny), zn = wrap_idx(jz, g.nz);
    const int trow = g.tnx * ((yn >> 3) + g.tny * (zn >> 3));
    const int lrow = ((yn & 7) << 3) | ((zn & 7) << 6);
    int sl[4], lc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int xn = g.xper ? wrap_idx(bx + i, g.nx) : bx + i;
      sl[i] = e.tile_slot[(xn >> 3) + trow];
      lc[i] = (xn & 7) | lrow;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (sl[i] < 0) continue;  // never: the first interpolation pass checked every stencil node
      const unsigned long long *gq = e.gcg + (size_t)sl[i] * 1536;
      const float h = 0.5f / e.macro[(size_t)sl[i] * 512 + lc[i]].x;
      const float d = r[i] * wyz;
#pragma unroll
      for (int c = 0; c < 3; ++c) v[c] += (from_fix(gq[512 * c + lc[i]]) * h) * d;
    }
  }
  const float qx = group16_sum(v[0]), qy = group16_sum(v[1]), qz = group16_sum(v[2]);
  if (live && sub == 0) {
    float q[3] = {qx, qy, qz};
    if (e.slip) {  // n . (S p n)
      q[0] = e.Nrm[k] * qx + e.Nrm[n + k] * qy + e.Nrm[2 * (size_t)n + k] * qz;
      q[1] = q[2] = 0.f;
    }
    float p[3];
    cg_direction(e, k, cg_scal(e, 1, j), j == 0, p);
    float *qv = e.cg + 9 * (size_t)n, *pv = e.cg + 6 * (size_t)n;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      qv[c * n + k] = q[c];
      pv[c * n + k] = p[c];
      pq[c] = p[c] * q[c];
    }
  }
  if (sub == 0)
#pragma unroll
    for (int c = 0; c < 3; ++c) s_pq[mk][c] = pq[c];
  __syncthreads();
  if (tid < 3) {
    float t = 0.f;
    for (int q = 0; q < kInterpMk; ++q) t += s_pq[q][tid];
    cg_pq(e)[4 * (size_t)item + tid] = t;
  }
}

// Step j of conjugate gradients for markers item*kCgWG ... On the last step
// also the outputs: F = G / dV, the record's spread value G, and the wrench
// partials per interpolation item (the layout wrench_sum reads).
__device__ inline void cg_update_item(const EnvView &e, const FrameF &fr, int item, int j, bool last) {
#pragma clang fp contract(on)  // as interp_item
  const int n = e.n, k = item * kCgWG + (int)threadIdx.x;
  float pq[3], alpha[3];
  cg_sum3(cg_pq(e), interp_items(n), pq);  // every workgroup, in row order
  const float *rz = cg_scal(e, 0, j);
#pragma unroll
  for (int c = 0; c < 3; ++c) alpha[c] = pq[c] > 0.f ? rz[c] / pq[c] : 0.f;
  float rzn[3] = {0.f, 0.f, 0.f}, part[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (k < n) {
    float *G = e.cg, *r = e.cg + 3 * (size_t)n;
    const float *p = e.cg + 6 * (size_t)n, *q = e.cg + 9 * (size_t)n;
    const float p2 = 2.0f * e.mstate[k];
    float Gk[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float a = alpha[c];
      Gk[c] = G[c * n + k] + a * p[c * n + k];
      const float rk = r[c * n + k] - a * q[c * n + k];
      G[c * n + k] = Gk[c];
      r[c * n + k] = rk;
      rzn[c] = rk * (p2 * rk);
    }
    if (last) {
      if (e.slip) {  // the normal force gamma n
        const float gam = Gk[0];
        Gk[0] = gam * e.Nrm[k];
        Gk[1] = gam * e.Nrm[n + k];
        Gk[2] = gam * e.Nrm[2 * (size_t)n + k];
      }
      const float idv = 1.0f / e.dv[k];
      float *rec = e.rec + (size_t)k * REC;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        e.F[c * n + k] = Gk[c] * idv;
        rec[16 + c] = Gk[c];
      }
      const float Uk[3] = {e.U[k], e.U[n + k], e.U[2 * n + k]};
      const float rx = e.X[k] - fr.org[0], ry = e.X[n + k] - fr.org[1], rzz = e.X[2 * n + k] - fr.org[2];
      part[0] = -Gk[0];
      part[1] = -Gk[1];
      part[2] = -Gk[2];
      part[3] = -(ry * Gk[2] - rzz * Gk[1]);
      part[4] = -(rzz * Gk[0] - rx * Gk[2]);
      part[5] = -(rx * Gk[1] - ry * Gk[0]);
      part[6] = Gk[0] * Uk[0] + Gk[1] * Uk[1] + Gk[2] * Uk[2];
    }
  }
  if (!last) {
    cg_part3(rzn, cg_rzp(e) + 4 * (size_t)item);
    if (cg_last_arrival(e.counters + 1, cg_items(n))) {
      float t[3];
      cg_sum3(cg_rzp(e), cg_items(n), t);
      if (threadIdx.x < 3) {
        const float rz0 = cg_scal(e, 0, j)[threadIdx.x];
        cg_scal(e, 0, j + 1)[threadIdx.x] = t[threadIdx.x];
        cg_scal(e, 1, j + 1)[threadIdx.x] = rz0 != 0.f ? t[threadIdx.x] / rz0 : 0.f;
      }
    }
    return;
  }
  // groups of kInterpMk consecutive markers (aligned lanes of one wave) form
  // one interpolation item
#pragma unroll
  for (int qd = 0; qd < 7; ++qd)
    for (int o = kInterpMk / 2; o > 0; o >>= 1) part[qd] += shfl_xor_f(part[qd], o);
  const int it = k / kInterpMk;
  if ((k % kInterpMk) == 0 && k < n)
#pragma unroll
    for (int qd = 0; qd < 7; ++qd) e.partials[(size_t)it * 8 + qd] = part[qd];
}

template <bool ROT>
__global__ void __launch_bounds__(kCgWG) k_cg_init(EnvView e, FrameF fr) { cg_init_item<ROT>(e, fr, blockIdx.x); }

// Spreading of step j's search direction into gcg.
__global__ void __launch_bounds__(WG) k_spread_cg(EnvView e, int j) {
  const int items = n_active_of(e) * kSpreadSplit;
  const float *beta = cg_scal(e, 1, j);
  for (int item = blockIdx.x; item < items; item += gridDim.x)
    spread_item<true>(e, item, threadIdx.x, e.gcg, beta, j == 0);
}

// Grid: exactly interp_items(n) workgroups (the last-arrival count).
__global__ void __launch_bounds__(WG) k_cg_apply(EnvView e, int j) {
  cg_apply_item(e, xcd_item(blockIdx.x, gridDim.x), threadIdx.x, j);
}

// Grid: at least cg_items(n) workgroups; the first cg_items(n) take the
// markers, and all of them clear gcg for the next step's spread (not after
// the last step: the next lattice step's macro pass clears it).
__global__ void __launch_bounds__(kCgWG) k_cg_update(EnvView e, FrameF fr, int j, int last) {
  if ((int)blockIdx.x < cg_items(e.n)) cg_update_item(e, fr, blockIdx.x, j, last != 0);
  if (last) return;
  const size_t words = (size_t)n_active_of(e) * 1536;
  for (size_t q = (size_t)blockIdx.x * kCgWG + threadIdx.x; q < words; q += (size_t)gridDim.x * kCgWG) e.gcg[q] = 0ull;
}

// Block reduction of 8 floats over the workgroup.
__device__ inline void block_sum8(float v[8], float *smem /* [16][8] + 8 */) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = wave_sum(v[q]);
  if (lane == 0)
    for (int q = 0; q < 8; ++q) smem[wv * 8 + q] = v[q];
  __syncthreads();
  if (threadIdx.x < 8) {
    float s = 0.f;
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) s += smem[w * 8 + threadIdx.x];
    smem[128 + threadIdx.x] = s;
  }
  __syncthreads();
  for (int q = 0; q < 8; ++q) v[q] = smem[128 + q];
}

// Fluid force, torque about `center`, and power sum F.U dV, for the whole body
// (blockIdx.x == 0) or one bone's blend-weighted share (blockIdx.x == 1 + b).
__global__ void __launch_bounds__(1024) k_wrench(const float *__restrict__ X, const float *__restrict__ U,
                                                 const float *__restrict__ F, const float *__restrict__ dv,
                                                 const int *__restrict__ bone, const float *__restrict__ weight,
                                                 int n, float c0, float c1, float c2, float *__restrict__ out) {
  __shared__ float smem[16 * 8 + 8];
  const int b = (int)blockIdx.x - 1;
  float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    float wk = 1.0f;
    if (b >= 0) wk = (bone[k] == b ? weight[k] : 0.f) + (bone[n + k] == b ? weight[n + k] : 0.f);
    const float s = wk * dv[k];
    const float fx = F[k] * s, fy = F[n + k] * s, fz = F[2 * n + k] * s;
    const float rx = X[k] - c0, ry = X[n + k] - c1, rz = X[2 * n + k] - c2;
    v[0] -= fx;
    v[1] -= fy;
    v[2] -= fz;
    v[3] -= ry * fz - rz * fy;
    v[4] -= rz * fx - rx * fz;
    v[5] -= rx * fy - ry * fx;
    v[6] += fx * U[k] + fy * U[n + k] + fz * U[2 * n + k];
  }
  block_sum8(v, smem);
  if (threadIdx.x < 8) out[blockIdx.x * 8 + threadIdx.x] = threadIdx.x < 7 ? v[threadIdx.x] : 0.f;
}

}  // namespace lbmib
