// Immersed-boundary kernels: skinning, tile binning, interpolation with direct
// forcing, gather-form spreading and the body wrench.
//
// The immersed force lives only in "active" 8x8x8 tiles: tiles that some
// marker's 4x4x4 Peskin stencil touches. Each step rebuilds the active set:
//   k_skin_mark     skin markers (linear blend skinning), wrap/check range,
//                   flag the tiles each stencil touches
//   k_active        compact the flags into a slot map and an active list
//   k_macro         density and unforced velocity of every active-tile cell
//   k_interp        one wave64 per marker, one lane per stencil node: weights,
//                   wave-level sums -> U*_k, rho_k, direct forcing F_k, and the
//                   body wrench reduced in workgroup order
//   k_spread        per (active tile, part): LDS fixed-point accumulation of
//                   the markers touching the tile, merged into the tile's
//                   fixed-point force - order-independent (deterministic)
//   k_wrench        per-bone wrench for the body-forces query
#pragma once

#include "fluid.hpp"

namespace lbmib {

struct IBArgs {
  GridArgs g;
  FrameF fr;
  int n, nbones;
  float alpha2;  // 2 * alpha (direct-forcing gain)
  int cap;       // active-tile capacity
};

// Marker record written by k_interp, read by k_spread: Peskin weights of the
// four stencil nodes per axis, the stencil base node per axis and F_k dV_k.
constexpr int REC = 20;  // floats: w[12], base[3], pad, fdv[3], pad

__device__ inline int stencil_base(float X) { return (int)floorf(X) - 1; }

// Distinct tiles along one axis touched by nodes base..base+3 (wrapped when
// periodic). At most 3.
__device__ inline int axis_tiles(int base, int n, bool per, int out[3]) {
  int cnt = 0;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    int j = base + s;
    if (per) j = wrap_idx(j, n);
    int t = j >> 3;
    bool dup = false;
    for (int q = 0; q < cnt; ++q) dup |= out[q] == t;
    if (!dup && cnt < 3) out[cnt++] = t;
  }
  return cnt;
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

// Linear blend skinning, domain handling and active-tile marking (one thread
// per marker). Periodic axes: X is wrapped into [0, n). Open x: markers must
// satisfy 2 <= X < nx - 3 so the stencil stays on nodes 1 .. nx-2; others
// raise the range guard and are clamped so that every access stays in bounds.
// Every tile a marker's stencil touches gets flag 1 (plain stores of one
// value: no atomics). mbase[k] keeps the stencil base node per axis for the
// spreading scan. Thread 0 also clears the active-tile counter of this step.
// Launched with 64-thread-aligned blocks: wave c (markers 64c .. 64c+63) also
// writes chunk_box[c], the range of tiles its markers' stencils touch per
// axis (whole axis when a stencil wraps), so spreading can skip chunks.
__global__ void k_skin_mark(const float *__restrict__ xrest, const int *__restrict__ bone,
                            const float *__restrict__ weight, const float *__restrict__ pose, float *__restrict__ X,
                            float *__restrict__ U, short4 *__restrict__ mbase, int *__restrict__ tile_flag,
                            int4 *__restrict__ chunk_box, int *__restrict__ counters, IBArgs a,
                            int *__restrict__ guard) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = a.n;
  if (k == 0) counters[0] = 0;
  const int tns[3] = {a.g.tnx, a.g.tny, (a.g.nz + 7) >> 3};
  int lo[3] = {1 << 20, 1 << 20, 1 << 20}, hi[3] = {-1, -1, -1};
  if (k < n) {
  const float r0 = xrest[k], r1 = xrest[n + k], r2 = xrest[2 * n + k];
  float p[3] = {0.f, 0.f, 0.f}, v[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    int b = bone[j * n + k];
    float w = weight[j * n + k];
    if ((unsigned)b >= (unsigned)a.nbones) {
      atomicOr(guard, (int)GUARD_BONE);
      b = 0;
      w = 0.f;
    }
    const float *P = pose + 24 * b;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      p[r] += w * (P[3 * r] * r0 + P[3 * r + 1] * r1 + P[3 * r + 2] * r2 + P[9 + r]);
      v[r] += w * (P[12 + 3 * r] * r0 + P[12 + 3 * r + 1] * r1 + P[12 + 3 * r + 2] * r2 + P[21 + r]);
    }
  }
  const int dims[3] = {a.g.nx, a.g.ny, a.g.nz};
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const float nn = (float)dims[ax];
    const bool per = ax > 0 || a.g.xper;
    if (per) {
      float q = p[ax] - nn * floorf(p[ax] / nn);
      if (!(q >= 0.f && q < nn)) q = 0.f;
      p[ax] = q;
    } else if (!(p[ax] >= 2.0f && p[ax] < nn - 3.0f)) {
      atomicOr(guard, (int)GUARD_MARKER_RANGE);
      p[ax] = (p[ax] >= 2.0f) ? nn - 3.5f : 2.0f;
    }
    X[ax * n + k] = p[ax];
    U[ax * n + k] = v[ax];
  }
  const int bs[3] = {stencil_base(p[0]), stencil_base(p[1]), stencil_base(p[2])};
  mbase[k] = make_short4((short)bs[0], (short)bs[1], (short)bs[2], 0);
  int tx[3], ty[3], tz[3];
  const int nxt = axis_tiles(bs[0], a.g.nx, a.g.xper, tx);
  const int nyt = axis_tiles(bs[1], a.g.ny, true, ty);
  const int nzt = axis_tiles(bs[2], a.g.nz, true, tz);
  for (int i = 0; i < nzt; ++i)
    for (int j = 0; j < nyt; ++j)
      for (int l = 0; l < nxt; ++l) tile_flag[tx[l] + a.g.tnx * (ty[j] + a.g.tny * tz[i])] = 1;
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
      lo[ax] = min(lo[ax], __shfl_xor(lo[ax], o, 64));
      hi[ax] = max(hi[ax], __shfl_xor(hi[ax], o, 64));
    }
  }
  if ((threadIdx.x & 63) == 0 && k < n)
    chunk_box[k >> 6] = make_int4(lo[0] | (hi[0] << 16), lo[1] | (hi[1] << 16), lo[2] | (hi[2] << 16), 0);
}

// Compaction of the flagged tiles (1024 tiles per workgroup): slots in
// workgroup order from one atomic per workgroup. Slot numbering only decides
// storage locations, never results. Clears the flags for the next step.
__global__ void __launch_bounds__(1024) k_active(int *__restrict__ tile_flag, int *__restrict__ tile_slot,
                                                 int *__restrict__ active, int *__restrict__ counters, int ntiles,
                                                 int cap, int *__restrict__ guard) {
  __shared__ int s_w[16];
  __shared__ int s_base;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int t = blockIdx.x * 1024 + tid;
  int f = 0;
  if (t < ntiles) {
    f = tile_flag[t] != 0;
    tile_flag[t] = 0;
  }
  const unsigned long long bal = __ballot(f);
  if (lane == 0) s_w[wv] = __popcll(bal);
  __syncthreads();
  if (tid == 0) {
    int tot = 0;
    for (int q = 0; q < 16; ++q) tot += s_w[q];
    s_base = tot ? atomicAdd(&counters[0], tot) : 0;
  }
  __syncthreads();
  int pre = s_base;
  for (int q = 0; q < wv; ++q) pre += s_w[q];
  pre += __popcll(bal & ((1ull << lane) - 1ull));
  if (t < ntiles) {
    if (f && pre < cap) {
      tile_slot[t] = pre;
      active[pre] = t;
    } else {
      tile_slot[t] = -1;
      if (f) atomicOr(guard, (int)GUARD_CAPACITY);
    }
  }
}

// Density and unforced velocity u* (frame force, no IB force) of every cell
// of every active tile (grid-stride over slots, 512 threads = the tile).
// Also clears the tile's fixed-point immersed force for this step.
template <class S, bool ROT>
__global__ void __launch_bounds__(512) k_macro(const typename S::T *__restrict__ src, const int *__restrict__ active,
                                               const int *__restrict__ counters, float4 *__restrict__ macro,
                                               unsigned long long *__restrict__ gfix, IBArgs a) {
  const int tid = threadIdx.x;
  const int n_active = min(counters[0], a.cap);
  const GridArgs &g = a.g;
  for (int slot = blockIdx.x; slot < n_active; slot += gridDim.x) {
    const int t = active[slot];
    const int tx = t % g.tnx, ty = (t / g.tnx) % g.tny, tz = t / (g.tnx * g.tny);
    const int x = tx * 8 + (tid & 7), y = ty * 8 + ((tid >> 3) & 7), z = tz * 8 + (tid >> 6);
    float4 out = make_float4(1.f, 0.f, 0.f, 0.f);
    if (x < g.nx && y < g.ny && z < g.nz && (g.xper || (x > 0 && x < g.nx - 1))) {
      const int xm = g.xper ? wrap_idx(x - 1, g.nx) : x - 1;
      const int xp = g.xper ? wrap_idx(x + 1, g.nx) : x + 1;
      float f[Q];
      pull27<S>(src, g.plane, g.nx, g.ny, xm, x, xp, wrap_idx(y - 1, g.ny), y, wrap_idx(y + 1, g.ny),
                wrap_idx(z - 1, g.nz), z, wrap_idx(z + 1, g.nz), f);
      float rho, mx, my, mz;
      moments(f, rho, mx, my, mz);
      float ax, ay, az;
      frame_a0<ROT>(a.fr, (float)x, (float)y, (float)z, ax, ay, az);
      float ux, uy, uz;
      const float ir = 1.0f / rho;
      solve_coriolis<ROT>(a.fr, mx * ir + 0.5f * ax, my * ir + 0.5f * ay, mz * ir + 0.5f * az, ux, uy, uz);
      out = make_float4(rho, ux, uy, uz);
    }
    macro[(size_t)slot * 512 + tid] = out;
    unsigned long long *gp = gfix + (size_t)slot * 1536;
    gp[tid] = 0ull;
    gp[512 + tid] = 0ull;
    gp[1024 + tid] = 0ull;
  }
}

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One wave64 per marker (16 per workgroup); lane l is stencil node
// (l & 3, (l >> 2) & 3, l >> 4).
// pass 0: U*_k = sum u* delta, rho_k = sum rho delta, F_k = 2 alpha rho_k (U_k - U*_k).
// pass p > 0 (multi-direct forcing): the interpolated velocity includes the
// current immersed force, u = u* + (I + [omega]x)^-1 g / (2 rho), and
// F_k += 2 alpha rho_k (U_k - U_k^interp).
// On the last pass (partials != nullptr): the fluid's force, torque about
// the frame origin and power, summed per workgroup into partials[block][8];
// k_spread adds them up in workgroup order.
template <bool ROT, bool MDF>
__global__ void __launch_bounds__(1024) k_interp(const float *__restrict__ X, const float *__restrict__ U,
                                                 const float *__restrict__ dv, float *__restrict__ F,
                                                 float *__restrict__ mstate, float *__restrict__ rec,
                                                 const int *__restrict__ tile_slot, const float4 *__restrict__ macro,
                                                 const unsigned long long *__restrict__ gfix, IBArgs a,
                                                 int *__restrict__ guard, float *__restrict__ partials) {
  __shared__ float s_part[16][8];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int k = blockIdx.x * 16 + wv;
  const int n = a.n;
  const GridArgs &g = a.g;
  float part[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (k < n) {
    const float Xk[3] = {X[k], X[n + k], X[2 * n + k]};
    const int s3[3] = {lane & 3, (lane >> 2) & 3, lane >> 4};
    const int dims[3] = {g.nx, g.ny, g.nz};
    int base[3], node[3];
    float w[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      base[ax] = stencil_base(Xk[ax]);
      const int j = base[ax] + s3[ax];
      w[ax] = peskin4(Xk[ax] - (float)j);
      node[ax] = (ax > 0 || g.xper) ? wrap_idx(j, dims[ax]) : j;
    }
    const int t = (node[0] >> 3) + g.tnx * ((node[1] >> 3) + g.tny * (node[2] >> 3));
    const int s = tile_slot[t];
    float rho = 0.f, ux = 0.f, uy = 0.f, uz = 0.f;
    if (s >= 0) {
      const int lc = (node[0] & 7) | ((node[1] & 7) << 3) | ((node[2] & 7) << 6);
      const float4 m = macro[(size_t)s * 512 + lc];
      rho = m.x;
      ux = m.y;
      uy = m.z;
      uz = m.w;
      if (MDF) {
        const unsigned long long *gp = gfix + (size_t)s * 1536;
        const float h = 0.5f / rho;
        float dx, dy, dz;
        solve_coriolis<ROT>(a.fr, from_fix(gp[lc]) * h, from_fix(gp[512 + lc]) * h, from_fix(gp[1024 + lc]) * h, dx,
                            dy, dz);
        ux += dx;
        uy += dy;
        uz += dz;
      }
    } else {
      atomicOr(guard, (int)GUARD_CAPACITY);
    }
    const float d = w[0] * w[1] * w[2];
    const float sr = wave_sum(rho * d), sx = wave_sum(ux * d), sy = wave_sum(uy * d), sz = wave_sum(uz * d);
    float *r = rec + (size_t)k * REC;
    if (lane < 4) r[lane] = w[0];                                 // s3 = (lane, 0, 0)
    if ((lane & 3) == 0 && lane < 16) r[4 + (lane >> 2)] = w[1];  // s3 = (0, lane/4, 0)
    if ((lane & 15) == 0) r[8 + (lane >> 4)] = w[2];              // s3 = (0, 0, lane/16)
    if (lane == 0) {
      // inc = this pass's force; the record carries inc dV because the
      // spreading kernel adds each pass into the step's accumulated g
      float rk;
      float Fk[3], inc[3];
      const float Uk[3] = {U[k], U[n + k], U[2 * n + k]};
      const float Ui[3] = {sx, sy, sz};
      if (!MDF) {
        rk = sr;
        mstate[k] = rk;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          mstate[(c + 1) * (size_t)n + k] = Ui[c];
          inc[c] = a.alpha2 * rk * (Uk[c] - Ui[c]);
          Fk[c] = inc[c];
        }
      } else {
        rk = mstate[k];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          inc[c] = a.alpha2 * rk * (Uk[c] - Ui[c]);
          Fk[c] = F[c * n + k] + inc[c];
        }
      }
      const float dvk = dv[k];
      float fd[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        F[c * n + k] = Fk[c];
        fd[c] = Fk[c] * dvk;
        r[16 + c] = inc[c] * dvk;
        r[12 + c] = __int_as_float(base[c]);
      }
      // fluid on body: -F dV; torque (X - x0) x (-F dV); power F.U dV
      const float rx = Xk[0] - a.fr.org[0], ry = Xk[1] - a.fr.org[1], rz = Xk[2] - a.fr.org[2];
      part[0] = -fd[0];
      part[1] = -fd[1];
      part[2] = -fd[2];
      part[3] = -(ry * fd[2] - rz * fd[1]);
      part[4] = -(rz * fd[0] - rx * fd[2]);
      part[5] = -(rx * fd[1] - ry * fd[0]);
      part[6] = fd[0] * Uk[0] + fd[1] * Uk[1] + fd[2] * Uk[2];
    }
  }
  if (partials == nullptr) return;  // uniform over the grid
  if (lane == 0)
    for (int q = 0; q < 7; ++q) s_part[wv][q] = part[q];
  __syncthreads();
  if (threadIdx.x < 8) {
    float sum = 0.f;
    if (threadIdx.x < 7)
      for (int q = 0; q < 16; ++q) sum += s_part[q][threadIdx.x];
    partials[(size_t)blockIdx.x * 8 + threadIdx.x] = sum;
  }
}

__device__ inline float bcast(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}

__device__ inline bool box_hits(int packed, int t) { return t >= (packed & 0xFFFF) && t <= (packed >> 16); }

// Spreading accumulates in 64-bit fixed point: every contribution is rounded
// to a multiple of 2^-40 (see fluid.hpp, to_fix / from_fix) and summed as an
// integer. Integer addition is associative, so sums do not depend on the order
// in which waves or workgroups add - the result is deterministic.
constexpr int kSpreadSplit = 4;  // workgroups per active tile

// Spreading, gather form: g(x) = sum_k F_k dV_k delta(x - X_k) over the active
// tiles. Work item = (tile, part), kSpreadSplit parts per tile, 1024 threads.
// Wave w of part p owns marker chunks c = 16 p + w (mod 16 kSpreadSplit)
// (64 markers each). It loads 64 of its chunk boxes at once and keeps the
// chunks whose box meets the tile; in each such chunk every lane tests its own
// marker and loads its record, and the hits are broadcast one by one to the 64
// lanes (one per stencil node), which add their node's contribution into the
// workgroup's LDS tile with 64-bit LDS atomics. Each workgroup then adds its
// nonzero cells into the tile's fixed-point force (one global atomic per
// cell and component; k_macro zeroed it this step).
// Workgroup 0 first adds the interpolation kernel's wrench partials in order.
__global__ void __launch_bounds__(1024) k_spread(const float *__restrict__ rec, const short4 *__restrict__ mbase,
                                                 const int4 *__restrict__ chunk_box,
                                                 const int *__restrict__ active, const int *__restrict__ counters,
                                                 unsigned long long *__restrict__ gfix, IBArgs a,
                                                 const float *__restrict__ partials, int nparts,
                                                 float *__restrict__ wrench) {
  __shared__ unsigned long long s_acc[3][512];
  __shared__ float s_red[1024];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const GridArgs &g = a.g;
  const int n = a.n;
  const int nchunks = (n + 63) >> 6;
  if (blockIdx.x == 0 && wrench != nullptr) {
    const int col = tid & 7, row0 = tid >> 3;
    float acc = 0.f;
    if (col < 7)
      for (int b = row0; b < nparts; b += 128) acc += partials[(size_t)b * 8 + col];
    s_red[tid] = acc;
    __syncthreads();
    if (tid < 8) {
      float sum = 0.f;
      for (int r2 = 0; r2 < 128; ++r2) sum += s_red[r2 * 8 + tid];
      wrench[tid] = tid < 7 ? sum : 0.f;
    }
  }
  const int n_items = min(counters[0], a.cap) * kSpreadSplit;
  const int stride = 16 * kSpreadSplit;
  for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
    const int slot = item / kSpreadSplit, part = item % kSpreadSplit;
    const int t = active[slot];
    const int tx = t % g.tnx, ty = (t / g.tnx) % g.tny, tz = t / (g.tnx * g.tny);
    for (int q = tid; q < 3 * 512; q += 1024) (&s_acc[0][0])[q] = 0ull;
    __syncthreads();
    const int c_first = part * 16 + wv;
    for (int it = 0; c_first + stride * 64 * it < nchunks; ++it) {
      const int cl = c_first + stride * (lane + 64 * it);  // chunk examined by this lane
      bool pass = false;
      if (cl < nchunks) {
        const int4 box = chunk_box[cl];
        pass = box_hits(box.x, tx) && box_hits(box.y, ty) && box_hits(box.z, tz);
      }
      unsigned long long cbal = __ballot(pass);
      while (cbal) {
        const int jc = __ffsll((long long)cbal) - 1;
        cbal &= cbal - 1ull;
        const int k = (c_first + stride * (jc + 64 * it)) * 64 + lane;
        bool hit = false;
        if (k < n) {
          const short4 b = mbase[k];
          hit = axis_touches(b.x, g.nx, g.xper, tx) && axis_touches(b.y, g.ny, true, ty) &&
                axis_touches(b.z, g.nz, true, tz);
        }
        if (hit) {
          // this lane's marker: walk its 4x4x4 stencil, adding the nodes that
          // fall in the tile
          float r[20];
          const float4 *rp = reinterpret_cast<const float4 *>(rec + (size_t)k * REC);
#pragma unroll
          for (int q = 0; q < 5; ++q) {
            const float4 v = rp[q];
            r[4 * q] = v.x;
            r[4 * q + 1] = v.y;
            r[4 * q + 2] = v.z;
            r[4 * q + 3] = v.w;
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
    unsigned long long *gp = gfix + (size_t)slot * 1536;
    for (int q = tid; q < 3 * 512; q += 1024) {
      const unsigned long long v = (&s_acc[0][0])[q];
      if (v != 0ull) atomicAdd(&gp[q], v);
    }
    __syncthreads();
  }
}

// Block reduction of 8 floats over 1024 threads.
__device__ inline void block_sum8(float v[8], float *smem /* [16][8] */) {
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
