// Immersed-boundary kernels: skinning, tile binning, interpolation with direct
// forcing, gather-form spreading and the body wrench.
//
// The immersed force lives only in "active" 8x8x8 tiles: tiles that some
// marker's 4x4x4 Peskin stencil touches. Each step rebuilds the active set:
//   k_skin_count    skin markers (linear blend skinning), wrap/check range,
//                   count markers per touched tile
//   k_tile_scan     one workgroup: tile counts -> slots, list offsets; clears
//                   the counts for the next step
//   k_fill_macro    per active tile: ordered list of its markers (increasing
//                   marker index, so spreading is deterministic) and the
//                   density and unforced velocity of its 512 cells
//   k_interp        one wave64 per marker, one lane per stencil node: weights,
//                   wave-level sums -> U*_k, rho_k, direct forcing F_k
//   k_spread        per active tile, one wave per 4x4x4 octant, marker records
//                   staged in LDS: g(x) = sum_k F_k dV_k delta(x - X_k) with no
//                   global atomics
//   k_wrench        one workgroup: force, torque, power of the fluid on the body
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

// Linear blend skinning, domain handling and tile counting (one thread per marker).
// Periodic axes: X is wrapped into [0, n). Open x: markers must satisfy
// 2 <= X < nx - 3 so the stencil stays on nodes 1 .. nx-2; others raise the
// range guard and are clamped so that every access stays in bounds.
__global__ void k_skin_count(const float *__restrict__ xrest, const int *__restrict__ bone,
                             const float *__restrict__ weight, const float *__restrict__ pose, float *__restrict__ X,
                             float *__restrict__ U, int *__restrict__ tile_count, IBArgs a, int *__restrict__ guard) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = a.n;
  if (k >= n) return;
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
  int tx[3], ty[3], tz[3];
  const int nxt = axis_tiles(stencil_base(p[0]), a.g.nx, a.g.xper, tx);
  const int nyt = axis_tiles(stencil_base(p[1]), a.g.ny, true, ty);
  const int nzt = axis_tiles(stencil_base(p[2]), a.g.nz, true, tz);
  for (int i = 0; i < nzt; ++i)
    for (int j = 0; j < nyt; ++j)
      for (int l = 0; l < nxt; ++l) atomicAdd(&tile_count[tx[l] + a.g.tnx * (ty[j] + a.g.tny * tz[i])], 1);
}

// Single workgroup: exclusive scans of (count > 0) and count over all tiles.
// counters[0] = number of active tiles (capped), counters[1] = list entries.
__global__ void __launch_bounds__(1024) k_tile_scan(int *__restrict__ tile_count, int *__restrict__ tile_slot,
                                                    int *__restrict__ active, int *__restrict__ tile_off,
                                                    int *__restrict__ tile_len, int *__restrict__ counters,
                                                    int ntiles, int cap, int *__restrict__ guard) {
  __shared__ int s_act[1024];
  __shared__ int s_sum[1024];
  const int tid = threadIdx.x;
  const int chunk = (ntiles + 1023) / 1024;
  const int t0 = min(tid * chunk, ntiles), t1 = min(t0 + chunk, ntiles);
  int act = 0, sum = 0;
  for (int t = t0; t < t1; ++t) {
    int c = tile_count[t];
    act += c > 0;
    sum += c;
  }
  s_act[tid] = act;
  s_sum[tid] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int va = tid >= off ? s_act[tid - off] : 0;
    int vs = tid >= off ? s_sum[tid - off] : 0;
    __syncthreads();
    s_act[tid] += va;
    s_sum[tid] += vs;
    __syncthreads();
  }
  int slot = s_act[tid] - act, pos = s_sum[tid] - sum;
  bool over = false;
  for (int t = t0; t < t1; ++t) {
    int c = tile_count[t];
    if (c > 0) {
      if (slot < cap) {
        tile_slot[t] = slot;
        active[slot] = t;
        tile_off[slot] = pos;
        tile_len[slot] = c;
      } else {
        tile_slot[t] = -1;
        over = true;
      }
      ++slot;
      pos += c;
    } else {
      tile_slot[t] = -1;
    }
    tile_count[t] = 0;
  }
  if (over) atomicOr(guard, (int)GUARD_CAPACITY);
  if (tid == 1023) {
    counters[0] = min(s_act[1023], cap);
    counters[1] = s_sum[1023];
  }
}

// Per active tile (grid-stride over slots, 512 threads = the tile's cells):
// (a) list of the markers touching the tile, in increasing marker index;
// (b) density and unforced velocity u* (frame force, no IB force) per cell.
template <class S, bool ROT>
__global__ void __launch_bounds__(512) k_fill_macro(const typename S::T *__restrict__ src, const float *__restrict__ X,
                                                    const int *__restrict__ active, const int *__restrict__ tile_off,
                                                    const int *__restrict__ tile_len, const int *__restrict__ counters,
                                                    int *__restrict__ pairs, float4 *__restrict__ macro, IBArgs a) {
  __shared__ int s_cnt[8];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n_active = counters[0];
  const GridArgs &g = a.g;
  for (int slot = blockIdx.x; slot < n_active; slot += gridDim.x) {
    const int t = active[slot];
    const int tx = t % g.tnx, ty = (t / g.tnx) % g.tny, tz = t / (g.tnx * g.tny);
    const int off = tile_off[slot], len = tile_len[slot];
    int running = 0;
    for (int base = 0; base < a.n; base += 512) {
      const int k = base + tid;
      bool hit = false;
      if (k < a.n) {
        hit = axis_touches(stencil_base(X[k]), g.nx, g.xper, tx) &&
              axis_touches(stencil_base(X[a.n + k]), g.ny, true, ty) &&
              axis_touches(stencil_base(X[2 * a.n + k]), g.nz, true, tz);
      }
      const unsigned long long bal = __ballot(hit);
      if (lane == 0) s_cnt[wv] = __popcll(bal);
      __syncthreads();
      int woff = 0, total = 0;
      for (int q = 0; q < 8; ++q) {
        woff += q < wv ? s_cnt[q] : 0;
        total += s_cnt[q];
      }
      const int pos = running + woff + __popcll(bal & ((1ull << lane) - 1ull));
      if (hit && pos < len) pairs[off + pos] = k;
      running += total;
      __syncthreads();
    }
    // cell of this thread
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
  }
}

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One wave64 per marker; lane l is stencil node (l & 3, (l >> 2) & 3, l >> 4).
// pass 0: U*_k = sum u* delta, rho_k = sum rho delta, F_k = 2 alpha rho_k (U_k - U*_k).
// pass p > 0 (multi-direct forcing): the interpolated velocity includes the
// current immersed force, u = u* + (I + [omega]x)^-1 g / (2 rho), and
// F_k += 2 alpha rho_k (U_k - U_k^interp).
template <bool ROT, bool MDF>
__global__ void __launch_bounds__(256) k_interp(const float *__restrict__ X, const float *__restrict__ U,
                                                const float *__restrict__ dv, float *__restrict__ F,
                                                float *__restrict__ mstate, float *__restrict__ rec,
                                                const int *__restrict__ tile_slot, const float4 *__restrict__ macro,
                                                const float *__restrict__ gbuf, IBArgs a, int *__restrict__ guard) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int n = a.n;
  if (k >= n) return;
  const GridArgs &g = a.g;
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
      const float *gp = gbuf + (size_t)s * 1536;
      const float h = 0.5f / rho;
      float dx, dy, dz;
      solve_coriolis<ROT>(a.fr, gp[lc] * h, gp[512 + lc] * h, gp[1024 + lc] * h, dx, dy, dz);
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
  if (lane < 4) r[lane] = w[0];                             // s3 = (lane, 0, 0)
  if ((lane & 3) == 0 && lane < 16) r[4 + (lane >> 2)] = w[1];  // s3 = (0, lane/4, 0)
  if ((lane & 15) == 0) r[8 + (lane >> 4)] = w[2];          // s3 = (0, 0, lane/16)
  if (lane == 0) {
    float rk;
    float Fk[3];
    const float Uk[3] = {U[k], U[n + k], U[2 * n + k]};
    const float Ui[3] = {sx, sy, sz};
    if (!MDF) {
      rk = sr;
      mstate[k] = rk;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        mstate[(c + 1) * (size_t)n + k] = Ui[c];
        Fk[c] = a.alpha2 * rk * (Uk[c] - Ui[c]);
      }
    } else {
      rk = mstate[k];
#pragma unroll
      for (int c = 0; c < 3; ++c) Fk[c] = F[c * n + k] + a.alpha2 * rk * (Uk[c] - Ui[c]);
    }
    const float dvk = dv[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      F[c * n + k] = Fk[c];
      r[16 + c] = Fk[c] * dvk;
      r[12 + c] = __int_as_float(base[c]);
    }
  }
}

// Per active tile (grid-stride over slots, 512 threads): wave w owns the
// 4x4x4 octant (w & 1, (w >> 1) & 1, w >> 2) of the tile, lane l one cell of
// it. The tile's marker list is staged through LDS in chunks; each wave keeps
// the markers whose stencil meets its octant (order preserved) and every lane
// accumulates its own cell's force in a register.
__global__ void __launch_bounds__(512) k_spread(const float *__restrict__ rec, const int *__restrict__ active,
                                                const int *__restrict__ tile_off, const int *__restrict__ tile_len,
                                                const int *__restrict__ counters, const int *__restrict__ pairs,
                                                float *__restrict__ gbuf, IBArgs a) {
  __shared__ float s_rec[512 * REC];
  __shared__ unsigned short s_idx[8][512];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const GridArgs &g = a.g;
  const int n_active = counters[0];
  for (int slot = blockIdx.x; slot < n_active; slot += gridDim.x) {
    const int t = active[slot];
    const int tx = t % g.tnx, ty = (t / g.tnx) % g.tny, tz = t / (g.tnx * g.tny);
    const int ox = tx * 8 + 4 * (wv & 1), oy = ty * 8 + 4 * ((wv >> 1) & 1), oz = tz * 8 + 4 * (wv >> 2);
    const int cx = ox + (lane & 3), cy = oy + ((lane >> 2) & 3), cz = oz + (lane >> 4);
    const int off = tile_off[slot], len = tile_len[slot];
    float gx = 0.f, gy = 0.f, gz = 0.f;
    for (int c0 = 0; c0 < len; c0 += 512) {
      const int m = min(512, len - c0);
      if (tid < m) {
        const float *src = rec + (size_t)pairs[off + c0 + tid] * REC;
#pragma unroll
        for (int q = 0; q < REC; ++q) s_rec[tid * REC + q] = src[q];
      }
      __syncthreads();
      // ordered filter of the chunk for this wave's octant
      int cnt = 0;
      for (int e0 = 0; e0 < m; e0 += 64) {
        const int e = e0 + lane;
        bool hit = false;
        if (e < m) {
          const float *r = s_rec + e * REC;
          const int bx = __float_as_int(r[12]), by = __float_as_int(r[13]), bz = __float_as_int(r[14]);
          int dx = wrap_idx(ox - bx, g.nx), dy = wrap_idx(oy - by, g.ny), dz = wrap_idx(oz - bz, g.nz);
          hit = (dx <= 3 || dx >= g.nx - 3) && (dy <= 3 || dy >= g.ny - 3) && (dz <= 3 || dz >= g.nz - 3);
        }
        const unsigned long long bal = __ballot(hit);
        if (hit) s_idx[wv][cnt + __popcll(bal & ((1ull << lane) - 1ull))] = (unsigned short)e;
        cnt += __popcll(bal);
      }
      __syncthreads();
      for (int q = 0; q < cnt; ++q) {
        const float *r = s_rec + s_idx[wv][q] * REC;
        int dx = wrap_idx(cx - __float_as_int(r[12]), g.nx);
        int dy = wrap_idx(cy - __float_as_int(r[13]), g.ny);
        int dz = wrap_idx(cz - __float_as_int(r[14]), g.nz);
        if (dx < 4 && dy < 4 && dz < 4) {
          const float d = r[dx] * r[4 + dy] * r[8 + dz];
          gx += r[16] * d;
          gy += r[17] * d;
          gz += r[18] * d;
        }
      }
      __syncthreads();
    }
    const int lc = (cx & 7) | ((cy & 7) << 3) | ((cz & 7) << 6);
    float *gp = gbuf + (size_t)slot * 1536;
    gp[lc] = gx;
    gp[512 + lc] = gy;
    gp[1024 + lc] = gz;
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
