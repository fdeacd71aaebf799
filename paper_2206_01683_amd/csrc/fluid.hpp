// Lattice Boltzmann kernels: the fused pull-stream + collide step and the
// state conversion kernels.
//
// State layout: two buffers of 27 populations per cell (planes or rows, see
// GridArgs), x fastest. A buffer holds the post-collision values f*(x, n-1),
// stored as deviations f* - w_i; the pre-collision state of step n is the
// pull f_i(x, n) = f*_i(x - c_i, n-1). One step reads the current buffer and
// writes the other.
#pragma once

#include "env.hpp"

namespace lbmib {

// Pull the 27 pre-collision populations of node (xs, y, z): f_i with
// DEV = false, the deviations h_i = f_i - w_i with DEV = true. The x
// neighbour indices xm/xp are given by the caller (periodic wrap or interior
// node). Offsets are 64-bit (27 populations of a large lattice pass 2^32
// elements).
template <class S, bool DEV = false, class P>
__device__ inline void pull27(P src, const GridArgs &g, int xm, int xs, int xp, int ym, int y, int yp, int zm, int z,
                              int zp, float f[Q]) {
  const int xx[3] = {xp, xs, xm};  // indexed by cx + 1: source x = xs - cx
  const int yy[3] = {yp, y, ym};
  const int zz[3] = {zp, z, zm};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const uint32_t row = (uint32_t)zz[cz_of(i) + 1] * (uint32_t)g.ny + (uint32_t)yy[cy_of(i) + 1];
    const size_t at = pop_idx(g, i, row, (uint32_t)xx[cx_of(i) + 1]);
    f[i] = DEV ? S::load_dev(src + at, i) : S::load(src + at, i);
  }
}

__device__ inline void moments(const float f[Q], float &rho, float &mx, float &my, float &mz) {
  rho = 0.f;
  mx = my = mz = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    rho += f[i];
    if (cx_of(i) == 1) mx += f[i];
    if (cx_of(i) == -1) mx -= f[i];
    if (cy_of(i) == 1) my += f[i];
    if (cy_of(i) == -1) my -= f[i];
    if (cz_of(i) == 1) mz += f[i];
    if (cz_of(i) == -1) mz -= f[i];
  }
}

__device__ inline float cdot(int i, float ax, float ay, float az) {
  float r = 0.f;
  if (cx_of(i) == 1) r += ax;
  if (cx_of(i) == -1) r -= ax;
  if (cy_of(i) == 1) r += ay;
  if (cy_of(i) == -1) r -= ay;
  if (cz_of(i) == 1) r += az;
  if (cz_of(i) == -1) r -= az;
  return r;
}

// Immersed force is kept as 64-bit fixed point with 2^-40 resolution (see
// the spreading kernel): contributions are summed as integers, so the result
// does not depend on summation order.
// float -> nearest multiple of 2^-40, as two's complement: adding 1.5 * 2^52
// to the scaled value in double precision leaves the rounded integer in the
// low mantissa bits (valid for |v| < 2^11).
__device__ inline unsigned long long to_fix(float v) {
  const double magic = 6755399441055744.0;  // 1.5 * 2^52
  const double d = (double)v * 1099511627776.0 + magic;
  return (unsigned long long)(__double_as_longlong(d) - __double_as_longlong(magic));
}
__device__ inline float from_fix(unsigned long long q) {
  return (float)((double)(long long)q * (1.0 / 1099511627776.0));
}

// Immersed-boundary force density at cell (x, y, z): zero outside active tiles.
__device__ inline void load_g(const GridArgs &g, const int *__restrict__ tile_slot,
                              const unsigned long long *__restrict__ gfix, int x, int y, int z, float &gx, float &gy,
                              float &gz) {
  gx = gy = gz = 0.f;
  if (tile_slot == nullptr) return;
  int t = (x >> 3) + g.tnx * ((y >> 3) + g.tny * (z >> 3));
  int s = ((const gmem<int> *)tile_slot)[t];
  if (s >= 0) {
    int lc = (x & 7) | ((y & 7) << 3) | ((z & 7) << 6);
    const gmem<unsigned long long> *gp = (const gmem<unsigned long long> *)gfix + (size_t)s * 1536;
    gx = from_fix(gp[lc]);
    gy = from_fix(gp[512 + lc]);
    gz = from_fix(gp[1024 + lc]);
  }
}

// One lattice Boltzmann step for every node:
//   interior node: f*_i = f_i - (f_i - f^eq_i(rho,u))/tau + (1 - 1/(2tau)) w_i
//                  [3(c_i - u) + 9 (c_i.u) c_i].F,  u = (m + F/2)/rho,
//                  F = g + rho a_ni(x, u)  (Eq. (3), solved exactly)
//   open-face node x_b with inward neighbour x_f (same y, z):
//                  f*_i(x_b) = f^eq_i(rho_f, u_b) + (1 - 1/tau)(f_i(x_f) - f^eq_i(rho_f, u_f))
//                  + (1 - 1/(2tau)) w_i [3(c_i - u_b) + 9 (c_i.u_b) c_i].F_b,
//                  u_f the forced velocity at x_f, u_b the face velocity
//                  (velocity face) or u_f (outflow), F_b = rho_f a_ni(x_b, u_b).
// The open-face lanes reuse the interior arithmetic: replacing f_i by
// f_i + f^eq_i(rho_f, u_b) - f^eq_i(rho_f, u_f) makes the BGK formula with
// (rho_f, u_b, F_b) produce exactly the extrapolated values.
//
// A cell of the collide and, for a boundary lane, the inward neighbour
// (xs, ys, zs) whose populations it reads.
struct CellAt {
  int x, y, z, xs, ys, zs;
};

// Cell (x, y, z) and, on an open face, the inward neighbour whose
// populations it reads (its source node). YZ: y or z may have open faces
// (otherwise both are periodic).
template <bool XPER, bool YZ = false>
__device__ inline CellAt cell_at(const GridArgs &g, int x, int y, int z) {
  CellAt c;
  c.x = x;
  c.y = y;
  c.z = z;
  c.xs = XPER ? x : (x == 0 ? 1 : (x == g.nx - 1 ? g.nx - 2 : x));
  c.ys = (YZ && !g.yper) ? (y == 0 ? 1 : (y == g.ny - 1 ? g.ny - 2 : y)) : y;
  c.zs = (YZ && !g.zper) ? (z == 0 ? 1 : (z == g.nz - 1 ? g.nz - 2 : z)) : z;
  return c;
}

// The 27 populations pulled to the source node of c.
template <class S, bool XPER, bool YZ = false>
__device__ inline void collide_pull(const EnvView &e, int cur, const CellAt &c, float f[Q]) {
  using T = typename S::T;
  const gmem<T> *__restrict__ src = (const gmem<T> *)e.f[cur];
  const GridArgs &g = e.g;
  const int xs = c.xs, y = c.y, z = c.z;
  int xm, xp;
  if (XPER) {
    xm = xs == 0 ? g.nx - 1 : xs - 1;
    xp = xs == g.nx - 1 ? 0 : xs + 1;
  } else {
    xm = xs - 1;
    xp = xs + 1;
  }
  int ys = y, zs = z, ym, yp, zm, zp;
  if (YZ && !g.yper) {
    ys = c.ys;
    ym = ys - 1;
    yp = ys + 1;
  } else {
    ym = y == 0 ? g.ny - 1 : y - 1;
    yp = y == g.ny - 1 ? 0 : y + 1;
  }
  if (YZ && !g.zper) {
    zs = c.zs;
    zm = zs - 1;
    zp = zs + 1;
  } else {
    zm = z == 0 ? g.nz - 1 : z - 1;
    zp = z == g.nz - 1 ? 0 : z + 1;
  }
  pull27<S, true>(src, g, xm, xs, xp, ym, ys, yp, zm, zs, zp, f);
}

// First half of collide_cell: locate the cell and pull its 27 populations
// (for a boundary lane, those of its inward neighbour). False past the
// lattice.
template <class S, bool XPER, bool YZ = false>
__device__ inline bool collide_load(const EnvView &e, int cur, int lb, int tx, int ty, CellAt &c, float f[Q]) {
  int x, y, z;
  if (!cell_of(e, lb, tx, ty, x, y, z)) return false;
  c = cell_at<XPER, YZ>(e.g, x, y, z);
  collide_pull<S, XPER, YZ>(e, cur, c, f);
  return true;
}

// Second half: moments, forcing, BGK + Guo (or the open-face extrapolation)
// and the 27 stores of f*(n). TRT: the two-relaxation-time collision instead
// of BGK (even and odd parts of f relax at omega+ and omega-, Guo's source
// split the same way).
template <class S, bool XPER, bool ROT, bool YZ = false, bool TRT = false>
__device__ inline void collide_finish(const EnvView &e, const FrameF &fr, int cur, const CellAt &c, float f[Q]) {
  // multiply-adds fused within a source expression only, so that this
  // arithmetic rounds the same way in every kernel it is inlined into (the
  // single-lattice, batched and persistent collides give the same bits)
#pragma clang fp contract(on)
  using T = typename S::T;
  gmem<T> *__restrict__ dst = (gmem<T> *)e.f[cur ^ 1];
  const int *__restrict__ tile_slot = e.ib ? e.tile_slot : nullptr;
  const GridArgs &g = e.g;
  const int x = c.x, y = c.y, z = c.z, xs = c.xs;
  const int ys = YZ ? c.ys : y, zs = YZ ? c.zs : z;
  const bool lo_face = !XPER && x == 0;
  const bool face = (!XPER && (x == 0 || x == g.nx - 1)) || (YZ && (ys != y || zs != z));
  // f holds the deviations h_i = f_i - w_i: sum h = rho - 1, sum h c = m
  float drho, mx, my, mz;
  moments(f, drho, mx, my, mz);
  const float rho = 1.0f + drho;
  const float irho = 1.0f / rho;

  float gx, gy, gz;
  load_g(g, tile_slot, e.gfix, xs, ys, zs, gx, gy, gz);
  float ax, ay, az;
  frame_a0<ROT>(fr, (float)xs, (float)ys, (float)zs, ax, ay, az);
  float ux, uy, uz;
  solve_coriolis<ROT>(fr, mx * irho + 0.5f * (gx * irho + ax), my * irho + 0.5f * (gy * irho + ay),
                      mz * irho + 0.5f * (gz * irho + az), ux, uy, uz);
  float Fx, Fy, Fz;
  if (!face) {
    float wx = 0.f, wy = 0.f, wz = 0.f;
    if (ROT) cross3(fr.omg, ux, uy, uz, wx, wy, wz);
    Fx = gx + rho * (ax - 2.0f * wx);
    Fy = gy + rho * (ay - 2.0f * wy);
    Fz = gz + rho * (az - 2.0f * wz);
  } else {
    // (ux,uy,uz) is u_f; choose u_b and shift f by f^eq(u_b) - f^eq(u_f).
    // The inlet velocity is picked by value (fr.uhi or fr.ulo), never through
    // a pointer into fr: where fr is a local, that would put it in scratch.
    int bc;
    bool use_hi;
    if (!YZ) {
      bc = lo_face ? g.bc_lo : g.bc_hi;
      use_hi = !lo_face;
    } else {
      // first velocity face of this node: x low, x high, y low, y high, z low, z high
      bc = 2;
      use_hi = false;
      if (!XPER && x != xs && (x == 0 ? g.bc_lo : g.bc_hi) == 1) {
        bc = 1;
        use_hi = x != 0;
      } else if ((ys != y && (y == 0 ? g.bc_y[0] : g.bc_y[1]) == 1) ||
                 (zs != z && (z == 0 ? g.bc_z[0] : g.bc_z[1]) == 1)) {
        bc = 1;
      }
    }
    const float ufx = use_hi ? fr.uhi[0] : fr.ulo[0], ufy = use_hi ? fr.uhi[1] : fr.ulo[1],
                ufz = use_hi ? fr.uhi[2] : fr.ulo[2];
    float bx = bc == 1 ? ufx : ux, by = bc == 1 ? ufy : uy, bz = bc == 1 ? ufz : uz;
    const float ub2 = bx * bx + by * by + bz * bz, uf2 = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const float cb = cdot(i, bx, by, bz), cf = cdot(i, ux, uy, uz);
      f[i] += w_of(i) * rho * (3.0f * (cb - cf) + 4.5f * (cb * cb - cf * cf) - 1.5f * (ub2 - uf2));
    }
    float ax2, ay2, az2;
    frame_a0<ROT>(fr, (float)x, (float)y, (float)z, ax2, ay2, az2);
    float wx = 0.f, wy = 0.f, wz = 0.f;
    if (ROT) cross3(fr.omg, bx, by, bz, wx, wy, wz);
    ux = bx;
    uy = by;
    uz = bz;
    Fx = rho * (ax2 - 2.0f * wx);
    Fy = rho * (ay2 - 2.0f * wy);
    Fz = rho * (az2 - 2.0f * wz);
  }

  const float u2 = ux * ux + uy * uy + uz * uz;
  if (!(u2 < 0.16f)) atomicOr(e.guard, (int)GUARD_UNSTABLE);

  // BGK + Guo on the deviations, evaluated on opposite pairs (i, 26 - i):
  // c_j = -c_i, so the equilibrium and forcing split into parts even and odd
  // in c. h*_i = h_i - (h_i - heq_i)/tau + S_i with
  // heq_i = f^eq_i - w_i = w_i [(rho - 1) + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u^2)].
  const float Ah = -1.5f * u2;
  const float uF = ux * Fx + uy * Fy + uz * Fz;
  gmem<T> *__restrict__ d = dst + pop_idx(g, 0, (uint32_t)z * (uint32_t)g.ny + (uint32_t)y, (uint32_t)x);
  if constexpr (!TRT) {
    const float E = e.inv_tau * rho;
    const float B = e.inv_tau * drho;
    const float P = e.pref;
#pragma unroll
    for (int i = 0; i < 13; ++i) {
      const int j = 26 - i;
      const float w = w_of(i);
      const float cu = cdot(i, ux, uy, uz);
      const float cF = cdot(i, Fx, Fy, Fz);
      const float even = w * (E * (Ah + 4.5f * cu * cu) + B) + (w * P) * (9.0f * cu * cF - 3.0f * uF);
      const float odd = (w * E) * (3.0f * cu) + (w * P) * (3.0f * cF);
      S::store_dev(d + (size_t)i * g.ps, e.omt * f[i] + even + odd, i);
      S::store_dev(d + (size_t)j * g.ps, e.omt * f[j] + even - odd, j);
    }
    {
      const float w = w_of(13);
      S::store_dev(d + (size_t)13 * g.ps, e.omt * f[13] + w * (E * Ah + B) - (w * P) * 3.0f * uF, 13);
    }
  } else {
    // h*_i = h_i - w+ (h+_i - heq+_i) - w- (h-_i - heq-_i) + (1 - w+/2) S+_i + (1 - w-/2) S-_i
    //      = a h_i + b h_j + [w+ heq+_i + (1 - w+/2) S+_i] + [w- heq-_i + (1 - w-/2) S-_i],
    // a = 1 - (w+ + w-)/2, b = (w- - w+)/2; the bracketed parts are even and
    // odd in c, as in BGK with its single rate split in two.
    const float Ep = e.trt.wp * rho, Em = e.trt.wm * rho, Bp = e.trt.wp * drho;
    const float Pp = e.trt.pp, Pm = e.trt.pm, a = e.trt.a, b = e.trt.b;
#pragma unroll
    for (int i = 0; i < 13; ++i) {
      const int j = 26 - i;
      const float w = w_of(i);
      const float cu = cdot(i, ux, uy, uz);
      const float cF = cdot(i, Fx, Fy, Fz);
      const float even = w * (Ep * (Ah + 4.5f * cu * cu) + Bp) + (w * Pp) * (9.0f * cu * cF - 3.0f * uF);
      const float odd = (w * Em) * (3.0f * cu) + (w * Pm) * (3.0f * cF);
      S::store_dev(d + (size_t)i * g.ps, a * f[i] + b * f[j] + even + odd, i);
      S::store_dev(d + (size_t)j * g.ps, a * f[j] + b * f[i] + even - odd, j);
    }
    {
      const float w = w_of(13);
      S::store_dev(d + (size_t)13 * g.ps, (1.0f - e.trt.wp) * f[13] + w * (Ep * Ah + Bp) - (w * Pp) * 3.0f * uF,
                   13);
    }
  }
}

// One cell of logical block lb (tile shape e.bx x e.by, see cell_of), thread
// (tx, ty); `cur` is the buffer holding f*(n-1), the other one receives f*(n).
template <class S, bool XPER, bool ROT, bool YZ = false, bool TRT = false>
__device__ inline void collide_cell(const EnvView &e, const FrameF &fr, int cur, int lb, int tx, int ty) {
  CellAt c;
  float f[Q];
  if (collide_load<S, XPER, YZ>(e, cur, lb, tx, ty, c, f)) collide_finish<S, XPER, ROT, YZ, TRT>(e, fr, cur, c, f);
}

// Single-lattice launch: blockDim = (e.bx, e.by), logical block = hardware
// workgroup index. (Mapping blocks so that each XCD, which takes workgroups
// b with b % 8 equal, sweeps a contiguous eighth of the domain measured 3%
// slower on the fish: consecutive workgroups then share no lines in L2, and
// interleaving them over the XCDs spreads each plane's traffic evenly.)
template <class S, bool XPER, bool ROT, bool YZ = false, bool TRT = false>
__global__ void __launch_bounds__(512) k_collide(EnvView e, FrameF fr, int cur) {
  const int lb = blockIdx.x;
  if (lb >= e.nblocks) return;
  collide_cell<S, XPER, ROT, YZ, TRT>(e, fr, cur, lb, threadIdx.x, threadIdx.y);
}

// f_i(x) of the caller's canonical pre-collision field -> stored buffer, i.e.
// stored_i(x) = f_i(x + c_i) - w_i (periodic wrap; clamped at open faces,
// where the value is never read).
template <class S>
__global__ void k_load_canonical(const float *__restrict__ fin, typename S::T *__restrict__ dst, GridArgs g) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx) return;
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  for (int i = 0; i < Q; ++i) {
    int sx = x + cx_of(i), sy = wrap_idx(y + cy_of(i), g.ny), sz = wrap_idx(z + cz_of(i), g.nz);
    sx = g.xper ? wrap_idx(sx, g.nx) : min(max(sx, 0), g.nx - 1);
    float v = fin[(size_t)i * n + ((size_t)sz * g.ny + sy) * g.nx + sx];
    S::store_plain(dst + pop_idx(g, i, (uint32_t)z * g.ny + y, x), v, i);
  }
}

// Equilibrium state f_i(x) = f^eq_i(rho0(x), u0(x)) written pre-shifted (and as
// deviations) as above.
template <class S>
__global__ void k_init_equilibrium(const float *__restrict__ rho0, const float *__restrict__ u0,
                                   typename S::T *__restrict__ dst, GridArgs g) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx) return;
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  for (int i = 0; i < Q; ++i) {
    int sx = x + cx_of(i), sy = wrap_idx(y + cy_of(i), g.ny), sz = wrap_idx(z + cz_of(i), g.nz);
    sx = g.xper ? wrap_idx(sx, g.nx) : min(max(sx, 0), g.nx - 1);
    size_t s = ((size_t)sz * g.ny + sy) * g.nx + sx;
    float r = rho0 ? rho0[s] : 1.0f;
    float ux = u0 ? u0[s] : 0.f, uy = u0 ? u0[n + s] : 0.f, uz = u0 ? u0[2 * n + s] : 0.f;
    float cu = cdot(i, ux, uy, uz);
    float v = w_of(i) * r * (1.0f + 3.0f * cu + 4.5f * cu * cu - 1.5f * (ux * ux + uy * uy + uz * uz));
    S::store_plain(dst + pop_idx(g, i, (uint32_t)z * g.ny + y, x), v, i);
  }
}

// Stored buffer -> canonical pre-collision populations (pull with wrap/clamp).
template <class S>
__global__ void k_read_canonical(const typename S::T *__restrict__ src, float *__restrict__ fout, GridArgs g) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx) return;
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  for (int i = 0; i < Q; ++i) {
    int sx = x - cx_of(i), sy = wrap_idx(y - cy_of(i), g.ny), sz = wrap_idx(z - cz_of(i), g.nz);
    sx = g.xper ? wrap_idx(sx, g.nx) : min(max(sx, 0), g.nx - 1);
    fout[(size_t)i * n + ((size_t)z * g.ny + y) * g.nx + x] =
        S::load(src + pop_idx(g, i, (uint32_t)sz * g.ny + sy, sx), i);
  }
}

// Density and frame-forced velocity (no immersed-boundary force) of the
// pre-collision state at every node.
template <class S, bool ROT>
__global__ void k_macros(const typename S::T *__restrict__ src, GridArgs g, FrameF fr, float *__restrict__ rho_out,
                         float *__restrict__ u_out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx) return;
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  int xm = x - 1, xp = x + 1;
  if (g.xper) {
    xm = wrap_idx(xm, g.nx);
    xp = wrap_idx(xp, g.nx);
  } else {
    xm = max(xm, 0);
    xp = min(xp, g.nx - 1);
  }
  float f[Q];  // deviations h_i
  pull27<S, true>(src, g, xm, x, xp, wrap_idx(y - 1, g.ny), y, wrap_idx(y + 1, g.ny),
                  wrap_idx(z - 1, g.nz), z, wrap_idx(z + 1, g.nz), f);
  float drho, mx, my, mz;
  moments(f, drho, mx, my, mz);
  const float rho = 1.0f + drho;
  float ax, ay, az;
  frame_a0<ROT>(fr, (float)x, (float)y, (float)z, ax, ay, az);
  float ux, uy, uz;
  solve_coriolis<ROT>(fr, mx / rho + 0.5f * ax, my / rho + 0.5f * ay, mz / rho + 0.5f * az, ux, uy, uz);
  size_t id = ((size_t)z * g.ny + y) * g.nx + x;
  if (rho_out) rho_out[id] = rho;
  if (u_out) {
    u_out[id] = ux;
    u_out[n + id] = uy;
    u_out[2 * n + id] = uz;
  }
}

}  // namespace lbmib
