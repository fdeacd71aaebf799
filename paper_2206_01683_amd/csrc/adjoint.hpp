// Discrete adjoint of one immersed-boundary lattice Boltzmann step (reverse
// mode of exactly the arithmetic of the forward step, float32 storage,
// explicit direct forcing, non-rotating frame).
//
// Forward step n (state A = post-collision populations of step n-1):
//   f = pull(A); rho, m per node; u* = m/rho + a0/2 (a0 = -frame acceleration)
//   markers: X, U from the pose; rho_k = sum W rho, U*_k = sum W u*,
//   F_k = 2 alpha rho_k (U_k - U*_k), g = sum_k W F_k dV_k  (W = Peskin weights)
//   interior: u = (m + g/2)/rho + a0/2, F = g + rho a0,
//             f*_i = (1-1/tau) f_i + f^eq_i(rho,u)/tau + S_i(u, F)
//   open faces: f*_i(x_b) = f^eq_i(rho_f,u_b) + (1-1/tau)(f_i(x_f) - f^eq_i(rho_f,u_f)) + S_i(u_b, rho_f a0)
//   A' = f*; per-step objective J_n = wF . F_body + wP P with F_body = -sum F_k dV_k,
//   P = sum F_k . U_k dV_k.
// Given lam' = dJ/dA' this computes lam = dJ/dA (for the part of J from step
// n on) and the step's dJ/d(bone pose). Passes, with the forward IB data of
// step n recomputed beforehand (skin, tiles, band macros, interpolation,
// spreading):
//   1 k_adj_gbar      gbar = dJ/dg on active-tile cells (collide + face adjoint);
//                     the open faces' density and momentum adjoints at x_f
//   2 k_adj_markers   per marker: Fbar, rhobar_k, U*bar_k, Ubar_k, Xbar_k
//                     (Xbar includes the derivative of the Peskin weights)
//   3 k_adj_spread    spread (rhobar_k, U*bar_k) onto the band in 64-bit fixed
//                     point (order-independent)
//   4 k_adj_collide   every cell: fbar from the collide adjoint and the band
//                     IB terms, push-streamed into lam (324 B per cell);
//                     the x_f lanes add the open faces' extrapolation adjoint
//   5 k_adj_pose_part per (bone, marker range, step): dJ/dR, dJ/dt, dJ/dRdot,
//     k_adj_pose_sum  dJ/dtdot partials, then their sum in a fixed order (per
//                     step, or once for all steps of a segment)
#pragma once

#include "ib.hpp"

namespace lbmib {

constexpr int kPoseSplit = 16;  // workgroups per bone in the pose adjoint

struct AdjArgs {
  float wF[3];                        // objective weight on the fluid force on the body
  float wP;                           // objective weight on the power
  float a0[3];                        // frame acceleration term a0 = -acc (uniform: no rotation)
  const float *__restrict__ lam_next;  // in the population layout (GridArgs)
  float *__restrict__ lam_prev;        // in the population layout
  float *__restrict__ gbar;            // [cap][3][512]
  unsigned long long *__restrict__ adjfix;  // [cap][4][512]: spread rhobar, U*bar (fixed point)
  float *__restrict__ mbar;            // [6][n]: Xbar (3), Ubar (3)
  float *__restrict__ facebuf;         // [2][4][ny*nz]: open faces' rhobar, mbar (3) at x_f
  float bc_u_lo[3], bc_u_hi[3];        // face velocities
};

// d phi / d r of Peskin's 4-point kernel
__device__ inline float peskin4_d(float r) {
  const float a = fabsf(r);
  float d = 0.f;
  if (a <= 1.0f) {
    const float s = __builtin_sqrtf(fmaxf(1.0f + 4.0f * a - 4.0f * a * a, 1e-30f));
    d = 0.125f * (-2.0f + (2.0f - 4.0f * a) / s);
  } else if (a <= 2.0f) {
    const float s = __builtin_sqrtf(fmaxf(-7.0f + 12.0f * a - 4.0f * a * a, 1e-30f));
    d = 0.125f * (-2.0f - (6.0f - 4.0f * a) / s);
  }
  return r < 0.f ? -d : d;
}

// Moments of lam weighted with w_i, used by the BGK + Guo adjoints:
// S0 = sum l w, S1 = sum l w c, S2 = sum l w (c.u) c, Scu = sum l w (c.u),
// Scu2 = sum l w (c.u)^2, SF = sum l w (c.F) c.
struct LamSums {
  float S0, S1[3], S2[3], Scu, Scu2, SF[3];
};

__device__ inline LamSums lam_sums(const float lam[Q], float ux, float uy, float uz, float Fx, float Fy, float Fz) {
  LamSums s{};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float lw = lam[i] * w_of(i);
    const float cu = cdot(i, ux, uy, uz), cF = cdot(i, Fx, Fy, Fz);
    const int c[3] = {cx_of(i), cy_of(i), cz_of(i)};
    s.S0 += lw;
    s.Scu += lw * cu;
    s.Scu2 += lw * cu * cu;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (c[a] != 0) {
        const float sg = (float)c[a];
        s.S1[a] += sg * lw;
        s.S2[a] += sg * lw * cu;
        s.SF[a] += sg * lw * cF;
      }
    }
  }
  return s;
}

// Adjoint of the interior BGK + Guo collision at one node with pre-collision
// f (moments rho, m), force g and lam = dJ/df*. Returns rhobar, mbar (the
// parts that reach f through rho and m: fbar_j += rhobar + c_j . mbar) and
// gbar; the direct part (1 - 1/tau) lam_j is added by the caller.
__device__ inline void adj_collide_node(const float lam[Q], float rho, const float m[3], const float g[3],
                                       const AdjArgs &A, float inv_tau, float pref, float &rhobar, float mbar[3],
                                       float gbar[3]) {
  const float ir = 1.0f / rho;
  float u[3], F[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u[a] = m[a] * ir + 0.5f * (g[a] * ir + A.a0[a]);
    F[a] = g[a] + rho * A.a0[a];
  }
  const float u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const LamSums s = lam_sums(lam, u[0], u[1], u[2], F[0], F[1], F[2]);
  rhobar = inv_tau * (s.S0 * (1.0f - 1.5f * u2) + 3.0f * s.Scu + 4.5f * s.Scu2);
  float ub[3], Fb[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ub[a] = inv_tau * rho * (3.0f * s.S1[a] + 9.0f * s.S2[a] - 3.0f * u[a] * s.S0) +
            pref * (-3.0f * F[a] * s.S0 + 9.0f * s.SF[a]);
    Fb[a] = pref * (3.0f * s.S1[a] - 3.0f * u[a] * s.S0 + 9.0f * s.S2[a]);
  }
  float q = 0.f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    gbar[a] = Fb[a] + 0.5f * ir * ub[a];
    rhobar += Fb[a] * A.a0[a];
    q += ub[a] * (m[a] + 0.5f * g[a]);
    mbar[a] = ub[a] * ir;
  }
  rhobar -= q * ir * ir;
}

// Adjoint of a face node's extrapolation, seen from its inward neighbour x_f
// (moments rho, m, force g at x_f): lam_b = dJ/df*(x_b). Returns the parts of
// fbar(x_f): direct (1 - 1/tau) lam_b is added by the caller, plus rhobar,
// mbar, and gbar(x_f).
__device__ inline void adj_face(const float lamb[Q], float rho, const float m[3], const float g[3],
                                const float ubc[3], bool velocity_face, const AdjArgs &A, float omt, float pref,
                                float &rhobar, float mbar[3], float gbar[3]) {
  const float ir = 1.0f / rho;
  float uf[3], ub[3], Fbd[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    uf[a] = m[a] * ir + 0.5f * (g[a] * ir + A.a0[a]);
    ub[a] = velocity_face ? ubc[a] : uf[a];
    Fbd[a] = rho * A.a0[a];
  }
  const float ub2 = ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2];
  const float uf2 = uf[0] * uf[0] + uf[1] * uf[1] + uf[2] * uf[2];
  const LamSums sb = lam_sums(lamb, ub[0], ub[1], ub[2], Fbd[0], Fbd[1], Fbd[2]);
  const LamSums sf = lam_sums(lamb, uf[0], uf[1], uf[2], 0.f, 0.f, 0.f);
  rhobar = (sb.S0 * (1.0f - 1.5f * ub2) + 3.0f * sb.Scu + 4.5f * sb.Scu2) -
           omt * (sf.S0 * (1.0f - 1.5f * uf2) + 3.0f * sf.Scu + 4.5f * sf.Scu2);
  float ubb[3], ufb[3], Fbb[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Fbb[a] = pref * (3.0f * sb.S1[a] - 3.0f * ub[a] * sb.S0 + 9.0f * sb.S2[a]);
    ubb[a] = rho * (3.0f * sb.S1[a] + 9.0f * sb.S2[a] - 3.0f * ub[a] * sb.S0) +
             pref * (-3.0f * Fbd[a] * sb.S0 + 9.0f * sb.SF[a]);
    ufb[a] = -omt * rho * (3.0f * sf.S1[a] + 9.0f * sf.S2[a] - 3.0f * uf[a] * sf.S0);
    if (!velocity_face) ufb[a] += ubb[a];
    rhobar += Fbb[a] * A.a0[a];
  }
  float q = 0.f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    mbar[a] = ufb[a] * ir;
    gbar[a] = 0.5f * ir * ufb[a];
    q += ufb[a] * (m[a] + 0.5f * g[a]);
  }
  rhobar -= q * ir * ir;
}

// lam (in the population layout) of every direction at x in row `row`
__device__ inline void load_lam(const float *__restrict__ lam, const GridArgs &g, uint32_t row, int x, float l[Q]) {
  const float *__restrict__ p = lam + pop_idx(g, 0, row, (uint32_t)x);
#pragma unroll
  for (int i = 0; i < Q; ++i) l[i] = p[(size_t)i * g.ps];
}

// ------------------------------------------------------------------ pass 1 --
// gbar on the cells of active tile `slot` (state A in e.f[0]); clears the
// tile's fixed-point IB adjoint accumulator.
__device__ inline void adj_gbar_item(const EnvView &e, const AdjArgs &A, int slot, int tid) {
  const GridArgs &g = e.g;
  const float *__restrict__ src = static_cast<const float *>(e.f[0]);
  const int t = e.active[slot];
  const int tx = t % g.tnx, ty = (t / g.tnx) % g.tny, tz = t / (g.tnx * g.tny);
  const int x = tx * 8 + (tid & 7), y = ty * 8 + ((tid >> 3) & 7), z = tz * 8 + (tid >> 6);
  float gb[3] = {0.f, 0.f, 0.f};
  if (x < g.nx && y < g.ny && z < g.nz && (g.xper || (x > 0 && x < g.nx - 1))) {
    const int xm = g.xper ? wrap_idx(x - 1, g.nx) : x - 1;
    const int xp = g.xper ? wrap_idx(x + 1, g.nx) : x + 1;
    float f[Q];
    pull27<StoreF32>(src, g, xm, x, xp, wrap_idx(y - 1, g.ny), y, wrap_idx(y + 1, g.ny),
                     wrap_idx(z - 1, g.nz), z, wrap_idx(z + 1, g.nz), f);
    float rho, m[3];
    moments(f, rho, m[0], m[1], m[2]);
    float gg[3];
    load_g(g, e.tile_slot, e.gfix, x, y, z, gg[0], gg[1], gg[2]);
    const uint32_t row = (uint32_t)z * g.ny + y;
    float lam[Q];
    load_lam(A.lam_next, g, row, x, lam);
    float rb, mb[3];
    adj_collide_node(lam, rho, m, gg, A, e.inv_tau, e.pref, rb, mb, gb);
    if (!g.xper && (x == 1 || x == g.nx - 2)) {
      const bool lo = x == 1;
      load_lam(A.lam_next, g, row, lo ? 0 : g.nx - 1, lam);
      float rb2, mb2[3], gb2[3];
      adj_face(lam, rho, m, gg, lo ? A.bc_u_lo : A.bc_u_hi, (lo ? g.bc_lo : g.bc_hi) == 1, A, e.omt, e.pref, rb2,
               mb2, gb2);
      for (int a = 0; a < 3; ++a) gb[a] += gb2[a];
    }
  }
  float *gp = A.gbar + (size_t)slot * 1536;
  gp[tid] = gb[0];
  gp[512 + tid] = gb[1];
  gp[1024 + tid] = gb[2];
  unsigned long long *ap = A.adjfix + (size_t)slot * 2048;
  for (int q = 0; q < 4; ++q) ap[q * 512 + tid] = 0ull;
}

// ------------------------------------------------------------------ pass 2 --
// Markers 8*item .. 8*item+7, one wave64 each, lane = stencil node. The
// forward quantities of the step (X, U, F, rho_k, U*_k, band macros) are
// those of the recomputed forward IB phases.
__device__ inline void adj_marker_item(const EnvView &e, const AdjArgs &A, int item, int tid) {
  const int lane = tid & 63, wv = tid >> 6;
  const int k = item * kWavePer + wv;
  const int n = e.n;
  if (k >= n) return;
  const GridArgs &g = e.g;
  const float Xk[3] = {e.X[k], e.X[n + k], e.X[2 * n + k]};
  const int s3[3] = {lane & 3, (lane >> 2) & 3, lane >> 4};
  const int dims[3] = {g.nx, g.ny, g.nz};
  int base[3], node[3];
  float w[3], dw[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    base[ax] = stencil_base(Xk[ax]);
    const int j = base[ax] + s3[ax];
    w[ax] = peskin4(Xk[ax] - (float)j);
    dw[ax] = peskin4_d(Xk[ax] - (float)j);  // d/dX of phi(X - j)
    node[ax] = (ax > 0 || g.xper) ? wrap_idx(j, dims[ax]) : j;
  }
  const int t = (node[0] >> 3) + g.tnx * ((node[1] >> 3) + g.tny * (node[2] >> 3));
  const int s = e.tile_slot[t];
  float gb[3] = {0.f, 0.f, 0.f}, mac[4] = {1.f, 0.f, 0.f, 0.f};
  if (s >= 0) {
    const int lc = (node[0] & 7) | ((node[1] & 7) << 3) | ((node[2] & 7) << 6);
    const float *gp = A.gbar + (size_t)s * 1536;
    gb[0] = gp[lc];
    gb[1] = gp[512 + lc];
    gb[2] = gp[1024 + lc];
    const float4 mm = e.macro[(size_t)s * 512 + lc];
    mac[0] = mm.x;
    mac[1] = mm.y;
    mac[2] = mm.z;
    mac[3] = mm.w;
  }
  const float W = w[0] * w[1] * w[2];
  float G[3];
  for (int a = 0; a < 3; ++a) G[a] = wave_sum(W * gb[a]);
  const float dvk = e.dv[k], rk = e.mstate[k];
  float Fk[3], Uk[3], Us[3], Fb[3], Usb[3], Ub[3];
  float rkb = 0.f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Fk[a] = e.F[a * n + k];
    Uk[a] = e.U[a * n + k];
    Us[a] = e.mstate[(a + 1) * (size_t)n + k];
    Fb[a] = dvk * (G[a] - A.wF[a] + A.wP * Uk[a]);
    rkb += e.alpha2 * Fb[a] * (Uk[a] - Us[a]);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Usb[a] = -e.alpha2 * rk * Fb[a];
    Ub[a] = e.alpha2 * rk * Fb[a] + A.wP * Fk[a] * dvk;
  }
  // Xbar: sum over nodes of grad_X W times d(consumers of W)/dW
  const float c = dvk * (Fk[0] * gb[0] + Fk[1] * gb[1] + Fk[2] * gb[2]) + mac[0] * rkb +
                  mac[1] * Usb[0] + mac[2] * Usb[1] + mac[3] * Usb[2];
  const float gX = wave_sum(dw[0] * w[1] * w[2] * c);
  const float gY = wave_sum(w[0] * dw[1] * w[2] * c);
  const float gZ = wave_sum(w[0] * w[1] * dw[2] * c);
  float *r = e.rec + (size_t)k * REC;
  if (lane < 4) r[lane] = w[0];
  if ((lane & 3) == 0 && lane < 16) r[4 + (lane >> 2)] = w[1];
  if ((lane & 15) == 0) r[8 + (lane >> 4)] = w[2];
  if (lane == 0) {
    r[12] = __int_as_float(base[0]);
    r[13] = __int_as_float(base[1]);
    r[14] = __int_as_float(base[2]);
    r[15] = rkb;
    r[16] = Usb[0];
    r[17] = Usb[1];
    r[18] = Usb[2];
    A.mbar[k] = gX;
    A.mbar[n + k] = gY;
    A.mbar[2 * n + k] = gZ;
    A.mbar[3 * n + k] = Ub[0];
    A.mbar[4 * n + k] = Ub[1];
    A.mbar[5 * n + k] = Ub[2];
  }
}

// ------------------------------------------------------------------ pass 3 --
// Spreading of (rhobar_k, U*bar_k) onto active tile (slot, part), as
// spread_item but with four components from record slots 15..18.
__device__ inline void adj_spread_item(const EnvView &e, const AdjArgs &A, int item, int tid) {
  __shared__ unsigned long long s_acc[4][512];
  const int lane = tid & 63, wv = tid >> 6;
  const GridArgs &g = e.g;
  const int n = e.n;
  const int nchunks = (n + 63) >> 6;
  const int slot = item / kSpreadSplit, part = item % kSpreadSplit;
  const int t = e.active[slot];
  const int tx = t % g.tnx, ty = (t / g.tnx) % g.tny, tz = t / (g.tnx * g.tny);
  for (int q = tid; q < 4 * 512; q += WG) (&s_acc[0][0])[q] = 0ull;
  __syncthreads();
  const int stride = (WG / 64) * kSpreadSplit;
  const int c_first = part * (WG / 64) + wv;
  for (int it = 0; c_first + stride * 64 * it < nchunks; ++it) {
    const int cl = c_first + stride * (lane + 64 * it);
    bool pass = false;
    if (cl < nchunks) {
      const int4 box = e.chunk_box[cl];
      pass = box_hits(box.x, tx) && box_hits(box.y, ty) && box_hits(box.z, tz);
    }
    unsigned long long cbal = __ballot(pass);
    while (cbal) {
      const int jc = __ffsll((long long)cbal) - 1;
      cbal &= cbal - 1ull;
      const int k = (c_first + stride * (jc + 64 * it)) * 64 + lane;
      bool hit = false;
      if (k < n) {
        const short4 b = e.mbase[k];
        hit = axis_touches(b.x, g.nx, g.xper, tx) && axis_touches(b.y, g.ny, true, ty) &&
              axis_touches(b.z, g.nz, true, tz);
      }
      if (hit) {
        float r[20];
        const float4 *rp = reinterpret_cast<const float4 *>(e.rec + (size_t)k * REC);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const float4 v = rp[q];
          r[4 * q] = v.x;
          r[4 * q + 1] = v.y;
          r[4 * q + 2] = v.z;
          r[4 * q + 3] = v.w;
        }
        const int bx = __float_as_int(r[12]), by = __float_as_int(r[13]), bz = __float_as_int(r[14]);
        int lx[4], ly[4], lz[4];
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
#pragma unroll
              for (int cc = 0; cc < 4; ++cc) atomicAdd(&s_acc[cc][lc], to_fix(r[15 + cc] * d));
            }
          }
        }
      }
    }
  }
  __syncthreads();
  unsigned long long *ap = A.adjfix + (size_t)slot * 2048;
  for (int q = tid; q < 4 * 512; q += WG) {
    const unsigned long long v = (&s_acc[0][0])[q];
    if (v != 0ull) atomicAdd(&ap[q], v);
  }
  __syncthreads();
}

// ------------------------------------------------------------------ pass 4 --
// Every cell: fbar = (1 - 1/tau) lam + collide adjoint + the band IB terms,
// then push-streamed: lam_prev_i(x - c_i) = fbar_i(x). Open-face nodes have
// fbar = 0 and also clear the entries no node streams into (c_x pointing out
// of the domain). The face extrapolation's share of fbar(x_f) is added by the
// x_f lanes from pass 1's face results.
template <bool XPER>
__device__ inline void adj_collide_cell(const EnvView &e, const AdjArgs &A, int lb, int tx, int ty) {
  const GridArgs &g = e.g;
  const float *__restrict__ src = static_cast<const float *>(e.f[0]);
  int x, y, z;
  if (!cell_of(e, lb, tx, ty, x, y, z)) return;
  const int ym = y == 0 ? g.ny - 1 : y - 1;
  const int yp = y == g.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? g.nz - 1 : z - 1;
  const int zp = z == g.nz - 1 ? 0 : z + 1;
  const uint32_t row = (uint32_t)z * g.ny + y;
  float fb[Q];
  const bool face = !XPER && (x == 0 || x == g.nx - 1);
  if (face) {
#pragma unroll
    for (int i = 0; i < Q; ++i) fb[i] = 0.f;
  } else {
    int xm, xp;
    if (XPER) {
      xm = x == 0 ? g.nx - 1 : x - 1;
      xp = x == g.nx - 1 ? 0 : x + 1;
    } else {
      xm = x - 1;
      xp = x + 1;
    }
    float f[Q];
    pull27<StoreF32>(src, g, xm, x, xp, ym, y, yp, zm, z, zp, f);
    float rho, m[3];
    moments(f, rho, m[0], m[1], m[2]);
    float gg[3];
    load_g(g, e.ib ? e.tile_slot : nullptr, e.gfix, x, y, z, gg[0], gg[1], gg[2]);
    float lam[Q];
    load_lam(A.lam_next, g, row, x, lam);
    float rb, mb[3], gb[3];
    adj_collide_node(lam, rho, m, gg, A, e.inv_tau, e.pref, rb, mb, gb);
#pragma unroll
    for (int i = 0; i < Q; ++i) fb[i] = e.omt * lam[i];
    // immersed-boundary terms: rhobar, U*bar spread onto the band reach f
    // through u* = m/rho + a0/2 and rho
    if (e.ib) {
      const int t = (x >> 3) + g.tnx * ((y >> 3) + g.tny * (z >> 3));
      const int s = e.tile_slot[t];
      if (s >= 0) {
        const int lc = (x & 7) | ((y & 7) << 3) | ((z & 7) << 6);
        const unsigned long long *ap = A.adjfix + (size_t)s * 2048;
        const float rib = from_fix(ap[lc]);
        const float ub[3] = {from_fix(ap[512 + lc]), from_fix(ap[1024 + lc]), from_fix(ap[1536 + lc])};
        const float ir = 1.0f / rho;
        float q = 0.f;
        for (int a = 0; a < 3; ++a) {
          mb[a] += ub[a] * ir;
          q += ub[a] * m[a];
        }
        rb += rib - q * ir * ir;
      }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) fb[i] += rb + (float)cx_of(i) * mb[0] + (float)cy_of(i) * mb[1] + (float)cz_of(i) * mb[2];
    if (!XPER && (x == 1 || x == g.nx - 2)) {
      // the open face's extrapolation reads f(x_f): its adjoint (pass 1) plus
      // the direct part (1 - 1/tau) lam_b of the face node
      const int nyz = g.ny * g.nz, yz = z * g.ny + y;
      const bool lo = x == 1;
      const float *fp = A.facebuf + (size_t)(lo ? 0 : 1) * 4 * nyz;
      const float rF = fp[yz], m0 = fp[nyz + yz], m1 = fp[2 * nyz + yz], m2 = fp[3 * nyz + yz];
      const float *__restrict__ lb_ = A.lam_next + pop_idx(g, 0, (uint32_t)yz, lo ? 0 : g.nx - 1);
#pragma unroll
      for (int i = 0; i < Q; ++i)
        fb[i] += e.omt * lb_[(size_t)i * g.ps] + rF + (float)cx_of(i) * m0 + (float)cy_of(i) * m1 +
                 (float)cz_of(i) * m2;
    }
  }
  // push: lam_prev_i(x - c_i) = fbar_i(x)
  const int yy[3] = {yp, y, ym};  // indexed by c + 1: target y - c
  const int zz[3] = {zp, z, zm};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int tx_ = x - cx_of(i);
    if (XPER) {
      tx_ = tx_ < 0 ? tx_ + g.nx : (tx_ >= g.nx ? tx_ - g.nx : tx_);
    } else if (tx_ < 0 || tx_ >= g.nx) {
      continue;
    }
    const uint32_t trow = (uint32_t)zz[cz_of(i) + 1] * g.ny + yy[cy_of(i) + 1];
    __builtin_nontemporal_store(fb[i], A.lam_prev + pop_idx(g, i, trow, (uint32_t)tx_));
  }
  if (face) {
    // entries of this face node pulled by no node: c_x pointing out of the domain
    const int cxo = x == 0 ? -1 : 1;
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if (cx_of(i) == cxo) A.lam_prev[pop_idx(g, i, row, (uint32_t)x)] = 0.f;
  }
}

// Face extrapolation adjoint of face node `id` (side id / (ny nz): 0 is
// x = 0, 1 is x = nx-1), seen from its inward neighbour x_f: the parts of
// fbar(x_f) that go through x_f's density and momentum (rhobar, mbar), stored
// for the x_f lane of the collide adjoint, which adds them and the direct
// part (1 - 1/tau) lam_b to its own pushes.
__device__ inline void adj_face_item(const EnvView &e, const AdjArgs &A, int id) {
  const GridArgs &g = e.g;
  const int nyz = g.ny * g.nz;
  const int side = id / nyz, yz = id - side * nyz;
  const int y = yz % g.ny, z = yz / g.ny;
  const bool lo = side == 0;
  const int x = lo ? 1 : g.nx - 2;
  const float *__restrict__ src = static_cast<const float *>(e.f[0]);
  const int ym = y == 0 ? g.ny - 1 : y - 1;
  const int yp = y == g.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? g.nz - 1 : z - 1;
  const int zp = z == g.nz - 1 ? 0 : z + 1;
  float f[Q];
  pull27<StoreF32>(src, g, x - 1, x, x + 1, ym, y, yp, zm, z, zp, f);
  float rho, m[3];
  moments(f, rho, m[0], m[1], m[2]);
  float gg[3];
  load_g(g, e.ib ? e.tile_slot : nullptr, e.gfix, x, y, z, gg[0], gg[1], gg[2]);
  float lam[Q];
  load_lam(A.lam_next, g, (uint32_t)yz, lo ? 0 : g.nx - 1, lam);
  float rb, mb[3], gb[3];
  adj_face(lam, rho, m, gg, lo ? A.bc_u_lo : A.bc_u_hi, (lo ? g.bc_lo : g.bc_hi) == 1, A, e.omt, e.pref, rb, mb, gb);
  float *fp = A.facebuf + (size_t)side * 4 * nyz;
  fp[yz] = rb;
  fp[nyz + yz] = mb[0];
  fp[2 * nyz + yz] = mb[1];
  fp[3 * nyz + yz] = mb[2];
}

template <bool XPER>
__global__ void __launch_bounds__(512) k_adj_collide(EnvView e, AdjArgs A) {
  const int lb = blockIdx.x;
  if (lb >= e.nblocks) return;
  adj_collide_cell<XPER>(e, A, lb, threadIdx.x, threadIdx.y);
}

constexpr int kFacePerBlock = 64;  // face nodes per workgroup (one wave): strided loads, spread over many CUs

// Pass 1 in one launch: workgroups [0, face_blocks) take kFacePerBlock open
// face nodes each (adj_face_item), the rest the active tiles (adj_gbar_item;
// none without a body).
__global__ void __launch_bounds__(WG) k_adj_gbar(EnvView e, AdjArgs A, int face_blocks) {
  if ((int)blockIdx.x < face_blocks) {
    const int id = blockIdx.x * kFacePerBlock + threadIdx.x;
    if (threadIdx.x < kFacePerBlock && id < 2 * e.g.ny * e.g.nz) adj_face_item(e, A, id);
    return;
  }
  if (!e.ib) return;
  const int na = n_active_of(e);
  const int nb = gridDim.x - face_blocks;
  for (int slot = blockIdx.x - face_blocks; slot < na; slot += nb) adj_gbar_item(e, A, slot, threadIdx.x);
}

__global__ void __launch_bounds__(WG) k_adj_markers(EnvView e, AdjArgs A) {
  adj_marker_item(e, A, blockIdx.x, threadIdx.x);
}

__global__ void __launch_bounds__(WG) k_adj_spread(EnvView e, AdjArgs A) {
  const int items = n_active_of(e) * kSpreadSplit;
  for (int item = blockIdx.x; item < items; item += gridDim.x) adj_spread_item(e, A, item, threadIdx.x);
}

// ------------------------------------------------------------------ pass 5 --
// Pose adjoint: X = sum_b w (R xrest + t), U = sum_b w (Rdot xrest + tdot).
// Workgroup (b, p, t) sums the terms of bone b over the p-th of kPoseSplit
// marker ranges of step t (marker adjoints mbar + t mstride, [6][n]) into
// pbar + t pstride, [nbones][kPoseSplit][24]; k_adj_pose_sum adds the
// kPoseSplit partials in order into pose_bar[t][b] (deterministic). One
// launch covers one step, or every step of a segment.
__global__ void __launch_bounds__(256) k_adj_pose_part(EnvView e, const float *__restrict__ mbar_base,
                                                       size_t mstride, float *__restrict__ pbar_base,
                                                       size_t pstride) {
  __shared__ float s_red[4][24];
  const int b = blockIdx.x, p = blockIdx.y;
  const float *__restrict__ mbar = mbar_base + mstride * blockIdx.z;
  float *__restrict__ pbar = pbar_base + pstride * blockIdx.z;
  const int n = e.n;
  const int chunk = (n + kPoseSplit - 1) / kPoseSplit;
  const int k0 = p * chunk, k1 = min(n, k0 + chunk);
  float acc[24];
#pragma unroll
  for (int q = 0; q < 24; ++q) acc[q] = 0.f;
  for (int k = k0 + (int)threadIdx.x; k < k1; k += 256) {
    const float wk = (e.bone[k] == b ? e.weight[k] : 0.f) + (e.bone[n + k] == b ? e.weight[n + k] : 0.f);
    const float xr[3] = {e.xrest[k], e.xrest[n + k], e.xrest[2 * n + k]};
    const float xb[3] = {wk * mbar[k], wk * mbar[n + k], wk * mbar[2 * n + k]};
    const float ub[3] = {wk * mbar[3 * n + k], wk * mbar[4 * n + k], wk * mbar[5 * n + k]};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc[3 * r + c] += xb[r] * xr[c];
        acc[12 + 3 * r + c] += ub[r] * xr[c];
      }
      acc[9 + r] += xb[r];
      acc[21 + r] += ub[r];
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 24; ++q) {
    const float v = wave_sum(acc[q]);
    if (lane == 0) s_red[wv][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < 24)
    pbar[((size_t)b * kPoseSplit + p) * 24 + threadIdx.x] =
        ((s_red[0][threadIdx.x] + s_red[1][threadIdx.x]) + s_red[2][threadIdx.x]) + s_red[3][threadIdx.x];
}

// grid (nbones, steps): pose_bar[t][b][q] += sum_p pbar_t[b][p][q], p in order.
__global__ void __launch_bounds__(64) k_adj_pose_sum(const float *__restrict__ pbar_base, size_t pstride,
                                                      float *__restrict__ pose_bar, int nbones) {
  const int b = blockIdx.x, q = threadIdx.x;
  if (q >= 24) return;
  const float *__restrict__ pbar = pbar_base + pstride * blockIdx.y;
  float v[kPoseSplit];
#pragma unroll
  for (int p = 0; p < kPoseSplit; ++p) v[p] = pbar[((size_t)b * kPoseSplit + p) * 24 + q];
  float s = 0.f;
#pragma unroll
  for (int p = 0; p < kPoseSplit; ++p) s += v[p];
  pose_bar[((size_t)blockIdx.y * nbones + b) * 24 + q] += s;
}

}  // namespace lbmib
