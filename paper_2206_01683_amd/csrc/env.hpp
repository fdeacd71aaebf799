// Device-side description of one lattice and its immersed body ("environment").
// Every kernel of the library works on an EnvView: the single-lattice
// launches pass one by value, the batched launches index an array of them.
#pragma once

#include "lattice.hpp"

namespace lbmib {

struct GridArgs {
  int nx, ny, nz;
  uint32_t plane;  // a population buffer holds 27 * plane elements
  // Population layout: element (i, x, y, z) at row * rs + i * ps + x with
  // row = z * ny + y. Planes: ps = plane, rs = nx ([27][nz][ny][nx], each
  // population a plane of its own). Rows: ps = nx, rs = 27 * nx
  // ([nz][ny][27][nx], the 27 populations of one (y, z) row side by side).
  uint32_t ps, rs;
  int xper;        // 1: x periodic
  int bc_lo, bc_hi;
  int tnx, tny;    // 8^3 tile grid (x, y extents)
  int yper, zper;  // 1: y (z) periodic; otherwise both faces open
  int bc_y[2], bc_z[2];
};

// Rates of the two-relaxation-time collision: omega+, omega-, the source
// factors 1 - omega+/2 and 1 - omega-/2, and a = 1 - (omega+ + omega-)/2,
// b = (omega- - omega+)/2 (f*_i = a f_i + b f_opp(i) + ...).
struct TrtRates {
  float wp, wm, pp, pm, a, b;
};

struct EnvView {
  GridArgs g;
  float inv_tau, omt, pref;     // 1/tau, 1 - 1/tau, 1 - 1/(2 tau)
  TrtRates trt;                 // used by the TRT collide only
  int two_rate;                 // collision: 1 TRT (rates in trt), 0 BGK
  int storage;                  // population format: Store*::kind (0 F32, 1 F16, 2 BF16)
  int bx, by, gx, gy, nblocks;  // collide tile shape and its block grid (by = 0: linear, see cell_of)
  void *f[2];                   // population buffers
  // immersed boundary
  int ib;                       // a body is present this step
  int n, nbones, cap, ntiles;
  float alpha2;                 // 2 * direct-forcing gain
  const float *xrest, *weight, *dv;
  int slip;                     // slip wall: force along the skinned normals Nrm only
  const float *nrest;           // [3][n] rest normals (slip)
  float *Nrm;                   // [3][n] skinned unit normals of this step (slip)
  const int *bone;
  float *X, *U, *F;
  int *tile_flag, *tile_slot, *active, *counters, *guard;
  short4 *mbase;
  int4 *chunk_box;
  float *partials;
  float4 *macro;
  unsigned long long *gfix;
  unsigned *sched;              // scheduling words of the overlapped step (single lattice), or null
  float *rec, *mstate;
  // implicit velocity correction (null with direct forcing)
  unsigned long long *gcg;      // fixed-point spread of the search direction, as gfix
  float *cg;                    // G, r, p, q, each [3][n]
  float *cgpart;                // dot-product partials: p.q [interp items][4], r.z [2][cg items][4]
  // per-run device inputs of the batched forms, indexed by step
  const float *poses;    // [nsteps][nbones][24]
  const double *frames;  // [nsteps][18] (lbm_frame layout)
  float *wrench;         // [nsteps][8] or null
  int rot;               // some frame rotates
  int cur0;              // buffer holding the state at the start of the run
};

// Element offset of population i at x in row `row` (= z * ny + y).
__device__ inline size_t pop_idx(const GridArgs &g, int i, uint32_t row, uint32_t x) {
  return (size_t)row * g.rs + (size_t)i * g.ps + x;
}

// Cell of thread (tx, ty) in logical collide block lb. Tile shapes bx x by
// cover x-rows and y in 2-D blocks (z from the block index); the linear shape
// (by = 0) gives each block bx consecutive cells of the x-fastest order, rows
// and planes wrapped, so no lane idles at ragged row ends. False past the
// lattice.
__device__ inline bool cell_of(const EnvView &e, int lb, int tx, int ty, int &x, int &y, int &z) {
  if (e.by == 0) {
    const uint32_t cell = (uint32_t)lb * (uint32_t)e.bx + (uint32_t)tx;
    const uint32_t row = cell / (uint32_t)e.g.nx;
    x = (int)(cell - row * (uint32_t)e.g.nx);
    z = (int)(row / (uint32_t)e.g.ny);
    y = (int)(row - (uint32_t)z * (uint32_t)e.g.ny);
    return z < e.g.nz;
  }
  const int bxi = lb % e.gx;
  const int rest = lb / e.gx;
  const int byi = rest % e.gy;
  z = rest / e.gy;
  x = bxi * e.bx + tx;
  y = byi * e.by + ty;
  return x < e.g.nx && y < e.g.ny;
}

// lbm_frame (18 doubles) -> float32 frame constants
template <class P>
__device__ inline FrameF frame_from(P d) {
  FrameF f;
  for (int a = 0; a < 3; ++a) {
    f.acc[a] = (float)d[a];
    f.omg[a] = (float)d[3 + a];
    f.alp[a] = (float)d[6 + a];
    f.org[a] = (float)d[9 + a];
    f.ulo[a] = (float)d[12 + a];
    f.uhi[a] = (float)d[15 + a];
  }
  return f;
}

}  // namespace lbmib
