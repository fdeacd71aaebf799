// D3Q27 lattice, population storage formats and per-node physics shared by
// the kernels of this library (device side only).
//
// Lattice: c_i in {-1,0,1}^3 with i = (cx+1) + 3(cy+1) + 9(cz+1), so the rest
// velocity is i = 13 and the opposite of i is 26 - i. Weights by |c|^2:
// 8/27, 2/27, 1/54, 1/216 (c_s^2 = 1/3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmib {

constexpr int Q = 27;
__host__ __device__ constexpr int cx_of(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cy_of(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz_of(int i) { return i / 9 - 1; }
__host__ __device__ constexpr int c2_of(int i) {
  return cx_of(i) * cx_of(i) + cy_of(i) * cy_of(i) + cz_of(i) * cz_of(i);
}
__host__ __device__ constexpr float w_of(int i) {
  return c2_of(i) == 0 ? 8.0f / 27.0f : c2_of(i) == 1 ? 2.0f / 27.0f : c2_of(i) == 2 ? 1.0f / 54.0f : 1.0f / 216.0f;
}

// Device memory seen through the global address space. A pointer read from
// memory (an EnvView in the batched forms' descriptor array) carries no
// address space, and the compiler then accesses it with flat instructions,
// which also count against the wait counter of LDS and scalar loads, so a
// wait for one of those waits for every population load in flight. The hot
// loads and stores go through pointers cast to this space instead.
template <class T>
using gmem = __attribute__((address_space(1))) T;
typedef float vfloat4 __attribute__((ext_vector_type(4)));  // float4 as a native vector (stores through gmem)

// ------------------------------------------------------------- storage ----
// Every format keeps h_i = f_i - w_i, the offset from the rest equilibrium:
// F32 as float, F16 / BF16 rounded to nearest even. The collide works on h
// directly (rho - 1 = sum h, m = sum h c), so the rounding of a stored value
// scales with |h| rather than with w_i; load / store convert to and from f
// for the kernels that want f.
struct StoreF32 {
  using T = float;
  static constexpr int kind = 0;
  template <class P>
  __device__ static inline float load_dev(P p, int) { return *p; }
  template <class P>
  __device__ static inline void store_dev(P p, float h, int) { __builtin_nontemporal_store(h, p); }
  template <class P>
  __device__ static inline float load(P p, int i) { return w_of(i) + *p; }
  template <class P>
  __device__ static inline void store(P p, float f, int i) { __builtin_nontemporal_store(f - w_of(i), p); }
  template <class P>
  __device__ static inline void store_plain(P p, float f, int i) { *p = f - w_of(i); }
};

struct StoreF16 {
  using T = _Float16;
  static constexpr int kind = 1;
  template <class P>
  __device__ static inline float load_dev(P p, int) { return (float)(*p); }
  template <class P>
  __device__ static inline void store_dev(P p, float h, int) { __builtin_nontemporal_store((_Float16)h, p); }
  template <class P>
  __device__ static inline float load(P p, int i) { return w_of(i) + (float)(*p); }
  template <class P>
  __device__ static inline void store(P p, float f, int i) {
    __builtin_nontemporal_store((_Float16)(f - w_of(i)), p);
  }
  template <class P>
  __device__ static inline void store_plain(P p, float f, int i) { *p = (_Float16)(f - w_of(i)); }
};

struct StoreBF16 {
  using T = uint16_t;
  static constexpr int kind = 2;
  __device__ static inline float to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
  __device__ static inline uint16_t to_h(float f) {
    // round to nearest, ties to even, on the upper 16 bits
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
  }
  template <class P>
  __device__ static inline float load_dev(P p, int) { return to_f(*p); }
  template <class P>
  __device__ static inline void store_dev(P p, float h, int) { __builtin_nontemporal_store(to_h(h), p); }
  template <class P>
  __device__ static inline float load(P p, int i) { return w_of(i) + to_f(*p); }
  template <class P>
  __device__ static inline void store(P p, float f, int i) { __builtin_nontemporal_store(to_h(f - w_of(i)), p); }
  template <class P>
  __device__ static inline void store_plain(P p, float f, int i) { *p = to_h(f - w_of(i)); }
};

// ------------------------------------------------------------- frames -----
// Per-step constants of Eq. (3) in float32.
struct FrameF {
  float acc[3], omg[3], alp[3], org[3], ulo[3], uhi[3];
};

__device__ inline void cross3(const float a[3], float bx, float by, float bz, float &ox, float &oy, float &oz) {
  ox = a[1] * bz - a[2] * by;
  oy = a[2] * bx - a[0] * bz;
  oz = a[0] * by - a[1] * bx;
}

// a0(x) = -acc - alpha x x' - omega x (omega x x'), x' = x - origin
template <bool ROT>
__device__ inline void frame_a0(const FrameF &fr, float px, float py, float pz, float &ax, float &ay, float &az) {
  ax = -fr.acc[0];
  ay = -fr.acc[1];
  az = -fr.acc[2];
  if (ROT) {
    float rx = px - fr.org[0], ry = py - fr.org[1], rz = pz - fr.org[2];
    float t0, t1, t2, s0, s1, s2, q0, q1, q2;
    cross3(fr.alp, rx, ry, rz, t0, t1, t2);
    cross3(fr.omg, rx, ry, rz, s0, s1, s2);
    cross3(fr.omg, s0, s1, s2, q0, q1, q2);
    ax -= t0 + q0;
    ay -= t1 + q1;
    az -= t2 + q2;
  }
}

// Solve u + omega x u = b exactly: u = (b - omega x b + (omega.b) omega)/(1 + |omega|^2)
template <bool ROT>
__device__ inline void solve_coriolis(const FrameF &fr, float bx, float by, float bz, float &ux, float &uy,
                                      float &uz) {
  if (!ROT) {
    ux = bx;
    uy = by;
    uz = bz;
    return;
  }
  float cxv, cyv, czv;
  cross3(fr.omg, bx, by, bz, cxv, cyv, czv);
  float wb = fr.omg[0] * bx + fr.omg[1] * by + fr.omg[2] * bz;
  float inv = 1.0f / (1.0f + fr.omg[0] * fr.omg[0] + fr.omg[1] * fr.omg[1] + fr.omg[2] * fr.omg[2]);
  ux = (bx - cxv + wb * fr.omg[0]) * inv;
  uy = (by - cyv + wb * fr.omg[1]) * inv;
  uz = (bz - czv + wb * fr.omg[2]) * inv;
}

// Peskin's 4-point kernel on one axis, |r| <= 2.
__device__ inline float peskin4(float r) {
  float a = fabsf(r);
  if (a <= 1.0f) return 0.125f * (3.0f - 2.0f * a + __builtin_sqrtf(fmaxf(1.0f + 4.0f * a - 4.0f * a * a, 0.0f)));
  if (a <= 2.0f) return 0.125f * (5.0f - 2.0f * a - __builtin_sqrtf(fmaxf(-7.0f + 12.0f * a - 4.0f * a * a, 0.0f)));
  return 0.0f;
}

__device__ inline int wrap_idx(int j, int n) {
  j = j < 0 ? j + n : j;
  return j >= n ? j - n : j;
}

// Device guard bits
enum : int { GUARD_UNSTABLE = 1, GUARD_MARKER_RANGE = 2, GUARD_CAPACITY = 4, GUARD_BONE = 8, GUARD_SCHEDULE = 16 };

}  // namespace lbmib
