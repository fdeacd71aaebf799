// Reference streaming kernels declared in include/hbm_ceiling.h: a copy, a
// read and the collide's access pattern without its arithmetic, for the
// practical HBM ceiling of the lattice Boltzmann step on this device.
#include <hip/hip_runtime.h>

#include "../../include/hbm_ceiling.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_copy(const f4 *__restrict__ a, f4 *__restrict__ b, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(a[i], b + i);
}

__global__ void __launch_bounds__(256) k_read(const f4 *__restrict__ a, size_t n, float *sink) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const f4 v = a[i];
    if (v.x == -12345.678f && v.y == 9876.5f) sink[0] = v.z + v.w;
  }
}

struct Dims {
  int nx, ny, nz;
  uint64_t ps, rs;
};

__global__ void __launch_bounds__(256) k_pull27(const float *__restrict__ src, float *__restrict__ dst, Dims d) {
  const uint64_t cell = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t row = cell / (uint64_t)d.nx;
  const int x = (int)(cell - row * (uint64_t)d.nx);
  const int z = (int)(row / (uint64_t)d.ny);
  const int y = (int)(row - (uint64_t)z * d.ny);
  if (z >= d.nz) return;
  const int xx[3] = {x == d.nx - 1 ? 0 : x + 1, x, x == 0 ? d.nx - 1 : x - 1};  // by cx + 1: x - cx
  const int yy[3] = {y == d.ny - 1 ? 0 : y + 1, y, y == 0 ? d.ny - 1 : y - 1};
  const int zz[3] = {z == d.nz - 1 ? 0 : z + 1, z, z == 0 ? d.nz - 1 : z - 1};
  float f[27];
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const uint64_t r = (uint64_t)zz[i / 9] * d.ny + yy[(i / 3) % 3];
    f[i] = src[r * d.rs + (uint64_t)i * d.ps + xx[i % 3]];
    s += f[i];
  }
  float *__restrict__ o = dst + row * d.rs + x;
#pragma unroll
  for (int i = 0; i < 27; ++i) __builtin_nontemporal_store(0.9f * f[i] + 1e-3f * s, o + (uint64_t)i * d.ps);
}

int launched() { return hipGetLastError() == hipSuccess ? 0 : -2; }

}  // namespace

extern "C" {

int hbm_copy(const void *src, void *dst, size_t bytes, void *hip_stream) {
  if (!src || !dst || bytes == 0 || bytes % 16 != 0) return -1;
  if (reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16) return -1;
  const size_t n = bytes / 16;
  k_copy<<<(unsigned)((n + 255) / 256), 256, 0, static_cast<hipStream_t>(hip_stream)>>>(
      static_cast<const f4 *>(src), static_cast<f4 *>(dst), n);
  return launched();
}

int hbm_read(const void *src, size_t bytes, float *sink, void *hip_stream) {
  if (!src || !sink || bytes == 0 || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(src) % 16) return -1;
  const size_t n = bytes / 16;
  k_read<<<(unsigned)((n + 255) / 256), 256, 0, static_cast<hipStream_t>(hip_stream)>>>(
      static_cast<const f4 *>(src), n, sink);
  return launched();
}

int hbm_pull27(const float *src, float *dst, int32_t nx, int32_t ny, int32_t nz, int64_t ps, int64_t rs,
               int32_t blocks_per_cu, void *hip_stream) {
  if (!src || !dst || src == dst || nx < 1 || ny < 1 || nz < 1 || ps < 1 || rs < 1) return -1;
  if (blocks_per_cu < 0 || blocks_per_cu > 32) return -1;
  const uint64_t cells = (uint64_t)nx * ny * nz;
  const bool planes = rs == nx && (uint64_t)ps >= cells;
  const bool rows = ps == nx && rs == 27 * (int64_t)nx;
  if (!planes && !rows) return -1;
  const uint64_t blocks = (cells + 255) / 256;
  if (blocks > 0x7fffffffull) return -1;
  // reserved, unused LDS: a size between the bounds for blocks_per_cu and
  // blocks_per_cu + 1 blocks of a 160 KiB compute unit, in whole KiB
  const size_t lds = blocks_per_cu > 0 ? (size_t)(2 * 160 * 1024 / (2 * blocks_per_cu + 1)) & ~(size_t)1023 : 0;
  k_pull27<<<(unsigned)blocks, 256, lds, static_cast<hipStream_t>(hip_stream)>>>(
      src, dst, Dims{nx, ny, nz, (uint64_t)ps, (uint64_t)rs});
  return launched();
}

}  // extern "C"
