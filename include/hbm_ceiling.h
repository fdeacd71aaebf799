/*
 * hbm_ceiling.h - reference streaming kernels for the HBM bandwidth a
 * bandwidth-bound lattice Boltzmann step can expect on one MI355X (gfx950).
 *
 * The step's roofline is the HBM peak; what simple kernels actually move on
 * the same device is the practical ceiling its collide is compared with: a
 * plain copy, a plain read, and the collide's own access pattern with the
 * arithmetic taken out (27 pulls from the neighbours x - c_i of a D3Q27
 * lattice, 27 stores at x), in either population layout.
 *
 * Conventions: device pointers, allocated and owned by the caller; work is
 * queued on hip_stream (hipStream_t, NULL = default stream) and the call
 * returns without synchronizing. Return value 0 on success, -1 for a bad
 * argument (nothing queued), -2 if the launch failed.
 */
#ifndef HBM_CEILING_H
#define HBM_CEILING_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* dst[k] = src[k] for `bytes` bytes (a multiple of 16, both pointers 16-byte
 * aligned, no overlap): one 16-byte load and one non-temporal 16-byte store
 * per thread, 256 threads per block. */
int hbm_copy(const void *src, void *dst, size_t bytes, void *hip_stream);

/* Read `bytes` bytes of src (a multiple of 16, 16-byte aligned), one 16-byte
 * load per thread; sink [1 float] is written only if a value equals a
 * sentinel no real input holds, so the loads cannot be removed. */
int hbm_read(const void *src, size_t bytes, float *sink, void *hip_stream);

/* The collide's memory traffic without its arithmetic, on an nx x ny x nz
 * periodic lattice of float32 populations: for every cell x,
 *   dst(i, x) = 0.9 src(i, x - c_i) + 1e-3 sum_j src(j, x - c_j),
 * c_i in {-1,0,1}^3 with i = (cx+1) + 3(cy+1) + 9(cz+1). Element (i, x, y, z)
 * of either buffer sits at (z ny + y) rs + i ps + x (the population layouts of
 * lbm_ib.h: planes ps >= nx ny nz, rs = nx; rows ps = nx, rs = 27 nx), so each
 * buffer holds at least (nz ny - 1) rs + 26 ps + nx floats.
 * 256 consecutive cells of the x-fastest order per block, non-temporal
 * stores. blocks_per_cu > 0 reserves unused LDS so that at most that many
 * blocks share a compute unit (the cap the library's F32 collide runs
 * under); 0 leaves occupancy to the registers. -1 if a size is < 1, the
 * strides do not give every element its own place, or blocks_per_cu is
 * outside 0..32. */
int hbm_pull27(const float *src, float *dst, int32_t nx, int32_t ny, int32_t nz, int64_t ps, int64_t rs,
               int32_t blocks_per_cu, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif
