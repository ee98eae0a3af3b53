/*
 * lbm_study.h -- memory-access study kernels (C ABI, same library as lbm.h).
 *
 * Re-runs on gfx950 the access-pattern experiments of Mawson & Revell,
 * Section 4.3:
 *   - aligned vs misaligned reads and writes over several large vectors,
 *     the patterns of the push and pull algorithms (Section 4.3, E1);
 *   - offset-by-one propagation of a row, done with direct misaligned
 *     loads, staged through LDS, or shifted across lanes with DPP
 *     (Section 4.3.2);
 *   - the fused push (Algorithm 2) and pull (Algorithm 3) iterations,
 *     one lattice point per work-item.
 *
 * All pointers are device pointers; work is enqueued on `hip_stream` (NULL =
 * null stream) and the calls return before it finishes. Arrays use the
 * paper's plain structure-of-arrays order f[i*N + c], c = (z*ny + y)*nx + x
 * (Section 4.1). Errors: LBM_ERR_INVALID for bad sizes/modes or NULL
 * pointers, LBM_ERR_DEVICE when the launch fails. No call allocates.
 */
#ifndef LBM_STUDY_H
#define LBM_STUDY_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * nvec independent vectors of n floats each (vector v at src + v*n):
 *   mode 0 (copy):  dst[v][k + woff] = src[v][k + roff]
 *   mode 1 (read):  sink[k] = sum_v src[v][k + roff]   (one write stream)
 *   mode 2 (write): dst[v][k + woff] = k + v            (no reads)
 * for k = 0 .. n - 2 (the last element is left out so that offsets 0 and 1
 * address the same count). roff, woff in {0, 1}; width = elements per
 * work-item, 1 (one 4-byte access) or 4 (one 16-byte access).
 * 1 <= nvec <= 32, n >= 8, n % 4 == 0 for width 4.
 */
lbm_status lbm_study_stream(int mode, const float* src, float* dst, float* sink, size_t n,
                            int nvec, int roff, int woff, int width, void* hip_stream);

/*
 * Offset-by-one propagation of nrows rows of nx floats, periodic within a
 * row: dst[r][x] = src[r][(x - 1) mod nx] (the e_x = +1 pull of a row).
 *   method 0: direct misaligned loads, one element per work-item;
 *   method 1: aligned loads staged through LDS, shifted read from LDS;
 *   method 2: aligned loads shifted across lanes with DPP (wave_shr:1),
 *             the wave-boundary element passed through LDS;
 *   method 3: direct misaligned 16-byte loads, four elements per work-item.
 * Methods 1 and 2 use one work-group per row: nx must be a multiple of 64
 * and at most 1024. Method 3 needs nx % 4 == 0.
 */
lbm_status lbm_study_shift(const float* src, float* dst, int nx, int nrows, int method,
                           void* hip_stream);

/*
 * The memory streams of the step without its stencil (Section 4.1: 19 loads
 * and 19 stores of 4 bytes per point): 19 planes per z-slab in the lattice
 * kernels' layout, plane (z, i) at element (z*19 + i)*nx*ny, row y at y*nx
 * within it. One row per wave, four points (16 bytes) per work-item, every
 * access aligned, the FP32 step's cache hints.
 *   mode 0 (copy):  dst = src     (19*N floats each)
 *   mode 1 (read):  reads src; sink is written only for data that never
 *                   occur (it may hold one float)
 *   mode 2 (write): dst[(z*19 + i)*nx*ny + y*nx + x..x+3] = {i, y*nx + x, 0, 1}
 * nx % 4 == 0, nx*ny*nz < 2^30, src and dst 16-byte aligned.
 */
lbm_status lbm_study_planes(int mode, const float* src, float* dst, float* sink, int nx, int ny,
                            int nz, void* hip_stream);

/*
 * One fused D3Q19 BGK iteration, FP32, one lattice point per work-item, on
 * plain [19][N] arrays `a` -> `b` (distinct), flags_dev [N] (0 fluid,
 * nonzero solid; walls are halfway bounce-back at rest; periodic box; no
 * body force).
 *   scheme 0, pull (Algorithm 3): a and b hold post-collision values s;
 *             gather p_i(x) = s_i(x - e_i) (misaligned reads), collide,
 *             aligned stores.
 *   scheme 1, push (Algorithm 2): a and b hold post-streaming values p;
 *             aligned local reads, collide, scatter s_i(x) to x + e_i
 *             (misaligned writes), or back into direction opp(i) of x when
 *             x + e_i is solid.
 * Both evolve the same recurrence: push applied to p = P s equals P applied
 * to the pull result, P being the streaming with bounce-back. Block size:
 * block_x threads along x (1..1024), one row per work-group row.
 */
lbm_status lbm_study_step(const float* a, float* b, const uint8_t* flags_dev, int nx, int ny,
                          int nz, float tau, int scheme, int block_x, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_STUDY_H */
