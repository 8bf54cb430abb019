/*
 * holo_plain.h -- C ABI of the plain per-angle ray-sum kernels
 * (libholo_plain.so).
 *
 * These are the deliberately simple forms of the ray-sum projector R_theta
 * (Sec. 2, Eq. 14) and of its adjoint R_theta^* (the back-projection of the
 * tomography step, Eq. 15), used only as the comparison baseline for the
 * fused library: one thread per ray or per voxel, every tap read from
 * global memory, one launch per angle.  They compute the same Joseph
 * discretisation as libholo.so (see holo.h):
 *
 *   p[z][i] = s(theta) sum_step ((1 - w) u[..][i0] + w u[..][i0 + 1])
 *
 * with unit steps along the dominant axis of the ray (y when
 * |cos| >= |sin|), the crossing f = c + (s_i - (step - c) sin) / cos (or the
 * same with sin and cos exchanged), i0 = floor(f), w = f - i0, taps outside
 * the grid dropped, s(theta) = 1 / max(|cos|, |sin|), c = W/2, s_i = i - c.
 * The crossing is formed in double precision, the sums in float.
 *
 * Layouts (device pointers, complex = interleaved float re/im):
 *   u, g_u  [H][W][W]   u[z][y][x]
 *   p, h    [H][W]      p[z][bin]
 *
 * Errors: 1 (invalid argument: NULL pointer, H < 1, W < 2, non-finite
 * theta) before any device work; 4 (HIP launch error).  Calls are
 * asynchronous on `stream` (a hipStream_t, NULL = default stream).
 */
#ifndef HOLO_PLAIN_H
#define HOLO_PLAIN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* p = R_theta u for one angle (overwrites p). */
int32_t holo_plain_radon(const void* u, int32_t H, int32_t W, double theta, void* p,
                         void* stream);

/* g_u += R_theta^T h for one angle: each voxel gathers the bins whose taps
 * reach it, with the weights the projector gave it. */
int32_t holo_plain_radon_adj(const void* h, int32_t H, int32_t W, double theta, void* g_u,
                             void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HOLO_PLAIN_H */
