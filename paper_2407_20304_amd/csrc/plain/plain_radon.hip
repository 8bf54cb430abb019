// Plain per-angle ray sums and their transpose (Eq. 14 and its adjoint):
// the comparison baseline for the fused kernels.  One thread per ray (bin,
// slice) or per voxel, global-memory taps, one launch per angle.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "holo_plain.h"

namespace {

constexpr int kBlock = 256;

struct Ray {
  double c, C, S;   // grid centre, cos, sin
  int walk_y;       // 1: unit steps along y, taps along x
  float scale;      // 1 / max(|cos|, |sin|)
};

Ray make_ray(int W, double theta) {
  Ray r;
  r.c = 0.5 * W;
  r.C = std::cos(theta);
  r.S = std::sin(theta);
  r.walk_y = std::fabs(r.C) >= std::fabs(r.S) ? 1 : 0;
  r.scale = (float)(1.0 / (r.walk_y ? std::fabs(r.C) : std::fabs(r.S)));
  return r;
}

// Fractional crossing of ray `bin` with line `step` of the walk axis.
__device__ inline double crossing(const Ray& r, int bin, int step) {
  const double s = (double)bin - r.c, t = (double)step - r.c;
  return r.walk_y ? r.c + (s - t * r.S) / r.C : r.c + (s - t * r.C) / r.S;
}

// Thread (bin, slice): walk the W steps and interpolate two taps per step.
__global__ void k_plain_radon(const float2* __restrict__ u, int H, int W, Ray r,
                              float2* __restrict__ p) {
  const int bin = blockIdx.x * kBlock + threadIdx.x;
  const int z = blockIdx.y;
  if (bin >= W || z >= H) return;
  const float2* slice = u + (size_t)z * W * W;
  float ax = 0.f, ay = 0.f;
  for (int step = 0; step < W; ++step) {
    const double f = crossing(r, bin, step);
    const double fl = floor(f);
    const int i0 = (int)fl;
    const float w = (float)(f - fl);
    if (i0 >= 0 && i0 < W) {
      const float2 v = r.walk_y ? slice[(size_t)step * W + i0] : slice[(size_t)i0 * W + step];
      ax += (1.f - w) * v.x;
      ay += (1.f - w) * v.y;
    }
    if (i0 + 1 >= 0 && i0 + 1 < W) {
      const float2 v = r.walk_y ? slice[(size_t)step * W + i0 + 1] : slice[(size_t)(i0 + 1) * W + step];
      ax += w * v.x;
      ay += w * v.y;
    }
  }
  p[(size_t)z * W + bin] = make_float2(ax * r.scale, ay * r.scale);
}

// Thread (x, y, slice): the bins whose crossing with this voxel's line of
// the walk lands within one index of it are found from the voxel's
// fractional bin position q (|i - q| < max(|cos|, |sin|) <= 1); each
// candidate's crossing is recomputed exactly as the projector forms it, so
// the weights are the projector's.
__global__ void k_plain_radon_adj(const float2* __restrict__ h, int H, int W, Ray r,
                                  float2* __restrict__ g) {
  const size_t n = (size_t)H * W * W;
  const size_t id = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= n) return;
  const int x = (int)(id % W), y = (int)((id / W) % W), z = (int)(id / ((size_t)W * W));
  const int step = r.walk_y ? y : x;     // this voxel's line of the walk
  const int tap = r.walk_y ? x : y;      // its index across the ray
  const double q = r.c + ((double)x - r.c) * r.C + ((double)y - r.c) * r.S;
  const int lo = (int)floor(q) - 2, hi = (int)floor(q) + 2;
  float ax = 0.f, ay = 0.f;
  for (int bin = lo; bin <= hi; ++bin) {
    if (bin < 0 || bin >= W) continue;
    const double f = crossing(r, bin, step);
    const double fl = floor(f);
    const int i0 = (int)fl;
    const float w = (float)(f - fl);
    float wt;
    if (i0 == tap) wt = 1.f - w;
    else if (i0 + 1 == tap) wt = w;
    else continue;
    const float2 v = h[(size_t)z * W + bin];
    ax += wt * v.x;
    ay += wt * v.y;
  }
  float2 o = g[id];
  o.x += ax * r.scale;
  o.y += ay * r.scale;
  g[id] = o;
}

bool args_ok(const void* a, const void* b, int H, int W, double theta) {
  return a && b && H >= 1 && W >= 2 && std::isfinite(theta);
}

}  // namespace

extern "C" int32_t holo_plain_radon(const void* u, int32_t H, int32_t W, double theta, void* p,
                                    void* stream) {
  if (!args_ok(u, p, H, W, theta)) return 1;
  const Ray r = make_ray(W, theta);
  dim3 grid((unsigned)((W + kBlock - 1) / kBlock), (unsigned)H);
  k_plain_radon<<<grid, kBlock, 0, (hipStream_t)stream>>>((const float2*)u, H, W, r, (float2*)p);
  return hipGetLastError() == hipSuccess ? 0 : 4;
}

extern "C" int32_t holo_plain_radon_adj(const void* h, int32_t H, int32_t W, double theta,
                                        void* g_u, void* stream) {
  if (!args_ok(h, g_u, H, W, theta)) return 1;
  const Ray r = make_ray(W, theta);
  const size_t n = (size_t)H * W * W;
  const size_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 0x7fffffffu) return 1;
  k_plain_radon_adj<<<(unsigned)blocks, kBlock, 0, (hipStream_t)stream>>>(
      (const float2*)h, H, W, r, (float2*)g_u);
  return hipGetLastError() == hipSuccess ? 0 : 4;
}
