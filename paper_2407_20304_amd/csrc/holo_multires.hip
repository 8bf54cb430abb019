// Data binning and grid refinement of the hierarchical schedule (Sec. 4:
// iterate on binned data, move the result to a grid twice as dense, go on
// with less binning).  Binning by b averages the intensities of b x b
// detector pixels (amplitudes: sqrt of the mean squared amplitude); moving to
// a grid f times denser replicates every cell.
#include <hip/hip_runtime.h>

#include <string>

#include "holo.h"
#include "holo_internal.hpp"

namespace holo {
holo_status set_last_error(holo_status st, const std::string& msg);
}

namespace {

constexpr int kBlock = 256;

unsigned grid_of(size_t n) {
  const size_t g = (n + kBlock - 1) / kBlock;
  return (unsigned)(g < 65536 ? (g ? g : 1) : 65536);
}

// out[f][y][x] = mean over the b x b block of in[f] (of in^2 with sqrt for
// amplitudes), summed in double.
__global__ void k_bin(const float* __restrict__ in, size_t n_out, int Ho, int Wo, int b,
                      int amplitude, float* __restrict__ out) {
  const int W = Wo * b;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n_out;
       i += (size_t)gridDim.x * kBlock) {
    const int x = (int)(i % Wo), y = (int)((i / Wo) % Ho);
    const size_t f = i / ((size_t)Wo * Ho);
    const float* src = in + (f * Ho * b + (size_t)y * b) * W + (size_t)x * b;
    double acc = 0.0;
    for (int r = 0; r < b; ++r)
      for (int c = 0; c < b; ++c) {
        const double v = src[(size_t)r * W + c];
        acc += amplitude ? v * v : v;
      }
    const double m = acc / ((double)b * b);
    out[i] = (float)(amplitude ? sqrt(m) : m);
  }
}

// out[z][y][x] = in[z / fz][y / f][x / f] for an output of nz x (H f) x (W f).
__global__ void k_replicate(const float2* __restrict__ in, size_t n_out, int Ho, int Wo, int f,
                            int fz, float2* __restrict__ out) {
  const int Hi = Ho / f, Wi = Wo / f;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n_out;
       i += (size_t)gridDim.x * kBlock) {
    const int x = (int)(i % Wo), y = (int)((i / Wo) % Ho);
    const size_t z = i / ((size_t)Wo * Ho);
    out[i] = in[((z / fz) * Hi + y / f) * Wi + x / f];
  }
}

holo_status fail(holo_status s, const std::string& m) { return holo::set_last_error(s, m); }

}  // namespace

extern "C" holo_status holo_bin_frames(const float* in, int64_t n_frames, int32_t H, int32_t W,
                                       int32_t b, int32_t amplitude, float* out, void* stream) {
  if (!in || !out) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_bin_frames: NULL pointer");
  if (n_frames < 1 || H < 1 || W < 1 || b < 1 || H % b || W % b)
    return fail(HOLO_ERR_INVALID_ARGUMENT,
                "holo_bin_frames: need n_frames, H, W, b >= 1 with b dividing H and W");
  if ((const void*)in == (const void*)out && b > 1)
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_bin_frames: out aliases in");
  const size_t n_out = (size_t)n_frames * (H / b) * (W / b);
  k_bin<<<grid_of(n_out), kBlock, 0, (hipStream_t)stream>>>(in, n_out, H / b, W / b, b,
                                                              amplitude ? 1 : 0, out);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? HOLO_OK
                         : fail(HOLO_ERR_HIP, std::string("holo_bin_frames: ") + hipGetErrorString(e));
}

static holo_status replicate(const holo_c64* in, int64_t n_in, int32_t H, int32_t W, int32_t f,
                             int32_t fz, holo_c64* out, void* stream, const char* fn) {
  if (!in || !out) return fail(HOLO_ERR_INVALID_ARGUMENT, std::string(fn) + ": NULL pointer");
  if (n_in < 1 || H < 1 || W < 1 || f < 1)
    return fail(HOLO_ERR_INVALID_ARGUMENT, std::string(fn) + ": sizes and factor must be >= 1");
  if ((const void*)in == (const void*)out)
    return fail(HOLO_ERR_INVALID_ARGUMENT, std::string(fn) + ": out aliases in");
  const size_t n_out = (size_t)n_in * fz * ((size_t)H * f) * ((size_t)W * f);
  k_replicate<<<grid_of(n_out), kBlock, 0, (hipStream_t)stream>>>(
      (const float2*)in, n_out, H * f, W * f, f, fz, (float2*)out);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? HOLO_OK
                         : fail(HOLO_ERR_HIP, std::string(fn) + ": " + hipGetErrorString(e));
}

extern "C" holo_status holo_upsample_frames(const holo_c64* in, int64_t n_frames, int32_t H,
                                            int32_t W, int32_t f, holo_c64* out, void* stream) {
  return replicate(in, n_frames, H, W, f, 1, out, stream, "holo_upsample_frames");
}

extern "C" holo_status holo_upsample_volume(const holo_c64* in, int32_t H, int32_t W, int32_t f,
                                            holo_c64* out, void* stream) {
  return replicate(in, H, W, W, f, f, out, stream, "holo_upsample_volume");
}
