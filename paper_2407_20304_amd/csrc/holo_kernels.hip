// HIP kernels of the holotomography gradient for gfx950 (MI355X).
//
// Frame stages (detector-plane work, HBM-bound):
//   pass A  rows:    phi = 1 + B(psi - 1), x = Q_j phi, row FFT * transfer * IFFT
//   pass B  columns: column FFT * transfer * IFFT -> v, residual and cost,
//                    column FFT * conj(transfer) * IFFT
//   pass C  rows:    row FFT * conj(transfer) * IFFT -> w,
//                    G_j += conj(phi) w (probe gradient), X := conj(Q_j) w
//   pass D  pixels:  g_psi = sum_j B^T X_j (gather), h = -i kappa conj(psi) g_psi
// Ray sums (bound by VALU and LDS operand delivery):
//   radon_fwd  Joseph ray sums, angle groups sharing row windows staged in
//              LDS by LDS-direct loads (16 lanes cover the 64 slices of one
//              bin group, each thread owns 4 slices x 4 bins), fused
//              exp(i kappa p) epilogue
//   radon_adj  transpose as a triangle-footprint gather over all angles
//              (a workgroup per 16 x 16 voxel tile and kAdjZT slices, each
//              thread a voxel pair along x and kAdjZT / 2 slices),
//              sinogram segments staged in LDS per angle group by
//              LDS-direct loads
// Positions and interpolation weights are formed in double precision (or as
// single-precision offsets of a few bins from double-precision bases); field
// arithmetic is single precision; costs and long ray sums are carried in
// double, the transpose's sums over angles in two levels of single precision.
#include <algorithm>

#include "holo_internal.hpp"
#include "fft_lds.hpp"

namespace holo {

typedef float f4a8 __attribute__((ext_vector_type(4), aligned(8)));

constexpr int kThreads = 256;

// Threads per row line.  From W = 1024 on a line spans two or more
// wavefronts: one wavefront per 1024-point line would need a private LDS
// line per wavefront, which halves the waves per CU, and that costs more in
// the row passes than their workgroup barriers.
__host__ __device__ constexpr int rows_tl(int W) { return fft_row_threads(W); }
__host__ __device__ constexpr int rows_lpw(int W) { return kThreads / rows_tl(W); }
// Lines (rows, or columns of a column tile) whose TL threads lie in one
// wavefront: their transforms need no workgroup barrier.
__host__ __device__ constexpr bool wave_lines(int TL) { return TL <= 64; }
__host__ __device__ constexpr int cols_tc(int H) { return H >= 2048 ? 4 : (H >= 1024 ? 8 : 16); }
// Pitch of one column line in the column kernels' LDS tile: the padded line
// plus 4, so that the tile loads (8 columns x 4 rows per LDS pass) hit
// distinct banks.
// Padded LDS position of element lt + e TL of a row line (see fpi).
template <int TL>
__device__ __forceinline__ int rowpos(int lp, int lt, int e) {
  return TL % 32 == 0 ? lp + e * (TL + TL / 32) : fpi(lt + e * TL);
}
__host__ __device__ constexpr int col_pitch(int H) { return fft_line_len(H) + 4; }

int rows_per_wg(int W) { return rows_lpw(W); }
int cols_per_wg(int H) { return cols_tc(H); }
bool fft_size_supported(int n) {
  switch (n) {
    case 64: case 128: case 192: case 256: case 384: case 512: case 1024: case 2048:
      return true;
    default:
      return false;
  }
}

// ---------------------------------------------------------------------------
// Demagnification / shift taps (bilinear, free space outside)
// ---------------------------------------------------------------------------

// Sample position of output index idx along one axis: c + m (idx - c) - t.
// The forward resample and its transpose call this same function, so both
// see bit-identical positions and weights.
__device__ __forceinline__ double src_pos(double c, double m, double t, int idx) {
  return c + m * ((double)idx - c) - t;
}

struct AxisTaps {
  int i0, i1;      // clamped in-range indices
  float w0, w1;    // weights (0 for taps outside the grid)
};

__device__ __forceinline__ AxisTaps fwd_taps(double c, double m, double t, int idx, int n) {
  double sp = src_pos(c, m, t, idx);
  double fl = floor(sp);
  int i0 = (int)fl;
  float w = (float)(sp - fl);
  AxisTaps a;
  bool v0 = (i0 >= 0) && (i0 < n);
  bool v1 = (i0 + 1 >= 0) && (i0 + 1 < n);
  a.w0 = v0 ? 1.0f - w : 0.0f;
  a.w1 = v1 ? w : 0.0f;
  a.i0 = v0 ? i0 : 0;
  a.i1 = v1 ? i0 + 1 : 0;
  return a;
}

// phi = 1 + sum of bilinear taps of (psi - 1) inside the grid.
__device__ __forceinline__ float2 sample_phi(const float2* __restrict__ psik, int W,
                                             const AxisTaps& ty, const AxisTaps& tx) {
  float2 a = psik[(size_t)ty.i0 * W + tx.i0];
  float2 b = psik[(size_t)ty.i0 * W + tx.i1];
  float2 c = psik[(size_t)ty.i1 * W + tx.i0];
  float2 d = psik[(size_t)ty.i1 * W + tx.i1];
  float w00 = ty.w0 * tx.w0, w01 = ty.w0 * tx.w1, w10 = ty.w1 * tx.w0, w11 = ty.w1 * tx.w1;
  float re = w00 * (a.x - 1.0f) + w01 * (b.x - 1.0f) + w10 * (c.x - 1.0f) + w11 * (d.x - 1.0f);
  float im = w00 * a.y + w01 * b.y + w10 * c.y + w11 * d.y;
  return make_float2(1.0f + re, im);
}

// Destination indices whose sample position lies within one pixel of source
// index `idx`, with the weight the forward resample gave to `idx` (taps of
// the transpose).  Three candidates cover every such index; unused ones get
// weight 0 and a clamped in-range index.
struct AdjTaps {
  int d[3];
  float w[3];
};

__device__ __forceinline__ AdjTaps adj_taps(double c, double m, double t, int idx, int n) {
  const double pre = ((double)idx - c + t) / m + c;
  const int d0 = (int)floor(pre) - 1;
  AdjTaps a;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int d = d0 + e;
    const bool ok = (d >= 0) && (d < n);
    const double sp = src_pos(c, m, t, d);
    const double fl = floor(sp);
    const int i0 = (int)fl;
    const float w = (float)(sp - fl);
    const float wt = (i0 == idx) ? 1.0f - w : ((i0 + 1 == idx) ? w : 0.0f);
    a.d[e] = ok ? d : 0;
    a.w[e] = ok ? wt : 0.0f;
  }
  return a;
}

__device__ __forceinline__ void shift_of(const DevGeom& g, int kglob, int j, double& ty, double& tx) {
  if (g.shift) {
    const float* s = g.shift + ((size_t)kglob * g.nd + j) * 2;
    ty = (double)s[0];
    tx = (double)s[1];
  } else {
    ty = 0.0;
    tx = 0.0;
  }
}

// Probe shifts (Eq. 9): S_s f is f sampled at (y - s_y, x - s_x) with linear
// interpolation on the periodic grid.  Circular shifts commute with the
// Fresnel propagator, so the shifted probe at plane j is S_s applied to
// Q_j = D_{rho_probe_j} q, and S_s^T = S_{-s}.
__device__ __forceinline__ float2 sample_circ(const float2* __restrict__ f, int H, int W,
                                              double yy, double xx) {
  // positions reduced onto [0, n] first, so any finite shift indexes in range
  yy -= (double)H * floor(yy / (double)H);
  xx -= (double)W * floor(xx / (double)W);
  const double fy = floor(yy), fx = floor(xx);
  const float wy = (float)(yy - fy), wx = (float)(xx - fx);
  int y0 = (int)fy % H, x0 = (int)fx % W;
  y0 += y0 < 0 ? H : 0;
  x0 += x0 < 0 ? W : 0;
  const int y1 = y0 + 1 == H ? 0 : y0 + 1, x1 = x0 + 1 == W ? 0 : x0 + 1;
  const float2 a = f[(size_t)y0 * W + x0], b = f[(size_t)y0 * W + x1];
  const float2 c = f[(size_t)y1 * W + x0], d = f[(size_t)y1 * W + x1];
  const float w00 = (1.f - wy) * (1.f - wx), w01 = (1.f - wy) * wx, w10 = wy * (1.f - wx),
              w11 = wy * wx;
  return make_float2(w00 * a.x + w01 * b.x + w10 * c.x + w11 * d.x,
                     w00 * a.y + w01 * b.y + w10 * c.y + w11 * d.y);
}

// ---------------------------------------------------------------------------
// Row kernels (lines of length W along the detector columns)
// ---------------------------------------------------------------------------

template <int W, bool PS>   // PS: probe shifts set
__global__ __launch_bounds__(kThreads) void k_pass_a(const float2* __restrict__ psi,
                                                     const float2* __restrict__ Q,
                                                     float2* __restrict__ X, DevGeom g,
                                                     int k_first) {
  constexpr int TL = rows_tl(W), LPW = rows_lpw(W), E = W / TL;
  __shared__ float2 s_tw[W];
  __shared__ float2 s_line[LPW][fft_line_len(W)];
  const int line = threadIdx.x / TL, lt = threadIdx.x % TL;
  const int lp = fpi(lt);   // padded position of the thread's first element
  const int z = blockIdx.x * LPW + line;
  const int f = blockIdx.y;
  const int k = f / g.nd, j = f % g.nd;
  for (int i = threadIdx.x; i < W; i += kThreads) s_tw[i] = g.twW[i];

  double ty, tx;
  shift_of(g, k_first + k, j, ty, tx);
  const double m = g.mag[j];
  const AxisTaps tyt = fwd_taps(g.cH, m, ty, z, g.H);
  const float2* psik = psi + (size_t)k * g.H * W;
  const float2* Qrow = Q + ((size_t)j * g.H + z) * W;
  const float* ps = PS ? g.pshift + ((size_t)(k_first + k) * g.nd + j) * 2 : nullptr;
  float2* L = s_line[line];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int s = lt + e * TL;
    const AxisTaps txt = fwd_taps(g.cW, m, tx, s, W);
    float2 qv;
    if constexpr (PS)
      qv = sample_circ(Q + (size_t)j * g.H * W, g.H, W, (double)z - ps[0], (double)s - ps[1]);
    else
      qv = Qrow[s];
    L[rowpos<TL>(lp, lt, e)] = cmul(qv, sample_phi(psik, W, tyt, txt));
  }
  if constexpr (wave_lines(TL)) __syncthreads();   // s_tw
  fft<W, TL, false, true, wave_lines(TL)>(L, s_tw, lt);
  const float2* ch = g.chirpW + (size_t)chirp_det(j) * W;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int s = lt + e * TL;
    L[rowpos<TL>(lp, lt, e)] = cmul(L[rowpos<TL>(lp, lt, e)], ch[s]);
  }
  fft<W, TL, true, true, wave_lines(TL)>(L, s_tw, lt);
  float2* out = X + ((size_t)f * g.H + z) * W;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int s = lt + e * TL;
    out[s] = L[rowpos<TL>(lp, lt, e)];
  }
}

template <int W, bool PS>   // PS: probe shifts set
__global__ __launch_bounds__(kThreads) void k_pass_c(float2* __restrict__ X,
                                                     const float2* __restrict__ psi,
                                                     const float2* __restrict__ Q,
                                                     float2* __restrict__ G,
                                                     float2* __restrict__ Pbuf, DevGeom g,
                                                     int accumulate, int k_first, int Kc) {
  constexpr int TL = rows_tl(W), LPW = rows_lpw(W), E = W / TL;
  __shared__ float2 s_tw[W];
  __shared__ float2 s_line[LPW][fft_line_len(W)];
  const int line = threadIdx.x / TL, lt = threadIdx.x % TL;
  const int lp = fpi(lt);   // padded position of the thread's first element
  const int z = blockIdx.x * LPW + line;
  const int j = blockIdx.y;
  for (int i = threadIdx.x; i < W; i += kThreads) s_tw[i] = g.twW[i];
  const double m = g.mag[j];
  const float2* Qrow = Q + ((size_t)j * g.H + z) * W;
  const float2* ch = g.chirpW + (size_t)chirp_det(j) * W;
  float2* L = s_line[line];
  float2 gacc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) gacc[e] = make_float2(0.f, 0.f);
  if constexpr (wave_lines(TL)) __syncthreads();   // s_tw

  for (int k = 0; k < Kc; ++k) {
    float2* row = X + (((size_t)k * g.nd + j) * g.H + z) * W;
#pragma unroll
    for (int e = 0; e < E; ++e) L[rowpos<TL>(lp, lt, e)] = row[lt + e * TL];
    fft<W, TL, false, true, wave_lines(TL)>(L, s_tw, lt);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int s = lt + e * TL;
      L[rowpos<TL>(lp, lt, e)] = cmulc(L[rowpos<TL>(lp, lt, e)], ch[s]);
    }
    fft<W, TL, true, true, wave_lines(TL)>(L, s_tw, lt);
    double ty, tx;
    shift_of(g, k_first + k, j, ty, tx);
    const AxisTaps tyt = fwd_taps(g.cH, m, ty, z, g.H);
    const float2* psik = psi + (size_t)k * g.H * W;
    const float* ps = PS ? g.pshift + ((size_t)(k_first + k) * g.nd + j) * 2 : nullptr;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int s = lt + e * TL;
      const float2 w = L[rowpos<TL>(lp, lt, e)];
      if (accumulate) {
        const AxisTaps txt = fwd_taps(g.cW, m, tx, s, W);
        const float2 phi = sample_phi(psik, W, tyt, txt);
        const float2 t = cmulc(w, phi);  // conj(phi) w
        if constexpr (PS) {              // shifted probes: summed after the chunk
          Pbuf[(((size_t)k * g.nd + j) * g.H + z) * W + s] = t;
        } else {
          gacc[e].x += t.x;
          gacc[e].y += t.y;
        }
      }
      float2 qv;
      if constexpr (PS)
        qv = sample_circ(Q + (size_t)j * g.H * W, g.H, W, (double)z - ps[0], (double)s - ps[1]);
      else
        qv = Qrow[s];
      row[s] = cmulc(w, qv);             // conj(Q_kj) w
    }
  }
  if (accumulate && !PS) {
    float2* grow = G + ((size_t)j * g.H + z) * W;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int s = lt + e * TL;
      float2 v = grow[s];
      grow[s] = make_float2(v.x + gacc[e].x, v.y + gacc[e].y);
    }
  }
}

template <int W>
__global__ __launch_bounds__(kThreads) void k_rows_prop(PropJobs jobs, DevGeom g) {
  constexpr int TL = rows_tl(W), LPW = rows_lpw(W), E = W / TL;
  __shared__ float2 s_tw[W];
  __shared__ float2 s_line[LPW][fft_line_len(W)];
  const int line = threadIdx.x / TL, lt = threadIdx.x % TL;
  const int lp = fpi(lt);   // padded position of the thread's first element
  const int z = blockIdx.x * LPW + line;
  const PropJob& jb = jobs.job[blockIdx.y];
  for (int i = threadIdx.x; i < W; i += kThreads) s_tw[i] = g.twW[i];
  const float2* in = jb.src + (size_t)z * W;
  float2* L = s_line[line];
#pragma unroll
  for (int e = 0; e < E; ++e) L[rowpos<TL>(lp, lt, e)] = in[lt + e * TL];
  if constexpr (wave_lines(TL)) __syncthreads();   // s_tw
  fft<W, TL, false, true, wave_lines(TL)>(L, s_tw, lt);
  const float2* ch = g.chirpW + (size_t)jb.chirp * W;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int s = lt + e * TL;
    L[rowpos<TL>(lp, lt, e)] = jb.conj ? cmulc(L[rowpos<TL>(lp, lt, e)], ch[s]) : cmul(L[rowpos<TL>(lp, lt, e)], ch[s]);
  }
  fft<W, TL, true, true, wave_lines(TL)>(L, s_tw, lt);
  float2* out = jb.dst + (size_t)z * W;
#pragma unroll
  for (int e = 0; e < E; ++e) out[lt + e * TL] = L[rowpos<TL>(lp, lt, e)];
}

// ---------------------------------------------------------------------------
// Column kernels (lines of length H along the detector rows)
// ---------------------------------------------------------------------------

template <int NT>
__device__ __forceinline__ void block_sum_store(double v, double* out) {
  // butterfly sum within each wave, then the wave sums in order: a fixed
  // summation order, so the result is reproducible bit for bit
  __shared__ double red[NT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) t += red[w];
    *out = t;
  }
}

// Amplitude functional (F2): r = 2 (v - a v/|v|) in place (v/|v| := 0 at
// |v| = 0), returns (|v| - a)^2.  Intensity functional (F1, `a` is then the
// intensity d): r = 4 (|v|^2 - d) v, returns (|v|^2 - d)^2.
__device__ __forceinline__ double residual(float2& v, float a, int functional) {
  if (functional) {
    const double e = (double)fmaf(v.x, v.x, v.y * v.y) - (double)a;
    const float sc = 4.0f * (float)e;
    v = make_float2(sc * v.x, sc * v.y);
    return e * e;
  }
  const float av = sqrtf(v.x * v.x + v.y * v.y);
  const double d = (double)av - (double)a;
  const float sc = av > 0.0f ? 2.0f * (1.0f - a / av) : 2.0f;
  v = make_float2(sc * v.x, sc * v.y);
  return d * d;
}

// Column workgroups are 512 threads (8 waves) so that two of them per CU
// keep 16 waves in flight with the column tile in LDS.  The tile order is
// remapped per XCD: neighbouring column tiles (the two halves of a cache
// line) are read and written through the same L2.
constexpr int kColThreads = 512;

// The dispatcher hands workgroup h of a 1-D grid to XCD h mod 8.  Remap so
// that each XCD walks a contiguous range of logical indices: neighbours in
// logical order then share that XCD's L2.
__device__ __forceinline__ int xcd_logical(int h, int n) {
  const int q = n >> 3, r = n & 7;
  const int x = h & 7, loc = h >> 3;
  return x * q + min(x, r) + loc;
}

template <int H, int MODE, int TC>
__global__ __launch_bounds__(kColThreads) void k_pass_b(const float2* __restrict__ src,
                                                        float2* __restrict__ X,
                                                        const float* __restrict__ amp,
                                                        double* __restrict__ Fpart, DevGeom g,
                                                        int ntiles) {
  constexpr int TLc = kColThreads / TC;
  constexpr int NPT = H * TC / kColThreads;       // tile elements per thread
  constexpr int RS = kColThreads / TC;            // tile rows between a thread's elements
  static_assert(H * TC % kColThreads == 0 && RS % 32 == 0, "column tile");
  constexpr bool kResidual = MODE == kColObj || MODE == kColGrad;
  __shared__ float2 s_tw[H];
  __shared__ float2 s_col[TC][col_pitch(H)];
  const int c = threadIdx.x / TLc, lt = threadIdx.x % TLc;
  const int W = g.W;
  const int L = xcd_logical(blockIdx.x, gridDim.x);
  const int tile = L % ntiles;
  const int s0 = tile * TC;
  const int f = L / ntiles;
  const int j = f % g.nd;
  // Element r of this thread is tile row z0 + r RS, column cc: global
  // offset g0 + r RS W, LDS position l0 + r (RS + RS / 32) of column cc
  // (RS is a multiple of 32, so the padding adds RS / 32 per step).  Every
  // global load of the tile and of the twiddles (and below, of the
  // amplitudes) is issued before the first is used, so their latencies
  // overlap.  The bases are re-made opaque before each phase so that the
  // per-element addresses are not kept live across the transforms.
  const int z0 = threadIdx.x / TC, cc = threadIdx.x % TC;
  const unsigned gstep = (unsigned)(RS * W);
  unsigned g0 = (unsigned)(z0 * W + cc);
  float2* l0 = &s_col[cc][fpi(z0)];
  constexpr int LSTEP = RS + RS / 32;
  const float2* in = (MODE == kColAdj ? src : X) + (size_t)f * H * W + s0;
  float2 t[NPT];
#pragma unroll
  for (int r = 0; r < NPT; ++r) t[r] = in[g0 + r * gstep];
#pragma unroll
  for (int r = 0; r < (H + kColThreads - 1) / kColThreads; ++r) {
    const int i = threadIdx.x + r * kColThreads;
    if (i < H) s_tw[i] = g.twH[i];
  }
#pragma unroll
  for (int r = 0; r < NPT; ++r) l0[r * LSTEP] = t[r];
  float2* Lc = s_col[c];
  const float2* ch = g.chirpH + (size_t)chirp_det(j) * H;
  constexpr bool WL = wave_lines(TLc);
  if (MODE != kColAdj) {
    if constexpr (WL) __syncthreads();   // tile and s_tw
    fft<H, TLc, false, true, WL>(Lc, s_tw, lt);
    for (int zz = lt; zz < H; zz += TLc) Lc[fpi(zz)] = cmul(Lc[fpi(zz)], ch[zz]);
    fft<H, TLc, true, true, WL>(Lc, s_tw, lt);
    __syncthreads();
  }
  if (kResidual) {
    asm volatile("" : "+v"(g0), "+v"(l0));
    const float* a = amp + (size_t)f * H * W + s0;
    float ar[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) ar[r] = a[g0 + r * gstep];
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
      float2 v = l0[r * LSTEP];
      acc += residual(v, ar[r], g.functional);
      l0[r * LSTEP] = v;
    }
    block_sum_store<kColThreads>(acc, Fpart + (size_t)f * ntiles + tile);
  }
  if (MODE == kColGrad || MODE == kColAdj) {
    if constexpr (WL) __syncthreads();   // tile (residual or load) and s_tw
    fft<H, TLc, false, true, WL>(Lc, s_tw, lt);
    for (int zz = lt; zz < H; zz += TLc) Lc[fpi(zz)] = cmulc(Lc[fpi(zz)], ch[zz]);
    fft<H, TLc, true, true, WL>(Lc, s_tw, lt);
    __syncthreads();
  }
  if (MODE != kColObj) {
    asm volatile("" : "+v"(g0), "+v"(l0));
    float2* out = X + (size_t)f * H * W + s0;
#pragma unroll
    for (int r = 0; r < NPT; ++r) out[g0 + r * gstep] = l0[r * LSTEP];
  }
}

template <int H>
__global__ __launch_bounds__(kColThreads) void k_cols_prop(PropJobs jobs, double* __restrict__ Fpart,
                                                           DevGeom g) {
  constexpr int TC = cols_tc(H), TLc = kColThreads / TC;
  __shared__ float2 s_tw[H];
  __shared__ float2 s_col[TC][col_pitch(H)];
  const int c = threadIdx.x / TLc, lt = threadIdx.x % TLc;
  const int W = g.W;
  const int s0 = blockIdx.x * TC;
  const PropJob& jb = jobs.job[blockIdx.y];
  for (int i = threadIdx.x; i < H; i += kColThreads) s_tw[i] = g.twH[i];
  const float2* in = jb.src + s0;
  for (int i = threadIdx.x; i < H * TC; i += kColThreads) {
    const int zz = i / TC, cc = i % TC;
    s_col[cc][fpi(zz)] = in[(size_t)zz * W + cc];
  }
  float2* L = s_col[c];
  const float2* ch = g.chirpH + (size_t)jb.chirp * H;
  constexpr bool WL = wave_lines(TLc);
  if constexpr (WL) __syncthreads();   // tile and s_tw
  fft<H, TLc, false, true, WL>(L, s_tw, lt);
  for (int zz = lt; zz < H; zz += TLc) L[fpi(zz)] = jb.conj ? cmulc(L[fpi(zz)], ch[zz]) : cmul(L[fpi(zz)], ch[zz]);
  fft<H, TLc, true, true, WL>(L, s_tw, lt);
  __syncthreads();
  if (jb.amp) {
    double acc = 0.0;
    const float* a = jb.amp + s0;
    for (int i = threadIdx.x; i < H * TC; i += kColThreads) {
      const int zz = i / TC, cc = i % TC;
      float2 v = s_col[cc][fpi(zz)];
      acc += residual(v, a[(size_t)zz * W + cc], g.functional);
      s_col[cc][fpi(zz)] = v;
    }
    block_sum_store<kColThreads>(acc, Fpart + (size_t)jb.fslot * gridDim.x + blockIdx.x);
    __syncthreads();
  }
  float2* out = jb.dst + s0;
  for (int i = threadIdx.x; i < H * TC; i += kColThreads) {
    const int zz = i / TC, cc = i % TC;
    out[(size_t)zz * W + cc] = s_col[cc][fpi(zz)];
  }
}

// ---------------------------------------------------------------------------
// Padded propagation: a line of n samples is set in the centre of a line of
// 2n (zeros outside), transformed there with the 2n-point transfer row, and
// the centre n samples are kept.  Rows and columns are separable halves of
// the padded 2-D propagation (the setting-in and cutting-out of one axis
// commute with the other axis' transform).
// ---------------------------------------------------------------------------

bool pad_size_supported(int n) { return fft_size_supported(n) && n <= 1024; }
int pad_col_tiles(int H, int W) { return W / cols_tc(2 * H); }

template <int W>
__global__ __launch_bounds__(kThreads) void k_rows_pad(PadJob jb, DevGeom g) {
  constexpr int N2 = 2 * W, TL = rows_tl(N2), LPW = rows_lpw(N2), E = N2 / TL;
  constexpr int OFF = W / 2;
  __shared__ float2 s_tw[N2];
  __shared__ float2 s_line[LPW][fft_line_len(N2)];
  const int line = threadIdx.x / TL, lt = threadIdx.x % TL;
  const int z = blockIdx.x * LPW + line;
  const int f = blockIdx.y;
  for (int i = threadIdx.x; i < N2; i += kThreads) s_tw[i] = g.tw2W[i];
  const float2* in = jb.src + (size_t)f * jb.src_step + (size_t)z * W;
  float2* L = s_line[line];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int n = lt + e * TL;
    L[fpi(n)] = (n >= OFF && n < OFF + W) ? in[n - OFF] : make_float2(0.f, 0.f);
  }
  if constexpr (wave_lines(TL)) __syncthreads();   // s_tw
  fft<N2, TL, false, true, wave_lines(TL)>(L, s_tw, lt);
  const float2* ch = g.chirp2W + (size_t)(jb.chirp0 + f % jb.cmod) * N2;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int n = lt + e * TL;
    L[fpi(n)] = jb.conj ? cmulc(L[fpi(n)], ch[n]) : cmul(L[fpi(n)], ch[n]);
  }
  fft<N2, TL, true, true, wave_lines(TL)>(L, s_tw, lt);
  float2* out = jb.dst + (size_t)f * g.H * W + (size_t)z * W;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int n = lt + e * TL;
    if (n >= OFF && n < OFF + W) out[n - OFF] = L[fpi(n)];
  }
}

template <int H>
__global__ __launch_bounds__(kColThreads) void k_cols_pad(PadJob jb, double* __restrict__ Fpart,
                                                          DevGeom g, int ntiles) {
  constexpr int N2 = 2 * H, TC = cols_tc(N2), TLc = kColThreads / TC;
  constexpr int OFF = H / 2;
  __shared__ float2 s_tw[N2];
  __shared__ float2 s_col[TC][col_pitch(N2)];
  const int c = threadIdx.x / TLc, lt = threadIdx.x % TLc;
  const int W = g.W;
  const int tile = blockIdx.x % ntiles, f = blockIdx.x / ntiles;
  const int s0 = tile * TC;
  const size_t HW = (size_t)H * W;
  for (int i = threadIdx.x; i < N2; i += kColThreads) s_tw[i] = g.tw2H[i];
  const float2* in = jb.src + (size_t)f * jb.src_step + s0;
  for (int i = threadIdx.x; i < N2 * TC; i += kColThreads) {
    const int zz = i / TC, cc = i % TC;
    s_col[cc][fpi(zz)] = (zz >= OFF && zz < OFF + H) ? in[(size_t)(zz - OFF) * W + cc]
                                                     : make_float2(0.f, 0.f);
  }
  float2* L = s_col[c];
  const float2* ch = g.chirp2H + (size_t)(jb.chirp0 + f % jb.cmod) * N2;
  constexpr bool WL = wave_lines(TLc);
  const bool cj = jb.mode == 0 && jb.conj;
  if constexpr (WL) __syncthreads();   // tile and s_tw
  fft<N2, TLc, false, true, WL>(L, s_tw, lt);
  for (int zz = lt; zz < N2; zz += TLc) L[fpi(zz)] = cj ? cmulc(L[fpi(zz)], ch[zz]) : cmul(L[fpi(zz)], ch[zz]);
  fft<N2, TLc, true, true, WL>(L, s_tw, lt);
  __syncthreads();
  if (jb.mode != 0) {
    // residual on the kept centre; the rest is cleared before the adjoint
    double acc = 0.0;
    const float* a = jb.amp + (size_t)f * HW + s0;
    for (int i = threadIdx.x; i < N2 * TC; i += kColThreads) {
      const int zz = i / TC, cc = i % TC;
      float2 v = make_float2(0.f, 0.f);
      if (zz >= OFF && zz < OFF + H) {
        v = s_col[cc][fpi(zz)];
        acc += residual(v, a[(size_t)(zz - OFF) * W + cc], g.functional);
      }
      s_col[cc][fpi(zz)] = v;
    }
    block_sum_store<kColThreads>(acc, Fpart + jb.fslot0 + (size_t)f * ntiles + tile);
    if (jb.mode == 2) return;
    if constexpr (WL) __syncthreads();
    fft<N2, TLc, false, true, WL>(L, s_tw, lt);
    for (int zz = lt; zz < N2; zz += TLc) L[fpi(zz)] = cmulc(L[fpi(zz)], ch[zz]);
    fft<N2, TLc, true, true, WL>(L, s_tw, lt);
    __syncthreads();
  }
  float2* out = jb.dst + (size_t)f * HW + s0;
  for (int i = threadIdx.x; i < H * TC; i += kColThreads) {
    const int zz = i / TC, cc = i % TC;
    out[(size_t)zz * W + cc] = s_col[cc][fpi(zz + OFF)];
  }
}

// x_kj = Q_kj phi_kj for every pixel of a chunk's frames (pass A without
// its row transform).
__global__ __launch_bounds__(kThreads) void k_frames_x(const float2* __restrict__ psi,
                                                       const float2* __restrict__ Q,
                                                       float2* __restrict__ X, DevGeom g,
                                                       int k_first, int Kc) {
  const size_t HW = (size_t)g.H * g.W;
  const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= HW * Kc * g.nd) return;
  const size_t fidx = i / HW;
  const int p = (int)(i % HW);
  const int z = p / g.W, s = p % g.W;
  const int k = (int)(fidx / g.nd), j = (int)(fidx % g.nd);
  double ty, tx;
  shift_of(g, k_first + k, j, ty, tx);
  const double m = g.mag[j];
  const AxisTaps tyt = fwd_taps(g.cH, m, ty, z, g.H);
  const AxisTaps txt = fwd_taps(g.cW, m, tx, s, g.W);
  float2 qv;
  if (g.pshift) {
    const float* ps = g.pshift + ((size_t)(k_first + k) * g.nd + j) * 2;
    qv = sample_circ(Q + (size_t)j * HW, g.H, g.W, (double)z - ps[0], (double)s - ps[1]);
  } else {
    qv = Q[(size_t)j * HW + p];
  }
  X[i] = cmul(qv, sample_phi(psi + (size_t)k * HW, g.W, tyt, txt));
}

// Pass C without its row transform: for every pixel of plane j, over the
// chunk's angles, G_j += conj(phi) w (or conj(phi) w into Pbuf with probe
// shifts) and X := conj(Q_kj) w.
__global__ __launch_bounds__(kThreads) void k_frames_c(float2* __restrict__ X,
                                                       const float2* __restrict__ psi,
                                                       const float2* __restrict__ Q,
                                                       float2* __restrict__ G,
                                                       float2* __restrict__ Pbuf, DevGeom g,
                                                       int accumulate, int k_first, int Kc) {
  const size_t HW = (size_t)g.H * g.W;
  const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= HW * g.nd) return;
  const int j = (int)(i / HW);
  const int p = (int)(i % HW);
  const int z = p / g.W, s = p % g.W;
  const double m = g.mag[j];
  float2 gacc = make_float2(0.f, 0.f);
  for (int k = 0; k < Kc; ++k) {
    float2* xp = X + ((size_t)k * g.nd + j) * HW + p;
    const float2 w = *xp;
    double ty, tx;
    shift_of(g, k_first + k, j, ty, tx);
    if (accumulate) {
      const AxisTaps tyt = fwd_taps(g.cH, m, ty, z, g.H);
      const AxisTaps txt = fwd_taps(g.cW, m, tx, s, g.W);
      const float2 t = cmulc(w, sample_phi(psi + (size_t)k * HW, g.W, tyt, txt));
      if (g.pshift) {
        Pbuf[((size_t)k * g.nd + j) * HW + p] = t;
      } else {
        gacc.x += t.x;
        gacc.y += t.y;
      }
    }
    float2 qv;
    if (g.pshift) {
      const float* ps = g.pshift + ((size_t)(k_first + k) * g.nd + j) * 2;
      qv = sample_circ(Q + (size_t)j * HW, g.H, g.W, (double)z - ps[0], (double)s - ps[1]);
    } else {
      qv = Q[(size_t)j * HW + p];
    }
    *xp = cmulc(w, qv);
  }
  if (accumulate && !g.pshift) {
    const float2 v = G[i];
    G[i] = make_float2(v.x + gacc.x, v.y + gacc.y);
  }
}

// ---------------------------------------------------------------------------
// Pass D: transpose of the demagnification, summed over planes, and the
// chain rule through psi = exp(i kappa p).
// ---------------------------------------------------------------------------

// Angles per pass-D workgroup: without object shifts the taps do not depend
// on the angle, so they are formed once for all of them.
constexpr int kPassDAngles = 4;

__global__ __launch_bounds__(kThreads) void k_pass_d(const float2* __restrict__ X,
                                                     const float2* __restrict__ psi,
                                                     float2* __restrict__ S, DevGeom g,
                                                     int k_first, int Kc) {
  // A workgroup covers 16 rows x 16 padded bins, bins fastest, of the
  // sinogram S[k][z][kAdjPad + s] (rows padded by kAdjPad zero bins on each
  // side) for kPassDAngles consecutive angles.  Workgroups over the padding
  // write its zeros.  The transposed resampling is separable, so its taps
  // are formed once per workgroup (once per angle with shifts): per plane,
  // the row taps of each of the 16 rows and the column taps of each of the
  // 16 bins.  Of the three candidates of an axis at most two adjacent ones
  // carry weight (the magnifications are >= 1, so the forward samples of
  // neighbouring destinations are at least one pixel apart), and only those
  // two are kept: four unconditional loads per plane and pixel.
  constexpr int SC = 16, ZR = kThreads / SC;
  static_assert(kMaxDist * 2 * SC <= kThreads, "one tap set per thread");
  __shared__ int s_d[kMaxDist][2 * SC][2];
  __shared__ float s_w[kMaxDist][2 * SC][2];
  const int H = g.H, W = g.W, Wp = sino_row(W);
  const int nsb = Wp / SC;
  const int z0 = (blockIdx.x / nsb) * ZR, sp0 = (blockIdx.x % nsb) * SC;
  const int r = threadIdx.x / SC, c = threadIdx.x % SC;
  const int z = z0 + r, sp = sp0 + c;
  const int s = sp - kAdjPad;
  const bool inside = s >= 0 && s < W;
  const int kb = blockIdx.y * kPassDAngles, ke = min(kb + kPassDAngles, Kc);
  for (int k = kb; k < ke; ++k) {
    if (k == kb || g.shift) {   // uniform over the workgroup
      if (k != kb) __syncthreads();   // the previous angle's taps are read
      if ((int)threadIdx.x < g.nd * 2 * SC) {
        // thread (j, e): plane j; e < 16 the taps of row z0 + e, else those
        // of bin sp0 + e - 16 (none for bins in the padding)
        const int j = threadIdx.x / (2 * SC), e = threadIdx.x % (2 * SC);
        double ty, tx;
        shift_of(g, k_first + k, j, ty, tx);
        const double m = g.mag[j];
        AdjTaps t;
        if (e < SC) {
          t = adj_taps(g.cH, m, ty, z0 + e, H);
        } else {
          const int sb = sp0 + e - SC - kAdjPad;
          if (sb >= 0 && sb < W) {
            t = adj_taps(g.cW, m, tx, sb, W);
          } else {
#pragma unroll
            for (int q = 0; q < 3; ++q) { t.d[q] = 0; t.w[q] = 0.f; }
          }
        }
        // the weighted pair: (0, 1) if candidate 0 has weight (candidate 2,
        // two destinations further on, then has none), else (1, 2)
        const int e0 = t.w[0] != 0.0f ? 0 : 1;
#pragma unroll
        for (int q = 0; q < 2; ++q) { s_d[j][e][q] = t.d[e0 + q]; s_w[j][e][q] = t.w[e0 + q]; }
      }
      __syncthreads();
    }
    float2* out = S + ((size_t)k * H + z) * Wp + sp;
    if (!inside) {
      *out = make_float2(0.f, 0.f);
      continue;
    }
    float ax = 0.f, ay = 0.f;
    for (int j = 0; j < g.nd; ++j) {
      const float2* Xj = X + ((size_t)k * g.nd + j) * H * W;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const float wz = s_w[j][r][a];
        const float2* Xr = Xj + (size_t)s_d[j][r][a] * W;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const float wt = wz * s_w[j][SC + c][b];
          const float2 v = Xr[s_d[j][SC + c][b]];   // in range; weight 0 if unused
          ax += wt * v.x;
          ay += wt * v.y;
        }
      }
    }
    const float2 ps = psi[((size_t)k * H + z) * W + s];
    // conj(psi) g
    const float cx = ps.x * ax + ps.y * ay;
    const float cy = ps.x * ay - ps.y * ax;
    // -i kappa (cx + i cy) = kappa cy - i kappa cx
    *out = make_float2(g.kappa * cy, -g.kappa * cx);
  }
}

// Z-blocked copies of the volume for the ray sums: ub[z / ZT][y][P + x][z % ZT]
// (walks along y) and uTb[z / ZT][x][P + y][z % ZT] (walks along x, i.e. the
// x/y-transposed volume), rows padded by P = kFwdPad zero columns on each
// side.  A workgroup moves a 16 x 16 x ZT brick; the workgroups at the
// first and last brick column also clear the padding of their 16 rows.
__global__ __launch_bounds__(kThreads) void k_block_volume(const float2* __restrict__ u,
                                                           float2* __restrict__ ub,
                                                           float2* __restrict__ uTb, int W) {
  constexpr int ZT = kVolZB, P = kFwdPad;
  __shared__ float2 brick[ZT][16][17];
  const int nt = W / 16, Wf = vol_row(W);
  const int x0 = (blockIdx.x % nt) * 16, y0 = (blockIdx.x / nt) * 16;
  const int zb = blockIdx.y;
  const size_t WW = (size_t)W * W, WWf = (size_t)W * Wf;
  // read along x (contiguous)
  for (int i = threadIdx.x; i < ZT * 256; i += kThreads) {
    const int xx = i & 15, yy = (i >> 4) & 15, zz = i >> 8;
    brick[zz][yy][xx] = u[(size_t)(zb * ZT + zz) * WW + (size_t)(y0 + yy) * W + x0 + xx];
  }
  __syncthreads();
  float2* bb = ub + (size_t)zb * WWf * ZT;
  float2* tb = uTb ? uTb + (size_t)zb * WWf * ZT : nullptr;
  // write with z fastest (contiguous 128-byte runs)
  for (int i = threadIdx.x; i < ZT * 256; i += kThreads) {
    const int zz = i % ZT, p = i / ZT;
    const int a = p & 15, b = p >> 4;
    bb[((size_t)(y0 + b) * Wf + P + x0 + a) * ZT + zz] = brick[zz][b][a];
    if (tb) tb[((size_t)(x0 + b) * Wf + P + y0 + a) * ZT + zz] = brick[zz][a][b];
  }
  // padding: rows y0..y0+15 of ub (brick column 0 / last) and rows
  // x0..x0+15 of uTb (brick row 0 / last)
  const float2 zero = make_float2(0.f, 0.f);
  const bool lo = x0 == 0, hi = x0 == W - 16;
  if (lo || hi) {
    for (int i = threadIdx.x; i < 16 * P * ZT; i += kThreads) {
      const int zz = i % ZT, c = (i / ZT) % P, r = i / (ZT * P);
      const int col = lo ? c : P + W + c;
      bb[((size_t)(y0 + r) * Wf + col) * ZT + zz] = zero;
    }
  }
  const bool tlo = y0 == 0, thi = y0 == W - 16;
  if (tb && (tlo || thi)) {
    for (int i = threadIdx.x; i < 16 * P * ZT; i += kThreads) {
      const int zz = i % ZT, c = (i / ZT) % P, r = i / (ZT * P);
      const int col = tlo ? c : P + W + c;
      tb[((size_t)(x0 + r) * Wf + col) * ZT + zz] = zero;
    }
  }
}

// ---------------------------------------------------------------------------
// Joseph ray sums and their transpose
// ---------------------------------------------------------------------------

// Forward.  A workgroup owns up to kFwdNA consecutive angles of one walk
// direction (one wave per angle), NB (16, or 8 for plans whose angle windows
// spread too far for 16) consecutive bins and kFwdZT slices.
// Within a wave, 16 consecutive lanes cover the 64 slices of one group of NB/4
// consecutive bins: lane l takes the slice pairs (2 (l % 16), + 1) and
// (32 + 2 (l % 16), + 1), so one tap position and weight serve 4 slices and
// each tap of a pair is one 16-byte LDS read.  The workgroup walks the rows
// of the volume one at a time: each row's column window that all its rays
// cross (shared by the angles of the group) is copied straight from memory
// into LDS, [column][slice], by LDS-direct loads two rows ahead of use
// (three row buffers), so staging costs no registers and no LDS writes by
// the waves.  The 16 lanes of one LDS pass read the 256 contiguous bytes of
// one column: free of bank conflicts.  Angles that walk along x read the
// x/y-transposed volume, so both walk directions use the same code.  The
// host groups angles so that every window fits.
template <int NB>
__global__ __launch_bounds__(kThreads, 2) void k_radon_fwd(const float2* __restrict__ u,
                                                         const float2* __restrict__ uT,  // z-blocked
                                                         float2* __restrict__ psi, DevGeom g,
                                                         const double* __restrict__ ang,
                                                         const int2* __restrict__ groups,
                                                         int g0, int ngroups, int c0, int c1) {
  constexpr int ZT = kFwdZT, SEG = kFwdSeg, ZB = kVolZB;
  constexpr int BPT = NB / 4;                       // bins per thread
  constexpr int NBUF = 3;                           // row buffers (loads run 2 rows ahead)
  constexpr int ROWF2 = SEG * ZT;                   // float2 per staged row
  constexpr int LPW = ROWF2 / (4 * 128);            // LDS-direct loads (16 B per lane) per wave per row
  constexpr int C4 = ZT / 2;                        // float4 per staged column
  static_assert(ZT == 64 && (NB == 16 || NB == 8) && LPW == 4 && kThreads == 256, "tiling");
  __shared__ float4 tile4[NBUF * ROWF2 / 2];
  __shared__ short s_xl[kMaxW];
  const int W = g.W, H = g.H;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int pz = lane & 15, bg = lane >> 4;
  // logical order: angle group fastest, then bin block, then slice block,
  // so the groups reading the same windows run together on one XCD
  const int L = xcd_logical(blockIdx.x, gridDim.x);
  const int gi = L % ngroups, rest = L / ngroups;
  const int nbb = W / NB;
  const int sb = (rest % nbb) * NB;
  const int s0 = sb + bg * BPT;                     // first bin of this thread
  const int z0 = (rest / nbb) * ZT;
  const int2 grp = groups[g0 + gi];
  const int gf = max(grp.x, c0), gl = min(grp.x + grp.y, c1);
  const int na = gl - gf;
  const bool active = wave < na;
  const int k = active ? gf + wave : gf;
  const double* aw = ang + (size_t)k * kAngleStride;
  const float2* vol = (aw[kBranch] != 0.0) ? uT : u;
  const double B = aw[kB], D = aw[kD];
  const double fA = aw[kA] + (double)s0 * B;
  const float Bf = (float)B;
  // Range of the per-row base that keeps every tap of the thread's bins and
  // its right neighbour inside the staged window.  Inside the volume the
  // host's grouping keeps every tap at least one column inside the window,
  // so the clamp changes nothing there; a window moved into the zero
  // padding reads zeros wherever the taps land.
  const float span = (float)(BPT - 1) * Bf;
  const float rel_lo = fmaxf(0.0f, -span), rel_hi = (float)(SEG - 1) - fmaxf(0.0f, span) - 0.01f;

  // window start of every row: lowest tap over the group's angles and the
  // block's end bins, minus one column of margin for rounding
  for (int r = threadIdx.x; r < W; r += kThreads) {
    double mn = 1e300;
    for (int a = 0; a < na; ++a) {
      const double* ap = ang + (size_t)(gf + a) * kAngleStride;
      const double fr = ap[kA] + (double)r * ap[kD];
      mn = fmin(mn, fmin(fr + (double)sb * ap[kB], fr + (double)(sb + NB - 1) * ap[kB]));
    }
    // a window wholly outside the volume is moved into the zero padding
    s_xl[r] = (short)min(max((int)floor(mn) - 1, -kFwdPad), W + kFwdPad - SEG);
  }
  __syncthreads();

  // The volume copies are slice-blocked and padded, vol[z / ZB][row][P + col][z % ZB].
  // Load i of wave w moves 1 KB: lane l brings slices 2 (l % 8) and
  // 2 (l % 8) + 1 of slice block (l / 8) % 4 of column 8 w + 2 i + l / 32,
  // which is where the [column][slice] row layout wants them (lane l lands
  // at byte 16 l of the load's 1 KB).
  const int Wf = vol_row(W);
  const size_t plane = (size_t)W * Wf * ZB;
  const float2* vl = vol + (size_t)(z0 / ZB + ((lane >> 3) & 3)) * plane +
                     (size_t)(kFwdPad + 8 * wave + (lane >> 5)) * ZB + 2 * (lane & 7);
  // The loads are issued as inline assembly: the compiler does not track
  // them, so it adds no waits of its own; the loop below waits for them
  // explicitly (vector-memory counter) before the barrier that publishes a
  // row.  M0 holds the wave's LDS destination of each load.
  const unsigned lds0 = (unsigned)(uintptr_t)(__attribute__((address_space(3))) float4*)tile4;
  auto issue = [&](int y) {
    const int xl = __builtin_amdgcn_readfirstlane((int)s_xl[y]);
    const float2* row = vl + ((size_t)y * Wf + xl) * ZB;
    const unsigned dst = __builtin_amdgcn_readfirstlane(
        lds0 + (unsigned)(((y % NBUF) * (ROWF2 / 2) + wave * (LPW * 64)) * 16));
#pragma unroll
    for (int i = 0; i < LPW; ++i)
      asm volatile(
          "s_mov_b32 m0, %0\n\t"
          "s_nop 0\n\t"
          "global_load_lds_dwordx4 %1, off"
          :
          : "s"(dst + 1024u * i), "v"(row + 2 * i * ZB)
          : "memory", "m0");
  };

  // accumulators: [bin][slice e] with slice 32 (e / 2) + 2 pz + e % 2
  float ax[BPT][4], ay[BPT][4];
  double ox[BPT][4], oy[BPT][4];
#pragma unroll
  for (int b = 0; b < BPT; ++b)
#pragma unroll
    for (int e = 0; e < 4; ++e) { ax[b][e] = ay[b][e] = 0.f; ox[b][e] = oy[b][e] = 0.0; }

  issue(0);
  if (W > 1) issue(1);
  for (int y = 0; y < W; ++y) {
    // this wave's loads of row y are complete (those of row y + 1 may be in
    // flight) and its LDS reads of row y - 1 have returned; the barrier then
    // publishes row y of every wave and retires row y - 1, whose buffer the
    // loads of row y + 2 reuse
    if (y + 1 < W) asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)" ::"n"(LPW) : "memory");
    else asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (y + 2 < W) issue(y + 2);
    if (active) {
      // tap position of the thread's first bin relative to the window, in
      // double precision; the other bins add b B (< 4 sqrt(2))
      float rel = (float)(fA + (double)y * D - (double)s_xl[y]);
      rel = fminf(fmaxf(rel, rel_lo), rel_hi);
      int tb = (y % NBUF) * (ROWF2 / 2) + pz;
      asm volatile("" : "+v"(tb));                     // one base register per row
      const float4* tr = tile4 + tb;
      // software pipeline: the taps of bin b + 1 are requested before bin b
      // is accumulated
      float4 v[BPT][2][2];                             // [bin][pair][tap]
      auto fetch_bin = [&](int b) {
        const float q = fmaf((float)b, Bf, rel);          // >= 0, < SEG - 1
        const float4* tp = tr + (int)q * C4;             // truncation = floor here
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          v[b][p][0] = tp[16 * p];
          v[b][p][1] = tp[C4 + 16 * p];
        }
      };
      fetch_bin(0);
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
        if (b + 1 < BPT) fetch_bin(b + 1);
        const float w1 = __builtin_amdgcn_fractf(fmaf((float)b, Bf, rel)), w0 = 1.0f - w1;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const float4 t0 = v[b][p][0], t1 = v[b][p][1];
          ax[b][2 * p] = fmaf(w1, t1.x, fmaf(w0, t0.x, ax[b][2 * p]));
          ay[b][2 * p] = fmaf(w1, t1.y, fmaf(w0, t0.y, ay[b][2 * p]));
          ax[b][2 * p + 1] = fmaf(w1, t1.z, fmaf(w0, t0.z, ax[b][2 * p + 1]));
          ay[b][2 * p + 1] = fmaf(w1, t1.w, fmaf(w0, t0.w, ay[b][2 * p + 1]));
        }
      }
      if ((y & 31) == 31) {
#pragma unroll
        for (int b = 0; b < BPT; ++b)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            ox[b][e] += (double)ax[b][e];
            oy[b][e] += (double)ay[b][e];
            ax[b][e] = ay[b][e] = 0.f;
          }
      }
    }
  }
  if (!active) return;
  const double scale = aw[kScale];
  const double kap = (double)g.kappa;
  const double twopi = 6.283185307179586476925;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float2 o[BPT];
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      const double px = (ox[b][e] + (double)ax[b][e]) * scale;
      const double py = (oy[b][e] + (double)ay[b][e]) * scale;
      double ph = kap * px;
      ph -= twopi * rint(ph / twopi);
      float sn, cs;
      sincosf((float)ph, &sn, &cs);
      const float mag = expf((float)(-kap * py));
      o[b] = make_float2(mag * cs, mag * sn);
    }
    // the thread's BPT bins of one slice are 8 BPT contiguous bytes
    const int z = z0 + 32 * (e >> 1) + 2 * pz + (e & 1);
    float4* dst = reinterpret_cast<float4*>(psi + ((size_t)(k - c0) * H + z) * W + s0);
#pragma unroll
    for (int b = 0; b < BPT; b += 2) dst[b / 2] = make_float4(o[b].x, o[b].y, o[b + 1].x, o[b + 1].y);
  }
}

// Transpose.  A workgroup owns a 16 x 16 voxel tile and kAdjZT slices; a
// thread owns a voxel pair along x and half of the slices (kAdjZT / 2).  It
// loops over all angles in groups of kAdjNA (one wave loads each angle of a
// group): the kAdjSeg bins of each slice that the tile projects onto are
// copied straight from the sinogram into LDS, [angle][slice][bin], by
// LDS-direct loads one group ahead of use (two group buffers); per slice a
// thread then reads the three consecutive bins that carry both voxels'
// weights.  The lanes of a wave read different bins of one 256-byte bin
// row: no bank conflicts.  Sinogram rows are zero-padded by kAdjPad bins, so a segment
// is read without bounds checks.  A voxel projecting to fractional bin q
// takes max(0, 1 - |i - q| / h) / h of bin i (h = max(|cos|, |sin|)) --
// exactly the weight Joseph's interpolation gave it.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_radon_adj(const float2* __restrict__ S,
                                                         float2* __restrict__ gu, DevGeom g,
                                                         const double* __restrict__ ang,
                                                         int K) {
  constexpr int ZT = kAdjZT, NA = kAdjNA, SEG = kAdjSeg, TW = kAdjWin;
  constexpr int NBUF = 2;                           // group buffers (loads run 1 group ahead)
  constexpr int GF2 = NA * ZT * SEG;                // float2 per staged group
  constexpr int LPW = ZT * SEG / 128;               // LDS-direct loads (1 KB) per wave per group
  static_assert(NA == kThreads / 64 && SEG == 32 && LPW == 4 && TW % NA == 0 && kAdjPad >= SEG,
                "staging layout");
  __shared__ float4 tile4[NBUF * GF2 / 2];
  // Per-angle set-up for a window of TW angles, double-buffered by window
  // parity: first staged bin, fractional bin of the tile corner relative to
  // it, cos, sin, 1/h and 1/h^2.
  __shared__ int s_sl[2][TW];
  __shared__ float s_f0[2][TW], s_c[2][TW], s_s[2][TW], s_ih[2][TW], s_ih2[2][TW];
  const float2* tile = reinterpret_cast<const float2*>(tile4);
  const int W = g.W, H = g.H, Wp = sino_row(W);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // logical order: tile x fastest, then tile y, then slice block
  const int L = xcd_logical(blockIdx.x, gridDim.x);
  const int nt = W / 16;
  const int x0 = (L % nt) * 16, y0 = ((L / nt) % nt) * 16;
  // thread: voxel pair (x, x + 1), x = x0 + 2 px, row y0 + dy, and the 8
  // slices of slice group sg of the block
  const int px = threadIdx.x & 7, dy = (threadIdx.x >> 3) & 15, sg = threadIdx.x >> 7;
  const int x = x0 + 2 * px, y = y0 + dy;
  const int z0 = (L / (nt * nt)) * ZT;
  const double X0 = (double)x0 - g.cW, X1 = X0 + 15.0;
  const double Y0 = (double)y0 - g.cW, Y1 = Y0 + 15.0;

  // Set-up of angle w * TW + t for threads t < TW, in double precision: the
  // first staged bin is the lowest projection of the tile's corners minus two
  // or three bins of margin (even, so each lane's bin pair is 16-byte
  // aligned), moved into [-kAdjPad, W + kAdjPad - SEG] (a segment
  // outside that range lies wholly off the detector, and the padding it is
  // moved to holds zeros); a voxel's fractional bin relative to it is
  // f0 + dx cos + dy sin, a small number that single precision holds to
  // ~1e-6 of a bin.
  auto setup_window = [&](int w) {
    const int slot = w & 1, t = threadIdx.x;
    if (t < TW) {
      const int kk = min(w * TW + t, K - 1);
      const double* ap = ang + (size_t)kk * kAngleStride;
      const double C = ap[kCos], Sn = ap[kSin], ih = ap[kInvH];
      const double q0 = g.cW + X0 * C + Y0 * Sn;
      int sl = (int)floor(g.cW + fmin(X0 * C, X1 * C) + fmin(Y0 * Sn, Y1 * Sn)) - 2;
      sl -= sl & 1;                                     // even: 16-byte aligned bin pairs
      sl = min(max(sl, -kAdjPad), W + kAdjPad - SEG);
      s_sl[slot][t] = sl;
      s_f0[slot][t] = (float)(q0 - (double)sl);
      s_c[slot][t] = (float)C;
      s_s[slot][t] = (float)Sn;
      s_ih[slot][t] = (float)ih;
      s_ih2[slot][t] = (float)(ih * ih);
    }
  };

  // The sinogram is S[k][z][kAdjPad + bin].  Load i of wave a (angle a of the
  // group) moves 1 KB: lane l brings bins 2 (l % 16) and 2 (l % 16) + 1 of
  // the segment of slice 4 i + l / 16, which lands at byte 16 l of the
  // load's 1 KB -- the [slice][bin] layout of that angle.  Issued as inline
  // assembly (M0 = LDS destination) so the compiler adds no waits of its
  // own; the loop waits for them explicitly.
  const size_t HWp = (size_t)H * Wp;
  const float2* Sl = S + (size_t)(z0 + (lane >> 4)) * Wp + kAdjPad + 2 * (lane & 15);
  const unsigned lds0 = (unsigned)(uintptr_t)(__attribute__((address_space(3))) float4*)tile4;
  auto issue = [&](int gidx) {
    const int k0 = gidx * NA;
    const int kk = min(k0 + wave, K - 1);                // past the end: never read back
    const int sl = __builtin_amdgcn_readfirstlane(s_sl[(k0 / TW) & 1][k0 % TW + wave]);
    const float2* src = Sl + (size_t)kk * HWp + sl;
    const unsigned dst = __builtin_amdgcn_readfirstlane(
        lds0 + (unsigned)((((gidx % NBUF) * GF2) + wave * ZT * SEG) * 8));
#pragma unroll
    for (int i = 0; i < LPW; ++i)
      asm volatile(
          "s_mov_b32 m0, %0\n\t"
          "s_nop 0\n\t"
          "global_load_lds_dwordx4 %1, off"
          :
          : "s"(dst + 1024u * i), "v"(src + (size_t)4 * i * Wp)
          : "memory", "m0");
  };

  constexpr int ZS = ZT / 2;                        // slices per thread
  float ax[2][ZS], ay[2][ZS];
  float ox[2][ZS], oy[2][ZS];
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int i = 0; i < ZS; ++i) { ax[v][i] = ay[v][i] = 0.f; ox[v][i] = oy[v][i] = 0.f; }

  const int ng = (K + NA - 1) / NA;
  constexpr int GPW = TW / NA;                      // groups per set-up window
  setup_window(0);
  __syncthreads();
  issue(0);
  for (int gi = 0; gi < ng; ++gi) {
    const int k0 = gi * NA;
    const int na = min(NA, K - k0);
    // this wave's loads of group gi are complete and its LDS reads of group
    // gi - 1 have returned; the barrier publishes group gi of every wave,
    // retires group gi - 1 (whose buffer the loads of gi + 1 reuse) and the
    // set-up window written below
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (gi + 1 < ng) issue(gi + 1);
    // the next window's set-up, written two groups before its first group
    // is issued, into the slot of the window before the current one
    if ((gi + 2) % GPW == 0 && (gi + 2) * NA < K) setup_window((gi + 2) / GPW);
    const int slot = (k0 / TW) & 1, base = k0 % TW;
    const float2* gb = tile + (gi % NBUF) * GF2;
    for (int a = 0; a < na; ++a) {
      // the pair's fractional bins q and q + cos; every bin with a nonzero
      // weight for either voxel (|i - q| < h <= 1) is one of jm .. jm + 2,
      // jm = floor(min of the two), and its weight is the footprint
      // max(0, 1 - |i - q| / h) / h = max(0, 1/h - |i - q| / h^2)
      const float ih = s_ih[slot][base + a], ih2 = s_ih2[slot][base + a];
      const float c = s_c[slot][base + a];
      const float qa = fmaf((float)dy, s_s[slot][base + a],
                            fmaf((float)(2 * px), c, s_f0[slot][base + a]));
      const float qb = qa + c;
      const float fl = floorf(fminf(qa, qb));
      const int jm = min(max((int)fl, 0), SEG - 3);
      float wt[2][3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float bin = (float)(jm + k);        // the bins actually read
        wt[0][k] = fmaxf(0.0f, fmaf(-fabsf(bin - qa), ih2, ih));
        wt[1][k] = fmaxf(0.0f, fmaf(-fabsf(bin - qb), ih2, ih));
      }
      const float2* tp = gb + a * ZT * SEG + sg * ZS * SEG + jm;
      // software pipeline: the three bins of slice i + LA are requested
      // before slice i is accumulated
      constexpr int LA = 3;
      static_assert(ZS == 8, "slice group");
      float2 r[ZS][3];
      auto fetch = [&](int i) {
        const float2* t = tp + i * SEG;
        r[i][0] = t[0];
        r[i][1] = t[1];
        r[i][2] = t[2];
      };
#pragma unroll
      for (int i = 0; i < LA; ++i) fetch(i);
#pragma unroll
      for (int i = 0; i < ZS; ++i) {
        if (i + LA < ZS) fetch(i + LA);
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          ax[v][i] = fmaf(wt[v][2], r[i][2].x, fmaf(wt[v][1], r[i][1].x, fmaf(wt[v][0], r[i][0].x, ax[v][i])));
          ay[v][i] = fmaf(wt[v][2], r[i][2].y, fmaf(wt[v][1], r[i][1].y, fmaf(wt[v][0], r[i][0].y, ay[v][i])));
        }
      }
    }
    // two-level single-precision sums: partials of up to 8 NA angles are
    // added into the outer sums
    if ((gi & 7) == 7 || gi + 1 >= ng) {
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int i = 0; i < ZS; ++i) {
          ox[v][i] += ax[v][i];
          oy[v][i] += ay[v][i];
          ax[v][i] = ay[v][i] = 0.f;
        }
    }
  }
  const size_t WW = (size_t)W * W;
#pragma unroll
  for (int i = 0; i < ZS; ++i) {
    float4* o = reinterpret_cast<float4*>(gu + (size_t)(z0 + sg * ZS + i) * WW + (size_t)y * W + x);
    *o = make_float4(ox[0][i], oy[0][i], ox[1][i], oy[1][i]);
  }
}

__global__ void k_fill(float2* __restrict__ p, size_t n, float2 value) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = value;
}

__global__ void k_sum_frames(const float2* __restrict__ G, int nd, const float2* __restrict__ extra,
                             float2* __restrict__ out, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    float2 acc = extra ? extra[i] : make_float2(0.f, 0.f);
    for (int j = 0; j < nd; ++j) {
      const float2 v = G[(size_t)j * n + i];
      acc.x += v.x;
      acc.y += v.y;
    }
    out[i] = acc;
  }
}

// Deterministic single-workgroup sum of double partials.
// Workgroup b sums parts[b per, min(n, (b + 1) per)) into out[b]; a fixed
// partition and order, so the total is reproducible bit for bit.
__global__ __launch_bounds__(kThreads) void k_reduce_sum(const double* __restrict__ parts, size_t n,
                                                         size_t per, double* __restrict__ out) {
  const size_t lo = (size_t)blockIdx.x * per, hi = min(n, lo + per);
  double acc = 0.0;
  for (size_t i = lo + threadIdx.x; i < hi; i += kThreads) acc += parts[i];
  block_sum_store<kThreads>(acc, out + blockIdx.x);
}

// ---------------------------------------------------------------------------
// Solver vector operations (complex64 vectors, double-precision products)
// ---------------------------------------------------------------------------

// Workgroup b sums Re(conj(a) b) over [b per, min(n, (b + 1) per)).
__global__ __launch_bounds__(kThreads) void k_dot_re(const float2* __restrict__ a,
                                                     const float2* __restrict__ b, size_t n,
                                                     size_t per, double* __restrict__ parts) {
  const size_t lo = (size_t)blockIdx.x * per, hi = min(n, lo + per);
  double acc = 0.0;
  for (size_t i = lo + threadIdx.x; i < hi; i += kThreads) {
    const float2 x = a[i], y = b[i];
    acc += (double)x.x * (double)y.x + (double)x.y * (double)y.y;
  }
  block_sum_store<kThreads>(acc, parts + blockIdx.x);
}

// out = x + t e
__global__ void k_axpy(const float2* __restrict__ x, const float2* __restrict__ e, float t,
                       float2* __restrict__ out, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    const float2 a = x[i], d = e[i];
    out[i] = make_float2(fmaf(t, d.x, a.x), fmaf(t, d.y, a.y));
  }
}

// eta = -g + beta eta, or eta = -g when `restart` (eta is then not read)
__global__ void k_cg_dir(const float2* __restrict__ g, float2* __restrict__ eta, float beta,
                         int restart, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    const float2 gv = g[i];
    if (restart) {
      eta[i] = make_float2(-gv.x, -gv.y);
    } else {
      const float2 e = eta[i];
      eta[i] = make_float2(fmaf(beta, e.x, -gv.x), fmaf(beta, e.y, -gv.y));
    }
  }
}

__global__ void k_real_to_c64(const float* __restrict__ a, float2* __restrict__ out, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) out[i] = make_float2(a[i], 0.f);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

#define HOLO_FOR_SIZES(X) X(64) X(128) X(192) X(256) X(384) X(512) X(1024) X(2048)

hipError_t launch_rows_prop(const DevGeom& g, const PropJobs& jobs, hipStream_t st) {
  if (jobs.n == 0) return hipSuccess;
  const dim3 grid(g.H / rows_per_wg(g.W), jobs.n);
  switch (g.W) {
#define CASE(N) case N: k_rows_prop<N><<<grid, kThreads, 0, st>>>(jobs, g); break;
    HOLO_FOR_SIZES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cols_prop(const DevGeom& g, const PropJobs& jobs, double* Fpart, hipStream_t st) {
  if (jobs.n == 0) return hipSuccess;
  const dim3 grid(g.W / cols_per_wg(g.H), jobs.n);
  switch (g.H) {
#define CASE(N) case N: k_cols_prop<N><<<grid, kColThreads, 0, st>>>(jobs, Fpart, g); break;
    HOLO_FOR_SIZES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define HOLO_FOR_PAD_SIZES(X) X(64) X(128) X(192) X(256) X(384) X(512) X(1024)

hipError_t launch_rows_pad(const DevGeom& g, const PadJob& jb, hipStream_t st) {
  if (jb.nframes == 0) return hipSuccess;
  if (!g.tw2W || !g.chirp2W) return hipErrorInvalidValue;
  const dim3 grid(g.H / rows_lpw(2 * g.W), jb.nframes);
  switch (g.W) {
#define CASE(N) case N: k_rows_pad<N><<<grid, kThreads, 0, st>>>(jb, g); break;
    HOLO_FOR_PAD_SIZES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cols_pad(const DevGeom& g, const PadJob& jb, double* Fpart, hipStream_t st) {
  if (jb.nframes == 0) return hipSuccess;
  if (!g.tw2H || !g.chirp2H || (jb.mode != 0 && (!jb.amp || !Fpart))) return hipErrorInvalidValue;
  const int ntiles = pad_col_tiles(g.H, g.W);
  const unsigned n = (unsigned)ntiles * (unsigned)jb.nframes;
  switch (g.H) {
#define CASE(N) case N: k_cols_pad<N><<<n, kColThreads, 0, st>>>(jb, Fpart, g, ntiles); break;
    HOLO_FOR_PAD_SIZES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// dst[r][s] = src[r * src_pitch + s] for rows r < rows, s < W.
__global__ __launch_bounds__(kThreads) void k_copy_rows(const float2* __restrict__ src,
                                                        size_t src_pitch, float2* __restrict__ dst,
                                                        size_t n, int W) {
  const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  dst[i] = src[(i / W) * src_pitch + i % W];
}

hipError_t launch_copy_rows(const float2* src, size_t src_pitch, float2* dst, size_t rows, int W,
                            hipStream_t st) {
  const size_t n = rows * (size_t)W;
  if (n == 0) return hipSuccess;
  k_copy_rows<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, st>>>(src, src_pitch, dst,
                                                                              n, W);
  return hipGetLastError();
}

hipError_t launch_frames_x(const DevGeom& g, const float2* psi, const float2* Q, float2* X,
                           int k_first, int Kc, hipStream_t st) {
  const size_t n = (size_t)g.H * g.W * Kc * g.nd;
  if (n == 0) return hipSuccess;
  k_frames_x<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, st>>>(psi, Q, X, g, k_first,
                                                                            Kc);
  return hipGetLastError();
}

hipError_t launch_frames_c(const DevGeom& g, float2* X, const float2* psi, const float2* Q,
                           float2* G, float2* Pbuf, int accumulate, int k_first, int Kc,
                           hipStream_t st) {
  const size_t n = (size_t)g.H * g.W * g.nd;
  k_frames_c<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, st>>>(
      X, psi, Q, G, Pbuf, g, accumulate, k_first, Kc);
  return hipGetLastError();
}

hipError_t launch_pass_a(const DevGeom& g, const float2* psi, const float2* Q, float2* X,
                         int k_first, int Kc, hipStream_t st) {
  const dim3 grid(g.H / rows_per_wg(g.W), Kc * g.nd);
  switch (g.W) {
#define CASE(N)                                                                 \
  case N:                                                                       \
    if (g.pshift)                                                               \
      k_pass_a<N, true><<<grid, kThreads, 0, st>>>(psi, Q, X, g, k_first);      \
    else                                                                        \
      k_pass_a<N, false><<<grid, kThreads, 0, st>>>(psi, Q, X, g, k_first);     \
    break;
    HOLO_FOR_SIZES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool col_tile_supported(int H, int tc) { return tc == cols_tc(H) || tc == cols_tc(H) / 2; }

template <int N, int TC>
static void pass_b_mode(int mode, unsigned grid, const float2* src, float2* X, const float* amp,
                        double* Fpart, const DevGeom& g, int ntiles, hipStream_t st) {
  switch (mode) {
    case kColFwd: k_pass_b<N, kColFwd, TC><<<grid, kColThreads, 0, st>>>(src, X, amp, Fpart, g, ntiles); break;
    case kColObj: k_pass_b<N, kColObj, TC><<<grid, kColThreads, 0, st>>>(src, X, amp, Fpart, g, ntiles); break;
    case kColGrad: k_pass_b<N, kColGrad, TC><<<grid, kColThreads, 0, st>>>(src, X, amp, Fpart, g, ntiles); break;
    default: k_pass_b<N, kColAdj, TC><<<grid, kColThreads, 0, st>>>(src, X, amp, Fpart, g, ntiles); break;
  }
}

// Pass B with g.col_tile columns per workgroup: the default cols_tc(H) or
// half of it (a tuning choice; the results are the same, only the cost
// partials are summed in a different grouping).
hipError_t launch_pass_b(const DevGeom& g, int mode, const float2* src, float2* X,
                         const float* amp, double* Fpart, int Kc, hipStream_t st) {
  if (mode != kColFwd && mode != kColObj && mode != kColGrad && mode != kColAdj)
    return hipErrorInvalidValue;
  const int tc = g.col_tile ? g.col_tile : cols_tc(g.H);
  if (!col_tile_supported(g.H, tc)) return hipErrorInvalidValue;
  const int ntiles = g.W / tc;
  const unsigned grid = (unsigned)ntiles * (unsigned)(Kc * g.nd);
  switch (g.H) {
#define CASE(N)                                                                     \
  case N:                                                                           \
    if (tc == cols_tc(N))                                                           \
      pass_b_mode<N, cols_tc(N)>(mode, grid, src, X, amp, Fpart, g, ntiles, st);    \
    else                                                                            \
      pass_b_mode<N, cols_tc(N) / 2>(mode, grid, src, X, amp, Fpart, g, ntiles, st); \
    break;
    HOLO_FOR_SIZES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pass_c(const DevGeom& g, float2* X, const float2* psi, const float2* Q,
                         float2* G, float2* Pbuf, int accumulate, int k_first, int Kc,
                         hipStream_t st) {
  const dim3 grid(g.H / rows_per_wg(g.W), g.nd);
  switch (g.W) {
#define CASE(N)                                                                            \
  case N:                                                                                  \
    if (g.pshift)                                                                          \
      k_pass_c<N, true><<<grid, kThreads, 0, st>>>(X, psi, Q, G, Pbuf, g, accumulate,       \
                                                   k_first, Kc);                            \
    else                                                                                   \
      k_pass_c<N, false><<<grid, kThreads, 0, st>>>(X, psi, Q, G, nullptr, g, accumulate,   \
                                                    k_first, Kc);                           \
    break;
    HOLO_FOR_SIZES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pass_d(const DevGeom& g, const float2* X, const float2* psi, float2* S,
                         int k_first, int Kc, hipStream_t st) {
  const dim3 grid((g.H / 16) * (sino_row(g.W) / 16), (Kc + kPassDAngles - 1) / kPassDAngles);
  k_pass_d<<<grid, kThreads, 0, st>>>(X, psi, S, g, k_first, Kc);
  return hipGetLastError();
}

// G_j[y][x] += sum over the chunk's angles k of Pbuf[k][j] sampled at
// (y + s_y, x + s_x): the transposed probe shift S_{-s_kj}.
__global__ __launch_bounds__(kThreads) void k_probe_shift_acc(float2* __restrict__ G,
                                                              const float2* __restrict__ Pbuf,
                                                              DevGeom g, int k_first, int Kc) {
  const size_t HW = (size_t)g.H * g.W;
  const int j = blockIdx.y;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < HW;
       i += (size_t)gridDim.x * kThreads) {
    const int y = (int)(i / g.W), x = (int)(i % g.W);
    float2 acc = G[(size_t)j * HW + i];
    for (int k = 0; k < Kc; ++k) {
      const float* ps = g.pshift + ((size_t)(k_first + k) * g.nd + j) * 2;
      const float2 v = sample_circ(Pbuf + ((size_t)k * g.nd + j) * HW, g.H, g.W,
                                   (double)y + ps[0], (double)x + ps[1]);
      acc.x += v.x;
      acc.y += v.y;
    }
    G[(size_t)j * HW + i] = acc;
  }
}

hipError_t launch_probe_shift_acc(const DevGeom& g, float2* G, const float2* Pbuf, int k_first,
                                  int Kc, hipStream_t st) {
  const size_t HW = (size_t)g.H * g.W;
  const unsigned gx = (unsigned)std::min<size_t>((HW + kThreads - 1) / kThreads, 4096);
  k_probe_shift_acc<<<dim3(gx, g.nd), kThreads, 0, st>>>(G, Pbuf, g, k_first, Kc);
  return hipGetLastError();
}

hipError_t launch_radon_fwd(const DevGeom& g, const float2* ub, const float2* uTb, float2* psi,
                            const double* ang, const int2* groups, int g0, int ngroups, int c0,
                            int c1, int nb, hipStream_t st) {
  const unsigned n = (unsigned)(g.W / nb) * (unsigned)(g.H / kFwdZT) * (unsigned)ngroups;
  if (nb == kFwdNB)
    k_radon_fwd<kFwdNB><<<n, kThreads, 0, st>>>(ub, uTb, psi, g, ang, groups, g0, ngroups, c0, c1);
  else if (nb == kFwdNB / 2)
    k_radon_fwd<kFwdNB / 2><<<n, kThreads, 0, st>>>(ub, uTb, psi, g, ang, groups, g0, ngroups, c0,
                                                    c1);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_radon_adj(const DevGeom& g, const float2* S, float2* gu, const double* ang,
                            int K, hipStream_t st) {
  const unsigned n = (unsigned)(g.W / 16) * (unsigned)(g.W / 16) * (unsigned)(g.H / kAdjZT);
  k_radon_adj<<<n, kThreads, 0, st>>>(S, gu, g, ang, K);
  return hipGetLastError();
}

hipError_t launch_block_volume(const DevGeom& g, const float2* u, float2* ub, float2* uTb,
                               hipStream_t st) {
  const dim3 grid((g.W / 16) * (g.W / 16), g.H / kVolZB);
  k_block_volume<<<grid, kThreads, 0, st>>>(u, ub, uTb, g.W);
  return hipGetLastError();
}

static unsigned grid_for(size_t n) {
  size_t b = (n + kThreads - 1) / kThreads;
  if (b > 65536) b = 65536;
  if (b == 0) b = 1;
  return (unsigned)b;
}

hipError_t launch_fill(float2* p, size_t n, float2 value, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_fill<<<grid_for(n), kThreads, 0, st>>>(p, n, value);
  return hipGetLastError();
}

hipError_t launch_fill_zero(float2* p, size_t n, hipStream_t st) {
  return launch_fill(p, n, make_float2(0.f, 0.f), st);
}

hipError_t launch_sum_frames(const float2* G, int nd, const float2* extra, float2* out, size_t n,
                             hipStream_t st) {
  k_sum_frames<<<grid_for(n), kThreads, 0, st>>>(G, nd, extra, out, n);
  return hipGetLastError();
}

hipError_t launch_dot_re(const float2* a1, const float2* b1, size_t n1, const float2* a2,
                         const float2* b2, size_t n2, double* parts, double* scratch, double* out,
                         hipStream_t st) {
  // fixed partitions of both parts, then the two-stage sum of the partials
  auto groups = [](size_t n) {
    return std::max<size_t>(1, std::min<size_t>(kDotParts / 2, (n + 65535) / 65536));
  };
  const size_t g1 = groups(n1), g2 = groups(n2);
  k_dot_re<<<(unsigned)g1, kThreads, 0, st>>>(a1, b1, n1, (n1 + g1 - 1) / g1, parts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_dot_re<<<(unsigned)g2, kThreads, 0, st>>>(a2, b2, n2, (n2 + g2 - 1) / g2, parts + g1);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_sum(parts, g1 + g2, scratch, out, st);
}

hipError_t launch_axpy(const float2* x, const float2* e, float t, float2* out, size_t n,
                       hipStream_t st) {
  k_axpy<<<grid_for(n), kThreads, 0, st>>>(x, e, t, out, n);
  return hipGetLastError();
}

hipError_t launch_cg_dir(const float2* g, float2* eta, float beta, int restart, size_t n,
                         hipStream_t st) {
  k_cg_dir<<<grid_for(n), kThreads, 0, st>>>(g, eta, beta, restart, n);
  return hipGetLastError();
}

hipError_t launch_real_to_c64(const float* a, float2* out, size_t n, hipStream_t st) {
  k_real_to_c64<<<grid_for(n), kThreads, 0, st>>>(a, out, n);
  return hipGetLastError();
}

hipError_t launch_reduce_sum(const double* parts, size_t n, double* scratch, double* out,
                             hipStream_t st) {
  // two stages: up to kReduceParts workgroups of consecutive partials, then one
  const size_t g = std::max<size_t>(1, std::min<size_t>(kReduceParts, (n + 8191) / 8192));
  const size_t per = (n + g - 1) / g;
  k_reduce_sum<<<(unsigned)g, kThreads, 0, st>>>(parts, n, per, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_reduce_sum<<<1, kThreads, 0, st>>>(scratch, g, g, out);
  return hipGetLastError();
}

}  // namespace holo
