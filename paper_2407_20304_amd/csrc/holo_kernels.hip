// HIP kernels of the holotomography gradient for gfx950 (MI355X).
//
// Frame stages (detector-plane work, HBM-bound):
//   pass A  rows:    phi = 1 + B(psi - 1), x = Q_j phi, row FFT * transfer * IFFT
//   pass B  columns: column FFT * transfer * IFFT -> v, residual and cost,
//                    column FFT * conj(transfer) * IFFT
//   pass C  rows:    row FFT * conj(transfer) * IFFT -> w,
//                    G_j += conj(phi) w (probe gradient), X := conj(Q_j) w
//   pass D  pixels:  g_psi = sum_j B^T X_j (gather), h = -i kappa conj(psi) g_psi
// (The ray sums R_k and their transpose are in holo_radon.hip.)
// Positions and interpolation weights are formed in double precision (or as
// single-precision offsets of a few bins from double-precision bases); field
// arithmetic is single precision; costs and long ray sums are carried in
// double, the transpose's sums over angles in two levels of single precision.
#include <algorithm>

#include "holo_internal.hpp"
#include "fft_lds.hpp"

namespace holo {

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
  constexpr bool WL = wave_lines(TL);
  __shared__ float2 s_tw[fft_line_len(W)];
  __shared__ float2 s_line[LPW][fft_line_len(W)];
  const int line = threadIdx.x / TL, lt = threadIdx.x % TL;
  const int z = blockIdx.x * LPW + line;
  const int f = blockIdx.y;
  const int k = f / g.nd, j = f % g.nd;
  for (int i = threadIdx.x; i < W; i += kThreads) s_tw[fpi(i)] = g.twW[i];

  double ty, tx;
  shift_of(g, k_first + k, j, ty, tx);
  const double m = g.mag[j];
  const AxisTaps tyt = fwd_taps(g.cH, m, ty, z, g.H);
  const float2* psik = psi + (size_t)k * g.H * W;
  const float2* Qrow = Q + ((size_t)j * g.H + z) * W;
  const float* ps = PS ? g.pshift + ((size_t)(k_first + k) * g.nd + j) * 2 : nullptr;
  const float2* ch = g.chirpW + (size_t)chirp_det(j) * W;
  // the thread's elements s = lt + e TL of the row, kept in registers
  // between the transforms (the line in LDS is only their exchange buffer)
  float2 v[E], cv[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int s = lt + e * TL;
    const AxisTaps txt = fwd_taps(g.cW, m, tx, s, W);
    float2 qv;
    if constexpr (PS)
      qv = sample_circ(Q + (size_t)j * g.H * W, g.H, W, (double)z - ps[0], (double)s - ps[1]);
    else
      qv = Qrow[s];
    v[e] = cmul(qv, sample_phi(psik, W, tyt, txt));
    cv[e] = ch[s];
  }
  if constexpr (WL) __syncthreads();   // s_tw (otherwise the first stage's barrier)
  float2* L = s_line[line];
  fft_e<W, TL, false, true, WL>(v, L, s_tw, lt);
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = cmul(v[e], cv[e]);
  fft_e<W, TL, true, true, WL>(v, L, s_tw, lt);
  float2* out = X + ((size_t)f * g.H + z) * W;
#pragma unroll
  for (int e = 0; e < E; ++e) out[lt + e * TL] = v[e];
}

template <int W, bool PS>   // PS: probe shifts set
__global__ __launch_bounds__(kThreads) void k_pass_c(float2* __restrict__ X,
                                                     const float2* __restrict__ psi,
                                                     const float2* __restrict__ Q,
                                                     float2* __restrict__ G,
                                                     float2* __restrict__ Pbuf, DevGeom g,
                                                     int accumulate, int k_first, int Kc) {
  constexpr int TL = rows_tl(W), LPW = rows_lpw(W), E = W / TL;
  __shared__ float2 s_tw[fft_line_len(W)];
  __shared__ float2 s_line[LPW][fft_line_len(W)];
  const int line = threadIdx.x / TL, lt = threadIdx.x % TL;
  const int lp = fpi(lt);   // padded position of the thread's first element
  const int z = blockIdx.x * LPW + line;
  const int j = blockIdx.y;
  for (int i = threadIdx.x; i < W; i += kThreads) s_tw[fpi(i)] = g.twW[i];
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
  __shared__ float2 s_tw[fft_line_len(W)];
  __shared__ float2 s_line[LPW][fft_line_len(W)];
  const int line = threadIdx.x / TL, lt = threadIdx.x % TL;
  const int lp = fpi(lt);   // padded position of the thread's first element
  const int z = blockIdx.x * LPW + line;
  const PropJob& jb = jobs.job[blockIdx.y];
  for (int i = threadIdx.x; i < W; i += kThreads) s_tw[fpi(i)] = g.twW[i];
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
  __shared__ float2 s_tw[fft_line_len(H)];
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
    if (i < H) s_tw[fpi(i)] = g.twH[i];
  }
#pragma unroll
  for (int r = 0; r < NPT; ++r) l0[r * LSTEP] = t[r];
  // The thread's column elements zz = lt + e TLc stay in registers around
  // the transforms; the tile column in LDS is their exchange buffer, and the
  // tile itself is only touched to load, to store and for the residual
  // (whose amplitudes are read in the coalesced tile order).
  constexpr int EC = H / TLc;
  float2* Lc = s_col[c];
  const float2* ch = g.chirpH + (size_t)chirp_det(j) * H;
  constexpr bool WL = wave_lines(TLc);
  float2 v[EC];
  __syncthreads();   // tile and s_tw
#pragma unroll
  for (int e = 0; e < EC; ++e) v[e] = Lc[fpi(lt + e * TLc)];
  if (MODE != kColAdj) {
    fft_e<H, TLc, false, true, WL>(v, Lc, s_tw, lt);
#pragma unroll
    for (int e = 0; e < EC; ++e) v[e] = cmul(v[e], ch[lt + e * TLc]);
    fft_e<H, TLc, true, true, WL>(v, Lc, s_tw, lt);
  }
  if (kResidual) {
    fft_sync<WL>();                    // the column's exchange reads are done
#pragma unroll
    for (int e = 0; e < EC; ++e) Lc[fpi(lt + e * TLc)] = v[e];
    asm volatile("" : "+v"(g0), "+v"(l0));
    const float* a = amp + (size_t)f * H * W + s0;
    float ar[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) ar[r] = a[g0 + r * gstep];
    __syncthreads();
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
      float2 t = l0[r * LSTEP];
      acc += residual(t, ar[r], g.functional);
      l0[r * LSTEP] = t;
    }
    // (its barrier also publishes the residual writes)
    block_sum_store<kColThreads>(acc, Fpart + (size_t)f * ntiles + tile);
#pragma unroll
    for (int e = 0; e < EC; ++e) v[e] = Lc[fpi(lt + e * TLc)];
  }
  if (MODE == kColGrad || MODE == kColAdj) {
    fft_e<H, TLc, false, true, WL>(v, Lc, s_tw, lt);
#pragma unroll
    for (int e = 0; e < EC; ++e) v[e] = cmulc(v[e], ch[lt + e * TLc]);
    fft_e<H, TLc, true, true, WL>(v, Lc, s_tw, lt);
  }
  if (MODE != kColObj) {
    __syncthreads();                   // every column's exchange reads are done
#pragma unroll
    for (int e = 0; e < EC; ++e) Lc[fpi(lt + e * TLc)] = v[e];
    __syncthreads();
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
  __shared__ float2 s_tw[fft_line_len(H)];
  __shared__ float2 s_col[TC][col_pitch(H)];
  const int c = threadIdx.x / TLc, lt = threadIdx.x % TLc;
  const int W = g.W;
  const int s0 = blockIdx.x * TC;
  const PropJob& jb = jobs.job[blockIdx.y];
  for (int i = threadIdx.x; i < H; i += kColThreads) s_tw[fpi(i)] = g.twH[i];
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
  __shared__ float2 s_tw[fft_line_len(N2)];
  __shared__ float2 s_line[LPW][fft_line_len(N2)];
  const int line = threadIdx.x / TL, lt = threadIdx.x % TL;
  const int z = blockIdx.x * LPW + line;
  const int f = blockIdx.y;
  for (int i = threadIdx.x; i < N2; i += kThreads) s_tw[fpi(i)] = g.tw2W[i];
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
  __shared__ float2 s_tw[fft_line_len(N2)];
  __shared__ float2 s_col[TC][col_pitch(N2)];
  const int c = threadIdx.x / TLc, lt = threadIdx.x % TLc;
  const int W = g.W;
  const int tile = blockIdx.x % ntiles, f = blockIdx.x / ntiles;
  const int s0 = tile * TC;
  const size_t HW = (size_t)H * W;
  for (int i = threadIdx.x; i < N2; i += kColThreads) s_tw[fpi(i)] = g.tw2H[i];
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
  // side; with g.sino_mirror, rows of angles with cos < 0 are stored
  // reversed, bin s at kAdjPad + W - 1 - s) for kPassDAngles consecutive
  // angles.  Workgroups over the padding
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
    // rows of angles with cos < 0 reversed for the Joseph transpose
    const bool mir = g.sino_mirror && g.ang[(size_t)(k_first + k) * kAngleStride + kCos] < 0.0;
    float2* out = S + ((size_t)k * H + z) * Wp + (mir ? Wp - 1 - sp : sp);
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
