// Fourier-slice ray sums and their transpose for gfx950 (the alternative
// discretisation of R_k; see holo.h, HOLO_PROJECTOR_FOURIER).
//
// The projection of a slice at angle theta is the inverse W-point DFT of the
// slice's discrete-time Fourier transform F(xi) = sum u[y][x]
// e^{-2 pi i xi.(x', y') / W} sampled at xi = m (cos, sin), m = -W/2 .. W/2
// (the two Nyquist samples averaged).  F is evaluated by gridding: the slice,
// divided by the Fourier transform of the spreading kernel, is embedded in an
// M x M grid (M = 2W, twice oversampled) and transformed by 2-D FFT; F(xi)
// is then the kernel-weighted sum of the KW x KW grid values around grid
// position 2 xi.  The kernel is exp(beta (sqrt(1 - (2x/KW)^2) - 1)) on
// |x| < KW/2 (the "exponential of semicircle" shape); with KW = 8 and
// beta = 2.3 KW the gridding error is a few 1e-8 relative.  The transpose
// runs the same steps backwards: per angle a DFT of the bin line, the polar
// samples spread onto the grid (written as a gather: every grid point sums
// the samples within its kernel reach, found from its polar angle through a
// table of the angles sorted modulo pi, so no atomics and a fixed order),
// inverse 2-D FFT, the centre W x W, divided by the kernel's transform.
//
// Slices are processed in slabs of kFsSlab: the grid of a slab (and, in the
// transpose, its polar samples of every angle) lives in the workspace.  The
// forward writes psi = exp(i kappa p) of every angle into the sinogram
// buffer (the frame passes copy one chunk at a time from there; pass D then
// overwrites the chunk with h, which the transpose reads).
#include "holo_internal.hpp"
#include "fft_lds.hpp"

namespace holo {

namespace {

constexpr int kT = 256;            // threads of the line kernels
constexpr int kColT = 512;         // threads of the column kernels
constexpr int KW = kFsWidth;       // kernel taps per axis

__host__ __device__ constexpr int fs_tl(int N) { return fft_row_threads(N); }
__host__ __device__ constexpr int fs_lpw(int N) { return kT / fs_tl(N); }
__host__ __device__ constexpr int fs_tc(int M) { return M >= 2048 ? 4 : (M >= 1024 ? 8 : 16); }
__host__ __device__ constexpr int fs_pitch(int M) { return fft_line_len(M) + 4; }
__host__ __device__ constexpr bool fs_wave(int TL) { return TL <= 64; }

// Kernel value at distance x (grid units) from a sample.
__device__ __forceinline__ float es_kernel(float x, float beta) {
  const float z = x * (2.0f / (float)KW);
  const float r = 1.0f - z * z;
  return r > 0.0f ? expf(beta * (sqrtf(r) - 1.0f)) : 0.0f;
}

// Grid index of centred position l (-M/2 - KW <= l < M/2 + KW).
__device__ __forceinline__ int wrap(int l, int M) { return l < 0 ? l + M : (l >= M ? l - M : l); }

}  // namespace

// ---------------------------------------------------------------------------
// Forward: rows (deapodise, embed, FFT), columns (FFT), gridding + inverse
// DFT per (slice, angle) line + exp(i kappa p).
// ---------------------------------------------------------------------------

// Row y of slice z of the slab: u[z][y][.] / (phihat(x') phihat(y')) placed
// at x' mod M (x' = x - W/2), transformed, stored as grid row y' mod M.
template <int W>
__global__ __launch_bounds__(kT) void k_fs_rows(const float2* __restrict__ u,
                                                float2* __restrict__ G, FsArgs f,
                                                const float2* __restrict__ tw) {
  constexpr int M = 2 * W, TL = fs_tl(M), LPW = fs_lpw(M), E = M / TL;
  __shared__ float2 s_tw[M];
  __shared__ float2 s_line[LPW][fft_line_len(M)];
  const int line = threadIdx.x / TL, lt = threadIdx.x % TL;
  const int L = blockIdx.x * LPW + line;            // z * W + y
  const int z = L / W, y = L % W;
  for (int i = threadIdx.x; i < M; i += kT) s_tw[i] = tw[i];
  const float2* row = u + (size_t)L * W;
  const float dy = f.dinv[y];
  float2* Ln = s_line[line];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int n = lt + e * TL;
    const int xp = n < W / 2 ? n : n - M;             // x' of grid column n
    float2 v = make_float2(0.f, 0.f);
    if (xp >= -W / 2 && xp < W / 2) {
      const int x = xp + W / 2;
      const float s = dy * f.dinv[x];
      const float2 a = row[x];
      v = make_float2(s * a.x, s * a.y);
    }
    Ln[fpi(n)] = v;
  }
  if constexpr (fs_wave(TL)) __syncthreads();
  fft<M, TL, false, true, fs_wave(TL)>(Ln, s_tw, lt);
  const int yp = y - W / 2;
  float2* out = G + ((size_t)z * M + (yp < 0 ? yp + M : yp)) * M;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int n = lt + e * TL;
    out[n] = Ln[fpi(n)];
  }
}

// Column transforms of the slab's grids.  Forward: only the W rows y' mod M
// hold data (the others are zero), all M rows are written.  Inverse (the
// transpose): all M rows are read, only those W rows are written.
template <int W, bool INV>
__global__ __launch_bounds__(kColT) void k_fs_cols(float2* __restrict__ G,
                                                   const float2* __restrict__ tw) {
  constexpr int M = 2 * W, TC = fs_tc(M), TLc = kColT / TC;
  __shared__ float2 s_tw[M];
  __shared__ float2 s_col[TC][fs_pitch(M)];
  const int c = threadIdx.x / TLc, lt = threadIdx.x % TLc;
  constexpr int ntiles = M / TC;
  const int z = blockIdx.x / ntiles, s0 = (blockIdx.x % ntiles) * TC;
  float2* g = G + (size_t)z * M * M + s0;
  for (int i = threadIdx.x; i < M; i += kColT) s_tw[i] = tw[i];
  for (int i = threadIdx.x; i < M * TC; i += kColT) {
    const int r = i / TC, cc = i % TC;
    const bool data = INV || r < W / 2 || r >= M - W / 2;
    s_col[cc][fpi(r)] = data ? g[(size_t)r * M + cc] : make_float2(0.f, 0.f);
  }
  float2* Lc = s_col[c];
  constexpr bool WL = fs_wave(TLc);
  if constexpr (WL) __syncthreads();
  fft<M, TLc, INV, true, WL>(Lc, s_tw, lt);
  __syncthreads();
  for (int i = threadIdx.x; i < M * TC; i += kColT) {
    const int r = i / TC, cc = i % TC;
    if (!INV || r < W / 2 || r >= M - W / 2) g[(size_t)r * M + cc] = s_col[cc][fpi(r)];
  }
}

// One (slice, angle) line per TL threads: F(m (cos, sin)) by gridding for
// m = -W/2 .. W/2, the line Q[m mod W] = (-1)^m F (Nyquist samples averaged),
// p = IDFT(Q) / W, psi = exp(i kappa p) written to the sinogram row
// S[k][z0 + z][kAdjPad + s].
template <int W>
__global__ __launch_bounds__(kT) void k_fs_project(const float2* __restrict__ G,
                                                   float2* __restrict__ S, FsArgs f,
                                                   const float2* __restrict__ twW, int H,
                                                   int z0, int nlines, float kappa) {
  constexpr int M = 2 * W, TL = fs_tl(W), LPW = fs_lpw(W), E = W / TL;
  __shared__ float2 s_tw[W];
  __shared__ float2 s_line[LPW][fft_line_len(W)];
  const int line = threadIdx.x / TL, lt = threadIdx.x % TL;
  // z * K + k, angles fastest; lines past the last only join the transforms
  const int L0 = blockIdx.x * LPW + line;
  const bool live = L0 < nlines;
  const int L = live ? L0 : nlines - 1;
  const int z = L / f.K, k = L % f.K;
  for (int i = threadIdx.x; i < W; i += kT) s_tw[i] = twW[i];
  const double* ap = f.ang + (size_t)(f.k0 + k) * kAngleStride;
  const double C = 2.0 * ap[kCos], Sn = 2.0 * ap[kSin];    // grid units per m
  const float2* g = G + (size_t)z * M * M;
  const float beta = f.beta;
  // F at m: the KW x KW grid values around (m C, m Sn); taps start at
  // floor(pos) - KW/2 + 1, so every distance lies in (-KW/2, KW/2]
  auto grid_at = [&](int m) {
    const double gx = (double)m * C, gy = (double)m * Sn;
    const double fx = floor(gx), fy = floor(gy);
    const int lx0 = (int)fx - KW / 2 + 1, ly0 = (int)fy - KW / 2 + 1;
    const float rx = (float)(gx - fx) + (float)(KW / 2 - 1);   // distance to tap 0
    const float ry = (float)(gy - fy) + (float)(KW / 2 - 1);
    float wx[KW];
#pragma unroll
    for (int b = 0; b < KW; ++b) wx[b] = es_kernel(rx - (float)b, beta);
    int cx[KW];
#pragma unroll
    for (int b = 0; b < KW; ++b) cx[b] = wrap(lx0 + b, M);
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int a = 0; a < KW; ++a) {
      const float2* gr = g + (size_t)wrap(ly0 + a, M) * M;
      float sx = 0.f, sy = 0.f;
#pragma unroll
      for (int b = 0; b < KW; ++b) {
        const float2 v = gr[cx[b]];
        sx = fmaf(wx[b], v.x, sx);
        sy = fmaf(wx[b], v.y, sy);
      }
      const float wy = es_kernel(ry - (float)a, beta);
      acc.x = fmaf(wy, sx, acc.x);
      acc.y = fmaf(wy, sy, acc.y);
    }
    return acc;
  };
  float2* Ln = s_line[line];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int mp = lt + e * TL;                     // m + W/2
    const int m = mp - W / 2;
    float2 v = grid_at(m);
    if (mp == 0) {                                  // Nyquist: average of -W/2 and +W/2
      const float2 v2 = grid_at(W / 2);
      v = make_float2(0.5f * (v.x + v2.x), 0.5f * (v.y + v2.y));
    }
    if (m & 1) v = make_float2(-v.x, -v.y);         // (-1)^m: bins start at s = -W/2
    Ln[fpi(m < 0 ? m + W : m)] = v;
  }
  if constexpr (fs_wave(TL)) __syncthreads();
  fft<W, TL, true, true, fs_wave(TL)>(Ln, s_tw, lt);
  const double twopi = 6.283185307179586476925;
  const int Wp = W + 2 * kAdjPad;
  float2* out = S + ((size_t)k * H + z0 + z) * Wp + kAdjPad;
  if (!live) return;                                // after the last barrier
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int s = lt + e * TL;
    const float2 p = Ln[fpi(s)];
    double ph = (double)kappa * ((double)p.x / (double)W);
    ph -= twopi * rint(ph / twopi);
    float sn, cs;
    sincosf((float)ph, &sn, &cs);
    const float mag = expf(-kappa * (p.y / (float)W));
    out[s] = make_float2(mag * cs, mag * sn);
  }
}

// ---------------------------------------------------------------------------
// Transpose: DFT per (slice, angle) line, gather-spread, inverse columns,
// inverse rows + deapodisation.
// ---------------------------------------------------------------------------

// A[z][k][m + W/2] = (-1)^m DFT(h)[m mod W] / W for m = -W/2 .. W/2, the two
// Nyquist entries halved (the transpose of the forward's line step).
template <int W>
__global__ __launch_bounds__(kT) void k_fs_line_T(const float2* __restrict__ S,
                                                  float2* __restrict__ A, FsArgs f,
                                                  const float2* __restrict__ twW, int H,
                                                  int z0, int nlines) {
  constexpr int TL = fs_tl(W), LPW = fs_lpw(W), E = W / TL;
  __shared__ float2 s_tw[W];
  __shared__ float2 s_line[LPW][fft_line_len(W)];
  const int line = threadIdx.x / TL, lt = threadIdx.x % TL;
  const int L0 = blockIdx.x * LPW + line;
  const bool live = L0 < nlines;
  const int L = live ? L0 : nlines - 1;
  const int z = L / f.K, k = L % f.K;
  for (int i = threadIdx.x; i < W; i += kT) s_tw[i] = twW[i];
  const int Wp = W + 2 * kAdjPad;
  const float2* in = S + ((size_t)k * H + z0 + z) * Wp + kAdjPad;
  float2* Ln = s_line[line];
#pragma unroll
  for (int e = 0; e < E; ++e) Ln[fpi(lt + e * TL)] = in[lt + e * TL];
  if constexpr (fs_wave(TL)) __syncthreads();
  fft<W, TL, false, true, fs_wave(TL)>(Ln, s_tw, lt);
  float2* out = A + (size_t)L * (W + 2);
  if (!live) return;                                // after the last barrier
  const float sc = 1.0f / (float)W;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int mp = lt + e * TL;
    const int m = mp - W / 2;
    float2 v = Ln[fpi(m < 0 ? m + W : m)];
    float s = (m & 1) ? -sc : sc;
    if (mp == 0) s *= 0.5f;
    v = make_float2(s * v.x, s * v.y);
    out[mp] = v;
    if (mp == 0) out[W] = v;                        // m = +W/2 shares the halved value
  }
}

// Every grid point of the slab sums kernel-weighted polar samples within its
// reach (the transpose of the gridding), for all kFsSlab slices at once.
template <int W>
__global__ __launch_bounds__(kT) void k_fs_spread(const float2* __restrict__ A,
                                                  float2* __restrict__ G, FsArgs f, int nz) {
  constexpr int M = 2 * W;
  const int idx = blockIdx.x * kT + threadIdx.x;
  if (idx >= M * M) return;
  const int lx = idx % M, ly = idx / M;
  const int cx = lx < M / 2 ? lx : lx - M, cy = ly < M / 2 ? ly : ly - M;
  // periodic images of the point that polar samples (radius <= M/2) can reach
  const int ax = cx < -M / 2 + KW / 2 ? cx + M : (cx >= M / 2 - KW / 2 ? cx - M : cx);
  const int ay = cy < -M / 2 + KW / 2 ? cy + M : (cy >= M / 2 - KW / 2 ? cy - M : cy);
  const float beta = f.beta;
  constexpr float kReach = (float)KW * 0.70710678f + 0.05f;   // KW/2 * sqrt(2)
  float2 acc[kFsSlab];
#pragma unroll
  for (int z = 0; z < kFsSlab; ++z) acc[z] = make_float2(0.f, 0.f);
  const size_t zstride = (size_t)f.K * (W + 2);
  for (int im = 0; im < 4; ++im) {
    const int px = (im & 1) ? ax : cx, py = (im & 2) ? ay : cy;
    if (((im & 1) && ax == cx) || ((im & 2) && ay == cy)) continue;
    const float r = sqrtf((float)px * px + (float)py * py);
    if (r > 0.5f * (float)M + (float)KW) continue;
    // sorted positions of the angles whose line passes within reach
    int seg_lo[2], seg_hi[2], nseg = 1;
    if (r <= kReach) {
      seg_lo[0] = 0;
      seg_hi[0] = f.n_angles;
    } else {
      const float dl = asinf(fminf(1.0f, kReach / r));
      float phi = atan2f((float)py, (float)px);
      if (phi < 0.f) phi += 3.14159265358979f;
      if (phi >= 3.14159265358979f) phi -= 3.14159265358979f;
      const float sc = (float)kFsBins / 3.14159265358979f;
      int b0 = (int)floorf((phi - dl) * sc) - 1, b1 = (int)floorf((phi + dl) * sc) + 1;
      if (b1 - b0 + 1 >= kFsBins) {
        seg_lo[0] = 0;
        seg_hi[0] = f.n_angles;
      } else if (b0 < 0) {
        seg_lo[0] = f.bin_first[b0 + kFsBins];
        seg_hi[0] = f.n_angles;
        seg_lo[1] = 0;
        seg_hi[1] = f.bin_first[b1 + 1];
        nseg = 2;
      } else if (b1 >= kFsBins) {
        seg_lo[0] = f.bin_first[b0];
        seg_hi[0] = f.n_angles;
        seg_lo[1] = 0;
        seg_hi[1] = f.bin_first[b1 - kFsBins + 1];
        nseg = 2;
      } else {
        seg_lo[0] = f.bin_first[b0];
        seg_hi[0] = f.bin_first[b1 + 1];
      }
    }
    for (int sgi = 0; sgi < nseg; ++sgi) {
      for (int sp = seg_lo[sgi]; sp < seg_hi[sgi]; ++sp) {
        const int kk = f.sorted_k[sp];
        if (kk < f.k0 || kk >= f.k0 + f.K) continue;
        const double* ap = f.ang + (size_t)kk * kAngleStride;
        const double C = 2.0 * ap[kCos], Sn = 2.0 * ap[kSin];
        // m range from the dominant axis of the line
        const bool xd = fabs(C) >= fabs(Sn);
        const double e = xd ? C : Sn, pd = xd ? (double)px : (double)py;
        const double mc = pd / e, hw = 0.5 * (double)KW / fabs(e);
        int m0 = (int)ceil(mc - hw), m1 = (int)floor(mc + hw);
        m0 = max(m0, -W / 2);
        m1 = min(m1, W / 2);
        const float2* ak = A + (size_t)(kk - f.k0) * (W + 2) + W / 2;
        for (int m = m0; m <= m1; ++m) {
          const float dx = (float)((double)px - (double)m * C);
          const float dy = (float)((double)py - (double)m * Sn);
          if (fabsf(dx) >= 0.5f * (float)KW || fabsf(dy) >= 0.5f * (float)KW) continue;
          const float w = es_kernel(dx, beta) * es_kernel(dy, beta);
#pragma unroll
          for (int z = 0; z < kFsSlab; ++z) {
            if (z < nz) {
              const float2 a = ak[z * zstride + m];
              acc[z].x = fmaf(w, a.x, acc[z].x);
              acc[z].y = fmaf(w, a.y, acc[z].y);
            }
          }
        }
      }
    }
  }
#pragma unroll
  for (int z = 0; z < kFsSlab; ++z)
    if (z < nz) G[(size_t)z * M * M + idx] = acc[z];
}

// Row y' mod M of the slab's grid: inverse transform, the W entries x' mod M,
// divided by phihat(x') phihat(y') -> g_u[z][y][x].
template <int W>
__global__ __launch_bounds__(kT) void k_fs_rows_T(const float2* __restrict__ G,
                                                  float2* __restrict__ gu, FsArgs f,
                                                  const float2* __restrict__ tw) {
  constexpr int M = 2 * W, TL = fs_tl(M), LPW = fs_lpw(M), E = M / TL;
  __shared__ float2 s_tw[M];
  __shared__ float2 s_line[LPW][fft_line_len(M)];
  const int line = threadIdx.x / TL, lt = threadIdx.x % TL;
  const int L = blockIdx.x * LPW + line;
  const int z = L / W, y = L % W;
  for (int i = threadIdx.x; i < M; i += kT) s_tw[i] = tw[i];
  const int yp = y - W / 2;
  const float2* in = G + ((size_t)z * M + (yp < 0 ? yp + M : yp)) * M;
  float2* Ln = s_line[line];
#pragma unroll
  for (int e = 0; e < E; ++e) Ln[fpi(lt + e * TL)] = in[lt + e * TL];
  if constexpr (fs_wave(TL)) __syncthreads();
  fft<M, TL, true, true, fs_wave(TL)>(Ln, s_tw, lt);
  const float dy = f.dinv[y];
  float2* out = gu + (size_t)L * W;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int n = lt + e * TL;
    const int xp = n < W / 2 ? n : n - M;
    if (xp >= -W / 2 && xp < W / 2) {
      const int x = xp + W / 2;
      const float s = dy * f.dinv[x];
      const float2 v = Ln[fpi(n)];
      out[x] = make_float2(s * v.x, s * v.y);
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

bool fs_size_supported(int W) {
  switch (W) {
    case 64: case 128: case 192: case 256: case 384: case 512: case 1024:
      return true;
    default:
      return false;
  }
}

#define HOLO_FS_SIZES(X) X(64) X(128) X(192) X(256) X(384) X(512) X(1024)

hipError_t launch_fs_forward_slab(const DevGeom& g, const FsArgs& f, const float2* u_slab,
                                  float2* G, float2* S, int z0, int nz, hipStream_t st) {
  const int W = g.W;
  if (!g.tw2W || nz < 1 || nz > kFsSlab) return hipErrorInvalidValue;
  switch (W) {
#define CASE(N)                                                                                \
  case N: {                                                                                    \
    constexpr int M = 2 * N;                                                                   \
    k_fs_rows<N><<<(unsigned)(nz * N / fs_lpw(M)), kT, 0, st>>>(u_slab, G, f, g.tw2W);         \
    k_fs_cols<N, false><<<(unsigned)(nz * (M / fs_tc(M))), kColT, 0, st>>>(G, g.tw2W);         \
    const unsigned nl = (unsigned)nz * (unsigned)f.K;                                          \
    k_fs_project<N><<<(nl + fs_lpw(N) - 1) / fs_lpw(N), kT, 0, st>>>(G, S, f, g.twW, g.H, z0, \
                                                                    (int)nl, g.kappa);        \
    break;                                                                                     \
  }
    HOLO_FS_SIZES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fs_adjoint_slab(const DevGeom& g, const FsArgs& f, const float2* S,
                                  float2* A, float2* G, float2* gu_slab, int z0, int nz,
                                  hipStream_t st) {
  const int W = g.W;
  if (!g.tw2W || nz < 1 || nz > kFsSlab) return hipErrorInvalidValue;
  switch (W) {
#define CASE(N)                                                                              \
  case N: {                                                                                  \
    constexpr int M = 2 * N;                                                                 \
    const unsigned nl = (unsigned)nz * (unsigned)f.K;                                        \
    k_fs_line_T<N><<<(nl + fs_lpw(N) - 1) / fs_lpw(N), kT, 0, st>>>(S, A, f, g.twW, g.H, z0,   \
                                                                   (int)nl);                  \
    k_fs_spread<N><<<(unsigned)((M * M + kT - 1) / kT), kT, 0, st>>>(A, G, f, nz);          \
    k_fs_cols<N, true><<<(unsigned)(nz * (M / fs_tc(M))), kColT, 0, st>>>(G, g.tw2W);        \
    k_fs_rows_T<N><<<(unsigned)(nz * N / fs_lpw(M)), kT, 0, st>>>(G, gu_slab, f, g.tw2W);    \
    break;                                                                                   \
  }
    HOLO_FS_SIZES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace holo
