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
  __shared__ float2 s_tw[fft_line_len(M)];
  __shared__ float2 s_line[LPW][fft_line_len(M)];
  const int line = threadIdx.x / TL, lt = threadIdx.x % TL;
  const int L = blockIdx.x * LPW + line;            // z * W + y
  const int z = L / W, y = L % W;
  for (int i = threadIdx.x; i < M; i += kT) s_tw[fpi(i)] = tw[i];
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
  __shared__ float2 s_tw[fft_line_len(M)];
  __shared__ float2 s_col[TC][fs_pitch(M)];
  const int c = threadIdx.x / TLc, lt = threadIdx.x % TLc;
  constexpr int ntiles = M / TC;
  const int z = blockIdx.x / ntiles, s0 = (blockIdx.x % ntiles) * TC;
  float2* g = G + (size_t)z * M * M + s0;
  for (int i = threadIdx.x; i < M; i += kColT) s_tw[fpi(i)] = tw[i];
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
  __shared__ float2 s_tw[fft_line_len(W)];
  __shared__ float2 s_line[LPW][fft_line_len(W)];
  const int line = threadIdx.x / TL, lt = threadIdx.x % TL;
  // z * K + k, angles fastest; lines past the last only join the transforms
  const int L0 = blockIdx.x * LPW + line;
  const bool live = L0 < nlines;
  const int L = live ? L0 : nlines - 1;
  const int z = L / f.K, k = L % f.K;
  for (int i = threadIdx.x; i < W; i += kT) s_tw[fpi(i)] = twW[i];
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

// A[k][m + W/2][z] = (-1)^m DFT(h)[m mod W] / W for m = -W/2 .. W/2, the two
// Nyquist entries halved (the transpose of the forward's line step); the
// slab's slices are innermost (kFsSlab of them, 64 bytes), so the spread
// reads all slices of a polar sample from one cache line.
template <int W>
__global__ __launch_bounds__(kT) void k_fs_line_T(const float2* __restrict__ S,
                                                  float2* __restrict__ A, FsArgs f,
                                                  const float2* __restrict__ twW, int H,
                                                  int z0, int nlines) {
  constexpr int TL = fs_tl(W), LPW = fs_lpw(W), E = W / TL;
  __shared__ float2 s_tw[fft_line_len(W)];
  __shared__ float2 s_line[LPW][fft_line_len(W)];
  const int line = threadIdx.x / TL, lt = threadIdx.x % TL;
  const int L0 = blockIdx.x * LPW + line;
  const bool live = L0 < nlines;
  const int L = live ? L0 : nlines - 1;
  const int z = L / f.K, k = L % f.K;
  for (int i = threadIdx.x; i < W; i += kT) s_tw[fpi(i)] = twW[i];
  const int Wp = W + 2 * kAdjPad;
  const float2* in = S + ((size_t)k * H + z0 + z) * Wp + kAdjPad;
  float2* Ln = s_line[line];
#pragma unroll
  for (int e = 0; e < E; ++e) Ln[fpi(lt + e * TL)] = in[lt + e * TL];
  if constexpr (fs_wave(TL)) __syncthreads();
  fft<W, TL, false, true, fs_wave(TL)>(Ln, s_tw, lt);
  float2* out = A + (size_t)k * (W + 1) * kFsSlab + z;
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
    out[(size_t)mp * kFsSlab] = v;
    if (mp == 0) out[(size_t)W * kFsSlab] = v;      // m = +W/2 shares the halved value
  }
}

// Every grid point of the slab sums the kernel-weighted polar samples within
// its reach (the transpose of the gridding), for all slices of the slab at
// once.  A workgroup owns a 16 x 16 tile of grid points.  The lines that can
// reach any point of the tile are those within d = 8 sqrt(2) + KW sqrt(2)/2
// of the tile centre: an angle window around the centre's polar angle
// (found through the table of angles sorted modulo pi), and on each line the
// samples m with |2m - c.e| <= d (at most 18).  The window is taken in
// batches of kSpBatch lines: the batch's samples (all slab slices, 64
// contiguous bytes per sample) are copied into LDS, then every point gathers
// from there.  Tiles near the grid edge also visit the periodic images of
// the tile that polar samples (radius <= M/2) can reach.
constexpr int kSpTile = 16, kSpBatch = 48, kSpM = 20;

template <int W>
__global__ __launch_bounds__(kT) void k_fs_spread(const float2* __restrict__ A,
                                                  float2* __restrict__ G, FsArgs f, int nz) {
  constexpr int M = 2 * W, NT = M / kSpTile;
  __shared__ float4 s_a[kSpBatch * kSpM * 4];
  __shared__ double s_c[kSpBatch], s_s[kSpBatch];
  __shared__ float s_ih[kSpBatch];
  __shared__ int s_m0[kSpBatch], s_nm[kSpBatch], s_kk[kSpBatch];
  __shared__ int s_seg[2][2], s_nseg;
  const int tx = blockIdx.x % NT, ty = blockIdx.x / NT;
  const int lx = tx * kSpTile + (threadIdx.x & 15), ly = ty * kSpTile + (threadIdx.x >> 4);
  const int idx = ly * M + lx;
  // centred coordinates (a tile never straddles M/2, a multiple of 16)
  const int cx = lx < M / 2 ? lx : lx - M, cy = ly < M / 2 ? ly : ly - M;
  const int tcx0 = tx * kSpTile < M / 2 ? tx * kSpTile : tx * kSpTile - M;
  const int tcy0 = ty * kSpTile < M / 2 ? ty * kSpTile : ty * kSpTile - M;
  const double ccx = tcx0 + 7.5, ccy = tcy0 + 7.5;             // tile centre
  const double d = 8.0 * 1.4142135623730951 + 0.5 * KW * 1.4142135623730951 + 0.05;
  const float beta = f.beta;
  const float4* A4 = reinterpret_cast<const float4*>(A);
  float2 acc[kFsSlab];
#pragma unroll
  for (int z = 0; z < kFsSlab; ++z) acc[z] = make_float2(0.f, 0.f);

  for (int im = 0; im < 9; ++im) {
    const int ox = (im % 3 - 1) * M, oy = (im / 3 - 1) * M;
    const double icx = ccx + ox, icy = ccy + oy;
    const double rc = sqrt(icx * icx + icy * icy);
    if (rc > 0.5 * M + d) continue;                              // uniform over the tile
    // the tile's angle window: sorted positions, one or two segments
    if (threadIdx.x == 0) {
      int nseg = 1;
      if (rc <= d) {
        s_seg[0][0] = 0;
        s_seg[0][1] = f.n_angles;
      } else {
        const double dl = asin(fmin(1.0, d / rc));
        double phi = atan2(icy, icx);
        const double pi = 3.14159265358979323846;
        if (phi < 0.0) phi += pi;
        if (phi >= pi) phi -= pi;
        const double sc = (double)kFsBins / pi;
        const int b0 = (int)floor((phi - dl) * sc) - 1, b1 = (int)floor((phi + dl) * sc) + 1;
        if (b1 - b0 + 1 >= kFsBins) {
          s_seg[0][0] = 0;
          s_seg[0][1] = f.n_angles;
        } else if (b0 < 0) {
          s_seg[0][0] = f.bin_first[b0 + kFsBins];
          s_seg[0][1] = f.n_angles;
          s_seg[1][0] = 0;
          s_seg[1][1] = f.bin_first[b1 + 1];
          nseg = 2;
        } else if (b1 >= kFsBins) {
          s_seg[0][0] = f.bin_first[b0];
          s_seg[0][1] = f.n_angles;
          s_seg[1][0] = 0;
          s_seg[1][1] = f.bin_first[b1 - kFsBins + 1];
          nseg = 2;
        } else {
          s_seg[0][0] = f.bin_first[b0];
          s_seg[0][1] = f.bin_first[b1 + 1];
        }
      }
      s_nseg = nseg;
    }
    __syncthreads();
    const int nseg = s_nseg;
    const double px = (double)(cx + ox), py = (double)(cy + oy);
    for (int sg = 0; sg < nseg; ++sg) {
      const int lo = s_seg[sg][0], hi = s_seg[sg][1];
      for (int b0 = lo; b0 < hi; b0 += kSpBatch) {
        const int nb = min(kSpBatch, hi - b0);
        // the batch's lines: direction, the tile's sample range
        if ((int)threadIdx.x < nb) {
          const int t = threadIdx.x;
          const int kk = f.sorted_k[b0 + t];
          int m0 = 0, nm = 0;
          double C = 0.0, Sn = 0.0;
          float ih = 0.f;
          if (kk >= f.k0 && kk < f.k0 + f.K) {
            const double* ap = f.ang + (size_t)kk * kAngleStride;
            C = 2.0 * ap[kCos];
            Sn = 2.0 * ap[kSin];
            ih = (float)ap[kInvH];
            const double ce = 0.5 * (icx * C + icy * Sn);           // c.e in grid units
            m0 = max((int)ceil(0.5 * (ce - d)), -W / 2);
            const int m1 = min((int)floor(0.5 * (ce + d)), W / 2);
            nm = max(0, m1 - m0 + 1);
          }
          s_c[t] = C;
          s_s[t] = Sn;
          s_ih[t] = ih;
          s_m0[t] = m0;
          s_nm[t] = nm;
          s_kk[t] = kk - f.k0;
        }
        __syncthreads();
        // copy the batch's samples into LDS: line t, sample j, quarter q
        for (int i = threadIdx.x; i < nb * kSpM * 4; i += kT) {
          const int q = i & 3, j = (i >> 2) % kSpM, t = (i >> 2) / kSpM;
          if (j < s_nm[t])
            s_a[i] = A4[((size_t)s_kk[t] * (W + 1) + (s_m0[t] + j + W / 2)) * 4 + q];
        }
        __syncthreads();
        for (int t = 0; t < nb; ++t) {
          const int nm = s_nm[t];
          if (nm == 0) continue;
          const double C = s_c[t], Sn = s_s[t];
          const double ihd = (double)s_ih[t];
          const bool xd = fabs(C) >= fabs(Sn);
          const double e = xd ? C : Sn, pd = xd ? px : py;
          const double mc = 0.5 * pd * (e >= 0.0 ? ihd : -ihd), hw = 0.25 * (double)KW * ihd;
          const int m0 = s_m0[t];
          const int ma = max((int)ceil(mc - hw), m0), mb = min((int)floor(mc + hw), m0 + nm - 1);
          for (int m = ma; m <= mb; ++m) {
            const float dx = (float)(px - (double)m * C);
            const float dy = (float)(py - (double)m * Sn);
            if (fabsf(dx) >= 0.5f * (float)KW || fabsf(dy) >= 0.5f * (float)KW) continue;
            const float w = es_kernel(dx, beta) * es_kernel(dy, beta);
            const float4* sa = s_a + (t * kSpM + (m - m0)) * 4;
#pragma unroll
            for (int z2 = 0; z2 < kFsSlab / 2; ++z2) {
              if (2 * z2 < nz) {
                const float4 a = sa[z2];
                acc[2 * z2].x = fmaf(w, a.x, acc[2 * z2].x);
                acc[2 * z2].y = fmaf(w, a.y, acc[2 * z2].y);
                acc[2 * z2 + 1].x = fmaf(w, a.z, acc[2 * z2 + 1].x);
                acc[2 * z2 + 1].y = fmaf(w, a.w, acc[2 * z2 + 1].y);
              }
            }
          }
        }
        __syncthreads();
      }
    }
    __syncthreads();                 // every thread is done with s_seg before it changes
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
  __shared__ float2 s_tw[fft_line_len(M)];
  __shared__ float2 s_line[LPW][fft_line_len(M)];
  const int line = threadIdx.x / TL, lt = threadIdx.x % TL;
  const int L = blockIdx.x * LPW + line;
  const int z = L / W, y = L % W;
  for (int i = threadIdx.x; i < M; i += kT) s_tw[fpi(i)] = tw[i];
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
    k_fs_spread<N><<<(unsigned)((M / kSpTile) * (M / kSpTile)), kT, 0, st>>>(A, G, f, nz);  \
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
