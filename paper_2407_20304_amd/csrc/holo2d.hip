// Batched independent single-angle, multi-plane retrievals (psi is the
// unknown; Eq. 10 and Eq. 11 with N_theta = 1, own probe and reference per
// instance), for instances of uneven square sizes in one packed layout.
//
// Every pass is one launch over all instances and planes: a host-built table
// lists one item per workgroup (instance, plane/job, first line), the kernel
// switches on the instance's edge length to the FFT specialised for it.
//   probe   rows+columns: Q_j = D_{rho_probe_j} q, P = D_1 q, reference cost
//           and residual r_ref, the columns of D_{-1} on r_ref
//   A       rows: phi = 1 + B_j(psi - 1), x = Q_j phi, row propagation
//   B       columns: propagation, residual, cost, adjoint propagation
//   C       rows: adjoint propagation -> w, X = conj(Q_j) w, G_j = conj(phi) w
//           and at once the rows of D_{-rho_probe_j} on G_j; the rows of
//           D_{-1} on r_ref
//   Gq      per column tile: the columns of every D_{-rho_probe_j} G_j,
//           summed over j before one inverse transform, plus D_{-1} r_ref:
//           g_q = sum_j D_{-rho_probe_j} G_j + D_{-1} r_ref
//   gather  g_psi = sum_j B_j^T X_j
//   reduce  per-instance cost from double partials
#include "holo2d_internal.hpp"
#include "fft_lds.hpp"

namespace holo {

constexpr int kT2 = 256;

__host__ __device__ constexpr int b_rows_tl(int n) { return fft_row_threads(n); }
__host__ __device__ constexpr int b_rows_lpw(int n) { return kT2 / fft_row_threads(n); }
// Columns per column-pass workgroup: 8 from 384 on, so that the tile of a
// batch whose instances are at most 512 px fits 37 KB of LDS (four
// workgroups per CU instead of two).
__host__ __device__ constexpr int b_cols_tc(int n) { return n >= 384 ? 8 : 16; }
// Pitch of one column line of the tile: the padded line plus 4, so that the
// tile loads (columns of consecutive threads at one row) spread over banks.
__host__ __device__ constexpr int b_col_pitch(int n) { return fft_line_len(n) + 4; }
// LDS of one column workgroup of size n: twiddles plus the tile.
__host__ __device__ constexpr int b_cols_lds(int n) { return fft_line_len(n) + b_cols_tc(n) * b_col_pitch(n); }

// The probe-gradient column pass keeps every plane's spectrum sum in
// registers next to the plane being transformed: 4 columns per workgroup
// (64 threads per column) keep that to 2 x n / 64 elements per thread.
__host__ __device__ constexpr int b_gq_tc(int) { return 4; }
__host__ __device__ constexpr int b_gq_lds(int n) { return fft_line_len(n) + b_gq_tc(n) * b_col_pitch(n); }

int b2_rows_per_wg(int n) { return b_rows_lpw(n); }
int b2_cols_per_wg(int n) { return b_cols_tc(n); }
int b2_gq_per_wg(int n) { return b_gq_tc(n); }
bool b2_size_supported(int n) {
  switch (n) {
    case 64: case 128: case 192: case 256: case 384: case 512: case 1024: return true;
    default: return false;
  }
}

// LDS budget shared by every specialisation (twiddles + lines / columns).
constexpr int kRowLds = 1024 + 3072;          // float2 elements
// column-kernel LDS (float2) for batches up to 512 px and with 1024 px
constexpr int kColLdsSmall = b_cols_lds(512), kColLdsLarge = b_cols_lds(1024);
static_assert(b_cols_lds(384) <= kColLdsSmall && b_cols_lds(256) <= kColLdsSmall &&
                  b_cols_lds(192) <= kColLdsSmall && b_cols_lds(128) <= kColLdsSmall &&
                  b_cols_lds(64) <= kColLdsSmall,
              "small column LDS covers every size up to 512");

__device__ __forceinline__ double b_src_pos(double c, double m, int idx) {
  return fma(m, (double)idx - c, c);
}

struct BTaps {
  int i0, i1;
  float w0, w1;
};

__device__ __forceinline__ BTaps b_fwd_taps(double c, double m, int idx, int n) {
  const double sp = b_src_pos(c, m, idx);
  const double fl = floor(sp);
  const int i0 = (int)fl;
  const float w = (float)(sp - fl);
  BTaps t;
  const bool v0 = i0 >= 0 && i0 < n, v1 = i0 + 1 >= 0 && i0 + 1 < n;
  t.w0 = v0 ? 1.0f - w : 0.0f;
  t.w1 = v1 ? w : 0.0f;
  t.i0 = v0 ? i0 : 0;
  t.i1 = v1 ? i0 + 1 : 0;
  return t;
}

__device__ __forceinline__ float2 b_phi(const float2* __restrict__ psi, int n, const BTaps& ty,
                                        const BTaps& tx) {
  const float2 a = psi[(size_t)ty.i0 * n + tx.i0], b = psi[(size_t)ty.i0 * n + tx.i1];
  const float2 c = psi[(size_t)ty.i1 * n + tx.i0], d = psi[(size_t)ty.i1 * n + tx.i1];
  const float w00 = ty.w0 * tx.w0, w01 = ty.w0 * tx.w1, w10 = ty.w1 * tx.w0, w11 = ty.w1 * tx.w1;
  return make_float2(1.0f + w00 * (a.x - 1.f) + w01 * (b.x - 1.f) + w10 * (c.x - 1.f) + w11 * (d.x - 1.f),
                     w00 * a.y + w01 * b.y + w10 * c.y + w11 * d.y);
}

// ---------------------------------------------------------------------------
// Rows
// ---------------------------------------------------------------------------

template <int N>
__device__ __forceinline__ void b_rows_body(const B2Args& A, const B2Item& it, float2* lds) {
  constexpr int TL = b_rows_tl(N), LPW = b_rows_lpw(N), E = N / TL;
  static_assert((LPW + 1) * fft_line_len(N) <= kRowLds, "twiddles and row lines fit the LDS");
  float2* s_tw = lds;
  const int line = threadIdx.x / TL, lt = threadIdx.x % TL;
  // lines stored padded (element s at fpi(s)): conflict-free FFT stages
  float2* L = lds + fft_line_len(N) + line * fft_line_len(N);
  const B2Inst in = A.inst[it.inst];
  for (int i = threadIdx.x; i < N; i += kT2) s_tw[fpi(i)] = in.tw[i];
  const int z = it.line0 + line;
  const size_t fr = (size_t)N * N;
  const int j = it.job;
  const int nd = A.nd;
  const double c = N / 2.0;
  const float2* src;
  float2* dst;
  int chirp;
  bool conj;
  switch (A.mode) {
    case kB2RowsProbe:   // q -> Q_j (job < nd) or P (job == nd)
      src = A.q + in.off;
      dst = (j < nd) ? A.Q + in.off * nd + j * fr : A.P + in.off;
      chirp = (j < nd) ? nd + j : 2 * nd;
      conj = false;
      break;
    case kB2RowsA:
      src = nullptr;
      dst = A.X + in.off * nd + j * fr;
      chirp = j;
      conj = false;
      break;
    default:             // kB2RowsC, kB2RowsCGq
      if (j < nd) {
        src = A.X + in.off * nd + j * fr;
        dst = A.X + in.off * nd + j * fr;
        chirp = j;
      } else {           // reference residual -> rows of D_{-1}
        src = A.P + in.off;
        dst = A.P + in.off;
        chirp = 2 * nd;
      }
      conj = true;
      break;
  }
  // The thread's row elements s = lt + e TL stay in registers from load to
  // store; the line in LDS is only the transforms' exchange buffer.
  float2 v[E];
  if (A.mode == kB2RowsA) {
    const double m = A.mag[j];
    const BTaps ty = b_fwd_taps(c, m, z, N);
    const float2* psi = A.psi + in.off;
    const float2* Qr = A.Q + in.off * nd + j * fr + (size_t)z * N;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int s = lt + e * TL;
      v[e] = cmul(Qr[s], b_phi(psi, N, ty, b_fwd_taps(c, m, s, N)));
    }
  } else {
    const float2* r = src + (size_t)z * N;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = r[lt + e * TL];
  }
  // A line within one wavefront synchronises only there (s_tw is behind
  // the barrier; otherwise the first stage's barrier covers it).
  constexpr bool WL = TL <= 64;
  if constexpr (WL) __syncthreads();
  fft_e<N, TL, false, true, WL>(v, L, s_tw, lt);
  const float2* ch = in.chirp + (size_t)chirp * N;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int s = lt + e * TL;
    v[e] = conj ? cmulc(v[e], ch[s]) : cmul(v[e], ch[s]);
  }
  fft_e<N, TL, true, true, WL>(v, L, s_tw, lt);
  float2* o = dst + (size_t)z * N;
  if ((A.mode == kB2RowsC || A.mode == kB2RowsCGq) && j < nd) {
    // X = conj(Q_j) w; with the probe gradient, G_j = conj(phi) w goes
    // through the rows of D_{-rho_probe_j} at once
    const bool gq = A.mode == kB2RowsCGq;
    const float2* Qr = A.Q + in.off * nd + j * fr + (size_t)z * N;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int s = lt + e * TL;
      o[s] = cmulc(v[e], Qr[s]);
    }
    if (gq) {
      const double m = A.mag[j];
      const BTaps ty = b_fwd_taps(c, m, z, N);
      const float2* psi = A.psi + in.off;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int s = lt + e * TL;
        v[e] = cmulc(v[e], b_phi(psi, N, ty, b_fwd_taps(c, m, s, N)));
      }
      fft_e<N, TL, false, true, WL>(v, L, s_tw, lt);
      const float2* cq = in.chirp + (size_t)(nd + j) * N;
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = cmulc(v[e], cq[lt + e * TL]);
      fft_e<N, TL, true, true, WL>(v, L, s_tw, lt);
      float2* Gr = A.G + in.off * nd + j * fr + (size_t)z * N;
#pragma unroll
      for (int e = 0; e < E; ++e) Gr[lt + e * TL] = v[e];
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) o[lt + e * TL] = v[e];
  }
  (void)LPW;
}

// (four waves per SIMD: the padded twiddle addresses would otherwise take
// it just past 128 VGPRs)
__global__ __launch_bounds__(kT2) __attribute__((amdgpu_waves_per_eu(4))) void k2_rows(
    B2Args A, const B2Item* __restrict__ items) {
  __shared__ float2 lds[kRowLds];
  const B2Item it = items[blockIdx.x];
  switch (A.inst[it.inst].n) {
#define CASE(N) case N: b_rows_body<N>(A, it, lds); break;
    CASE(64) CASE(128) CASE(192) CASE(256) CASE(384) CASE(512) CASE(1024)
#undef CASE
    default: break;
  }
}

// ---------------------------------------------------------------------------
// Columns
// ---------------------------------------------------------------------------

// Amplitude functional (F2): r = 2 (v - a v/|v|) in place (v/|v| := 0 at
// |v| = 0), returns (|v| - a)^2.  Intensity functional (F1, `a` is then the
// intensity d): r = 4 (|v|^2 - d) v, returns (|v|^2 - d)^2.
__device__ __forceinline__ double b_residual(float2& v, float a, int functional) {
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

__device__ __forceinline__ void b_block_sum(double v, double* out) {
  __shared__ double red[kT2];
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int o = kT2 / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

template <int N>
__device__ __forceinline__ void b_cols_body(const B2Args& A, const B2Item& it, float2* lds) {
  constexpr int TC = b_cols_tc(N), TLc = kT2 / TC;
  float2* s_tw = lds;
  const int cidx = threadIdx.x / TLc, lt = threadIdx.x % TLc;
  // column lines stored padded (element zz at fpi(zz)), pitch b_col_pitch
  constexpr int CP = b_col_pitch(N);
  float2* col0 = lds + fft_line_len(N);
  float2* Lc = col0 + cidx * CP;
  const B2Inst in = A.inst[it.inst];
  for (int i = threadIdx.x; i < N; i += kT2) s_tw[fpi(i)] = in.tw[i];
  const size_t fr = (size_t)N * N;
  const int j = it.job, nd = A.nd;
  const int s0 = it.line0;
  float2* frame;
  const float* amp = nullptr;
  int chirp;
  bool adj_after = false;
  if (A.mode == kB2ColsProbe) {
    frame = (j < nd) ? A.Q + in.off * nd + j * fr : A.P + in.off;
    chirp = (j < nd) ? nd + j : 2 * nd;
    if (j == nd) {                 // reference: residual, then D_{-1} columns
      amp = A.amp_ref + in.off;
      adj_after = A.want_gq != 0;
    }
  } else {                         // kB2ColsB
    frame = A.X + in.off * nd + j * fr;
    chirp = j;
    amp = A.amp ? A.amp + in.off * nd + j * fr : nullptr;
    adj_after = A.amp != nullptr && A.want_grad;
  }
  for (int i = threadIdx.x; i < N * TC; i += kT2) {
    const int zz = i / TC, cc = i % TC;
    col0[cc * CP + fpi(zz)] = frame[(size_t)zz * N + s0 + cc];
  }
  const float2* ch = in.chirp + (size_t)chirp * N;
  // The thread's column elements zz = lt + e TLc stay in registers around
  // the transforms; the tile is touched to load, to store and for the
  // residual (amplitudes read in the coalesced tile order).
  constexpr int EC = N / TLc;
  constexpr bool WL = TLc <= 64;
  float2 v[EC];
  __syncthreads();   // tile and s_tw
#pragma unroll
  for (int e = 0; e < EC; ++e) v[e] = Lc[fpi(lt + e * TLc)];
  fft_e<N, TLc, false, true, WL>(v, Lc, s_tw, lt);
#pragma unroll
  for (int e = 0; e < EC; ++e) v[e] = cmul(v[e], ch[lt + e * TLc]);
  fft_e<N, TLc, true, true, WL>(v, Lc, s_tw, lt);
  if (amp) {
    fft_sync<WL>();   // the column's exchange reads are done
#pragma unroll
    for (int e = 0; e < EC; ++e) Lc[fpi(lt + e * TLc)] = v[e];
    __syncthreads();
    double acc = 0.0;
    for (int i = threadIdx.x; i < N * TC; i += kT2) {
      const int zz = i / TC, cc = i % TC;
      float2 t = col0[cc * CP + fpi(zz)];
      acc += b_residual(t, amp[(size_t)zz * N + s0 + cc], A.functional);
      col0[cc * CP + fpi(zz)] = t;
    }
    b_block_sum(acc, A.Fpart + it.slot);   // (its barriers publish the residual)
#pragma unroll
    for (int e = 0; e < EC; ++e) v[e] = Lc[fpi(lt + e * TLc)];
  }
  if (adj_after) {
    fft_e<N, TLc, false, true, WL>(v, Lc, s_tw, lt);
#pragma unroll
    for (int e = 0; e < EC; ++e) v[e] = cmulc(v[e], ch[lt + e * TLc]);
    fft_e<N, TLc, true, true, WL>(v, Lc, s_tw, lt);
  }
  if (A.mode == kB2ColsB && A.amp && !A.want_grad) return;  // objective only
  __syncthreads();   // every column's exchange reads are done
#pragma unroll
  for (int e = 0; e < EC; ++e) Lc[fpi(lt + e * TLc)] = v[e];
  __syncthreads();
  for (int i = threadIdx.x; i < N * TC; i += kT2) {
    const int zz = i / TC, cc = i % TC;
    frame[(size_t)zz * N + s0 + cc] = col0[cc * CP + fpi(zz)];
  }
}

// Work item of workgroup h in a launch of n items for the column kernels.
// The dispatcher hands workgroup h to XCD h mod 8; here each XCD takes runs
// of kXcdRun consecutive items (neighbouring column tiles, whose row pieces
// share cache lines, then share that XCD's L2), and the runs of the eight
// XCDs interleave over the item list, so every XCD gets a mix of the
// instance sizes.  Items past the last whole round keep their own index.
constexpr int kXcdRun = 8;
__device__ __forceinline__ int xcd_runs(int h, int n) {
  constexpr int R = 8 * kXcdRun;
  if (h >= (n / R) * R) return h;
  const int x = h & 7, l = h >> 3;
  return (l / kXcdRun) * R + x * kXcdRun + l % kXcdRun;
}

// LDS: the host launches the small instantiation only for batches whose
// largest instance is at most 512 px.
template <int LDS>
__global__ __launch_bounds__(kT2) void k2_cols(B2Args A, const B2Item* __restrict__ items) {
  __shared__ float2 lds[LDS];
  const B2Item it = items[xcd_runs(blockIdx.x, gridDim.x)];
  switch (A.inst[it.inst].n) {
#define CASE(N) \
  case N:       \
    if constexpr (b_cols_lds(N) <= LDS) b_cols_body<N>(A, it, lds); \
    break;
    CASE(64) CASE(128) CASE(192) CASE(256) CASE(384) CASE(512) CASE(1024)
#undef CASE
    default: break;
  }
}

// Probe gradient of one column tile: every plane's G_j (rows already
// through D_{-rho_probe_j}) is loaded, its columns transformed and weighted
// by the conjugate column transfer factors, and the spectra are summed in
// registers (each thread keeps the column elements it owns); one inverse
// transform of the sum, plus the reference term D_{-1} r_ref, is g_q.
template <int N>
__device__ __forceinline__ void b_cols_gq_sum(const B2Args& A, const B2Item& it, float2* lds) {
  constexpr int TC = b_gq_tc(N), TLc = kT2 / TC, EC = N / TLc;
  static_assert(N % TLc == 0, "column elements per thread");
  float2* s_tw = lds;
  const int cidx = threadIdx.x / TLc, lt = threadIdx.x % TLc;
  constexpr int CP = b_col_pitch(N);
  float2* col0 = lds + fft_line_len(N);
  float2* Lc = col0 + cidx * CP;
  const B2Inst in = A.inst[it.inst];
  for (int i = threadIdx.x; i < N; i += kT2) s_tw[fpi(i)] = in.tw[i];
  const size_t fr = (size_t)N * N;
  const int nd = A.nd, s0 = it.line0;
  constexpr bool WL = TLc <= 64;
  float2 acc[EC];
#pragma unroll
  for (int e = 0; e < EC; ++e) acc[e] = make_float2(0.f, 0.f);
  for (int j = 0; j < nd; ++j) {
    const float2* frame = A.G + in.off * nd + j * fr;
    __syncthreads();   // the previous plane's tile has been read
    for (int i = threadIdx.x; i < N * TC; i += kT2) {
      const int zz = i / TC, cc = i % TC;
      col0[cc * CP + fpi(zz)] = frame[(size_t)zz * N + s0 + cc];
    }
    __syncthreads();
    float2 v[EC];
#pragma unroll
    for (int e = 0; e < EC; ++e) v[e] = Lc[fpi(lt + e * TLc)];
    fft_e<N, TLc, false, true, WL>(v, Lc, s_tw, lt);
    const float2* ch = in.chirp + (size_t)(nd + j) * N;
#pragma unroll
    for (int e = 0; e < EC; ++e) {
      const float2 t = cmulc(v[e], ch[lt + e * TLc]);
      acc[e].x += t.x;
      acc[e].y += t.y;
    }
  }
  fft_e<N, TLc, true, true, WL>(acc, Lc, s_tw, lt);
  __syncthreads();   // every column's exchange reads are done
#pragma unroll
  for (int e = 0; e < EC; ++e) Lc[fpi(lt + e * TLc)] = acc[e];
  __syncthreads();
  const float2* ref = A.P + in.off;
  float2* gq = A.g_q + in.off;
  for (int i = threadIdx.x; i < N * TC; i += kT2) {
    const int zz = i / TC, cc = i % TC;
    const size_t o = (size_t)zz * N + s0 + cc;
    const float2 v = col0[cc * CP + fpi(zz)], r = ref[o];
    gq[o] = make_float2(v.x + r.x, v.y + r.y);
  }
}

template <int LDS>
__global__ __launch_bounds__(kT2) __attribute__((amdgpu_waves_per_eu(4))) void k2_gq_sum(B2Args A, const B2Item* __restrict__ items) {
  __shared__ float2 lds[LDS];
  const B2Item it = items[xcd_runs(blockIdx.x, gridDim.x)];
  switch (A.inst[it.inst].n) {
#define CASE(N) \
  case N:       \
    if constexpr (b_gq_lds(N) <= LDS) b_cols_gq_sum<N>(A, it, lds); \
    break;
    CASE(64) CASE(128) CASE(192) CASE(256) CASE(384) CASE(512) CASE(1024)
#undef CASE
    default: break;
  }
}

// ---------------------------------------------------------------------------
// Gather (B^T over planes) and per-instance reduction
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kT2) void k2_gather(B2Args A, const B2Item* __restrict__ items) {
  const B2Item it = items[blockIdx.x];
  const B2Inst in = A.inst[it.inst];
  const int n = in.n;
  const int p = it.line0 + threadIdx.x;
  if (p >= n * n) return;
  const int z = p / n, s = p % n;
  const size_t fr = (size_t)n * n;
  float ax = 0.f, ay = 0.f;
  for (int j = 0; j < A.nd; ++j) {
    // the two weighted taps of each axis (from the plan's table): four
    // unconditional loads
    const B2AdjTap tz = in.adj[j * n + z], ts = in.adj[j * n + s];
    const float2* Xj = A.X + in.off * A.nd + j * fr;
    const int rz[2] = {tz.d0, tz.d1}, rs[2] = {ts.d0, ts.d1};
    const float wz[2] = {tz.w0, tz.w1}, ws[2] = {ts.w0, ts.w1};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const float wt = wz[a] * ws[b];
        const float2 v = Xj[(size_t)rz[a] * n + rs[b]];   // in range
        ax += wt * v.x;
        ay += wt * v.y;
      }
    }
  }
  A.g_psi[in.off + p] = make_float2(ax, ay);
}

__global__ __launch_bounds__(kT2) void k2_reduce(const double* __restrict__ parts,
                                                 const int2* __restrict__ ranges,
                                                 double* __restrict__ F) {
  const int2 r = ranges[blockIdx.x];
  double acc = 0.0;
  for (int i = r.x + threadIdx.x; i < r.y; i += kT2) acc += parts[i];
  b_block_sum(acc, F + blockIdx.x);
}

hipError_t launch_b2_rows(const B2Args& A, const B2Item* items, int n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k2_rows<<<n, kT2, 0, st>>>(A, items);
  return hipGetLastError();
}

hipError_t launch_b2_cols(const B2Args& A, const B2Item* items, int n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (A.max_n <= 512)
    k2_cols<kColLdsSmall><<<n, kT2, 0, st>>>(A, items);
  else
    k2_cols<kColLdsLarge><<<n, kT2, 0, st>>>(A, items);
  return hipGetLastError();
}

hipError_t launch_b2_gq_sum(const B2Args& A, const B2Item* items, int n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (!A.g_q || !A.P) return hipErrorInvalidValue;
  if (A.max_n <= 512)
    k2_gq_sum<b_gq_lds(512)><<<n, kT2, 0, st>>>(A, items);
  else
    k2_gq_sum<b_gq_lds(1024)><<<n, kT2, 0, st>>>(A, items);
  return hipGetLastError();
}

hipError_t launch_b2_gather(const B2Args& A, const B2Item* items, int n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (!A.g_psi) return hipErrorInvalidValue;
  k2_gather<<<n, kT2, 0, st>>>(A, items);
  return hipGetLastError();
}

hipError_t launch_b2_reduce(const double* parts, const int2* ranges, int n_inst, double* F,
                            hipStream_t st) {
  k2_reduce<<<n_inst, kT2, 0, st>>>(parts, ranges, F);
  return hipGetLastError();
}

}  // namespace holo
