// Joseph ray sums R_k (Eq. 14) and their transpose for gfx950 (MI355X).
//
//   block_volume  z-blocked copies of the volume (and of its x/y transpose)
//                 with zero-padded rows, read by the forward
//   radon_fwd     Joseph ray sums, angle groups sharing row windows staged in
//                 LDS by LDS-direct loads (16 lanes cover the 64 slices of
//                 one bin group, each thread owns 4 slices x 4 bins), fused
//                 exp(i kappa p) epilogue
//   radon_adj     transpose as a triangle-footprint gather over all angles
//                 (a workgroup per 16 x 16 voxel tile and kAdjZT slices,
//                 each thread a 2 x 2 voxel block and kAdjZT / 4 slices,
//                 angles in two classes by the sign of sin), sinogram
//                 segments staged in LDS per angle group by LDS-direct loads
// Both are bound by VALU issue and LDS operand delivery, not by HBM: every
// voxel is revisited once per angle.
#include <type_traits>

#include "holo_internal.hpp"

namespace holo {

// Z-blocked copies of the volume for the ray sums: ub[z / ZT][y][P + x][z % ZT]
// (walks along y) and uTb[z / ZT][x][P + y][z % ZT] (walks along x, i.e. the
// x/y-transposed volume), rows padded by P = kFwdPad zero columns on each
// side.  A workgroup moves a 16 x 16 x ZT brick; the workgroups at the
// first and last brick column also clear the padding of their 16 rows.
__global__ __launch_bounds__(kThreads) void k_block_volume(const float2* __restrict__ u,
                                                           float2* __restrict__ ub,
                                                           float2* __restrict__ uTb, int W) {
  constexpr int ZT = kVolZB, P = kFwdPad;
  // one 16 x 17 plane per slice, planes 274 elements apart: the write phase
  // reads down the slices (the 16 lanes of consecutive z at one position,
  // the next 16 at the neighbouring one), which a plane stride of 272 put
  // on two bank pairs; 274 = 18 (mod 32) spreads the 16 slices over the
  // even bank pairs and their neighbours over the odd ones
  constexpr int PL = 16 * 17 + 2;
  __shared__ float2 brick[ZT * PL];
  const int nt = W / 16, Wf = vol_row(W);
  const int x0 = (blockIdx.x % nt) * 16, y0 = (blockIdx.x / nt) * 16;
  const int zb = blockIdx.y;
  const size_t WW = (size_t)W * W, WWf = (size_t)W * Wf;
  // read along x (contiguous)
  for (int i = threadIdx.x; i < ZT * 256; i += kThreads) {
    const int xx = i & 15, yy = (i >> 4) & 15, zz = i >> 8;
    brick[zz * PL + yy * 17 + xx] = u[(size_t)(zb * ZT + zz) * WW + (size_t)(y0 + yy) * W + x0 + xx];
  }
  __syncthreads();
  float2* bb = ub + (size_t)zb * WWf * ZT;
  float2* tb = uTb ? uTb + (size_t)zb * WWf * ZT : nullptr;
  // write with z fastest (contiguous 128-byte runs)
  for (int i = threadIdx.x; i < ZT * 256; i += kThreads) {
    const int zz = i % ZT, p = i / ZT;
    const int a = p & 15, b = p >> 4;
    bb[((size_t)(y0 + b) * Wf + P + x0 + a) * ZT + zz] = brick[zz * PL + b * 17 + a];
    if (tb) tb[((size_t)(x0 + b) * Wf + P + y0 + a) * ZT + zz] = brick[zz * PL + a * 17 + b];
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
// direction (one wave per angle), NB (16 by default, or 8: a tuning choice)
// consecutive bins and kFwdZT slices.
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
// thread owns a 2 x 2 voxel block (an x pair in two neighbouring rows) and
// a quarter of the slices (kAdjZT / 4, one slice group per wave).  It loops
// over all angles in groups of kAdjNA (one wave loads each angle of a
// group): the kAdjSeg bins of each slice that the tile projects onto are
// copied straight from the sinogram into LDS, [angle][slice][bin], by
// LDS-direct loads one group ahead of use (two group buffers); per slice a
// thread then reads the four consecutive bins that carry its four voxels'
// weights (8 bytes of LDS per voxel and slice).  The lanes of a wave read
// bins of one 256-byte bin row: no bank conflicts.  The angles come in two
// classes, each in a list of its own (ascending angle indices): after the
// reversal of the rows with cos < 0, sin >= 0 (class 0) or sin < 0 (class
// 1).  Within a class the lowest-projecting voxel of every block is the
// same one, so each class runs a loop specialised for it; each class is
// padded to whole groups with dummy angles whose segment is the zero
// padding of a row.  Sinogram rows are zero-padded by kAdjPad bins, so a segment
// is read without bounds checks.  A voxel projecting to fractional bin q
// takes max(0, 1 - |i - q| / h) / h of bin i (h = max(|cos|, |sin|)) --
// exactly the weight Joseph's interpolation gave it.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_radon_adj(const float2* __restrict__ S,
                                                         float2* __restrict__ gu, DevGeom g,
                                                         const double* __restrict__ ang,
                                                         int k0, const int* __restrict__ ord0,
                                                         int n0, const int* __restrict__ ord1,
                                                         int n1) {
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
  __shared__ int s_sl[2][TW], s_row[2][TW];
  __shared__ float s_f0[2][TW], s_c[2][TW], s_s[2][TW], s_ih[2][TW], s_ih2[2][TW];
  const float2* tile = reinterpret_cast<const float2*>(tile4);
  const int W = g.W, H = g.H, Wp = sino_row(W);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // logical order: slice blocks slowest; within one, the tiles in square
  // groups of GS x GS (x fastest within a group, groups in rows), so the
  // workgroups resident on one XCD cover a compact patch of the slice block
  // whose sinogram segments, per angle, are few and stay in that XCD's L2
  const int L = xcd_logical(blockIdx.x, gridDim.x);
  const int nt = W / 16;
  const int GS = (nt % 8 == 0) ? 8 : (nt % 4 == 0) ? 4 : (nt % 2 == 0) ? 2 : 1;
  const int tl = L % (nt * nt), grp = tl / (GS * GS), in_grp = tl % (GS * GS);
  const int x0 = ((grp % (nt / GS)) * GS + in_grp % GS) * 16;
  const int y0 = ((grp / (nt / GS)) * GS + in_grp / GS) * 16;
  // thread: voxels (x, y), (x + 1, y), (x, y + 1), (x + 1, y + 1),
  // x = x0 + 2 px, y = y0 + 2 py, and the 4 slices of slice group sg (its
  // wave) of the block
  const int px = threadIdx.x & 7, py = (threadIdx.x >> 3) & 7, sg = threadIdx.x >> 6;
  const int x = x0 + 2 * px, y = y0 + 2 * py;
  const int z0 = (L / (nt * nt)) * ZT;
  const double X0 = (double)x0 - g.cW, X1 = X0 + 15.0;
  const double Y0 = (double)y0 - g.cW, Y1 = Y0 + 15.0;

  // Position p of the angle sequence: class 0's list padded to a multiple of
  // NA, then class 1's.  Returns the angle (a dummy repeats its class's last
  // angle) and whether it is a dummy.
  const int G0 = (n0 + NA - 1) / NA, G1 = (n1 + NA - 1) / NA;
  const int ng = G0 + G1, Kp = ng * NA;
  auto angle_at = [&](int p, bool& dummy) {
    if (p < G0 * NA) {
      dummy = p >= n0;
      return ord0[min(p, n0 - 1)];
    }
    p -= G0 * NA;
    dummy = p >= n1;
    return ord1[min(p, n1 - 1)];
  };

  // Set-up of position w * TW + t for threads t < TW, in double precision: the
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
      bool dummy;
      const int kk = angle_at(min(w * TW + t, Kp - 1), dummy);
      const double* ap = ang + (size_t)kk * kAngleStride;
      // an angle with cos < 0 has its row stored reversed: it is the angle
      // theta - pi, direction (-cos, -sin), positions W - 1 - q
      const bool mir = ap[kCos] < 0.0;
      const double C = mir ? -ap[kCos] : ap[kCos], Sn = mir ? -ap[kSin] : ap[kSin];
      const double ih = ap[kInvH];
      const double cq = mir ? (double)(W - 1) - g.cW : g.cW;
      const double q0 = cq + X0 * C + Y0 * Sn;
      int sl = (int)floor(cq + fmin(X0 * C, X1 * C) + fmin(Y0 * Sn, Y1 * Sn)) - 2;
      sl -= sl & 1;                                     // even: 16-byte aligned bin pairs
      sl = min(max(sl, -kAdjPad), W + kAdjPad - SEG);
      // a dummy reads the zero padding left of its row; its weights are
      // zero there too (its taps fall far right of the segment)
      if (dummy) sl = -kAdjPad;
      s_sl[slot][t] = sl;
      s_row[slot][t] = kk - k0;
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
    const int p0 = gidx * NA;
    const int sl = __builtin_amdgcn_readfirstlane(s_sl[(p0 / TW) & 1][p0 % TW + wave]);
    const int row = __builtin_amdgcn_readfirstlane(s_row[(p0 / TW) & 1][p0 % TW + wave]);
    const float2* src = Sl + (size_t)row * HWp + sl;
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

  constexpr int ZS = ZT / 4;                        // slices per thread
  static_assert(ZS == 4 && NA == 4, "slice group per wave");
  // accumulators [voxel v = dx + 2 dy][slice]
  float ax[4][ZS], ay[4][ZS];
  float ox[4][ZS], oy[4][ZS];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int i = 0; i < ZS; ++i) { ax[v][i] = ay[v][i] = 0.f; ox[v][i] = oy[v][i] = 0.f; }

  constexpr int GPW = TW / NA;                      // groups per set-up window
  setup_window(0);
  __syncthreads();
  issue(0);
  // One group of NA angles of one class.
  auto group = [&](int gi, auto sneg) {
    constexpr bool SNEG = decltype(sneg)::value;
    const int p0 = gi * NA;
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
    if ((gi + 2) % GPW == 0 && (gi + 2) * NA < Kp) setup_window((gi + 2) / GPW);
    const int slot = (p0 / TW) & 1, base = p0 % TW;
    const float2* gb = tile + (gi % NBUF) * GF2;
    // One angle.  Its row has cos >= 0 (rows of angles with cos < 0 are
    // stored reversed), so the block's lowest fractional bin q belongs to
    // voxel (x, y) in class 0 and to (x, y + 1) in class 1 (SNEG); the
    // others lie at q + cos (the x neighbour of the lowest), q + |sin| (its
    // y neighbour) and q + cos + |sin| (the opposite corner), with
    // 1 <= cos + |sin| <= sqrt(2).  Every bin with a nonzero weight
    // (|i - q'| < h <= 1) is one of jm .. jm + 3, jm = floor(q): bins jm,
    // jm + 1 for the lowest voxel, jm .. jm + 2 for its two neighbours and
    // jm + 1 .. jm + 3 for the opposite corner; the weight is the footprint
    // max(0, 1/h - |i - q'| / h^2).
    constexpr int VL = SNEG ? 2 : 0, VX = SNEG ? 3 : 1, VY = SNEG ? 0 : 2, VXY = SNEG ? 1 : 3;
#pragma unroll 1
    for (int a = 0; a < NA; ++a) {
      const float ih = s_ih[slot][base + a], ih2 = s_ih2[slot][base + a];
      const float c = s_c[slot][base + a], sn = s_s[slot][base + a];
      const float as = SNEG ? -sn : sn;
      const float q = fmaf((float)(2 * py + (SNEG ? 1 : 0)), sn,
                           fmaf((float)(2 * px), c, s_f0[slot][base + a]));
      const int jm = min(max((int)floorf(q), 0), SEG - 4);
      const float d = q - (float)jm;                   // lowest voxel relative to bin jm
      auto wt = [&](float dist) { return fmaxf(0.0f, fmaf(-fabsf(dist), ih2, ih)); };
      const float dX = d + c, dY = d + as, dXY = dX + as;
      const float wL0 = wt(d), wL1 = wt(1.0f - d);
      const float wX0 = wt(dX), wX1 = wt(1.0f - dX), wX2 = wt(2.0f - dX);
      const float wY0 = wt(dY), wY1 = wt(1.0f - dY), wY2 = wt(2.0f - dY);
      const float wXY1 = wt(1.0f - dXY), wXY2 = wt(2.0f - dXY), wXY3 = wt(3.0f - dXY);
      const float2* tp = gb + a * ZT * SEG + sg * ZS * SEG + jm;
      // software pipeline: the four bins of slice i + LA are requested
      // before slice i is accumulated
      constexpr int LA = 1;
      float2 r[ZS][4];
      auto fetch = [&](int i) {
        const float2* t = tp + i * SEG;
#pragma unroll
        for (int b = 0; b < 4; ++b) r[i][b] = t[b];
      };
#pragma unroll
      for (int i = 0; i < LA; ++i) fetch(i);
#pragma unroll
      for (int i = 0; i < ZS; ++i) {
        if (i + LA < ZS) fetch(i + LA);
        const float2 r0 = r[i][0], r1 = r[i][1], r2 = r[i][2], r3 = r[i][3];
        ax[VL][i] = fmaf(wL1, r1.x, fmaf(wL0, r0.x, ax[VL][i]));
        ay[VL][i] = fmaf(wL1, r1.y, fmaf(wL0, r0.y, ay[VL][i]));
        ax[VX][i] = fmaf(wX2, r2.x, fmaf(wX1, r1.x, fmaf(wX0, r0.x, ax[VX][i])));
        ay[VX][i] = fmaf(wX2, r2.y, fmaf(wX1, r1.y, fmaf(wX0, r0.y, ay[VX][i])));
        ax[VY][i] = fmaf(wY2, r2.x, fmaf(wY1, r1.x, fmaf(wY0, r0.x, ax[VY][i])));
        ay[VY][i] = fmaf(wY2, r2.y, fmaf(wY1, r1.y, fmaf(wY0, r0.y, ay[VY][i])));
        ax[VXY][i] = fmaf(wXY3, r3.x, fmaf(wXY2, r2.x, fmaf(wXY1, r1.x, ax[VXY][i])));
        ay[VXY][i] = fmaf(wXY3, r3.y, fmaf(wXY2, r2.y, fmaf(wXY1, r1.y, ay[VXY][i])));
      }
    }
    // two-level single-precision sums: partials of up to 8 NA angles are
    // added into the outer sums
    if ((gi & 7) == 7 || gi + 1 >= ng) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int i = 0; i < ZS; ++i) {
          ox[v][i] += ax[v][i];
          oy[v][i] += ay[v][i];
          ax[v][i] = ay[v][i] = 0.f;
        }
    }
  };
  for (int gi = 0; gi < G0; ++gi) group(gi, std::integral_constant<bool, false>());
  for (int gi = G0; gi < ng; ++gi) group(gi, std::integral_constant<bool, true>());
  const size_t WW = (size_t)W * W;
#pragma unroll
  for (int i = 0; i < ZS; ++i) {
    float2* o = gu + (size_t)(z0 + sg * ZS + i) * WW + (size_t)y * W + x;
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
      *reinterpret_cast<float4*>(o + (size_t)dy * W) =
          make_float4(ox[2 * dy][i], oy[2 * dy][i], ox[2 * dy + 1][i], oy[2 * dy + 1][i]);
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

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
                            int k0, const int* ord0, int n0, const int* ord1, int n1,
                            hipStream_t st) {
  // the kernel reads the rows of angles with cos < 0 reversed
  if (!g.sino_mirror || n0 < 0 || n1 < 0 || n0 + n1 < 1) return hipErrorInvalidValue;
  const unsigned n = (unsigned)(g.W / 16) * (unsigned)(g.W / 16) * (unsigned)(g.H / kAdjZT);
  k_radon_adj<<<n, kThreads, 0, st>>>(S, gu, g, ang, k0, ord0, n0, ord1, n1);
  return hipGetLastError();
}

hipError_t launch_block_volume(const DevGeom& g, const float2* u, float2* ub, float2* uTb,
                               hipStream_t st) {
  const dim3 grid((g.W / 16) * (g.W / 16), g.H / kVolZB);
  k_block_volume<<<grid, kThreads, 0, st>>>(u, ub, uTb, g.W);
  return hipGetLastError();
}

}  // namespace holo
