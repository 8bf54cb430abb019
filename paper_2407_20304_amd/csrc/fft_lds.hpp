// In-LDS complex FFT of one line per thread group, for gfx950.
//
// Stockham autosort formulation: for each radix-R stage with P = product of
// the radices already applied, butterfly i (0 <= i < N/R) reads
// x[i + j N/R], multiplies input j by W_{PR}^{j (i mod P)}, applies an R-point
// DFT and writes output j to y[(i / P) P R + (i mod P) + j P].  Input and
// output are in natural order, so the transfer-function multiply in between
// indexes frequencies directly.  Each stage reads all its inputs into
// registers, synchronises, and writes in place, so one LDS line per transform
// suffices.
//
// Lengths are 2^a (radices 8, then 4 or 2; a plan ending in 4, 4 ends in
// one radix-16 stage instead when the line has N / 16 threads) and 3 * 2^a
// (one radix-3 stage first).  Twiddles come from a table tw[m] = exp(-2 pi i m / N) built in
// double precision on the host and staged in LDS by the caller in the padded
// layout of the lines (tw[m] at fpi(m), fft_line_len(N) elements): a stage
// reads the twiddles j k N / (P R) of its butterflies, strided by up to
// N / 8 entries, which the plain layout puts on a few banks.
#pragma once
#include <hip/hip_runtime.h>

namespace holo {

__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
__host__ __device__ constexpr int pow2_floor(int n) { return n <= 1 ? 1 : 2 * pow2_floor(n / 2); }

__host__ __device__ constexpr int fft_has3(int N) { return N % 3 == 0 ? 1 : 0; }
__host__ __device__ constexpr int fft_log2m(int N) { return ilog2(fft_has3(N) ? N / 3 : N); }

__host__ __device__ constexpr int fft_nstages(int N) {
  return fft_has3(N) +
         (fft_log2m(N) % 3 == 0 ? fft_log2m(N) / 3
          : fft_log2m(N) % 3 == 2 ? fft_log2m(N) / 3 + 1
          : (fft_log2m(N) >= 3 ? fft_log2m(N) / 3 + 1 : 1));
}

// Radix of stage t of the power-of-two part (2^L): 8 ... 8 then {}, {4},
// {4, 4} or {2}.
__host__ __device__ constexpr int fft_radix_pow2(int L, int t) {
  return (L % 3 == 0) ? 8
         : (L % 3 == 2) ? (t < L / 3 ? 8 : 4)
         : (L >= 3 ? (t < L / 3 - 1 ? 8 : 4) : 2);
}

// Radix of stage s of an N-point transform (one radix-3 stage first).
__host__ __device__ constexpr int fft_radix(int N, int s) {
  return (fft_has3(N) && s == 0) ? 3 : fft_radix_pow2(fft_log2m(N), s - fft_has3(N));
}

__host__ __device__ constexpr int fft_pstride(int N, int s) {
  return s == 0 ? 1 : fft_pstride(N, s - 1) * fft_radix(N, s - 1);
}

// Plans for a given number of threads per line.  A power of two whose
// radix plan ends in {4, 4} ends in one radix-16 stage instead when that
// stage has exactly one butterfly per thread (N / 16 == TL): one LDS round
// trip fewer per transform, no idle threads.
__host__ __device__ constexpr bool fft_use16(int N, int TL) {
  return !fft_has3(N) && fft_log2m(N) % 3 == 1 && fft_log2m(N) >= 4 && N / 16 == TL;
}
__host__ __device__ constexpr int fft_nstages_tl(int N, int TL) {
  return fft_nstages(N) - (fft_use16(N, TL) ? 1 : 0);
}
__host__ __device__ constexpr int fft_radix_tl(int N, int TL, int s) {
  return fft_use16(N, TL) && s == fft_nstages_tl(N, TL) - 1 ? 16 : fft_radix(N, s);
}
__host__ __device__ constexpr int fft_pstride_tl(int N, int TL, int s) {
  return s == 0 ? 1 : fft_pstride_tl(N, TL, s - 1) * fft_radix_tl(N, TL, s - 1);
}

// Threads that share one line in the row kernels: a power of two near N/8.
__host__ __device__ constexpr int fft_row_threads(int N) { return pow2_floor(N / 8); }

// Padded line layout (PADDED transforms): element n of a line is stored at
// n + n / 32, one spare slot per 32 elements (one bank cycle of 8-byte
// elements).  Contiguous accesses stay conflict-free, and the first radix-8
// stage, which writes with a stride of 8 elements (8 lanes of an LDS pass on
// one bank in a plain layout), becomes conflict-free too.
__host__ __device__ constexpr int fft_line_len(int N) { return N + N / 32; }
__device__ __forceinline__ int fpi(int n) { return (int)((unsigned)n + ((unsigned)n >> 5)); }
template <bool PADDED>
__device__ __forceinline__ int fidx(int n) { return PADDED ? fpi(n) : n; }
// padded length of a compile-time step
template <bool PADDED>
__host__ __device__ constexpr int pstep(int d) { return PADDED ? d + d / 32 : d; }

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int R, bool INV> struct Dft;

template <bool INV> struct Dft<2, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
  }
};

template <bool INV> struct Dft<3, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    const float s3 = 0.86602540378443864676f;  // sin(2 pi / 3)
    float2 t = cadd(v[1], v[2]);
    float2 d = csub(v[1], v[2]);
    float2 m = make_float2(v[0].x - 0.5f * t.x, v[0].y - 0.5f * t.y);
    float2 jd = mul_mi<INV>(d);  // -i d (forward) / +i d (inverse)
    v[0] = cadd(v[0], t);
    v[1] = make_float2(m.x + s3 * jd.x, m.y + s3 * jd.y);
    v[2] = make_float2(m.x - s3 * jd.x, m.y - s3 * jd.y);
  }
};

template <bool INV> struct Dft<4, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    float2 a2 = cadd(v[1], v[3]), a3 = mul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(a0, a2);
    v[2] = csub(a0, a2);
    v[1] = cadd(a1, a3);
    v[3] = csub(a1, a3);
  }
};

template <bool INV> struct Dft<8, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    const float r = 0.70710678118654752440f;
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV>::run(e);
    Dft<4, INV>::run(o);
    // o_k *= exp(-+ 2 pi i k / 8)
    float2 t1 = INV ? make_float2(r * (o[1].x - o[1].y), r * (o[1].x + o[1].y))
                    : make_float2(r * (o[1].x + o[1].y), r * (o[1].y - o[1].x));
    float2 t2 = mul_mi<INV>(o[2]);
    float2 t3 = INV ? make_float2(-r * (o[3].x + o[3].y), r * (o[3].x - o[3].y))
                    : make_float2(r * (o[3].y - o[3].x), -r * (o[3].x + o[3].y));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], t1);
    v[5] = csub(e[1], t1);
    v[2] = cadd(e[2], t2);
    v[6] = csub(e[2], t2);
    v[3] = cadd(e[3], t3);
    v[7] = csub(e[3], t3);
  }
};

// Ordering between the phases of a transform.  WAVE: each line is owned by
// threads of a single wavefront.  A wavefront's LDS accesses are performed
// in issue order, so a wavefront-scope fence (which only stops the compiler
// from moving accesses across it) orders them for every lane of the line;
// the other wavefronts of the workgroup go on without waiting.  Otherwise a
// workgroup barrier.
template <bool WAVE>
__device__ __forceinline__ void fft_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// 16-point DFT as 4 x 4: x[4 n1 + n2] -> 4-point DFTs over n1, twiddles
// W16^(n2 k1), 4-point DFTs over n2 -> X[k1 + 4 k2].
template <bool INV> struct Dft<16, INV> {
  // W16^m = exp(-+2 pi i m / 16) for the products m = n2 k1 that occur
  __device__ __forceinline__ static float2 w16(int m) {
    const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;
    const float r = 0.70710678118654752440f;
    float2 w = m == 1 ? make_float2(c1, -s1)
             : m == 2 ? make_float2(r, -r)
             : m == 3 ? make_float2(s1, -c1)
             : m == 4 ? make_float2(0.0f, -1.0f)
             : m == 6 ? make_float2(-r, -r)
                      : make_float2(-c1, s1);   // m == 9
    if (INV) w.y = -w.y;
    return w;
  }
  __device__ __forceinline__ static void run(float2* v) {
    float2 a[4][4];   // a[n2][k1]
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      float2 t[4] = {v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]};
      Dft<4, INV>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1)
        a[n2][k1] = (n2 == 0 || k1 == 0) ? t[k1] : cmul(t[k1], w16(n2 * k1));
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      Dft<4, INV>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
    }
  }
};

// One Stockham stage on `line` (LDS), executed by TL threads (thread lt).
template <int N, int TL, int R, int P, bool INV, bool PADDED, bool WAVE>
__device__ __forceinline__ void fft_stage(float2* line, const float2* tw, int lt) {
  constexpr int NB = N / R;
  constexpr int IT = (NB + TL - 1) / TL;
  // Padded addresses as a per-butterfly base plus compile-time steps:
  // fpi(b + j d) = fpi(b) + j d + (j d) / 32 whenever the base's offset
  // within its group of 32 never changes which group step j d lands in.
  // Reads (b = i < NB, d = NB): NB a multiple of 32 or a divisor of 32.
  // Writes (b = (i - k) R + k, d = P): P a multiple of 32, or P dividing 32
  // with P R a divisor or a multiple of 32.  Other strides (around a radix-3
  // stage) map each address on its own.
  constexpr bool RLIN = !PADDED || NB % 32 == 0 || 32 % NB == 0;
  constexpr bool WLIN = !PADDED || P % 32 == 0 ||
                        (32 % P == 0 && (32 % (P * R) == 0 || (P * R) % 32 == 0));
  float2 v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int i = lt + it * TL;
    if (NB % TL == 0 || i < NB) {
      if constexpr (RLIN) {
        const int rb = fidx<PADDED>(i);
#pragma unroll
        for (int j = 0; j < R; ++j) v[it][j] = line[rb + pstep<PADDED>(j * NB)];
      } else {
#pragma unroll
        for (int j = 0; j < R; ++j) v[it][j] = line[fidx<PADDED>(i + j * NB)];
      }
    }
  }
  fft_sync<WAVE>();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int i = lt + it * TL;
    if (NB % TL == 0 || i < NB) {
      const int k = i % P;
      if (P > 1) {
#pragma unroll
        for (int j = 1; j < R; ++j) {
          float2 w = tw[fpi(j * k * (N / (P * R)))];
          if (INV) w.y = -w.y;
          v[it][j] = cmul(v[it][j], w);
        }
      }
      Dft<R, INV>::run(v[it]);
      const int base = (i - k) * R + k;
      if constexpr (WLIN) {
        const int wb = fidx<PADDED>(base);
#pragma unroll
        for (int j = 0; j < R; ++j) line[wb + pstep<PADDED>(j * P)] = v[it][j];
      } else {
#pragma unroll
        for (int j = 0; j < R; ++j) line[fidx<PADDED>(base + j * P)] = v[it][j];
      }
    }
  }
  fft_sync<WAVE>();
}

// Register-chained form.  Thread lt holds the line elements e[m] =
// x[lt + m TL] (m < N / TL).  When every stage of the plan gives each
// thread the same number of butterflies (N / R a multiple of TL for every
// radix R), those are exactly the inputs of its first-stage butterflies
// (i = lt + it TL reads x[i + j N / R]) and the outputs of its last-stage
// butterflies (written to i + j N / R, since the last stage has P = N / R).
// The first stage then reads registers and the last writes them: a
// transform costs one LDS round trip fewer than its stage count, and the
// work between a forward and an inverse transform (a transfer-function
// multiply, a residual) needs none.
template <int N, int TL, int S = 0>
__host__ __device__ constexpr bool fft_even_stages() {
  if constexpr (S >= fft_nstages_tl(N, TL)) {
    return true;
  } else {
    return (N / fft_radix_tl(N, TL, S)) % TL == 0 && fft_even_stages<N, TL, S + 1>();
  }
}

template <int N, int TL, int R, int P, bool INV, bool PADDED, bool WAVE, bool IN_REG, bool OUT_REG,
          int E>
__device__ __forceinline__ void fft_stage_e(float2 (&e)[E], float2* line, const float2* tw,
                                            int lt) {
  constexpr int NB = N / R;
  constexpr int IT = NB / TL;
  static_assert(NB % TL == 0 && E == N / TL, "even stages");
  constexpr bool RLIN = !PADDED || NB % 32 == 0 || 32 % NB == 0;
  constexpr bool WLIN = !PADDED || P % 32 == 0 ||
                        (32 % P == 0 && (32 % (P * R) == 0 || (P * R) % 32 == 0));
  float2 v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int i = lt + it * TL;
    if constexpr (IN_REG) {
#pragma unroll
      for (int j = 0; j < R; ++j) v[it][j] = e[it + j * IT];
    } else if constexpr (RLIN) {
      const int rb = fidx<PADDED>(i);
#pragma unroll
      for (int j = 0; j < R; ++j) v[it][j] = line[rb + pstep<PADDED>(j * NB)];
    } else {
#pragma unroll
      for (int j = 0; j < R; ++j) v[it][j] = line[fidx<PADDED>(i + j * NB)];
    }
  }
  // every thread's reads of the line (this stage's, or the previous
  // transform's last stage) are done before it is overwritten
  if constexpr (!OUT_REG) fft_sync<WAVE>();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int i = lt + it * TL;
    const int k = i % P;
    if (P > 1) {
#pragma unroll
      for (int j = 1; j < R; ++j) {
        float2 w = tw[fpi(j * k * (N / (P * R)))];
        if (INV) w.y = -w.y;
        v[it][j] = cmul(v[it][j], w);
      }
    }
    Dft<R, INV>::run(v[it]);
    if constexpr (OUT_REG) {
#pragma unroll
      for (int j = 0; j < R; ++j) e[it + j * IT] = v[it][j];
    } else {
      const int base = (i - k) * R + k;
      if constexpr (WLIN) {
        const int wb = fidx<PADDED>(base);
#pragma unroll
        for (int j = 0; j < R; ++j) line[wb + pstep<PADDED>(j * P)] = v[it][j];
      } else {
#pragma unroll
        for (int j = 0; j < R; ++j) line[fidx<PADDED>(base + j * P)] = v[it][j];
      }
    }
  }
  if constexpr (!OUT_REG) fft_sync<WAVE>();
}

template <int N, int TL, bool INV, bool PADDED, bool WAVE, int S, int E>
__device__ __forceinline__ void fft_stages_e(float2 (&e)[E], float2* line, const float2* tw,
                                             int lt) {
  constexpr int NS = fft_nstages_tl(N, TL);
  if constexpr (S < NS) {
    fft_stage_e<N, TL, fft_radix_tl(N, TL, S), fft_pstride_tl(N, TL, S), INV, PADDED, WAVE, S == 0,
                S == NS - 1>(e, line, tw, lt);
    fft_stages_e<N, TL, INV, PADDED, WAVE, S + 1>(e, line, tw, lt);
  }
}

template <int N, int TL, bool INV, bool PADDED, bool WAVE, int S>
__device__ __forceinline__ void fft_stages(float2* line, const float2* tw, int lt) {
  if constexpr (S < fft_nstages_tl(N, TL)) {
    fft_stage<N, TL, fft_radix_tl(N, TL, S), fft_pstride_tl(N, TL, S), INV, PADDED, WAVE>(line, tw,
                                                                                         lt);
    fft_stages<N, TL, INV, PADDED, WAVE, S + 1>(line, tw, lt);
  }
}

// Unnormalised DFT of `line` (forward: exp(-2 pi i jk/N); INV: exp(+...)).
// All threads of the workgroup must call it (it synchronises); the line must
// be fully written before the call.  PADDED: the line is stored padded
// (element n at fpi(n), fft_line_len(N) elements), otherwise plain.  `tw`
// holds the N twiddles.  WAVE (each line owned by one wavefront, TL <= 64):
// the transform synchronises only within the wavefront, so LDS data written
// by other wavefronts (the twiddles, a tile loaded across lines) must be
// behind a workgroup barrier before the call.
template <int N, int TL, bool INV, bool PADDED = false, bool WAVE = false>
__device__ __forceinline__ void fft(float2* line, const float2* tw, int lt) {
  static_assert(!WAVE || (TL <= 64 && 64 % TL == 0), "wavefront-owned lines");
  fft_sync<WAVE>();
  fft_stages<N, TL, INV, PADDED, WAVE, 0>(line, tw, lt);
}

// Unnormalised DFT of the line whose elements x[lt + m TL] thread lt holds in
// e[m]; on return e[m] holds X[lt + m TL].  `line` (fft_line_len(N) elements
// if PADDED) is the exchange buffer of the line: its contents are
// overwritten, and every thread of the line must call.  The twiddles obey
// the rules of fft(); no other ordering is needed around the call: the
// transform neither reads the line before writing it nor leaves anything
// in it that the caller reads.  Plans whose stages are not even (lengths
// 3 * 2^a for some thread counts) go through the line-based transform.
template <int N, int TL, bool INV, bool PADDED = true, bool WAVE = false>
__device__ __forceinline__ void fft_e(float2 (&e)[N / TL], float2* line, const float2* tw,
                                      int lt) {
  static_assert(!WAVE || (TL <= 64 && 64 % TL == 0), "wavefront-owned lines");
  static_assert(N % TL == 0, "whole elements per thread");
  if constexpr (fft_even_stages<N, TL>()) {
    fft_stages_e<N, TL, INV, PADDED, WAVE, 0>(e, line, tw, lt);
  } else {
    fft_sync<WAVE>();
#pragma unroll
    for (int m = 0; m < N / TL; ++m) line[fidx<PADDED>(lt + m * TL)] = e[m];
    fft<N, TL, INV, PADDED, WAVE>(line, tw, lt);
#pragma unroll
    for (int m = 0; m < N / TL; ++m) e[m] = line[fidx<PADDED>(lt + m * TL)];
  }
}

}  // namespace holo
