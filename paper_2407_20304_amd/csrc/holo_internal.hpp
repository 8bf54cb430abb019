// Internal interface between the host runtime (holo_api.cpp) and the HIP
// kernels (holo_kernels.hip, holo_radon.hip, holo_fs.hip).  Not part of the
// public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace holo {

constexpr int kThreads = 256;   // threads per workgroup of the 1-D kernels
constexpr int kMaxDist = 8;
// Per-angle constants (double): see AngleCols.
constexpr int kAngleStride = 8;
enum AngleCols {
  kCos = 0,     // cos(theta)
  kSin = 1,     // sin(theta)
  kInvH = 2,    // 1 / max(|cos|, |sin|)  (footprint half-width h = max(...))
  kBranch = 3,  // 0: walk along y, taps along x;  1: walk along x, taps along y
  kA = 4,       // tap position f = A + bin * B + step * D (fractional index)
  kB = 5,
  kD = 6,
  kScale = 7    // path length per step, 1 / max(|cos|, |sin|)
};
// Class of an angle in the transpose: its direction, taken as theta - pi
// (-cos, -sin) when cos < 0 (the rows the transpose reads reversed), has
// sin >= 0 (class 0) or sin < 0 (class 1).
inline int adj_class(const double* a) {
  const double s = a[kCos] < 0.0 ? -a[kSin] : a[kSin];
  return s < 0.0 ? 1 : 0;
}

// Geometry and device tables as the kernels see them.
struct DevGeom {
  int H, W, nd;
  int n_angles;              // angles of the plan (shift table stride)
  double cH, cW;             // grid centres H/2, W/2
  double mag[kMaxDist];      // m~_j
  float kappa;
  const float2* twW;         // [W]  exp(-2 pi i m / W)
  const float2* twH;         // [H]
  const float2* chirpW;      // [3 nd + 1][W] transfer factors, times 1/W
  const float2* chirpH;      // [3 nd + 1][H] transfer factors, times 1/H
  const float* shift;        // [n_angles][nd][2] (t_y, t_x) or nullptr
  int functional;            // residual: 0 amplitude (F2 and the conventional
                             // functional), 1 intensity (F1)
  const float* pshift;       // [n_angles][nd][2] (s_y, s_x) probe shifts or nullptr
  // padded propagation (lines set in the centre of lines twice as long):
  // twiddles and transfer rows of lengths 2W and 2H, or nullptr
  const float2* tw2W;        // [2W]
  const float2* tw2H;        // [2H]
  const float2* chirp2W;     // [2 nd + 1][2W], times 1/(2W)
  const float2* chirp2H;     // [2 nd + 1][2H], times 1/(2H)
  int col_tile;              // columns per pass-B workgroup (0: the default)
  // Joseph plans store the sinogram rows of angles with cos < 0 with the
  // bin axis reversed (as the angle theta - pi): pass D writes them so and
  // the transpose reads them so, which makes cos >= 0 for every angle it sees
  const double* ang;         // [n_angles][kAngleStride] plan angle table
  int sino_mirror;
};

// Fourier-slice projector (holo_fs.hip): gridding kernel taps per axis,
// slices per slab, and the bins of the transpose's angle-window table.
constexpr int kFsWidth = 8;
constexpr int kFsSlab = 8;
constexpr int kFsBins = 4096;
struct FsArgs {
  int K, k0;                 // the call's angles: plan angles k0 .. k0 + K - 1
  int n_angles;              // plan angles
  float beta;                // kernel shape exp(beta (sqrt(1 - (2x/KW)^2) - 1))
  const float* dinv;         // [W] 1 / (Fourier transform of the kernel) at x - W/2
  const double* ang;         // plan angle table (kAngleStride doubles per angle)
  const int* sorted_k;       // [n_angles] plan angles sorted by theta mod pi
  const int* bin_first;      // [kFsBins + 1] first sorted position at or past bin b
};

// One padded propagation over a set of frames (H x W each): frame f reads
// src + f * src_step and writes dst + f * H * W; its transfer row is
// chirp0 + f % cmod (conjugated when conj).  Rows apply the transfer only.
// Columns: mode 0 the transfer only; mode 1 the transfer, the residual
// against amp + f * H * W (cost into Fpart[fslot0 + f * ntiles + tile]) and
// then the conjugate transfer; mode 2 the transfer and the residual's cost
// only (nothing written).
struct PadJob {
  const float2* src;
  float2* dst;
  const float* amp;
  long long src_step;
  int nframes, chirp0, cmod, conj, mode, fslot0;
};

// Transfer-function table rows: detector step of plane j, probe step of
// plane j, and the reference step rho = 1.
__host__ __device__ inline int chirp_det(int j) { return j; }
__host__ __device__ inline int chirp_probe(int nd, int j) { return nd + j; }
__host__ __device__ inline int chirp_ref(int nd) { return 2 * nd; }
__host__ __device__ inline int chirp_rows(int nd) { return 2 * nd + 1; }

// One propagation job of the probe-side kernels (rows or columns).
struct PropJob {
  const float2* src;
  float2* dst;
  const float* amp;          // non-null: replace the field by the residual
  int chirp;                 // table row
  int conj;                  // 1: use the conjugate transfer (D_{-rho})
  int fslot;                 // index into Fpart for the residual's cost
};
constexpr int kMaxJobs = 12;
struct PropJobs {
  PropJob job[kMaxJobs];
  int n;
};

enum ColMode { kColFwd = 0, kColObj = 1, kColGrad = 2, kColAdj = 3 };

// Launch geometry helpers shared by host and device.
int rows_per_wg(int W);      // lines of W handled by one 256-thread workgroup
int cols_per_wg(int H);      // columns of length H per workgroup
bool fft_size_supported(int n);
// Pass B's column tile: cols_per_wg(H) (the default) or half of it.
bool col_tile_supported(int H, int tc);
// Ray-sum tiling (see the kernels): forward angle-group size, slices and
// bins per workgroup, staged rows per block and staged columns per row;
// transpose slices per thread, angles per staged group and bins per staged
// segment; slice blocking of the forward's volume copies.
constexpr int kFwdNA = 4, kFwdZT = 64, kFwdNB = 16, kFwdYB = 2, kFwdSeg = 32;
constexpr int kAdjZT = 16, kAdjNA = 4, kAdjSeg = 32;
constexpr int kAdjWin = 64;   // angles per transpose set-up window
constexpr int kVolZB = 16;
// Zero bins on each side of every row of the sinogram read by the transpose,
// stored S[k][z][kAdjPad + bin]: a staged segment is then always valid
// memory (segments wholly off the detector are moved into the padding,
// which reads as zeros).
constexpr int kAdjPad = kAdjSeg;
inline __host__ __device__ int sino_row(int W) { return W + 2 * kAdjPad; }
// Zero columns on each side of every row of the forward's volume copies: a
// staged row window is then always valid memory (windows wholly outside the
// volume are moved into the padding, which reads as zeros).
constexpr int kFwdPad = kFwdSeg;
inline __host__ __device__ int vol_row(int W) { return W + 2 * kFwdPad; }
// Largest detector edge (the forward kernel keeps one window start per row).
constexpr int kMaxW = 2048;

// Launchers (all asynchronous on `st`; return hipSuccess or the launch error).
hipError_t launch_rows_prop(const DevGeom& g, const PropJobs& jobs, hipStream_t st);
hipError_t launch_cols_prop(const DevGeom& g, const PropJobs& jobs, double* Fpart, hipStream_t st);
hipError_t launch_pass_a(const DevGeom& g, const float2* psi, const float2* Q, float2* X,
                         int k_first, int Kc, hipStream_t st);
// Padded propagation (row and column halves) and the elementwise parts of
// passes A and C that surround it when the plan propagates padded.
bool pad_size_supported(int n);
int pad_col_tiles(int H, int W);  // column tiles per frame of the padded column pass
hipError_t launch_rows_pad(const DevGeom& g, const PadJob& jb, hipStream_t st);
hipError_t launch_cols_pad(const DevGeom& g, const PadJob& jb, double* Fpart, hipStream_t st);
// Fourier-slice forward of slices z0 .. z0 + nz - 1 (nz <= kFsSlab): psi of
// every angle of the call into S[k][z][kAdjPad + s]; and its transpose from
// h in S into g_u of those slices.  G: kFsSlab grids of (2W)^2; A:
// kFsSlab * K * (W + 2) polar samples.
bool fs_size_supported(int W);
hipError_t launch_fs_forward_slab(const DevGeom& g, const FsArgs& f, const float2* u_slab,
                                  float2* G, float2* S, int z0, int nz, hipStream_t st);
hipError_t launch_fs_adjoint_slab(const DevGeom& g, const FsArgs& f, const float2* S,
                                  float2* A, float2* G, float2* gu_slab, int z0, int nz,
                                  hipStream_t st);
hipError_t launch_copy_rows(const float2* src, size_t src_pitch, float2* dst, size_t rows,
                            int W, hipStream_t st);
hipError_t launch_frames_x(const DevGeom& g, const float2* psi, const float2* Q, float2* X,
                           int k_first, int Kc, hipStream_t st);
hipError_t launch_frames_c(const DevGeom& g, float2* X, const float2* psi, const float2* Q,
                           float2* G, float2* Pbuf, int accumulate, int k_first, int Kc,
                           hipStream_t st);
hipError_t launch_pass_b(const DevGeom& g, int mode, const float2* src, float2* X,
                         const float* amp, double* Fpart, int Kc, hipStream_t st);
hipError_t launch_pass_c(const DevGeom& g, float2* X, const float2* psi, const float2* Q,
                         float2* G, float2* Pbuf, int accumulate, int k_first, int Kc,
                         hipStream_t st);
// G_j += sum_k S_{-s_kj}(Pbuf[k][j]) for the Kc angles of a chunk (probe shifts).
hipError_t launch_probe_shift_acc(const DevGeom& g, float2* G, const float2* Pbuf, int k_first,
                                  int Kc, hipStream_t st);
hipError_t launch_pass_d(const DevGeom& g, const float2* X, const float2* psi, float2* S,
                         int k_first, int Kc, hipStream_t st);
hipError_t launch_radon_fwd(const DevGeom& g, const float2* ub, const float2* uTb, float2* psi,
                            const double* ang, const int2* groups, int g0, int ngroups, int c0,
                            int c1, int nb, hipStream_t st);
// Transpose of the ray sums over angles k0 + [0, n0 + n1): S holds their rows
// (row k - k0), ang the plan's whole angle table; ord0 / ord1 list the angles
// of class 0 / 1 (sin >= 0 / < 0 once rows with cos < 0 are reversed) in
// ascending order.
hipError_t launch_radon_adj(const DevGeom& g, const float2* S, float2* gu, const double* ang,
                            int k0, const int* ord0, int n0, const int* ord1, int n1,
                            hipStream_t st);
hipError_t launch_block_volume(const DevGeom& g, const float2* u, float2* ub, float2* uTb,
                               hipStream_t st);
hipError_t launch_fill_zero(float2* p, size_t n, hipStream_t st);
hipError_t launch_fill(float2* p, size_t n, float2 value, hipStream_t st);
hipError_t launch_sum_frames(const float2* G, int nd, const float2* extra, float2* out,
                             size_t n, hipStream_t st);
// Deterministic two-stage sum of n doubles; `scratch` holds kReduceParts.
constexpr int kReduceParts = 256;
hipError_t launch_reduce_sum(const double* parts, size_t n, double* scratch, double* out,
                             hipStream_t st);
// Solver vector operations.  launch_dot_re: *out = Re <a1, b1> + Re <a2, b2>
// in double, deterministic; `parts` holds kDotParts, `scratch` kReduceParts.
constexpr int kDotParts = 1024;
hipError_t launch_dot_re(const float2* a1, const float2* b1, size_t n1, const float2* a2,
                         const float2* b2, size_t n2, double* parts, double* scratch, double* out,
                         hipStream_t st);
hipError_t launch_axpy(const float2* x, const float2* e, float t, float2* out, size_t n,
                       hipStream_t st);
hipError_t launch_cg_dir(const float2* g, float2* eta, float beta, int restart, size_t n,
                         hipStream_t st);
hipError_t launch_real_to_c64(const float* a, float2* out, size_t n, hipStream_t st);

// The dispatcher hands workgroup h of a 1-D grid to XCD h mod 8.  Remap so
// that each XCD walks a contiguous range of logical indices: neighbours in
// logical order then share that XCD's L2.
__device__ __forceinline__ int xcd_logical(int h, int n) {
  const int q = n >> 3, r = n & 7;
  const int x = h & 7, loc = h >> 3;
  return x * q + min(x, r) + loc;
}

}  // namespace holo
