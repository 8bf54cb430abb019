// Internal interface of the batched single-angle retrievals (holo2d.hip and
// holo2d_api.cpp).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace holo {

// Transpose of the bilinear demagnification along one axis: the two source
// indices that give destination index idx a weight, and those weights
// (unused entries have index 0 and weight 0).
struct B2AdjTap {
  int d0, d1;
  float w0, w1;
};

struct B2Inst {
  int n;                   // square edge
  long long off;           // element offset of the instance's frame
  const float2* tw;        // [n] twiddles
  const float2* chirp;     // [2 nd + 1][n] transfer rows (det_j, probe_j, ref), times 1/n
  const B2AdjTap* adj;     // [nd][n] transposed demagnification taps of an axis
};

struct B2Item {
  int inst, job, line0, slot;
};

// Passes of the batched gradient (one launch each):
//   kB2RowsProbe  rows of D_{rho_probe_j} q (jobs < nd) and of D_1 q (job nd)
//   kB2ColsProbe  their columns; job nd: reference residual and cost, then
//                 (want_gq) the columns of D_{-1} on it
//   kB2RowsA      pass A rows;  kB2ColsB  pass B columns
//   kB2RowsC      pass C rows (no probe gradient)
//   kB2RowsCGq    pass C rows, then the rows of D_{-rho_probe_j} on G_j;
//                 job nd: the rows of D_{-1} on the reference residual
//   kB2ColsGqSum  per column tile: the columns of D_{-rho_probe_j} on every
//                 G_j summed in the frequency domain, one inverse transform,
//                 plus the reference term -> g_q
enum B2Mode {
  kB2RowsProbe = 0, kB2RowsA, kB2RowsC, kB2RowsCGq,
  kB2ColsProbe, kB2ColsB, kB2ColsGqSum
};

struct B2Args {
  int mode, nd, want_grad, want_ref;
  int want_gq;             // the probe gradient is wanted (and the reference term with it)
  int functional;          // 0: amplitude (F2), 1: intensity (F1)
  int max_n;               // largest instance size of the batch
  double mag[8];
  const B2Inst* inst;
  const float2* psi;
  const float2* q;
  const float* amp;        // nullptr: forward fields only
  const float* amp_ref;
  float2* Q;               // [inst][nd] frames
  float2* P;               // [inst] reference field / residual / gradient
  float2* X;               // [inst][nd] frames (output v in forward mode)
  float2* G;               // [inst][nd] frames
  float2* g_psi;
  float2* g_q;
  double* Fpart;
};

int b2_rows_per_wg(int n);
int b2_cols_per_wg(int n);
int b2_gq_per_wg(int n);
bool b2_size_supported(int n);

hipError_t launch_b2_rows(const B2Args& A, const B2Item* items, int n, hipStream_t st);
hipError_t launch_b2_cols(const B2Args& A, const B2Item* items, int n, hipStream_t st);
hipError_t launch_b2_gq_sum(const B2Args& A, const B2Item* items, int n, hipStream_t st);
hipError_t launch_b2_gather(const B2Args& A, const B2Item* items, int n, hipStream_t st);
hipError_t launch_b2_reduce(const double* parts, const int2* ranges, int n_inst, double* F,
                            hipStream_t st);

}  // namespace holo
