// Internal interface of the batched single-angle retrievals (holo2d.hip and
// holo2d_api.cpp).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace holo {

struct B2Inst {
  int n;                   // square edge
  long long off;           // element offset of the instance's frame
  const float2* tw;        // [n] twiddles
  const float2* chirp;     // [2 nd + 1][n] transfer rows (det_j, probe_j, ref), times 1/n
};

struct B2Item {
  int inst, job, line0, slot;
};

enum B2Mode {
  kB2RowsProbe = 0, kB2RowsRef, kB2RowsA, kB2RowsC, kB2RowsGq,
  kB2ColsProbe, kB2ColsRef, kB2ColsB, kB2ColsGq
};

struct B2Args {
  int mode, nd, want_grad, want_ref;
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
bool b2_size_supported(int n);

hipError_t launch_b2_rows(const B2Args& A, const B2Item* items, int n, hipStream_t st);
hipError_t launch_b2_cols(const B2Args& A, const B2Item* items, int n, hipStream_t st);
hipError_t launch_b2_gather(const B2Args& A, const B2Item* items, int n, hipStream_t st);
hipError_t launch_b2_reduce(const double* parts, const int2* ranges, int n_inst, double* F,
                            hipStream_t st);

}  // namespace holo
