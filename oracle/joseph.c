/*
 * joseph.c -- the oracle's Joseph ray sums and their literal transpose in
 * plain C, double precision.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by oracle/holo_oracle.py for problems too
 * large for its NumPy loops (the 256^3 x 360-angle, 1024^3 and 2048^2 x 512
 * checks).  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may reach it.  It shares no code, header or table with the HIP library.
 *
 * Definition (Sec. 2, Eq. 14: R_k is the Radon transform at angle theta_k;
 * its discretisation is the Joseph reading): for slice z, bin i and
 * s = i - W/2, with C = cos(theta), S = sin(theta), c = W/2,
 *   |C| >= |S|:  p = (1/|C|) sum_{y < W} lerp_x(u[z][y][:], c + (s - (y - c) S) / C)
 *   otherwise:   p = (1/|S|) sum_{x < W} lerp_y(u[z][:][x], c + (s - (x - c) C) / S)
 * where lerp at f takes (1 - w) g[floor f] + w g[floor f + 1], w = f - floor f,
 * and drops taps outside [0, W).  The transpose scatters every ray sum back
 * with the same weights.  These are the loops of `radon` and `radon_T` in
 * holo_oracle.py; the only liberty taken is the loop order (blocks of slices
 * in parallel, the taps of one step computed once for the slices of a
 * block), which changes nothing but the order of the double-precision sums.
 *
 * Layouts: complex values are interleaved (re, im).
 *   u   float  [H][W][W][2]   complex64 volume, widened to double on read
 *   p   double [n][nz][W][2]  ray sums of slices z0 .. z0 + nz - 1
 *   h   double [n][nz][W][2]  sinogram of nz slices (transpose input)
 *   g   double [nz][W][W][2]  transpose output for those slices
 * Return value: 0 on success, 1 for bad sizes, 2 if a thread's scratch
 * allocation failed.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { kSlab = 4 };   /* slices per work item */

/* Taps of one walk step for every bin: i0[i], w[i] and the path factor;
 * returns the axis (0: taps index x in row `step`; 1: taps index y in
 * column `step`). */
static int taps(int W, double theta, int step, long *i0, double *w, double *scale) {
  const double c = W / 2.0, C = cos(theta), S = sin(theta);
  const int along_y = fabs(C) >= fabs(S);
  for (int i = 0; i < W; ++i) {
    const double s = (double)i - c;
    const double f = along_y ? c + (s - ((double)step - c) * S) / C
                             : c + (s - ((double)step - c) * C) / S;
    const double fl = floor(f);
    i0[i] = (long)fl;
    w[i] = f - fl;
  }
  *scale = 1.0 / (along_y ? fabs(C) : fabs(S));
  return along_y ? 0 : 1;
}

int joseph_radon(const float *u, int H, int W, const double *theta, int n, int z0, int nz,
                 double *p) {
  if (H < 1 || W < 1 || n < 1 || z0 < 0 || nz < 1 || z0 + nz > H) return 1;
  int bad = 0;
  const int nblk = (nz + kSlab - 1) / kSlab;
#pragma omp parallel
  {
    long *i0 = (long *)malloc(sizeof(long) * W);
    double *w = (double *)malloc(sizeof(double) * W);
    if (!i0 || !w) {
#pragma omp atomic write
      bad = 1;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int b = 0; b < nblk; ++b) {
        const int za = b * kSlab, zb = za + kSlab < nz ? za + kSlab : nz;
        for (int k = 0; k < n; ++k) {
          for (int zz = za; zz < zb; ++zz)
            memset(p + ((size_t)k * nz + zz) * W * 2, 0, sizeof(double) * 2 * W);
          for (int step = 0; step < W; ++step) {
            double scale;
            const int axis = taps(W, theta[k], step, i0, w, &scale);
            for (int zz = za; zz < zb; ++zz) {
              const float *us = u + (size_t)(z0 + zz) * W * W * 2;
              double *pk = p + ((size_t)k * nz + zz) * W * 2;
              for (int i = 0; i < W; ++i) {
                for (int t = 0; t < 2; ++t) {
                  const long idx = i0[i] + t;
                  if (idx < 0 || idx >= W) continue;
                  const double wt = (t == 0 ? 1.0 - w[i] : w[i]) * scale;
                  const float *gv = axis == 0 ? us + 2 * ((size_t)step * W + idx)
                                              : us + 2 * ((size_t)idx * W + step);
                  pk[2 * i] += wt * (double)gv[0];
                  pk[2 * i + 1] += wt * (double)gv[1];
                }
              }
            }
          }
        }
      }
    }
    free(i0);
    free(w);
  }
  return bad ? 2 : 0;
}

int joseph_radon_T(const double *h, int W, const double *theta, int n, int nz, double *g) {
  if (W < 1 || n < 1 || nz < 1) return 1;
  int bad = 0;
  const int nblk = (nz + kSlab - 1) / kSlab;
#pragma omp parallel
  {
    long *i0 = (long *)malloc(sizeof(long) * W);
    double *w = (double *)malloc(sizeof(double) * W);
    if (!i0 || !w) {
#pragma omp atomic write
      bad = 1;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int b = 0; b < nblk; ++b) {
        const int za = b * kSlab, zb = za + kSlab < nz ? za + kSlab : nz;
        memset(g + (size_t)za * W * W * 2, 0, sizeof(double) * 2 * (size_t)W * W * (zb - za));
        for (int k = 0; k < n; ++k) {
          for (int step = 0; step < W; ++step) {
            double scale;
            const int axis = taps(W, theta[k], step, i0, w, &scale);
            for (int zz = za; zz < zb; ++zz) {
              const double *hk = h + ((size_t)k * nz + zz) * W * 2;
              double *gs = g + (size_t)zz * W * W * 2;
              for (int i = 0; i < W; ++i) {
                for (int t = 0; t < 2; ++t) {
                  const long idx = i0[i] + t;
                  if (idx < 0 || idx >= W) continue;
                  const double wt = (t == 0 ? 1.0 - w[i] : w[i]) * scale;
                  double *o = axis == 0 ? gs + 2 * ((size_t)step * W + idx)
                                        : gs + 2 * ((size_t)idx * W + step);
                  o[0] += wt * hk[2 * i];
                  o[1] += wt * hk[2 * i + 1];
                }
              }
            }
          }
        }
      }
    }
    free(i0);
    free(w);
  }
  return bad ? 2 : 0;
}
