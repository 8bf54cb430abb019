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
 * in parallel, the taps of one angle tabled once for the slices of a block,
 * the walk along x summed ray by ray), which changes nothing but the order
 * of the double-precision sums.
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
#include <omp.h>
#include <stdlib.h>
#include <string.h>

enum { kSlab = 16 };   /* at most this many slices per work item */

/* Slices per work item: up to kSlab, fewer when there are too few slices
 * to keep every thread busy. */
static int slab_of(int nz) {
  int s = nz / omp_get_max_threads();
  return s < 1 ? 1 : (s > kSlab ? kSlab : s);
}

/* Taps of every (step, bin) of one angle: for the walk along y (|C| >= |S|,
 * axis 0) entry [step][i], otherwise [i][step], so that the loops below run
 * through memory in order.  i0 = floor f, w = f - floor f; returns the axis
 * and the path factor 1/max(|C|, |S|). */
static int tap_table(int W, double theta, int *i0, double *w, double *scale) {
  const double c = W / 2.0, C = cos(theta), S = sin(theta);
  const int along_y = fabs(C) >= fabs(S);
  for (int step = 0; step < W; ++step) {
    for (int i = 0; i < W; ++i) {
      const double s = (double)i - c;
      const double f = along_y ? c + (s - ((double)step - c) * S) / C
                               : c + (s - ((double)step - c) * C) / S;
      const double fl = floor(f);
      const size_t e = along_y ? (size_t)step * W + i : (size_t)i * W + step;
      i0[e] = (int)fl;
      w[e] = f - fl;
    }
  }
  *scale = 1.0 / (along_y ? fabs(C) : fabs(S));
  return along_y ? 0 : 1;
}

int joseph_radon(const float *u, int H, int W, const double *theta, int n, int z0, int nz,
                 double *p) {
  if (H < 1 || W < 1 || n < 1 || z0 < 0 || nz < 1 || z0 + nz > H) return 1;
  int bad = 0;
  const int slab = slab_of(nz);
  const int nblk = (nz + slab - 1) / slab;
  const size_t WW = (size_t)W * W;
#pragma omp parallel
  {
    int *i0 = (int *)malloc(sizeof(int) * WW);
    double *w = (double *)malloc(sizeof(double) * WW);
    if (!i0 || !w) {
#pragma omp atomic write
      bad = 1;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int b = 0; b < nblk * n; ++b) {
        const int k = b / nblk;
        const int za = (b % nblk) * slab, zb = za + slab < nz ? za + slab : nz;
        double scale;
        const int axis = tap_table(W, theta[k], i0, w, &scale);
        for (int zz = za; zz < zb; ++zz) {
          const float *us = u + (size_t)(z0 + zz) * WW * 2;
          double *pk = p + ((size_t)k * nz + zz) * W * 2;
          memset(pk, 0, sizeof(double) * 2 * W);
          if (axis == 0) {            /* taps along x in row `step` */
            for (int step = 0; step < W; ++step) {
              const float *row = us + (size_t)step * W * 2;
              for (int i = 0; i < W; ++i) {
                const size_t e = (size_t)step * W + i;
                for (int t = 0; t < 2; ++t) {
                  const long idx = (long)i0[e] + t;
                  if (idx < 0 || idx >= W) continue;
                  const double wt = (t == 0 ? 1.0 - w[e] : w[e]) * scale;
                  pk[2 * i] += wt * (double)row[2 * idx];
                  pk[2 * i + 1] += wt * (double)row[2 * idx + 1];
                }
              }
            }
          } else {                    /* taps along y in column `step` */
            for (int i = 0; i < W; ++i) {
              double re = 0.0, im = 0.0;
              for (int step = 0; step < W; ++step) {
                const size_t e = (size_t)i * W + step;
                for (int t = 0; t < 2; ++t) {
                  const long idx = (long)i0[e] + t;
                  if (idx < 0 || idx >= W) continue;
                  const double wt = (t == 0 ? 1.0 - w[e] : w[e]) * scale;
                  const float *gv = us + 2 * ((size_t)idx * W + step);
                  re += wt * (double)gv[0];
                  im += wt * (double)gv[1];
                }
              }
              pk[2 * i] = re;
              pk[2 * i + 1] = im;
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
  const int slab = slab_of(nz);
  const int nblk = (nz + slab - 1) / slab;
  const size_t WW = (size_t)W * W;
#pragma omp parallel
  {
    int *i0 = (int *)malloc(sizeof(int) * WW);
    double *w = (double *)malloc(sizeof(double) * WW);
    if (!i0 || !w) {
#pragma omp atomic write
      bad = 1;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int b = 0; b < nblk; ++b) {
        const int za = b * slab, zb = za + slab < nz ? za + slab : nz;
        memset(g + (size_t)za * WW * 2, 0, sizeof(double) * 2 * WW * (zb - za));
        for (int k = 0; k < n; ++k) {
          double scale;
          const int axis = tap_table(W, theta[k], i0, w, &scale);
          for (int zz = za; zz < zb; ++zz) {
            const double *hk = h + ((size_t)k * nz + zz) * W * 2;
            double *gs = g + (size_t)zz * WW * 2;
            for (int a = 0; a < W; ++a) {      /* axis 0: a = step; axis 1: a = bin */
              for (int bb = 0; bb < W; ++bb) { /* axis 0: bb = bin; axis 1: bb = step */
                const size_t e = (size_t)a * W + bb;
                const int i = axis == 0 ? bb : a, step = axis == 0 ? a : bb;
                for (int t = 0; t < 2; ++t) {
                  const long idx = (long)i0[e] + t;
                  if (idx < 0 || idx >= W) continue;
                  const double wt = (t == 0 ? 1.0 - w[e] : w[e]) * scale;
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
