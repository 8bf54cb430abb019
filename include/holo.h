/*
 * holo.h -- C ABI of the MI355X holotomography gradient library (libholo.so).
 *
 * The library evaluates the joint object-and-probe holotomography objective
 * and its gradients on one AMD Instinct MI355X (gfx950):
 *
 *   psi_k  = exp(i kappa R_k u)                     joint model, Sec. 5 Eq. (17)
 *   phi_kj = M_{1/m~_j} S_{t_kj}(psi_k)             demagnify + shift, Sec. 2 Eq. (8)-(9)
 *   Q_j    = D_{rho_probe_j}(q)                     probe at plane j, Eq. (8)
 *   v_kj   = D_{rho_det_j}(Q_j . phi_kj)            detector field, Eq. (8) / Thm A.3
 *   F(u,q) = sum_kj || |v_kj| - a_kj ||^2
 *          + || |D_1 q| - a_ref ||^2                amplitude functional F2, Eq. (10)
 *
 * and the gradients of Eq. (11) and the display after it, extended to u by the
 * chain rule through exp and R.  Everything is dimensionless: lengths are
 * detector pixels after the data rescaling d~ = m0^2 M_{1/m0} d (Eq. 9 text),
 * distances are multiples of zeta_0 = z_0 (Z - z_0) / Z, and
 *   rho_det_j   = zeta_j / (m~_j^2 zeta_0) = (m0 - m~_j) / (m~_j (m0 - 1)),
 *   rho_probe_j = omega_j / zeta_0         = m0 (m~_j - 1) / (m~_j (m0 - 1)),
 * with m~_j = z_j / z_0 and m0 = Z / z_0 (Thm A.3).  D_rho is the Fresnel
 * transfer function exp(-i pi rho (kx^2/W^2 + ky^2/H^2) / N_F0) applied by FFT
 * on the unpadded periodic H x W grid (Appendix A, kernel P_Z); it is unitary
 * and D_rho^H = D_{-rho}.
 *
 * Discretisations (the paper names the operators but not their grids):
 *   R_k  Joseph ray sums: unit steps along the dominant axis of the ray,
 *        linear interpolation across it, path factor 1/max(|cos|,|sin|).
 *        Voxel (ix, iy) sits at (ix - W/2, iy - W/2); bin i sits at
 *        s = i - W/2 with s = x cos(theta) + y sin(theta).
 *   M S  bilinear sampling at src = c + m~ (x - c) - t (c = n/2 per axis);
 *        outside the psi grid the transmission is 1 (free space).
 *   |v|=0  the residual uses v/|v| := 0.
 *
 * Gradient convention: g = dF/dRe + i dF/dIm (the paper's 2 L*(...)); this is
 * also PyTorch's convention for the gradient of a real loss.
 *
 * Memory layouts (all device pointers, row-major, complex = interleaved
 * float re/im, i.e. the layout of torch.complex64):
 *   u, g_u    [H][W][W]                      u[z][y][x], z = detector row
 *   q, g_q    [H][W]
 *   amp       [n_angles][n_dist][H][W] float  a_kj = sqrt(d~_kj)
 *   amp_ref   [H][W] float                    a_ref = sqrt(d~r)
 *   v, w      [k1-k0][n_dist][H][W]           detector-plane frames
 *
 * Sizes: H and W must each be one of 64, 128, 192, 256, 384, 512, 1024,
 * 2048 (FFT lengths 2^a and 3*2^a handled in LDS), and 1 <= n_dist <= 8.
 *
 * Ownership and execution: every device buffer, including the workspace, is
 * owned by the caller.  A call validates its arguments on the host, returns a
 * non-OK status before enqueueing anything if they are wrong, and otherwise
 * enqueues kernels on `stream` (a hipStream_t; NULL = the default stream) and
 * returns without synchronising.  Outputs are overwritten, never
 * accumulated.  Scalars (F) are written to device memory as double.  The
 * plan's first compute call uploads small constant tables to the current
 * device (one hipMalloc owned by the plan, freed by holo_plan_destroy); later
 * calls on that plan must use the same device.  A plan may be used by one
 * stream at a time.  Device faults surface at the caller's synchronisation.
 */
#ifndef HOLO_H
#define HOLO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } holo_c64;

typedef enum {
  HOLO_OK = 0,
  HOLO_ERR_INVALID_ARGUMENT = 1,   /* NULL pointer, bad range, bad geometry  */
  HOLO_ERR_UNSUPPORTED_SIZE = 2,   /* H or W not a supported FFT length     */
  HOLO_ERR_WORKSPACE_TOO_SMALL = 3,
  HOLO_ERR_HIP = 4,                /* a HIP runtime call or launch failed   */
  HOLO_ERR_OUT_OF_HOST_MEMORY = 5
} holo_status;

/* Geometry of one reconstruction problem (all host memory, copied by
 * holo_plan_create; the caller may free it afterwards). */
typedef struct {
  int32_t det_rows;        /* H: detector rows = volume slices z            */
  int32_t det_cols;        /* W: detector columns = in-plane volume edge    */
  int32_t n_angles;        /* N_theta >= 1                                  */
  int32_t n_dist;          /* N_z, number of sample planes, 1..8            */
  const double* theta;     /* [n_angles] projection angles, radians         */
  const double* mag_rel;   /* [n_dist] m~_j = z_j / z_0 >= 1 (plane 0 = 1)  */
  double m0;               /* Z / z_0 > 1 (Table 1: 300)                    */
  double fresnel0;         /* N_F0 = Delta^2 / (lambda zeta_0) > 0          */
  double kappa;            /* 2 pi Delta / lambda: phase per unit u per voxel */
  const float* shift;      /* [n_angles][n_dist][2] = (t_y, t_x) sample
                              shifts in pixels (Eq. 9), or NULL for none   */
  int32_t chunk;           /* angles per chunk of the frame stages; 0 = 64  */
} holo_geom;

typedef struct holo_plan holo_plan;

/* Validate `geom` and build the host-side plan (no device work).
 * Errors: INVALID_ARGUMENT (NULL, n_angles < 1, n_dist outside 1..8,
 * m0 <= 1, fresnel0 <= 0, non-finite values, mag_rel < 1), UNSUPPORTED_SIZE. */
holo_status holo_plan_create(const holo_geom* geom, holo_plan** out);

/* Free a plan and its device tables.  NULL is accepted. */
holo_status holo_plan_destroy(holo_plan* plan);

/* Bytes of device workspace every compute call of this plan needs. */
holo_status holo_workspace_bytes(const holo_plan* plan, size_t* bytes);

/* Probe shifts s_kj of Eq. (9): Q_kj = D_{rho_probe_j}(S_{s_kj} q) with S_s
 * the shift by s = (s_y, s_x) pixels, f sampled at (y - s_y, x - s_x) with
 * linear interpolation on the periodic H x W grid (so S_s commutes with the
 * propagators and the kernels shift Q_j = D_{rho_probe_j} q directly).
 * `shifts` is host memory [n_angles][n_dist][2], copied; NULL removes the
 * shifts.  Setting shifts grows the workspace by chunk * n_dist frames
 * (query holo_workspace_bytes again).  Errors: INVALID_ARGUMENT (NULL plan,
 * non-finite shift).  Host-only; the device copy is refreshed by the next
 * compute call. */
holo_status holo_plan_set_probe_shifts(holo_plan* plan, const float* shifts);

/* Angles per chunk (the frames of one chunk are formed, back-propagated and
 * dropped before the next; the workspace grows with it).  set_chunk changes
 * the plan's workspace size (query holo_workspace_bytes again); chunks below
 * the plan's largest forward angle group (at most 4 angles) are rejected
 * with INVALID_ARGUMENT; values above n_angles are clamped.  Host-only. */
holo_status holo_plan_set_chunk(holo_plan* plan, int32_t chunk);
holo_status holo_plan_get_chunk(const holo_plan* plan, int32_t* chunk);

/* Autotuner of the chunk size: one untimed gradient, then one gradient per
 * candidate timed with HIP events on `stream` (times_ms[n_cand], may be
 * NULL); the fastest candidate becomes the plan's chunk and is returned in
 * *best_chunk.  The inputs and outputs are those of holo_grad (all
 * required); `ws` must hold the workspace of the largest candidate
 * (WORKSPACE_TOO_SMALL otherwise, before any device work).  Synchronises
 * `stream`.  The chunk is a launch-shape choice: results agree with any
 * other chunk to rounding. */
holo_status holo_plan_autotune(holo_plan* plan, const holo_c64* u, const holo_c64* q,
                               const float* amp, const float* amp_ref, double* F,
                               holo_c64* g_u, holo_c64* g_q, const int32_t* candidates,
                               int32_t n_cand, void* ws, size_t ws_bytes,
                               int32_t* best_chunk, float* times_ms, void* stream);

/* Launch-shape parameters ("tiles") that change the speed of a compute call
 * but not its results (beyond the summation grouping of the cost):
 *   CHUNK     angles per chunk (holo_plan_set_chunk);
 *   COL_TILE  columns per workgroup of the fused column pass: 0 (the
 *             default: 16 for H <= 512, 8 for H = 1024, 4 for H = 2048) or
 *             half of the default;
 *   FS_SLAB   slices per slab of the Fourier-slice projector: 1, 2, 4 or 8
 *             (default 8);
 *   FWD_BINS  bins per workgroup of the forward ray sums, 16 (default) or
 *             8 (smaller staged windows, so more angles share one;
 *             setting it regroups the angles, and it is refused if the chunk
 *             is smaller than the new largest group).
 *   OVERLAP   1: Joseph's forward ray sums of the next chunk run on a second
 *             stream of the library's, concurrently with the current chunk's
 *             frame passes (two psi buffers in the workspace; the calls still
 *             order all their work after the caller's stream's earlier work
 *             and before its later work, also under graph capture); 0
 *             (default): one stream.  The results are the same.
 * holo_plan_set_tile validates and sets one (the workspace size can change
 * with CHUNK and OVERLAP; query holo_workspace_bytes again); holo_plan_get_tile reads
 * it.  holo_plan_autotune_tile is holo_plan_autotune for any of them: one
 * untimed gradient, then one gradient per candidate value timed with HIP
 * events on `stream`; the fastest becomes the plan's value.  Errors:
 * INVALID_ARGUMENT (NULL, unknown parameter, a value outside the ones
 * above), WORKSPACE_TOO_SMALL (autotune: the largest candidate's workspace
 * does not fit).  Set and get are host-only; autotune synchronises
 * `stream`. */
typedef enum {
  HOLO_TUNE_CHUNK = 0,
  HOLO_TUNE_COL_TILE = 1,
  HOLO_TUNE_FS_SLAB = 2,
  HOLO_TUNE_FWD_BINS = 3,
  HOLO_TUNE_OVERLAP = 4
} holo_tune_param;
holo_status holo_plan_set_tile(holo_plan* plan, int32_t param, int32_t value);
holo_status holo_plan_get_tile(const holo_plan* plan, int32_t param, int32_t* value);
holo_status holo_plan_autotune_tile(holo_plan* plan, int32_t param, const holo_c64* u,
                                    const holo_c64* q, const float* amp, const float* amp_ref,
                                    double* F, holo_c64* g_u, holo_c64* g_q,
                                    const int32_t* candidates, int32_t n_cand, void* ws,
                                    size_t ws_bytes, int32_t* best, float* times_ms,
                                    void* stream);

/* The least-squares functional that holo_fwd, holo_adj, holo_objective,
 * holo_grad*, holo_cg (and the residual they form) evaluate on this plan.
 *   AMPLITUDE (default): F2 of Eq. (10),
 *     sum || |v_kj| - a_kj ||^2 + || |D_1 q| - a_ref ||^2,
 *     amp and amp_ref hold the amplitudes a = sqrt(d~).
 *   INTENSITY: F1 of Eq. (9),
 *     sum || |v_kj|^2 - d~_kj ||^2 + || |D_1 q|^2 - d~r ||^2,
 *     amp and amp_ref then hold the intensities d~ themselves; the residual
 *     is 4 (|v|^2 - d~) v.
 *   CONVENTIONAL: the flat-field functional of Eq. (16), the model with
 *     the probe replaced by 1 (Sec. 2: q = 1 gives the conventional form)
 *     and no reference term,
 *     sum || |D_{rho_det_j}(M_{1/m~_j} S_{t_kj} psi_k)| - a_kj ||^2,
 *     amp holding sqrt(d_kj / d^r) (data divided by the reference image).
 *     q and amp_ref must still be non-NULL but are not read, g_q is
 *     written as 0 (F does not depend on q), holo_fwd gives the probe-free
 *     fields and holo_cg leaves q unchanged.
 * Errors: INVALID_ARGUMENT (NULL plan, unknown value).  Host-only. */
typedef enum {
  HOLO_FUNCTIONAL_AMPLITUDE = 0,
  HOLO_FUNCTIONAL_INTENSITY = 1,
  HOLO_FUNCTIONAL_CONVENTIONAL = 2
} holo_functional;
holo_status holo_plan_set_functional(holo_plan* plan, int32_t functional);

/* Propagation on a padded grid (Appendix A: D_Z is a convolution over the
 * whole plane).  pad = 1 (default): every propagation is the transfer
 * function on the periodic H x W grid.  pad = 2: every propagation of the
 * model (probe to plane j, plane j to the detector, the reference, and
 * their adjoints, also in holo_probe_init) sets the field in the centre of
 * a 2H x 2W grid with zeros outside, applies that grid's transfer function
 * (same pixel size) and keeps the centre H x W: the fields are taken as zero
 * outside the field of view instead of periodic.  The frame stages then run
 * as separate elementwise, row and column launches (slower than the fused
 * passes of pad = 1).  The workspace size does not change.  Probe shifts
 * are not taken with pad = 2: they are applied to the propagated probe,
 * which equals shifting before the propagation only on the periodic grid.
 * Errors: INVALID_ARGUMENT (NULL plan, pad not 1 or 2, pad = 2 on a plan
 * with probe shifts, and holo_plan_set_probe_shifts on a padded plan),
 * UNSUPPORTED_SIZE (pad = 2 with det_rows or det_cols above 1024).
 * Host-only. */
holo_status holo_plan_set_padding(holo_plan* plan, int32_t pad);

/* The discretisation of the ray sums R_k (Eq. 14 names the Radon transform
 * only).
 *   JOSEPH (default): the ray-driven sums of the header above.
 *   FOURIER: the Fourier slice theorem evaluated on each slice's
 *     discrete-time Fourier transform, F(xi) = sum u[z][y][x]
 *     exp(-2 pi i xi.(x', y') / W), at xi = m (cos, sin), m = -W/2 .. W/2
 *     (the two Nyquist samples averaged), inverted by the W-point DFT at the
 *     bins s = i - W/2; equivalently p[i] = sum u D_W(s_i - (x' cos +
 *     y' sin)) with D_W(d) = sin(pi d) / (W tan(pi d / W)): line integrals
 *     of each slice's trigonometric interpolant, no path factor.  Evaluated
 *     by gridding on a twice-oversampled frequency grid (8-tap kernel,
 *     approximation error a few 1e-8 relative) with O(W^2 log W + N_theta W)
 *     work per slice instead of O(N_theta W^2).  Its transpose is the exact
 *     transpose of the same computation.  Needs det_cols <= 1024; changes
 *     the workspace (8 grids of (2W)^2 and 8 N_theta (W + 2) samples in
 *     place of the ray sums' slice-blocked volume copies; query
 *     holo_workspace_bytes again).
 * Errors: INVALID_ARGUMENT (NULL plan, unknown value), UNSUPPORTED_SIZE
 * (FOURIER with det_cols above 1024).  Host-only. */
typedef enum {
  HOLO_PROJECTOR_JOSEPH = 0,
  HOLO_PROJECTOR_FOURIER = 1
} holo_projector;
holo_status holo_plan_set_projector(holo_plan* plan, int32_t projector);

/* Forward model: v_kj for the angles k0 <= k < k1 (Eq. 8 with Eq. 17). */
holo_status holo_fwd(holo_plan* plan, const holo_c64* u, const holo_c64* q,
                     int32_t k0, int32_t k1, holo_c64* v,
                     void* ws, size_t ws_bytes, void* stream);

/* Adjoint of the linearised forward model: (g_u, g_q) = J^H w with
 * J = d v / d(u, q) over the angles k0 <= k < k1 (v is holomorphic in u and
 * q, so this is the vector-Jacobian product).  Either output may be NULL. */
holo_status holo_adj(holo_plan* plan, const holo_c64* u, const holo_c64* q,
                     int32_t k0, int32_t k1, const holo_c64* w,
                     holo_c64* g_u, holo_c64* g_q,
                     void* ws, size_t ws_bytes, void* stream);

/* Objective F(u, q) of Eq. (10) over all angles, written to F_dev[0]. */
holo_status holo_objective(holo_plan* plan, const holo_c64* u, const holo_c64* q,
                           const float* amp, const float* amp_ref, double* F_dev,
                           void* ws, size_t ws_bytes, void* stream);

/* Objective and gradients in one sweep.  F_dev, g_u and g_q may each be
 * NULL; with g_u == NULL the R^T sweep is skipped. */
holo_status holo_grad(holo_plan* plan, const holo_c64* u, const holo_c64* q,
                      const float* amp, const float* amp_ref,
                      double* F_dev, holo_c64* g_u, holo_c64* g_q,
                      void* ws, size_t ws_bytes, void* stream);

/* holo_grad with g_q = NULL: gradient with respect to the object only. */
holo_status holo_grad_object(holo_plan* plan, const holo_c64* u, const holo_c64* q,
                             const float* amp, const float* amp_ref,
                             double* F_dev, holo_c64* g_u,
                             void* ws, size_t ws_bytes, void* stream);

/* holo_grad with g_u = NULL: gradient with respect to the probe only (the
 * forward ray sums still run; the R^T sweep does not). */
holo_status holo_grad_probe(holo_plan* plan, const holo_c64* u, const holo_c64* q,
                            const float* amp, const float* amp_ref,
                            double* F_dev, holo_c64* g_q,
                            void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * The solver around the gradient (Sec. 2: conjugate gradients with the
 * Dai-Yuan formula, Eq. 12-13, and the initial probe).
 * ------------------------------------------------------------------------- */

/* Initial probe q_out = D_{-1}(amp_ref): the reference amplitude with zero
 * phase propagated back to sample plane 0 (Sec. 2, initial guess).  amp_ref
 * [H][W] float and q_out [H][W] complex are device pointers; q_out may not
 * alias amp_ref.  Asynchronous on `stream`; needs no workspace. */
holo_status holo_probe_init(holo_plan* plan, const float* amp_ref, holo_c64* q_out,
                            void* stream);

/* Workspace of holo_cg: holo_workspace_bytes plus three vectors the size of
 * (u, q) (gradient, search direction, trial point) and a few kB of partials. */
holo_status holo_cg_workspace_bytes(const holo_plan* plan, size_t* bytes);

/* `iters` iterations of conjugate gradients with the Dai-Yuan formula on the
 * joint objective F(u, q) of Eq. (10) with Eq. (17):
 *   x = (u, q), <a, b> = Re sum conj(a) b over both parts,
 *   eta_0 = -g_0,  x_{m+1} = x_m + gamma_m eta_m,
 *   eta_{m+1} = -g_{m+1} + ||g_{m+1}||^2 / <g_{m+1} - g_m, eta_m> eta_m
 *   (restart eta = -g when that denominator is not positive).
 * gamma_m: halving from a trial step until F does not increase; the first
 * trial of the first iteration is step0 > 0, later ones start at twice the
 * previous accepted step; after 30 halvings the step is 0 and x stays.
 * u [H][W][W] and q [H][W] (device) are read as the starting point and
 * overwritten with the final iterate.  Host outputs: F_hist[iters + 1] (F
 * before the first and after every iteration), and optionally
 * steps[iters] (accepted gamma, 0 if none) and halvings[iters] (halvings of
 * the accepted trial; 31 if none was accepted).  Inner products and F are
 * formed in double on the device.  The line search decides on the host, so
 * the call returns only when the iterations are done (it synchronises
 * `stream`).  Argument errors are returned before any device work. */
holo_status holo_cg(holo_plan* plan, holo_c64* u, holo_c64* q,
                    const float* amp, const float* amp_ref,
                    int32_t iters, double step0,
                    double* F_hist, double* steps, int32_t* halvings,
                    void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Hierarchical schedule (Sec. 4): iterate on binned data, move the result to
 * a grid twice as dense, continue with less binning.  A problem binned by b
 * is the same model on pixels b times larger: H/b x W/b detector,
 * W/b x W/b x H/b volume, fresnel0 * b^2, kappa * b, shifts / b.
 * ------------------------------------------------------------------------- */

/* out[f][y][x] = mean of in[f] over the b x b block (y b .. y b + b - 1,
 * x b .. x b + b - 1), summed in double; with `amplitude` != 0 the data are
 * amplitudes and out = sqrt(mean in^2) (intensities are averaged).  in
 * [n_frames][H][W] float, out [n_frames][H/b][W/b] float (device).
 * Errors: INVALID_ARGUMENT (NULL, sizes < 1, b not dividing H and W, out
 * aliasing in for b > 1). */
holo_status holo_bin_frames(const float* in, int64_t n_frames, int32_t H, int32_t W, int32_t b,
                            int32_t amplitude, float* out, void* stream);

/* Move complex frames [n_frames][H][W] (or a volume [H][W][W]) to the grid
 * f times denser by replication: out[n][f H][f W] with out[.][y][x] =
 * in[.][y / f][x / f] (the volume also along z: out[f H][f W][f W]).
 * Errors: INVALID_ARGUMENT (NULL, sizes or f < 1, out aliasing in). */
holo_status holo_upsample_frames(const holo_c64* in, int64_t n_frames, int32_t H, int32_t W,
                                 int32_t f, holo_c64* out, void* stream);
holo_status holo_upsample_volume(const holo_c64* in, int32_t H, int32_t W, int32_t f,
                                 holo_c64* out, void* stream);

/* ---------------------------------------------------------------------------
 * Batched independent single-angle retrievals (Eq. 10 and Eq. 11 with one
 * projection, psi the unknown, own probe and reference per instance).
 *
 * Instance i is an n_i x n_i problem (n_i one of 64, 128, 192, 256, 384, 512,
 * 1024) with n_dist planes; all instances share the geometry (m~_j, m0, N_F0)
 * and have no shifts.  Arrays are packed: with off_i from holo2d_offsets and
 * T = sum_i n_i^2,
 *   psi, q, g_psi, g_q   [T] complex; instance i at element off_i, row-major
 *   amp, v               [n_dist * T]; instance i at n_dist * off_i, laid out
 *                        [n_dist][n_i][n_i] (float for amp, complex for v)
 *   amp_ref              [T] float
 *   F                    [n_inst] double, one objective per instance
 * Every pass is one launch over all instances.  Same ownership, validation
 * and stream rules as above.
 * ------------------------------------------------------------------------- */
typedef struct holo2d_plan holo2d_plan;

/* Errors: INVALID_ARGUMENT (NULL, n_inst < 1, n_dist outside 1..8, m0 <= 1,
 * fresnel0 <= 0, mag_rel < 1), UNSUPPORTED_SIZE (an unsupported n_i). */
holo_status holo2d_plan_create(int32_t n_inst, const int32_t* sizes, int32_t n_dist,
                               const double* mag_rel, double m0, double fresnel0,
                               holo2d_plan** out);
holo_status holo2d_plan_destroy(holo2d_plan* plan);
/* The functional holo2d_objective and holo2d_grad evaluate, as
 * holo_plan_set_functional: HOLO_FUNCTIONAL_AMPLITUDE (default, F2 of
 * Eq. 10) or HOLO_FUNCTIONAL_INTENSITY (F1 of Eq. 9; amp and amp_ref then
 * hold intensities).  Errors: INVALID_ARGUMENT (NULL plan, unknown value).
 * Host-only. */
holo_status holo2d_plan_set_functional(holo2d_plan* plan, int32_t functional);
/* offsets[n_inst] (elements) and total T of the packed layout. */
holo_status holo2d_offsets(const holo2d_plan* plan, int64_t* offsets, int64_t* total);
holo_status holo2d_workspace_bytes(const holo2d_plan* plan, size_t* bytes);
/* Detector fields v of every instance and plane (Eq. 8 with N_theta = 1). */
holo_status holo2d_fwd(holo2d_plan* plan, const holo_c64* psi, const holo_c64* q, holo_c64* v,
                       void* ws, size_t ws_bytes, void* stream);
/* Objective of every instance (Eq. 10 with the reference term). */
holo_status holo2d_objective(holo2d_plan* plan, const holo_c64* psi, const holo_c64* q,
                             const float* amp, const float* amp_ref, double* F,
                             void* ws, size_t ws_bytes, void* stream);
/* Objectives and gradients; F, g_psi and g_q may each be NULL. */
holo_status holo2d_grad(holo2d_plan* plan, const holo_c64* psi, const holo_c64* q,
                        const float* amp, const float* amp_ref, double* F,
                        holo_c64* g_psi, holo_c64* g_q, void* ws, size_t ws_bytes,
                        void* stream);

/* holo2d_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no workspace argument, and the call performs no hipMalloc, hipFree or
 * other allocation.  The plan's constant tables and the workspace are placed
 * in one static device array of HOLO2D_SCRATCH_MAX_BYTES per GPU, which the
 * library holds from its load until the process ends; each call rewrites
 * the tables there (stream-ordered before its kernels).  The caller still
 * passes every input and output (device pointers, as holo2d_grad; F, g_psi
 * and g_q may each be NULL).  Results equal holo2d_grad's.
 * All calls on one GPU share that GPU's array: calls that overlap on one GPU
 * (different streams or threads without ordering between them) race and
 * give wrong results; calls ordered on one stream are safe.
 * holo2d_noalloc_bytes gives the bytes a plan needs in the array.
 * Errors: INVALID_ARGUMENT (NULL plan, psi, q, amp or amp_ref),
 * WORKSPACE_TOO_SMALL (the plan needs more than HOLO2D_SCRATCH_MAX_BYTES;
 * returned before any device work), HIP. */
#define HOLO2D_SCRATCH_MAX_BYTES (128u << 20)
holo_status holo2d_noalloc_bytes(const holo2d_plan* plan, size_t* bytes);
holo_status holo2d_grad_noalloc(holo2d_plan* plan, const holo_c64* psi, const holo_c64* q,
                                const float* amp, const float* amp_ref, double* F,
                                holo_c64* g_psi, holo_c64* g_q, void* stream);

/* Kernel classes for the timing diagnostics below. */
enum {
  HOLO_K_RADON_FWD = 0,  /* ray sums + exp, one launch per angle chunk          */
  HOLO_K_RADON_ADJ = 1,  /* transpose of the ray sums, one launch per call      */
  HOLO_K_PASS_A = 2,     /* demagnify, probe product, row propagation           */
  HOLO_K_PASS_B = 3,     /* column propagation, residual, adjoint columns       */
  HOLO_K_PASS_C = 4,     /* adjoint rows, probe-gradient accumulation           */
  HOLO_K_PASS_D = 5,     /* transpose of the demagnification, chain rule        */
  HOLO_K_PROBE = 6,      /* probe-side propagations and the reference term      */
  HOLO_K_OTHER = 7,      /* transposed volume copy, fills, sums, reductions     */
  HOLO_K_SOLVER = 8,     /* holo_cg's inner products, updates and copies        */
  HOLO_K_COUNT = 9
};

/* Diagnostics.  holo_timing_enable(plan, 1) clears the counters and makes
 * every later compute call of the plan record a HIP event pair around each
 * kernel launch, on the call's stream; holo_timing_enable(plan, 0) stops
 * recording.  holo_timing_read waits for the recorded events and returns,
 * for one kernel class, the summed kernel time in milliseconds and the number
 * of launches recorded since the counters were cleared.  Errors:
 * INVALID_ARGUMENT (NULL plan or outputs, class out of range), HIP. */
holo_status holo_timing_enable(holo_plan* plan, int32_t on);
holo_status holo_timing_read(holo_plan* plan, int32_t kernel_class,
                             double* total_ms, int64_t* launches);

/* The angle groups of the forward ray sums (diagnostics): consecutive
 * angles of one walk direction, at most 4, never crossing a chunk, whose
 * rays share one staged column window per (block of FWD_BINS bins, row); the
 * plan forms them so that every tap of every row lies at least one column
 * inside its window.  Writes *n_groups and, for i < min(capacity,
 * *n_groups), the first angle and the angle count of group i.  Errors:
 * INVALID_ARGUMENT (NULL plan or n_groups; NULL first or count with
 * capacity > 0).  Host-only. */
holo_status holo_plan_ray_groups(const holo_plan* plan, int32_t* first, int32_t* count,
                                 int32_t capacity, int32_t* n_groups);

/* Message describing the last non-OK status returned on this thread. */
const char* holo_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HOLO_H */
