// Host runtime and C ABI of libholo.so (see include/holo.h).
//
// A plan holds the validated geometry, the transfer-function and twiddle
// tables (built in double precision on the host), the per-angle ray-sum
// constants and the workspace layout.  A compute call enqueues, on the
// caller's stream:
//   probe stage      Q_j = D_{rho_probe_j} q; reference field D_1 q, its cost
//                    and gradient D_{-1}(r_ref)
//   per angle chunk  ray sums + exp -> psi; pass A (rows) -> pass B (columns,
//                    residual) -> pass C (rows, probe gradient) -> pass D
//                    (transpose of the demagnification, chain rule) -> h
//   after the chunks R^T over all angles -> g_u;  g_q = sum_j D_{-rho_probe_j}
//                    G_j + reference gradient;  F = sum of double partials
#include "../../include/holo.h"
#include "holo_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace holo;

namespace {

thread_local std::string g_last_error;

holo_status fail(holo_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

enum Mode { kFwd, kAdj, kObj, kGrad };

}  // namespace

namespace holo {
// Shared with the batched entry points (holo2d_api.cpp).
holo_status set_last_error(holo_status st, const std::string& msg) { return fail(st, msg); }
}  // namespace holo

struct holo_plan {
  int H = 0, W = 0, n_angles = 0, nd = 0, chunk = 64;
  int functional = HOLO_FUNCTIONAL_AMPLITUDE;
  int max_group = 1;                        // largest forward angle group
  double m0 = 0, fresnel0 = 0, kappa = 0;
  std::vector<double> theta, mag;
  std::vector<float> shift;                 // empty = no shifts
  std::vector<float> pshift;                // probe shifts, empty = none
  bool pshift_dirty = false;                // device copy older than pshift
  int fwd_nb = kFwdNB;                      // bins per forward workgroup (16 or 8)
  bool groups_dirty = false;                // device copy older than groups
  std::vector<double> ang;                  // [n_angles][kAngleStride]
  std::vector<float2> twW, twH, chirpW, chirpH;
  // padded propagation (reading P1): 1 = periodic, 2 = padded; the tables
  // of lengths 2W and 2H exist when both edges are at most 1024
  int pad = 1;
  std::vector<float2> tw2W, tw2H, chirp2W, chirp2H;
  // Fourier-slice projector (reading F1): HOLO_PROJECTOR_*, and its tables
  // (built when W <= 1024): 1 / kernel transform, angles sorted modulo pi,
  // first sorted position of every angle bin
  int projector = HOLO_PROJECTOR_JOSEPH;
  // launch-shape choices (the autotuner's tiles): pass B's columns per
  // workgroup (0 = default) and the Fourier-slice slab depth
  int col_tile = 0;
  int fs_slab = kFsSlab;
  // Joseph's forward of the next chunk on a second stream, concurrent with
  // the current chunk's frame passes (two psi buffers); the stream and its
  // fork/join events are made on the first call that needs them
  int overlap = 0;
  hipStream_t side = nullptr;
  hipEvent_t ov_ev[5] = {};
  std::vector<float> fs_dinv;
  std::vector<int> fs_sorted, fs_bins;
  size_t off_fsdinv = 0, off_fssorted = 0, off_fsbins = 0;
  size_t off_fsG = 0, off_fsA = 0;
  bool any_xwalk = false;
  // forward ray-sum angle groups: consecutive angles of one walk direction
  // whose staged row windows fit (first, count); group_of[k] = group index
  std::vector<int2> groups;
  std::vector<int> group_of;
  // transpose angle classes (sin >= 0 / < 0 once rows with cos < 0 are
  // reversed): class 0's angles in ascending order, then class 1's
  std::vector<int> adj_order;
  int adj_n0 = 0;
  // workspace layout (byte offsets)
  size_t off_Q = 0, off_G = 0, off_P = 0, off_ub = 0, off_uTb = 0, off_psi = 0, off_X = 0, off_S = 0,
         off_F = 0, ws_bytes = 0, n_fpart = 0, off_psi2 = 0;
  // device tables (lazily uploaded on the first compute call)
  void* d_tables = nullptr;
  int device = -1;
  size_t off_twW = 0, off_twH = 0, off_chW = 0, off_chH = 0, off_ang = 0, off_shift = 0,
         off_groups = 0, off_pshift = 0, table_bytes = 0, off_Pbuf = 0, off_adjord = 0;
  size_t off_tw2W = 0, off_tw2H = 0, off_ch2W = 0, off_ch2H = 0;
  // timing diagnostics
  bool timing = false;
  std::vector<hipEvent_t> ev_free;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  double t_ms[HOLO_K_COUNT] = {0};
  int64_t t_n[HOLO_K_COUNT] = {0};
};

static void build_chirp(std::vector<float2>& out, int n, const std::vector<double>& rhos,
                        double fresnel0) {
  // exp(-i pi rho k^2 / (N_F0 n^2)) / n with k the signed integer frequency
  out.resize(rhos.size() * (size_t)n);
  for (size_t r = 0; r < rhos.size(); ++r) {
    for (int i = 0; i < n; ++i) {
      const double k = (2 * i < n) ? i : i - n;
      // phase in turns, reduced before the trigonometric evaluation
      double turns = -0.5 * rhos[r] * k * k / (fresnel0 * (double)n * (double)n);
      turns -= std::floor(turns);
      const double ph = 2.0 * M_PI * turns;
      out[r * n + i] = make_float2((float)(std::cos(ph) / n), (float)(std::sin(ph) / n));
    }
  }
}

static void build_twiddles(std::vector<float2>& out, int n) {
  out.resize(n);
  for (int m = 0; m < n; ++m) {
    const double ph = -2.0 * M_PI * (double)m / (double)n;
    out[m] = make_float2((float)std::cos(ph), (float)std::sin(ph));
  }
}

static bool is_finite(double x) { return std::isfinite(x); }

// Fourier-slice tables.  The gridding kernel exp(beta (sqrt(1 - (2x/KW)^2) - 1))
// on |x| < KW/2 has the transform phihat(k) = int phi(x) cos(2 pi k x / M) dx
// (M = 2W grid points); with x = (KW/2) sin(t) the integrand is smooth, and
// Simpson's rule on t in [0, pi/2] gives it to double precision.
static double fs_beta() { return 2.3 * kFsWidth; }

static void build_fs_tables(holo_plan* P) {
  const int W = P->W;
  const double M = 2.0 * W, h = 0.5 * kFsWidth, beta = fs_beta();
  const int n = 4096;                           // Simpson intervals (even)
  P->fs_dinv.resize(W);
  for (int x = 0; x < W; ++x) {
    const double k = (double)(x - W / 2);
    double acc = 0.0;
    for (int i = 0; i <= n; ++i) {
      const double t = 0.5 * M_PI * i / n;
      const double f = std::exp(beta * (std::cos(t) - 1.0)) * std::cos(2.0 * M_PI * k * h * std::sin(t) / M) *
                       h * std::cos(t);
      acc += f * ((i == 0 || i == n) ? 1.0 : (i % 2 ? 4.0 : 2.0));
    }
    const double phihat = 2.0 * acc * (0.5 * M_PI / n) / 3.0;   // both halves
    P->fs_dinv[x] = (float)(1.0 / phihat);
  }
  // angles sorted by theta mod pi, and the first sorted position of every
  // bin [b pi / B, (b + 1) pi / B)
  std::vector<double> tm(P->n_angles);
  for (int k = 0; k < P->n_angles; ++k) {
    double t = std::fmod(P->theta[k], M_PI);
    if (t < 0) t += M_PI;
    if (t >= M_PI) t -= M_PI;
    tm[k] = t;
  }
  P->fs_sorted.resize(P->n_angles);
  for (int k = 0; k < P->n_angles; ++k) P->fs_sorted[k] = k;
  std::stable_sort(P->fs_sorted.begin(), P->fs_sorted.end(),
                   [&](int a, int b) { return tm[a] < tm[b]; });
  P->fs_bins.assign(kFsBins + 1, P->n_angles);
  int pos = 0;
  for (int b = 0; b <= kFsBins; ++b) {
    const double lo = M_PI * b / kFsBins;
    while (pos < P->n_angles && tm[P->fs_sorted[pos]] < lo) ++pos;
    P->fs_bins[b] = b == kFsBins ? P->n_angles : pos;
  }
}

// Can angles [a, b) share the staged row windows of the forward ray sums?
// For each (bin block, row) the window starts one column below the lowest
// tap, floor(mn) - 1.  Tap positions are affine in bin and row, so over the
// group's angles and the block's end bins the highest tap mx is convex in
// the row and the lowest mn concave: their span mx - mn is largest at the
// first or the last row.  A span of at most kFwdSeg - 4 there keeps every
// tap of every row below column kFwdSeg - 2 of its window
// (mx - floor(mn) + 1 < kFwdSeg - 2): the tap and its right neighbour stay
// inside the staged kFwdSeg columns, and the kernel's clamp of the tap base
// (to at most kFwdSeg - 1.01 for the highest tap) only ever acts on windows
// moved into the zero padding.
static bool fwd_group_fits(const holo_plan* P, int a, int b, int nb) {
  const int W = P->W;
  for (int sb = 0; sb < W; sb += nb) {
    for (int r : {0, W - 1}) {
      double mn = 1e300, mx = -1e300;
      for (int k = a; k < b; ++k) {
        const double* g = &P->ang[(size_t)k * kAngleStride];
        for (int bin : {sb, sb + nb - 1}) {
          const double f = g[kA] + (double)bin * g[kB] + (double)r * g[kD];
          mn = std::fmin(mn, f);
          mx = std::fmax(mx, f);
        }
      }
      if (mx - mn > (double)(kFwdSeg - 4)) return false;
    }
  }
  return true;
}

// Forward ray-sum groups for bin blocks of nb bins (never larger than a
// chunk): consecutive angles of one walk direction whose windows fit.
static void form_groups(holo_plan* P, int nb, std::vector<int2>& groups,
                        std::vector<int>& group_of, int& max_group) {
  const int na_max = std::min(kFwdNA, P->chunk);
  groups.clear();
  group_of.assign(P->n_angles, 0);
  max_group = 1;
  for (int a = 0; a < P->n_angles;) {
    int b = a + 1;
    while (b < P->n_angles && b - a < na_max &&
           P->ang[(size_t)b * kAngleStride + kBranch] == P->ang[(size_t)a * kAngleStride + kBranch] &&
           fwd_group_fits(P, a, b + 1, nb))
      ++b;
    for (int k = a; k < b; ++k) group_of[k] = (int)groups.size();
    groups.push_back(make_int2(a, b - a));
    max_group = std::max(max_group, b - a);
    a = b;
  }
}

static void set_fwd_bins(holo_plan* P, int nb) {
  P->fwd_nb = nb;
  form_groups(P, nb, P->groups, P->group_of, P->max_group);
  P->groups_dirty = true;
}

// Workspace layout of a plan (depends on its chunk).
static void layout_workspace(holo_plan* P) {
  const size_t fr = (size_t)P->H * P->W * sizeof(float2);
  size_t o = 0;
  P->off_Q = o;   o = align_up(o + fr * P->nd);
  P->off_G = o;   o = align_up(o + fr * P->nd);
  P->off_P = o;   o = align_up(o + fr);
  // z-blocked copies of the volume read by the ray sums (one per walk
  // direction), rows padded by kFwdPad zero columns on each side
  // (not used by the Fourier-slice projector)
  const size_t vb = P->projector == HOLO_PROJECTOR_FOURIER
                        ? 0 : (size_t)P->H * P->W * vol_row(P->W) * sizeof(float2);
  P->off_ub = o;  o = align_up(o + vb);
  P->off_uTb = o; o = align_up(o + (P->any_xwalk ? vb : 0));
  P->off_psi = o; o = align_up(o + fr * P->chunk);
  // the second psi buffer of the overlapped forward (Joseph's ray sums only)
  const bool two_psi = P->overlap && P->projector == HOLO_PROJECTOR_JOSEPH;
  P->off_psi2 = o; o = align_up(o + (two_psi ? fr * P->chunk : 0));
  P->off_X = o;   o = align_up(o + fr * P->chunk * P->nd);
  // sinogram rows carry kAdjPad zero bins on each side
  P->off_S = o;   o = align_up(o + (size_t)P->H * sino_row(P->W) * sizeof(float2) * P->n_angles);
  // cost slots: the reference term's column tiles, then every frame's; sized
  // for the most tiles any column pass of the plan can use (the padded pass,
  // or pass B at half its default tile), so tuning never resizes them
  const size_t pt = P->chirp2W.empty() ? 0 : (size_t)pad_col_tiles(P->H, P->W);
  const size_t ref_tiles = std::max((size_t)(P->W / cols_per_wg(P->H)), pt);
  const size_t tiles = std::max((size_t)(P->W / (cols_per_wg(P->H) / 2)), pt);
  P->n_fpart = ref_tiles + tiles * (size_t)P->n_angles * P->nd;
  // cost partials, then the reduction's stage-one sums
  P->off_F = o;   o = align_up(o + (P->n_fpart + kReduceParts) * sizeof(double));
  // with probe shifts: conj(phi) w of every frame of a chunk
  P->off_Pbuf = o; o = align_up(o + (P->pshift.empty() ? 0 : fr * P->chunk * P->nd));
  // Fourier-slice projector: the grids of one slab and its polar samples
  const bool fs = P->projector == HOLO_PROJECTOR_FOURIER;
  const size_t M = 2 * (size_t)P->W;
  P->off_fsG = o; o = align_up(o + (fs ? (size_t)kFsSlab * M * M * sizeof(float2) : 0));
  P->off_fsA = o;
  o = align_up(o + (fs ? (size_t)kFsSlab * P->n_angles * (P->W + 2) * sizeof(float2) : 0));
  P->ws_bytes = o;
}

extern "C" holo_status holo_plan_create(const holo_geom* geom, holo_plan** out) {
  if (!out) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_create: out is NULL");
  *out = nullptr;
  if (!geom) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_create: geom is NULL");
  const holo_geom& G = *geom;
  if (G.n_angles < 1) return fail(HOLO_ERR_INVALID_ARGUMENT, "n_angles must be >= 1");
  if (G.n_dist < 1 || G.n_dist > kMaxDist)
    return fail(HOLO_ERR_INVALID_ARGUMENT, "n_dist must be in 1..8");
  if (!G.theta || !G.mag_rel) return fail(HOLO_ERR_INVALID_ARGUMENT, "theta/mag_rel is NULL");
  if (!fft_size_supported(G.det_rows) || !fft_size_supported(G.det_cols))
    return fail(HOLO_ERR_UNSUPPORTED_SIZE,
                "det_rows and det_cols must each be one of 64,128,192,256,384,512,1024,2048 (got " +
                    std::to_string(G.det_rows) + "x" + std::to_string(G.det_cols) + ")");
  if (!(is_finite(G.m0) && G.m0 > 1.0)) return fail(HOLO_ERR_INVALID_ARGUMENT, "m0 must be finite and > 1");
  if (!(is_finite(G.fresnel0) && G.fresnel0 > 0.0))
    return fail(HOLO_ERR_INVALID_ARGUMENT, "fresnel0 must be finite and > 0");
  if (!is_finite(G.kappa)) return fail(HOLO_ERR_INVALID_ARGUMENT, "kappa must be finite");
  if (G.chunk < 0) return fail(HOLO_ERR_INVALID_ARGUMENT, "chunk must be >= 0");
  for (int j = 0; j < G.n_dist; ++j)
    if (!(is_finite(G.mag_rel[j]) && G.mag_rel[j] >= 1.0))
      return fail(HOLO_ERR_INVALID_ARGUMENT, "mag_rel[j] must be finite and >= 1");
  for (int k = 0; k < G.n_angles; ++k)
    if (!is_finite(G.theta[k])) return fail(HOLO_ERR_INVALID_ARGUMENT, "theta must be finite");
  if (G.shift) {
    for (size_t i = 0; i < (size_t)G.n_angles * G.n_dist * 2; ++i)
      if (!std::isfinite(G.shift[i])) return fail(HOLO_ERR_INVALID_ARGUMENT, "shift must be finite");
  }

  holo_plan* P = new (std::nothrow) holo_plan();
  if (!P) return fail(HOLO_ERR_OUT_OF_HOST_MEMORY, "holo_plan_create: out of host memory");
  try {
    P->H = G.det_rows;
    P->W = G.det_cols;
    P->n_angles = G.n_angles;
    P->nd = G.n_dist;
    P->chunk = G.chunk > 0 ? G.chunk : 64;
    if (P->chunk > P->n_angles) P->chunk = P->n_angles;
    P->m0 = G.m0;
    P->fresnel0 = G.fresnel0;
    P->kappa = G.kappa;
    P->theta.assign(G.theta, G.theta + G.n_angles);
    P->mag.assign(G.mag_rel, G.mag_rel + G.n_dist);
    if (G.shift) P->shift.assign(G.shift, G.shift + (size_t)G.n_angles * G.n_dist * 2);

    // Per-angle ray constants.  Walk along y when |cos| >= |sin|: the ray of
    // bin i crosses row `step` at x = c + ((i - c) - (step - c) sin) / cos;
    // otherwise walk along x with the roles of the axes exchanged.
    const double c = P->W / 2.0;
    P->ang.resize((size_t)P->n_angles * kAngleStride);
    for (int k = 0; k < P->n_angles; ++k) {
      const double C = std::cos(P->theta[k]), S = std::sin(P->theta[k]);
      double* a = &P->ang[(size_t)k * kAngleStride];
      a[kCos] = C;
      a[kSin] = S;
      const double h = std::fmax(std::fabs(C), std::fabs(S));
      a[kInvH] = 1.0 / h;
      a[kScale] = 1.0 / h;
      if (std::fabs(C) >= std::fabs(S)) {
        a[kBranch] = 0.0;
        a[kB] = 1.0 / C;
        a[kD] = -S / C;
        a[kA] = c - c / C + c * S / C;
      } else {
        a[kBranch] = 1.0;
        a[kB] = 1.0 / S;
        a[kD] = -C / S;
        a[kA] = c - c / S + c * C / S;
        P->any_xwalk = true;
      }
    }

    // Forward ray-sum groups for blocks of kFwdNB bins (8-bin blocks are a
    // tuning choice, holo_plan_set_tile).
    set_fwd_bins(P, kFwdNB);
    // Transpose angle classes.
    for (int cls = 0; cls < 2; ++cls)
      for (int k = 0; k < P->n_angles; ++k)
        if (adj_class(&P->ang[(size_t)k * kAngleStride]) == cls) P->adj_order.push_back(k);
    P->adj_n0 = (int)(std::count_if(P->adj_order.begin(), P->adj_order.end(), [&](int k) {
      return adj_class(&P->ang[(size_t)k * kAngleStride]) == 0;
    }));

    // Transfer-function tables: detector steps, probe steps, reference.
    std::vector<double> rhos(chirp_rows(P->nd));
    for (int j = 0; j < P->nd; ++j) {
      const double m = P->mag[j];
      rhos[chirp_det(j)] = (P->m0 - m) / (m * (P->m0 - 1.0));
      rhos[chirp_probe(P->nd, j)] = P->m0 * (m - 1.0) / (m * (P->m0 - 1.0));
    }
    rhos[chirp_ref(P->nd)] = 1.0;
    build_chirp(P->chirpW, P->W, rhos, P->fresnel0);
    build_chirp(P->chirpH, P->H, rhos, P->fresnel0);
    build_twiddles(P->twW, P->W);
    build_twiddles(P->twH, P->H);
    if (pad_size_supported(P->H) && pad_size_supported(P->W)) {
      build_chirp(P->chirp2W, 2 * P->W, rhos, P->fresnel0);
      build_chirp(P->chirp2H, 2 * P->H, rhos, P->fresnel0);
      build_twiddles(P->tw2H, 2 * P->H);
    }
    if (fs_size_supported(P->W)) {
      build_twiddles(P->tw2W, 2 * P->W);
      build_fs_tables(P);
    }

    layout_workspace(P);

    // Device table layout.
    size_t t = 0;
    P->off_twW = t;   t = align_up(t + P->twW.size() * sizeof(float2));
    P->off_twH = t;   t = align_up(t + P->twH.size() * sizeof(float2));
    P->off_chW = t;   t = align_up(t + P->chirpW.size() * sizeof(float2));
    P->off_chH = t;   t = align_up(t + P->chirpH.size() * sizeof(float2));
    P->off_ang = t;   t = align_up(t + P->ang.size() * sizeof(double));
    P->off_shift = t; t = align_up(t + P->shift.size() * sizeof(float));
    P->off_groups = t; t = align_up(t + (size_t)P->n_angles * sizeof(int2));
    P->off_adjord = t; t = align_up(t + (size_t)P->n_angles * sizeof(int));
    // probe shifts (room for all of them, filled when set)
    P->off_pshift = t; t = align_up(t + (size_t)P->n_angles * P->nd * 2 * sizeof(float));
    P->off_tw2W = t;  t = align_up(t + P->tw2W.size() * sizeof(float2));
    P->off_tw2H = t;  t = align_up(t + P->tw2H.size() * sizeof(float2));
    P->off_ch2W = t;  t = align_up(t + P->chirp2W.size() * sizeof(float2));
    P->off_ch2H = t;  t = align_up(t + P->chirp2H.size() * sizeof(float2));
    P->off_fsdinv = t;  t = align_up(t + P->fs_dinv.size() * sizeof(float));
    P->off_fssorted = t; t = align_up(t + P->fs_sorted.size() * sizeof(int));
    P->off_fsbins = t;  t = align_up(t + P->fs_bins.size() * sizeof(int));
    P->table_bytes = t + 256;
  } catch (const std::bad_alloc&) {
    delete P;
    return fail(HOLO_ERR_OUT_OF_HOST_MEMORY, "holo_plan_create: out of host memory");
  }
  *out = P;
  return HOLO_OK;
}

extern "C" holo_status holo_plan_destroy(holo_plan* P) {
  if (!P) return HOLO_OK;
  for (auto& pe : P->ev_pending) {
    (void)hipEventSynchronize(pe.second.second);
    (void)hipEventDestroy(pe.second.first);
    (void)hipEventDestroy(pe.second.second);
  }
  for (hipEvent_t e : P->ev_free) (void)hipEventDestroy(e);
  if (P->side) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != P->device) (void)hipSetDevice(P->device);
    (void)hipStreamSynchronize(P->side);
    for (hipEvent_t& e : P->ov_ev)
      if (e) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(P->side);
    if (cur != P->device && cur >= 0) (void)hipSetDevice(cur);
  }
  if (P->d_tables) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != P->device) (void)hipSetDevice(P->device);
    (void)hipFree(P->d_tables);
    if (cur != P->device && cur >= 0) (void)hipSetDevice(cur);
  }
  delete P;
  return HOLO_OK;
}

extern "C" holo_status holo_workspace_bytes(const holo_plan* P, size_t* bytes) {
  if (!P || !bytes) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_workspace_bytes: NULL argument");
  *bytes = P->ws_bytes;
  return HOLO_OK;
}

extern "C" const char* holo_last_error(void) { return g_last_error.c_str(); }

namespace {

holo_status hip_fail(hipError_t e, const char* where) {
  return fail(HOLO_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HOLO_HIP(call)                                  \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #call);   \
  } while (0)

hipEvent_t take_event(holo_plan* P) {
  if (!P->ev_free.empty()) {
    hipEvent_t e = P->ev_free.back();
    P->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Run one launcher, bracketed by an event pair when timing is on.
template <class F>
hipError_t timed(holo_plan* P, int cls, hipStream_t st, F&& launch) {
  if (!P->timing) return launch();
  hipEvent_t a = take_event(P), b = take_event(P);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, st);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, st);
  if (e != hipSuccess) return e;
  P->ev_pending.push_back({cls, {a, b}});
  return hipSuccess;
}

holo_status drain_events(holo_plan* P) {
  for (auto& pe : P->ev_pending) {
    HOLO_HIP(hipEventSynchronize(pe.second.second));
    float ms = 0.f;
    HOLO_HIP(hipEventElapsedTime(&ms, pe.second.first, pe.second.second));
    P->t_ms[pe.first] += ms;
    P->t_n[pe.first] += 1;
    P->ev_free.push_back(pe.second.first);
    P->ev_free.push_back(pe.second.second);
  }
  P->ev_pending.clear();
  return HOLO_OK;
}

holo_status ensure_tables(holo_plan* P) {
  int dev = -1;
  HOLO_HIP(hipGetDevice(&dev));
  if (P->d_tables) {
    if (dev != P->device)
      return fail(HOLO_ERR_INVALID_ARGUMENT, "plan tables live on device " + std::to_string(P->device) +
                                                 ", current device is " + std::to_string(dev));
    if (P->pshift_dirty && !P->pshift.empty())
      HOLO_HIP(hipMemcpy((char*)P->d_tables + P->off_pshift, P->pshift.data(),
                         P->pshift.size() * sizeof(float), hipMemcpyHostToDevice));
    P->pshift_dirty = false;
    if (P->groups_dirty)
      HOLO_HIP(hipMemcpy((char*)P->d_tables + P->off_groups, P->groups.data(),
                         P->groups.size() * sizeof(int2), hipMemcpyHostToDevice));
    P->groups_dirty = false;
    return HOLO_OK;
  }
  const size_t bytes = P->table_bytes;
  void* d = nullptr;
  HOLO_HIP(hipMalloc(&d, bytes));
  char* b = (char*)d;
  auto put = [&](size_t off, const void* src, size_t n) -> hipError_t {
    return n ? hipMemcpy(b + off, src, n, hipMemcpyHostToDevice) : hipSuccess;
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = put(P->off_twW, P->twW.data(), P->twW.size() * sizeof(float2));
  if (e == hipSuccess) e = put(P->off_twH, P->twH.data(), P->twH.size() * sizeof(float2));
  if (e == hipSuccess) e = put(P->off_chW, P->chirpW.data(), P->chirpW.size() * sizeof(float2));
  if (e == hipSuccess) e = put(P->off_chH, P->chirpH.data(), P->chirpH.size() * sizeof(float2));
  if (e == hipSuccess) e = put(P->off_ang, P->ang.data(), P->ang.size() * sizeof(double));
  if (e == hipSuccess) e = put(P->off_shift, P->shift.data(), P->shift.size() * sizeof(float));
  if (e == hipSuccess) e = put(P->off_groups, P->groups.data(), P->groups.size() * sizeof(int2));
  if (e == hipSuccess) e = put(P->off_adjord, P->adj_order.data(), P->adj_order.size() * sizeof(int));
  if (e == hipSuccess) e = put(P->off_pshift, P->pshift.data(), P->pshift.size() * sizeof(float));
  if (e == hipSuccess) e = put(P->off_tw2W, P->tw2W.data(), P->tw2W.size() * sizeof(float2));
  if (e == hipSuccess) e = put(P->off_tw2H, P->tw2H.data(), P->tw2H.size() * sizeof(float2));
  if (e == hipSuccess) e = put(P->off_ch2W, P->chirp2W.data(), P->chirp2W.size() * sizeof(float2));
  if (e == hipSuccess) e = put(P->off_ch2H, P->chirp2H.data(), P->chirp2H.size() * sizeof(float2));
  if (e == hipSuccess) e = put(P->off_fsdinv, P->fs_dinv.data(), P->fs_dinv.size() * sizeof(float));
  if (e == hipSuccess) e = put(P->off_fssorted, P->fs_sorted.data(), P->fs_sorted.size() * sizeof(int));
  if (e == hipSuccess) e = put(P->off_fsbins, P->fs_bins.data(), P->fs_bins.size() * sizeof(int));
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(e, "uploading plan tables");
  }
  P->d_tables = d;
  P->device = dev;
  P->pshift_dirty = false;
  P->groups_dirty = false;
  return HOLO_OK;
}

DevGeom make_geom(const holo_plan* P) {
  DevGeom g;
  g.H = P->H;
  g.W = P->W;
  g.nd = P->nd;
  g.n_angles = P->n_angles;
  g.cH = P->H / 2.0;
  g.cW = P->W / 2.0;
  for (int j = 0; j < kMaxDist; ++j) g.mag[j] = j < P->nd ? P->mag[j] : 1.0;
  g.kappa = (float)P->kappa;
  const char* b = (const char*)P->d_tables;
  g.twW = (const float2*)(b + P->off_twW);
  g.twH = (const float2*)(b + P->off_twH);
  g.chirpW = (const float2*)(b + P->off_chW);
  g.chirpH = (const float2*)(b + P->off_chH);
  g.shift = P->shift.empty() ? nullptr : (const float*)(b + P->off_shift);
  // the conventional functional has the amplitude residual
  g.functional = P->functional == HOLO_FUNCTIONAL_INTENSITY ? 1 : 0;
  g.pshift = P->pshift.empty() ? nullptr : (const float*)(b + P->off_pshift);
  const bool tabs = !P->chirp2W.empty();
  g.tw2W = P->tw2W.empty() ? nullptr : (const float2*)(b + P->off_tw2W);
  g.tw2H = tabs ? (const float2*)(b + P->off_tw2H) : nullptr;
  g.chirp2W = tabs ? (const float2*)(b + P->off_ch2W) : nullptr;
  g.chirp2H = tabs ? (const float2*)(b + P->off_ch2H) : nullptr;
  g.col_tile = P->col_tile;
  g.ang = (const double*)(b + P->off_ang);
  g.sino_mirror = P->projector == HOLO_PROJECTOR_JOSEPH ? 1 : 0;
  return g;
}

holo_status run(holo_plan* P, Mode mode, const holo_c64* u_, const holo_c64* q_, int k0, int k1,
                const holo_c64* w_in_, holo_c64* v_out_, const float* amp, const float* amp_ref,
                double* F, holo_c64* gu_, holo_c64* gq_, void* ws, size_t ws_bytes, void* stream_) {
  const float2* u = (const float2*)u_;
  const float2* q = (const float2*)q_;
  const float2* w_in = (const float2*)w_in_;
  float2* v_out = (float2*)v_out_;
  float2* gu = (float2*)gu_;
  float2* gq = (float2*)gq_;
  hipStream_t st = (hipStream_t)stream_;

  if (!ws) return fail(HOLO_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (ws_bytes < P->ws_bytes)
    return fail(HOLO_ERR_WORKSPACE_TOO_SMALL, "workspace needs " + std::to_string(P->ws_bytes) +
                                                  " bytes, got " + std::to_string(ws_bytes));
  holo_status ts = ensure_tables(P);
  if (ts != HOLO_OK) return ts;

  const DevGeom g = make_geom(P);
  const int H = P->H, W = P->W, nd = P->nd;
  const size_t HW = (size_t)H * W;
  char* wsb = (char*)ws;
  float2* Q = (float2*)(wsb + P->off_Q);
  float2* Gacc = (float2*)(wsb + P->off_G);
  float2* Pref = (float2*)(wsb + P->off_P);
  float2* ub = (float2*)(wsb + P->off_ub);
  float2* uTb = (float2*)(wsb + P->off_uTb);
  float2* psi = (float2*)(wsb + P->off_psi);
  float2* X = (float2*)(wsb + P->off_X);
  float2* S = (float2*)(wsb + P->off_S);
  double* Fpart = (double*)(wsb + P->off_F);
  float2* Pbuf = P->pshift.empty() ? nullptr : (float2*)(wsb + P->off_Pbuf);
  const double* d_ang = (const double*)((const char*)P->d_tables + P->off_ang);
  const bool padded = P->pad == 2;
  // cost slots: ref_tiles of the reference term (the probe-side column
  // launch), then `tiles` per frame (the frame column launches)
  const int ref_tiles = padded ? pad_col_tiles(H, W) : W / cols_per_wg(H);
  const int tiles = padded ? pad_col_tiles(H, W)
                           : W / (P->col_tile ? P->col_tile : cols_per_wg(H));
  // a padded propagation over `n` frames (see PadJob)
  auto pj = [&](const float2* src, float2* dst, long long step, int n, int chirp0, int cmod,
                int conj, int pmode, const float* a, int fslot0) {
    PadJob jb;
    jb.src = src;
    jb.dst = dst;
    jb.amp = a;
    jb.src_step = step;
    jb.nframes = n;
    jb.chirp0 = chirp0;
    jb.cmod = cmod;
    jb.conj = conj;
    jb.mode = pmode;
    jb.fslot0 = fslot0;
    return jb;
  };
  const long long hw = (long long)HW;

  // The conventional functional is the model with q = 1 and no reference
  // term: F does not depend on q, so g_q = 0.
  const bool conv = P->functional == HOLO_FUNCTIONAL_CONVENTIONAL;
  const bool want_F = (mode == kObj || mode == kGrad) && F;
  const bool want_gq = (mode == kAdj || mode == kGrad) && gq && !conv;
  const bool want_gu = (mode == kAdj || mode == kGrad) && gu;
  const bool with_ref = (mode == kObj || mode == kGrad) && !conv;

  // Probe stage.
  if (conv) {
    HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] {
      return launch_fill(Q, nd * HW, make_float2(1.f, 0.f), st);
    }));
    if ((mode == kAdj || mode == kGrad) && gq)
      HOLO_HIP(timed(P, HOLO_K_OTHER, st, [&] { return launch_fill_zero(gq, HW, st); }));
  } else if (padded) {
    const int cp = chirp_probe(nd, 0), cr = chirp_ref(nd);
    const PadJob rq = pj(q, Q, 0, nd, cp, nd, 0, 0, nullptr, 0);
    const PadJob cq = pj(Q, Q, hw, nd, cp, nd, 0, 0, nullptr, 0);
    HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] { return launch_rows_pad(g, rq, st); }));
    HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] { return launch_cols_pad(g, cq, Fpart, st); }));
    if (with_ref) {
      // the reference field, its residual (cost slots 0 .. ref_tiles - 1) and,
      // for the probe gradient, its adjoint propagation
      const PadJob rr = pj(q, Pref, 0, 1, cr, 1, 0, 0, nullptr, 0);
      const PadJob cr2 = pj(Pref, Pref, hw, 1, cr, 1, 0, want_gq ? 1 : 2, amp_ref, 0);
      HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] { return launch_rows_pad(g, rr, st); }));
      HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] { return launch_cols_pad(g, cr2, Fpart, st); }));
      if (want_gq) {
        const PadJob ra = pj(Pref, Pref, hw, 1, cr, 1, 1, 0, nullptr, 0);
        HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] { return launch_rows_pad(g, ra, st); }));
      }
    }
  } else {
    PropJobs rj{}, cj{};
    for (int j = 0; j < nd; ++j) {
      rj.job[rj.n++] = PropJob{q, Q + j * HW, nullptr, chirp_probe(nd, j), 0, 0};
      cj.job[cj.n++] = PropJob{Q + j * HW, Q + j * HW, nullptr, chirp_probe(nd, j), 0, 0};
    }
    if (with_ref) {
      rj.job[rj.n++] = PropJob{q, Pref, nullptr, chirp_ref(nd), 0, 0};
      cj.job[cj.n++] = PropJob{Pref, Pref, amp_ref, chirp_ref(nd), 0, 0};
    }
    HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] { return launch_rows_prop(g, rj, st); }));
    HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] { return launch_cols_prop(g, cj, Fpart, st); }));
    if (with_ref && want_gq) {
      PropJobs r2{}, c2{};
      r2.job[r2.n++] = PropJob{Pref, Pref, nullptr, chirp_ref(nd), 1, 0};
      c2.job[c2.n++] = PropJob{Pref, Pref, nullptr, chirp_ref(nd), 1, 0};
      HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] { return launch_rows_prop(g, r2, st); }));
      HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] { return launch_cols_prop(g, c2, Fpart, st); }));
    }
  }
  // Fourier-slice projector: psi of every angle of the call into the
  // sinogram buffer now, slab by slab; the chunks copy theirs from there
  const bool fs = P->projector == HOLO_PROJECTOR_FOURIER;
  FsArgs fa{};
  float2* fsG = (float2*)(wsb + P->off_fsG);
  float2* fsA = (float2*)(wsb + P->off_fsA);
  const int Wp = sino_row(W);
  if (fs) {
    const char* tb = (const char*)P->d_tables;
    fa.K = k1 - k0;
    fa.k0 = k0;
    fa.n_angles = P->n_angles;
    fa.beta = (float)fs_beta();
    fa.dinv = (const float*)(tb + P->off_fsdinv);
    fa.ang = d_ang;
    fa.sorted_k = (const int*)(tb + P->off_fssorted);
    fa.bin_first = (const int*)(tb + P->off_fsbins);
    for (int z0 = 0; z0 < H; z0 += P->fs_slab) {
      const int nz = std::min(P->fs_slab, H - z0);
      HOLO_HIP(timed(P, HOLO_K_RADON_FWD, st, [&] {
        return launch_fs_forward_slab(g, fa, u + (size_t)z0 * W * W, fsG, S, z0, nz, st);
      }));
    }
  } else {
    bool xwalk = false;
    for (int k = k0; k < k1; ++k) xwalk |= P->ang[(size_t)k * kAngleStride + kBranch] != 0.0;
    HOLO_HIP(timed(P, HOLO_K_OTHER, st, [&] {
      return launch_block_volume(g, u, ub, xwalk ? uTb : nullptr, st);
    }));
  }
  if (want_gq) HOLO_HIP(timed(P, HOLO_K_OTHER, st, [&] { return launch_fill_zero(Gacc, nd * HW, st); }));

  const bool frames_back = want_gq || want_gu;
  const int2* d_groups = (const int2*)((const char*)P->d_tables + P->off_groups);
  // Chunks [c0, c1): whole ray-sum groups (clipped to [k0, k1)), at most
  // `chunk` angles.
  std::vector<int2> chunks;
  for (int c0 = k0, c1 = k0; c0 < k1; c0 = c1) {
    c1 = c0;
    while (c1 < k1) {
      const int2 gr = P->groups[P->group_of[c1]];
      const int end = std::min(gr.x + gr.y, k1);
      if (end - c0 > P->chunk) break;
      c1 = end;
    }
    if (c1 == c0) c1 = std::min(c0 + P->chunk, k1);
    chunks.push_back(make_int2(c0, c1));
  }
  // With the overlap on, chunk i + 1's forward runs on the side stream
  // (into the other psi buffer) while chunk i's frame passes run on the
  // caller's stream: the forward waits for the frames that last read its
  // buffer (chunk i - 1), the frames for their own forward.
  const bool ovl = P->overlap && !fs && chunks.size() > 1;
  float2* psib[2] = {psi, ovl ? (float2*)(wsb + P->off_psi2) : psi};
  hipStream_t sf = st;
  if (ovl) {
    if (!P->side) {
      // made all together or not at all
      hipStream_t side = nullptr;
      hipEvent_t ev[5] = {};
      hipError_t e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
      for (int i = 0; i < 5 && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
      if (e != hipSuccess) {
        for (hipEvent_t x : ev)
          if (x) (void)hipEventDestroy(x);
        if (side) (void)hipStreamDestroy(side);
        return fail(HOLO_ERR_HIP, std::string("overlapped forward: ") + hipGetErrorString(e));
      }
      P->side = side;
      for (int i = 0; i < 5; ++i) P->ov_ev[i] = ev[i];
    }
    sf = P->side;
    // the side stream starts after everything so far on the caller's
    // stream (the volume copies, the probe stage)
    HOLO_HIP(hipEventRecord(P->ov_ev[0], st));
    HOLO_HIP(hipStreamWaitEvent(sf, P->ov_ev[0], 0));
  }
  hipEvent_t* ev_fwd = P->ov_ev + 1;      // [chunk parity]: forward done
  hipEvent_t* ev_frames = P->ov_ev + 3;   // [chunk parity]: its frames done
  auto forward = [&](size_t ci) -> hipError_t {
    const int c0 = chunks[ci].x, c1 = chunks[ci].y;
    const int gfirst = P->group_of[c0], glast = P->group_of[c1 - 1];
    hipError_t e = timed(P, HOLO_K_RADON_FWD, sf, [&] {
      return launch_radon_fwd(g, ub, uTb, psib[ci & 1], d_ang, d_groups, gfirst,
                              glast - gfirst + 1, c0, c1, P->fwd_nb, sf);
    });
    if (e == hipSuccess && ovl) e = hipEventRecord(ev_fwd[ci & 1], sf);
    return e;
  };
  if (ovl) HOLO_HIP(forward(0));
  for (size_t ci = 0; ci < chunks.size(); ++ci) {
    const int c0 = chunks[ci].x, c1 = chunks[ci].y;
    const int Kc = c1 - c0;
    float2* const psi_c = psib[ci & 1];
    if (fs) {
      HOLO_HIP(timed(P, HOLO_K_OTHER, st, [&] {
        return launch_copy_rows(S + (size_t)(c0 - k0) * H * Wp + kAdjPad, Wp, psi_c,
                                (size_t)Kc * H, W, st);
      }));
    } else if (ovl) {
      HOLO_HIP(hipStreamWaitEvent(st, ev_fwd[ci & 1], 0));
      if (ci + 1 < chunks.size()) {
        if (ci >= 1) HOLO_HIP(hipStreamWaitEvent(sf, ev_frames[(ci + 1) & 1], 0));
        HOLO_HIP(forward(ci + 1));
      }
    } else {
      HOLO_HIP(forward(ci));
    }
    double* Fc = Fpart + ref_tiles + (size_t)tiles * (c0 - k0) * nd;
    if (padded) {
      // the unfused sequence: elementwise pass A, padded rows, padded
      // columns (with the residual and the adjoint columns), padded adjoint
      // rows, elementwise pass C
      const int nf = Kc * nd;
      float2* F0 = mode == kFwd ? v_out + (size_t)(c0 - k0) * nd * HW : X;
      if (mode != kAdj) {
        HOLO_HIP(timed(P, HOLO_K_PASS_A, st, [&] {
          return launch_frames_x(g, psi_c, Q, F0, c0, Kc, st);
        }));
        const PadJob rf = pj(F0, F0, hw, nf, chirp_det(0), nd, 0, 0, nullptr, 0);
        HOLO_HIP(timed(P, HOLO_K_PASS_A, st, [&] { return launch_rows_pad(g, rf, st); }));
      }
      PadJob cf;
      if (mode == kFwd) {
        cf = pj(F0, F0, hw, nf, chirp_det(0), nd, 0, 0, nullptr, 0);
      } else if (mode == kAdj) {
        cf = pj(w_in + (size_t)(c0 - k0) * nd * HW, X, hw, nf, chirp_det(0), nd, 1, 0, nullptr, 0);
      } else {
        cf = pj(X, X, hw, nf, chirp_det(0), nd, 0, frames_back ? 1 : 2,
                amp + (size_t)c0 * nd * HW, (int)(Fc - Fpart));
      }
      HOLO_HIP(timed(P, HOLO_K_PASS_B, st, [&] { return launch_cols_pad(g, cf, Fpart, st); }));
      if ((mode == kGrad || mode == kAdj) && frames_back) {
        const PadJob ra = pj(X, X, hw, nf, chirp_det(0), nd, 1, 0, nullptr, 0);
        HOLO_HIP(timed(P, HOLO_K_PASS_C, st, [&] { return launch_rows_pad(g, ra, st); }));
        HOLO_HIP(timed(P, HOLO_K_PASS_C, st, [&] {
          return launch_frames_c(g, X, psi_c, Q, Gacc, Pbuf, want_gq ? 1 : 0, c0, Kc, st);
        }));
        if (want_gq && Pbuf)
          HOLO_HIP(timed(P, HOLO_K_PASS_C, st, [&] {
            return launch_probe_shift_acc(g, Gacc, Pbuf, c0, Kc, st);
          }));
        if (want_gu)
          HOLO_HIP(timed(P, HOLO_K_PASS_D, st, [&] {
            return launch_pass_d(g, X, psi_c, S + (size_t)(c0 - k0) * H * sino_row(W), c0, Kc, st);
          }));
      }
      if (ovl) HOLO_HIP(hipEventRecord(ev_frames[ci & 1], st));
      continue;
    }
    switch (mode) {
      case kFwd: {
        float2* v = v_out + (size_t)(c0 - k0) * nd * HW;
        HOLO_HIP(timed(P, HOLO_K_PASS_A, st, [&] { return launch_pass_a(g, psi_c, Q, v, c0, Kc, st); }));
        HOLO_HIP(timed(P, HOLO_K_PASS_B, st, [&] {
          return launch_pass_b(g, kColFwd, nullptr, v, nullptr, nullptr, Kc, st);
        }));
        break;
      }
      case kObj:
      case kGrad: {
        HOLO_HIP(timed(P, HOLO_K_PASS_A, st, [&] { return launch_pass_a(g, psi_c, Q, X, c0, Kc, st); }));
        const float* a = amp + (size_t)c0 * nd * HW;
        HOLO_HIP(timed(P, HOLO_K_PASS_B, st, [&] {
          return launch_pass_b(g, frames_back ? kColGrad : kColObj, nullptr, X, a, Fc, Kc, st);
        }));
        break;
      }
      case kAdj: {
        const float2* w = w_in + (size_t)(c0 - k0) * nd * HW;
        HOLO_HIP(timed(P, HOLO_K_PASS_B, st, [&] {
          return launch_pass_b(g, kColAdj, w, X, nullptr, nullptr, Kc, st);
        }));
        break;
      }
    }
    if ((mode == kGrad || mode == kAdj) && frames_back) {
      HOLO_HIP(timed(P, HOLO_K_PASS_C, st, [&] {
        return launch_pass_c(g, X, psi_c, Q, Gacc, Pbuf, want_gq ? 1 : 0, c0, Kc, st);
      }));
      if (want_gq && Pbuf)
        HOLO_HIP(timed(P, HOLO_K_PASS_C, st, [&] {
          return launch_probe_shift_acc(g, Gacc, Pbuf, c0, Kc, st);
        }));
      if (want_gu)
        HOLO_HIP(timed(P, HOLO_K_PASS_D, st, [&] {
          return launch_pass_d(g, X, psi_c, S + (size_t)(c0 - k0) * H * sino_row(W), c0, Kc, st);
        }));
    }
    if (ovl) HOLO_HIP(hipEventRecord(ev_frames[ci & 1], st));
  }
  if (want_gu && fs) {
    for (int z0 = 0; z0 < H; z0 += P->fs_slab) {
      const int nz = std::min(P->fs_slab, H - z0);
      HOLO_HIP(timed(P, HOLO_K_RADON_ADJ, st, [&] {
        return launch_fs_adjoint_slab(g, fa, S, fsA, fsG, gu + (size_t)z0 * W * W, z0, nz, st);
      }));
    }
  } else if (want_gu) {
    // each class's angles within [k0, k1): a contiguous run of its list
    const int* ord = (const int*)((const char*)P->d_tables + P->off_adjord);
    const auto b0 = P->adj_order.begin(), e0 = b0 + P->adj_n0, e1 = P->adj_order.end();
    const int lo0 = (int)(std::lower_bound(b0, e0, k0) - b0);
    const int hi0 = (int)(std::lower_bound(b0, e0, k1) - b0);
    const int lo1 = (int)(std::lower_bound(e0, e1, k0) - b0);
    const int hi1 = (int)(std::lower_bound(e0, e1, k1) - b0);
    HOLO_HIP(timed(P, HOLO_K_RADON_ADJ, st, [&] {
      return launch_radon_adj(g, S, gu, d_ang, k0, ord + lo0, hi0 - lo0, ord + lo1, hi1 - lo1, st);
    }));
  }
  if (want_gq) {
    if (padded) {
      const int cp = chirp_probe(nd, 0);
      const PadJob rg = pj(Gacc, Gacc, hw, nd, cp, nd, 1, 0, nullptr, 0);
      const PadJob cg = pj(Gacc, Gacc, hw, nd, cp, nd, 1, 0, nullptr, 0);
      HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] { return launch_rows_pad(g, rg, st); }));
      HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] { return launch_cols_pad(g, cg, Fpart, st); }));
    } else {
      PropJobs rj{}, cj{};
      for (int j = 0; j < nd; ++j) {
        rj.job[rj.n++] = PropJob{Gacc + j * HW, Gacc + j * HW, nullptr, chirp_probe(nd, j), 1, 0};
        cj.job[cj.n++] = PropJob{Gacc + j * HW, Gacc + j * HW, nullptr, chirp_probe(nd, j), 1, 0};
      }
      HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] { return launch_rows_prop(g, rj, st); }));
      HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] { return launch_cols_prop(g, cj, Fpart, st); }));
    }
    HOLO_HIP(timed(P, HOLO_K_OTHER, st, [&] {
      return launch_sum_frames(Gacc, nd, with_ref ? Pref : nullptr, gq, HW, st);
    }));
  }
  if (want_F) {
    // the first ref_tiles slots hold the reference term's cost
    const size_t first = with_ref ? 0 : (size_t)ref_tiles;
    const size_t n = ref_tiles + (size_t)tiles * (k1 - k0) * nd - first;
    HOLO_HIP(timed(P, HOLO_K_OTHER, st, [&] {
      return launch_reduce_sum(Fpart + first, n, Fpart + P->n_fpart, F, st);
    }));
  }
  return HOLO_OK;
}

holo_status check_common(holo_plan* P, const holo_c64* u, const holo_c64* q, const char* fn) {
  if (!P) return fail(HOLO_ERR_INVALID_ARGUMENT, std::string(fn) + ": plan is NULL");
  if (!u || !q) return fail(HOLO_ERR_INVALID_ARGUMENT, std::string(fn) + ": u or q is NULL");
  return HOLO_OK;
}

}  // namespace

extern "C" holo_status holo_fwd(holo_plan* P, const holo_c64* u, const holo_c64* q, int32_t k0,
                                int32_t k1, holo_c64* v, void* ws, size_t ws_bytes, void* stream) {
  holo_status s = check_common(P, u, q, "holo_fwd");
  if (s != HOLO_OK) return s;
  if (!v) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_fwd: v is NULL");
  if (k0 < 0 || k1 > P->n_angles || k0 >= k1)
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_fwd: need 0 <= k0 < k1 <= n_angles");
  return run(P, kFwd, u, q, k0, k1, nullptr, v, nullptr, nullptr, nullptr, nullptr, nullptr, ws,
             ws_bytes, stream);
}

extern "C" holo_status holo_adj(holo_plan* P, const holo_c64* u, const holo_c64* q, int32_t k0,
                                int32_t k1, const holo_c64* w, holo_c64* g_u, holo_c64* g_q,
                                void* ws, size_t ws_bytes, void* stream) {
  holo_status s = check_common(P, u, q, "holo_adj");
  if (s != HOLO_OK) return s;
  if (!w) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_adj: w is NULL");
  if (k0 < 0 || k1 > P->n_angles || k0 >= k1)
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_adj: need 0 <= k0 < k1 <= n_angles");
  return run(P, kAdj, u, q, k0, k1, w, nullptr, nullptr, nullptr, nullptr, g_u, g_q, ws, ws_bytes,
             stream);
}

extern "C" holo_status holo_objective(holo_plan* P, const holo_c64* u, const holo_c64* q,
                                      const float* amp, const float* amp_ref, double* F, void* ws,
                                      size_t ws_bytes, void* stream) {
  holo_status s = check_common(P, u, q, "holo_objective");
  if (s != HOLO_OK) return s;
  if (!amp || !amp_ref || !F)
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_objective: amp, amp_ref or F is NULL");
  return run(P, kObj, u, q, 0, P->n_angles, nullptr, nullptr, amp, amp_ref, F, nullptr, nullptr, ws,
             ws_bytes, stream);
}

extern "C" holo_status holo_grad(holo_plan* P, const holo_c64* u, const holo_c64* q,
                                 const float* amp, const float* amp_ref, double* F, holo_c64* g_u,
                                 holo_c64* g_q, void* ws, size_t ws_bytes, void* stream) {
  holo_status s = check_common(P, u, q, "holo_grad");
  if (s != HOLO_OK) return s;
  if (!amp || !amp_ref) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_grad: amp or amp_ref is NULL");
  return run(P, kGrad, u, q, 0, P->n_angles, nullptr, nullptr, amp, amp_ref, F, g_u, g_q, ws,
             ws_bytes, stream);
}

extern "C" holo_status holo_grad_object(holo_plan* P, const holo_c64* u, const holo_c64* q,
                                        const float* amp, const float* amp_ref, double* F,
                                        holo_c64* g_u, void* ws, size_t ws_bytes, void* stream) {
  if (!g_u) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_grad_object: g_u is NULL");
  return holo_grad(P, u, q, amp, amp_ref, F, g_u, nullptr, ws, ws_bytes, stream);
}

extern "C" holo_status holo_grad_probe(holo_plan* P, const holo_c64* u, const holo_c64* q,
                                       const float* amp, const float* amp_ref, double* F,
                                       holo_c64* g_q, void* ws, size_t ws_bytes, void* stream) {
  if (!g_q) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_grad_probe: g_q is NULL");
  return holo_grad(P, u, q, amp, amp_ref, F, nullptr, g_q, ws, ws_bytes, stream);
}

// ---------------------------------------------------------------------------
// Solver: Dai-Yuan conjugate gradients and the initial probe
// ---------------------------------------------------------------------------

namespace {

struct CgLayout {
  size_t nu, nq;                       // complex elements of u and q
  size_t off_gu, off_gq, off_eu, off_eq, off_xu, off_xq, off_d, bytes;
};

CgLayout cg_layout(const holo_plan* P) {
  CgLayout L{};
  L.nu = (size_t)P->H * P->W * P->W;
  L.nq = (size_t)P->H * P->W;
  size_t o = P->ws_bytes;
  L.off_gu = o; o = align_up(o + L.nu * sizeof(float2));
  L.off_gq = o; o = align_up(o + L.nq * sizeof(float2));
  L.off_eu = o; o = align_up(o + L.nu * sizeof(float2));
  L.off_eq = o; o = align_up(o + L.nq * sizeof(float2));
  L.off_xu = o; o = align_up(o + L.nu * sizeof(float2));
  L.off_xq = o; o = align_up(o + L.nq * sizeof(float2));
  // doubles: F, three inner products, dot partials, reduction scratch
  L.off_d = o;  o = align_up(o + (4 + kDotParts + kReduceParts) * sizeof(double));
  L.bytes = o;
  return L;
}

}  // namespace

extern "C" holo_status holo_probe_init(holo_plan* P, const float* amp_ref, holo_c64* q_out,
                                       void* stream) {
  if (!P) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_probe_init: plan is NULL");
  if (!amp_ref || !q_out)
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_probe_init: amp_ref or q_out is NULL");
  if ((const void*)amp_ref == (const void*)q_out)
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_probe_init: q_out aliases amp_ref");
  holo_status ts = ensure_tables(P);
  if (ts != HOLO_OK) return ts;
  hipStream_t st = (hipStream_t)stream;
  const DevGeom g = make_geom(P);
  float2* q = (float2*)q_out;
  HOLO_HIP(timed(P, HOLO_K_PROBE, st,
                 [&] { return launch_real_to_c64(amp_ref, q, (size_t)P->H * P->W, st); }));
  // D_{-1}: the reference step with the conjugate transfer, rows then columns
  if (P->pad == 2) {
    PadJob jb{q, q, nullptr, (long long)P->H * P->W, 1, chirp_ref(P->nd), 1, 1, 0, 0};
    HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] { return launch_rows_pad(g, jb, st); }));
    HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] { return launch_cols_pad(g, jb, nullptr, st); }));
    return HOLO_OK;
  }
  PropJobs rj{}, cj{};
  rj.job[rj.n++] = PropJob{q, q, nullptr, chirp_ref(P->nd), 1, 0};
  cj.job[cj.n++] = PropJob{q, q, nullptr, chirp_ref(P->nd), 1, 0};
  HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] { return launch_rows_prop(g, rj, st); }));
  HOLO_HIP(timed(P, HOLO_K_PROBE, st, [&] { return launch_cols_prop(g, cj, nullptr, st); }));
  return HOLO_OK;
}

extern "C" holo_status holo_cg_workspace_bytes(const holo_plan* P, size_t* bytes) {
  if (!P || !bytes) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_cg_workspace_bytes: NULL argument");
  *bytes = cg_layout(P).bytes;
  return HOLO_OK;
}

extern "C" holo_status holo_cg(holo_plan* P, holo_c64* u_, holo_c64* q_, const float* amp,
                               const float* amp_ref, int32_t iters, double step0, double* F_hist,
                               double* steps, int32_t* halvings, void* ws, size_t ws_bytes,
                               void* stream) {
  holo_status s = check_common(P, u_, q_, "holo_cg");
  if (s != HOLO_OK) return s;
  if (!amp || !amp_ref) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_cg: amp or amp_ref is NULL");
  if (!F_hist) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_cg: F_hist is NULL");
  if (iters < 0) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_cg: iters must be >= 0");
  if (!(step0 > 0.0) || !std::isfinite(step0))
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_cg: step0 must be positive and finite");
  if (!ws) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_cg: workspace is NULL");
  const CgLayout L = cg_layout(P);
  if (ws_bytes < L.bytes)
    return fail(HOLO_ERR_WORKSPACE_TOO_SMALL, "holo_cg: workspace needs " +
                                                  std::to_string(L.bytes) + " bytes, got " +
                                                  std::to_string(ws_bytes));
  constexpr int kMaxHalvings = 30;
  hipStream_t st = (hipStream_t)stream;
  char* wsb = (char*)ws;
  float2* u = (float2*)u_;
  float2* q = (float2*)q_;
  float2* gu = (float2*)(wsb + L.off_gu);
  float2* gq = (float2*)(wsb + L.off_gq);
  float2* eu = (float2*)(wsb + L.off_eu);
  float2* eq = (float2*)(wsb + L.off_eq);
  float2* xu = (float2*)(wsb + L.off_xu);
  float2* xq = (float2*)(wsb + L.off_xq);
  double* dF = (double*)(wsb + L.off_d);
  double* ddot = dF + 1;
  double* dparts = dF + 4;
  double* dscratch = dparts + kDotParts;
  auto c64 = [](float2* p) { return (holo_c64*)p; };
  auto fetch = [&](const double* dev, double* host) -> holo_status {
    HOLO_HIP(hipMemcpyAsync(host, dev, sizeof(double), hipMemcpyDeviceToHost, st));
    HOLO_HIP(hipStreamSynchronize(st));
    return HOLO_OK;
  };
  auto dot = [&](const float2* a1, const float2* b1, const float2* a2, const float2* b2,
                 double* host) -> holo_status {
    HOLO_HIP(timed(P, HOLO_K_SOLVER, st, [&] {
      return launch_dot_re(a1, b1, L.nu, a2, b2, L.nq, dparts, dscratch, ddot, st);
    }));
    return fetch(ddot, host);
  };
#define HOLO_TRY(call)                      \
  do {                                      \
    holo_status s_ = (call);                \
    if (s_ != HOLO_OK) return s_;           \
  } while (0)

  double F = 0.0;
  HOLO_TRY(run(P, kGrad, c64(u), c64(q), 0, P->n_angles, nullptr, nullptr, amp, amp_ref, dF,
               c64(gu), c64(gq), ws, P->ws_bytes, stream));
  HOLO_TRY(fetch(dF, &F));
  F_hist[0] = F;
  auto direction = [&](float beta, int restart) -> holo_status {
    HOLO_HIP(timed(P, HOLO_K_SOLVER, st, [&] { return launch_cg_dir(gu, eu, beta, restart, L.nu, st); }));
    HOLO_HIP(timed(P, HOLO_K_SOLVER, st, [&] { return launch_cg_dir(gq, eq, beta, restart, L.nq, st); }));
    return HOLO_OK;
  };
  HOLO_TRY(direction(0.f, 1));
  double gamma_try = step0;
  for (int m = 0; m < iters; ++m) {
    double d_old = 0.0;   // <g_m, eta_m>, for the Dai-Yuan denominator
    HOLO_TRY(dot(gu, eu, gq, eq, &d_old));
    double t = gamma_try;
    int h = 0;
    bool accepted = false;
    for (; h <= kMaxHalvings; ++h, t *= 0.5) {
      const float tf = (float)t;
      HOLO_HIP(timed(P, HOLO_K_SOLVER, st, [&] { return launch_axpy(u, eu, tf, xu, L.nu, st); }));
      HOLO_HIP(timed(P, HOLO_K_SOLVER, st, [&] { return launch_axpy(q, eq, tf, xq, L.nq, st); }));
      double Ft = 0.0;
      HOLO_TRY(run(P, kObj, c64(xu), c64(xq), 0, P->n_angles, nullptr, nullptr, amp, amp_ref, dF,
                   nullptr, nullptr, ws, P->ws_bytes, stream));
      HOLO_TRY(fetch(dF, &Ft));
      if (Ft <= F) {
        accepted = true;
        break;
      }
    }
    if (!accepted) {   // x stays; the next iteration repeats the same search
      F_hist[m + 1] = F;
      if (steps) steps[m] = 0.0;
      if (halvings) halvings[m] = kMaxHalvings + 1;
      continue;
    }
    HOLO_HIP(timed(P, HOLO_K_SOLVER, st, [&] {
      return hipMemcpyAsync(u, xu, L.nu * sizeof(float2), hipMemcpyDeviceToDevice, st);
    }));
    HOLO_HIP(timed(P, HOLO_K_SOLVER, st, [&] {
      return hipMemcpyAsync(q, xq, L.nq * sizeof(float2), hipMemcpyDeviceToDevice, st);
    }));
    HOLO_TRY(run(P, kGrad, c64(u), c64(q), 0, P->n_angles, nullptr, nullptr, amp, amp_ref, dF,
                 c64(gu), c64(gq), ws, P->ws_bytes, stream));
    HOLO_TRY(fetch(dF, &F));
    double gg = 0.0, g_eta = 0.0;
    HOLO_TRY(dot(gu, gu, gq, gq, &gg));
    HOLO_TRY(dot(gu, eu, gq, eq, &g_eta));
    const double den = g_eta - d_old;
    const bool restart = !(den > 0.0);
    const double beta = restart ? 0.0 : gg / den;
    HOLO_TRY(direction((float)beta, restart ? 1 : 0));
    F_hist[m + 1] = F;
    if (steps) steps[m] = t;
    if (halvings) halvings[m] = h;
    gamma_try = 2.0 * t;
  }
#undef HOLO_TRY
  HOLO_HIP(hipStreamSynchronize(st));
  return HOLO_OK;
}

extern "C" holo_status holo_plan_set_probe_shifts(holo_plan* P, const float* shifts) {
  if (!P) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_set_probe_shifts: plan is NULL");
  const size_t n = (size_t)P->n_angles * P->nd * 2;
  if (shifts && P->pad == 2)
    return fail(HOLO_ERR_INVALID_ARGUMENT,
                "holo_plan_set_probe_shifts: padded propagation does not take probe shifts");
  if (shifts) {
    for (size_t i = 0; i < n; ++i)
      if (!std::isfinite(shifts[i]))
        return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_set_probe_shifts: shifts must be finite");
    P->pshift.assign(shifts, shifts + n);
  } else {
    P->pshift.clear();
  }
  P->pshift_dirty = true;
  layout_workspace(P);
  return HOLO_OK;
}

extern "C" holo_status holo_plan_set_chunk(holo_plan* P, int32_t chunk) {
  if (!P) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_set_chunk: plan is NULL");
  if (chunk < P->max_group)
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_set_chunk: chunk must be >= " +
                                               std::to_string(P->max_group) +
                                               " (the largest forward angle group)");
  P->chunk = std::min<int>(chunk, P->n_angles);
  layout_workspace(P);
  return HOLO_OK;
}

extern "C" holo_status holo_plan_get_chunk(const holo_plan* P, int32_t* chunk) {
  if (!P || !chunk) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_get_chunk: NULL argument");
  *chunk = P->chunk;
  return HOLO_OK;
}

// The launch-shape parameters the tile autotuner can choose.
static holo_status tile_check(const holo_plan* P, int param, int value, const char* fn) {
  switch (param) {
    case HOLO_TUNE_CHUNK:
      if (value < P->max_group)
        return fail(HOLO_ERR_INVALID_ARGUMENT, std::string(fn) + ": chunk " +
                                                   std::to_string(value) + " is below " +
                                                   std::to_string(P->max_group));
      return HOLO_OK;
    case HOLO_TUNE_COL_TILE:
      if (value != 0 && !col_tile_supported(P->H, value))
        return fail(HOLO_ERR_INVALID_ARGUMENT,
                    std::string(fn) + ": column tile must be 0, " +
                        std::to_string(cols_per_wg(P->H)) + " or " +
                        std::to_string(cols_per_wg(P->H) / 2));
      return HOLO_OK;
    case HOLO_TUNE_FS_SLAB:
      if (value != 1 && value != 2 && value != 4 && value != kFsSlab)
        return fail(HOLO_ERR_INVALID_ARGUMENT, std::string(fn) + ": slab must be 1, 2, 4 or 8");
      return HOLO_OK;
    case HOLO_TUNE_OVERLAP:
      if (value != 0 && value != 1)
        return fail(HOLO_ERR_INVALID_ARGUMENT, std::string(fn) + ": overlap must be 0 or 1");
      return HOLO_OK;
    case HOLO_TUNE_FWD_BINS: {
      if (value != kFwdNB && value != kFwdNB / 2)
        return fail(HOLO_ERR_INVALID_ARGUMENT, std::string(fn) + ": forward bins must be 8 or 16");
      // the chunk must still hold the largest angle group
      std::vector<int2> g;
      std::vector<int> go;
      int mg = 1;
      form_groups(const_cast<holo_plan*>(P), value, g, go, mg);
      if (P->chunk < mg)
        return fail(HOLO_ERR_INVALID_ARGUMENT, std::string(fn) + ": the chunk is smaller than "
                                                                 "an angle group of that size");
      return HOLO_OK;
    }
    default:
      return fail(HOLO_ERR_INVALID_ARGUMENT, std::string(fn) + ": unknown parameter");
  }
}

static int tile_get(const holo_plan* P, int param) {
  return param == HOLO_TUNE_CHUNK ? P->chunk
         : param == HOLO_TUNE_COL_TILE ? P->col_tile
         : param == HOLO_TUNE_FS_SLAB ? P->fs_slab
         : param == HOLO_TUNE_OVERLAP ? P->overlap : P->fwd_nb;
}

static void tile_put(holo_plan* P, int param, int value) {
  if (param == HOLO_TUNE_CHUNK) P->chunk = std::min<int>(value, P->n_angles);
  else if (param == HOLO_TUNE_COL_TILE) P->col_tile = value;
  else if (param == HOLO_TUNE_FS_SLAB) P->fs_slab = value;
  else if (param == HOLO_TUNE_OVERLAP) P->overlap = value;
  else if (value != P->fwd_nb) set_fwd_bins(P, value);
  layout_workspace(P);
}

extern "C" holo_status holo_plan_set_tile(holo_plan* P, int32_t param, int32_t value) {
  if (!P) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_set_tile: plan is NULL");
  holo_status s = tile_check(P, param, value, "holo_plan_set_tile");
  if (s != HOLO_OK) return s;
  tile_put(P, param, value);
  return HOLO_OK;
}

extern "C" holo_status holo_plan_get_tile(const holo_plan* P, int32_t param, int32_t* value) {
  if (!P || !value) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_get_tile: NULL argument");
  if (param < HOLO_TUNE_CHUNK || param > HOLO_TUNE_OVERLAP)
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_get_tile: unknown parameter");
  *value = tile_get(P, param);
  return HOLO_OK;
}

extern "C" holo_status holo_plan_autotune(holo_plan* P, const holo_c64* u, const holo_c64* q,
                                          const float* amp, const float* amp_ref, double* F,
                                          holo_c64* g_u, holo_c64* g_q, const int32_t* candidates,
                                          int32_t n_cand, void* ws, size_t ws_bytes,
                                          int32_t* best_chunk, float* times_ms, void* stream) {
  return holo_plan_autotune_tile(P, HOLO_TUNE_CHUNK, u, q, amp, amp_ref, F, g_u, g_q, candidates,
                                 n_cand, ws, ws_bytes, best_chunk, times_ms, stream);
}

extern "C" holo_status holo_plan_autotune_tile(holo_plan* P, int32_t param, const holo_c64* u,
                                               const holo_c64* q, const float* amp,
                                               const float* amp_ref, double* F, holo_c64* g_u,
                                               holo_c64* g_q, const int32_t* candidates,
                                               int32_t n_cand, void* ws, size_t ws_bytes,
                                               int32_t* best_chunk, float* times_ms,
                                               void* stream) {
  holo_status s = check_common(P, u, q, "holo_plan_autotune");
  if (s != HOLO_OK) return s;
  if (!amp || !amp_ref || !F || !g_u || !g_q || !candidates || !best_chunk || !ws)
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_autotune: NULL argument");
  if (n_cand < 1) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_autotune: no candidates");
  if (param < HOLO_TUNE_CHUNK || param > HOLO_TUNE_OVERLAP)
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_autotune: unknown parameter");
  const int chunk0 = tile_get(P, param);
  size_t need = 0;
  for (int i = 0; i < n_cand; ++i) {
    s = tile_check(P, param, candidates[i], "holo_plan_autotune");
    if (s != HOLO_OK) {
      tile_put(P, param, chunk0);
      return s;
    }
    tile_put(P, param, candidates[i]);
    need = std::max(need, P->ws_bytes);
  }
  tile_put(P, param, chunk0);
  if (ws_bytes < need)
    return fail(HOLO_ERR_WORKSPACE_TOO_SMALL, "holo_plan_autotune: workspace needs " +
                                                  std::to_string(need) + " bytes, got " +
                                                  std::to_string(ws_bytes));
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HOLO_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(HOLO_ERR_HIP, "holo_plan_autotune: hipEventCreate failed");
  }
  auto grad = [&]() {
    return run(P, kGrad, u, q, 0, P->n_angles, nullptr, nullptr, amp, amp_ref, F, g_u, g_q, ws,
               ws_bytes, stream);
  };
  // One untimed gradient first (device tables, code load), then one timed
  // gradient per candidate; the fastest becomes the plan's value.
  int best = chunk0;
  float best_ms = 0.f;
  s = grad();
  for (int i = 0; i < n_cand && s == HOLO_OK; ++i) {
    tile_put(P, param, candidates[i]);
    float ms = 0.f;
    if (hipEventRecord(e0, st) != hipSuccess) { s = fail(HOLO_ERR_HIP, "hipEventRecord"); break; }
    s = grad();
    if (s != HOLO_OK) break;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      s = fail(HOLO_ERR_HIP, "holo_plan_autotune: event timing failed");
      break;
    }
    if (times_ms) times_ms[i] = ms;
    if (i == 0 || ms < best_ms) {
      best_ms = ms;
      best = tile_get(P, param);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  tile_put(P, param, s == HOLO_OK ? best : chunk0);
  if (s == HOLO_OK) *best_chunk = best;
  return s;
}

extern "C" holo_status holo_plan_ray_groups(const holo_plan* P, int32_t* first, int32_t* count,
                                            int32_t capacity, int32_t* n_groups) {
  if (!P || !n_groups)
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_ray_groups: plan or n_groups is NULL");
  *n_groups = (int32_t)P->groups.size();
  if (capacity > 0 && (!first || !count))
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_ray_groups: first or count is NULL");
  const int n = std::min<int>(capacity, (int)P->groups.size());
  for (int i = 0; i < n; ++i) {
    first[i] = P->groups[i].x;
    count[i] = P->groups[i].y;
  }
  return HOLO_OK;
}

extern "C" holo_status holo_plan_set_projector(holo_plan* P, int32_t projector) {
  if (!P) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_set_projector: plan is NULL");
  if (projector != HOLO_PROJECTOR_JOSEPH && projector != HOLO_PROJECTOR_FOURIER)
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_set_projector: unknown projector");
  if (projector == HOLO_PROJECTOR_FOURIER && P->fs_dinv.empty())
    return fail(HOLO_ERR_UNSUPPORTED_SIZE,
                "holo_plan_set_projector: the Fourier-slice projector needs det_cols <= 1024");
  P->projector = projector;
  layout_workspace(P);
  return HOLO_OK;
}

extern "C" holo_status holo_plan_set_padding(holo_plan* P, int32_t pad) {
  if (!P) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_set_padding: plan is NULL");
  if (pad != 1 && pad != 2)
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_set_padding: pad must be 1 or 2");
  if (pad == 2 && P->chirp2W.empty())
    return fail(HOLO_ERR_UNSUPPORTED_SIZE,
                "holo_plan_set_padding: padded propagation needs det_rows and det_cols <= 1024");
  if (pad == 2 && !P->pshift.empty())
    return fail(HOLO_ERR_INVALID_ARGUMENT,
                "holo_plan_set_padding: padded propagation does not take probe shifts");
  P->pad = pad;
  return HOLO_OK;
}

extern "C" holo_status holo_plan_set_functional(holo_plan* P, int32_t functional) {
  if (!P) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_set_functional: plan is NULL");
  if (functional != HOLO_FUNCTIONAL_AMPLITUDE && functional != HOLO_FUNCTIONAL_INTENSITY &&
      functional != HOLO_FUNCTIONAL_CONVENTIONAL)
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_plan_set_functional: unknown functional");
  P->functional = functional;
  return HOLO_OK;
}

extern "C" holo_status holo_timing_enable(holo_plan* P, int32_t on) {
  if (!P) return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_timing_enable: plan is NULL");
  if (on) {
    holo_status s = drain_events(P);
    if (s != HOLO_OK) return s;
    for (int c = 0; c < HOLO_K_COUNT; ++c) {
      P->t_ms[c] = 0.0;
      P->t_n[c] = 0;
    }
  }
  P->timing = on != 0;
  return HOLO_OK;
}

extern "C" holo_status holo_timing_read(holo_plan* P, int32_t cls, double* total_ms,
                                        int64_t* launches) {
  if (!P || !total_ms || !launches)
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_timing_read: NULL argument");
  if (cls < 0 || cls >= HOLO_K_COUNT)
    return fail(HOLO_ERR_INVALID_ARGUMENT, "holo_timing_read: kernel class out of range");
  holo_status s = drain_events(P);
  if (s != HOLO_OK) return s;
  *total_ms = P->t_ms[cls];
  *launches = P->t_n[cls];
  return HOLO_OK;
}
