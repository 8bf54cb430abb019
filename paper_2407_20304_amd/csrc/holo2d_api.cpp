// Host runtime and C ABI of the batched single-angle retrievals
// (holo2d_* in include/holo.h).
#include "../../include/holo.h"
#include "holo2d_internal.hpp"
#include "holo_internal.hpp"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace holo;

namespace holo {
holo_status set_last_error(holo_status st, const std::string& msg);
}

namespace {

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct ItemList {
  std::vector<B2Item> items;
  size_t off = 0;   // byte offset in the device table buffer
};

}  // namespace

struct holo2d_plan {
  int n_inst = 0, nd = 0;
  int functional = 0;                     // holo_functional
  double m0 = 0, fresnel0 = 0;
  std::vector<double> mag;
  std::vector<int> sizes;
  std::vector<long long> off;
  long long total = 0;
  std::vector<int> dsizes;                // distinct sizes
  std::vector<std::vector<float2>> tw, chirp;
  std::vector<std::vector<B2AdjTap>> adj;  // per distinct size: [nd][n]
  ItemList rows_probe, rows_probe_noref, rows_nd, rows_cgq, cols_probe, cols_probe_noref,
      cols_nd, cols_gq, gather;
  std::vector<int2> ranges;               // per-instance cost-partial slots
  int n_slots = 0;
  // device tables
  size_t off_inst = 0, off_ranges = 0, table_bytes = 0;
  std::vector<size_t> off_tw, off_chirp, off_adj;
  void* d_tables = nullptr;
  int device = -1;
  // workspace (bytes)
  size_t ws_Q = 0, ws_P = 0, ws_X = 0, ws_G = 0, ws_F = 0, ws_bytes = 0;
  // table image of holo2d_grad_noalloc, built for the static array's address
  std::vector<char> noalloc_image;
  const void* noalloc_base = nullptr;
};

static holo_status fail2(holo_status s, const std::string& m) { return holo::set_last_error(s, m); }

// Transposed demagnification taps of one axis of an n-point frame for
// magnification m (Eq. 8's resampling B_j, bilinear, free space outside):
// the forward samples destination d at c + m (d - c) from the two pixels
// around it, so source pixel idx receives weight from the destinations
// whose sample lies within one pixel of it -- at most two adjacent ones,
// as m >= 1, among the three candidates around (idx - c) / m + c.  The
// arithmetic is the forward's (the sample position as one fused
// multiply-add), so each weight is the forward's own.
static B2AdjTap adj_tap(double c, double m, int idx, int n) {
  const int d0 = (int)std::floor(((double)idx - c) / m + c) - 1;
  int d[3];
  float w[3];
  for (int e = 0; e < 3; ++e) {
    const int dd = d0 + e;
    const double sp = std::fma(m, (double)dd - c, c);
    const double fl = std::floor(sp);
    const int i0 = (int)fl;
    const float f = (float)(sp - fl);
    const float wt = i0 == idx ? 1.0f - f : (i0 + 1 == idx ? f : 0.0f);
    const bool ok = dd >= 0 && dd < n;
    d[e] = ok ? dd : 0;
    w[e] = ok ? wt : 0.0f;
  }
  const int e0 = w[0] != 0.0f ? 0 : 1;
  return {d[e0], d[e0 + 1], w[e0], w[e0 + 1]};
}

static void chirp_rows(std::vector<float2>& out, int n, const std::vector<double>& rhos,
                       double nf) {
  out.resize(rhos.size() * (size_t)n);
  for (size_t r = 0; r < rhos.size(); ++r)
    for (int i = 0; i < n; ++i) {
      const double k = (2 * i < n) ? i : i - n;
      double turns = -0.5 * rhos[r] * k * k / (nf * (double)n * (double)n);
      turns -= std::floor(turns);
      const double ph = 2.0 * M_PI * turns;
      out[r * n + i] = make_float2((float)(std::cos(ph) / n), (float)(std::sin(ph) / n));
    }
}

extern "C" holo_status holo2d_plan_create(int32_t n_inst, const int32_t* sizes, int32_t n_dist,
                                          const double* mag_rel, double m0, double fresnel0,
                                          holo2d_plan** out) {
  if (!out) return fail2(HOLO_ERR_INVALID_ARGUMENT, "holo2d_plan_create: out is NULL");
  *out = nullptr;
  if (n_inst < 1 || !sizes) return fail2(HOLO_ERR_INVALID_ARGUMENT, "need n_inst >= 1 and sizes");
  if (n_dist < 1 || n_dist > 8 || !mag_rel)
    return fail2(HOLO_ERR_INVALID_ARGUMENT, "n_dist must be in 1..8 with mag_rel given");
  if (!(std::isfinite(m0) && m0 > 1.0)) return fail2(HOLO_ERR_INVALID_ARGUMENT, "m0 must be > 1");
  if (!(std::isfinite(fresnel0) && fresnel0 > 0.0))
    return fail2(HOLO_ERR_INVALID_ARGUMENT, "fresnel0 must be > 0");
  for (int j = 0; j < n_dist; ++j)
    if (!(std::isfinite(mag_rel[j]) && mag_rel[j] >= 1.0))
      return fail2(HOLO_ERR_INVALID_ARGUMENT, "mag_rel[j] must be finite and >= 1");
  for (int i = 0; i < n_inst; ++i)
    if (!b2_size_supported(sizes[i]))
      return fail2(HOLO_ERR_UNSUPPORTED_SIZE,
                   "instance sizes must be one of 64,128,192,256,384,512,1024 (got " +
                       std::to_string(sizes[i]) + ")");
  holo2d_plan* P = new (std::nothrow) holo2d_plan();
  if (!P) return fail2(HOLO_ERR_OUT_OF_HOST_MEMORY, "out of host memory");
  try {
    P->n_inst = n_inst;
    P->nd = n_dist;
    P->m0 = m0;
    P->fresnel0 = fresnel0;
    P->mag.assign(mag_rel, mag_rel + n_dist);
    P->sizes.assign(sizes, sizes + n_inst);
    P->off.resize(n_inst);
    for (int i = 0; i < n_inst; ++i) {
      P->off[i] = P->total;
      P->total += (long long)sizes[i] * sizes[i];
    }
    P->dsizes = P->sizes;
    std::sort(P->dsizes.begin(), P->dsizes.end());
    P->dsizes.erase(std::unique(P->dsizes.begin(), P->dsizes.end()), P->dsizes.end());
    std::vector<double> rhos(2 * n_dist + 1);
    for (int j = 0; j < n_dist; ++j) {
      const double m = P->mag[j];
      rhos[j] = (m0 - m) / (m * (m0 - 1.0));
      rhos[n_dist + j] = m0 * (m - 1.0) / (m * (m0 - 1.0));
    }
    rhos[2 * n_dist] = 1.0;
    for (int n : P->dsizes) {
      std::vector<float2> t(n);
      for (int m = 0; m < n; ++m) {
        const double ph = -2.0 * M_PI * (double)m / (double)n;
        t[m] = make_float2((float)std::cos(ph), (float)std::sin(ph));
      }
      P->tw.push_back(t);
      std::vector<float2> c;
      chirp_rows(c, n, rhos, fresnel0);
      P->chirp.push_back(c);
      std::vector<B2AdjTap> a((size_t)n_dist * n);
      for (int j = 0; j < n_dist; ++j)
        for (int idx = 0; idx < n; ++idx) a[(size_t)j * n + idx] = adj_tap(n / 2.0, P->mag[j], idx, n);
      P->adj.push_back(a);
    }
    // work items, largest instances first
    std::vector<int> order(n_inst);
    for (int i = 0; i < n_inst; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return P->sizes[a] > P->sizes[b]; });
    P->ranges.assign(n_inst, make_int2(0, 0));
    std::vector<int> slot_base(n_inst);
    int slots = 0;
    for (int i = 0; i < n_inst; ++i) {
      const int n = P->sizes[i];
      const int per = n / b2_cols_per_wg(n);
      slot_base[i] = slots;
      P->ranges[i] = make_int2(slots, slots + per * (n_dist + 1));
      slots += per * (n_dist + 1);
    }
    P->n_slots = slots;
    for (int i : order) {
      const int n = P->sizes[i];
      const int lpw = b2_rows_per_wg(n), tc = b2_cols_per_wg(n);
      // job n_dist of the probe and pass-C rows is the reference term
      for (int j = 0; j <= n_dist; ++j)
        for (int z = 0; z < n; z += lpw) {
          P->rows_probe.items.push_back({i, j, z, 0});
          P->rows_cgq.items.push_back({i, j, z, 0});
          if (j < n_dist) {
            P->rows_probe_noref.items.push_back({i, j, z, 0});
            P->rows_nd.items.push_back({i, j, z, 0});
          }
        }
      for (int j = 0; j <= n_dist; ++j)
        for (int s = 0; s < n; s += tc) {
          // cost slots: plane j's column tiles, then the reference's
          const int slot = slot_base[i] + (j < n_dist ? j : n_dist) * (n / tc) + s / tc;
          P->cols_probe.items.push_back({i, j, s, slot});
          if (j < n_dist) {
            P->cols_probe_noref.items.push_back({i, j, s, 0});
            P->cols_nd.items.push_back({i, j, s, slot});
          }
        }
      for (int s = 0; s < n; s += b2_gq_per_wg(n)) P->cols_gq.items.push_back({i, 0, s, 0});
      for (int p = 0; p < n * n; p += 256) P->gather.items.push_back({i, 0, p, 0});
    }
    // device table layout
    size_t t = 0;
    for (size_t d = 0; d < P->dsizes.size(); ++d) {
      P->off_tw.push_back(t);
      t = al(t + P->tw[d].size() * sizeof(float2));
      P->off_chirp.push_back(t);
      t = al(t + P->chirp[d].size() * sizeof(float2));
      P->off_adj.push_back(t);
      t = al(t + P->adj[d].size() * sizeof(B2AdjTap));
    }
    P->off_inst = t;
    t = al(t + sizeof(B2Inst) * n_inst);
    for (ItemList* L : {&P->rows_probe, &P->rows_probe_noref, &P->rows_nd, &P->rows_cgq,
                        &P->cols_probe, &P->cols_probe_noref, &P->cols_nd, &P->cols_gq,
                        &P->gather}) {
      L->off = t;
      t = al(t + sizeof(B2Item) * L->items.size());
    }
    P->off_ranges = t;
    t = al(t + sizeof(int2) * n_inst);
    P->table_bytes = t;
    // workspace
    const size_t fr = (size_t)P->total * sizeof(float2);
    size_t w = 0;
    P->ws_Q = w; w = al(w + fr * n_dist);
    P->ws_P = w; w = al(w + fr);
    P->ws_X = w; w = al(w + fr * n_dist);
    P->ws_G = w; w = al(w + fr * n_dist);
    P->ws_F = w; w = al(w + sizeof(double) * (size_t)slots);
    P->ws_bytes = w;
  } catch (const std::bad_alloc&) {
    delete P;
    return fail2(HOLO_ERR_OUT_OF_HOST_MEMORY, "out of host memory");
  }
  *out = P;
  return HOLO_OK;
}

extern "C" holo_status holo2d_plan_set_functional(holo2d_plan* P, int32_t functional) {
  if (!P) return fail2(HOLO_ERR_INVALID_ARGUMENT, "holo2d_plan_set_functional: NULL plan");
  if (functional != HOLO_FUNCTIONAL_AMPLITUDE && functional != HOLO_FUNCTIONAL_INTENSITY &&
      functional != HOLO_FUNCTIONAL_CONVENTIONAL)
    return fail2(HOLO_ERR_INVALID_ARGUMENT,
                 "holo2d_plan_set_functional: functional must be 0 (amplitude), 1 (intensity) or "
                 "2 (conventional)");
  P->functional = functional;
  return HOLO_OK;
}

extern "C" holo_status holo2d_plan_destroy(holo2d_plan* P) {
  if (!P) return HOLO_OK;
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

extern "C" holo_status holo2d_offsets(const holo2d_plan* P, int64_t* offsets, int64_t* total) {
  if (!P || !offsets || !total) return fail2(HOLO_ERR_INVALID_ARGUMENT, "holo2d_offsets: NULL argument");
  for (int i = 0; i < P->n_inst; ++i) offsets[i] = P->off[i];
  *total = P->total;
  return HOLO_OK;
}

extern "C" holo_status holo2d_workspace_bytes(const holo2d_plan* P, size_t* bytes) {
  if (!P || !bytes) return fail2(HOLO_ERR_INVALID_ARGUMENT, "holo2d_workspace_bytes: NULL argument");
  *bytes = P->ws_bytes;
  return HOLO_OK;
}

namespace {

#define B2_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) return fail2(HOLO_ERR_HIP, std::string(#call) + ": " + \
                                                         hipGetErrorString(e_)); \
  } while (0)

// The device image of a plan's constant tables (twiddles, transfer rows,
// instance descriptors, work items, cost-slot ranges) for tables placed at
// device address `base`: the instance descriptors hold pointers into it.
void b2_table_image(const holo2d_plan* P, const char* base, std::vector<char>& h) {
  h.assign(P->table_bytes, 0);
  for (size_t d = 0; d < P->dsizes.size(); ++d) {
    std::copy((const char*)P->tw[d].data(), (const char*)(P->tw[d].data() + P->tw[d].size()),
              h.data() + P->off_tw[d]);
    std::copy((const char*)P->chirp[d].data(),
              (const char*)(P->chirp[d].data() + P->chirp[d].size()), h.data() + P->off_chirp[d]);
    std::copy((const char*)P->adj[d].data(), (const char*)(P->adj[d].data() + P->adj[d].size()),
              h.data() + P->off_adj[d]);
  }
  std::vector<B2Inst> inst(P->n_inst);
  for (int i = 0; i < P->n_inst; ++i) {
    const size_t k = std::lower_bound(P->dsizes.begin(), P->dsizes.end(), P->sizes[i]) -
                     P->dsizes.begin();
    inst[i].n = P->sizes[i];
    inst[i].off = P->off[i];
    inst[i].tw = (const float2*)(base + P->off_tw[k]);
    inst[i].chirp = (const float2*)(base + P->off_chirp[k]);
    inst[i].adj = (const B2AdjTap*)(base + P->off_adj[k]);
  }
  std::copy((const char*)inst.data(), (const char*)(inst.data() + inst.size()),
            h.data() + P->off_inst);
  for (const ItemList* L : {&P->rows_probe, &P->rows_probe_noref, &P->rows_nd, &P->rows_cgq,
                            &P->cols_probe, &P->cols_probe_noref, &P->cols_nd, &P->cols_gq,
                            &P->gather})
    std::copy((const char*)L->items.data(), (const char*)(L->items.data() + L->items.size()),
              h.data() + L->off);
  std::copy((const char*)P->ranges.data(), (const char*)(P->ranges.data() + P->ranges.size()),
            h.data() + P->off_ranges);
}

holo_status b2_tables(holo2d_plan* P) {
  int dev = -1;
  B2_HIP(hipGetDevice(&dev));
  if (P->d_tables) {
    if (dev != P->device)
      return fail2(HOLO_ERR_INVALID_ARGUMENT, "plan tables live on another device");
    return HOLO_OK;
  }
  void* d = nullptr;
  B2_HIP(hipMalloc(&d, P->table_bytes));
  std::vector<char> h;
  b2_table_image(P, (const char*)d, h);
  hipError_t e = hipMemcpy(d, h.data(), P->table_bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return fail2(HOLO_ERR_HIP, std::string("uploading batch tables: ") + hipGetErrorString(e));
  }
  P->d_tables = d;
  P->device = dev;
  return HOLO_OK;
}

enum B2Run { kB2Fwd, kB2Obj, kB2Grad };

// Enqueue the passes of one call.  `tb` holds the plan's device tables (as
// laid out by b2_table_image for that address), `w` the workspace.
holo_status b2_launch(holo2d_plan* P, B2Run run, const char* tb, char* w, const holo_c64* psi,
                      const holo_c64* q, const float* amp, const float* amp_ref,
                      holo_c64* v_out, double* F, holo_c64* g_psi, holo_c64* g_q,
                      hipStream_t st) {
  auto items = [&](const ItemList& L) { return (const B2Item*)(tb + L.off); };
  // The conventional functional: the model with q = 1 and no reference
  // term (amplitude residual); F does not depend on q, so g_q = 0.
  const bool conv = P->functional == HOLO_FUNCTIONAL_CONVENTIONAL;
  B2Args A{};
  A.nd = P->nd;
  A.functional = P->functional == HOLO_FUNCTIONAL_INTENSITY ? 1 : 0;
  A.max_n = P->dsizes.back();
  for (int j = 0; j < P->nd; ++j) A.mag[j] = P->mag[j];
  A.inst = (const B2Inst*)(tb + P->off_inst);
  A.psi = (const float2*)psi;
  A.q = (const float2*)q;
  A.amp_ref = amp_ref;
  A.Q = (float2*)(w + P->ws_Q);
  A.P = (float2*)(w + P->ws_P);
  A.X = run == kB2Fwd ? (float2*)v_out : (float2*)(w + P->ws_X);
  A.G = (float2*)(w + P->ws_G);
  A.Fpart = (double*)(w + P->ws_F);
  const bool want_ref = run != kB2Fwd && !conv;
  const bool grad = run == kB2Grad && (g_psi || g_q);
  const bool want_gq = grad && g_q && !conv;
  A.want_ref = want_ref ? 1 : 0;
  A.want_grad = grad ? 1 : 0;
  A.want_gq = want_gq ? 1 : 0;
  A.g_psi = grad ? (float2*)g_psi : nullptr;
  A.g_q = want_gq ? (float2*)g_q : nullptr;

  // probe stage
  if (conv) {
    B2_HIP(launch_fill(A.Q, (size_t)P->total * P->nd, make_float2(1.f, 0.f), st));
    // the reference's cost slots stay zero (a double 0 is all-zero bits)
    if (run != kB2Fwd) B2_HIP(launch_fill_zero((float2*)A.Fpart, (size_t)P->n_slots, st));
    if (grad && g_q) B2_HIP(launch_fill_zero((float2*)g_q, (size_t)P->total, st));
  } else {
    A.mode = kB2RowsProbe;
    const ItemList& rp = want_ref ? P->rows_probe : P->rows_probe_noref;
    B2_HIP(launch_b2_rows(A, items(rp), (int)rp.items.size(), st));
    A.mode = kB2ColsProbe;
    const ItemList& cp = want_ref ? P->cols_probe : P->cols_probe_noref;
    B2_HIP(launch_b2_cols(A, items(cp), (int)cp.items.size(), st));
  }
  // pass A and pass B
  A.mode = kB2RowsA;
  B2_HIP(launch_b2_rows(A, items(P->rows_nd), (int)P->rows_nd.items.size(), st));
  A.amp = run == kB2Fwd ? nullptr : amp;
  A.mode = kB2ColsB;
  B2_HIP(launch_b2_cols(A, items(P->cols_nd), (int)P->cols_nd.items.size(), st));
  if (grad) {
    // pass C (with the probe gradient's rows and the reference rows when
    // g_q is wanted), then g_q per column tile and g_psi by the gather
    A.mode = want_gq ? kB2RowsCGq : kB2RowsC;
    const ItemList& rc = want_gq ? P->rows_cgq : P->rows_nd;
    B2_HIP(launch_b2_rows(A, items(rc), (int)rc.items.size(), st));
    if (want_gq) {
      A.mode = kB2ColsGqSum;
      B2_HIP(launch_b2_gq_sum(A, items(P->cols_gq), (int)P->cols_gq.items.size(), st));
    }
    if (g_psi) B2_HIP(launch_b2_gather(A, items(P->gather), (int)P->gather.items.size(), st));
  }
  if (F && run != kB2Fwd)
    B2_HIP(launch_b2_reduce(A.Fpart, (const int2*)(tb + P->off_ranges), P->n_inst, F, st));
  return HOLO_OK;
}

holo_status b2_run(holo2d_plan* P, B2Run run, const holo_c64* psi, const holo_c64* q,
                   const float* amp, const float* amp_ref, holo_c64* v_out, double* F,
                   holo_c64* g_psi, holo_c64* g_q, void* ws, size_t ws_bytes, void* stream) {
  if (!psi || !q) return fail2(HOLO_ERR_INVALID_ARGUMENT, "psi or q is NULL");
  if (!ws) return fail2(HOLO_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (ws_bytes < P->ws_bytes)
    return fail2(HOLO_ERR_WORKSPACE_TOO_SMALL, "workspace needs " + std::to_string(P->ws_bytes) +
                                                   " bytes, got " + std::to_string(ws_bytes));
  holo_status ts = b2_tables(P);
  if (ts != HOLO_OK) return ts;
  return b2_launch(P, run, (const char*)P->d_tables, (char*)ws, psi, q, amp, amp_ref, v_out, F,
                   g_psi, g_q, (hipStream_t)stream);
}

}  // namespace

extern "C" holo_status holo2d_fwd(holo2d_plan* P, const holo_c64* psi, const holo_c64* q,
                                  holo_c64* v, void* ws, size_t ws_bytes, void* stream) {
  if (!P || !v) return fail2(HOLO_ERR_INVALID_ARGUMENT, "holo2d_fwd: plan or v is NULL");
  return b2_run(P, kB2Fwd, psi, q, nullptr, nullptr, v, nullptr, nullptr, nullptr, ws, ws_bytes,
                stream);
}

extern "C" holo_status holo2d_objective(holo2d_plan* P, const holo_c64* psi, const holo_c64* q,
                                        const float* amp, const float* amp_ref, double* F,
                                        void* ws, size_t ws_bytes, void* stream) {
  if (!P || !amp || !amp_ref || !F)
    return fail2(HOLO_ERR_INVALID_ARGUMENT, "holo2d_objective: NULL argument");
  return b2_run(P, kB2Obj, psi, q, amp, amp_ref, nullptr, F, nullptr, nullptr, ws, ws_bytes,
                stream);
}

extern "C" holo_status holo2d_grad(holo2d_plan* P, const holo_c64* psi, const holo_c64* q,
                                   const float* amp, const float* amp_ref, double* F,
                                   holo_c64* g_psi, holo_c64* g_q, void* ws, size_t ws_bytes,
                                   void* stream) {
  if (!P || !amp || !amp_ref) return fail2(HOLO_ERR_INVALID_ARGUMENT, "holo2d_grad: NULL argument");
  return b2_run(P, kB2Grad, psi, q, amp, amp_ref, nullptr, F, g_psi, g_q, ws, ws_bytes, stream);
}

// ---------------------------------------------------------------------------
// holo2d_grad without allocation: the plan's tables and the workspace live in
// one static device array per GPU.
// ---------------------------------------------------------------------------

// Each GPU holds its own copy from the library's load until the process
// ends.  Host code never uses this name as an address: the device address of
// the current GPU's copy comes from hipGetSymbolAddress (scratch_address).
static __device__ __align__(256) unsigned char scratch[HOLO2D_SCRATCH_MAX_BYTES];

namespace {

constexpr size_t kScratchBytes = size_t(HOLO2D_SCRATCH_MAX_BYTES);
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

holo_status scratch_address(void** out) {
  int dev = -1;
  B2_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail2(HOLO_ERR_INVALID_ARGUMENT, "holo2d_grad_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail2(HOLO_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                     hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HOLO_OK;
}

}  // namespace

extern "C" holo_status holo2d_noalloc_bytes(const holo2d_plan* P, size_t* bytes) {
  if (!P || !bytes) return fail2(HOLO_ERR_INVALID_ARGUMENT, "holo2d_noalloc_bytes: NULL argument");
  *bytes = al(P->table_bytes) + P->ws_bytes;
  return HOLO_OK;
}

extern "C" holo_status holo2d_grad_noalloc(holo2d_plan* P, const holo_c64* psi, const holo_c64* q,
                                           const float* amp, const float* amp_ref, double* F,
                                           holo_c64* g_psi, holo_c64* g_q, void* stream) {
  if (!P || !psi || !q || !amp || !amp_ref)
    return fail2(HOLO_ERR_INVALID_ARGUMENT, "holo2d_grad_noalloc: NULL argument");
  const size_t need = al(P->table_bytes) + P->ws_bytes;
  if (need > kScratchBytes)
    return fail2(HOLO_ERR_WORKSPACE_TOO_SMALL,
                 "holo2d_grad_noalloc: the plan needs " + std::to_string(need) +
                     " bytes of scratch, the static array holds " + std::to_string(kScratchBytes) +
                     " (use holo2d_grad with a caller workspace)");
  void* base = nullptr;
  holo_status s = scratch_address(&base);
  if (s != HOLO_OK) return s;
  char* tb = (char*)base;
  // Tables first: every call rewrites them (another plan's call may have
  // left its own there), ordered on the stream before this call's kernels.
  if (P->noalloc_base != base) {
    b2_table_image(P, tb, P->noalloc_image);
    P->noalloc_base = base;
  }
  hipStream_t st = (hipStream_t)stream;
  B2_HIP(hipMemcpyAsync(tb, P->noalloc_image.data(), P->table_bytes, hipMemcpyHostToDevice, st));
  return b2_launch(P, kB2Grad, tb, tb + al(P->table_bytes), psi, q, amp, amp_ref, nullptr, F,
                   g_psi, g_q, st);
}
