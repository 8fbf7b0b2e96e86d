// Host runtime and C ABI of the hybrid weight-window sweep library (see
// include/hww.h for the contract of every entry point).  The runtime owns no
// device memory: it carves the caller's workspace into banks, queues, tally
// sets and solver scratch, and queues kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hww.h"
#include "hww_internal.h"

using namespace hww;

namespace {

constexpr double kSegSlack = 2.0;   // segment capacity / fair share of a work-group
constexpr double kOvfShare = 0.5;   // overflow capacity / fair share of a region
constexpr int kBlock = 512;         // threads per sweep work-group (default; see hww_autotune)
constexpr int kTile = 256;          // particles a wave claims per tile (default)
constexpr int64_t kUnitParticles = 8192;  // start particles per batched work unit and launch
constexpr int kGridMax = 1024;      // work-groups of a batched launch at most
// Replicas of a batch fall in LDS classes by what one sweep unit's histogram
// needs: at most a quarter of a compute unit's LDS (class 0, four work-groups
// of 256 threads per compute unit by default), at most half (class 1, two of
// 512), more (class 2, one of 1024, which may also keep the cell records in
// LDS).  Each class is a persistent launch of its own, so small replicas are
// not held to one work-group per compute unit by the largest one.
constexpr int kBatchClasses = 3;

int batch_class(size_t hist_lds) {
  return hist_lds <= kLdsBytes / 4 ? 0 : (hist_lds <= kLdsBytes / 2 ? 1 : 2);
}

struct Layout {
  int64_t total = 0;
  BankGeom geom{};
  bool cells_lds = false;  // the sweep keeps the per-cell records in LDS
  int64_t dcap = 0;
  int64_t off_edges, off_sigt, off_sigs, off_cells, off_win, off_cfis;
  // Comb scratch (comb = 1): n_hist histories, slots census slots.
  int64_t n_hist = 0, comb_slots = 0, off_c_cnt = 0, off_c_cur = 0, off_c_order = 0, off_c_wq = 0, off_c_blk = 0,
          off_c_misc = 0;
  int64_t off_bank[2], off_segcnt[2], off_ovfcnt[2], off_q;
  int64_t off_tal[2], off_tsum[2], off_bnd[2], off_tracks, off_counters, off_wstart, off_wnext;
  int64_t off_err, off_status, off_scratch, off_factor, off_phi_out, off_J_out;
  int64_t off_F_out, off_P_out;
  int64_t off_m_sig, off_m_F, off_m_P, off_m_phi0, off_m_J0, off_m_w, off_m_hist, off_m_fac, off_m_fact, off_m_G,
      off_m_g, off_m_dw;
};

int64_t align_up(int64_t v) { return (v + 255) & ~int64_t(255); }

struct Carver {
  int64_t cur = 0;
  int64_t take(int64_t bytes) {
    const int64_t o = cur;
    cur = align_up(cur + bytes);
    return o;
  }
};

bool real_bytes(int precision, int64_t *rb) {
  if (precision == HWW_FP64) { *rb = 8; return true; }
  if (precision == HWW_FP32) { *rb = 4; return true; }
  return false;
}

// Launch shape of one problem.  The grid is B * K persistent work-groups.
// When the per-cell records fit in LDS beside the histogram, one work-group
// of 1024 threads per compute unit of a 256-CU MI355X keeps them there (no
// dependent global load per flight); otherwise two of 512 threads per
// compute unit when the histogram allows it, else one.
int segments_per_batch(int I, int B, int nc, int precision, bool *cells_lds) {
  const size_t cb = precision == HWW_FP32 ? lds_cell_bytes<float>() : lds_cell_bytes<double>();
  int target;
  if (sweep_lds_bytes(I, nc, 64, cb) <= kLdsBytes) {
    *cells_lds = true;
    target = 256;
  } else {
    *cells_lds = false;
    target = sweep_lds_bytes(I, nc, 64) <= kLdsBytes / 2 ? 512 : 256;
  }
  int K = (target + B / 2) / B;
  if (K < 1) K = 1;
  if (K > 64) K = 64;
  return K;
}

// Segments per batch of a replica of a batched problem: about
// kUnitParticles start particles per unit and launch.
int member_segments(const hww_problem &p) {
  const int64_t per = (int64_t)p.n_batches * p.n_chunks * kUnitParticles;
  int64_t K = (p.n_src + per - 1) / per;
  if (K < 1) K = 1;
  if (K > 64) K = 64;
  return (int)K;
}

// Workspace layout of one problem.  A replica of a batch (member = true)
// has no daughter buffers (the batch's are shared) and no march arrays.
void make_layout(const hww_problem &p, Layout *L, bool member = false) {
  const int64_t I = p.n_cells, B = p.n_batches, nc = p.n_chunks, R = B * nc;
  int64_t rb = 8;
  real_bytes(p.precision, &rb);
  bool cells_lds = false;
  const int K = member ? member_segments(p) : segments_per_batch((int)I, (int)B, (int)nc, p.precision, &cells_lds);
  L->cells_lds = cells_lds;
  BankGeom &G = L->geom;
  G.K = K;
  const double share = (double)p.bank_capacity / (double)R;
  G.seg_cap = (int64_t)std::ceil(kSegSlack * share / K) + 64;
  G.ovf_cap = (int64_t)std::ceil(kOvfShare * share) + 1024;
  G.stride = (int64_t)K * G.seg_cap + G.ovf_cap;
  // Daughter slots per work-group buffer: its share of the bank, four times
  // that for combed (supercritical) problems, whose windows split whole
  // generations at the wave front.
  L->dcap = std::max<int64_t>(4096, (p.comb ? 4 : 1) * ((p.bank_capacity + B * K - 1) / (B * K)));
  const int64_t slots = R * G.stride;
  const int64_t dslots = member ? 0 : 2 * B * K * L->dcap;
  Carver c;
  L->off_edges = c.take(8 * (I + 1));
  L->off_sigt = c.take(8 * I);
  L->off_sigs = c.take(8 * I);
  L->off_cells = c.take(4 * rb * I);
  L->off_win = c.take(sizeof(Window) * I);
  L->off_cfis = c.take(p.sigma_f ? 8 * I : 0);
  for (int k = 0; k < 2; ++k) {
    L->off_bank[k] = c.take(0);
    // (x, mu), w, lin, (src, e, cell) streams
    c.take(2 * rb * slots);
    c.take(8 * slots);
    c.take(8 * slots);
    c.take(sizeof(Tag) * slots);
    L->off_segcnt[k] = c.take(4 * R * K);
    L->off_ovfcnt[k] = c.take(4 * R);
  }
  L->off_q = c.take(0);
  c.take(2 * rb * dslots);
  c.take(sizeof(WTau) * dslots);
  c.take(8 * dslots);
  c.take(sizeof(Tag) * dslots);
  for (int k = 0; k < 2; ++k) {
    L->off_tal[k] = c.take(8 * B * I * 6);
    L->off_tsum[k] = c.take(8 * kSumCopies * 6 * I);
    L->off_bnd[k] = c.take(8 * B * 6);
  }
  L->off_tracks = c.take(8 * I);
  L->off_counters = c.take(8 * 2 * C_NCOUNTERS);
  L->off_wstart = c.take(8 * nc);
  L->off_wnext = c.take(8 * nc);
  L->off_err = c.take(4);
  L->off_status = c.take(4);
  L->off_scratch = c.take(8 * 24 * (I + 4));
  L->off_factor = c.take(8 * 4 * (2 * I + 3));
  L->off_phi_out = c.take(8 * (I + 2));
  L->off_J_out = c.take(8 * (I + 1));
  L->off_F_out = c.take(8 * (I + 2));
  L->off_P_out = c.take(8 * 2);
  // Deterministic march of up to n_steps steps and its adjoint.
  const int64_t N1 = member ? 0 : (int64_t)p.n_steps + 1, n = member ? 0 : 2 * I + 3;
  L->off_m_sig = c.take(8 * 2 * I);
  L->off_m_F = c.take(8 * N1 * (I + 2));
  L->off_m_P = c.take(8 * N1 * 2);
  L->off_m_phi0 = c.take(8 * (I + 2));
  L->off_m_J0 = c.take(8 * (I + 1));
  L->off_m_w = c.take(8 * N1 * (I + 2));
  L->off_m_hist = c.take(8 * N1 * n);
  L->off_m_fac = c.take(8 * 3 * n);
  L->off_m_fact = c.take(8 * 3 * n);
  L->off_m_G = c.take(8);
  L->off_m_g = c.take(8 * 2 * I);
  L->off_m_dw = c.take(8 * N1 * (I + 2));
  if (p.comb && !member) {
    L->n_hist = std::max<int64_t>(p.n_src, p.bank_capacity);
    L->comb_slots = slots;
    L->off_c_cnt = c.take(8 * (L->n_hist + 1));
    L->off_c_cur = c.take(4 * L->n_hist);
    L->off_c_order = c.take(8 * slots);
    L->off_c_wq = c.take(8 * slots);
    L->off_c_blk = c.take(8 * comb_scan_blocks(std::max<int64_t>(L->n_hist + 1, slots)));
    L->off_c_misc = c.take(8 * 8);
  }
  L->total = c.cur;
}

template <typename Real>
Bank<Real> bank_view(char *ws, int64_t off, int64_t off_seg, int64_t off_ovf, int64_t slots) {
  Bank<Real> b;
  int64_t o = off;
  auto take = [&](int64_t bytes) {
    char *p = ws + o;
    o = align_up(o + bytes);
    return p;
  };
  b.xm = reinterpret_cast<XMu<Real> *>(take(sizeof(XMu<Real>) * slots));
  b.w = reinterpret_cast<double *>(take(8 * slots));
  b.lin = reinterpret_cast<uint64_t *>(take(8 * slots));
  b.tag = reinterpret_cast<Tag *>(take(sizeof(Tag) * slots));
  b.segcnt = reinterpret_cast<uint32_t *>(ws + off_seg);
  b.ovfcnt = reinterpret_cast<uint32_t *>(ws + off_ovf);
  return b;
}

template <typename Real>
Queue<Real> queue_view(char *ws, int64_t off, int64_t slots) {
  Queue<Real> q;
  int64_t o = off;
  auto take = [&](int64_t bytes) {
    char *p = ws + o;
    o = align_up(o + bytes);
    return p;
  };
  q.xm = reinterpret_cast<XMu<Real> *>(take(sizeof(XMu<Real>) * slots));
  q.wt = reinterpret_cast<WTau *>(take(sizeof(WTau) * slots));
  q.lin = reinterpret_cast<uint64_t *>(take(8 * slots));
  q.tag = reinterpret_cast<Tag *>(take(sizeof(Tag) * slots));
  return q;
}

std::string g_init_error;

}  // namespace

// Fixed device workspace of hww_init_problem_static, for callers that cannot
// allocate device memory.  Every GPU the library runs on holds one copy of
// it until the process ends.  Host code never passes this name to a kernel
// or a copy: it stands in for the array on the host only.  The device
// address of each GPU's copy comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[HWW_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
char *g_static_ptr[kMaxDevices];   // device address of each GPU's `scratch` (null until looked up)
bool g_static_busy[kMaxDevices];   // a live handle works in that GPU's copy

// Device address of the current device's copy of the static workspace.
// Looked up once per device, with that device current.  Caller holds
// g_static_mu.
int static_workspace(int dev, char **ptr, std::string *why) {
  if (!g_static_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return HWW_E_DEVICE;
    }
    g_static_ptr[dev] = static_cast<char *>(p);
  }
  *ptr = g_static_ptr[dev];
  return HWW_OK;
}

// Launch shapes the tuner measured, kept for the life of the process: a
// later problem of the same kind takes its shape without measuring.  The
// key is the device, the flight precision, fission, the chunk and batch
// counts, work-groups per batch and the LDS placement of the cell records
// (single problems), or the LDS class and the replica count (batches), and
// the power-of-two buckets of the cell count and the start particles.
struct TuneKey {
  int dev, fp32, fission, batch, cls, nc, B, K, cells, cells_bucket, particles_bucket, replicas;
  bool operator==(const TuneKey &o) const { return std::memcmp(this, &o, sizeof(TuneKey)) == 0; }
};
struct TuneShape {
  int block, tile, grid;
  float ms;
};
std::mutex g_tune_mu;
std::vector<std::pair<TuneKey, TuneShape>> g_tune_cache;

int log2_bucket(int64_t v) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < v) ++b;
  return b;
}

bool tune_lookup(const TuneKey &k, TuneShape *out) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (const auto &e : g_tune_cache)
    if (e.first == k) {
      *out = e.second;
      return true;
    }
  return false;
}

void tune_store(const TuneKey &k, const TuneShape &v) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (auto &e : g_tune_cache)
    if (e.first == k) {
      e.second = v;
      return;
    }
  g_tune_cache.emplace_back(k, v);
}

}  // namespace

struct hww_handle {
  hww_problem p{};
  int I = 0, B = 0, nc = 0, R = 0, K = 1;
  Layout L;
  hipStream_t stream = nullptr;
  char *ws = nullptr;
  double *edges, *sig_t, *sig_s;
  Window *win;
  int fp32 = 0;
  // Particle streams in the flight precision of the problem (one set used).
  Bank<double> bank[2];
  Queue<double> dq;
  CellData<double> *cells;
  Bank<float> bank32[2];
  Queue<float> dq32;
  CellData<float> *cells32;
  double *tal[2], *tsum[2], *bnd[2];
  unsigned long long *tracks, *counters;
  double *wstart, *wnext;
  uint32_t *err;
  int32_t *status;
  double *scratch, *factor, *phi_out, *J_out;
  double *cfis = nullptr;  // (sigma_s + sigma_f) / sigma_t, fission problems only
  int64_t src_bound = 0;   // history ids of the start and census banks are below this
  double nu_f = 0.0;
  int track_moments = 3;   // track-length moments scored per segment

  int start_bank = 0;  // census bank = 1 - start_bank
  int cur_tal = 0;
  int step = 0, next_chunk = 0;
  int ww_on = 0;
  int fatal = 0;
  double factor_theta = -1.0;  // theta of the LU factors in the workspace
  // Writes into each tally set (sweeps, clears) and the set and count whose
  // batch sums of the initial condition the LOSM scratch holds.
  uint64_t tal_epoch[2] = {0, 0};
  int ic_buf = -1;
  uint64_t ic_epoch = 0;
  size_t lds = 0;
  int block = kBlock, tile = kTile;  // sweep launch shape of a single problem (batches: per LDS class)
  bool cells_lds = false;      // the sweep keeps the per-cell records in LDS
  int is_view = 0;             // a replica of a batch, for reads only
  int static_dev = -1;        // device whose static workspace the handle uses (-1: caller's)
  // Batch of replicas (is_batch): the replicas are handles of their own
  // whose small per-replica arrays live in shared arrays of the batch.
  int is_batch = 0;
  std::vector<hww_handle *> rep;
  int max_I = 0, max_K = 0, cus = 256;
  uint32_t n_units = 0;
  // LDS classes of a batch: unit range, launch LDS, cell placement and shape.
  struct BatchClass {
    uint32_t u0 = 0, u1 = 0;
    size_t lds = 0;
    int cells_mode = 0, block = 1024, tile = kTile, grid = 0;
    int64_t starts = 0;  // start particles of its replicas
    int n_rep = 0, max_cells = 0;
  };
  BatchClass bcls[kBatchClasses];
  void *desc = nullptr;              // ReplicaDesc<Real>[n]
  uint32_t *units = nullptr, *work = nullptr;
  LosmReplica *losm_tab = nullptr;
  BeginStepArgs *bs_tab = nullptr;   // [2][n]
  double *phi_cat = nullptr, *J_cat = nullptr;
  unsigned long long *counters_all = nullptr;
  uint32_t *segcnt_all[2] = {nullptr, nullptr}, *ovfcnt_all[2] = {nullptr, nullptr};
  int64_t n_seg_all = 0, n_ovf_all = 0, n_phi_all = 0, n_J_all = 0;
  int64_t bdcap = 0;                 // daughter slots per buffer of a batched launch
  Queue<double> bq;
  Queue<float> bq32;
  int losm_wil = 0;
  int n_launch = 0;            // sweep launches of the current step
  int timing = 1;              // record HIP events around every sweep launch
  int64_t launch_count = 0;    // sweep launches since init (timed or not)
  int step_ev0 = 0;            // first event pair of the current step
  std::vector<hipEvent_t> ev;  // start/stop pairs of every sweep launch since init
  std::vector<double> dx_host;  // cell widths (normalised tally reads)
  MarchArgs march{};           // last deterministic march (its state stays in the workspace)
  int march_ok = 0;
  int ev_used = 0;             // pairs recorded
  int ev_summed = 0;           // pairs already added into ms_summed
  double ms_summed = 0.0;
  std::string msg;
};

namespace {

int fail(hww_handle *h, int code, const std::string &m) {
  if (h) h->msg = m;
  else g_init_error = m;
  return code;
}

int check_hip(hww_handle *h, hipError_t e, const char *what) {
  if (e == hipSuccess) return HWW_OK;
  return fail(h, HWW_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(h, expr)                                \
  do {                                                 \
    int rc__ = check_hip((h), (expr), #expr);          \
    if (rc__ != HWW_OK) return rc__;                   \
  } while (0)

int validate(const hww_problem *p, std::string *why) {
  if (!p) { *why = "problem is NULL"; return HWW_E_INVALID_ARG; }
  if (p->n_cells < 1 || !p->edges || !p->sigma_t || !p->sigma_s) { *why = "bad mesh or cross sections"; return HWW_E_INVALID_ARG; }
  if (!(p->speed > 0.0) || !(p->dt > 0.0) || p->n_steps < 1) { *why = "speed, dt and n_steps must be positive"; return HWW_E_INVALID_ARG; }
  if (p->n_src < 0 || p->n_src > 0xFFFFFFFFll) { *why = "n_src out of range"; return HWW_E_INVALID_ARG; }
  if (p->bank_capacity < p->n_src || p->bank_capacity < 1 || p->bank_capacity > (int64_t)1 << 34) { *why = "bank_capacity out of range"; return HWW_E_INVALID_ARG; }
  if (p->n_batches < 1 || p->n_batches > 64) { *why = "n_batches must be 1..64"; return HWW_E_INVALID_ARG; }
  if (p->n_chunks < 1 || p->n_chunks > 8) { *why = "n_chunks must be 1..8"; return HWW_E_INVALID_ARG; }
  if (p->replica >= (1u << 28)) { *why = "replica must be < 2^28"; return HWW_E_INVALID_ARG; }
  int64_t rb;
  if (!real_bytes(p->precision, &rb)) { *why = "unsupported precision"; return HWW_E_INVALID_ARG; }
  for (int i = 0; i < p->n_cells; ++i) {
    if (!(p->edges[i + 1] > p->edges[i])) { *why = "edges must ascend"; return HWW_E_INVALID_ARG; }
    if (!(p->sigma_t[i] > 0.0) || !(p->sigma_s[i] >= 0.0) || p->sigma_s[i] > p->sigma_t[i] ||
        !std::isfinite(p->sigma_t[i])) { *why = "need 0 < sigma_t, 0 <= sigma_s <= sigma_t"; return HWW_E_INVALID_ARG; }
    if (p->sigma_f && (!(p->sigma_f[i] >= 0.0) || p->sigma_s[i] + p->sigma_f[i] > p->sigma_t[i])) {
      *why = "need 0 <= sigma_f, sigma_s + sigma_f <= sigma_t"; return HWW_E_INVALID_ARG;
    }
  }
  if (p->sigma_f && (!(p->nu_f >= 0.0) || !(p->nu_f < 1.0e6))) { *why = "nu_f must be in [0, 1e6)"; return HWW_E_INVALID_ARG; }
  if (p->comb < 0 || p->comb > 2) { *why = "comb must be 0, 1 or 2"; return HWW_E_INVALID_ARG; }
  if (p->track_moments < 0 || p->track_moments > 3) { *why = "track_moments must be 0..3"; return HWW_E_INVALID_ARG; }
  if (!(p->src_x >= p->edges[0] && p->src_x <= p->edges[p->n_cells])) { *why = "src_x outside the mesh"; return HWW_E_INVALID_ARG; }
  if (sweep_lds_bytes(p->n_cells, p->n_chunks, 64) > 160 * 1024) { *why = "too many cells for the LDS histogram (I <= 3136 with 2..8 chunks, 3137 with 1)"; return HWW_E_INVALID_ARG; }
  return HWW_OK;
}

// Census-bank occupancy from the device counts (synchronises).
int census_total(hww_handle *h, int bank_idx, uint64_t *total) {
  std::vector<uint32_t> seg((size_t)h->R * h->K), ovf(h->R);
  HIPCHK(h, hipMemcpyAsync(seg.data(), h->bank[bank_idx].segcnt, 4 * seg.size(), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(ovf.data(), h->bank[bank_idx].ovfcnt, 4 * ovf.size(), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  uint64_t t = 0;
  for (uint32_t c : seg) t += std::min<uint64_t>(c, (uint64_t)h->L.geom.seg_cap);
  for (uint32_t c : ovf) t += std::min<uint64_t>(c, (uint64_t)h->L.geom.ovf_cap);
  *total = t;
  return HWW_OK;
}

// Read the device error word and the census occupancy; map them to an ABI
// code.  Errors are sticky: the problem must be re-initialised.
int poll_batch(hww_handle *h);

int error_status(hww_handle *h, uint32_t e, uint64_t cen);

int poll_errors(hww_handle *h) {
  if (h->is_batch) return poll_batch(h);
  uint32_t e = 0;
  HIPCHK(h, hipMemcpyAsync(&e, h->err, 4, hipMemcpyDeviceToHost, h->stream));
  uint64_t cen = 0;
  int rc = census_total(h, 1 - h->start_bank, &cen);
  if (rc != HWW_OK) return rc;
  return error_status(h, e, cen);
}

// The ABI code of an error word read from the device and a census size.
int error_status(hww_handle *h, uint32_t e, uint64_t cen) {
  if (e & (ERR_CAPACITY | ERR_SPLIT | ERR_GENERATIONS | ERR_DAUGHTERS)) {
    h->fatal = HWW_E_CAPACITY;
    return fail(h, HWW_E_CAPACITY, (e & ERR_SPLIT) ? "a split exceeded 1e9 daughters"
                                   : (e & ERR_GENERATIONS) ? "too many daughter generations"
                                   : (e & ERR_DAUGHTERS) ? "a work-group's daughter buffer overflowed"
                                                         : "bank segment overflow");
  }
  if (cen > (uint64_t)h->p.bank_capacity) {
    h->fatal = HWW_E_CAPACITY;
    return fail(h, HWW_E_CAPACITY, "census bank exceeds bank_capacity");
  }
  if (e & ERR_NUMERIC) {
    h->fatal = HWW_E_NUMERIC;
    return fail(h, HWW_E_NUMERIC, "non-finite or non-positive window, or zero pivot in the LOSM solve");
  }
  if (e & ERR_COMB_WEIGHT) {
    h->fatal = HWW_E_NUMERIC;
    return fail(h, HWW_E_NUMERIC, "a census combed without waiting had a weight that was not positive and finite");
  }
  return HWW_OK;
}

template <typename Real>
SweepArgs<Real> base_args(hww_handle *h) {
  SweepArgs<Real> a{};
  a.I = h->I; a.B = h->B; a.nc = h->nc;
  a.v = h->p.speed; a.inv_v = 1.0 / h->p.speed; a.dt = h->p.dt;
  a.seed = h->p.seed; a.key1 = h->p.replica << 4;
  a.win = h->win;
  a.cfis = h->cfis;
  a.nu_f = h->nu_f;
  a.track_moments = h->track_moments;
  a.ww_on = h->ww_on;
  a.geom = h->L.geom;
  if constexpr (sizeof(Real) == 8) {
    a.cells = h->cells;
    a.in_bank = h->bank[h->start_bank];
    a.census = h->bank[1 - h->start_bank];
    a.dq = h->dq;
  } else {
    a.cells = h->cells32;
    a.in_bank = h->bank32[h->start_bank];
    a.census = h->bank32[1 - h->start_bank];
    a.dq = h->dq32;
  }
  a.dcap = h->L.dcap;
  a.tal = h->tal[h->cur_tal];
  a.tsum = h->tsum[h->cur_tal];
  a.bnd = h->bnd[h->cur_tal];
  a.tracks = h->tracks;
  a.counters = h->counters;
  a.wnext = h->wnext;
  a.err = h->err;
  return a;
}

// The persistent launch of LDS class ci of a batch for one chunk.
template <typename Real>
int launch_class(hww_handle *h, int ci, int chunk, int k) {
  const hww_handle::BatchClass &c = h->bcls[ci];
  if (c.u1 == c.u0) return HWW_OK;
  BatchSweepArgs<Real> a{};
  a.desc = reinterpret_cast<const ReplicaDesc<Real> *>(h->desc);
  a.units = h->units + c.u0;
  a.n_units = c.u1 - c.u0;
  a.work = h->work + 2 * ci;
  a.par = k & 1;
  a.start_bank = h->start_bank;
  a.chunk = chunk;
  a.ww_on = h->ww_on;
  a.tile = c.tile;
  if constexpr (sizeof(Real) == 8) a.dq = h->bq;
  else a.dq = h->bq32;
  a.dcap = h->bdcap;
  a.err = h->err;
  HIPCHK(h, launch_sweep_batch<Real>(a, c.cells_mode, c.grid, c.block, c.lds, h->stream));
  return HWW_OK;
}

template <typename Real>
int launch_chunk(hww_handle *h, int chunk, int k) {
  if (h->is_batch) {
    ++h->tal_epoch[h->cur_tal];
    for (int ci = 0; ci < kBatchClasses; ++ci) {
      const int rc = launch_class<Real>(h, ci, chunk, k);
      if (rc != HWW_OK) return rc;
    }
    return HWW_OK;
  }
  SweepArgs<Real> a = base_args<Real>(h);
  a.chunk = chunk;
  a.tile = h->tile;
  ++h->tal_epoch[h->cur_tal];
  HIPCHK(h, launch_sweep<Real>(a, h->cells_lds, h->B * h->K, h->block, h->lds, h->stream));
  return HWW_OK;
}

int zero_counts(hww_handle *h, int k) {
  HIPCHK(h, launch_fill_u32(h->bank[k].segcnt, 0u, (int64_t)h->R * h->K, h->stream));
  HIPCHK(h, launch_fill_u32(h->bank[k].ovfcnt, 0u, h->R, h->stream));
  return HWW_OK;
}

// Point the handle's arrays into its part of the workspace.
void carve_handle(hww_handle *h, const hww_problem &problem, char *ws, const Layout &L, hipStream_t stream) {
  h->p = problem;
  h->dx_host.resize(problem.n_cells);
  for (int i = 0; i < problem.n_cells; ++i) h->dx_host[i] = problem.edges[i + 1] - problem.edges[i];
  h->p.edges = h->p.sigma_t = h->p.sigma_s = h->p.sigma_f = nullptr;
  h->cfis = problem.sigma_f ? reinterpret_cast<double *>(ws + L.off_cfis) : nullptr;
  h->nu_f = problem.sigma_f ? problem.nu_f : 0.0;
  h->src_bound = problem.n_src;
  h->track_moments = problem.track_moments == 0 ? 3 : problem.track_moments;
  h->I = problem.n_cells;
  h->B = problem.n_batches;
  h->nc = problem.n_chunks;
  h->R = h->B * h->nc;
  h->L = L;
  h->K = L.geom.K;
  h->cells_lds = L.cells_lds;
  const size_t cb = problem.precision == HWW_FP32 ? lds_cell_bytes<float>() : lds_cell_bytes<double>();
  h->lds = sweep_lds_bytes(h->I, h->nc, h->K, h->cells_lds ? cb : 0);
  h->block = h->cells_lds ? 1024 : kBlock;
  h->stream = stream;
  h->ws = ws;
  const int64_t slots = (int64_t)h->R * L.geom.stride;
  h->edges = reinterpret_cast<double *>(ws + L.off_edges);
  h->sig_t = reinterpret_cast<double *>(ws + L.off_sigt);
  h->sig_s = reinterpret_cast<double *>(ws + L.off_sigs);
  h->cells = reinterpret_cast<CellData<double> *>(ws + L.off_cells);
  h->win = reinterpret_cast<Window *>(ws + L.off_win);
  for (int k = 0; k < 2; ++k) {
    h->bank[k] = bank_view<double>(ws, L.off_bank[k], L.off_segcnt[k], L.off_ovfcnt[k], slots);
    h->bank32[k] = bank_view<float>(ws, L.off_bank[k], L.off_segcnt[k], L.off_ovfcnt[k], slots);
    h->tal[k] = reinterpret_cast<double *>(ws + L.off_tal[k]);
    h->tsum[k] = reinterpret_cast<double *>(ws + L.off_tsum[k]);
    h->bnd[k] = reinterpret_cast<double *>(ws + L.off_bnd[k]);
  }
  h->fp32 = problem.precision == HWW_FP32;
  h->dq = queue_view<double>(ws, L.off_q, 2 * (int64_t)h->B * h->K * L.dcap);
  h->dq32 = queue_view<float>(ws, L.off_q, 2 * (int64_t)h->B * h->K * L.dcap);
  h->cells32 = reinterpret_cast<CellData<float> *>(ws + L.off_cells);
  h->tracks = reinterpret_cast<unsigned long long *>(ws + L.off_tracks);
  h->counters = reinterpret_cast<unsigned long long *>(ws + L.off_counters);
  h->wstart = reinterpret_cast<double *>(ws + L.off_wstart);
  h->wnext = reinterpret_cast<double *>(ws + L.off_wnext);
  h->err = reinterpret_cast<uint32_t *>(ws + L.off_err);
  h->status = reinterpret_cast<int32_t *>(ws + L.off_status);
  h->scratch = reinterpret_cast<double *>(ws + L.off_scratch);
  h->factor = reinterpret_cast<double *>(ws + L.off_factor);
  h->phi_out = reinterpret_cast<double *>(ws + L.off_phi_out);
  h->J_out = reinterpret_cast<double *>(ws + L.off_J_out);
}

// Upload the mesh, clear every accumulator and build the source bank at t^0
// (the census bank of step 0, bank 1; its tallies fill set 0).  Queues work
// only; the caller polls.
int prime_handle(hww_handle *h, const hww_problem &problem) {
  const int I = h->I;
  std::vector<CellData<double>> cd(I);
  std::vector<CellData<float>> cf(I);
  for (int i = 0; i < I; ++i) {
    cd[i].xl = problem.edges[i];
    cd[i].xr = problem.edges[i + 1];
    cd[i].inv_sig = 1.0 / problem.sigma_t[i];
    cd[i].c = problem.sigma_s[i] / problem.sigma_t[i];
    cf[i].xl = (float)cd[i].xl;
    cf[i].xr = (float)cd[i].xr;
    cf[i].inv_sig = (float)cd[i].inv_sig;
    cf[i].c = (float)cd[i].c;
  }
  HIPCHK(h, hipMemcpyAsync(h->edges, problem.edges, 8 * (I + 1), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(h->sig_t, problem.sigma_t, 8 * I, hipMemcpyHostToDevice, h->stream));
  // The low-order balance takes sigma_s + nu_f sigma_f (Eq. balance); a
  // collision below (sigma_s + sigma_f) / sigma_t and above the scattering
  // ratio is a fission.
  std::vector<double> sig_lo(problem.sigma_s, problem.sigma_s + I), cfis_h;
  if (problem.sigma_f) {
    cfis_h.resize(I);
    for (int i = 0; i < I; ++i) {
      sig_lo[i] = problem.sigma_s[i] + problem.nu_f * problem.sigma_f[i];
      cfis_h[i] = (problem.sigma_s[i] + problem.sigma_f[i]) / problem.sigma_t[i];
    }
    HIPCHK(h, hipMemcpyAsync(h->cfis, cfis_h.data(), 8 * I, hipMemcpyHostToDevice, h->stream));
  }
  HIPCHK(h, hipMemcpyAsync(h->sig_s, sig_lo.data(), 8 * I, hipMemcpyHostToDevice, h->stream));
  if (h->fp32)
    HIPCHK(h, hipMemcpyAsync(h->cells32, cf.data(), sizeof(CellData<float>) * I, hipMemcpyHostToDevice, h->stream));
  else
    HIPCHK(h, hipMemcpyAsync(h->cells, cd.data(), sizeof(CellData<double>) * I, hipMemcpyHostToDevice, h->stream));
  for (int k = 0; k < 2; ++k) {
    if (zero_counts(h, k) != HWW_OK) return HWW_E_DEVICE;
    HIPCHK(h, launch_fill_f64(h->tal[k], 0.0, (int64_t)h->B * I * 6, h->stream));
    HIPCHK(h, launch_fill_f64(h->tsum[k], 0.0, (int64_t)kSumCopies * 6 * I, h->stream));
    HIPCHK(h, launch_fill_f64(h->bnd[k], 0.0, (int64_t)h->B * 6, h->stream));
  }
  HIPCHK(h, launch_fill_u32(reinterpret_cast<uint32_t *>(h->tracks), 0u, 2 * (int64_t)I, h->stream));
  HIPCHK(h, launch_fill_u32(reinterpret_cast<uint32_t *>(h->counters), 0u, 4 * C_NCOUNTERS, h->stream));
  HIPCHK(h, launch_fill_f64(h->wstart, 0.0, h->nc, h->stream));
  HIPCHK(h, launch_fill_f64(h->wnext, 0.0, h->nc, h->stream));
  HIPCHK(h, launch_fill_f64(reinterpret_cast<double *>(h->win), 0.0, 4 * (int64_t)I, h->stream));
  HIPCHK(h, launch_fill_u32(h->err, 0u, 1, h->stream));
  HIPCHK(h, launch_fill_u32(reinterpret_cast<uint32_t *>(h->status), 0u, 1, h->stream));
  h->start_bank = 0;
  h->cur_tal = 0;
  h->ic_buf = -1;
  SourceArgs sa{};
  sa.I = I; sa.B = h->B; sa.nc = h->nc;
  sa.v = problem.speed; sa.dt = problem.dt; sa.src_x = problem.src_x;
  sa.n_src = problem.n_src; sa.seed = problem.seed; sa.key1 = problem.replica << 4;
  sa.edges = h->edges; sa.geom = h->L.geom;
  sa.tal = h->tal[0]; sa.tsum = h->tsum[0]; sa.wnext = h->wnext; sa.err = h->err;
  if (h->fp32)
    HIPCHK(h, launch_source<float>(sa, h->bank32[1], h->B * h->K, 256, h->lds, h->stream));
  else
    HIPCHK(h, launch_source<double>(sa, h->bank[1], h->B * h->K, 256, h->lds, h->stream));
  h->step = 0;
  h->next_chunk = h->nc;
  return HWW_OK;
}

void destroy_events(hww_handle *h) {
  for (auto &e : h->ev)
    if (e) (void)hipEventDestroy(e);
  h->ev.clear();
}

// ---------------------------------------------------------------- batches --
// Workspace of a batch: shared arrays first (replica and unit tables, the
// replicas' counters, segment counts and solve outputs side by side
// so that one copy reads them all, the daughter buffers of the persistent
// grid), then one member layout per replica.
struct BatchLayout {
  int64_t total = 0;
  std::vector<Layout> L;
  std::vector<int64_t> base;
  std::vector<uint32_t> units;
  int64_t off_desc, off_units, off_work, off_err, off_counters, off_seg[2], off_ovf[2], off_phi, off_J,
      off_losm, off_bs, off_q;
  int64_t n_seg = 0, n_ovf = 0, n_phi = 0, n_J = 0, dcap = 0;
  int max_I = 0, max_K = 0;
  std::vector<int> cls;                // LDS class of each replica
  uint32_t cls_u0[kBatchClasses] = {}, cls_u1[kBatchClasses] = {};  // unit range of each class
};

int make_batch_layout(const hww_problem *probs, int n, BatchLayout *BL, std::string *why) {
  if (!probs || n < 1 || n > 65535) { *why = "need 1..65535 problems"; return HWW_E_INVALID_ARG; }
  for (int r = 0; r < n; ++r) {
    const int rc = validate(&probs[r], why);
    if (rc != HWW_OK) { *why = "replica " + std::to_string(r) + ": " + *why; return rc; }
    if (probs[r].sigma_f || probs[r].comb) {
      *why = "replica " + std::to_string(r) + ": fission and combing need a single problem";
      return HWW_E_INVALID_ARG;
    }
    if (probs[r].precision != probs[0].precision || probs[r].n_chunks != probs[0].n_chunks ||
        probs[r].n_steps != probs[0].n_steps) {
      *why = "replicas must share precision, n_chunks and n_steps";
      return HWW_E_INVALID_ARG;
    }
  }
  const int nc = probs[0].n_chunks;
  BL->L.resize(n);
  std::vector<int> order(n);
  for (int r = 0; r < n; ++r) {
    make_layout(probs[r], &BL->L[r], true);
    order[r] = r;
    const Layout &L = BL->L[r];
    BL->max_I = std::max(BL->max_I, probs[r].n_cells);
    BL->max_K = std::max(BL->max_K, L.geom.K);
    const int64_t R = (int64_t)probs[r].n_batches * nc;
    BL->n_seg += R * L.geom.K;
    BL->n_ovf += R;
    BL->n_phi += probs[r].n_cells + 2;
    BL->n_J += probs[r].n_cells + 1;
    BL->dcap = std::max(BL->dcap, (probs[r].bank_capacity + (int64_t)probs[r].n_batches * L.geom.K - 1) /
                                      ((int64_t)probs[r].n_batches * L.geom.K));
  }
  BL->dcap = std::max<int64_t>(BL->dcap, 4096);
  if (sweep_lds_bytes(BL->max_I, nc, BL->max_K) > 160 * 1024) { *why = "too many cells for the LDS histogram"; return HWW_E_INVALID_ARG; }
  // Units: by LDS class, in a class the biggest replicas first; the units of
  // one batch next to each other.
  BL->cls.resize(n);
  for (int r = 0; r < n; ++r) BL->cls[r] = batch_class(sweep_lds_bytes(probs[r].n_cells, nc, BL->L[r].geom.K));
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (BL->cls[a] != BL->cls[b]) return BL->cls[a] < BL->cls[b];
    return probs[a].n_src > probs[b].n_src;
  });
  BL->units.clear();
  for (int ci = 0; ci < kBatchClasses; ++ci) {
    BL->cls_u0[ci] = (uint32_t)BL->units.size();
    for (int r : order)
      if (BL->cls[r] == ci)
        for (int b = 0; b < probs[r].n_batches; ++b)
          for (int j = 0; j < BL->L[r].geom.K; ++j) BL->units.push_back(((uint32_t)r << 16) | ((uint32_t)b << 8) | (uint32_t)j);
    BL->cls_u1[ci] = (uint32_t)BL->units.size();
  }
  int64_t rb = 8;
  real_bytes(probs[0].precision, &rb);
  Carver c;
  BL->off_desc = c.take((int64_t)n * (int64_t)std::max(sizeof(ReplicaDesc<double>), sizeof(ReplicaDesc<float>)));
  BL->off_units = c.take(4 * (int64_t)BL->units.size());
  BL->off_work = c.take(8 * kBatchClasses);
  BL->off_err = c.take(4);
  BL->off_counters = c.take(8 * 2 * C_NCOUNTERS * (int64_t)n);
  for (int k = 0; k < 2; ++k) {
    BL->off_seg[k] = c.take(4 * BL->n_seg);
    BL->off_ovf[k] = c.take(4 * BL->n_ovf);
  }
  BL->off_phi = c.take(8 * BL->n_phi);
  BL->off_J = c.take(8 * BL->n_J);
  BL->off_losm = c.take((int64_t)sizeof(LosmReplica) * n);
  BL->off_bs = c.take((int64_t)sizeof(BeginStepArgs) * 2 * n);
  const int64_t qslots = 2 * (int64_t)kGridMax * BL->dcap;
  BL->off_q = c.take(0);
  c.take(2 * rb * qslots);
  c.take(sizeof(WTau) * qslots);
  c.take(8 * qslots);
  c.take(sizeof(Tag) * qslots);
  BL->base.resize(n);
  for (int r = 0; r < n; ++r) BL->base[r] = c.take(BL->L[r].total);
  BL->total = c.cur;
  return HWW_OK;
}

size_t replica_cell_bytes(const hww_handle *r) {
  return r->fp32 ? lds_cell_bytes<float>() : lds_cell_bytes<double>();
}
bool replica_cells_lds(const hww_handle *r) {
  return sweep_lds_bytes(r->I, r->nc, r->K, replica_cell_bytes(r)) <= kLdsBytes;
}

template <typename Real>
ReplicaDesc<Real> replica_desc(hww_handle *r) {
  ReplicaDesc<Real> d{};
  d.I = r->I; d.B = r->B; d.nc = r->nc;
  d.v = r->p.speed; d.inv_v = 1.0 / r->p.speed; d.dt = r->p.dt;
  d.seed = r->p.seed; d.key1 = r->p.replica << 4;
  d.win = r->win;
  d.track_moments = r->track_moments;
  d.cells_lds = replica_cells_lds(r) ? 1 : 0;
  d.geom = r->L.geom;
  for (int k = 0; k < 2; ++k) {
    if constexpr (sizeof(Real) == 8) d.bank[k] = r->bank[k];
    else d.bank[k] = r->bank32[k];
    d.tal[k] = r->tal[k];
    d.tsum[k] = r->tsum[k];
    d.bnd[k] = r->bnd[k];
  }
  if constexpr (sizeof(Real) == 8) d.cells = r->cells;
  else d.cells = r->cells32;
  d.tracks = r->tracks;
  d.counters = r->counters;
  d.wnext = r->wnext;
  return d;
}

LosmArgs replica_losm_args(hww_handle *r) {
  LosmArgs a{};
  a.I = r->I; a.B = r->B; a.nc = r->nc;
  a.v = r->p.speed; a.dt = r->p.dt; a.n_src = (double)r->p.n_src;
  a.edges = r->edges; a.sig_t = r->sig_t; a.sig_s = r->sig_s;
  a.wstart = r->wstart; a.wnext = r->wnext;
  a.scratch = r->scratch; a.factor = r->factor;
  a.win = r->win;
  a.phi_out = r->phi_out; a.J_out = r->J_out; a.err = r->err; a.status = r->status;
  a.F_out = reinterpret_cast<double *>(r->ws + r->L.off_F_out);
  a.P_out = reinterpret_cast<double *>(r->ws + r->L.off_P_out);
  return a;
}

BeginStepArgs begin_args(hww_handle *h) {
  BeginStepArgs bs{};
  bs.segcnt = h->bank[1 - h->start_bank].segcnt;
  bs.ovfcnt = h->bank[1 - h->start_bank].ovfcnt;
  bs.tal = h->tal[h->cur_tal]; bs.tsum = h->tsum[h->cur_tal]; bs.bnd = h->bnd[h->cur_tal];
  bs.tracks = h->tracks; bs.counters = h->counters;
  bs.wstart = h->wstart; bs.wnext = h->wnext;
  bs.n_seg = (int64_t)h->R * h->K; bs.n_ovf = h->R;
  bs.n_tal = (int64_t)h->B * h->I * 6; bs.n_tsum = (int64_t)kSumCopies * 6 * h->I; bs.n_bnd = (int64_t)h->B * 6; bs.n_tracks = h->I;
  bs.nc = h->nc;
  return bs;
}

// Swap the start and census banks and the tally sets (batch and replicas).
void flip_banks(hww_handle *h) {
  h->start_bank = 1 - h->start_bank;
  h->cur_tal = 1 - h->cur_tal;
  for (hww_handle *r : h->rep) {
    r->start_bank = h->start_bank;
    r->cur_tal = h->cur_tal;
  }
}

// Queue the clearing of the new step's accumulators (after flip_banks).
int begin_step(hww_handle *h) {
  ++h->tal_epoch[h->cur_tal];
  if (h->is_batch) {
    HIPCHK(h, launch_begin_step_batch(h->bs_tab + (size_t)h->start_bank * h->rep.size(), (int)h->rep.size(),
                                      (int64_t)64 * h->max_I * 6, h->stream));
  } else {
    HIPCHK(h, launch_begin_step(begin_args(h), h->stream));
  }
  return HWW_OK;
}

void sync_replica_state(hww_handle *h) {
  for (hww_handle *r : h->rep) {
    r->step = h->step;
    r->next_chunk = h->next_chunk;
    r->start_bank = h->start_bank;
    r->cur_tal = h->cur_tal;
    r->ww_on = h->ww_on;
    r->factor_theta = h->factor_theta;
  }
}

int poll_batch(hww_handle *h) {
  uint32_t e = 0;
  HIPCHK(h, hipMemcpyAsync(&e, h->err, 4, hipMemcpyDeviceToHost, h->stream));
  const int cb = 1 - h->start_bank;
  std::vector<uint32_t> seg((size_t)h->n_seg_all), ovf((size_t)h->n_ovf_all);
  HIPCHK(h, hipMemcpyAsync(seg.data(), h->segcnt_all[cb], 4 * seg.size(), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(ovf.data(), h->ovfcnt_all[cb], 4 * ovf.size(), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (e & (ERR_CAPACITY | ERR_SPLIT | ERR_GENERATIONS | ERR_DAUGHTERS)) {
    h->fatal = HWW_E_CAPACITY;
    return fail(h, HWW_E_CAPACITY, (e & ERR_SPLIT) ? "a split exceeded 1e9 daughters"
                                   : (e & ERR_GENERATIONS) ? "too many daughter generations"
                                   : (e & ERR_DAUGHTERS) ? "a work-group's daughter buffer overflowed"
                                                         : "bank segment overflow");
  }
  for (size_t q = 0; q < h->rep.size(); ++q) {
    hww_handle *r = h->rep[q];
    const int64_t so = r->bank[cb].segcnt - h->segcnt_all[cb], oo = r->bank[cb].ovfcnt - h->ovfcnt_all[cb];
    uint64_t t = 0;
    for (int64_t j = 0; j < (int64_t)r->R * r->K; ++j) t += std::min<uint64_t>(seg[so + j], (uint64_t)r->L.geom.seg_cap);
    for (int64_t j = 0; j < r->R; ++j) t += std::min<uint64_t>(ovf[oo + j], (uint64_t)r->L.geom.ovf_cap);
    if (t > (uint64_t)r->p.bank_capacity) {
      h->fatal = HWW_E_CAPACITY;
      return fail(h, HWW_E_CAPACITY, "census bank of replica " + std::to_string(q) + " exceeds bank_capacity");
    }
  }
  if (e & ERR_NUMERIC) {
    h->fatal = HWW_E_NUMERIC;
    return fail(h, HWW_E_NUMERIC, "non-finite or non-positive window, or zero pivot in the LOSM solve");
  }
  return HWW_OK;
}

// Counters of the batch or problem: part 0 this step, 1 since init.
int read_counters(hww_handle *h, int part, unsigned long long out[C_NCOUNTERS]) {
  const size_t n = h->is_batch ? h->rep.size() : 1;
  std::vector<unsigned long long> all(n * 2 * C_NCOUNTERS);
  HIPCHK(h, hipMemcpyAsync(all.data(), h->is_batch ? h->counters_all : h->counters, 8 * all.size(),
                           hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int q = 0; q < C_NCOUNTERS; ++q) out[q] = 0;
  for (size_t r = 0; r < n; ++r)
    for (int q = 0; q < C_NCOUNTERS; ++q) {
      const unsigned long long v = all[(r * 2 + part) * C_NCOUNTERS + q];
      if (q == C_GENERATIONS) out[q] = std::max(out[q], v);
      else out[q] += v;
    }
  return HWW_OK;
}

void fill_stats(hww_handle *h, const unsigned long long *cnt, hww_step_stats *stats) {
  stats->segments = cnt[C_SEGMENTS];
  stats->collisions = cnt[C_COLLISIONS];
  stats->scatters = cnt[C_SCATTERS];
  stats->absorptions = cnt[C_ABSORPTIONS];
  stats->crossings = cnt[C_CROSSINGS];
  stats->leaks = cnt[C_LEAKS];
  stats->census = cnt[C_CENSUS];
  stats->splits = cnt[C_SPLITS];
  stats->daughters = cnt[C_DAUGHTERS];
  stats->rr_kill = cnt[C_RR_KILL];
  stats->rr_survive = cnt[C_RR_SURVIVE];
  stats->histories = cnt[C_HISTORIES];
  stats->generations = cnt[C_GENERATIONS];
  stats->fissions = cnt[C_FISSIONS];
  stats->fission_births = cnt[C_FISSION_BIRTHS];
  const uint64_t rec = h->fp32 ? 36 : 44, drec = h->fp32 ? 44 : 52;
  stats->bytes_moved = cnt[C_HISTORIES] * rec + cnt[C_CENSUS] * rec + cnt[C_DAUGHTERS] * 2 * drec;
}

// Default launch shape of a batch: as many work-groups per compute unit as
// the LDS histogram and the thread limit allow, up to four.
int default_grid(hww_handle *h, size_t lds, int block) {
  int wpc = 4;
  while (wpc > 1 && ((size_t)wpc * lds > 160 * 1024 || wpc * block > 2048)) --wpc;
  return std::min(kGridMax, h->cus * wpc);
}

}  // namespace

extern "C" {

int64_t hww_workspace_bytes(const hww_problem *problem) {
  std::string why;
  if (validate(problem, &why) != HWW_OK) return HWW_E_INVALID_ARG;
  Layout L;
  make_layout(*problem, &L);
  return L.total;
}

int hww_init_problem(const hww_problem *problem, void *dev_workspace, int64_t ws_bytes, void *hip_stream,
                     hww_handle **out) {
  std::string why;
  if (!out) return fail(nullptr, HWW_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int rc = validate(problem, &why);
  if (rc != HWW_OK) return fail(nullptr, rc, why);
  Layout L;
  make_layout(*problem, &L);
  if (!dev_workspace || ws_bytes < L.total) return fail(nullptr, HWW_E_INVALID_ARG, "workspace too small");
  if (reinterpret_cast<uintptr_t>(dev_workspace) % 256 != 0) return fail(nullptr, HWW_E_INVALID_ARG, "workspace not 256-byte aligned");

  hww_handle *h = new hww_handle();
  carve_handle(h, *problem, reinterpret_cast<char *>(dev_workspace), L, reinterpret_cast<hipStream_t>(hip_stream));
  rc = prime_handle(h, *problem);
  if (rc == HWW_OK) rc = poll_errors(h);
  if (rc != HWW_OK) {
    g_init_error = h->msg;
    destroy_events(h);
    delete h;
    return rc;
  }
  *out = h;
  return HWW_OK;
}

int hww_init_problem_static(const hww_problem *problem, void *hip_stream, hww_handle **out) {
  std::string why;
  if (!out) return fail(nullptr, HWW_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int rc = validate(problem, &why);
  if (rc != HWW_OK) return fail(nullptr, rc, why);
  Layout L;
  make_layout(*problem, &L);
  if (L.total > (int64_t)HWW_STATIC_WORKSPACE_BYTES)
    return fail(nullptr, HWW_E_INVALID_ARG,
                "problem needs " + std::to_string(L.total) + " workspace bytes; the static workspace holds " +
                    std::to_string((int64_t)HWW_STATIC_WORKSPACE_BYTES));
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(nullptr, HWW_E_DEVICE, "no current device (or its ordinal is >= 64)");
  if (hip_stream) {
    hipDevice_t sdev = -1;
    if (hipStreamGetDevice(reinterpret_cast<hipStream_t>(hip_stream), &sdev) != hipSuccess || sdev != dev)
      return fail(nullptr, HWW_E_INVALID_ARG, "the stream does not belong to the current device");
  }
  char *ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_busy[dev]) return fail(nullptr, HWW_E_STATE, "a live handle already uses this device's static workspace");
    rc = static_workspace(dev, &ws, &why);
    if (rc != HWW_OK) return fail(nullptr, rc, why);
    g_static_busy[dev] = true;
  }
  hww_handle *h = new hww_handle();
  h->static_dev = dev;
  // prime_handle clears every accumulator the previous user of the array
  // left behind; the banks and queues are read only below their counts.
  carve_handle(h, *problem, ws, L, reinterpret_cast<hipStream_t>(hip_stream));
  rc = prime_handle(h, *problem);
  if (rc == HWW_OK) rc = poll_errors(h);
  if (rc != HWW_OK) {
    g_init_error = h->msg;
    hww_destroy(h);
    return rc;
  }
  *out = h;
  return HWW_OK;
}

int hww_set_windows(hww_handle *h, const double *centre, double rho) {
  if (!h) return HWW_E_INVALID_ARG;
  if (h->is_view) return fail(h, HWW_E_STATE, "a replica view is read-only");
  if (!centre) {
    h->ww_on = 0;
    sync_replica_state(h);
    return HWW_OK;
  }
  if (!(rho >= 1.0) || !std::isfinite(rho)) return fail(h, HWW_E_INVALID_ARG, "rho must be >= 1");
  std::vector<hww_handle *> targets = h->is_batch ? h->rep : std::vector<hww_handle *>{h};
  int64_t total = 0;
  for (hww_handle *t : targets) total += t->I;
  std::vector<Window> w3((size_t)total);
  for (int64_t i = 0; i < total; ++i) {
    if (!(centre[i] > 0.0) || !std::isfinite(centre[i])) return fail(h, HWW_E_NUMERIC, "window centres must be positive and finite");
    w3[i].ww = centre[i];
    w3[i].ceil = centre[i] * rho;
    w3[i].floor = centre[i] / rho;
    w3[i].pad = 0.0;
  }
  int64_t o = 0;
  for (hww_handle *t : targets) {
    HIPCHK(h, hipMemcpyAsync(t->win, w3.data() + o, sizeof(Window) * (size_t)t->I, hipMemcpyHostToDevice, h->stream));
    o += t->I;
  }
  // The host vector must outlive the copies.
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->ww_on = 1;
  sync_replica_state(h);
  return HWW_OK;
}

int hww_sweep_step(hww_handle *h, int32_t step, int32_t chunk, hww_step_stats *stats) {
  if (!h) return HWW_E_INVALID_ARG;
  if (h->is_view) return fail(h, HWW_E_STATE, "a replica view is read-only");
  if (h->fatal) return fail(h, h->fatal, "an earlier error left the problem invalid");
  if (chunk < 0 || chunk >= h->nc) return fail(h, HWW_E_INVALID_ARG, "chunk out of range");
  if (chunk == 0) {
    if (h->next_chunk != h->nc || step != h->step + 1 || step > h->p.n_steps)
      return fail(h, HWW_E_STATE, "step out of order");
    // The census bank of the finished step becomes the start bank.
    flip_banks(h);
    int rc = begin_step(h);
    if (rc != HWW_OK) return rc;
    h->step = step;
    h->next_chunk = 0;
    h->n_launch = 0;
    h->step_ev0 = h->ev_used;
  } else if (step != h->step || chunk != h->next_chunk) {
    return fail(h, HWW_E_STATE, "chunk out of order");
  }

  const int k = h->ev_used;
  if (h->timing) {
    while ((int)h->ev.size() < 2 * (k + 1)) {
      hipEvent_t e = nullptr;
      // Timing only: no system-scope fence at the record (the stream is
      // synchronised before any elapsed time is read).
      HIPCHK(h, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      h->ev.push_back(e);
    }
    HIPCHK(h, hipEventRecord(h->ev[2 * k], h->stream));
  }
  const int lrc = h->fp32 ? launch_chunk<float>(h, chunk, (int)(h->launch_count & 1))
                          : launch_chunk<double>(h, chunk, (int)(h->launch_count & 1));
  if (lrc != HWW_OK) return lrc;
  if (h->timing) {
    HIPCHK(h, hipEventRecord(h->ev[2 * k + 1], h->stream));
    h->ev_used = k + 1;
  }
  h->launch_count += 1;
  h->n_launch += 1;
  h->next_chunk = chunk + 1;
  sync_replica_state(h);
  if (!stats) return HWW_OK;

  unsigned long long cnt[C_NCOUNTERS];
  int rc = read_counters(h, 0, cnt);
  if (rc != HWW_OK) return rc;
  rc = poll_errors(h);
  if (rc != HWW_OK) return rc;
  fill_stats(h, cnt, stats);
  stats->launches = (uint64_t)h->n_launch;
  double ms = 0.0;
  for (int q = h->step_ev0; q < h->ev_used; ++q) {
    float t = 0.0f;
    HIPCHK(h, hipEventElapsedTime(&t, h->ev[2 * q], h->ev[2 * q + 1]));
    ms += t;
  }
  stats->kernel_ms = ms;
  return HWW_OK;
}

int hww_comb(hww_handle *h, int64_t n_target, int64_t *n_before, double *w_total) {
  if (!h) return HWW_E_INVALID_ARG;
  if (h->is_batch || h->is_view) return fail(h, HWW_E_STATE, "combing needs a single problem");
  if (h->fatal) return fail(h, h->fatal, "an earlier error left the problem invalid");
  if (!h->p.comb) return fail(h, HWW_E_STATE, "the problem was initialised without comb workspace");
  if (n_target < 1 || n_target > h->p.bank_capacity || n_target > 0xFFFFFFFFll)
    return fail(h, HWW_E_INVALID_ARG, "n_target must be in 1..bank_capacity and < 2^32");
  if (h->step < 1 || h->next_chunk != h->nc) return fail(h, HWW_E_STATE, "combing needs a finished step");
  const Layout &L = h->L;
  const BankGeom &G = L.geom;
  // Every region of the new bank must fit its segments and overflow.
  for (int b = 0; b < h->B; ++b)
    for (int c = 0; c < h->nc; ++c) {
      const int64_t n_b = n_target > b ? (n_target - b + h->B - 1) / h->B : 0;
      const int64_t n_bc = n_b > c ? (n_b - c + h->nc - 1) / h->nc : 0;
      const int64_t per = std::min<int64_t>(G.seg_cap, (n_bc + G.K - 1) / G.K);
      if (n_bc - (int64_t)G.K * per > G.ovf_cap) return fail(h, HWW_E_CAPACITY, "a region of the combed bank overflows");
    }
  auto fill = [&](CombArgs<double> &a) {
    a.G = G;
    a.B = h->B; a.nc = h->nc; a.R = h->R;
    a.n_hist = h->src_bound;
    a.cap = L.comb_slots;
    a.n_target = n_target;
    a.no_wait = (!n_before && !w_total) ? 1 : 0;
    a.by_index = h->p.comb == 2 ? 1 : 0;
    a.seed = h->p.seed; a.key1 = h->p.replica << 4; a.step = (uint32_t)h->step;
    a.cnt = reinterpret_cast<unsigned long long *>(h->ws + L.off_c_cnt);
    a.cur = reinterpret_cast<uint32_t *>(h->ws + L.off_c_cur);
    a.order = reinterpret_cast<unsigned long long *>(h->ws + L.off_c_order);
    a.wq = reinterpret_cast<unsigned long long *>(h->ws + L.off_c_wq);
    a.blk = reinterpret_cast<unsigned long long *>(h->ws + L.off_c_blk);
    a.misc = reinterpret_cast<unsigned long long *>(h->ws + L.off_c_misc);
    a.wnext = h->wnext;
    a.err = h->err;
  };
  CombArgs<double> a{};
  CombArgs<float> a32{};
  fill(a);
  a.src_bank = h->bank[1 - h->start_bank];
  a.dst_bank = h->bank[h->start_bank];
  if (h->fp32) {
    a32.src_bank = h->bank32[1 - h->start_bank];
    a32.dst_bank = h->bank32[h->start_bank];
    a32.G = a.G; a32.B = a.B; a32.nc = a.nc; a32.R = a.R; a32.n_hist = a.n_hist; a32.cap = a.cap;
    a32.n_target = a.n_target; a32.no_wait = a.no_wait; a32.by_index = a.by_index; a32.seed = a.seed; a32.key1 = a.key1; a32.step = a.step;
    a32.cnt = a.cnt; a32.cur = a.cur; a32.order = a.order; a32.wq = a.wq; a32.blk = a.blk; a32.misc = a.misc;
    a32.wnext = a.wnext; a32.err = a.err;
  }
  HIPCHK(h, h->fp32 ? launch_comb<float>(a32, h->stream) : launch_comb<double>(a, h->stream));
  if (a.no_wait) {
    // The combed bank (empty if the census was) becomes the census bank;
    // errors reach the error word, read at the next synchronising call.
    h->start_bank = 1 - h->start_bank;
    h->src_bound = std::max<int64_t>(h->src_bound, n_target);
    return HWW_OK;
  }
  unsigned long long misc[8];
  uint32_t e = 0;
  HIPCHK(h, hipMemcpyAsync(misc, a.misc, sizeof misc, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(&e, h->err, 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  const int64_t n = (int64_t)misc[1];
  if (n_before) *n_before = n;
  if (w_total) *w_total = 0.0;
  if (n > 0) {
    // The kernels after the count do nothing unless the largest weight is
    // positive and finite; an empty census stays empty.
    double m;
    std::memcpy(&m, &misc[0], 8);
    if (!(m > 0.0) || !std::isfinite(m)) return fail(h, HWW_E_NUMERIC, "census weights must be positive and finite");
    // The combed bank becomes the census bank; its histories are 0..n_target-1.
    h->start_bank = 1 - h->start_bank;
    h->src_bound = std::max<int64_t>(h->src_bound, n_target);
  }
  // The census is the n_target copies after a comb, still empty otherwise.
  const int rc = error_status(h, e, n > 0 ? (uint64_t)n_target : 0u);
  if (rc != HWW_OK) return rc;
  if (n == 0) return HWW_OK;
  if (w_total) std::memcpy(w_total, &misc[2], 8);
  return HWW_OK;
}

int hww_read_run_stats(hww_handle *h, hww_step_stats *stats) {
  if (!h || !stats) return HWW_E_INVALID_ARG;
  unsigned long long cnt[C_NCOUNTERS];
  int rc = read_counters(h, 1, cnt);
  if (rc != HWW_OK) return rc;
  rc = poll_errors(h);
  if (rc != HWW_OK) return rc;
  for (; h->ev_summed < h->ev_used; ++h->ev_summed) {
    float t = 0.0f;
    HIPCHK(h, hipEventElapsedTime(&t, h->ev[2 * h->ev_summed], h->ev[2 * h->ev_summed + 1]));
    h->ms_summed += t;
  }
  fill_stats(h, cnt, stats);
  stats->launches = (uint64_t)h->launch_count;
  stats->kernel_ms = h->ms_summed;
  return HWW_OK;
}

// The batch sums of the initial-condition set stay in the LOSM scratch from
// one solve to the next while that tally set is not written: the semi-
// implicit solve of a step and the implicit solves of the next share them.
// A replica view of a batch sees no sweeps of its own and never caches.
static int ic_cached(const hww_handle *h, int buf) {
  return !h->is_view && h->ic_buf == buf && h->ic_epoch == h->tal_epoch[buf];
}
static void note_ic(hww_handle *h, int buf) {
  if (h->is_view) return;
  h->ic_buf = buf;
  h->ic_epoch = h->tal_epoch[buf];
}

int hww_solve_losm(hww_handle *h, const hww_losm_opts *o, double *phi_out, double *J_out) {
  if (!h || !o) return HWW_E_INVALID_ARG;
  if (h->is_view) return fail(h, HWW_E_STATE, "a replica view is read-only");
  if (h->fatal) return fail(h, h->fatal, "an earlier error left the problem invalid");
  if (!(o->theta > 0.0 && o->theta <= 1.0) || o->ma_k < 0 || o->filter < 0 || o->filter > 2 || o->kappa < 0)
    return fail(h, HWW_E_INVALID_ARG, "bad LOSM options");
  if (o->lagged && (o->implicit || !o->apply_windows))
    return fail(h, HWW_E_INVALID_ARG, "lagged windows are set at the start of a step");
  if (o->closure_track && !o->lagged && h->track_moments < 2)
    return fail(h, HWW_E_INVALID_ARG, "track-length closures need the K tally (track_moments 0, 2 or 3)");
  if (o->lagged && h->step == 0 && h->next_chunk == h->nc) {
    // The source has no track-length flux: the first step runs with the
    // windows as they are (none unless set).
    if (phi_out) std::memset(phi_out, 0, 8 * (size_t)(h->is_batch ? h->n_phi_all : h->I + 2));
    if (J_out) std::memset(J_out, 0, 8 * (size_t)(h->is_batch ? h->n_J_all : h->I + 1));
    return HWW_OK;
  }
  if (o->apply_windows && (!(o->rho >= 1.0) || !(o->eps_min > 0.0 && o->eps_min <= 1.0)))
    return fail(h, HWW_E_INVALID_ARG, "bad window options");
  if (h->is_batch) {
    if (!o->implicit) {
      if (h->next_chunk != h->nc || h->step >= h->p.n_steps) return fail(h, HWW_E_STATE, "semi-implicit solve needs a finished step");
    } else if (h->step < 1 || h->next_chunk < 1 || h->next_chunk >= h->nc) {
      return fail(h, HWW_E_STATE, "implicit solve needs a step in progress");
    }
    LosmCall c{};
    c.cur = h->cur_tal;
    c.implicit = o->implicit; c.next_chunk = h->next_chunk; c.filter = o->filter; c.ma_k = o->ma_k;
    c.closure_track = o->lagged ? 1 : o->closure_track; c.apply_windows = o->apply_windows; c.export_only = 0;
    c.kappa = o->kappa; c.lagged = o->lagged; c.window_scale = o->window_scale ? 1 : 0;
    c.refactor = (o->theta != h->factor_theta) ? 1 : 0;
    c.work_in_lds = h->losm_wil;
    c.theta = o->theta; c.eps_min = o->eps_min; c.rho = o->rho;
    const int ib = o->implicit ? 1 - h->cur_tal : h->cur_tal;
    c.ic_cached = ic_cached(h, ib);
    HIPCHK(h, launch_losm_batch(h->losm_tab, (int)h->rep.size(), h->max_I, c, h->stream));
    note_ic(h, ib);
    h->factor_theta = o->theta;
    if (o->apply_windows) h->ww_on = 1;
    sync_replica_state(h);
    if (phi_out || J_out) {
      if (phi_out) HIPCHK(h, hipMemcpyAsync(phi_out, h->phi_cat, 8 * (size_t)h->n_phi_all, hipMemcpyDeviceToHost, h->stream));
      if (J_out) HIPCHK(h, hipMemcpyAsync(J_out, h->J_cat, 8 * (size_t)h->n_J_all, hipMemcpyDeviceToHost, h->stream));
      return poll_errors(h);
    }
    return HWW_OK;
  }
  LosmArgs a{};
  a.I = h->I; a.B = h->B; a.nc = h->nc;
  a.v = h->p.speed; a.dt = h->p.dt; a.n_src = (double)h->p.n_src;
  a.edges = h->edges; a.sig_t = h->sig_t; a.sig_s = h->sig_s;
  if (!o->implicit) {
    if (h->next_chunk != h->nc || h->step >= h->p.n_steps) return fail(h, HWW_E_STATE, "semi-implicit solve needs a finished step");
    a.tsum_ic = h->tsum[h->cur_tal]; a.bnd_ic = h->bnd[h->cur_tal];
    a.tsum_cl = a.tsum_ic; a.bnd_cl = a.bnd_ic;
  } else {
    if (h->step < 1 || h->next_chunk < 1 || h->next_chunk >= h->nc) return fail(h, HWW_E_STATE, "implicit solve needs a step in progress");
    a.tsum_ic = h->tsum[1 - h->cur_tal]; a.bnd_ic = h->bnd[1 - h->cur_tal];
    a.tsum_cl = h->tsum[h->cur_tal]; a.bnd_cl = h->bnd[h->cur_tal];
  }
  a.wstart = h->wstart; a.wnext = h->wnext; a.next_chunk = h->next_chunk;
  a.theta = o->theta; a.implicit = o->implicit; a.filter = o->filter; a.ma_k = o->ma_k;
  a.closure_track = o->lagged ? 1 : o->closure_track; a.apply_windows = o->apply_windows;
  a.kappa = o->kappa; a.lagged = o->lagged; a.window_scale = o->window_scale ? 1 : 0;
  a.eps_min = o->eps_min; a.rho = o->rho;
  a.scratch = h->scratch; a.factor = h->factor;
  a.refactor = (o->theta != h->factor_theta) ? 1 : 0;
  a.win = h->win;
  a.phi_out = h->phi_out; a.J_out = h->J_out; a.err = h->err; a.status = h->status;
  const int ib = o->implicit ? 1 - h->cur_tal : h->cur_tal;
  a.ic_cached = ic_cached(h, ib);
  if (a.refactor) HIPCHK(h, launch_fill_u32(reinterpret_cast<uint32_t *>(h->status), 0u, 1, h->stream));
  HIPCHK(h, launch_losm(a, h->stream));
  note_ic(h, ib);
  h->factor_theta = o->theta;
  if (o->apply_windows) h->ww_on = 1;
  if (phi_out || J_out) {
    if (phi_out) HIPCHK(h, hipMemcpyAsync(phi_out, h->phi_out, 8 * (size_t)(h->I + 2), hipMemcpyDeviceToHost, h->stream));
    if (J_out) HIPCHK(h, hipMemcpyAsync(J_out, h->J_out, 8 * (size_t)(h->I + 1), hipMemcpyDeviceToHost, h->stream));
    return poll_errors(h);
  }
  return HWW_OK;
}

int hww_read_closures(hww_handle *h, double *F, double *P, double *phi, double *J) {
  if (!h || !F || !P || !phi || !J) return HWW_E_INVALID_ARG;
  if (h->is_batch) return fail(h, HWW_E_STATE, "read the closures of a replica through hww_batch_replica");
  if (h->fatal) return fail(h, h->fatal, "an earlier error left the problem invalid");
  if (h->next_chunk != h->nc) return fail(h, HWW_E_STATE, "closures need a finished step");
  LosmArgs a{};
  a.I = h->I; a.B = h->B; a.nc = h->nc;
  a.v = h->p.speed; a.dt = h->p.dt; a.n_src = (double)h->p.n_src;
  a.edges = h->edges; a.sig_t = h->sig_t; a.sig_s = h->sig_s;
  a.tsum_ic = h->tsum[h->cur_tal]; a.bnd_ic = h->bnd[h->cur_tal];
  a.tsum_cl = a.tsum_ic; a.bnd_cl = a.bnd_ic;
  a.wstart = h->wstart; a.wnext = h->wnext; a.next_chunk = h->next_chunk;
  a.theta = h->factor_theta > 0.0 ? h->factor_theta : 0.5;
  a.implicit = 0; a.filter = 0; a.apply_windows = 0;
  a.scratch = h->scratch; a.factor = h->factor;
  a.refactor = (a.theta != h->factor_theta) ? 1 : 0;
  a.win = h->win;
  a.phi_out = h->phi_out; a.J_out = h->J_out; a.err = h->err; a.status = h->status;
  a.export_only = 1;
  a.F_out = reinterpret_cast<double *>(h->ws + h->L.off_F_out);
  a.P_out = reinterpret_cast<double *>(h->ws + h->L.off_P_out);
  a.ic_cached = ic_cached(h, h->cur_tal);
  if (a.refactor) HIPCHK(h, launch_fill_u32(reinterpret_cast<uint32_t *>(h->status), 0u, 1, h->stream));
  HIPCHK(h, launch_losm(a, h->stream));
  note_ic(h, h->cur_tal);
  h->factor_theta = a.theta;
  const int I = h->I;
  HIPCHK(h, hipMemcpyAsync(F, a.F_out, 8 * (size_t)(I + 2), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(P, a.P_out, 16, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(phi, h->phi_out, 8 * (size_t)(I + 2), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(J, h->J_out, 8 * (size_t)(I + 1), hipMemcpyDeviceToHost, h->stream));
  return poll_errors(h);
}

int hww_losm_march(hww_handle *h, const double *sigma_t, const double *sigma_s, double theta, int32_t n_steps,
                   const double *F, const double *P, const double *phi0, const double *J0, const double *weights,
                   double *phi_hist, double *J_hist, double *G) {
  if (!h || !sigma_t || !sigma_s || !F || !P || !phi0 || !J0 || !weights || !G) return HWW_E_INVALID_ARG;
  if (h->is_batch || h->is_view) return fail(h, HWW_E_STATE, "the march runs on a single problem");
  if (n_steps < 1 || n_steps > h->p.n_steps) return fail(h, HWW_E_INVALID_ARG, "n_steps out of range");
  if (!(theta > 0.0 && theta <= 1.0)) return fail(h, HWW_E_INVALID_ARG, "theta must be in (0, 1]");
  const int I = h->I;
  for (int i = 0; i < I; ++i)
    if (!(sigma_t[i] > 0.0) || !(sigma_s[i] >= 0.0) || !std::isfinite(sigma_t[i]) || !std::isfinite(sigma_s[i]))
      return fail(h, HWW_E_INVALID_ARG, "march cross sections must be positive and finite");
  const Layout &L = h->L;
  char *ws = h->ws;
  MarchArgs &a = h->march;
  a = MarchArgs{};
  a.I = I; a.n_steps = n_steps; a.v = h->p.speed; a.dt = h->p.dt; a.theta = theta;
  a.edges = h->edges;
  double *msig = reinterpret_cast<double *>(ws + L.off_m_sig);
  a.sig_t = msig; a.sig_s = msig + I;
  a.F = reinterpret_cast<double *>(ws + L.off_m_F);
  a.P = reinterpret_cast<double *>(ws + L.off_m_P);
  a.phi0 = reinterpret_cast<double *>(ws + L.off_m_phi0);
  a.J0 = reinterpret_cast<double *>(ws + L.off_m_J0);
  a.w = reinterpret_cast<double *>(ws + L.off_m_w);
  a.hist = reinterpret_cast<double *>(ws + L.off_m_hist);
  a.factor = reinterpret_cast<double *>(ws + L.off_m_fac);
  a.factor_t = reinterpret_cast<double *>(ws + L.off_m_fact);
  a.G = reinterpret_cast<double *>(ws + L.off_m_G);
  a.g_t = reinterpret_cast<double *>(ws + L.off_m_g);
  a.g_s = a.g_t + I;
  a.err = h->err;
  const size_t N1 = (size_t)n_steps + 1, M = (size_t)I + 2, n = 2 * (size_t)I + 3;
  HIPCHK(h, hipMemcpyAsync(msig, sigma_t, 8 * I, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(msig + I, sigma_s, 8 * I, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(const_cast<double *>(a.F), F, 8 * N1 * M, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(const_cast<double *>(a.P), P, 8 * N1 * 2, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(const_cast<double *>(a.phi0), phi0, 8 * M, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(const_cast<double *>(a.J0), J0, 8 * (M - 1), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(const_cast<double *>(a.w), weights, 8 * N1 * M, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, launch_march(a, h->stream));
  HIPCHK(h, hipMemcpyAsync(G, a.G, 8, hipMemcpyDeviceToHost, h->stream));
  std::vector<double> hist;
  if (phi_hist || J_hist) {
    hist.resize(N1 * n);
    HIPCHK(h, hipMemcpyAsync(hist.data(), a.hist, 8 * N1 * n, hipMemcpyDeviceToHost, h->stream));
  }
  int rc = poll_errors(h);
  if (rc != HWW_OK) return rc;
  for (size_t s = 0; s < N1; ++s) {
    if (phi_hist)
      for (size_t i = 0; i < M; ++i) phi_hist[s * M + i] = hist[s * n + 2 * i];
    if (J_hist)
      for (size_t j = 0; j + 1 < M; ++j) J_hist[s * (M - 1) + j] = hist[s * n + 2 * j + 1];
  }
  h->march_ok = 1;
  return HWW_OK;
}

int hww_losm_adjoint(hww_handle *h, const double *dG_dphi, double *grad_sigma_t, double *grad_sigma_s) {
  if (!h || !grad_sigma_t || !grad_sigma_s) return HWW_E_INVALID_ARG;
  if (h->is_batch || h->is_view || !h->march_ok) return fail(h, HWW_E_STATE, "the adjoint needs a preceding hww_losm_march");
  if (h->I > 4 * 1024) return fail(h, HWW_E_INVALID_ARG, "the adjoint handles I <= 4096");
  MarchArgs a = h->march;
  if (dG_dphi) {
    double *dw = reinterpret_cast<double *>(h->ws + h->L.off_m_dw);
    const size_t N1 = (size_t)a.n_steps + 1, M = (size_t)h->I + 2;
    HIPCHK(h, hipMemcpyAsync(dw, dG_dphi, 8 * N1 * M, hipMemcpyHostToDevice, h->stream));
    a.w = dw;
  }
  HIPCHK(h, launch_adjoint(a, h->stream));
  HIPCHK(h, hipMemcpyAsync(grad_sigma_t, a.g_t, 8 * (size_t)h->I, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(grad_sigma_s, a.g_s, 8 * (size_t)h->I, hipMemcpyDeviceToHost, h->stream));
  return poll_errors(h);
}

// Normalise a tally array of handle h in place (Eqs. phi-mc, ct-mc): track
// sums w*l over N_src dx dt, time-layer sums v*w over N_src dx, face sums
// w f(mu)/|mu| over N_src dt; other kinds are left as they are.
static void normalise_tallies(const hww_handle *h, int32_t kind, double *o) {
  const double N = (double)h->p.n_src, dt = h->p.dt;
  const int64_t I = h->I, B = h->B;
  if (kind == HWW_TALLY_CELLS || kind == HWW_TALLY_PREV_CELLS) {
    for (int64_t b = 0; b < B; ++b)
      for (int64_t i = 0; i < I; ++i) {
        double *c = o + (b * I + i) * 6;
        const double nt = N * h->dx_host[i] * dt, nc = N * h->dx_host[i];
        for (int k = 0; k < 3; ++k) c[k] /= nt;
        for (int k = 3; k < 6; ++k) c[k] /= nc;
      }
  } else if (kind == HWW_TALLY_BOUNDARY || kind == HWW_TALLY_PREV_BOUNDARY) {
    for (int64_t k = 0; k < B * 6; ++k) o[k] /= N * dt;
  }
}

int hww_read_tallies(hww_handle *h, int32_t kind, int32_t raw, void *out, int64_t out_bytes) {
  if (!h || !out) return HWW_E_INVALID_ARG;
  if (h->is_batch) {
    int64_t need = 0;
    for (hww_handle *r : h->rep) {
      const int64_t I = r->I, B = r->B;
      switch (kind) {
        case HWW_TALLY_CELLS: case HWW_TALLY_PREV_CELLS: need += 8 * B * I * 6; break;
        case HWW_TALLY_BOUNDARY: case HWW_TALLY_PREV_BOUNDARY: need += 8 * B * 6; break;
        case HWW_TALLY_TRACKS: need += 8 * I; break;
        case HWW_TALLY_WINDOWS: need += 8 * 3 * I; break;
        case HWW_TALLY_BANK_COUNTS: need += 16; break;
        default: return fail(h, HWW_E_INVALID_ARG, "unknown tally kind");
      }
    }
    if (out_bytes != need) return fail(h, HWW_E_INVALID_ARG, "out_bytes does not match the tally kind");
    char *o = static_cast<char *>(out);
    for (hww_handle *r : h->rep) {
      int64_t sz = 0;
      switch (kind) {
        case HWW_TALLY_CELLS: case HWW_TALLY_PREV_CELLS: sz = 8 * (int64_t)r->B * r->I * 6; break;
        case HWW_TALLY_BOUNDARY: case HWW_TALLY_PREV_BOUNDARY: sz = 8 * (int64_t)r->B * 6; break;
        case HWW_TALLY_TRACKS: sz = 8 * (int64_t)r->I; break;
        case HWW_TALLY_WINDOWS: sz = 8 * 3 * (int64_t)r->I; break;
        default: sz = 16; break;
      }
      const int rc = hww_read_tallies(r, kind, raw, o, sz);
      if (rc != HWW_OK) return fail(h, rc, r->msg);
      o += sz;
    }
    return poll_errors(h);
  }
  const int64_t I = h->I, B = h->B;
  const void *src = nullptr;
  int64_t bytes = 0;
  switch (kind) {
    case HWW_TALLY_CELLS: src = h->tal[h->cur_tal]; bytes = 8 * B * I * 6; break;
    case HWW_TALLY_BOUNDARY: src = h->bnd[h->cur_tal]; bytes = 8 * B * 6; break;
    case HWW_TALLY_TRACKS: src = h->tracks; bytes = 8 * I; break;
    case HWW_TALLY_PREV_CELLS: src = h->tal[1 - h->cur_tal]; bytes = 8 * B * I * 6; break;
    case HWW_TALLY_PREV_BOUNDARY: src = h->bnd[1 - h->cur_tal]; bytes = 8 * B * 6; break;
    case HWW_TALLY_WINDOWS: src = h->win; bytes = 8 * 3 * I; break;
    case HWW_TALLY_BANK_COUNTS: bytes = 16; break;
    default: return fail(h, HWW_E_INVALID_ARG, "unknown tally kind");
  }
  if (out_bytes != bytes) return fail(h, HWW_E_INVALID_ARG, "out_bytes does not match the tally kind");
  if (kind == HWW_TALLY_BANK_COUNTS) {
    uint64_t counts[2] = {0, 0};
    if (h->step > 0) {
      int rc = census_total(h, h->start_bank, &counts[0]);
      if (rc != HWW_OK) return rc;
    }
    int rc = census_total(h, 1 - h->start_bank, &counts[1]);
    if (rc != HWW_OK) return rc;
    std::memcpy(out, counts, 16);
    return HWW_OK;
  }
  if (kind == HWW_TALLY_WINDOWS) {
    std::vector<Window> wv(I);
    HIPCHK(h, hipMemcpyAsync(wv.data(), h->win, sizeof(Window) * I, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    double *o = static_cast<double *>(out);
    for (int64_t i = 0; i < I; ++i) {
      o[i] = h->ww_on ? wv[i].ww : 0.0;
      o[I + i] = h->ww_on ? wv[i].ceil : 0.0;
      o[2 * I + i] = h->ww_on ? wv[i].floor : 0.0;
    }
    return poll_errors(h);
  }
  HIPCHK(h, hipMemcpyAsync(out, src, bytes, hipMemcpyDeviceToHost, h->stream));
  const int rc = poll_errors(h);
  if (rc == HWW_OK && !raw) normalise_tallies(h, kind, static_cast<double *>(out));
  return rc;
}

int hww_read_bank(hww_handle *h, int32_t which, int64_t cap, int64_t *count, double *x, double *mu, double *w,
                  uint32_t *src, uint64_t *lin, uint32_t *e, int32_t *cell, int32_t *chunk) {
  if (!h || !count || (which != 0 && which != 1)) return HWW_E_INVALID_ARG;
  if (h->is_batch) return fail(h, HWW_E_INVALID_ARG, "read the bank of a replica through hww_batch_replica");
  if (which == 0 && h->step == 0) {
    *count = 0;
    return HWW_OK;
  }
  const int bi = which == 0 ? h->start_bank : 1 - h->start_bank;
  const Bank<double> &bk = h->bank[bi];
  const BankGeom &G = h->L.geom;
  std::vector<uint32_t> seg((size_t)h->R * h->K), ovf(h->R);
  HIPCHK(h, hipMemcpyAsync(seg.data(), bk.segcnt, 4 * seg.size(), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(ovf.data(), bk.ovfcnt, 4 * ovf.size(), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  int64_t total = 0;
  for (int r = 0; r < h->R; ++r) {
    for (int j = 0; j < h->K; ++j) total += std::min<int64_t>(seg[(size_t)r * h->K + j], G.seg_cap);
    total += std::min<int64_t>(ovf[r], G.ovf_cap);
  }
  *count = total;
  if (total > cap) return fail(h, HWW_E_INVALID_ARG, "cap smaller than the bank");
  int64_t o = 0;
  for (int r = 0; r < h->R; ++r) {
    for (int j = 0; j <= h->K; ++j) {
      const int64_t n = j < h->K ? std::min<int64_t>(seg[(size_t)r * h->K + j], G.seg_cap)
                                 : std::min<int64_t>(ovf[r], G.ovf_cap);
      if (n == 0) continue;
      const int64_t k = (int64_t)r * G.stride + (int64_t)j * G.seg_cap;
      std::vector<XMu<double>> xm(n);
      std::vector<XMu<float>> xmf(h->fp32 ? n : 0);
      std::vector<Tag> tg(n);
      if (h->fp32)
        HIPCHK(h, hipMemcpyAsync(xmf.data(), h->bank32[bi].xm + k, sizeof(XMu<float>) * n, hipMemcpyDeviceToHost,
                                 h->stream));
      else
        HIPCHK(h, hipMemcpyAsync(xm.data(), bk.xm + k, sizeof(XMu<double>) * n, hipMemcpyDeviceToHost, h->stream));
      // The w, lineage and tag streams sit at precision-dependent offsets.
      const Tag *tag_d = h->fp32 ? h->bank32[bi].tag : bk.tag;
      const double *w_d = h->fp32 ? h->bank32[bi].w : bk.w;
      const uint64_t *lin_d = h->fp32 ? h->bank32[bi].lin : bk.lin;
      HIPCHK(h, hipMemcpyAsync(tg.data(), tag_d + k, sizeof(Tag) * n, hipMemcpyDeviceToHost, h->stream));
      if (w) HIPCHK(h, hipMemcpyAsync(w + o, w_d + k, 8 * n, hipMemcpyDeviceToHost, h->stream));
      if (lin) HIPCHK(h, hipMemcpyAsync(lin + o, lin_d + k, 8 * n, hipMemcpyDeviceToHost, h->stream));
      HIPCHK(h, hipStreamSynchronize(h->stream));
      for (int64_t q = 0; q < n; ++q) {
        if (h->fp32) {
          xm[q].x = xmf[q].x;
          xm[q].mu = xmf[q].mu;
        }
        if (x) x[o + q] = xm[q].x;
        if (mu) mu[o + q] = xm[q].mu;
        if (src) src[o + q] = tg[q].src;
        if (e) e[o + q] = tg[q].e;
        if (cell) cell[o + q] = tg[q].cell;
        if (chunk) chunk[o + q] = r % h->nc;
      }
      o += n;
    }
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return HWW_OK;
}

int64_t hww_batch_workspace_bytes(const hww_problem *problems, int32_t n) {
  std::string why;
  BatchLayout BL;
  if (make_batch_layout(problems, n, &BL, &why) != HWW_OK) return HWW_E_INVALID_ARG;
  return BL.total;
}

int hww_init_batch(const hww_problem *problems, int32_t n, void *dev_workspace, int64_t ws_bytes, void *hip_stream,
                   hww_handle **out) {
  std::string why;
  if (!out) return fail(nullptr, HWW_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  BatchLayout BL;
  int rc = make_batch_layout(problems, n, &BL, &why);
  if (rc != HWW_OK) return fail(nullptr, rc, why);
  if (!dev_workspace || ws_bytes < BL.total) return fail(nullptr, HWW_E_INVALID_ARG, "workspace too small");
  if (reinterpret_cast<uintptr_t>(dev_workspace) % 256 != 0) return fail(nullptr, HWW_E_INVALID_ARG, "workspace not 256-byte aligned");
  char *ws = reinterpret_cast<char *>(dev_workspace);
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);

  hww_handle *h = new hww_handle();
  h->is_batch = 1;
  h->p = problems[0];
  h->p.edges = h->p.sigma_t = h->p.sigma_s = nullptr;
  h->nc = problems[0].n_chunks;
  h->fp32 = problems[0].precision == HWW_FP32;
  h->stream = stream;
  h->ws = ws;
  h->max_I = BL.max_I;
  h->max_K = BL.max_K;
  {
    // Per LDS class: the launch's LDS holds the largest need of its
    // replicas.  In class 2 (one work-group per compute unit) a replica
    // keeps its cell records in LDS when they fit beside its histogram.
    int fit[kBatchClasses] = {}, cnt[kBatchClasses] = {};
    const size_t cb = h->fp32 ? lds_cell_bytes<float>() : lds_cell_bytes<double>();
    for (int r = 0; r < n; ++r) {
      const int I = problems[r].n_cells, K = BL.L[r].geom.K, ci = BL.cls[r];
      const bool f = ci == 2 && sweep_lds_bytes(I, h->nc, K, cb) <= kLdsBytes;
      fit[ci] += f ? 1 : 0;
      ++cnt[ci];
      h->bcls[ci].lds = std::max(h->bcls[ci].lds, sweep_lds_bytes(I, h->nc, K, f ? cb : 0));
      h->bcls[ci].starts += problems[r].n_src;
      h->bcls[ci].n_rep += 1;
      h->bcls[ci].max_cells = std::max(h->bcls[ci].max_cells, I);
    }
    for (int ci = 0; ci < kBatchClasses; ++ci) {
      hww_handle::BatchClass &c = h->bcls[ci];
      c.u0 = BL.cls_u0[ci];
      c.u1 = BL.cls_u1[ci];
      c.cells_mode = fit[ci] == 0 ? 0 : (fit[ci] == cnt[ci] ? 1 : 2);
      c.block = ci == 0 ? 256 : (ci == 1 ? 512 : 1024);
      c.tile = kTile;
    }
  }
  h->n_units = (uint32_t)BL.units.size();
  h->desc = ws + BL.off_desc;
  h->units = reinterpret_cast<uint32_t *>(ws + BL.off_units);
  h->work = reinterpret_cast<uint32_t *>(ws + BL.off_work);
  h->err = reinterpret_cast<uint32_t *>(ws + BL.off_err);
  h->counters_all = reinterpret_cast<unsigned long long *>(ws + BL.off_counters);
  for (int k = 0; k < 2; ++k) {
    h->segcnt_all[k] = reinterpret_cast<uint32_t *>(ws + BL.off_seg[k]);
    h->ovfcnt_all[k] = reinterpret_cast<uint32_t *>(ws + BL.off_ovf[k]);
  }
  h->phi_cat = reinterpret_cast<double *>(ws + BL.off_phi);
  h->J_cat = reinterpret_cast<double *>(ws + BL.off_J);
  h->losm_tab = reinterpret_cast<LosmReplica *>(ws + BL.off_losm);
  h->bs_tab = reinterpret_cast<BeginStepArgs *>(ws + BL.off_bs);
  h->n_seg_all = BL.n_seg; h->n_ovf_all = BL.n_ovf;
  h->n_phi_all = BL.n_phi; h->n_J_all = BL.n_J;
  h->bdcap = BL.dcap;
  h->bq = queue_view<double>(ws, BL.off_q, 2 * (int64_t)kGridMax * BL.dcap);
  h->bq32 = queue_view<float>(ws, BL.off_q, 2 * (int64_t)kGridMax * BL.dcap);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
    h->cus = cus;
  for (int ci = 0; ci < kBatchClasses; ++ci) h->bcls[ci].grid = default_grid(h, h->bcls[ci].lds, h->bcls[ci].block);
  (void)losm_batch_lds(h->max_I, &h->losm_wil);

  auto bail = [&](int code) {
    g_init_error = h->msg;
    hww_destroy(h);
    return code;
  };
  // Replicas: member layouts whose small arrays sit in the shared ones.
  int64_t so = 0, oo = 0, po = 0, jo = 0;
  h->rep.resize(n, nullptr);
  for (int r = 0; r < n; ++r) {
    hww_handle *m = new hww_handle();
    h->rep[r] = m;
    carve_handle(m, problems[r], ws + BL.base[r], BL.L[r], stream);
    m->is_view = 1;
    const int64_t R = (int64_t)m->R, K = m->K;
    for (int k = 0; k < 2; ++k) {
      m->bank[k].segcnt = m->bank32[k].segcnt = h->segcnt_all[k] + so;
      m->bank[k].ovfcnt = m->bank32[k].ovfcnt = h->ovfcnt_all[k] + oo;
    }
    so += R * K;
    oo += R;
    m->counters = h->counters_all + (int64_t)r * 2 * C_NCOUNTERS;
    m->phi_out = h->phi_cat + po;
    m->J_out = h->J_cat + jo;
    po += m->I + 2;
    jo += m->I + 1;
    m->err = h->err;
    rc = prime_handle(m, problems[r]);
    if (rc != HWW_OK) {
      h->msg = "replica " + std::to_string(r) + ": " + m->msg;
      return bail(rc);
    }
  }
  HIPCHK(h, launch_fill_u32(h->work, 0u, 2 * kBatchClasses, h->stream));
  // Device tables.
  std::vector<ReplicaDesc<double>> d64(n);
  std::vector<ReplicaDesc<float>> d32(n);
  std::vector<LosmReplica> lt(n);
  std::vector<BeginStepArgs> bs(2 * (size_t)n);
  for (int r = 0; r < n; ++r) {
    hww_handle *m = h->rep[r];
    if (h->fp32) d32[r] = replica_desc<float>(m);
    else d64[r] = replica_desc<double>(m);
    lt[r].a = replica_losm_args(m);
    for (int k = 0; k < 2; ++k) {
      lt[r].tsum[k] = m->tsum[k];
      lt[r].bnd[k] = m->bnd[k];
      m->start_bank = m->cur_tal = k;
      bs[(size_t)k * n + r] = begin_args(m);
    }
    m->start_bank = m->cur_tal = 0;
  }
  if (h->fp32)
    rc = check_hip(h, hipMemcpyAsync(h->desc, d32.data(), sizeof(ReplicaDesc<float>) * n, hipMemcpyHostToDevice, stream), "desc");
  else
    rc = check_hip(h, hipMemcpyAsync(h->desc, d64.data(), sizeof(ReplicaDesc<double>) * n, hipMemcpyHostToDevice, stream), "desc");
  if (rc == HWW_OK) rc = check_hip(h, hipMemcpyAsync(h->units, BL.units.data(), 4 * BL.units.size(), hipMemcpyHostToDevice, stream), "units");
  if (rc == HWW_OK) rc = check_hip(h, hipMemcpyAsync(h->losm_tab, lt.data(), sizeof(LosmReplica) * n, hipMemcpyHostToDevice, stream), "losm table");
  if (rc == HWW_OK) rc = check_hip(h, hipMemcpyAsync(h->bs_tab, bs.data(), sizeof(BeginStepArgs) * bs.size(), hipMemcpyHostToDevice, stream), "step table");
  if (rc == HWW_OK) rc = check_hip(h, hipStreamSynchronize(stream), "sync");
  if (rc == HWW_OK) rc = poll_errors(h);
  if (rc != HWW_OK) return bail(rc);
  h->start_bank = 0;
  h->cur_tal = 0;
  h->step = 0;
  h->next_chunk = h->nc;
  sync_replica_state(h);
  *out = h;
  return HWW_OK;
}

int hww_batch_replica(hww_handle *h, int32_t r, hww_handle **view) {
  if (!h || !view) return HWW_E_INVALID_ARG;
  *view = nullptr;
  if (!h->is_batch) return fail(h, HWW_E_STATE, "not a batch");
  if (r < 0 || r >= (int32_t)h->rep.size()) return fail(h, HWW_E_INVALID_ARG, "replica out of range");
  *view = h->rep[r];
  return HWW_OK;
}

int hww_autotune(hww_handle *h, hww_tune_result *best) {
  if (!h || !best) return HWW_E_INVALID_ARG;
  if (h->is_view) return fail(h, HWW_E_STATE, "a replica view is read-only");
  if (h->fatal) return fail(h, h->fatal, "an earlier error left the problem invalid");
  if (h->step != 0) return fail(h, HWW_E_STATE, "the tuner runs before the first sweep");
  std::vector<hww_handle *> reps = h->is_batch ? h->rep : std::vector<hww_handle *>{h};
  // Save what a trial sweep changes beyond the banks and tally sets that the
  // first real step clears anyway: the source chunk weights and the counters.
  std::vector<double> wsave(reps.size() * (size_t)h->nc);
  const size_t ncnt = reps.size() * 2 * C_NCOUNTERS;
  std::vector<unsigned long long> csave(ncnt);
  unsigned long long *cdev = h->is_batch ? h->counters_all : h->counters;
  for (size_t r = 0; r < reps.size(); ++r)
    HIPCHK(h, hipMemcpyAsync(wsave.data() + r * h->nc, reps[r]->wnext, 8 * h->nc, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(csave.data(), cdev, 8 * ncnt, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(h, hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
  HIPCHK(h, hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
  auto clear_work = [&]() -> int {
    if (h->is_batch) HIPCHK(h, launch_fill_u32(h->work, 0u, 2 * kBatchClasses, h->stream));
    return HWW_OK;
  };
  // One trial: chunk 0 of step 1 under the shape (of a batch: LDS class ci
  // only), timed by events on the stream.
  auto trial = [&](int ci, int block, int tile, int grid, float *ms) -> int {
    if (h->is_batch) {
      h->bcls[ci].block = block;
      h->bcls[ci].tile = tile;
      h->bcls[ci].grid = grid;
    } else {
      h->block = block;
      h->tile = tile;
    }
    int rc = clear_work();
    if (rc != HWW_OK) return rc;
    flip_banks(h);
    rc = begin_step(h);
    if (rc == HWW_OK) rc = check_hip(h, hipEventRecord(e0, h->stream), "event");
    if (rc == HWW_OK) {
      if (h->is_batch) rc = h->fp32 ? launch_class<float>(h, ci, 0, 0) : launch_class<double>(h, ci, 0, 0);
      else rc = h->fp32 ? launch_chunk<float>(h, 0, 0) : launch_chunk<double>(h, 0, 0);
    }
    if (rc == HWW_OK) rc = check_hip(h, hipEventRecord(e1, h->stream), "event");
    if (rc == HWW_OK) rc = check_hip(h, hipStreamSynchronize(h->stream), "sync");
    if (rc == HWW_OK) rc = check_hip(h, hipEventElapsedTime(ms, e0, e1), "event");
    flip_banks(h);
    return rc;
  };
  const int blocks[3] = {256, 512, 1024};
  const int tiles[4] = {64, 128, 256, 512};
  int trials = 0, report = 0;
  float total_ms = 0.0f;
  int rc = HWW_OK;
  const int ncls = h->is_batch ? kBatchClasses : 1;
  int dev = 0;
  (void)hipGetDevice(&dev);
  for (int ci = 0; rc == HWW_OK && ci < ncls; ++ci) {
    if (h->is_batch && h->bcls[ci].u1 == h->bcls[ci].u0) continue;
    if (h->is_batch && h->bcls[ci].starts > h->bcls[report].starts) report = ci;
    TuneKey key;
    std::memset(&key, 0, sizeof key);
    key.dev = dev;
    key.fp32 = h->fp32;
    key.nc = h->nc;
    key.batch = h->is_batch;
    if (h->is_batch) {
      key.cls = ci;
      key.cells = h->bcls[ci].cells_mode;
      key.cells_bucket = log2_bucket(h->bcls[ci].max_cells);
      key.particles_bucket = log2_bucket(h->bcls[ci].starts);
      key.replicas = log2_bucket(h->bcls[ci].n_rep);
    } else {
      key.fission = h->cfis != nullptr;
      key.B = h->B;
      key.K = h->K;
      key.cells = h->cells_lds;
      key.cells_bucket = log2_bucket(h->I);
      key.particles_bucket = log2_bucket(h->p.n_src);
    }
    TuneShape hit;
    if (tune_lookup(key, &hit)) {
      if (h->is_batch) {
        h->bcls[ci].block = hit.block;
        h->bcls[ci].tile = hit.tile;
        h->bcls[ci].grid = hit.grid;
      } else {
        h->block = hit.block;
        h->tile = hit.tile;
      }
      total_ms += hit.ms;
      continue;
    }
    const size_t lds = h->is_batch ? h->bcls[ci].lds : h->lds;
    int bb = h->is_batch ? h->bcls[ci].block : h->block;
    int bt = h->is_batch ? h->bcls[ci].tile : h->tile;
    int bg = h->is_batch ? h->bcls[ci].grid : 0;
    float ms = 0.0f, best_ms = 0.0f;
    bool have = false;
    rc = trial(ci, bb, bt, bg, &ms);  // warm-up
    for (int bi = 0; rc == HWW_OK && bi < 3; ++bi) {
      std::vector<int> grids;
      if (h->is_batch) {
        for (int wpc = 1; wpc <= 4; ++wpc)
          if ((size_t)wpc * lds <= 160 * 1024 && wpc * blocks[bi] <= 2048 && h->cus * wpc <= kGridMax)
            grids.push_back(h->cus * wpc);
      } else {
        grids.push_back(0);
      }
      for (int g : grids)
        for (int ti = 0; rc == HWW_OK && ti < 4; ++ti) {
          float m = 0.0f, mbest = 1e30f;
          for (int rep = 0; rc == HWW_OK && rep < 2; ++rep) {
            rc = trial(ci, blocks[bi], tiles[ti], g, &m);
            mbest = std::min(mbest, m);
          }
          ++trials;
          if (rc == HWW_OK && (!have || mbest < best_ms)) {
            have = true;
            best_ms = mbest;
            bb = blocks[bi];
            bt = tiles[ti];
            bg = g;
          }
        }
    }
    if (h->is_batch) {
      h->bcls[ci].block = bb;
      h->bcls[ci].tile = bt;
      h->bcls[ci].grid = bg;
    } else {
      h->block = bb;
      h->tile = bt;
    }
    if (rc == HWW_OK && have) tune_store(key, TuneShape{bb, bt, bg, best_ms});
    total_ms += best_ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != HWW_OK) return rc;
  // Restore the state of step 0.
  for (size_t r = 0; r < reps.size(); ++r) {
    HIPCHK(h, hipMemcpyAsync(reps[r]->wnext, wsave.data() + r * h->nc, 8 * h->nc, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, launch_fill_f64(reps[r]->tal[1], 0.0, (int64_t)reps[r]->B * reps[r]->I * 6, h->stream));
    HIPCHK(h, launch_fill_f64(reps[r]->tsum[1], 0.0, (int64_t)kSumCopies * 6 * reps[r]->I, h->stream));
    HIPCHK(h, launch_fill_f64(reps[r]->bnd[1], 0.0, (int64_t)reps[r]->B * 6, h->stream));
    HIPCHK(h, launch_fill_u32(reinterpret_cast<uint32_t *>(reps[r]->tracks), 0u, 2 * (int64_t)reps[r]->I, h->stream));
  }
  HIPCHK(h, hipMemcpyAsync(cdev, csave.data(), 8 * ncnt, hipMemcpyHostToDevice, h->stream));
  h->ic_buf = -1;
  rc = clear_work();
  if (rc != HWW_OK) return rc;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  rc = poll_errors(h);
  if (rc != HWW_OK) return rc;
  if (h->is_batch) {
    best->block = h->bcls[report].block;
    best->tile = h->bcls[report].tile;
    best->grid = h->bcls[report].grid;
  } else {
    best->block = h->block;
    best->tile = h->tile;
    best->grid = h->B * h->K;
  }
  best->trials = trials;
  best->ms = total_ms;
  return HWW_OK;
}

int hww_set_timing(hww_handle *h, int32_t on) {
  if (!h) return HWW_E_INVALID_ARG;
  if (h->is_view) return fail(h, HWW_E_STATE, "a replica view is read-only");
  h->timing = on ? 1 : 0;
  return HWW_OK;
}

int hww_sync(hww_handle *h) {
  if (!h) return HWW_E_INVALID_ARG;
  return poll_errors(h);
}

const char *hww_last_error(const hww_handle *h) {
  return h ? h->msg.c_str() : g_init_error.c_str();
}

void hww_destroy(hww_handle *h) {
  if (!h || h->is_view) return;
  (void)hipStreamSynchronize(h->stream);
  destroy_events(h);
  for (hww_handle *r : h->rep) delete r;
  if (h->static_dev >= 0) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static_busy[h->static_dev] = false;
  }
  delete h;
}

}  // extern "C"
