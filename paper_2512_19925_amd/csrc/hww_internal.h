// Internal definitions shared by the HIP kernels and the host runtime of the
// hybrid weight-window sweep library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hww {

// Device error bits (ORed into one word of the workspace).
enum : uint32_t { ERR_CAPACITY = 1u, ERR_NUMERIC = 2u, ERR_SPLIT = 4u, ERR_GENERATIONS = 8u, ERR_DAUGHTERS = 16u,
                  ERR_COMB_WEIGHT = 32u };

// Counter slots (per step, uint64).
enum {
  C_SEGMENTS = 0, C_COLLISIONS, C_SCATTERS, C_ABSORPTIONS, C_CROSSINGS, C_LEAKS, C_CENSUS,
  C_SPLITS, C_DAUGHTERS, C_RR_KILL, C_RR_SURVIVE, C_HISTORIES, C_GENERATIONS, C_FISSIONS, C_FISSION_BIRTHS,
  C_NCOUNTERS = 16
};

// Random-number slots of the keying contract: key = (seed, (replica << 4) | slot),
// counter = (src, lineage lo, lineage hi, event index).
enum { SLOT_FLIGHT = 0, SLOT_EVENT = 1, SLOT_START = 2, SLOT_BIRTH = 3, SLOT_LIN_EVENT = 4,
       SLOT_LIN_START = 5, SLOT_FISSION_DIR = 6, SLOT_COMB = 7 };

// Work-group-local daughter generations per launch before giving up.
constexpr int kMaxGenerations = 4096;

// Batch-summed tallies: every sweep work-group adds its histogram into copy
// (work-group index mod kSumCopies) of [copy][6][I] (column-major), besides
// its batch's row of [B][I][6]; an LOSM solve adds the copies up.  More copies
// would spread the atomics of the flush over more addresses, but the flushes
// of a launch are spread in time enough that one copy does not slow the
// sweep, and each further copy costs the solve loads.
constexpr int kSumCopies = 1;

// Position and direction of a particle (one 16-byte load in FP64).
template <typename Real>
struct alignas(2 * sizeof(Real)) XMu {
  Real x, mu;
};
// Identity of a particle: source history, event index, cell.
struct Tag {
  uint32_t src, e;
  int32_t cell;
};
// Weight and remaining time of a daughter (one 16-byte load).
struct alignas(16) WTau {
  double w, tau;
};
// Per-cell data read by every flight, in the flight precision: edges,
// 1/sigma_t, sigma_s/sigma_t.
template <typename Real>
struct alignas(4 * sizeof(Real)) CellData {
  Real xl, xr, inv_sig, c;
};
// Per-cell weight window: centre, ceiling, floor.
struct alignas(32) Window {
  double ww, ceil, floor, pad;
};

// Particle bank as four structure-of-arrays streams.  Region (batch b,
// chunk c) holds the particles of batch b whose next step starts in chunk c.
// It is cut into K segments of seg_cap slots, segment j written only by
// work-group j of batch b (so appends need only a work-group-local counter),
// and one overflow segment of ovf_cap slots shared through a device atomic.
template <typename Real>
struct Bank {
  XMu<Real> *xm;
  double *w;
  uint64_t *lin;
  Tag *tag;
  uint32_t *segcnt;  // [B][nc][K]
  uint32_t *ovfcnt;  // [B][nc]
};

struct BankGeom {
  int32_t K;
  int64_t seg_cap, ovf_cap, stride;  // stride = K * seg_cap + ovf_cap slots per region
};

// Daughter buffers: two per work-group, dcap slots each.
template <typename Real>
struct Queue {
  XMu<Real> *xm;
  WTau *wt;
  uint64_t *lin;
  Tag *tag;
};

template <typename Real>
struct SweepArgs {
  int32_t I, B, nc;
  double v, inv_v, dt;
  uint32_t seed, key1;  // key1 = replica << 4
  const CellData<Real> *cells;  // [I]
  const Window *win;       // [I]
  const double *cfis;      // [I] (sigma_s + sigma_f) / sigma_t, or null: no fission
  double nu_f;             // mean neutrons per fission
  int32_t track_moments;   // 3: phi, J, K per segment; 2: phi, K; 1: phi
  int32_t ww_on;
  int32_t chunk;
  int32_t tile;            // start-bank / daughter tile a wave claims at a time
  BankGeom geom;
  Bank<Real> in_bank;
  Bank<Real> census;
  Queue<Real> dq;
  int64_t dcap;
  double *tal;                     // [B][I][6]
  double *tsum;                    // [kSumCopies][6][I] batch sums of tal
  double *bnd;                     // [B][2][3]
  unsigned long long *tracks;      // [I]
  unsigned long long *counters;    // [2][C_NCOUNTERS]: this step, since init
  double *wnext;                   // [nc]
  uint32_t *err;
};

// One replica of a batched problem: everything a sweep unit of the replica
// needs, with both banks and both tally sets; the launch
// selects the current ones.
template <typename Real>
struct ReplicaDesc {
  int32_t I, B, nc;
  double v, inv_v, dt;
  uint32_t seed, key1;
  const CellData<Real> *cells;
  const Window *win;
  int32_t track_moments;
  int32_t cells_lds;   // the replica's cell records fit in LDS beside its histogram
  BankGeom geom;
  Bank<Real> bank[2];
  double *tal[2], *tsum[2], *bnd[2];
  unsigned long long *tracks, *counters;
  double *wnext;
};

// Persistent launch over the work units (replica, batch, segment) of all
// replicas: unit code = replica << 16 | batch << 8 | segment.
template <typename Real>
struct BatchSweepArgs {
  const ReplicaDesc<Real> *desc;
  const uint32_t *units;
  uint32_t n_units;
  uint32_t *work;      // [2] unit counters; launch parity `par` uses work[par]
  int32_t par;         // unit counter of this launch (the other one is cleared for the next)
  int32_t start_bank;  // start bank and current tally set
  int32_t chunk, ww_on, tile;
  Queue<Real> dq;      // daughter buffers: 2 per work-group of the grid
  int64_t dcap;
  uint32_t *err;
};

// Uniform comb of a census bank (src_bank, geometry G, R = B * nc regions)
// into dst_bank.  Scratch: per-history counts and offsets (n_hist + 1),
// cursors (n_hist), the canonical order of the census slots and the
// integer weights / their prefix sums (cap each), scan block sums, and
// misc[8] = {max weight bits, census count, W, eu, xi bits, ...}.
template <typename Real>
struct CombArgs {
  Bank<Real> src_bank, dst_bank;
  BankGeom G;
  int32_t B, nc, R;
  int64_t n_hist;              // bound on src values + 1 of the census
  int64_t cap;                 // bound on census particles
  int64_t n_target;
  int32_t by_index;            // 1: teeth spaced in particle index, each copy keeping its
                               // particle's weight times n / n_target; 0: spaced in
                               // cumulative weight, every copy of weight W / n_target
  int32_t no_wait;             // 1: the host will not read the census size, so an empty or
                               // invalid census leaves an empty combed bank (and, if
                               // invalid, ERR_COMB_WEIGHT) for it to take as the census
  uint32_t seed, key1, step;
  unsigned long long *cnt;     // [n_hist + 1] counts, then exclusive offsets
  uint32_t *cur;               // [n_hist]
  unsigned long long *order;   // [cap] slot index of the census particle at each canonical position
  unsigned long long *wq;      // [cap] integer weights, then inclusive prefix sums
  unsigned long long *blk;     // scan block sums
  unsigned long long *misc;    // [8]: largest weight's bits, count, total weight, -, long histories
  double *wnext;               // [nc]
  uint32_t *err;
};

struct BeginStepArgs {
  uint32_t *segcnt, *ovfcnt;
  double *tal, *tsum, *bnd;
  unsigned long long *tracks, *counters;
  double *wstart, *wnext;
  int64_t n_seg, n_ovf, n_tal, n_tsum, n_bnd, n_tracks;
  int32_t nc;
};

struct SourceArgs {
  int32_t I, B, nc;
  double v, dt, src_x;
  int64_t n_src;
  uint32_t seed, key1;
  const double *edges;
  BankGeom geom;
  double *tal;   // census part of [B][I][6]
  double *tsum;  // and of its batch sums
  double *wnext;
  uint32_t *err;
};

struct LosmArgs {
  int32_t I, B, nc;
  double v, dt, n_src;
  const double *edges, *sig_t, *sig_s;
  const double *tsum_ic, *bnd_ic;  // tally set of the initial condition (census at t^{n-1}):
                                   // batch-sum copies [kSumCopies][6][I], faces [B][2][3]
  const double *tsum_cl, *bnd_cl;  // tally set of the closures (same as the initial condition's
                                   // when semi-implicit)
  const double *wstart, *wnext;   // [nc] chunk weights of the start bank / census bank
  int32_t next_chunk;             // chunks already swept in the step (implicit solve)
  double theta;
  int32_t implicit, filter, ma_k, closure_track, apply_windows;
  int32_t kappa, lagged;          // Fourier cutoff; windows from the previous step's track flux
  int32_t window_scale;           // 1: centres as printed (max 1), 0: times start weight / n_src
  double eps_min, rho;
  double *scratch;                // >= 24 * (I + 4) doubles
  double *factor;                 // [4][2I+3] LU factors of the system for `theta`, old-time diagonal
  int32_t refactor;               // 1: (re)compute the factors first
  int32_t work_in_lds;            // set by the launcher: grid functions fit in LDS
  int32_t ic_cached;              // 1: the initial condition's sums are already in the scratch
  int32_t export_only;            // 1: write phi^{n-1}, J^{n-1}, F^{n-1}, P^{n-1} and stop
  double *F_out, *P_out;          // I+2, 2 (device) for export_only
  Window *win;                    // [I] window centres, ceilings, floors
  double *phi_out, *J_out;        // I+2, I+1 (device)
  uint32_t *err;
  int32_t *status;                // 0 ok, else error bits of this solve
};

// One replica of a batched LOSM solve: its arguments with both tally sets;
// the per-call options come from LosmCall.
struct LosmReplica {
  LosmArgs a;
  const double *tsum[2], *bnd[2];
};
struct LosmCall {
  int32_t cur;  // current tally set
  int32_t implicit, next_chunk, filter, ma_k, closure_track, apply_windows, export_only, refactor, work_in_lds;
  int32_t kappa, lagged, ic_cached, window_scale;
  double theta, eps_min, rho;
};

// Deterministic LOSM march and its adjoint (one work-group each).
struct MarchArgs {
  int32_t I, n_steps;
  double v, dt, theta;
  const double *edges, *sig_t, *sig_s;  // cross sections of the march
  const double *F, *P;                  // (n_steps+1) x (I+2), (n_steps+1) x 2
  const double *phi0, *J0;              // I+2, I+1
  const double *w;                      // (n_steps+1) x (I+2) functional weights on phi
  double *factor, *factor_t;            // 3 (2I+3) each: factors of A and A^T
  double *hist;                         // (n_steps+1) x (2I+3) interleaved u^n
  double *G;                            // functional value
  double *g_t, *g_s;                    // I each
  uint32_t *err;
};

// Dynamic LDS of the sweep and source kernels: [I][6] + nc + 6 doubles for
// the histogram, then 32-bit words for segment counts, counters, the tile counter and
// the start-bank tile table.  A sweep that keeps the per-cell records in
// LDS puts them first (cell_bytes per cell: CellData and Window).
__host__ __device__ inline size_t lds_doubles(int I, int nc) { return (size_t)I * 6 + nc + 6; }
__host__ __device__ inline size_t lds_words(int I, int K) { return (size_t)I + 16 + 8 + 2 + 2 + 2 + 1 + 1 + (K + 2) + (K + 1); }
inline size_t sweep_lds_bytes(int I, int nc, int K, size_t cell_bytes = 0) {
  return (size_t)I * cell_bytes + lds_doubles(I, nc) * 8 + lds_words(I, K) * 4;
}
template <typename Real>
constexpr size_t lds_cell_bytes() { return sizeof(CellData<Real>) + sizeof(Window); }
constexpr size_t kLdsBytes = 160 * 1024;  // LDS of one gfx950 compute unit

// Launchers (defined in the .hip files).
template <typename Real>
hipError_t launch_sweep(const SweepArgs<Real> &a, bool cells_lds, int grid, int block, size_t lds, hipStream_t s);
template <typename Real>
hipError_t launch_source(const SourceArgs &a, const Bank<Real> &bank, int grid, int block, size_t lds,
                         hipStream_t s);
template <typename Real>
hipError_t launch_sweep_batch(const BatchSweepArgs<Real> &a, int cells_mode, int grid, int block, size_t lds,
                              hipStream_t s);
hipError_t launch_losm(const LosmArgs &a, hipStream_t s);
hipError_t launch_losm_batch(const LosmReplica *tab, int n, int max_I, const LosmCall &c, hipStream_t s);
size_t losm_batch_lds(int max_I, int *work_in_lds);
hipError_t launch_begin_step_batch(const BeginStepArgs *tab, int n, int64_t max_tal, hipStream_t s);
template <typename Real>
hipError_t launch_comb(const CombArgs<Real> &a, hipStream_t s);
int64_t comb_scan_blocks(int64_t n);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s);
hipError_t launch_rotate_chunks(double *wstart, double *wnext, int nc, hipStream_t s);
hipError_t launch_begin_step(const BeginStepArgs &a, hipStream_t s);
hipError_t launch_march(const MarchArgs &a, hipStream_t s);
hipError_t launch_adjoint(const MarchArgs &a, hipStream_t s);

}  // namespace hww
