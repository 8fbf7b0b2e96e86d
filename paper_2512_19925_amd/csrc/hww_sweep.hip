// Particle sweep of one chunk of a time step of the hybrid weight-window
// Monte Carlo method (Shaw & Anistratov, arXiv 2512.19925): flight,
// collision and census of a 1D slab bank (Sec. 3, Eq. HO_transport),
// track-length and time-crossing tallies (Sec. 3, Eqs. phi-mc, ct-mc),
// and split / Russian roulette against weight windows (Sec. 2).
//
// Launch shape: grid = B * K work-groups; work-group g serves batch
// b = g mod B and owns segment j = g / B of every census region of that
// batch.  Consequences:
//  - all lanes of a wave belong to one batch, so the work-group keeps the
//    batch's tallies in an LDS histogram flushed to HBM once per launch;
//  - census appends need only a work-group-local LDS counter (a shared
//    overflow segment takes what does not fit);
//  - daughters split off by the work-group go to its own buffer and are
//    transported by the same work-group in further generations, so no
//    work-group ever waits for another and the host never waits at all.
// Each wave keeps its 64 lanes busy: a lane whose particle ends (census,
// leak, absorption, roulette) refills from the wave's current tile.
#include "hww_internal.h"
#include "hww_rng_dev.h"

namespace hww {

// Daughters of a generation that waves out of their own tiles take early
// even when no wave has tiles of its own left.
constexpr uint32_t kDrainSmall = 256;
// A wave whose lanes each have at most this many daughters to write lets
// every lane write its own; above it the wave writes them 64 at a time.
constexpr uint32_t kLaneDaughters = 4;

// Window and event actions of a lane (bit flags).
enum : uint32_t { WW_ROULETTE = 1u, WW_SPLIT = 2u, EV_DRAW = 4u, EV_SCATTER = 8u, EV_FISSION = 16u,
                  FIS_BIRTHS = 32u };

// ln v of a positive normal v by fixed steps, so that every IEEE-double
// implementation of the same steps (the CPU check of this sweep has one)
// gives the same bits: v = (1 + f) 2^k with 1 + f in [sqrt(1/2), sqrt(2)),
// s = f / (2 + f), ln(1 + f) = 2 atanh(s) = f - (h - s (h + R)) with
// h = f^2 / 2 and R = sum_{j=1..9} 2 z^j / (2j + 1), z = s^2 (the rounding
// of s only touches the small s (h + R) term), plus k ln 2 with ln 2 split
// in two doubles.  Within one ulp of ln v.
__device__ __forceinline__ double log_r(double v) {
  int k;
  double m = frexp(v, &k);
  if (m < 0.70710678118654752440) {
    m = m * 2.0;
    k = k - 1;
  }
  const double f = m - 1.0;
  const double s = f / (2.0 + f);
  const double z = s * s;
  double q = 2.0 / 19.0;
  q = __builtin_fma(q, z, 2.0 / 17.0);
  q = __builtin_fma(q, z, 2.0 / 15.0);
  q = __builtin_fma(q, z, 2.0 / 13.0);
  q = __builtin_fma(q, z, 2.0 / 11.0);
  q = __builtin_fma(q, z, 2.0 / 9.0);
  q = __builtin_fma(q, z, 2.0 / 7.0);
  q = __builtin_fma(q, z, 2.0 / 5.0);
  q = __builtin_fma(q, z, 2.0 / 3.0);
  const double R = z * q;
  const double h = 0.5 * f * f;
  const double kd = (double)k;
  const double c = __builtin_fma(kd, 2.3190468138462996e-17, s * (h + R));
  const double u = f - (h - c);
  return __builtin_fma(kd, 0.69314718055994528623, u);
}
__device__ __forceinline__ float log_r(float v) { return logf(v); }

__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
  return (uint32_t)__popcll(m & __lanemask_lt());
}

__device__ __forceinline__ int first_lane(uint64_t m) { return __ffsll((long long)m) - 1; }

// Cell of x; a point on an interior edge belongs to the cell it moves into.
__device__ __forceinline__ int32_t find_cell(const double *edges, int I, double x, double mu) {
  if (x <= edges[0]) return 0;
  if (x >= edges[I]) return I - 1;
  int32_t lo = 0, hi = I;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) / 2;
    if (edges[mid] <= x) lo = mid; else hi = mid;
  }
  if (x == edges[lo] && mu < 0.0 && lo > 0) lo -= 1;
  return lo;
}

// Events of a lane in one pass of the event loop (bit flags), counted per
// wave by ballots: no per-lane counter registers.  A lane can pass a
// start-of-step check and a post-event check in the same pass, so the
// start-of-step outcomes that leave it alive have bits of their own.
enum : uint32_t {
  EVB_CENSUS = 1u, EVB_LEAK = 2u, EVB_CROSS = 4u, EVB_SCATTER = 8u, EVB_ABSORB = 16u,
  EVB_RR_SURVIVE = 32u, EVB_RR_KILL = 64u, EVB_SPLIT = 128u, EVB_START_SURVIVE = 256u, EVB_START_SPLIT = 512u,
  EVB_FISSION = 1024u
};
constexpr int kEventKinds = 11;
constexpr uint32_t kRareEvents = EVB_LEAK | EVB_RR_SURVIVE | EVB_RR_KILL | EVB_SPLIT | EVB_START_SURVIVE |
                                 EVB_START_SPLIT | EVB_FISSION;
__device__ constexpr int kEventSlot[kEventKinds] = {C_CENSUS, C_LEAKS, C_CROSSINGS, C_SCATTERS, C_ABSORPTIONS,
                                                    C_RR_SURVIVE, C_RR_KILL, C_SPLITS, C_RR_SURVIVE, C_SPLITS,
                                                    C_FISSIONS};

// Shared-memory carve-up common to the sweep and source kernels.
struct Lds {
  double *hist;     // [I][6]
  double *wnext;    // [nc]
  double *bnd;      // [6]
  uint32_t *trk;    // [I]
  uint32_t *cnt;    // [16]
  uint32_t *ccnt;   // [8]   census appends of this work-group per chunk
  uint32_t *dcnt;   // [2]   daughter slots taken in each buffer
  uint32_t *dready; // [2]   daughters of each buffer written (visible to the work-group)
  uint32_t *dtake;  // [2]   daughters taken from a buffer while it is still written
  uint32_t *obusy;  // [1]   waves still taking tiles of their own in this generation
  uint32_t *dcur;   // [1]   tile counter: start-bank tiles (generation 0), then daughter slots
  uint32_t *tstart; // [K+2] first tile of each start-bank segment
  uint32_t *nseg;   // [K+1] particles of each start-bank segment
};


__device__ inline Lds carve(double *raw, int I, int nc, int K) {
  Lds L;
  L.hist = raw;
  L.wnext = raw + (size_t)I * 6;
  L.bnd = L.wnext + nc;
  L.trk = reinterpret_cast<uint32_t *>(L.bnd + 6);
  L.cnt = L.trk + I;
  L.ccnt = L.cnt + 16;
  L.dcnt = L.ccnt + 8;
  L.dready = L.dcnt + 2;
  L.dtake = L.dready + 2;
  L.obusy = L.dtake + 2;
  L.dcur = L.obusy + 1;
  L.tstart = L.dcur + 1;
  L.nseg = L.tstart + (K + 2);
  return L;
}

__device__ inline void zero_lds(double *raw, int I, int nc, int K) {
  const size_t nd = lds_doubles(I, nc);
  for (size_t t = threadIdx.x; t < nd; t += blockDim.x) raw[t] = 0.0;
  uint32_t *w = reinterpret_cast<uint32_t *>(raw + nd);
  const size_t nw = lds_words(I, K);
  for (size_t t = threadIdx.x; t < nw; t += blockDim.x) w[t] = 0u;
}

// Flush the work-group histogram of batch b (nonzero entries only) into
// the batch's row and into copy `copy` of the batch sums.
__device__ inline void flush_tallies(const Lds &L, int I, int nc, int b, double *tal, double *tsum, int copy,
                                     double *bnd, unsigned long long *tracks, double *wnext) {
  double *tal_b = tal + (size_t)b * I * 6;
  double *sum_c = tsum + (size_t)copy * 6 * I;
  for (int j = threadIdx.x; j < I * 6; j += blockDim.x) {
    const double val = L.hist[j];
    if (val != 0.0) {
      unsafeAtomicAdd(&tal_b[j], val);
      const int i = j / 6, k = j - 6 * i;
      unsafeAtomicAdd(&sum_c[k * I + i], val);
    }
  }
  if (tracks) {
    for (int j = threadIdx.x; j < I; j += blockDim.x) {
      const uint32_t t = L.trk[j];
      if (t != 0) atomicAdd(&tracks[j], (unsigned long long)t);
    }
  }
  if (bnd && threadIdx.x < 6) {
    const double val = L.bnd[threadIdx.x];
    if (val != 0.0) unsafeAtomicAdd(&bnd[b * 6 + threadIdx.x], val);
  }
  if (threadIdx.x < (unsigned)nc) {
    const double val = L.wnext[threadIdx.x];
    if (val != 0.0) unsafeAtomicAdd(&wnext[threadIdx.x], val);
  }
}

template <typename Real>
__device__ inline void store_record(const Bank<Real> &bk, int64_t k, Real x, Real mu, double w,
                                    uint64_t lin, uint32_t src, uint32_t e, int32_t cell) {
  XMu<Real> xm;
  xm.x = x;
  xm.mu = mu;
  bk.xm[k] = xm;
  bk.w[k] = w;
  bk.lin[k] = lin;
  Tag t;
  t.src = src;
  t.e = e;
  t.cell = cell;
  bk.tag[k] = t;
}

// Append the census particles of the wave to the regions (b, c) of their
// next-step chunks c: each census lane takes the next slot of its chunk's
// count in the work-group (one LDS atomic), in the work-group's own segment
// j; what does not fit goes to the shared overflow segment.  The order of
// the records within a segment is free (the bank is a multiset).
template <typename Real>
__device__ inline void census_append(const Bank<Real> &bk, const BankGeom &G, uint32_t *ccnt, uint32_t *ovfcnt_b,
                                     int64_t region_b0, int nc, int j, bool mine, int c, Real x, Real mu,
                                     double w, uint64_t lin, uint32_t src, uint32_t e, int32_t cell,
                                     uint32_t *err) {
  const int lane = (int)__lane_id();
  if (__ballot(mine) == 0) return;
  uint32_t slot = 0;
  if (mine) slot = atomicAdd(&ccnt[c], 1u);
  const bool in_seg = mine && slot < (uint32_t)G.seg_cap;
  // Region (b, c) starts c strides after the batch's first region; segment
  // j of a region j seg_cap slots in.
  int64_t k = -1;
  if (in_seg) k = region_b0 + (int64_t)j * G.seg_cap + (int64_t)c * G.stride + (int64_t)slot;
  if (__ballot(mine && !in_seg) != 0) {
    for (int cc = 0; cc < nc; ++cc) {
      const bool over = mine && !in_seg && c == cc;
      const uint64_t om = __ballot(over);
      if (om == 0) continue;
      const int ol = first_lane(om);
      uint32_t ob = 0;
      if (lane == ol) ob = atomicAdd(&ovfcnt_b[cc], (uint32_t)__popcll(om));
      ob = __shfl(ob, ol);
      if (over) {
        const uint64_t os = (uint64_t)ob + rank_below(om);
        if (os < (uint64_t)G.ovf_cap) k = region_b0 + (int64_t)cc * G.stride + (int64_t)G.K * G.seg_cap + (int64_t)os;
        else atomicOr(err, ERR_CAPACITY);
      }
    }
  }
  if (k >= 0) store_record(bk, k, x, mu, w, lin, src, e, cell);
}

// One work unit: the particles of chunk A.chunk in the start-bank region of
// batch b, tiles jseg, jseg + K, jseg + 2K, ... of it (claimed by the waves
// through a work-group counter in LDS), and all their daughters, with census
// appends into segment jseg of the batch's regions.  The work-group's
// daughter buffers are number qslot of nq.  With kCellsLds the per-cell
// records are copied into LDS first.  Starts and ends with the LDS free for
// reuse.  kFission compiles the fission branch of collisions in (problems
// with fission cross sections); without it the kernel is the plain sweep.
template <typename Real, bool kCellsLds, bool kFission>
__device__ __forceinline__ void sweep_unit(const SweepArgs<Real> &A, int b, int jseg, int qslot, int nq,
                                           double *lds_raw) {
  const int I = A.I, nc = A.nc;
  const BankGeom G = A.geom;
  const int K = G.K;
  const uint32_t TILE = (uint32_t)A.tile;
  const CellData<Real> *cellp = A.cells;
  const Window *winp = A.win;
  const int tid = threadIdx.x;
  const int r_in = b * nc + A.chunk;
  const int64_t in_region = (int64_t)r_in * G.stride;
  // Sizes of the start region's segments (lane s of wave 0 takes segment s,
  // the overflow segment at s = K; with K = 64 lane 0 takes the overflow
  // segment as well) and this unit's census counts, loaded before the LDS
  // set-up so that their latency overlaps it.
  uint32_t n_s = 0, n_ovf64 = 0, cen = 0;
  if (tid < 64) {
    if (tid < K) n_s = (uint32_t)min((int64_t)A.in_bank.segcnt[r_in * K + tid], G.seg_cap);
    else if (tid == K) n_s = (uint32_t)min((int64_t)A.in_bank.ovfcnt[r_in], G.ovf_cap);
    if (K == 64 && tid == 0) n_ovf64 = (uint32_t)min((int64_t)A.in_bank.ovfcnt[r_in], G.ovf_cap);
  }
  if (tid < nc) cen = A.census.segcnt[(b * nc + tid) * K + jseg];
  if constexpr (kCellsLds) {
    CellData<Real> *sc = reinterpret_cast<CellData<Real> *>(lds_raw);
    Window *sw = reinterpret_cast<Window *>(sc + I);
    for (int j = threadIdx.x; j < I; j += blockDim.x) {
      sc[j] = A.cells[j];
      sw[j] = A.win[j];
    }
    cellp = sc;
    winp = sw;
    lds_raw = reinterpret_cast<double *>(sw + I);
  }
  Lds L = carve(lds_raw, I, nc, K);
  zero_lds(lds_raw, I, nc, K);
  __syncthreads();
  // Tile table: first tile of each start segment (a wave-wide prefix sum of
  // the segments' tile counts) and the total.
  if (tid < 64) {
    const uint32_t t_s = (n_s + TILE - 1u) / TILE;
    uint32_t incl = t_s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o);
      if (tid >= o) incl += y;
    }
    if (tid <= K) {
      L.nseg[tid] = n_s;
      L.tstart[tid] = incl - t_s;
    }
    const uint32_t total = __shfl(incl, 63);
    if (tid == 0) {
      if (K == 64) {
        L.nseg[64] = n_ovf64;
        L.tstart[64] = total;
        L.tstart[65] = total + (n_ovf64 + TILE - 1u) / TILE;
      } else {
        L.tstart[K + 1] = total;
      }
      L.obusy[0] = blockDim.x >> 6;
    }
  }
  if (tid < nc) L.ccnt[tid] = cen;
  __syncthreads();

  const uint32_t lane = __lane_id();
  const double v = A.v;
  const Real v_r = (Real)A.v, inv_v_r = (Real)A.inv_v, dt_r = (Real)A.dt;
  const int64_t dstride = A.dcap;

  // Lane state: position, direction and remaining time in the flight
  // precision, weight in FP64.
  Real x = 0, mu = 0, tau = 0;
  double w = 0.0;
  int32_t cell = 0;
  uint32_t src = 0, e = 0;
  uint64_t lin = 0;
  bool active = false;
  // Window check still due for the lane's particle in its cell: the
  // start-of-step check of a particle just loaded from the bank, or the
  // check after a crossing (made at the top of the next pass, where the new
  // cell's record is read anyway; the particle does nothing in between).
  uint32_t pend = 0u;
  // Pending split or fission of this lane: the daughters copy the lane
  // state (a fission daughter draws its own direction).
  uint32_t nd = 0;
  uint64_t lin_base = 0;
  uint32_t e_d = 0;
  bool fis = false;
  uint32_t evb = 0u;  // EVB_* events not yet counted
  uint32_t pub = 0u;  // daughters the wave has written but not yet counted as written
  int out_buf = 0;

  // Count the wave's pending events (converged): the common kinds into
  // wave-uniform totals (scalar registers) added to the work-group counters
  // once, at the end of the unit; the rare ones into the work-group
  // counters behind a single ballot.  Crossings are not counted here; every
  // segment adds one to its cell's track counter, so they follow from the
  // segment total at the end.
  auto count_kind = [&](int q) {
    const uint64_t m = __ballot(((evb >> q) & 1u) != 0u);
    if (m != 0 && lane == 0) atomicAdd(&L.cnt[kEventSlot[q]], (uint32_t)__popcll(m));
  };
  uint32_t n_census = 0, n_scatter = 0, n_absorb = 0, n_hist = 0;  // n_hist: start particles taken
  auto count_events = [&]() {
    n_census += (uint32_t)__popcll(__ballot((evb & EVB_CENSUS) != 0u));
    n_scatter += (uint32_t)__popcll(__ballot((evb & EVB_SCATTER) != 0u));
    n_absorb += (uint32_t)__popcll(__ballot((evb & EVB_ABSORB) != 0u));
    if (__ballot((evb & kRareEvents) != 0u) != 0) {
      count_kind(1);
#pragma unroll
      for (int q = 5; q < kEventKinds; ++q) count_kind(q);
    }
    evb = 0u;
  };

  // Count the wave's written daughters as written (for the waves that take
  // daughters early) once the release fence has made the records visible
  // to the work-group.
  auto publish = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane == 0) atomicAdd(&L.dready[out_buf], pub);
    pub = 0u;
  };

  // Write the pending daughters of all lanes of the wave into the work-
  // group's buffer `out_buf` (converged call).
  auto flush_daughters = [&]() {
    const uint32_t cntd = nd > 1 ? nd - 1 : 0;
    uint32_t incl = cntd;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t t = __shfl_up(incl, o);
      if ((int)lane >= o) incl += t;
    }
    const uint32_t total = __shfl(incl, 63);
    if (total != 0) {
      // Split daughters are counted here; fission neutrons at the fission.
      uint32_t nsplit = (kFission && fis) ? 0u : cntd;
      if (kFission && __ballot(fis && cntd != 0) != 0) {
        for (int o = 32; o >= 1; o >>= 1) nsplit += __shfl_xor(nsplit, o);
      } else {
        nsplit = total;
      }
      if (lane == 0 && nsplit != 0) atomicAdd(&L.cnt[C_DAUGHTERS], nsplit);
      uint32_t base = 0;
      if (lane == 0) base = atomicAdd(&L.dcnt[out_buf], total);
      base = __shfl(base, 0);
      if ((uint64_t)base + total > (uint64_t)A.dcap && lane == 0) atomicOr(A.err, ERR_DAUGHTERS);
      const int64_t qb = ((int64_t)out_buf * nq + qslot) * dstride;
      // Daughter q = 1..n of a lane goes to slot base + (its lane's offset
      // in the wave) + q - 1, with lineage base + q.
      auto write_daughter = [&](uint32_t g, uint32_t q, Real dx, Real dmu, double dw, Real dtau, uint32_t dsrc,
                                uint64_t dlin, uint32_t de, int32_t dcell, bool dfis) {
        const uint64_t slot = (uint64_t)base + g;
        if (slot >= (uint64_t)A.dcap) return;
        const int64_t k = qb + (int64_t)slot;
        XMu<Real> xm;
        xm.x = dx;
        xm.mu = dmu;
        if (kFission && dfis) {
          uint32_t rd[4];
          draw(A.seed, A.key1, SLOT_FISSION_DIR, dsrc, dlin + q, de, rd);
          xm.mu = (Real)2 * uflight<Real>(rd[0], rd[1]) - (Real)1;
        }
        A.dq.xm[k] = xm;
        WTau wt;
        wt.w = dw;
        wt.tau = (double)dtau;
        A.dq.wt[k] = wt;
        A.dq.lin[k] = dlin + q;
        Tag tg;
        tg.src = dsrc;
        tg.e = de;
        tg.cell = dcell;
        A.dq.tag[k] = tg;
      };
      const uint32_t excl = incl - cntd;
      if (__ballot(cntd > kLaneDaughters) == 0) {
        // Few per lane: each lane writes its own.
        for (uint32_t q = 1; q <= cntd; ++q)
          write_daughter(excl + q - 1, q, x, mu, w, tau, src, lin_base, e_d, cell, kFission && fis);
      } else {
        // Many in some lane (a heavy split): the wave writes 64 daughters
        // per pass, lane l the (64 j + l)-th of the wave, reading its
        // parent's state from the parent's lane.
        for (uint32_t j0 = 0; j0 < total; j0 += 64) {
          const uint32_t g = j0 + lane;
          // Parent: the first lane whose inclusive count exceeds g.
          int sl = 0;
#pragma unroll
          for (int step = 32; step >= 1; step >>= 1)
            if (__shfl(incl, sl + step - 1) <= g) sl += step;
          if (sl > 63) sl = 63;
          const Real px = __shfl(x, sl), pmu = __shfl(mu, sl), ptau = __shfl(tau, sl);
          const double pw = __shfl(w, sl);
          const uint32_t psrc = __shfl(src, sl), pe = __shfl(e_d, sl), pexcl = __shfl(excl, sl);
          const int32_t pcell = __shfl(cell, sl);
          const uint64_t plin = __shfl(lin_base, sl);
          const bool pfis = kFission && __shfl((int)fis, sl) != 0;
          if (g < total) write_daughter(g, g - pexcl + 1, px, pmu, pw, ptau, psrc, plin, pe, pcell, pfis);
        }
      }
      pub += total;
      publish();
    }
    nd = 0;
  };

  // Weight-window check of the lane's particle in its cell (Sec. 2), in
  // two parts so that the random draws of all lanes of a wave are made by
  // one converged call per kind.  classify() decides from the weight alone:
  // 0 inside the window, WW_ROULETTE below the floor, WW_SPLIT above the
  // ceiling (an impossible split raises an error and ends the particle).
  auto classify = [&](const Window &wd) -> uint32_t {
    if (!A.ww_on) return 0u;
    if (w > wd.ceil) {
      const double ndf = ceil(w / wd.ww);
      if (!(ndf >= 2.0) || ndf > 1.0e9) {
        atomicOr(A.err, ERR_SPLIT);
        active = false;
        return 0u;
      }
      if (ndf - 1.0 > (double)A.dcap) {
        atomicOr(A.err, ERR_DAUGHTERS);
        active = false;
        return 0u;
      }
      return WW_SPLIT;
    }
    return w < wd.floor ? WW_ROULETTE : 0u;
  };
  // Roulette with the uniform xi: survive at the window centre or die.
  auto roulette = [&](double xi, double ww, bool at_start) {
    if (xi < w / ww) {
      w = ww;
      evb |= at_start ? EVB_START_SURVIVE : EVB_RR_SURVIVE;
    } else {
      evb |= EVB_RR_KILL;
      active = false;
    }
  };
  // Split into N_d = ceil(w / ww) equal daughters; the lane keeps daughter
  // 0, the others take lineage base + j and the event index e_daughter.
  auto split = [&](const uint32_t r[4], double ww, uint32_t e_daughter, bool at_start) {
    const double ndf = ceil(w / ww);
    lin_base = (uint64_t)r[0] | ((uint64_t)r[1] << 32);
    nd = (uint32_t)ndf;
    w = w / ndf;
    e_d = e_daughter;
    evb |= at_start ? EVB_START_SPLIT : EVB_SPLIT;
  };

  int gen = 0;
  uint32_t n_list = 0;  // daughters to transport in a generation >= 1
  for (;;) {
    const bool from_bank = (gen == 0);
    const int in_buf = (gen + 1) & 1;  // buffer written by the previous generation
    out_buf = gen & 1;
    const int64_t in_qbase = ((int64_t)in_buf * nq + qslot) * dstride;
    const int64_t out_qbase = ((int64_t)out_buf * nq + qslot) * dstride;

    int64_t tile_base = 0;
    uint32_t tile_next = 0, tile_end = 0;
    bool tile_bank = false;  // the current tile is of start particles (else daughters)
    bool exhausted = false;  // this generation's own tiles are all taken
    for (;;) {
      // ---------------------------------------------------------- refill --
      const uint64_t need_m = __ballot(!active);
      if (need_m != 0) {
        if (tile_next == tile_end) {
          int64_t tb = -1;
          uint32_t tl = 0;
          if (lane == 0 && !exhausted) {
            if (from_bank) {
              // Tiles of this unit: jseg, jseg + K, ... of the region.
              const uint32_t t = (uint32_t)jseg + (uint32_t)K * atomicAdd(L.dcur, 1u);
              if (t < L.tstart[K + 1]) {
                int s = K;
                while (L.tstart[s] > t) --s;
                const uint32_t off = (t - L.tstart[s]) * TILE;
                tl = min(TILE, L.nseg[s] - off);
                tb = in_region + (s < K ? (int64_t)s * G.seg_cap : (int64_t)K * G.seg_cap) + off;
              }
            } else {
              const uint32_t t0 = atomicAdd(L.dcur, TILE);
              if (t0 < n_list) {
                tl = min(TILE, n_list - t0);
                tb = in_qbase + t0;
              }
            }
          }
          const bool own = __shfl(tb, 0) >= 0;
          if (!own && !exhausted) {
            exhausted = true;
            if (lane == 0) atomicSub(L.obusy, 1u);
          }
          // With its own tiles gone, the wave takes daughters that this
          // generation has already written to its output buffer, when every
          // slot reserved so far is written (then all slots below the count
          // are): while another wave still has tiles of its own, or while
          // the generation has made few daughters.  A wave that finds none
          // leaves the generation, so a long cascade of daughters would be
          // left to the last waves; past kDrainSmall daughters it goes to the
          // next generation instead, which all waves share.
          if (lane == 0 && !own) {
            const bool busy = __hip_atomic_load(L.obusy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0u;
            const uint32_t r = __hip_atomic_load(&L.dready[out_buf], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
            const uint32_t c = __hip_atomic_load(&L.dcnt[out_buf], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (r == c && (busy || c <= kDrainSmall)) {
              const uint32_t lim = min(r, (uint32_t)A.dcap);
              uint32_t t = __hip_atomic_load(&L.dtake[out_buf], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
              while (t < lim) {
                const uint32_t nt = min(t + TILE, lim);
                const uint32_t old = atomicCAS(&L.dtake[out_buf], t, nt);
                if (old == t) {
                  tb = out_qbase + t;
                  tl = nt - t;
                  break;
                }
                t = old;
              }
            }
          }
          tb = __shfl(tb, 0);
          tl = __shfl(tl, 0);
          if (!own && tb >= 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
          if (tb >= 0) {
            tile_base = tb;
            tile_next = 0;
            tile_end = tl;
            tile_bank = own && from_bank;
          }
        }
        const uint32_t avail = tile_end - tile_next;
        if (avail != 0) {
          const uint32_t take = min((uint32_t)__popcll(need_m), avail);
          const uint32_t rk = rank_below(need_m);
          if (!active && rk < take) {
            const int64_t k = tile_base + (int64_t)(tile_next + rk);
            if (tile_bank) {
              const XMu<Real> xm = A.in_bank.xm[k];
              const Tag tg = A.in_bank.tag[k];
              x = xm.x;
              mu = xm.mu;
              w = A.in_bank.w[k];
              lin = A.in_bank.lin[k];
              src = tg.src;
              e = tg.e;
              cell = tg.cell;
              tau = dt_r;
              active = true;
              pend = 1u;
            } else {
              const XMu<Real> xm = A.dq.xm[k];
              const WTau wt = A.dq.wt[k];
              const Tag tg = A.dq.tag[k];
              x = xm.x;
              mu = xm.mu;
              w = wt.w;
              tau = (Real)wt.tau;
              lin = A.dq.lin[k];
              src = tg.src;
              e = tg.e;
              cell = tg.cell;
              active = true;
              pend = 0u;
            }
          }
          if (tile_bank) n_hist += take;
          tile_next += take;
        }
      }
      if (__ballot(active) == 0) {
        count_events();
        if (exhausted && tile_next == tile_end) break;
        continue;
      }

      // ------------------------------------------------ cell, window check --
      // The cell's flight record and its window, read together; then the
      // pending checks: the start-of-step one draws from slot 2 (roulette)
      // or 5 (split lineage) at the particle's event index, the one after a
      // crossing from slot 1 (roulette) or 4 (split lineage) at the index of
      // the crossing event, e - 1 (Sec. 2; one converged draw for all).
      CellData<Real> cd{};
      Window wd{};
      if (active) {
        cd = cellp[cell];
        if (A.ww_on) wd = winp[cell];
      }
      uint32_t ck = 0u;
      if (pend != 0u && active) ck = classify(wd);
      if (__ballot(ck != 0u) != 0) {
        if (ck != 0u) {
          const bool st = pend == 1u;
          const int slot = ck == WW_SPLIT ? (st ? SLOT_LIN_START : SLOT_LIN_EVENT) : (st ? SLOT_START : SLOT_EVENT);
          uint32_t r[4];
          draw_lane(A.seed, A.key1, slot, src, lin, st ? e : e - 1u, r);
          if (ck == WW_SPLIT) split(r, wd.ww, e, st);
          else roulette(u53(r[2], r[3]), wd.ww, st);
        }
        if (__ballot(nd > 1) != 0) flush_daughters();
        nd = 0;
      }
      pend = 0u;

      // --------------------------------------------------------- segment --
      bool at_census = false;
      int32_t next_chunk = 0;
      uint32_t act = 0u;  // EV_DRAW | EV_SCATTER | WW_ROULETTE | WW_SPLIT
      bool chk = false;   // window check due after a scatter
      uint32_t e_ev = 0u;
      if (active) {
        const int i = cell;
        uint32_t r[4];
        draw(A.seed, A.key1, SLOT_FLIGHT, src, lin, e, r);
        const Real ua = uflight<Real>(r[0], r[1]);
        const Real ub = uflight<Real>(r[2], r[3]);
        // Exponential flight distance with mean free path 1/sigma_t.
        const Real d_coll = -log_r((Real)1 - ua) * cd.inv_sig;
        const Real xl = cd.xl, xr = cd.xr;
        Real d_bnd;
        if (mu > (Real)0) d_bnd = (xr - x) / mu;
        else if (mu < (Real)0) d_bnd = (xl - x) / mu;
        else d_bnd = (Real)__builtin_inf();
        const Real d_cen = v_r * tau;
        int ev;
        Real l;
        if (d_cen <= d_bnd && d_cen <= d_coll) { ev = 0; l = d_cen; }
        else if (d_bnd <= d_coll) { ev = 1; l = d_bnd; }
        else { ev = 2; l = d_coll; }

        // Track-length tally of phi, J and K in cell i (Eq. phi-mc), in FP64.
        const double wl = w * (double)l;
        const double t1 = wl * (double)mu;
        atomicAdd(&L.hist[i * 6 + 0], wl);
        if (A.track_moments == 3) atomicAdd(&L.hist[i * 6 + 1], t1);
        if (A.track_moments >= 2) atomicAdd(&L.hist[i * 6 + 2], t1 * (double)mu);
        atomicAdd(&L.trk[i], 1u);
        e_ev = e;
        e = e_ev + 1;
        // Census and collision move the particle by mu l, kept in the cell.
        if (ev != 1) {
          Real xn = x + mu * l;
          if (xn < xl) xn = xl;
          if (xn > xr) xn = xr;
          x = xn;
        }

        if (ev == 0) {
          // The flight draw's second variate is unused at census: it picks
          // the chunk of the next step.
          next_chunk = (int32_t)(ub * (Real)nc);
          if (next_chunk >= nc) next_chunk = nc - 1;
          // Time-crossing tally at t^n (Eq. ct-mc): v*w per particle.
          const double vw = v * w;
          const double c1 = vw * (double)mu;
          atomicAdd(&L.hist[i * 6 + 3], vw);
          atomicAdd(&L.hist[i * 6 + 4], c1);
          atomicAdd(&L.hist[i * 6 + 5], c1 * (double)mu);
          atomicAdd(&L.wnext[next_chunk], w);
          evb |= EVB_CENSUS;
          at_census = true;
          active = false;
        } else {
          tau = tau - l * inv_v_r;
          if (ev == 1) {
            const bool out_l = (i == 0 && mu < (Real)0);
            const bool out_r = (i == I - 1 && mu > (Real)0);
            if (out_l || out_r) {
              // Edge-crossing estimators at the domain faces (w f(mu)/|mu|).
              const double mud = (double)mu;
              const double am = fabs(mud);
              double *f = L.bnd + (out_l ? 0 : 3);
              atomicAdd(&f[0], w / am);
              atomicAdd(&f[1], w * (0.5 - am) / am);
              atomicAdd(&f[2], w * (1.0 / 3.0 - mud * mud) / am);
              evb |= EVB_LEAK;
              active = false;
            } else {
              if (mu > (Real)0) { x = xr; cell = i + 1; }
              else { x = xl; cell = i - 1; }
              pend = 2u;
            }
          } else {
            if (ub < cd.c) {
              evb |= EVB_SCATTER;
              act = EV_DRAW | EV_SCATTER;
              chk = true;
            } else if (kFission && (double)ub < A.cfis[i]) {
              evb |= EVB_FISSION;
              act = EV_DRAW | EV_FISSION;
            } else {
              evb |= EVB_ABSORB;
              active = false;
            }
          }
        }
      }

      // Window check after a scatter (same cell: its window is in
      // registers); a roulette needs the event draw.
      if (chk) {
        const uint32_t c = classify(wd);
        act |= c;
        if (c == WW_ROULETTE) act |= EV_DRAW;
      }

      // Post-event draws, one converged call per kind: slot 1 gives the
      // scattering direction (first variate) and the roulette uniform
      // (second); slot 4 gives the lineage base of a split.  The window
      // check follows the new direction, as in the serial order.
      // A fission makes floor(nu_f + xi) neutrons (xi: second variate of
      // slot 1): the lane continues as the first with the direction of the
      // first variate, the others become daughters (lineage base of slot 4).
      uint32_t nf = 0;
      if (__ballot((act & EV_DRAW) != 0u) != 0) {
        if ((act & EV_DRAW) != 0u) {
          uint32_t r1[4];
          draw(A.seed, A.key1, SLOT_EVENT, src, lin, e_ev, r1);
          if (act & (EV_SCATTER | EV_FISSION)) mu = (Real)2 * uflight<Real>(r1[0], r1[1]) - (Real)1;
          if (act & WW_ROULETTE) roulette(u53(r1[2], r1[3]), wd.ww, false);
          if (kFission && (act & EV_FISSION)) {
            nf = (uint32_t)floor(A.nu_f + u53(r1[2], r1[3]));
            atomicAdd(&L.cnt[C_FISSION_BIRTHS], nf);
            if (nf == 0) active = false;
            else if (nf >= 2) act |= FIS_BIRTHS;
          }
        }
      }
      if (__ballot((act & (WW_SPLIT | FIS_BIRTHS)) != 0u) != 0) {
        if ((act & (WW_SPLIT | FIS_BIRTHS)) != 0u) {
          uint32_t r2[4];
          draw(A.seed, A.key1, SLOT_LIN_EVENT, src, lin, e_ev, r2);
          if (!kFission || (act & WW_SPLIT)) {
            split(r2, wd.ww, e, false);
          } else {
            lin_base = (uint64_t)r2[0] | ((uint64_t)r2[1] << 32);
            nd = nf;
            e_d = e;
            fis = true;
          }
        }
      }

      // -------------------------------------------------- census appends --
      census_append(A.census, G, L.ccnt, &A.census.ovfcnt[b * nc], (int64_t)(b * nc) * G.stride, nc, jseg,
                    at_census, next_chunk, x, mu, w, lin, src, e, cell, A.err);
      if (__ballot(nd > 1) != 0) flush_daughters();
      count_events();
      // Nothing of a split outlives the pass (this keeps the split state
      // out of the registers carried around the loop).
      nd = 0;
      lin_base = 0;
      e_d = 0;
      fis = false;
    }

    // ------------------------------------------- next daughter generation --
    // The daughters of this generation not taken while it ran: slots
    // taken .. n_list of its output buffer.
    __syncthreads();
    const uint32_t produced = L.dcnt[gen & 1], taken = L.dtake[gen & 1];
    const uint32_t next_list = produced < (uint32_t)A.dcap ? produced : (uint32_t)A.dcap;
    if (next_list <= taken) break;
    if (gen + 1 >= kMaxGenerations) {
      if (tid == 0) atomicOr(A.err, ERR_GENERATIONS);
      break;
    }
    __syncthreads();
    if (tid == 0) {
      L.dcnt[(gen + 1) & 1] = 0u;
      L.dready[(gen + 1) & 1] = 0u;
      L.dtake[(gen + 1) & 1] = 0u;
      L.obusy[0] = blockDim.x >> 6;
      L.dcur[0] = taken;
    }
    __syncthreads();
    n_list = next_list;
    ++gen;
  }

  if (lane == 0) {
    if (n_census) atomicAdd(&L.cnt[C_CENSUS], n_census);
    if (n_scatter) atomicAdd(&L.cnt[C_SCATTERS], n_scatter);
    if (n_absorb) atomicAdd(&L.cnt[C_ABSORPTIONS], n_absorb);
    if (n_hist) atomicAdd(&L.cnt[C_HISTORIES], n_hist);
  }
  // Segments: the sum of the per-cell track counters.  Every segment ends
  // in exactly one of census, leak, crossing or collision (scatter, fission
  // or absorption), which gives the crossings.
  __syncthreads();
  {
    uint32_t part = 0;
    for (int j = tid; j < I; j += blockDim.x) part += L.trk[j];
    for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o);
    if ((tid & 63) == 0 && part != 0) atomicAdd(&L.cnt[C_SEGMENTS], part);
  }
  __syncthreads();
  if (tid == 0) {
    L.cnt[C_COLLISIONS] = L.cnt[C_SCATTERS] + L.cnt[C_ABSORPTIONS] + L.cnt[C_FISSIONS];
    L.cnt[C_CROSSINGS] = L.cnt[C_SEGMENTS] - L.cnt[C_CENSUS] - L.cnt[C_LEAKS] - L.cnt[C_COLLISIONS];
  }
  __syncthreads();
  if (tid < nc) {
    const uint32_t cc = L.ccnt[tid];
    A.census.segcnt[(b * nc + tid) * K + jseg] = cc < (uint32_t)G.seg_cap ? cc : (uint32_t)G.seg_cap;
  }
  if (tid < C_NCOUNTERS && tid != C_GENERATIONS) {
    const uint32_t t = L.cnt[tid];
    if (t != 0) {
      atomicAdd(&A.counters[tid], (unsigned long long)t);                // this step
      atomicAdd(&A.counters[C_NCOUNTERS + tid], (unsigned long long)t);  // since init
    }
  }
  if (tid == 0) {
    atomicMax(&A.counters[C_GENERATIONS], (unsigned long long)(gen + 1));
    atomicMax(&A.counters[C_NCOUNTERS + C_GENERATIONS], (unsigned long long)(gen + 1));
  }
  flush_tallies(L, I, nc, b, A.tal, A.tsum, qslot % kSumCopies, A.bnd, A.tracks, A.wnext);
}

// One problem: grid = B * K work-groups; work-group g is the unit
// (batch g mod B, segment g / B).
template <typename Real, bool kCellsLds, bool kFission>
__global__ void __launch_bounds__(1024) sweep_kernel(SweepArgs<Real> A) {
  extern __shared__ double lds_raw[];
  sweep_unit<Real, kCellsLds, kFission>(A, (int)(blockIdx.x % A.B), (int)(blockIdx.x / A.B), (int)blockIdx.x,
                              (int)gridDim.x, lds_raw);
}

// Many problems (replicas) in one persistent launch: each work-group claims
// units from the launch's counter until none is left.  The unit table lists
// the biggest replicas first and the units of one batch next to each other,
// so the units that share a batch's tiles run at the same time.  kCells:
// 0 no replica keeps its cell records in LDS, 1 all do, 2 each as its
// descriptor says (the launch's LDS holds the largest need).
template <typename Real, int kCells>
__global__ void __launch_bounds__(1024) sweep_batch_kernel(BatchSweepArgs<Real> P,
                                                           const ReplicaDesc<Real> *__restrict__ desc,
                                                           const uint32_t *__restrict__ units) {
  extern __shared__ double lds_raw[];
  __shared__ uint32_t s_unit;
  const int par = P.par;
  if (blockIdx.x == 0 && threadIdx.x == 0) P.work[1 - par] = 0u;
  for (;;) {
    if (threadIdx.x == 0) s_unit = atomicAdd(&P.work[par], 1u);
    __syncthreads();
    const uint32_t u = __builtin_amdgcn_readfirstlane(s_unit);
    if (u >= P.n_units) break;
    const uint32_t code = __builtin_amdgcn_readfirstlane(units[u]);
    const int r = (int)(code >> 16), b = (int)((code >> 8) & 0xFFu), jseg = (int)(code & 0xFFu);
    const ReplicaDesc<Real> &D = desc[r];
    SweepArgs<Real> A;
    A.I = D.I; A.B = D.B; A.nc = D.nc;
    A.v = D.v; A.inv_v = D.inv_v; A.dt = D.dt;
    // The key words feed an asm operand that must live in scalar registers.
    A.seed = __builtin_amdgcn_readfirstlane(D.seed);
    A.key1 = __builtin_amdgcn_readfirstlane(D.key1);
    A.cells = D.cells; A.win = D.win;
    A.track_moments = D.track_moments;
    A.cfis = nullptr; A.nu_f = 0.0;  // batches have no fission (kFission = false)
    A.ww_on = P.ww_on; A.chunk = P.chunk; A.tile = P.tile;
    A.geom = D.geom;
    A.in_bank = D.bank[P.start_bank];
    A.census = D.bank[1 - P.start_bank];
    A.dq = P.dq; A.dcap = P.dcap;
    A.tal = D.tal[P.start_bank]; A.tsum = D.tsum[P.start_bank]; A.bnd = D.bnd[P.start_bank];
    A.tracks = D.tracks; A.counters = D.counters; A.wnext = D.wnext;
    A.err = P.err;
    if (kCells == 1 || (kCells == 2 && D.cells_lds))
      sweep_unit<Real, true, false>(A, b, jseg, (int)blockIdx.x, (int)gridDim.x, lds_raw);
    else
      sweep_unit<Real, false, false>(A, b, jseg, (int)blockIdx.x, (int)gridDim.x, lds_raw);
    __syncthreads();
  }
}

// Source bank at t^0 (Sec. 5.1): unit-weight particles at src_x with
// isotropic directions from slot 3, appended to the census region of their
// batch and of their step-1 chunk; their census moments are the step-1
// initial condition.  Work-group (b, j) creates the sources s = b + B m,
// m = j, j + K, j + 2K, ... into its own segments.
template <typename Real>
__global__ void __launch_bounds__(1024) source_kernel(SourceArgs A, Bank<Real> bank) {
  extern __shared__ double lds_raw[];
  const int I = A.I, nc = A.nc;
  const BankGeom G = A.geom;
  const int K = G.K;
  Lds L = carve(lds_raw, I, nc, K);
  zero_lds(lds_raw, I, nc, K);
  __syncthreads();
  const int b = blockIdx.x % A.B;
  const int jseg = blockIdx.x / A.B;
  const int64_t n_b = (A.n_src > b) ? (A.n_src - b + A.B - 1) / A.B : 0;  // sources of batch b
  const int64_t n_j = (n_b > jseg) ? (n_b - jseg + K - 1) / K : 0;           // of which this work-group's
  const int64_t rounds = (n_j + blockDim.x - 1) / blockDim.x;
  const Real x0 = (Real)A.src_x;
  for (int64_t it = 0; it < rounds; ++it) {
    const int64_t mloc = it * blockDim.x + threadIdx.x;
    const bool live = mloc < n_j;
    const int64_t s = (int64_t)b + (int64_t)A.B * ((int64_t)jseg + (int64_t)K * mloc);
    Real mu = 0;
    int32_t cell = 0, chunk = 0;
    if (live) {
      uint32_t r[4];
      draw(A.seed, A.key1, SLOT_BIRTH, (uint32_t)s, 0ull, 0u, r);
      mu = (Real)2 * uflight<Real>(r[0], r[1]) - (Real)1;
      cell = find_cell(A.edges, I, (double)x0, (double)mu);
      chunk = (int32_t)(uflight<Real>(r[2], r[3]) * (Real)nc);
      if (chunk >= nc) chunk = nc - 1;
      const double vw = A.v * 1.0;
      const double c1 = vw * (double)mu;
      atomicAdd(&L.hist[cell * 6 + 3], vw);
      atomicAdd(&L.hist[cell * 6 + 4], c1);
      atomicAdd(&L.hist[cell * 6 + 5], c1 * (double)mu);
      atomicAdd(&L.wnext[chunk], 1.0);
    }
    census_append(bank, G, L.ccnt, &bank.ovfcnt[b * nc], (int64_t)(b * nc) * G.stride, nc, jseg, live, chunk,
                  x0, mu, 1.0, 0ull, (uint32_t)s, 0u, cell, A.err);
  }
  __syncthreads();
  if ((int)threadIdx.x < nc) {
    const uint32_t cc = L.ccnt[threadIdx.x];
    bank.segcnt[(b * nc + threadIdx.x) * K + jseg] = cc < (uint32_t)G.seg_cap ? cc : (uint32_t)G.seg_cap;
  }
  flush_tallies(L, I, nc, b, A.tal, A.tsum, (int)(blockIdx.x % kSumCopies), nullptr, nullptr, A.wnext);
}

// Clear the accumulators of a new time step and hand the census chunk
// weights of the finished step to the new one (one launch).
__device__ inline void begin_step_body(const BeginStepArgs &A) {
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = t0; j < A.n_seg; j += st) A.segcnt[j] = 0u;
  for (int64_t j = t0; j < A.n_ovf; j += st) A.ovfcnt[j] = 0u;
  for (int64_t j = t0; j < A.n_tal; j += st) A.tal[j] = 0.0;
  for (int64_t j = t0; j < A.n_tsum; j += st) A.tsum[j] = 0.0;
  for (int64_t j = t0; j < A.n_bnd; j += st) A.bnd[j] = 0.0;
  for (int64_t j = t0; j < A.n_tracks; j += st) A.tracks[j] = 0ull;
  for (int64_t j = t0; j < C_NCOUNTERS; j += st) A.counters[j] = 0ull;
  if (t0 < A.nc) {
    A.wstart[t0] = A.wnext[t0];
    A.wnext[t0] = 0.0;
  }
}

__global__ void begin_step_kernel(BeginStepArgs A) { begin_step_body(A); }

// All replicas of a batch: row blockIdx.y of the grid serves replica y.
__global__ void begin_step_batch_kernel(const BeginStepArgs *tab) { begin_step_body(tab[blockIdx.y]); }

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t n) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    p[j] = v;
}
__global__ void fill_f64_kernel(double *p, double v, int64_t n) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    p[j] = v;
}
__global__ void rotate_chunks_kernel(double *wstart, double *wnext, int nc) {
  const int j = threadIdx.x;
  if (j < nc) {
    wstart[j] = wnext[j];
    wnext[j] = 0.0;
  }
}

static hipError_t allow_lds(const void *fn, size_t lds, size_t *done) {
  if (lds > *done) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    *done = lds;
  }
  return hipSuccess;
}

template <typename Real>
hipError_t launch_sweep(const SweepArgs<Real> &a, bool cells_lds, int grid, int block, size_t lds, hipStream_t s) {
  static size_t done[4] = {64 * 1024, 64 * 1024, 64 * 1024, 64 * 1024};
  const bool fis = a.cfis != nullptr;
  const void *fn = fis ? (cells_lds ? reinterpret_cast<const void *>(&sweep_kernel<Real, true, true>)
                                    : reinterpret_cast<const void *>(&sweep_kernel<Real, false, true>))
                       : (cells_lds ? reinterpret_cast<const void *>(&sweep_kernel<Real, true, false>)
                                    : reinterpret_cast<const void *>(&sweep_kernel<Real, false, false>));
  hipError_t e = allow_lds(fn, lds, &done[(fis ? 2 : 0) + (cells_lds ? 1 : 0)]);
  if (e != hipSuccess) return e;
  if (fis) {
    if (cells_lds) hipLaunchKernelGGL((sweep_kernel<Real, true, true>), dim3(grid), dim3(block), lds, s, a);
    else hipLaunchKernelGGL((sweep_kernel<Real, false, true>), dim3(grid), dim3(block), lds, s, a);
  } else {
    if (cells_lds) hipLaunchKernelGGL((sweep_kernel<Real, true, false>), dim3(grid), dim3(block), lds, s, a);
    else hipLaunchKernelGGL((sweep_kernel<Real, false, false>), dim3(grid), dim3(block), lds, s, a);
  }
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_source(const SourceArgs &a, const Bank<Real> &bank, int grid, int block, size_t lds,
                         hipStream_t s) {
  static size_t done = 64 * 1024;
  hipError_t e = allow_lds(reinterpret_cast<const void *>(&source_kernel<Real>), lds, &done);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(source_kernel<Real>, dim3(grid), dim3(block), lds, s, a, bank);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_sweep_batch(const BatchSweepArgs<Real> &a, int cells_mode, int grid, int block, size_t lds,
                              hipStream_t s) {
  static size_t done[3] = {64 * 1024, 64 * 1024, 64 * 1024};
  const void *fn = cells_mode == 1   ? reinterpret_cast<const void *>(&sweep_batch_kernel<Real, 1>)
                   : cells_mode == 2 ? reinterpret_cast<const void *>(&sweep_batch_kernel<Real, 2>)
                                     : reinterpret_cast<const void *>(&sweep_batch_kernel<Real, 0>);
  hipError_t e = allow_lds(fn, lds, &done[cells_mode]);
  if (e != hipSuccess) return e;
  if (cells_mode == 1)
    hipLaunchKernelGGL((sweep_batch_kernel<Real, 1>), dim3(grid), dim3(block), lds, s, a, a.desc, a.units);
  else if (cells_mode == 2)
    hipLaunchKernelGGL((sweep_batch_kernel<Real, 2>), dim3(grid), dim3(block), lds, s, a, a.desc, a.units);
  else
    hipLaunchKernelGGL((sweep_batch_kernel<Real, 0>), dim3(grid), dim3(block), lds, s, a, a.desc, a.units);
  return hipGetLastError();
}

template hipError_t launch_sweep_batch<double>(const BatchSweepArgs<double> &, int, int, int, size_t, hipStream_t);
template hipError_t launch_sweep_batch<float>(const BatchSweepArgs<float> &, int, int, int, size_t, hipStream_t);
template hipError_t launch_sweep<double>(const SweepArgs<double> &, bool, int, int, size_t, hipStream_t);
template hipError_t launch_sweep<float>(const SweepArgs<float> &, bool, int, int, size_t, hipStream_t);
template hipError_t launch_source<double>(const SourceArgs &, const Bank<double> &, int, int, size_t, hipStream_t);
template hipError_t launch_source<float>(const SourceArgs &, const Bank<float> &, int, int, size_t, hipStream_t);

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)g), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)g), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_begin_step(const BeginStepArgs &a, hipStream_t s) {
  int64_t g = (a.n_tal + 255) / 256;
  if (g < 1) g = 1;
  if (g > 1024) g = 1024;
  hipLaunchKernelGGL(begin_step_kernel, dim3((unsigned)g), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_begin_step_batch(const BeginStepArgs *tab, int n, int64_t max_tal, hipStream_t s) {
  int64_t g = (max_tal + 255) / 256;
  if (g < 1) g = 1;
  if (g > 64) g = 64;
  hipLaunchKernelGGL(begin_step_batch_kernel, dim3((unsigned)g, (unsigned)n), dim3(256), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_rotate_chunks(double *wstart, double *wnext, int nc, hipStream_t s) {
  hipLaunchKernelGGL(rotate_chunks_kernel, dim3(1), dim3(64), 0, s, wstart, wnext, nc);
  return hipGetLastError();
}

}  // namespace hww
