// Particle sweep of one chunk of a time step of the hybrid weight-window
// Monte Carlo method (Shaw & Anistratov, arXiv 2512.19925): flight,
// collision and census of a 1D slab bank (Sec. 3, Eq. HO_transport),
// track-length and time-crossing tallies (Sec. 3, Eqs. phi-mc, ct-mc),
// and split / Russian roulette against weight windows (Sec. 2).
//
// Launch shape: grid = B * k work-groups.  Work-group g serves batch
// b = g mod B; all lanes of a wave therefore belong to one batch, so a
// work-group keeps its batch's tallies in an LDS histogram that is flushed
// to HBM once, with FP64 atomics, and census / daughter writes compact by
// wave ballot into batch-private regions with one atomic per wave.
//
// Each wave keeps its 64 lanes busy: a lane whose particle ends (census,
// leak, absorption, roulette) refills from the wave's current tile of the
// input list; tiles are claimed from a per-batch atomic cursor.
#include "hww_internal.h"

namespace hww {

static constexpr int TILE = 256;

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of the two published
// 32x32 -> 64 multiplies; key bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ void draw(uint32_t seed, uint32_t key1, int slot, uint32_t src,
                                     uint64_t lin, uint32_t e, uint32_t r[4]) {
  r[0] = src;
  r[1] = (uint32_t)lin;
  r[2] = (uint32_t)(lin >> 32);
  r[3] = e;
  philox4x32_10(r, seed, key1 | (uint32_t)slot);
}

// 53-bit uniform on [0,1) from the high bits of two words.
__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
  const double k = (double)(a >> 5) * 67108864.0 + (double)(b >> 6);
  return k * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
  return (uint32_t)__popcll(m & __lanemask_lt());
}

struct LaneCounters {
  uint32_t segments, collisions, scatters, absorptions, crossings, leaks, census;
  uint32_t splits, daughters, rr_kill, rr_survive, histories;
};

// Shared-memory layout of a work-group.
struct Lds {
  double *hist;    // [I][6]
  uint32_t *trk;   // [I]
  double *wnext;   // [nc]
  double *bnd;     // [6]
  uint32_t *cnt;   // [C_NCOUNTERS]
};

__device__ __forceinline__ void lds_add(double *p, double v) { atomicAdd(p, v); }

template <typename Real>
__global__ void __launch_bounds__(1024) sweep_kernel(SweepArgs<Real> A) {
  extern __shared__ double lds_raw[];
  const int I = A.I;
  Lds L;
  L.hist = lds_raw;
  L.wnext = lds_raw + (size_t)I * 6;
  L.bnd = L.wnext + A.nc;
  L.trk = reinterpret_cast<uint32_t *>(L.bnd + 6);
  L.cnt = L.trk + I;
  for (int j = threadIdx.x; j < I * 6 + A.nc + 6; j += blockDim.x) lds_raw[j] = 0.0;
  for (int j = threadIdx.x; j < I + C_NCOUNTERS; j += blockDim.x) L.trk[j] = 0u;
  __syncthreads();

  const int b = blockIdx.x % A.B;
  const uint32_t lane = lane_id();
  const bool from_bank = (A.gen == 0);
  uint32_t n_in = from_bank ? A.in_bank.count[b * A.nc + A.chunk] : A.in_q.count[b];
  // An overflowed list is already flagged; never read past its region.
  const int64_t in_cap = from_bank ? A.cap_r : A.cap_d;
  if ((int64_t)n_in > in_cap) n_in = (uint32_t)in_cap;
  const int64_t in_base = from_bank ? (int64_t)(b * A.nc + A.chunk) * A.cap_r : (int64_t)b * A.cap_d;
  const double v = A.v;

  // Lane state.
  double x = 0.0, mu = 0.0, w = 0.0, tau = 0.0;
  int32_t cell = 0;
  uint32_t src = 0, e = 0;
  uint64_t lin = 0;
  bool active = false;
  // Pending split of this lane: daughters copy the lane state.
  uint32_t nd = 0;
  uint64_t lin_base = 0;
  uint32_t e_d = 0;

  uint32_t tile_next = 0, tile_end = 0;
  bool exhausted = false;
  LaneCounters C = {};

  // Write the pending daughters of all lanes of the wave (converged call).
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
      uint32_t base = 0;
      if (lane == 0) base = atomicAdd(&A.out_q.count[b], total);
      base = __shfl(base, 0);
      if ((uint64_t)base + total > (uint64_t)A.cap_d) {
        if (lane == 0) atomicOr(A.err, ERR_CAPACITY);
      }
      const uint32_t start = base + incl - cntd;
      for (uint32_t j = 1; j <= cntd; ++j) {
        const uint64_t slot = (uint64_t)start + (j - 1);
        if (slot >= (uint64_t)A.cap_d) break;
        {
          const int64_t k = (int64_t)b * A.cap_d + (int64_t)slot;
          A.out_q.x[k] = (Real)x;
          A.out_q.mu[k] = (Real)mu;
          A.out_q.w[k] = w;
          A.out_q.tau[k] = tau;
          A.out_q.lin[k] = lin_base + j;
          A.out_q.src[k] = src;
          A.out_q.e[k] = e_d;
          A.out_q.cell[k] = cell;
        }
      }
    }
    nd = 0;
  };

  // Weight-window check of the lane's particle in its cell (Sec. 2).
  // kind 0: after an event at index e_ev; kind 1: start of step.
  // xi_slot: slot whose u_b is the roulette variate (drawn only if needed).
  auto ww_check = [&](int kind, uint32_t e_ev, uint32_t e_daughter, int xi_slot, bool have_xi,
                      double xi) {
    if (!A.ww_on) return;
    const double ww = A.centre[cell];
    if (w > A.wceil[cell]) {
      const double ndf = ceil(w / ww);
      if (!(ndf >= 2.0) || ndf > 1.0e9) {
        atomicOr(A.err, ERR_SPLIT);
        active = false;
        return;
      }
      if (ndf - 1.0 > (double)A.cap_d) {
        atomicOr(A.err, ERR_CAPACITY);
        active = false;
        return;
      }
      uint32_t r[4];
      draw(A.seed, A.key1, kind == 0 ? SLOT_LIN_EVENT : SLOT_LIN_START, src, lin, e_ev, r);
      lin_base = (uint64_t)r[0] | ((uint64_t)r[1] << 32);
      nd = (uint32_t)ndf;
      w = w / ndf;
      e_d = e_daughter;
      C.splits += 1;
      C.daughters += nd - 1;
    } else if (w < A.wfloor[cell]) {
      if (!have_xi) {
        uint32_t r[4];
        draw(A.seed, A.key1, xi_slot, src, lin, e_ev, r);
        xi = u53(r[2], r[3]);
      }
      if (xi < w / ww) {
        w = ww;
        C.rr_survive += 1;
      } else {
        C.rr_kill += 1;
        active = false;
      }
    }
  };

  for (;;) {
    // ---------------------------------------------------------- refill --
    const uint64_t need_m = __ballot(!active);
    if (need_m != 0) {
      if (tile_next == tile_end && !exhausted) {
        uint32_t t0 = 0;
        if (lane == 0) t0 = atomicAdd(&A.cursor[b], (uint32_t)TILE);
        t0 = __shfl(t0, 0);
        if (t0 >= n_in) {
          exhausted = true;
        } else {
          tile_next = t0;
          tile_end = min(t0 + (uint32_t)TILE, n_in);
        }
      }
      const uint32_t avail = tile_end - tile_next;
      if (avail != 0) {
        const uint32_t take = min((uint32_t)__popcll(need_m), avail);
        const uint32_t rk = rank_below(need_m);
        if (!active && rk < take) {
          const int64_t k = in_base + (int64_t)(tile_next + rk);
          if (from_bank) {
            x = (double)A.in_bank.x[k];
            mu = (double)A.in_bank.mu[k];
            w = A.in_bank.w[k];
            lin = A.in_bank.lin[k];
            src = A.in_bank.src[k];
            e = A.in_bank.e[k];
            cell = A.in_bank.cell[k];
            tau = A.dt;
            active = true;
            C.histories += 1;
            ww_check(1, e, e, SLOT_START, false, 0.0);
          } else {
            x = (double)A.in_q.x[k];
            mu = (double)A.in_q.mu[k];
            w = A.in_q.w[k];
            tau = A.in_q.tau[k];
            lin = A.in_q.lin[k];
            src = A.in_q.src[k];
            e = A.in_q.e[k];
            cell = A.in_q.cell[k];
            active = true;
          }
        }
        tile_next += take;
      }
      flush_daughters();
    }
    if (__ballot(active) == 0) {
      if (exhausted && tile_next == tile_end) break;
      continue;
    }

    // --------------------------------------------------------- segment --
    bool at_census = false;
    int32_t next_chunk = 0;
    if (active) {
      const int i = cell;
      uint32_t r[4];
      draw(A.seed, A.key1, SLOT_FLIGHT, src, lin, e, r);
      const double ua = u53(r[0], r[1]);
      const double ub = u53(r[2], r[3]);
      const double d_coll = -log(1.0 - ua) / A.sig_t[i];
      const double xl = A.edges[i], xr = A.edges[i + 1];
      double d_bnd;
      if (mu > 0.0) d_bnd = (xr - x) / mu;
      else if (mu < 0.0) d_bnd = (xl - x) / mu;
      else d_bnd = __builtin_inf();
      const double d_cen = v * tau;
      int ev;
      double l;
      if (d_cen <= d_bnd && d_cen <= d_coll) { ev = 0; l = d_cen; }
      else if (d_bnd <= d_coll) { ev = 1; l = d_bnd; }
      else { ev = 2; l = d_coll; }

      // Track-length tally of phi, J and K in cell i (Eq. phi-mc).
      const double wl = w * l;
      const double t1 = wl * mu;
      lds_add(&L.hist[i * 6 + 0], wl);
      lds_add(&L.hist[i * 6 + 1], t1);
      lds_add(&L.hist[i * 6 + 2], t1 * mu);
      atomicAdd(&L.trk[i], 1u);
      C.segments += 1;
      const uint32_t e_ev = e;
      e = e_ev + 1;

      if (ev == 0) {
        double xn = x + mu * l;
        if (xn < xl) xn = xl;
        if (xn > xr) xn = xr;
        x = xn;
        uint32_t rc[4];
        draw(A.seed, A.key1, SLOT_START, src, lin, e, rc);
        next_chunk = (int32_t)(u53(rc[0], rc[1]) * (double)A.nc);
        if (next_chunk >= A.nc) next_chunk = A.nc - 1;
        // Time-crossing tally at t^n (Eq. ct-mc): v*w per particle.
        const double vw = v * w;
        const double c1 = vw * mu;
        lds_add(&L.hist[i * 6 + 3], vw);
        lds_add(&L.hist[i * 6 + 4], c1);
        lds_add(&L.hist[i * 6 + 5], c1 * mu);
        lds_add(&L.wnext[next_chunk], w);
        C.census += 1;
        at_census = true;
        active = false;
      } else {
        tau = tau - l / v;
        if (ev == 1) {
          const bool out_l = (i == 0 && mu < 0.0);
          const bool out_r = (i == I - 1 && mu > 0.0);
          if (out_l || out_r) {
            // Edge-crossing estimators at the domain faces (w f(mu)/|mu|).
            const double am = fabs(mu);
            double *f = L.bnd + (out_l ? 0 : 3);
            lds_add(&f[0], w / am);
            lds_add(&f[1], w * (0.5 - am) / am);
            lds_add(&f[2], w * (1.0 / 3.0 - mu * mu) / am);
            C.leaks += 1;
            active = false;
          } else {
            if (mu > 0.0) { x = xr; cell = i + 1; }
            else { x = xl; cell = i - 1; }
            C.crossings += 1;
            ww_check(0, e_ev, e, SLOT_EVENT, false, 0.0);
          }
        } else {
          double xn = x + mu * l;
          if (xn < xl) xn = xl;
          if (xn > xr) xn = xr;
          x = xn;
          C.collisions += 1;
          if (ub < A.cratio[i]) {
            uint32_t r1[4];
            draw(A.seed, A.key1, SLOT_EVENT, src, lin, e_ev, r1);
            mu = 2.0 * u53(r1[0], r1[1]) - 1.0;
            C.scatters += 1;
            ww_check(0, e_ev, e, SLOT_EVENT, true, u53(r1[2], r1[3]));
          } else {
            C.absorptions += 1;
            active = false;
          }
        }
      }
    }

    // -------------------------------------------------- census compaction --
    const uint64_t cen_m = __ballot(at_census);
    if (cen_m != 0) {
      for (int c = 0; c < A.nc; ++c) {
        const uint64_t m = __ballot(at_census && next_chunk == c);
        if (m == 0) continue;
        const uint32_t leader = (uint32_t)(__ffsll((long long)m) - 1);
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&A.census.count[b * A.nc + c], (uint32_t)__popcll(m));
        base = __shfl(base, (int)leader);
        if (at_census && next_chunk == c) {
          const uint64_t slot = (uint64_t)base + rank_below(m);
          if (slot < (uint64_t)A.cap_r) {
            const int64_t k = (int64_t)(b * A.nc + c) * A.cap_r + (int64_t)slot;
            A.census.x[k] = (Real)x;
            A.census.mu[k] = (Real)mu;
            A.census.w[k] = w;
            A.census.lin[k] = lin;
            A.census.src[k] = src;
            A.census.e[k] = e;
            A.census.cell[k] = cell;
          } else {
            atomicOr(A.err, ERR_CAPACITY);
          }
        }
      }
    }
    if (__ballot(nd > 1) != 0) flush_daughters();
  }

  // Per-wave counter reduction into LDS.
  {
    uint32_t vals[12] = {C.segments, C.collisions, C.scatters, C.absorptions, C.crossings, C.leaks,
                         C.census, C.splits, C.daughters, C.rr_kill, C.rr_survive, C.histories};
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      uint32_t s = vals[q];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
      if (lane == 0 && s != 0) atomicAdd(&L.cnt[q], s);
    }
  }
  __syncthreads();

  // Flush the work-group histogram (nonzero entries only).
  double *tal_b = A.tal + (size_t)b * I * 6;
  for (int j = threadIdx.x; j < I * 6; j += blockDim.x) {
    const double val = L.hist[j];
    if (val != 0.0) unsafeAtomicAdd(&tal_b[j], val);
  }
  for (int j = threadIdx.x; j < I; j += blockDim.x) {
    const uint32_t t = L.trk[j];
    if (t != 0) atomicAdd(&A.tracks[j], (unsigned long long)t);
  }
  if (threadIdx.x < 6) {
    const double val = L.bnd[threadIdx.x];
    if (val != 0.0) unsafeAtomicAdd(&A.bnd[b * 6 + threadIdx.x], val);
  }
  if (threadIdx.x < (unsigned)A.nc) {
    const double val = L.wnext[threadIdx.x];
    if (val != 0.0) unsafeAtomicAdd(&A.wnext[threadIdx.x], val);
  }
  if (threadIdx.x < 12) {
    const uint32_t t = L.cnt[threadIdx.x];
    if (t != 0) atomicAdd(&A.counters[threadIdx.x], (unsigned long long)t);
  }
}

// Source bank at t^0 (Sec. 5.1): unit-weight particles at src_x with
// isotropic directions from slot 3, in the region of their batch and of the
// chunk of step 1; their census moments are the step-1 initial condition.
__global__ void __launch_bounds__(256) source_kernel(SourceArgs A, Bank<double> bank) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= A.n_src) return;
  uint32_t r[4];
  draw(A.seed, A.key1, SLOT_BIRTH, (uint32_t)s, 0ull, 0u, r);
  const double mu = 2.0 * u53(r[0], r[1]) - 1.0;
  const double x = A.src_x;
  // Cell of x; a point on an interior edge belongs to the cell it moves into.
  int32_t cell;
  if (x <= A.edges[0]) {
    cell = 0;
  } else if (x >= A.edges[A.I]) {
    cell = A.I - 1;
  } else {
    int32_t lo = 0, hi = A.I;
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) / 2;
      if (A.edges[mid] <= x) lo = mid; else hi = mid;
    }
    if (x == A.edges[lo] && mu < 0.0 && lo > 0) lo -= 1;
    cell = lo;
  }
  draw(A.seed, A.key1, SLOT_START, (uint32_t)s, 0ull, 0u, r);
  int32_t chunk = (int32_t)(u53(r[0], r[1]) * (double)A.nc);
  if (chunk >= A.nc) chunk = A.nc - 1;
  const int b = (int)(s % A.B);
  const int reg = b * A.nc + chunk;
  const uint32_t slot = atomicAdd(&bank.count[reg], 1u);
  if ((int64_t)slot >= A.cap_r) {
    atomicOr(A.err, ERR_CAPACITY);
    return;
  }
  const int64_t k = (int64_t)reg * A.cap_r + slot;
  bank.x[k] = x;
  bank.mu[k] = mu;
  bank.w[k] = 1.0;
  bank.lin[k] = 0ull;
  bank.src[k] = (uint32_t)s;
  bank.e[k] = 0u;
  bank.cell[k] = cell;
  const double vw = A.v * 1.0;
  const double c1 = vw * mu;
  double *t = A.tal + ((size_t)b * A.I + cell) * 6;
  unsafeAtomicAdd(&t[3], vw);
  unsafeAtomicAdd(&t[4], c1);
  unsafeAtomicAdd(&t[5], c1 * mu);
  unsafeAtomicAdd(&A.wnext[chunk], 1.0);
}

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

hipError_t launch_sweep_f64(const SweepArgs<double> &a, int grid, int block, size_t lds, hipStream_t s) {
  static size_t attr_lds = 64 * 1024;
  if (lds > attr_lds) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&sweep_kernel<double>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_lds = lds;
  }
  hipLaunchKernelGGL(sweep_kernel<double>, dim3(grid), dim3(block), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_source_f64(const SourceArgs &a, const Bank<double> &bank, hipStream_t s) {
  if (a.n_src == 0) return hipSuccess;
  const int64_t grid = (a.n_src + 255) / 256;
  hipLaunchKernelGGL(source_kernel, dim3((unsigned)grid), dim3(256), 0, s, a, bank);
  return hipGetLastError();
}

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

hipError_t launch_rotate_chunks(double *wstart, double *wnext, int nc, hipStream_t s) {
  hipLaunchKernelGGL(rotate_chunks_kernel, dim3(1), dim3(64), 0, s, wstart, wnext, nc);
  return hipGetLastError();
}

}  // namespace hww
