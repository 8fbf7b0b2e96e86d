// Uniform combing of a census bank (the population control of the paper's
// supercritical test problem, Sec. 5.1), in two readings.  By weight: the
// census particles are laid end to end in canonical order (src, lineage,
// event), each as long as its weight, and n_target equally spaced teeth with
// one random offset pick the particles that are copied, at weight
// W / n_target.  By index: the teeth are spaced n / n_target apart over the
// n particles in canonical order, every particle has the same chance, and
// each copy keeps its particle's weight times n / n_target (the reading under
// which the comb thins the many particles of weight near 1 at the source, as
// Sec. 5 remarks of the paper's), the weight taken in the integer unit below
// and the chunk weights from exact integer sums, so that rounding far below
// the unit (the summation order of the window solve) changes nothing after
// the comb.
//
// Order on the device: a counting sort by src (histogram, exclusive scan,
// scatter), then each history's particles ranked by (lineage, event): one
// lane per particle comparing its key with the rest of its history when the
// history has few, one work-group ranking through LDS tiles when it has many.
// Weights become integers in units of 2^eu (count * max weight < 2^(53 +
// eu)), so the inclusive prefix sums are exact and identical in any
// summation order, and each tooth finds its particle by binary search over
// them.  The census count and eu are read on the device, so the whole comb
// is one sequence of launches with one wait at its end.
#include <algorithm>

#include "hww_internal.h"
#include "hww_rng_dev.h"

namespace hww {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;                        // elements per thread in a scan tile
constexpr int kScanTile = kScanThreads * kScanPer;
constexpr int kSmallBin = 64;                      // histories ranked lane by lane up to this size

// The occupied slots of the census bank: each wavefront takes whole
// segments (K per region plus the overflow segment) and its lanes the slots
// below the segment's count, so the walk costs the census, not the bank's
// capacity.  f(q) is called for every occupied slot q.
template <typename Real, typename F>
__device__ inline void for_each_census_slot(const CombArgs<Real> &A, F &&f) {
  const BankGeom &G = A.G;
  const int64_t nseg = (int64_t)A.R * (G.K + 1);
  const int lane = threadIdx.x & 63;
  const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t sg = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; sg < nseg; sg += nwave) {
    const int64_t r = sg / (G.K + 1), sidx = sg - r * (G.K + 1);
    const int64_t n = sidx < G.K ? min((int64_t)A.src_bank.segcnt[r * G.K + sidx], G.seg_cap)
                                 : min((int64_t)A.src_bank.ovfcnt[r], G.ovf_cap);
    const int64_t base = r * G.stride + sidx * G.seg_cap;
    for (int64_t i = lane; i < n; i += 64) f(base + i);
  }
}

// Clears the history counts and cursors and the reduction cells.
template <typename Real>
__global__ void comb_clear_kernel(CombArgs<Real> A) {
  if (blockIdx.x == 0 && threadIdx.x < 8) A.misc[threadIdx.x] = 0ull;

  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= A.n_hist; i += (int64_t)gridDim.x * blockDim.x) {
    A.cnt[i] = 0ull;
    if (i < A.n_hist) A.cur[i] = 0u;
  }
}

// Census count n, unit exponent eu and whether the largest weight is
// positive and finite, from the reduction cells (misc[0] largest weight's
// bits, misc[1] count): every kernel after the count derives them alike.
struct CombScale {
  int64_t n;
  int eu;
  bool ok;
};
__device__ inline CombScale comb_scale(const unsigned long long *misc) {
  CombScale c;
  c.n = (int64_t)misc[1];
  const double m = __longlong_as_double((long long)misc[0]);
  c.ok = c.n > 0 && m > 0.0 && m <= 1.7976931348623157e308;
  int em = 0;
  if (c.ok) frexp(m, &em);
  int ln = 0;
  while (((int64_t)1 << ln) < c.n) ++ln;
  c.eu = em + ln - 53;
  return c;
}

// Histogram by history, census count and largest weight (positive doubles
// order like their bit patterns).
template <typename Real>
__global__ void __launch_bounds__(256) comb_count_kernel(CombArgs<Real> A) {
  __shared__ unsigned long long red[2][4];
  unsigned long long mx = 0, n = 0;
  for_each_census_slot(A, [&](int64_t q) {
    const uint32_t src = A.src_bank.tag[q].src;
    if ((int64_t)src >= A.n_hist) {
      atomicOr(A.err, ERR_CAPACITY);
      return;
    }
    atomicAdd(&A.cnt[src], 1ull);
    const unsigned long long wb = (unsigned long long)__double_as_longlong(A.src_bank.w[q]);
    mx = wb > mx ? wb : mx;
    ++n;
  });
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned long long t = __shfl_xor(mx, o);
    mx = t > mx ? t : mx;
    n += __shfl_xor(n, o);
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wv] = mx;
    red[1][wv] = n;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 4; ++k) {
      mx = red[0][k] > mx ? red[0][k] : mx;
      n += red[1][k];
    }
    if (n != 0) {
      atomicMax(&A.misc[0], mx);
      atomicAdd(&A.misc[1], n);
    }
  }
}

// Scan of a[0..n) in tiles of kScanTile: local scan of each tile and its
// total into blk; then the scan of the totals; then the tile offsets added.
__device__ inline unsigned long long block_excl_scan(unsigned long long v, unsigned long long *sh,
                                                     unsigned long long *total) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = blockDim.x >> 6;
  unsigned long long x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  if (t == 0) {
    unsigned long long acc = 0;
    for (int w = 0; w < nw; ++w) {
      const unsigned long long s = sh[w];
      sh[w] = acc;
      acc += s;
    }
    sh[32] = acc;
  }
  __syncthreads();
  const unsigned long long r = sh[wv] + x - v;
  *total = sh[32];
  __syncthreads();
  return r;
}

// The length is n, or the device value *n_dev when that is smaller (the
// host launches tiles for the bound; the tiles past the end do nothing).
__device__ inline int64_t scan_len(int64_t n, const unsigned long long *n_dev) {
  return n_dev ? min(n, (int64_t)*n_dev) : n;
}

__global__ void __launch_bounds__(kScanThreads) scan_tiles_kernel(unsigned long long *a, int64_t n_bound,
                                                                  const unsigned long long *n_dev,
                                                                  unsigned long long *blk, int inclusive) {
  __shared__ unsigned long long sh[48];
  const int64_t n = scan_len(n_bound, n_dev);
  if ((int64_t)blockIdx.x * kScanTile >= n) {
    if (threadIdx.x == 0) blk[blockIdx.x] = 0ull;
    return;
  }
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  unsigned long long v[kScanPer], s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = base + k < n ? a[base + k] : 0ull;
    s += v[k];
  }
  unsigned long long total;
  unsigned long long run = block_excl_scan(s, sh, &total);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const unsigned long long nx = run + v[k];
    if (base + k < n) a[base + k] = inclusive ? nx : run;
    run = nx;
  }
  if (threadIdx.x == 0) blk[blockIdx.x] = total;
}

// One work-group scans a[0..n) a block of kScanThreads at a time, carrying
// the running total: the top level of the tiled scan, and the whole scan of
// a short array.
__global__ void __launch_bounds__(kScanThreads) scan_one_kernel(unsigned long long *a, int64_t n, int inclusive) {
  __shared__ unsigned long long sh[48];
  unsigned long long carry = 0;
  for (int64_t b0 = 0; b0 < n; b0 += kScanThreads) {
    const int64_t i = b0 + threadIdx.x;
    const unsigned long long v = i < n ? a[i] : 0ull;
    unsigned long long total;
    const unsigned long long r = block_excl_scan(v, sh, &total);
    if (i < n) a[i] = carry + r + (inclusive ? v : 0ull);
    carry += total;
  }
}

__global__ void __launch_bounds__(kScanThreads) scan_add_kernel(unsigned long long *a, int64_t n_bound,
                                                                const unsigned long long *n_dev,
                                                                const unsigned long long *blk) {
  const int64_t n = scan_len(n_bound, n_dev);
  if ((int64_t)blockIdx.x * kScanTile >= n) return;
  const unsigned long long off = blk[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k)
    if (base + k < n) a[base + k] += off;
}

// Each census particle takes the next place of its history's range.
template <typename Real>
__global__ void comb_scatter_kernel(CombArgs<Real> A) {
  for_each_census_slot(A, [&](int64_t q) {
    const uint32_t src = A.src_bank.tag[q].src;
    if ((int64_t)src >= A.n_hist) return;
    const unsigned long long pos = A.cnt[src] + atomicAdd(&A.cur[src], 1u);
    A.order[pos] = (unsigned long long)q;
  });
}

template <typename Real>
__device__ inline bool key_less(const CombArgs<Real> &A, unsigned long long qa, unsigned long long qb) {
  const uint64_t la = A.src_bank.lin[qa], lb = A.src_bank.lin[qb];
  if (la != lb) return la < lb;
  return A.src_bank.tag[qa].e < A.src_bank.tag[qb].e;
}

// Canonical position of every census particle of a history with at most
// kSmallBin particles: its history's start plus the number of the history's
// particles of smaller (lineage, event), ties by current place.  The sorted
// slot indices go to wq.  Longer histories are listed for the work-group
// sort: misc[4] counts them, their ids go to cur[] (the cursors are free
// again after the scatter).
template <typename Real>
__global__ void comb_rank_small_kernel(CombArgs<Real> A) {
  const CombScale c = comb_scale(A.misc);
  if (!c.ok) return;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < c.n; p += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long q = A.order[p];
    const uint32_t s = A.src_bank.tag[q].src;
    const int64_t lo = (int64_t)A.cnt[s], m = (int64_t)A.cnt[s + 1] - lo;
    if (m > kSmallBin) {
      if (p == lo) {
        const unsigned long long slot = atomicAdd(&A.misc[4], 1ull);
        A.cur[slot] = s;
      }
      continue;
    }
    const uint64_t li = A.src_bank.lin[q];
    const uint32_t ei = A.src_bank.tag[q].e;
    int64_t rank = 0;
    for (int64_t j = lo; j < lo + m; ++j) {
      const unsigned long long qj = A.order[j];
      const uint64_t lj = A.src_bank.lin[qj];
      const uint32_t ej = A.src_bank.tag[qj].e;
      rank += (lj < li || (lj == li && (ej < ei || (ej == ei && j < p)))) ? 1 : 0;
    }
    A.wq[lo + rank] = q;
  }
}

// Histories with many particles: one work-group each; particle i goes to
// place (number of particles of smaller key, ties by current place), keys
// staged through LDS a tile at a time; the sorted slot indices go to wq.
template <typename Real>
__global__ void __launch_bounds__(1024) comb_sort_big_kernel(CombArgs<Real> A) {
  __shared__ uint64_t kl[1024];
  __shared__ uint32_t ke[1024];
  const int64_t nbig = (int64_t)A.misc[4];
  for (int64_t g = blockIdx.x; g < nbig; g += gridDim.x) {
    const int64_t s = A.cur[g];
    const int64_t lo = (int64_t)A.cnt[s], m = (int64_t)A.cnt[s + 1] - lo;
    for (int64_t i0 = 0; i0 < m; i0 += blockDim.x) {
      const int64_t i = i0 + threadIdx.x;
      uint64_t li = 0;
      uint32_t ei = 0;
      if (i < m) {
        const unsigned long long q = A.order[lo + i];
        li = A.src_bank.lin[q];
        ei = A.src_bank.tag[q].e;
      }
      int64_t rank = 0;
      for (int64_t j0 = 0; j0 < m; j0 += blockDim.x) {
        __syncthreads();
        const int64_t j = j0 + threadIdx.x;
        if (j < m) {
          const unsigned long long q = A.order[lo + j];
          kl[threadIdx.x] = A.src_bank.lin[q];
          ke[threadIdx.x] = A.src_bank.tag[q].e;
        }
        __syncthreads();
        const int64_t jn = min((int64_t)blockDim.x, m - j0);
        if (i < m)
          for (int64_t t = 0; t < jn; ++t) {
            const uint64_t lj = kl[t];
            const uint32_t ej = ke[t];
            const bool less = lj < li || (lj == li && (ej < ei || (ej == ei && j0 + t < i)));
            rank += less ? 1 : 0;
          }
      }
      if (i < m) A.wq[lo + rank] = A.order[lo + i];
    }
    __syncthreads();
  }
}

// The sorted slot indices move from wq to order, and wq takes the integer
// weights in units of 2^eu, in canonical order.
template <typename Real>
__global__ void comb_weights_kernel(CombArgs<Real> A) {
  // The history counts are done with; their first cells take the integer
  // chunk sums of a comb by index.
  if (blockIdx.x == 0 && threadIdx.x < 8) A.cnt[threadIdx.x] = 0ull;
  const CombScale c = comb_scale(A.misc);
  if (!c.ok) return;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < c.n; j += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long q = A.wq[j];
    A.order[j] = q;
    A.wq[j] = (unsigned long long)rint(ldexp(A.src_bank.w[q], -c.eu));
  }
}

// Place of comb copy k in the new bank: region (k mod B, (k / B) mod nc),
// the region's copies spread over its K segments in runs of `per`, the rest
// (if a run would pass seg_cap) in the overflow segment.
struct CombPlace {
  int64_t slot;
  bool ok;
};
__device__ __host__ inline void comb_region(int64_t H, int B, int nc, int b, int c, int64_t *n_bc) {
  const int64_t n_b = H > b ? (H - b + B - 1) / B : 0;
  *n_bc = n_b > c ? (n_b - c + nc - 1) / nc : 0;
}
__device__ inline CombPlace comb_place(int64_t k, int64_t H, int B, int nc, const BankGeom &G) {
  const int b = (int)(k % B);
  const int64_t t = k / B;
  const int c = (int)(t % nc);
  const int64_t q = t / nc;
  int64_t n_bc;
  comb_region(H, B, nc, b, c, &n_bc);
  const int64_t per = min(G.seg_cap, (n_bc + G.K - 1) / G.K);
  const int64_t r0 = ((int64_t)b * nc + c) * G.stride;
  CombPlace p{0, true};
  const int64_t s = q / per;
  if (s < G.K) {
    p.slot = r0 + s * G.seg_cap + (q - s * per);
  } else {
    const int64_t o = q - (int64_t)G.K * per;
    p.ok = o < G.ovf_cap;
    p.slot = r0 + (int64_t)G.K * G.seg_cap + o;
  }
  return p;
}

// Tooth k: by weight, the first particle whose inclusive prefix exceeds
// (k + xi) delta; by index, the particle at canonical position
// floor((k + xi) n / n_target).
template <typename Real>
__global__ void comb_teeth_kernel(CombArgs<Real> A) {
  const CombScale c = comb_scale(A.misc);
  if (!c.ok) return;
  const int64_t n = c.n;
  const int eu = c.eu;
  uint32_t r[4];
  draw(A.seed, A.key1, SLOT_COMB, A.step, 0ull, 0u, r);
  const double xi = u53(r[0], r[1]);
  const double W = (double)A.wq[n - 1];
  const double delta = A.by_index ? (double)n / (double)A.n_target : W / (double)A.n_target;
  const double w_out = ldexp(W, eu) / (double)A.n_target;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < A.n_target;
       k += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo;
    if (A.by_index) {
      lo = (int64_t)(((double)k + xi) * delta);
      if (lo >= n) lo = n - 1;
    } else {
      double t = ((double)k + xi) * delta;
      if (t >= W) t = W - 1.0;
      lo = 0;
      int64_t hi = n - 1;
      while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if ((double)A.wq[mid] > t) hi = mid;
        else lo = mid + 1;
      }
    }
    const unsigned long long q = A.order[lo];
    const CombPlace pl = comb_place(k, A.n_target, A.B, A.nc, A.G);
    if (!pl.ok) {
      atomicOr(A.err, ERR_CAPACITY);
      continue;
    }
    double wc = w_out;
    if (A.by_index) {
      const unsigned long long wi = A.wq[lo] - (lo > 0 ? A.wq[lo - 1] : 0ull);
      wc = ldexp((double)wi, eu) * delta;
      atomicAdd(&A.cnt[(int)((k / A.B) % A.nc)], wi);
    }
    A.dst_bank.xm[pl.slot] = A.src_bank.xm[q];
    A.dst_bank.w[pl.slot] = wc;
    A.dst_bank.lin[pl.slot] = (uint64_t)A.step;
    Tag tg;
    tg.src = (uint32_t)k;
    tg.e = 0u;
    tg.cell = A.src_bank.tag[q].cell;
    A.dst_bank.tag[pl.slot] = tg;
  }
}

// Segment counts of the new bank, chunk weights count * W / n_target and
// the total weight W for the host (misc[2]).  One work-group: a thread per
// segment, the chunk counts summed in LDS.
template <typename Real>
__global__ void __launch_bounds__(1024) comb_finish_kernel(CombArgs<Real> A) {
  __shared__ unsigned long long chunk[8];
  const CombScale cs = comb_scale(A.misc);
  const BankGeom &G = A.G;
  if (!cs.ok) {
    // Nothing combed.  When the host does not wait for the census size, it
    // takes the new bank as the census anyway: make that bank empty.
    if (!A.no_wait) return;
    for (int64_t t = threadIdx.x; t < (int64_t)A.R * G.K; t += blockDim.x) A.dst_bank.segcnt[t] = 0u;
    for (int t = threadIdx.x; t < A.R; t += blockDim.x) A.dst_bank.ovfcnt[t] = 0u;
    if (threadIdx.x < (unsigned)A.nc) A.wnext[threadIdx.x] = 0.0;
    if (threadIdx.x == 0 && cs.n > 0) atomicOr(A.err, ERR_COMB_WEIGHT);
    return;
  }
  if (threadIdx.x < 8) chunk[threadIdx.x] = 0ull;
  __syncthreads();
  const int64_t nseg = (int64_t)A.R * (G.K + 1);
  for (int64_t t = threadIdx.x; t < nseg; t += blockDim.x) {
    const int r = (int)(t / (G.K + 1)), s = (int)(t - (int64_t)r * (G.K + 1));
    const int b = r / A.nc, c = r % A.nc;
    int64_t n_bc;
    comb_region(A.n_target, A.B, A.nc, b, c, &n_bc);
    const int64_t per = min(G.seg_cap, (n_bc + G.K - 1) / G.K);
    if (s < G.K) {
      const int64_t left = n_bc - (int64_t)s * per;
      A.dst_bank.segcnt[(int64_t)r * G.K + s] = (uint32_t)(left < 0 ? 0 : (left < per ? left : per));
    } else {
      const int64_t over = n_bc - (int64_t)G.K * per;
      A.dst_bank.ovfcnt[r] = (uint32_t)(over > 0 ? over : 0);
      atomicAdd(&chunk[c], (unsigned long long)n_bc);
    }
  }
  __syncthreads();
  const double W = (double)A.wq[cs.n - 1];
  const double w_out = ldexp(W, cs.eu) / (double)A.n_target;
  if (threadIdx.x < (unsigned)A.nc)
    A.wnext[threadIdx.x] = A.by_index ? ldexp((double)A.cnt[threadIdx.x], cs.eu) * ((double)cs.n / (double)A.n_target)
                                      : (double)chunk[threadIdx.x] * w_out;
  if (threadIdx.x == 0) A.misc[2] = (unsigned long long)__double_as_longlong(ldexp(W, cs.eu));
}

// Scan of a[0..n) (n bounded by *n_dev when given): one work-group for a
// short array, else tiles, their totals, and the tile offsets added.
hipError_t scan(unsigned long long *a, int64_t n, const unsigned long long *n_dev, unsigned long long *blk,
                int inclusive, hipStream_t s) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 0) return hipSuccess;
  if (!n_dev && nb <= 4) {
    hipLaunchKernelGGL(scan_one_kernel, dim3(1), dim3(kScanThreads), 0, s, a, n, inclusive);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(scan_tiles_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, a, n, n_dev, blk, inclusive);
  hipLaunchKernelGGL(scan_one_kernel, dim3(1), dim3(kScanThreads), 0, s, blk, nb, 0);
  hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, a, n, n_dev, blk);
  return hipGetLastError();
}

unsigned grid_for(int64_t n, int block) {
  const int64_t g = (n + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

}  // namespace

int64_t comb_scan_blocks(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

template <typename Real>
hipError_t launch_comb(const CombArgs<Real> &a, hipStream_t s) {
  const int64_t nseg = (int64_t)a.R * (a.G.K + 1);
  const unsigned seg_grid = grid_for(nseg, 4);  // four wavefronts of 64 per work-group
  hipLaunchKernelGGL(comb_clear_kernel<Real>, dim3(grid_for(a.n_hist + 1, 256)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(comb_count_kernel<Real>, dim3(seg_grid), dim3(256), 0, s, a);
  hipError_t e = scan(a.cnt, a.n_hist + 1, nullptr, a.blk, 0, s);
  if (e != hipSuccess) return e;
  const unsigned cen_grid = grid_for(a.cap, 256);
  hipLaunchKernelGGL(comb_scatter_kernel<Real>, dim3(seg_grid), dim3(256), 0, s, a);
  hipLaunchKernelGGL(comb_rank_small_kernel<Real>, dim3(cen_grid), dim3(256), 0, s, a);
  hipLaunchKernelGGL(comb_sort_big_kernel<Real>, dim3(256), dim3(1024), 0, s, a);
  hipLaunchKernelGGL(comb_weights_kernel<Real>, dim3(cen_grid), dim3(256), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan(a.wq, a.cap, a.misc + 1, a.blk, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(comb_teeth_kernel<Real>, dim3(grid_for(a.n_target, 256)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(comb_finish_kernel<Real>, dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_comb<double>(const CombArgs<double> &, hipStream_t);
template hipError_t launch_comb<float>(const CombArgs<float> &, hipStream_t);

}  // namespace hww
