// Hybrid low-order second-moment (HLOSM) solve on the device (Shaw &
// Anistratov, arXiv 2512.19925, Sec. 3 Eqs. losm-disc and losm-disc-semi;
// moving-average filter of Sec. 4; window centres of Sec. 2 Eq. ww-center).
//
// The interleaved tridiagonal system of 2I+3 unknowns
// [phi_0, J_0, phi_1, J_1, ..., J_I, phi_{I+1}] has a matrix that depends
// only on the mesh, the cross sections, v, dt and theta, so its LU factors
// (Gaussian elimination without pivoting, the Thomas algorithm) are computed
// once per theta by losm_factor_kernel.  Each solve (losm_kernel, one
// work-group) then
//   1. adds up the batch-sum copies that the sweep's work-groups flushed, of
//      the initial-condition set (census at t^{n-1}) and of the closure set,
//      and the per-batch face tallies
//   2. forms phi^{n-1}, J^{n-1} at edges (linear interpolation of
//      cell-average currents), F^{n-1}, F^n, P_L, P_R
//   3. optionally moving-average filters F^n, F^{n-1}, phi^{n-1}, J^{n-1}
//   4. assembles the right-hand side
//   5. runs the forward and backward substitutions, each a first-order
//      affine recurrence, as a parallel scan over the work-group
//   6. sets the window centres s [(max(phi,0)/max phi)(1-eps) + eps],
//      ceiling and floor (Sec. 2 Eq. ww-c&f).
#include "hww_losm_dev.h"

namespace hww {

static constexpr int LOSM_THREADS = 1024;
static constexpr double kThird = 1.0 / 3.0;

// Thomas factors of the solve matrix for A.theta, then the old-time
// diagonal of every row: factor = [alpha | 1/den | gamma | bb], each 2I+3
// long.  The elimination runs on one lane, the diagonals on all; once per
// theta.
__device__ inline void losm_factor_body(const LosmArgs &A) {
  const double inv_vdt = 1.0 / (A.v * A.dt);
  const int n = 2 * A.I + 3;
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    double ba, bb, bc;
    losm_brow(A.I, A.edges, A.sig_t, A.sig_s, A.theta, inv_vdt, r, &ba, &bb, &bc);
    A.factor[3 * n + r] = bb;
  }
  if (threadIdx.x != 0) return;
  if (!losm_factor_seq(A.I, A.edges, A.sig_t, A.sig_s, A.theta, inv_vdt, false, A.factor)) {
    atomicOr(A.err, ERR_NUMERIC);
    *A.status = (int)ERR_NUMERIC;
  }
}

__global__ void losm_factor_kernel(LosmArgs A) {
  if (blockIdx.x != 0) return;
  losm_factor_body(A);
}

// Moving average (Sec. 4 Eq. moving_average) of value m of in[0..M) into
// out[m]: the mean over the 2k+1 values centred on it, the window shrunk
// symmetrically where it would leave the range; terms added in the order
// l = -k..k.
template <int K>
__device__ __forceinline__ double ma_full(const double *in, int m) {
  double x[2 * K + 1];
#pragma unroll
  for (int l = -K; l <= K; ++l) x[l + K] = in[m - l];
  double acc = 0.0;
#pragma unroll
  for (int l = 0; l <= 2 * K; ++l) acc += x[l];
  return acc * (1.0 / (double)(2 * K + 1));
}

__device__ inline void ma_point(const double *in, double *out, int M, int m, int k) {
  int km = k;
  if (m < km) km = m;
  if (M - 1 - m < km) km = M - 1 - m;
  // Full windows of the usual widths: the window's loads issued together.
  if (km == k && k >= 1 && k <= 4) {
    out[m] = k == 1 ? ma_full<1>(in, m) : k == 2 ? ma_full<2>(in, m) : k == 3 ? ma_full<3>(in, m) : ma_full<4>(in, m);
    return;
  }
  double acc = 0.0;
  for (int l = -km; l <= km; ++l) acc += in[m - l];
  out[m] = acc / (double)(2 * km + 1);
}

// Fourier low pass (Sec. 4, Eqs. fft and ifft) of in[0..M) into out: of the
// discrete Fourier transform keep the frequencies 0..kappa and their
// negatives (the real low pass; kappa >= M/2 keeps everything).  The kept
// coefficients go to xc (2 (M/2 + 1) doubles).  One wave per coefficient,
// then one thread per output value; the phase factors are advanced by
// complex multiplication (no table, so no LDS bank conflicts).
__device__ void fourier_filter_dev(const double *in, double *out, int M, int kappa, double *xc) {
  const int T = blockDim.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = T >> 6;
  const int kk = kappa < M / 2 ? kappa : M / 2;
  double *xr = xc, *xi = xc + (M / 2 + 1);
  for (int j = wv; j <= kk; j += nw) {
    // e^{-i 2 pi j m / M} at m = lane, advanced by e^{-i 2 pi 64 j / M}.
    double s0, c0, sd, cd;
    sincospi(2.0 * (double)(((int64_t)j * lane) % M) / (double)M, &s0, &c0);
    sincospi(2.0 * (double)((64 * (int64_t)j) % M) / (double)M, &sd, &cd);
    double zr = c0, zi = -s0;
    const double wr = cd, wi = -sd;
    double re = 0.0, im = 0.0;
    for (int m = lane; m < M; m += 64) {
      re += in[m] * zr;
      im += in[m] * zi;
      const double t = zr * wr - zi * wi;
      zi = zr * wi + zi * wr;
      zr = t;
    }
    for (int o = 32; o >= 1; o >>= 1) {
      re += __shfl_xor(re, o);
      im += __shfl_xor(im, o);
    }
    if (lane == 0) {
      xr[j] = re;
      xi[j] = im;
    }
  }
  __syncthreads();
  for (int m = tid; m < M; m += T) {
    double sm, cm;
    sincospi(2.0 * (double)m / (double)M, &sm, &cm);
    double zr = 1.0, zi = 0.0, acc = xr[0];
    for (int j = 1; j <= kk; ++j) {
      const double t = zr * cm - zi * sm;  // e^{i 2 pi j m / M}
      zi = zr * sm + zi * cm;
      zr = t;
      const double term = xr[j] * zr - xi[j] * zi;
      acc += (2 * j == M) ? term : 2.0 * term;
    }
    out[m] = acc / (double)M;
  }
  __syncthreads();
}

// Fourier low pass of the cell values f[1..I] of a grid function into the
// spare buffer, face values f[0], f[I+1] copied; the two pointers swap.
__device__ __forceinline__ void fourier_cells_swap(double *&f, double *&spare, int I, int kappa, double *xc) {
  fourier_filter_dev(f + 1, spare + 1, I, kappa, xc);
  if (threadIdx.x == 0) {
    spare[0] = f[0];
    spare[I + 1] = f[I + 1];
  }
  __syncthreads();
  double *t = f;
  f = spare;
  spare = t;
}

// Layout of a solve's working arrays (M = I + 2 doubles each): eight grid
// functions, in LDS when they fit (work_in_lds) else at the start of the
// global scratch; the initial condition's normalised batch sums after them
// in the global scratch (kept there for the later solves of the step); the
// Fourier coefficients after those.
__device__ inline double *losm_sums(const LosmArgs &A) { return A.scratch + 8 * (A.I + 2); }
__device__ inline double *losm_fourier_scratch(const LosmArgs &A) { return A.scratch + 12 * (A.I + 2) + 16; }

// kWil: where the working arrays live (0 global scratch, 1 LDS, 2 LDS with
// the Fourier coefficients too), fixed at compile time so that every access
// is a plain LDS or global one.
//
// The solve is a chain of dependent phases on one work-group, so its time
// is the latency of that chain.  All global reads of the inputs are issued
// at once at the start (the closure scale and the early-exit checks are
// wave-uniform values every wave computes for itself), and the phases meet
// at seven barriers.
template <int kWil>
__device__ __forceinline__ void losm_body(const LosmArgs &A, double *dyn) {
  const int I = A.I;
  const int M = I + 2;
  const int n = 2 * I + 3;
  const int tid = threadIdx.x;
  const int T = blockDim.x;
  double *u = dyn;  // [n] right-hand side, then solution
  double *S = kWil ? dyn + n : A.scratch;
  // Each thread's rows of the substitutions, loaded now to overlap the
  // first phases (up to kScanRows rows per thread, else read when used).
  constexpr int kScanRows = 4;
  const bool rows_in_regs = (n + T - 1) / T <= kScanRows;
  ScanRows<kScanRows> R;
  if (rows_in_regs) losm_scan_prefetch(A.factor, n, R);
  // Grid functions and four spare buffers; filters write into the spares and
  // the pointers swap.
  double *phi_o = S, *J_o = S + M, *F_o = S + 2 * M, *F_n = S + 3 * M;
  double *T1 = S + 4 * M, *T2 = S + 5 * M, *T3 = S + 6 * M, *T4 = S + 7 * M;
  double *gi_phi = losm_sums(A);
  double *gi_J = gi_phi + I;
  double *gi_K = gi_J + I;
  __shared__ double sp[64], sq[64];
  __shared__ double face[12];  // ic: phi L/R, P L/R, F L/R; cl: same
  __shared__ int bad;
  __shared__ double red[LOSM_THREADS / 64];

  // Wave-uniform set-up: a failed factorization stays failed; the closure
  // scale W_start / W_done (1 when semi-implicit; zero when no start weight
  // has been swept yet, so that no closures exist and the update is
  // skipped); the start weight of the step per source particle.
  const bool failed = *A.status != 0;
  double wtot = 0.0, wn = 0.0, wdone = 0.0;
  for (int q = 0; q < A.nc; ++q) {
    wtot += A.wstart[q];
    wn += A.wnext[q];
    if (q < A.next_chunk) wdone += A.wstart[q];
  }
  const double scale = A.implicit ? (wdone > 0.0 ? wtot / wdone : 0.0) : 1.0;
  const double s_w = (A.implicit ? wtot : wn) / A.n_src;
  const bool skip = A.implicit && !(scale > 0.0);
  if (tid == 0) bad = 0;

  // 1.-2. Batch sums of the tallies (the copies the sweep flushed),
  // normalised per source particle and cell width (and step for
  // track-length closures; the closure set scaled by W_start / W_done), and
  // the grid functions of the initial condition and the closures made from
  // them at once: the thread of cell c reads what grid point c + 1 needs,
  // the current of cell c + 1 included.
  for (int t = tid >> 6; t < 12; t += T >> 6) {
    // Face values, one wave each (lane = batch, B <= 64): t = (phi L,
    // phi R, P L, P R, F L, F R) of the initial-condition set (t < 6) and
    // of the closure set (t >= 6).  The waves write the boundary entries of
    // the grid functions themselves; the waves of P L and P R also add up
    // phi L and phi R for the boundary currents.
    const int bl = tid & 63;
    const int set = t / 6, q = t % 6;
    const int f = q & 1, kind = q >> 1;
    const double *bs = set == 0 ? A.bnd_ic : A.bnd_cl;
    double acc = bl < A.B ? bs[(bl * 2 + f) * 3 + kind] : 0.0;
    double acc0 = (t == 2 || t == 3) && bl < A.B ? A.bnd_ic[(bl * 2 + f) * 3] : 0.0;
    acc = wave_sum_f64(acc);
    if (t == 2 || t == 3) acc0 = wave_sum_f64(acc0);
    if (bl == 0) {
      const double v = (set == 0 ? 1.0 : scale) * acc / (A.n_src * A.dt);
      face[t] = v;
      const int e = f ? I + 1 : 0;
      if (t == 0 || t == 1) phi_o[e] = v;
      if (t == 2) J_o[0] = -0.5 * (acc0 / (A.n_src * A.dt)) + v;
      if (t == 3) J_o[I] = 0.5 * (acc0 / (A.n_src * A.dt)) - v;
      if (t == 4 || t == 5) {
        F_o[e] = v;
        if (!A.implicit) F_n[e] = v;
      }
      if ((t == 10 || t == 11) && A.implicit) F_n[e] = v;
    }
  }
  {
    const int kc = A.closure_track ? 0 : 3;
    for (int c = tid; c < I; c += T) {
      const int i = c + 1;
      const bool right = c + 1 < I;  // an interior edge to the right
      const double xl = A.edges[c], xr = A.edges[c + 1];
      const double xrr = right ? A.edges[c + 2] : xr;
      double p = 0.0, j = 0.0, k = 0.0, jn = 0.0;
      if (A.ic_cached) {
        p = gi_phi[c];
        j = gi_J[c];
        k = gi_K[c];
        if (right) jn = gi_J[c + 1];
      } else {
#pragma unroll
        for (int s = 0; s < kSumCopies; ++s) {
          const double *t = A.tsum_ic + (size_t)s * 6 * I;
          p += t[3 * I + c];
          j += t[4 * I + c];
          k += t[5 * I + c];
          if (right) jn += t[4 * I + c + 1];
        }
      }
      double cp = 0.0, ck = 0.0;
#pragma unroll
      for (int s = 0; s < kSumCopies; ++s) {
        const double *t = A.tsum_cl + (size_t)s * 6 * I;
        cp += t[kc * I + c];
        ck += t[(kc + 2) * I + c];
      }
      const double dl = xr - xl, dr = xrr - xr;
      const double norm = A.n_src * dl;
      // The solve runs on one compute unit, so its FP64 divisions are a
      // large share of its issue time: each divisor is inverted once.
      if (!A.ic_cached) {
        const double inv = 1.0 / norm;
        p = p * inv;
        j = j * inv;
        k = k * inv;
        if (right) jn = jn * (1.0 / (A.n_src * dr));  // as the next cell's thread scales its own
        gi_phi[c] = p;
        gi_J[c] = j;
        gi_K[c] = k;
      }
      const double normc = A.closure_track ? norm * A.dt : norm;
      const double sn = scale / normc;
      const double gcp = cp * sn, gck = ck * sn;
      phi_o[i] = p;
      const double fo = p * kThird - k;
      F_o[i] = fo;
      F_n[i] = A.implicit ? gcp * kThird - gck : fo;
      if (right) J_o[i] = (dr * j + dl * jn) / (dl + dr);
      if (A.lagged) {
        // Lagged windows: the shape is the previous step's Monte Carlo
        // track-length flux (the closure set read as track tallies).
        u[2 * i] = gcp;
        u[2 * i - 1] = 0.0;
      }
    }
    if (A.lagged && tid == 0) {
      u[0] = 0.0;
      u[2 * I + 1] = 0.0;
      u[2 * I + 2] = 0.0;
    }
  }
  __syncthreads();
  if (failed) return;
  if (skip) {
    for (int i = tid; i <= I + 1; i += T) A.phi_out[i] = 0.0;
    for (int i = tid; i <= I; i += T) A.J_out[i] = 0.0;
    return;
  }
  const double PL = A.implicit ? face[8] : face[2];
  const double PR = A.implicit ? face[9] : face[3];

  if (A.export_only) {
    // Closures and initial condition of the finished step, unfiltered.
    for (int i = tid; i <= I + 1; i += T) {
      A.phi_out[i] = phi_o[i];
      A.F_out[i] = F_o[i];
    }
    for (int i = tid; i <= I; i += T) A.J_out[i] = J_o[i];
    if (tid == 0) {
      A.P_out[0] = PL;
      A.P_out[1] = PR;
    }
    return;
  }

  if (!A.lagged) {
  // 3. filters of F^n, F^{n-1}, phi^{n-1} (cell values) and J^{n-1} (edges).
  if (A.filter == 1) {
    // Moving average of the cell values of phi (g = 0), F^{n-1} (2), F^n
    // (3) and of the edge values of J (1), grid function g at S + g M into
    // S + (4 + g) M, as one loop over all of their values (one copy of the
    // loop's code runs for all four); faces copied along.
    for (int g = 0; g < 4; ++g) {
      const int off = g == 1 ? 0 : 1, len = g == 1 ? I + 1 : I;
      for (int m = tid; m < len; m += T) ma_point(S + g * M + off, S + (4 + g) * M + off, len, m, A.ma_k);
    }
    if (tid == 0) {
      T1[0] = phi_o[0]; T1[I + 1] = phi_o[I + 1];
      T3[0] = F_o[0]; T3[I + 1] = F_o[I + 1];
      T4[0] = F_n[0]; T4[I + 1] = F_n[I + 1];
    }
    __syncthreads();
    phi_o = T1; J_o = T2; F_o = T3; F_n = T4;
  } else if (A.filter == 2) {
    // Fourier low pass, one grid function at a time.
    double *xc = kWil == 2 ? S + 8 * M : losm_fourier_scratch(A);
    fourier_cells_swap(F_n, T1, I, A.kappa, xc);
    fourier_cells_swap(F_o, T1, I, A.kappa, xc);
    fourier_cells_swap(phi_o, T1, I, A.kappa, xc);
    fourier_filter_dev(J_o, T1, I + 1, A.kappa, xc);
    double *old = J_o;
    J_o = T1;
    T1 = old;
  }

  // 4. right-hand side, 5. substitutions as parallel scans of affine
  // recurrences.  With the rows in registers each thread assembles the
  // rows it then scans first, so no barrier sits between the two.
  const double th = A.theta;
  if (rows_in_regs) {
    const int m = (n + T - 1) / T, r0 = tid * m, cnt = min(m, n - r0);
#pragma unroll
    for (int k = 0; k < kScanRows; ++k)
      if (k < cnt) u[r0 + k] = losm_rhs_bb(I, th, r0 + k, R.bb[k], phi_o, J_o, F_o, F_n, PL, PR);
    losm_solve_scans_rows(u, n, R, sp, sq);
  } else {
    for (int r = tid; r < n; r += T)
      u[r] = losm_rhs_bb(I, th, r, A.factor[3 * n + r], phi_o, J_o, F_o, F_n, PL, PR);
    __syncthreads();
    losm_solve_scans(u, n, A.factor, sp, sq);
  }
  }

  // 6. window centres (an empty bank has nothing to window: unchanged).
  // The largest flux by a wave maximum and one barrier; every thread then
  // reads the waves' maxima.
  if (A.apply_windows && s_w > 0.0) {
    double mx = -__builtin_inf();
    int nonfinite = 0;
    for (int i = tid; i < I; i += T) {
      const double p = u[2 * (i + 1)];
      if (!isfinite(p)) nonfinite = 1;
      if (p > mx) mx = p;
    }
    mx = wave_max_f64(mx);
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    if (nonfinite) atomicOr(&bad, 1);
    __syncthreads();
    const int lane = tid & 63;
    const double mm = wave_max_f64(lane < (T >> 6) ? red[lane] : -__builtin_inf());
    const double inv_mm = 1.0 / mm, inv_rho = 1.0 / A.rho;
    bool numeric = bad != 0, keep = false;
    // A lagged shape without any track flux (the first step) leaves the
    // windows as they are.
    if (!(mm > 0.0)) {
      if (A.lagged && !numeric) keep = true;
      else numeric = true;
    }
    if (numeric) {
      if (tid == 0) atomicOr(A.err, ERR_NUMERIC);
    } else if (!keep) {
      const double s = A.window_scale ? 1.0 : s_w;
      for (int i = tid; i < I; i += T) {
        const double p = u[2 * (i + 1)];
        const double rr = p > 0.0 ? p * inv_mm : 0.0;
        const double ww = s * (rr * (1.0 - A.eps_min) + A.eps_min);
        Window wd;
        wd.ww = ww;
        wd.ceil = ww * A.rho;
        wd.floor = ww * inv_rho;
        wd.pad = 0.0;
        A.win[i] = wd;
      }
    }
  }
  for (int i = tid; i <= I + 1; i += T) A.phi_out[i] = u[2 * i];
  for (int i = tid; i <= I; i += T) A.J_out[i] = u[2 * i + 1];
}

template <int kWil>
__global__ void __launch_bounds__(LOSM_THREADS) losm_kernel(LosmArgs A) {
  extern __shared__ double dyn[];
  losm_body<kWil>(A, dyn);
}

// Batched solves: replica r of the table takes block r (factor, solve); the
// call options are shared.
__device__ inline LosmArgs losm_batch_args(const LosmReplica &R, const LosmCall &c) {
  LosmArgs A = R.a;
  if (!c.implicit) {
    A.tsum_ic = R.tsum[c.cur]; A.bnd_ic = R.bnd[c.cur];
    A.tsum_cl = A.tsum_ic; A.bnd_cl = A.bnd_ic;
  } else {
    A.tsum_ic = R.tsum[1 - c.cur]; A.bnd_ic = R.bnd[1 - c.cur];
    A.tsum_cl = R.tsum[c.cur]; A.bnd_cl = R.bnd[c.cur];
  }
  A.next_chunk = c.next_chunk;
  A.theta = c.theta;
  A.implicit = c.implicit; A.filter = c.filter; A.ma_k = c.ma_k;
  A.kappa = c.kappa; A.lagged = c.lagged; A.ic_cached = c.ic_cached; A.window_scale = c.window_scale;
  A.closure_track = c.closure_track; A.apply_windows = c.apply_windows;
  A.eps_min = c.eps_min; A.rho = c.rho;
  A.refactor = c.refactor; A.work_in_lds = c.work_in_lds; A.export_only = c.export_only;
  return A;
}

__global__ void losm_factor_batch_kernel(const LosmReplica *tab, LosmCall c) {
  const LosmArgs A = losm_batch_args(tab[blockIdx.x], c);
  if (threadIdx.x == 0) *A.status = 0;
  losm_factor_body(A);
}

template <int kWil>
__global__ void __launch_bounds__(LOSM_THREADS) losm_batch_kernel(const LosmReplica *tab, LosmCall c) {
  extern __shared__ double dyn[];
  const LosmArgs A = losm_batch_args(tab[blockIdx.x], c);
  losm_body<kWil>(A, dyn);
}

// Dynamic LDS of a solve of I cells: the unknowns; then, when they fit
// beside the 16 KB of static LDS, the working grid functions (work_in_lds
// 1) and also the Fourier filter's coefficients (2).
static size_t losm_lds(int I, int *work_in_lds) {
  const size_t lds_min = (size_t)(2 * I + 3) * sizeof(double);
  const size_t lds_full = lds_min + (size_t)8 * (I + 2) * sizeof(double);
  const size_t lds_four = lds_full + (size_t)((I + 2) + 4) * sizeof(double);
  const size_t budget = 160 * 1024 - 2 * 1024;  // static LDS of the solve: about 1.3 KB
  *work_in_lds = lds_four <= budget ? 2 : (lds_full <= budget ? 1 : 0);
  return *work_in_lds == 2 ? lds_four : (*work_in_lds == 1 ? lds_full : lds_min);
}

static hipError_t allow_losm_lds(const void *fn, size_t lds, size_t *done) {
  if (lds > 32 * 1024 && lds > *done) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    *done = lds;
  }
  return hipSuccess;
}

size_t losm_batch_lds(int max_I, int *work_in_lds) { return losm_lds(max_I, work_in_lds); }

hipError_t launch_losm_batch(const LosmReplica *tab, int n, int max_I, const LosmCall &c, hipStream_t s) {
  if (c.refactor) {
    hipLaunchKernelGGL(losm_factor_batch_kernel, dim3(n), dim3(64), 0, s, tab, c);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  int wil = 0;
  const size_t lds = losm_lds(max_I, &wil);
  if (wil != c.work_in_lds) return hipErrorInvalidValue;
  static size_t done[3] = {0, 0, 0};
  const void *fn = wil == 2 ? reinterpret_cast<const void *>(&losm_batch_kernel<2>)
                 : wil == 1 ? reinterpret_cast<const void *>(&losm_batch_kernel<1>)
                            : reinterpret_cast<const void *>(&losm_batch_kernel<0>);
  {
    const hipError_t e = allow_losm_lds(fn, lds, &done[wil]);
    if (e != hipSuccess) return e;
  }
  if (wil == 2) hipLaunchKernelGGL(losm_batch_kernel<2>, dim3(n), dim3(LOSM_THREADS), lds, s, tab, c);
  else if (wil == 1) hipLaunchKernelGGL(losm_batch_kernel<1>, dim3(n), dim3(LOSM_THREADS), lds, s, tab, c);
  else hipLaunchKernelGGL(losm_batch_kernel<0>, dim3(n), dim3(LOSM_THREADS), lds, s, tab, c);
  return hipGetLastError();
}

hipError_t launch_losm(const LosmArgs &a, hipStream_t s) {
  if (a.refactor) {
    hipLaunchKernelGGL(losm_factor_kernel, dim3(1), dim3(64), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  LosmArgs b = a;
  const size_t lds = losm_lds(a.I, &b.work_in_lds);
  const int wil = b.work_in_lds;
  static size_t done[3] = {0, 0, 0};
  const void *fn = wil == 2 ? reinterpret_cast<const void *>(&losm_kernel<2>)
                 : wil == 1 ? reinterpret_cast<const void *>(&losm_kernel<1>)
                            : reinterpret_cast<const void *>(&losm_kernel<0>);
  {
    const hipError_t e = allow_losm_lds(fn, lds, &done[wil]);
    if (e != hipSuccess) return e;
  }
  if (wil == 2) hipLaunchKernelGGL(losm_kernel<2>, dim3(1), dim3(LOSM_THREADS), lds, s, b);
  else if (wil == 1) hipLaunchKernelGGL(losm_kernel<1>, dim3(1), dim3(LOSM_THREADS), lds, s, b);
  else hipLaunchKernelGGL(losm_kernel<0>, dim3(1), dim3(LOSM_THREADS), lds, s, b);
  return hipGetLastError();
}

}  // namespace hww
