// Deterministic LOSM march with frozen Monte Carlo closures and its
// hand-written adjoint (Shaw & Anistratov, arXiv 2512.19925, Sec. 3 Eqs.
// losm-disc): for given per-cell sigma_t, sigma_s, the march takes n fully
// implicit theta-scheme steps A u^n = B u^{n-1} + g^n from u^0 = (phi^0, J^0)
// with the closures F^n, P^n recorded from a Monte Carlo run, and evaluates
// G = sum_n sum_i w_{n,i} phi_i^n.  The adjoint solves
// A^T lambda^n = dG/du^n + B^T lambda^{n+1} backward in time and gives
// dG/dp = -sum_n lambda^n . (dA/dp u^n - dB/dp u^{n-1}) for p = sigma_t,i and
// sigma_s,i of every cell.  Both run in one work-group; the tridiagonal
// solves are the parallel scans of the LOSM solve.
#include "hww_losm_dev.h"

namespace hww {

static constexpr int MARCH_THREADS = 1024;

__global__ void __launch_bounds__(MARCH_THREADS) march_kernel(MarchArgs A) {
  const int I = A.I, n = 2 * I + 3, M = I + 2, N = A.n_steps;
  const int tid = threadIdx.x, T = blockDim.x;
  extern __shared__ double dyn[];
  double *u = dyn;             // [n]
  double *phi_o = u + n;       // [I+2]
  double *J_o = phi_o + M;     // [I+1]
  __shared__ double sp[MARCH_THREADS], sq[MARCH_THREADS];
  __shared__ int ok;
  __shared__ double red[MARCH_THREADS / 64];
  const double th = A.theta, inv_vdt = 1.0 / (A.v * A.dt);
  if (tid == 0) ok = losm_factor_seq(I, A.edges, A.sig_t, A.sig_s, th, inv_vdt, false, A.factor) ? 1 : 0;
  for (int i = tid; i < M; i += T) A.hist[2 * i] = A.phi0[i];
  for (int j = tid; j <= I; j += T) A.hist[2 * j + 1] = A.J0[j];
  __syncthreads();
  if (!ok) {
    if (tid == 0) atomicOr(A.err, ERR_NUMERIC);
    return;
  }
  double gacc = 0.0;
  for (int i = tid; i < M; i += T) gacc += A.w[i] * A.phi0[i];
  for (int s = 1; s <= N; ++s) {
    const double *prev = A.hist + (size_t)(s - 1) * n;
    for (int i = tid; i < M; i += T) phi_o[i] = prev[2 * i];
    for (int j = tid; j <= I; j += T) J_o[j] = prev[2 * j + 1];
    __syncthreads();
    const double *Fo = A.F + (size_t)(s - 1) * M, *Fn = A.F + (size_t)s * M;
    const double PL = A.P[2 * s], PR = A.P[2 * s + 1];
    for (int r = tid; r < n; r += T)
      u[r] = losm_rhs(I, A.edges, A.sig_t, A.sig_s, th, inv_vdt, r, phi_o, J_o, Fo, Fn, PL, PR);
    __syncthreads();
    losm_solve_scans(u, n, A.factor, sp, sq);
    double *cur = A.hist + (size_t)s * n;
    for (int r = tid; r < n; r += T) cur[r] = u[r];
    for (int i = tid; i < M; i += T) gacc += A.w[(size_t)s * M + i] * u[2 * i];
    __syncthreads();
  }
  for (int o = 32; o >= 1; o >>= 1) gacc += __shfl_xor(gacc, o);
  if ((tid & 63) == 0) red[tid >> 6] = gacc;
  __syncthreads();
  if (tid == 0) {
    double g = 0.0;
    for (int q = 0; q < (T >> 6); ++q) g += red[q];
    *A.G = g;
  }
}

__global__ void __launch_bounds__(MARCH_THREADS) adjoint_kernel(MarchArgs A) {
  const int I = A.I, n = 2 * I + 3, M = I + 2, N = A.n_steps;
  const int tid = threadIdx.x, T = blockDim.x;
  extern __shared__ double dyn[];
  double *u = dyn;        // [n] right-hand side, then lambda^s
  double *lam = u + n;    // [n] lambda^{s+1}
  __shared__ double sp[MARCH_THREADS], sq[MARCH_THREADS];
  __shared__ int ok;
  const double th = A.theta, inv_vdt = 1.0 / (A.v * A.dt);
  if (tid == 0) ok = losm_factor_seq(I, A.edges, A.sig_t, A.sig_s, th, inv_vdt, true, A.factor_t) ? 1 : 0;
  for (int r = tid; r < n; r += T) lam[r] = 0.0;
  __syncthreads();
  if (!ok) {
    if (tid == 0) atomicOr(A.err, ERR_NUMERIC);
    return;
  }
  // Each thread owns the cells i = tid + k T (k < 4: I <= 4096).
  double gt[4] = {0.0, 0.0, 0.0, 0.0}, gs[4] = {0.0, 0.0, 0.0, 0.0};
  for (int s = N; s >= 1; --s) {
    for (int r = tid; r < n; r += T) {
      double d = ((r & 1) == 0) ? A.w[(size_t)s * M + r / 2] : 0.0;
      if (s < N) {
        // (B^T lambda)_r collects rows r-1, r, r+1 of B.
        double ba, bb, bc;
        losm_brow(I, A.edges, A.sig_t, A.sig_s, th, inv_vdt, r, &ba, &bb, &bc);
        d += bb * lam[r];
        if (r + 1 < n) {
          losm_brow(I, A.edges, A.sig_t, A.sig_s, th, inv_vdt, r + 1, &ba, &bb, &bc);
          d += ba * lam[r + 1];
        }
        if (r - 1 >= 0) {
          losm_brow(I, A.edges, A.sig_t, A.sig_s, th, inv_vdt, r - 1, &ba, &bb, &bc);
          d += bc * lam[r - 1];
        }
      }
      u[r] = d;
    }
    __syncthreads();
    losm_solve_scans(u, n, A.factor_t, sp, sq);  // u = lambda^s
    const double *us = A.hist + (size_t)s * n, *uo = A.hist + (size_t)(s - 1) * n;
    for (int k = 0; k < 4; ++k) {
      const int i = tid + k * T;  // 0-based cell; balance row 2(i+1)
      if (i >= I) break;
      const int ci = i + 1;
      const double dx = A.edges[ci] - A.edges[ci - 1];
      const double db = th * dx * us[2 * ci] - (th - 1.0) * dx * uo[2 * ci];
      gt[k] -= u[2 * ci] * db;
      gs[k] += u[2 * ci] * db;
      for (int e = ci - 1; e <= ci; ++e) {
        const int r = 2 * e + 1;
        const double dm = th * 0.5 * dx * us[r] - (th - 1.0) * 0.5 * dx * uo[r];
        gt[k] -= u[r] * dm;
      }
    }
    __syncthreads();
    for (int r = tid; r < n; r += T) lam[r] = u[r];
    __syncthreads();
  }
  for (int k = 0; k < 4; ++k) {
    const int i = tid + k * T;
    if (i >= I) break;
    A.g_t[i] = gt[k];
    A.g_s[i] = gs[k];
  }
}

static hipError_t launch_single(const void *fn, void (*k)(MarchArgs), const MarchArgs &a, size_t lds, hipStream_t s,
                                size_t *done) {
  if (lds > 32 * 1024 && lds > *done) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    *done = lds;
  }
  hipLaunchKernelGGL(k, dim3(1), dim3(MARCH_THREADS), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_march(const MarchArgs &a, hipStream_t s) {
  static size_t done = 0;
  const size_t lds = (size_t)(2 * a.I + 3 + (a.I + 2) + (a.I + 1)) * sizeof(double);
  return launch_single(reinterpret_cast<const void *>(&march_kernel), march_kernel, a, lds, s, &done);
}

hipError_t launch_adjoint(const MarchArgs &a, hipStream_t s) {
  static size_t done = 0;
  const size_t lds = (size_t)2 * (2 * a.I + 3) * sizeof(double);
  return launch_single(reinterpret_cast<const void *>(&adjoint_kernel), adjoint_kernel, a, lds, s, &done);
}

}  // namespace hww
