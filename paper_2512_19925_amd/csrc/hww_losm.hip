// Hybrid low-order second-moment (HLOSM) solve on the device (Shaw &
// Anistratov, arXiv 2512.19925, Sec. 3 Eqs. losm-disc and losm-disc-semi;
// moving-average filter of Sec. 4; window centres of Sec. 2 Eq. ww-center).
//
// One work-group per system.  Phases, separated by barriers:
//   1. sum the per-batch tallies of the initial-condition set (census at
//      t^{n-1}, face tallies of step n-1) and of the closure set
//   2. grid functions: phi^{n-1}, J^{n-1} at edges (linear interpolation of
//      cell-average currents), F^{n-1}, F^n, P_L, P_R
//   3. optional moving-average filter of F^n, F^{n-1}, phi^{n-1}, J^{n-1}
//   4. assemble the interleaved tridiagonal system of 2I+3 unknowns
//      [phi_0, J_0, phi_1, J_1, ..., J_I, phi_{I+1}] and solve it
//   5. window centres s * [(max(phi,0)/max phi)(1-eps) + eps], ceiling and
//      floor (Sec. 2 Eq. ww-c&f)
#include "hww_internal.h"

namespace hww {

static constexpr int LOSM_THREADS = 1024;

__device__ void ma_filter_dev(const double *in, double *out, int M, int k) {
  for (int m = 1 + (int)threadIdx.x; m <= M; m += blockDim.x) {
    int km = k;
    if (m - 1 < km) km = m - 1;
    if (M - m < km) km = M - m;
    double acc = 0.0;
    for (int l = -km; l <= km; ++l) acc += in[m - l - 1];
    out[m - 1] = acc / (double)(2 * km + 1);
  }
}

__global__ void __launch_bounds__(LOSM_THREADS) losm_kernel(LosmArgs A) {
  const int I = A.I;
  const int M = I + 2;
  const int n = 2 * I + 3;
  const int tid = threadIdx.x;
  double *S = A.scratch;
  double *phi_o = S;
  double *J_o = phi_o + M;
  double *F_o = J_o + M;
  double *F_n = F_o + M;
  double *tmp = F_n + M;
  double *gi_phi = tmp + M;
  double *gi_J = gi_phi + I;
  double *gi_K = gi_J + I;
  double *gc_phi = gi_K + I;
  double *gc_K = gc_phi + I;
  double *a = gc_K + I;
  double *bb = a + n;
  double *c = bb + n;
  double *d = c + n;
  double *u = d + n;
  __shared__ double face[12];  // ic: phi L/R, P L/R, F L/R; cl: same
  __shared__ double sc[4];     // scale, s, max
  __shared__ int bad;
  __shared__ int skip;
  __shared__ double red[LOSM_THREADS / 64];

  if (tid == 0) {
    bad = 0;
    skip = 0;
    double wtot = 0.0, done = 0.0, wn = 0.0;
    for (int q = 0; q < A.nc; ++q) {
      wtot += A.wstart[q];
      if (q < A.next_chunk) done += A.wstart[q];
      wn += A.wnext[q];
    }
    if (A.implicit) {
      sc[0] = wtot / done;
      sc[1] = wtot / A.n_src;
      // No start weight swept yet: no closures exist, the update is skipped.
      if (!(done > 0.0)) skip = 1;
    } else {
      sc[0] = 1.0;
      sc[1] = wn / A.n_src;
    }
  }
  __syncthreads();
  if (skip) {
    for (int i = tid; i <= I + 1; i += blockDim.x) A.phi_out[i] = 0.0;
    for (int i = tid; i <= I; i += blockDim.x) A.J_out[i] = 0.0;
    if (tid == 0) *A.status = 0;
    return;
  }
  const double scale = sc[0];

  // 1. batch sums and normalisation per source particle.
  const int kc = A.closure_track ? 0 : 3;
  for (int i = tid; i < I; i += blockDim.x) {
    double p = 0.0, j = 0.0, k = 0.0, cp = 0.0, ck = 0.0;
    for (int b = 0; b < A.B; ++b) {
      const double *t = A.tal_ic + ((size_t)b * I + i) * 6;
      p += t[3];
      j += t[4];
      k += t[5];
      const double *tc = A.tal_cl + ((size_t)b * I + i) * 6;
      cp += tc[kc];
      ck += tc[kc + 2];
    }
    const double dxi = A.edges[i + 1] - A.edges[i];
    const double norm = A.n_src * dxi;
    gi_phi[i] = p / norm;
    gi_J[i] = j / norm;
    gi_K[i] = k / norm;
    const double normc = A.closure_track ? (A.n_src * dxi * A.dt) : norm;
    gc_phi[i] = scale * cp / normc;
    gc_K[i] = scale * ck / normc;
  }
  if (tid < 12) {
    const int set = tid / 6, q = tid % 6;
    const int f = q & 1, kind = q >> 1;  // q: (phi L, phi R, P L, P R, F L, F R)
    const double *bs = set == 0 ? A.bnd_ic : A.bnd_cl;
    double acc = 0.0;
    for (int b = 0; b < A.B; ++b) acc += bs[(b * 2 + f) * 3 + kind];
    face[tid] = (set == 0 ? 1.0 : scale) * acc / (A.n_src * A.dt);
  }
  __syncthreads();

  // 2. grid functions.
  for (int i = tid; i <= I + 1; i += blockDim.x) {
    if (i == 0) {
      phi_o[0] = face[0];
      F_o[0] = face[4];
      J_o[0] = -0.5 * face[0] + face[2];
    } else if (i == I + 1) {
      phi_o[I + 1] = face[1];
      F_o[I + 1] = face[5];
      J_o[I] = 0.5 * face[1] - face[3];
    } else {
      phi_o[i] = gi_phi[i - 1];
      F_o[i] = gi_phi[i - 1] / 3.0 - gi_K[i - 1];
      if (i <= I - 1) {
        const double dl = A.edges[i] - A.edges[i - 1], dr = A.edges[i + 1] - A.edges[i];
        J_o[i] = (dr * gi_J[i - 1] + dl * gi_J[i]) / (dl + dr);
      }
    }
  }
  __syncthreads();
  double PL, PR;
  if (!A.implicit) {
    for (int i = tid; i <= I + 1; i += blockDim.x) F_n[i] = F_o[i];
    PL = face[2];
    PR = face[3];
  } else {
    for (int i = tid; i <= I + 1; i += blockDim.x) {
      if (i == 0) F_n[0] = face[10];
      else if (i == I + 1) F_n[I + 1] = face[11];
      else F_n[i] = gc_phi[i - 1] / 3.0 - gc_K[i - 1];
    }
    PL = face[8];
    PR = face[9];
  }
  __syncthreads();

  // 3. moving-average filter.
  if (A.filter == 1) {
    double *arrs[3] = {F_n + 1, F_o + 1, phi_o + 1};
    for (int q = 0; q < 3; ++q) {
      ma_filter_dev(arrs[q], tmp, I, A.ma_k);
      __syncthreads();
      for (int i = tid; i < I; i += blockDim.x) arrs[q][i] = tmp[i];
      __syncthreads();
    }
    ma_filter_dev(J_o, tmp, I + 1, A.ma_k);
    __syncthreads();
    for (int i = tid; i <= I; i += blockDim.x) J_o[i] = tmp[i];
    __syncthreads();
  }

  // 4. assemble.
  const double th = A.theta;
  const double inv_vdt = 1.0 / (A.v * A.dt);
  for (int r = tid; r < n; r += blockDim.x) {
    if (r == 0) {
      a[0] = 0.0; bb[0] = 0.5; c[0] = 1.0; d[0] = PL;
    } else if (r == n - 1) {
      a[r] = 1.0; bb[r] = -0.5; c[r] = 0.0; d[r] = -PR;
    } else if ((r & 1) == 0) {
      const int i = r / 2;  // balance of cell i (1..I)
      const double dx = A.edges[i] - A.edges[i - 1];
      const double sa = A.sig_t[i - 1] - A.sig_s[i - 1];
      a[r] = -th;
      bb[r] = dx * inv_vdt + th * sa * dx;
      c[r] = th;
      d[r] = dx * inv_vdt * phi_o[i] + th * 0.0 * dx
           + (th - 1.0) * (J_o[i] - J_o[i - 1] + sa * dx * phi_o[i] - 0.0 * dx);
    } else {
      const int i = (r - 1) / 2;  // first moment at edge i (0..I)
      const double dxl = (i >= 1) ? A.edges[i] - A.edges[i - 1] : 0.0;
      const double dxr = (i <= I - 1) ? A.edges[i + 1] - A.edges[i] : 0.0;
      const double stl = (i >= 1) ? A.sig_t[i - 1] : 0.0;
      const double str = (i <= I - 1) ? A.sig_t[i] : 0.0;
      const double dxh = 0.5 * (dxr + dxl);
      const double sh = (stl * dxl + str * dxr) / (dxl + dxr);
      a[r] = -th / 3.0;
      bb[r] = dxh * inv_vdt + th * sh * dxh;
      c[r] = th / 3.0;
      d[r] = dxh * inv_vdt * J_o[i] + th * (F_n[i + 1] - F_n[i])
           + (th - 1.0) * ((phi_o[i + 1] - phi_o[i]) / 3.0 + sh * dxh * J_o[i] - (F_o[i + 1] - F_o[i]));
    }
  }
  __syncthreads();

  // Thomas elimination (no pivoting), one lane.
  if (tid == 0 && !bad) {
    double den = bb[0];
    if (den == 0.0 || !isfinite(den)) bad = 1;
    double cp = c[0] / den;
    double dp = d[0] / den;
    a[0] = cp;  // reuse a[] for c' and d[] for d'
    d[0] = dp;
    for (int i = 1; i < n && !bad; ++i) {
      den = bb[i] - a[i] * cp;
      if (den == 0.0 || !isfinite(den)) { bad = 1; break; }
      cp = (i < n - 1) ? c[i] / den : 0.0;
      dp = (d[i] - a[i] * dp) / den;
      a[i] = cp;
      d[i] = dp;
    }
    if (!bad) {
      double xn = d[n - 1];
      u[n - 1] = xn;
      for (int i = n - 2; i >= 0; --i) {
        xn = d[i] - a[i] * xn;
        u[i] = xn;
      }
    }
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) {
      atomicOr(A.err, ERR_NUMERIC);
      *A.status = (int)ERR_NUMERIC;
    }
    return;
  }
  for (int i = tid; i <= I + 1; i += blockDim.x) A.phi_out[i] = u[2 * i];
  for (int i = tid; i <= I; i += blockDim.x) A.J_out[i] = u[2 * i + 1];

  // 5. window centres (an empty bank has nothing to window: unchanged).
  if (A.apply_windows && sc[1] > 0.0) {
    double mx = -__builtin_inf();
    int nonfinite = 0;
    for (int i = tid; i < I; i += blockDim.x) {
      const double p = u[2 * (i + 1)];
      if (!isfinite(p)) nonfinite = 1;
      if (p > mx) mx = p;
    }
    for (int o = 32; o >= 1; o >>= 1) {
      const double t = __shfl_xor(mx, o);
      mx = t > mx ? t : mx;
    }
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    if (nonfinite) atomicOr(&bad, 1);
    __syncthreads();
    if (tid == 0) {
      double m = red[0];
      for (int q = 1; q < (int)(blockDim.x >> 6); ++q) m = red[q] > m ? red[q] : m;
      sc[2] = m;
      if (!(m > 0.0) || !(sc[1] > 0.0)) bad = 1;
    }
    __syncthreads();
    if (bad) {
      if (tid == 0) {
        atomicOr(A.err, ERR_NUMERIC);
        *A.status = (int)ERR_NUMERIC;
      }
      return;
    }
    const double m = sc[2], s = sc[1];
    for (int i = tid; i < I; i += blockDim.x) {
      const double p = u[2 * (i + 1)];
      const double rr = p > 0.0 ? p / m : 0.0;
      const double ww = s * (rr * (1.0 - A.eps_min) + A.eps_min);
      A.centre[i] = ww;
      A.wceil[i] = ww * A.rho;
      A.wfloor[i] = ww / A.rho;
    }
  }
  if (tid == 0) *A.status = 0;
}

hipError_t launch_losm(const LosmArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(losm_kernel, dim3(1), dim3(LOSM_THREADS), 0, s, a);
  return hipGetLastError();
}

}  // namespace hww
