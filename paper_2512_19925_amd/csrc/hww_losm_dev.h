// Device building blocks of the LOSM solves (Sec. 3, Eqs. losm-0, losm-1,
// losm-disc-bc): matrix and old-time coefficients of the interleaved
// tridiagonal system [phi_0, J_0, phi_1, J_1, ..., J_I, phi_{I+1}], its
// Thomas factors, and the substitutions as parallel scans of affine
// recurrences over one work-group.
#pragma once

#include "hww_internal.h"

namespace hww {

// Row r of the matrix: sub-diagonal a, diagonal b, super-diagonal c.
// The half-cell cross section at edge j averages the two cells touching it.
__device__ inline void losm_row(int I, const double *edges, const double *sig_t, const double *sig_s, double th,
                                double inv_vdt, int r, double *a, double *b, double *c) {
  const int n = 2 * I + 3;
  if (r == 0) {  // left boundary relation phi_0/2 + J_0 = 2 J_L + P_L
    *a = 0.0; *b = 0.5; *c = 1.0;
  } else if (r == n - 1) {  // right boundary relation J_I - phi_{I+1}/2 = 2 J_R - P_R
    *a = 1.0; *b = -0.5; *c = 0.0;
  } else if ((r & 1) == 0) {  // balance over cell i = r/2
    const int i = r / 2;
    const double dx = edges[i] - edges[i - 1];
    const double sa = sig_t[i - 1] - sig_s[i - 1];
    *a = -th;
    *b = dx * inv_vdt + th * sa * dx;
    *c = th;
  } else {  // first moment over the half cells around edge j = (r-1)/2
    const int j = (r - 1) / 2;
    const double dxl = (j >= 1) ? edges[j] - edges[j - 1] : 0.0;
    const double dxr = (j <= I - 1) ? edges[j + 1] - edges[j] : 0.0;
    const double stl = (j >= 1) ? sig_t[j - 1] : 0.0;
    const double str = (j <= I - 1) ? sig_t[j] : 0.0;
    const double dxh = 0.5 * (dxr + dxl);
    const double sh = (stl * dxl + str * dxr) / (dxl + dxr);
    *a = -th / 3.0;
    *b = dxh * inv_vdt + th * sh * dxh;
    *c = th / 3.0;
  }
}

// Coefficients of the old-time unknowns in row r of the right-hand side:
// d_r = ba u_{r-1} + bb u_r + bc u_{r+1} + closure terms.
__device__ inline void losm_brow(int I, const double *edges, const double *sig_t, const double *sig_s, double th,
                                 double inv_vdt, int r, double *ba, double *bb, double *bc) {
  const int n = 2 * I + 3;
  if (r == 0 || r == n - 1) {
    *ba = 0.0; *bb = 0.0; *bc = 0.0;
  } else if ((r & 1) == 0) {
    const int i = r / 2;
    const double dx = edges[i] - edges[i - 1];
    const double sa = sig_t[i - 1] - sig_s[i - 1];
    *ba = -(th - 1.0);
    *bb = dx * inv_vdt + (th - 1.0) * sa * dx;
    *bc = (th - 1.0);
  } else {
    const int j = (r - 1) / 2;
    const double dxl = (j >= 1) ? edges[j] - edges[j - 1] : 0.0;
    const double dxr = (j <= I - 1) ? edges[j + 1] - edges[j] : 0.0;
    const double stl = (j >= 1) ? sig_t[j - 1] : 0.0;
    const double str = (j <= I - 1) ? sig_t[j] : 0.0;
    const double dxh = 0.5 * (dxr + dxl);
    const double sh = (stl * dxl + str * dxr) / (dxl + dxr);
    *ba = -(th - 1.0) / 3.0;
    *bb = dxh * inv_vdt + (th - 1.0) * sh * dxh;
    *bc = (th - 1.0) / 3.0;
  }
}

// Right-hand side of row r from the old state (phi_o [I+2], J_o [I+1]), the
// closures at the old and new time (F_o, F_n [I+2]) and P_L, P_R.
__device__ inline double losm_rhs(int I, const double *edges, const double *sig_t, const double *sig_s, double th,
                                  double inv_vdt, int r, const double *phi_o, const double *J_o, const double *F_o,
                                  const double *F_n, double PL, double PR) {
  const int n = 2 * I + 3;
  if (r == 0) return PL;
  if (r == n - 1) return -PR;
  if ((r & 1) == 0) {
    const int i = r / 2;
    const double dx = edges[i] - edges[i - 1];
    const double sa = sig_t[i - 1] - sig_s[i - 1];
    return dx * inv_vdt * phi_o[i] + (th - 1.0) * (J_o[i] - J_o[i - 1] + sa * dx * phi_o[i]);
  }
  const int j = (r - 1) / 2;
  const double dxl = (j >= 1) ? edges[j] - edges[j - 1] : 0.0;
  const double dxr = (j <= I - 1) ? edges[j + 1] - edges[j] : 0.0;
  const double stl = (j >= 1) ? sig_t[j - 1] : 0.0;
  const double str = (j <= I - 1) ? sig_t[j] : 0.0;
  const double dxh = 0.5 * (dxr + dxl);
  const double sh = (stl * dxl + str * dxr) / (dxl + dxr);
  return dxh * inv_vdt * J_o[j] + th * (F_n[j + 1] - F_n[j])
       + (th - 1.0) * ((phi_o[j + 1] - phi_o[j]) / 3.0 + sh * dxh * J_o[j] - (F_o[j + 1] - F_o[j]));
}

// The same right-hand side with the old-time diagonal bb_r of row r (the
// coefficient of u_r in losm_brow) precomputed: no mesh or cross-section
// reads in the solve.
__device__ inline double losm_rhs_bb(int I, double th, int r, double bb, const double *phi_o, const double *J_o,
                                     const double *F_o, const double *F_n, double PL, double PR) {
  const int n = 2 * I + 3;
  if (r == 0) return PL;
  if (r == n - 1) return -PR;
  if ((r & 1) == 0) {
    const int i = r / 2;
    return bb * phi_o[i] + (th - 1.0) * (J_o[i] - J_o[i - 1]);
  }
  const int j = (r - 1) / 2;
  return bb * J_o[j] + th * (F_n[j + 1] - F_n[j])
       + (th - 1.0) * ((phi_o[j + 1] - phi_o[j]) * (1.0 / 3.0) - (F_o[j + 1] - F_o[j]));
}

// Thomas factors of the matrix (or of its transpose) for the forward
// recurrence d'_r = d_r/den_r + alpha_r d'_{r-1} and the backward one
// x_r = d'_r + gamma_r x_{r+1}: factor = [alpha | 1/den | gamma], each n long.
// One lane.  Returns false on a zero or non-finite pivot.
__device__ inline bool losm_factor_seq(int I, const double *edges, const double *sig_t, const double *sig_s,
                                       double th, double inv_vdt, bool transpose, double *factor) {
  const int n = 2 * I + 3;
  double *alpha = factor, *inv = factor + n, *gamma = factor + 2 * n;
  double cp = 0.0;
  double a_next, b_next, c_next;
  losm_row(I, edges, sig_t, sig_s, th, inv_vdt, 0, &a_next, &b_next, &c_next);
  double c_prev = 0.0;
  for (int r = 0; r < n; ++r) {
    const double a = a_next, b = b_next, c = c_next;
    if (r + 1 < n) losm_row(I, edges, sig_t, sig_s, th, inv_vdt, r + 1, &a_next, &b_next, &c_next);
    // transpose: sub-diagonal of row r is c_{r-1}, super-diagonal is a_{r+1}
    const double sub = transpose ? c_prev : a;
    const double sup = transpose ? (r + 1 < n ? a_next : 0.0) : c;
    c_prev = c;
    const double den = (r == 0) ? b : b - sub * cp;
    if (den == 0.0 || !isfinite(den)) return false;
    cp = (r < n - 1) ? sup / den : 0.0;
    alpha[r] = (r == 0) ? 0.0 : -sub / den;
    inv[r] = 1.0 / den;
    gamma[r] = -cp;
  }
  return true;
}

// Cross-lane moves by DPP (no LDS round trip): the value of another lane of
// the wave, chosen by the DPP control kCtrl, in the rows of kRowMask; lanes
// whose source lane lies outside their row, and lanes of other rows, get
// `old`.  Doubles move as two 32-bit halves.
enum : int { kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118,
             kDppWaveShr1 = 0x138, kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143 };

template <int kCtrl, int kRowMask = 0xF>
__device__ __forceinline__ double dpp_f64(double old, double v) {
  const uint64_t o = (uint64_t)__double_as_longlong(old), x = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)x, kCtrl, kRowMask, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(x >> 32), kCtrl,
                                                            kRowMask, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// One step of the affine-map scan: compose the lane's map with the map
// (pp, qq) of the lanes before it (identity (0, 1) where there are none).
template <int kCtrl, int kRowMask = 0xF>
__device__ __forceinline__ void affine_step(double &P, double &Q) {
  const double pp = dpp_f64<kCtrl, kRowMask>(0.0, P), qq = dpp_f64<kCtrl, kRowMask>(1.0, Q);
  P = P + Q * pp;
  Q = Q * qq;
}

// Inclusive scan of affine maps over the 64 lanes of a wave (Hillis-Steele
// within rows of 16, then the row ends broadcast to the rows after them).
__device__ __forceinline__ void affine_scan_wave(double &P, double &Q) {
  affine_step<kDppRowShr1>(P, Q);
  affine_step<kDppRowShr2>(P, Q);
  affine_step<kDppRowShr4>(P, Q);
  affine_step<kDppRowShr8>(P, Q);
  affine_step<kDppRowBcast15, 0xA>(P, Q);
  affine_step<kDppRowBcast31, 0xC>(P, Q);
}

// Largest value over the 64 lanes of a wave (every lane gets it).
__device__ __forceinline__ double wave_max_f64(double m) {
  const double lo = -__builtin_inf();
  double t;
  t = dpp_f64<kDppRowShr1>(lo, m); m = t > m ? t : m;
  t = dpp_f64<kDppRowShr2>(lo, m); m = t > m ? t : m;
  t = dpp_f64<kDppRowShr4>(lo, m); m = t > m ? t : m;
  t = dpp_f64<kDppRowShr8>(lo, m); m = t > m ? t : m;
  t = dpp_f64<kDppRowBcast15, 0xA>(lo, m); m = t > m ? t : m;
  t = dpp_f64<kDppRowBcast31, 0xC>(lo, m); m = t > m ? t : m;
  const uint64_t b = (uint64_t)__double_as_longlong(m);
  const uint32_t lo32 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
  const uint32_t hi32 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
  return __longlong_as_double((long long)(((uint64_t)hi32 << 32) | lo32));
}

// Sum over the 64 lanes of a wave (every lane gets it): an inclusive scan
// by DPP lane moves, then lane 63.
__device__ __forceinline__ double wave_sum_f64(double x) {
  x += dpp_f64<kDppRowShr1>(0.0, x);
  x += dpp_f64<kDppRowShr2>(0.0, x);
  x += dpp_f64<kDppRowShr4>(0.0, x);
  x += dpp_f64<kDppRowShr8>(0.0, x);
  x += dpp_f64<kDppRowBcast15, 0xA>(0.0, x);
  x += dpp_f64<kDppRowBcast31, 0xC>(0.0, x);
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo32 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
  const uint32_t hi32 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
  return __longlong_as_double((long long)(((uint64_t)hi32 << 32) | lo32));
}

// Scan of affine maps y -> p + q y across the work-group in thread order:
// returns, for thread t, the composition of the maps of threads 0..t-1
// applied to y = 0 (0 for thread 0).  Within a wave by DPP lane moves;
// across the (at most 16) waves through LDS with one barrier, after which
// every wave scans the wave totals itself.  sp, sq: >= 16 doubles each.
// Two calls need a barrier between them (the second one rewrites sp, sq).
__device__ inline double affine_scan_excl(double *sp, double *sq, double P, double Q) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = (int)(blockDim.x >> 6);
  affine_scan_wave(P, Q);
  // In-wave exclusive map (identity for lane 0).
  const double pe = dpp_f64<kDppWaveShr1>(0.0, P), qe = dpp_f64<kDppWaveShr1>(1.0, Q);
  if (lane == 63) {
    sp[wv] = P;
    sq[wv] = Q;
  }
  __syncthreads();
  if (wv == 0) return pe + qe * 0.0;
  // Inclusive scan of the wave totals in lanes 0..nw-1 (one row of 16); the
  // maps of waves 0..wv-1 are lane wv-1's.
  double p = lane < nw ? sp[lane] : 0.0, q = lane < nw ? sq[lane] : 1.0;
  affine_step<kDppRowShr1>(p, q);
  affine_step<kDppRowShr2>(p, q);
  affine_step<kDppRowShr4>(p, q);
  affine_step<kDppRowShr8>(p, q);
  const uint64_t b = (uint64_t)__double_as_longlong(p);
  const uint32_t lo32 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, wv - 1);
  const uint32_t hi32 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), wv - 1);
  const double pw = __longlong_as_double((long long)(((uint64_t)hi32 << 32) | lo32));
  return pe + qe * pw;
}

// Solve with the factors, in place: u holds the right-hand side on entry
// and the solution on return (all threads of the work-group call this).
__device__ inline void losm_solve_scans(double *u, int n, const double *factor, double *sp, double *sq) {
  const double *alpha = factor, *inv = factor + n, *gamma = factor + 2 * n;
  const int T = blockDim.x, tid = threadIdx.x;
  const int m = (n + T - 1) / T;
  {
    const int r0 = tid * m, r1 = min(r0 + m, n);
    double P = 0.0, Q = 1.0;
    for (int r = r0; r < r1; ++r) {
      const double al = alpha[r];
      P = u[r] * inv[r] + al * P;
      Q = al * Q;
    }
    double y = affine_scan_excl(sp, sq, P, Q);
    for (int r = r0; r < r1; ++r) {
      y = u[r] * inv[r] + alpha[r] * y;
      u[r] = y;
    }
  }
  __syncthreads();
  {
    const int tb = T - 1 - tid;  // mirrored block: the scan runs from the end
    const int b0 = tb * m, b1 = min(b0 + m, n);
    double P = 0.0, Q = 1.0;
    for (int r = b1 - 1; r >= b0; --r) {
      const double g = (r == n - 1) ? 0.0 : gamma[r];
      P = u[r] + g * P;
      Q = g * Q;
    }
    double y = affine_scan_excl(sp, sq, P, Q);
    for (int r = b1 - 1; r >= b0; --r) {
      const double g = (r == n - 1) ? 0.0 : gamma[r];
      y = u[r] + g * y;
      u[r] = y;
    }
  }
  __syncthreads();
}

// losm_solve_scans with each thread's factor entries loaded into registers
// beforehand (losm_scan_prefetch, at most MR rows per thread): the same
// arithmetic in the same order, without factor loads on the critical path.
// The factor array here is [alpha | 1/den | gamma | bb] (bb: the old-time
// diagonal of losm_rhs_bb).
template <int MR>
struct ScanRows {
  double al[MR], iv[MR], ga[MR], bb[MR];
};

template <int MR>
__device__ inline void losm_scan_prefetch(const double *factor, int n, ScanRows<MR> &R) {
  const int T = blockDim.x, tid = threadIdx.x;
  const int m = (n + T - 1) / T;
  const int r0 = tid * m, b0 = (T - 1 - tid) * m;
#pragma unroll
  for (int k = 0; k < MR; ++k) {
    const int r = r0 + k, rb = b0 + k;
    const bool f = k < m && r < n, b = k < m && rb < n;
    R.al[k] = f ? factor[r] : 0.0;
    R.iv[k] = f ? factor[n + r] : 0.0;
    R.bb[k] = f ? factor[3 * n + r] : 0.0;
    R.ga[k] = (b && rb != n - 1) ? factor[2 * n + rb] : 0.0;
  }
}

template <int MR>
__device__ inline void losm_solve_scans_rows(double *u, int n, const ScanRows<MR> &R, double *sp, double *sq) {
  const int T = blockDim.x, tid = threadIdx.x;
  const int m = (n + T - 1) / T;
  {
    const int r0 = tid * m, cnt = min(m, n - r0);
    double P = 0.0, Q = 1.0;
#pragma unroll
    for (int k = 0; k < MR; ++k)
      if (k < cnt) {
        P = u[r0 + k] * R.iv[k] + R.al[k] * P;
        Q = R.al[k] * Q;
      }
    double y = affine_scan_excl(sp, sq, P, Q);
#pragma unroll
    for (int k = 0; k < MR; ++k)
      if (k < cnt) {
        y = u[r0 + k] * R.iv[k] + R.al[k] * y;
        u[r0 + k] = y;
      }
  }
  __syncthreads();
  {
    const int b0 = (T - 1 - tid) * m, cnt = min(m, n - b0);
    double P = 0.0, Q = 1.0;
#pragma unroll
    for (int k = MR - 1; k >= 0; --k)
      if (k < cnt) {
        P = u[b0 + k] + R.ga[k] * P;
        Q = R.ga[k] * Q;
      }
    double y = affine_scan_excl(sp, sq, P, Q);
#pragma unroll
    for (int k = MR - 1; k >= 0; --k)
      if (k < cnt) {
        y = u[b0 + k] + R.ga[k] * y;
        u[b0 + k] = y;
      }
  }
  __syncthreads();
}

}  // namespace hww
