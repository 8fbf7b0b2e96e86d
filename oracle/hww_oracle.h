/*
 * hww_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, serial, FP64 CPU oracle of the hybrid weight-window (HWW)
 * time-dependent Monte Carlo method (Shaw & Anistratov, arXiv 2512.19925).
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no source with the GPU library; the two meet only through
 * the random-number keying contract, which each side implements on its own
 * from the published Philox4x32-10 definition.
 *
 * The pins of each function are listed at the top of hww_oracle.c.
 */
#ifndef HWW_ORACLE_H
#define HWW_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Tally kinds (per batch, per cell). */
enum { ORC_T_PHI = 0, ORC_T_J = 1, ORC_T_K = 2, ORC_C_PHI = 3, ORC_C_J = 4, ORC_C_K = 5 };
/* Boundary tally kinds (per batch, per face 0 = left, 1 = right). */
enum { ORC_B_PHI = 0, ORC_B_P = 1, ORC_B_F = 2 };
/* Event counters. */
enum {
  ORC_N_SEGMENTS = 0, ORC_N_COLLISIONS, ORC_N_SCATTERS, ORC_N_ABSORPTIONS,
  ORC_N_CROSSINGS, ORC_N_LEAKS, ORC_N_CENSUS, ORC_N_SPLITS, ORC_N_DAUGHTERS,
  ORC_N_RR_KILL, ORC_N_RR_SURVIVE, ORC_N_HISTORIES, ORC_N_FISSIONS, ORC_N_FISSION_BIRTHS,
  ORC_N_COUNTERS = 16
};

typedef struct orc_params {
  int32_t n_cells;
  const double *edges;    /* n_cells + 1, ascending */
  const double *sigma_t;  /* n_cells */
  const double *sigma_s;  /* n_cells */
  double speed, dt;
  int32_t n_steps;
  double src_x;
  int64_t n_src;
  int64_t bank_capacity;
  uint32_t seed, replica;
  int32_t n_batches;
  int32_t n_chunks;
  const double *sigma_f;  /* n_cells, or NULL: no fission */
  double nu_f;            /* mean number of neutrons per fission */
  int32_t track_moments;  /* track-length moments scored per segment: 0 or 3 phi, J, K; 2 phi, K; 1 phi */
} orc_params;

typedef struct orc_losm_opts {
  double theta;
  int32_t implicit;      /* 0: semi-implicit (lagged closures), 1: fully implicit */
  int32_t filter;        /* 0: none, 1: moving average, 2: Fourier low pass */
  int32_t ma_k;
  double eps_min;
  double rho;
  int32_t closure_track; /* 0: census (time-layer) closures, 1: track-length closures */
  int32_t apply_windows;
  int32_t kappa;         /* Fourier cutoff */
  int32_t lagged;        /* 1: windows from the previous step's track-length flux, no solve */
  int32_t window_scale;  /* 0: centres times s^n = start weight / N_src; 1: as printed (max centre 1) */
} orc_losm_opts;

typedef struct orc_sim orc_sim;

/* Philox4x32-10 block function. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* 53-bit uniform in [0,1) from two 32-bit words. */
double orc_u53(uint32_t a, uint32_t b);
/* ln x for a positive normal x by fixed steps (atanh series); the flight
 * distance -ln(1 - u) / sigma_t uses it. */
double orc_log(double x);

int orc_create(const orc_params *p, orc_sim **out);
void orc_destroy(orc_sim *s);
/* Restrict the simulation to the batches whose flag is nonzero (n_batches flags). */
int orc_set_batch_mask(orc_sim *s, const uint8_t *mask);
int orc_set_windows(orc_sim *s, const double *centre, double rho);
int orc_sweep_chunk(orc_sim *s, int32_t step, int32_t chunk);
/* Uniform combing of the census bank of the finished step into n_target
 * particles of equal weight (population control of the supercritical test
 * problem, Sec. 5.1).  n_before and w_total (nullable) return the census
 * size and the total weight that the comb distributes. */
int orc_comb(orc_sim *s, int64_t n_target, int64_t *n_before, double *w_total);
/* Reading of the comb: 0 (default) teeth spaced in cumulative weight, every
 * copy of weight W / n_target; 1 teeth spaced in particle index, every copy
 * keeping its particle's weight times n / n_target. */
int orc_set_comb_mode(orc_sim *s, int32_t mode);
int orc_solve_losm(orc_sim *s, const orc_losm_opts *o, double *phi_out, double *J_out);
/* Initial condition phi_o (I+2), J_o (I+1), F_o (I+2) and closures F_n
 * (I+2), P (2: P_L, P_R) of an HLOSM solve, before any filter:
 * implicit = 0 the semi-implicit solve at the start of the next step
 * (F_n = F_o, the lagged closures), 1 the fully implicit solve inside the
 * step after the chunks swept so far.  Returns 1 when no start weight has
 * been swept yet (no closures), -2 in the wrong state. */
int orc_losm_inputs(const orc_sim *s, int32_t implicit, int32_t closure_track, double *phi_o, double *J_o,
                    double *F_o, double *F_n, double *P);
/* Unfiltered closures F (I+2), P (2) and initial condition phi (I+2), J (I+1)
 * that the finished step hands to the next. */
int orc_get_closures(const orc_sim *s, double *F, double *P, double *phi, double *J);

/* Raw per-batch sums: cur = 1 current step, 0 previous step. */
int orc_get_tallies(const orc_sim *s, int32_t cur, double *cells /* B*I*6 */, double *bnd /* B*2*3 */);
int orc_get_counters(const orc_sim *s, uint64_t *out /* ORC_N_COUNTERS */);
int orc_get_tracks(const orc_sim *s, uint64_t *out /* I */);
int orc_get_windows(const orc_sim *s, double *centre, double *ceil_, double *floor_);
int orc_get_state(const orc_sim *s, int32_t *step, int32_t *next_chunk, double *w_start /* n_chunks */, double *w_next /* n_chunks */);
/* Bank dump: which = 0 start-of-step bank, 1 census bank being filled (at step 0: the source). */
int64_t orc_bank_size(const orc_sim *s, int32_t which);
int orc_get_bank(const orc_sim *s, int32_t which, double *x, double *mu, double *w,
                 uint32_t *src, uint64_t *lin, uint32_t *e, int32_t *cell, int32_t *chunk);

/* Stand-alone pieces (used by the pins). */
int orc_losm_step(int32_t I, const double *edges, const double *sig_t, const double *sig_s,
                  double speed, double dt, double theta,
                  const double *phi_old /* I+2 */, const double *J_old /* I+1 */,
                  const double *F_old /* I+2 */, const double *F_new /* I+2 */,
                  double PL, double PR, double JL, double JR,
                  const double *q_old /* I or NULL */, const double *q_new /* I or NULL */,
                  double *phi_new /* I+2 */, double *J_new /* I+1 */);
int orc_thomas(int32_t n, const double *a, const double *b, const double *c, const double *d, double *x);
/* March of n_steps fully implicit LOSM steps with frozen closures F
 * ((n_steps+1) x (I+2)) and P ((n_steps+1) x 2: P_L, P_R) from phi0, J0;
 * phi_hist (n_steps+1) x (I+2), J_hist (n_steps+1) x (I+1). */
int orc_losm_march(int32_t I, const double *edges, const double *sig_t, const double *sig_s, double v,
                   double dt, double theta, int32_t n_steps, const double *F, const double *P,
                   const double *phi0, const double *J0, double *phi_hist, double *J_hist);
/* Gradient of G = sum w[n][i] phi_hist[n][i] with respect to sigma_t, sigma_s. */
int orc_losm_adjoint(int32_t I, const double *edges, const double *sig_t, const double *sig_s, double v,
                     double dt, double theta, int32_t n_steps, const double *phi_hist, const double *J_hist,
                     const double *w, double *g_t, double *g_s);
void orc_ma_filter(const double *in, int32_t M, int32_t k, double *out);
void orc_fourier_filter(const double *in, int32_t M, int32_t kappa, double *out);
int orc_ww_centres(int32_t I, const double *phi_tilde, double eps_min, double scale, double *ww);

#ifdef __cplusplus
}
#endif
#endif
