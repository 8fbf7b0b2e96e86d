/*
 * hww_oracle.c -- TEST INFRASTRUCTURE ONLY (see hww_oracle.h).
 *
 * A plain, serial, obviously-correct FP64 implementation of one time step of
 * the hybrid weight-window Monte Carlo method of Shaw & Anistratov (arXiv
 * 2512.19925): flight, collision and census of a 1D slab particle bank with
 * isotropic scattering (transport equation, Sec. 3 Eq. HO_transport),
 * and fission (the nu_f Sigma_f term of that equation), track-length and
 * time-crossing tallies (Sec. 3 Eqs. phi-mc, ct-mc), uniform combing of the
 * census (the population control of Sec. 5.1),
 * splitting and Russian roulette against weight windows (Sec. 2, Eqs.
 * ww-c&f, ww-center), and the hybrid low-order second-moment (HLOSM)
 * solve that defines the window centres (Sec. 3 Eqs. losm-disc,
 * losm-disc-semi), with the moving-average filter of Sec. 4.
 *
 * Each history runs to completion before the next, with its split daughters
 * on a last-in-first-out stack.  Tally sums are Neumaier-compensated.
 *
 * Pins (tests/test_oracle_*.py):
 *   orc_philox4x32_10   published Philox4x32-10 known-answer vectors
 *   orc_u53             exact integer construction, range and moments
 *   orc_log             libm's log within one ulp over the flight range
 *                       (0, 1], 0 at 1, log identities at powers of two
 *   orc_thomas          dense LAPACK solve on random well-posed systems
 *   orc_losm_step       manufactured smooth solution: 2nd-order convergence
 *                       for theta = 1/2, 1st order for theta = 1; discrete
 *                       balance identity
 *   orc_ma_filter       brute-force sums, constants and linear functions kept
 *   orc_fourier_filter  numpy's real FFT low pass, identity for kappa >= M/2,
 *                       the mean for kappa = 0, single cosine modes kept or
 *                       removed exactly
 *   orc_ww_centres      max cell = scale exactly, floor eps*scale, shape
 *   orc_losm_inputs     closed-form uncollided (c = 0) time-layer cell
 *                       averages, edge currents (exact where J is linear),
 *                       face values and P_L, P_R on an unequal leaking mesh,
 *                       for the semi-implicit inputs and the scaled partial
 *                       closures of the implicit updates; orc_solve_losm is
 *                       the pinned LOSM step of the (filtered) inputs
 *   orc_losm_march      source-free manufactured solution with time-dependent
 *                       closures: 2nd order (CN), 1st order (BE)
 *   (tests/test_oracle_mutations.py plants ten plausible mistakes in these
 *   two and checks that each fails a pin)
 *   sweep (uncollided)  closed-form c = 0 pulse solution for all six tallies
 *   sweep (streaming)   exact geometric track lengths, single particles
 *   sweep (scattering)  exact weight/track conservation at c = 1 (analog),
 *                       closed-form moment solutions for 0 < c < 1
 *   sweep (one short    track length and census weight per cell against
 *    step)              the expectations over histories with at most one
 *                       collision (first order in the collisions)
 *   split / roulette    exact daughter count and weight sum, unbiased
 *                       roulette, HWW vs analog tallies agree statistically
 *   fission             nu_f = 1 fission identical to scattering (tallies,
 *                       counters, solves), exact multiplicity for integer
 *                       nu_f, closed-form pulse moments and the reference
 *                       pulse solution at c_eff = 1.1, low-order balance
 *                       with the nu_f sigma_f production term
 *   orc_comb            systematic-sampling property (floor/ceil copies of
 *                       every run, canonical order kept), equal weights
 *                       summing to the census weight, identities and
 *                       chunks, uniform offset over seeds; with teeth in
 *                       particle index: systematic sampling over the
 *                       particles, each copy's weight its particle's times
 *                       n / n_target, the census weight kept on average
 * Parity unpinned: the variance/FOM benefit of a particular window schedule
 * (the paper shows it only in figures).
 */
#include "hww_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  Ten rounds of two 32x32->64 multiplies with    */
/* the published multipliers and Weyl key increments.                       */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint64_t p0 = (uint64_t)M0 * c0;
    uint64_t p1 = (uint64_t)M1 * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53-bit uniform on [0,1): 27 high bits of a, 26 high bits of b. */
double orc_u53(uint32_t a, uint32_t b) {
  double k = (double)(a >> 5) * 67108864.0 + (double)(b >> 6);
  return k * (1.0 / 9007199254740992.0);
}

/* Natural logarithm of a positive normal x, as the flight distance uses it.
 * x = (1 + f) 2^k with 1 + f in [sqrt(1/2), sqrt(2)) (f exact).  With
 * s = f / (2 + f), ln(1 + f) = 2 atanh(s) = 2s + s R, R the rest of the
 * atanh series, and 2s = f - s f = f - h + s h (h = f^2 / 2), so
 * ln(1 + f) = f - (h - s (h + R)): the rounding of s only touches the small
 * s (h + R) term.  R = sum_{j=1..9} 2 z^j / (2j + 1), z = s^2 <= 0.0295 (the
 * first term left out is below 2^-54 relatively).  k ln 2 is added with
 * ln 2 split in two doubles.  Within one ulp of ln x.  The steps are fixed
 * (every product and sum named, fused multiply-adds where written), so any
 * implementation of the same steps in IEEE double gives the same bits;
 * libm's log differs from it in the last bit now and then. */
double orc_log(double x) {
  int k;
  double m = frexp(x, &k);
  if (m < 0.70710678118654752440) {
    m = m * 2.0;
    k = k - 1;
  }
  const double f = m - 1.0;
  const double s = f / (2.0 + f);
  const double z = s * s;
  double q = 2.0 / 19.0;
  q = fma(q, z, 2.0 / 17.0);
  q = fma(q, z, 2.0 / 15.0);
  q = fma(q, z, 2.0 / 13.0);
  q = fma(q, z, 2.0 / 11.0);
  q = fma(q, z, 2.0 / 9.0);
  q = fma(q, z, 2.0 / 7.0);
  q = fma(q, z, 2.0 / 5.0);
  q = fma(q, z, 2.0 / 3.0);
  const double R = z * q;
  const double h = 0.5 * f * f;
  const double kd = (double)k;
  const double c = fma(kd, 2.3190468138462996e-17, s * (h + R));
  const double u = f - (h - c);
  return fma(kd, 0.69314718055994528623, u);
}

/* Random-number slots of the keying contract. */
enum { SLOT_FLIGHT = 0, SLOT_EVENT = 1, SLOT_START = 2, SLOT_BIRTH = 3,
       SLOT_LIN_EVENT = 4, SLOT_LIN_START = 5, SLOT_FISSION_DIR = 6, SLOT_COMB = 7 };

static void draw(uint32_t seed, uint32_t replica, int slot, uint32_t src, uint64_t lin,
                 uint32_t e, double *ua, double *ub, uint32_t raw[4]) {
  uint32_t ctr[4] = {src, (uint32_t)lin, (uint32_t)(lin >> 32), e};
  uint32_t key[2] = {seed, (replica << 4) | (uint32_t)slot};
  uint32_t r[4];
  orc_philox4x32_10(ctr, key, r);
  if (ua) *ua = orc_u53(r[0], r[1]);
  if (ub) *ub = orc_u53(r[2], r[3]);
  if (raw) memcpy(raw, r, sizeof r);
}

/* ------------------------------------------------------------------------ */
/* Compensated accumulator                                                   */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;
static void nadd(nsum *a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
  else a->c += (v - t) + a->s;
  a->s = t;
}
static double nval(const nsum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* Simulation state                                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
  double x, mu, w, tau;
  int32_t cell;
  uint32_t src;
  uint64_t lin;
  uint32_t e;
  int32_t chunk; /* chunk of the step that starts from this particle */
} particle;

typedef struct {
  nsum *cells;   /* [B][I][6] */
  nsum *bnd;     /* [B][2][3] */
} tally_set;

struct orc_sim {
  int32_t I;
  double *edges, *sig_t, *sig_s, *cratio, *inv_sig_t;
  double *cfis;      /* (sigma_s + sigma_f) / sigma_t: collision is scatter below cratio, fission below cfis */
  double *sig_s_lo;  /* sigma_s + nu_f sigma_f: the production term of the low-order balance */
  double nu_f;
  int fission;
  int track_moments;  /* 3: phi, J, K; 2: phi, K; 1: phi */
  double v, inv_v, dt;
  int32_t n_steps;
  double src_x;
  int64_t n_src, cap;
  uint32_t seed, replica;
  int32_t B, n_chunks;
  uint8_t *batch_on;

  int ww_on;
  double *centre, *ceil_, *floor_;

  particle *start; int64_t n_start;
  particle *census; int64_t n_census;
  particle *stack; int64_t n_stack, cap_stack;

  tally_set cur, prev;
  uint64_t *tracks;                  /* [I] for the current step */
  uint64_t counters[ORC_N_COUNTERS]; /* current step */
  nsum *w_chunk_start;               /* [n_chunks] weight of the start bank per chunk */
  nsum *w_chunk_next;                /* [n_chunks] same, for the next step (filled at census) */
  int32_t step, next_chunk;
  int comb_mode;  /* 0: teeth spaced in cumulative weight, 1: spaced in particle index */
};

static int tally_alloc(tally_set *t, int B, int I) {
  t->cells = (nsum *)calloc((size_t)B * I * 6, sizeof(nsum));
  t->bnd = (nsum *)calloc((size_t)B * 2 * 3, sizeof(nsum));
  return (t->cells && t->bnd) ? 0 : -1;
}
static void tally_zero(tally_set *t, int B, int I) {
  memset(t->cells, 0, (size_t)B * I * 6 * sizeof(nsum));
  memset(t->bnd, 0, (size_t)B * 2 * 3 * sizeof(nsum));
}

/* Cell containing x; a point on an interior edge belongs to the cell the
 * particle moves into (mu >= 0: right, mu < 0: left). */
static int32_t find_cell(const orc_sim *s, double x, double mu) {
  int32_t lo = 0, hi = s->I; /* edges[lo] <= x < edges[hi] */
  if (x <= s->edges[0]) return 0;
  if (x >= s->edges[s->I]) return s->I - 1;
  while (hi - lo > 1) {
    int32_t mid = (lo + hi) / 2;
    if (s->edges[mid] <= x) lo = mid; else hi = mid;
  }
  if (x == s->edges[lo] && mu < 0.0 && lo > 0) lo -= 1;
  return lo;
}

/* Chunk (window-update interval) of the next step from a uniform variate. */
static int32_t chunk_from(const orc_sim *s, double u) {
  int32_t c = (int32_t)(u * (double)s->n_chunks);
  if (c >= s->n_chunks) c = s->n_chunks - 1;
  return c;
}

static int batch_of(const orc_sim *s, uint32_t src) { return (int)(src % (uint32_t)s->B); }

void orc_destroy(orc_sim *s) {
  if (!s) return;
  free(s->edges); free(s->sig_t); free(s->sig_s); free(s->cratio); free(s->inv_sig_t); free(s->batch_on);
  free(s->cfis); free(s->sig_s_lo);
  free(s->centre); free(s->ceil_); free(s->floor_);
  free(s->start); free(s->census); free(s->stack);
  free(s->cur.cells); free(s->cur.bnd); free(s->prev.cells); free(s->prev.bnd);
  free(s->tracks); free(s->w_chunk_start); free(s->w_chunk_next);
  free(s);
}

/* Add a census (time-crossing) contribution of a particle at t^n: the
 * cell-average flux at the time layer counts v*w per particle (Eq. ct-mc). */
static void census_tally(orc_sim *s, tally_set *t, const particle *p) {
  int b = batch_of(s, p->src);
  nsum *c = t->cells + ((size_t)b * s->I + p->cell) * 6;
  double vw = s->v * p->w;
  double t1 = vw * p->mu;
  nadd(&c[ORC_C_PHI], vw);
  nadd(&c[ORC_C_J], t1);
  nadd(&c[ORC_C_K], t1 * p->mu);
}

int orc_create(const orc_params *p, orc_sim **out) {
  if (!p || !out) return -1;
  *out = NULL;
  if (p->n_cells < 1 || !p->edges || !p->sigma_t || !p->sigma_s) return -1;
  if (!(p->speed > 0.0) || !(p->dt > 0.0) || p->n_steps < 1 || p->n_src < 0) return -1;
  if (p->n_batches < 1 || p->n_chunks < 1 || p->n_chunks > 16 || p->bank_capacity < p->n_src) return -1;
  if (p->n_src > 0xFFFFFFFFll) return -1;
  int I = p->n_cells;
  for (int i = 0; i < I; ++i) {
    if (!(p->edges[i + 1] > p->edges[i])) return -1;
    if (!(p->sigma_t[i] > 0.0) || !(p->sigma_s[i] >= 0.0) || p->sigma_s[i] > p->sigma_t[i]) return -1;
    if (p->sigma_f && (!(p->sigma_f[i] >= 0.0) || p->sigma_s[i] + p->sigma_f[i] > p->sigma_t[i])) return -1;
  }
  if (p->sigma_f && (!(p->nu_f >= 0.0) || !(p->nu_f < 1.0e6))) return -1;
  if (p->track_moments < 0 || p->track_moments > 3) return -1;
  if (!(p->src_x >= p->edges[0] && p->src_x <= p->edges[I])) return -1;

  orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
  if (!s) return -1;
  s->I = I; s->v = p->speed; s->dt = p->dt; s->n_steps = p->n_steps; s->src_x = p->src_x;
  s->n_src = p->n_src; s->cap = p->bank_capacity; s->seed = p->seed; s->replica = p->replica;
  s->B = p->n_batches; s->n_chunks = p->n_chunks;
  s->edges = (double *)malloc(sizeof(double) * (I + 1));
  s->sig_t = (double *)malloc(sizeof(double) * I);
  s->sig_s = (double *)malloc(sizeof(double) * I);
  s->cratio = (double *)malloc(sizeof(double) * I);
  s->inv_sig_t = (double *)malloc(sizeof(double) * I);
  s->cfis = (double *)malloc(sizeof(double) * I);
  s->sig_s_lo = (double *)malloc(sizeof(double) * I);
  s->centre = (double *)malloc(sizeof(double) * I);
  s->ceil_ = (double *)malloc(sizeof(double) * I);
  s->floor_ = (double *)malloc(sizeof(double) * I);
  s->batch_on = (uint8_t *)malloc(s->B);
  s->tracks = (uint64_t *)calloc(I, sizeof(uint64_t));
  s->w_chunk_start = (nsum *)calloc(s->n_chunks, sizeof(nsum));
  s->w_chunk_next = (nsum *)calloc(s->n_chunks, sizeof(nsum));
  s->start = (particle *)malloc(sizeof(particle) * (size_t)(s->cap > 0 ? s->cap : 1));
  s->census = (particle *)malloc(sizeof(particle) * (size_t)(s->cap > 0 ? s->cap : 1));
  s->cap_stack = 1024;
  s->stack = (particle *)malloc(sizeof(particle) * (size_t)s->cap_stack);
  if (!s->edges || !s->sig_t || !s->sig_s || !s->cratio || !s->inv_sig_t || !s->cfis || !s->sig_s_lo ||
      !s->centre || !s->ceil_ ||
      !s->floor_ || !s->batch_on || !s->tracks || !s->w_chunk_start || !s->w_chunk_next ||
      !s->start || !s->census || !s->stack ||
      tally_alloc(&s->cur, s->B, I) || tally_alloc(&s->prev, s->B, I)) {
    orc_destroy(s);
    return -1;
  }
  memcpy(s->edges, p->edges, sizeof(double) * (I + 1));
  memcpy(s->sig_t, p->sigma_t, sizeof(double) * I);
  memcpy(s->sig_s, p->sigma_s, sizeof(double) * I);
  s->fission = p->sigma_f != NULL;
  s->track_moments = p->track_moments == 0 ? 3 : p->track_moments;
  s->nu_f = s->fission ? p->nu_f : 0.0;
  for (int i = 0; i < I; ++i) {
    s->cratio[i] = s->sig_s[i] / s->sig_t[i];
    s->inv_sig_t[i] = 1.0 / s->sig_t[i];
    const double sf = s->fission ? p->sigma_f[i] : 0.0;
    s->cfis[i] = (s->sig_s[i] + sf) / s->sig_t[i];
    s->sig_s_lo[i] = s->sig_s[i] + s->nu_f * sf;
  }
  s->inv_v = 1.0 / s->v;
  memset(s->batch_on, 1, s->B);
  s->ww_on = 0;

  /* Source bank at t^0: isotropic unit-weight pulse at src_x (Sec. 5.1).
   * It is the census at t^0: it supplies the step-1 initial condition, and
   * its weight per chunk the scale of step 1. */
  s->n_census = 0;
  for (int64_t k = 0; k < s->n_src; ++k) {
    particle q;
    double ua, ub;
    draw(s->seed, s->replica, SLOT_BIRTH, (uint32_t)k, 0, 0, &ua, &ub, NULL);
    q.mu = 2.0 * ua - 1.0;
    q.x = s->src_x;
    q.w = 1.0;
    q.tau = s->dt;
    q.src = (uint32_t)k;
    q.lin = 0;
    q.e = 0;
    q.cell = find_cell(s, q.x, q.mu);
    q.chunk = chunk_from(s, ub);
    s->census[s->n_census++] = q;
  }
  for (int64_t k = 0; k < s->n_census; ++k) {
    census_tally(s, &s->cur, &s->census[k]);
    nadd(&s->w_chunk_next[s->census[k].chunk], s->census[k].w);
  }
  s->n_start = 0;
  s->step = 0;
  s->next_chunk = s->n_chunks; /* step 0 is complete */
  *out = s;
  return 0;
}

int orc_set_batch_mask(orc_sim *s, const uint8_t *mask) {
  if (!s || !mask) return -1;
  if (s->step != 0) return -2;
  memcpy(s->batch_on, mask, s->B);
  /* Recompute the t^0 census and chunk weights for the selected batches. */
  tally_zero(&s->cur, s->B, s->I);
  memset(s->w_chunk_next, 0, sizeof(nsum) * s->n_chunks);
  int64_t n = 0;
  for (int64_t k = 0; k < s->n_census; ++k) {
    if (!s->batch_on[batch_of(s, s->census[k].src)]) continue;
    s->census[n++] = s->census[k];
  }
  s->n_census = n;
  for (int64_t k = 0; k < n; ++k) {
    census_tally(s, &s->cur, &s->census[k]);
    nadd(&s->w_chunk_next[s->census[k].chunk], s->census[k].w);
  }
  return 0;
}

int orc_set_windows(orc_sim *s, const double *centre, double rho) {
  if (!s) return -1;
  if (!centre) { s->ww_on = 0; return 0; }
  if (!(rho >= 1.0) || !isfinite(rho)) return -1;
  for (int i = 0; i < s->I; ++i)
    if (!(centre[i] > 0.0) || !isfinite(centre[i])) return -5;
  for (int i = 0; i < s->I; ++i) {
    s->centre[i] = centre[i];
    s->ceil_[i] = centre[i] * rho;   /* Eq. ww-ceiling */
    s->floor_[i] = centre[i] / rho;  /* Eq. ww-floor */
  }
  s->ww_on = 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Sweep                                                                     */
/* ------------------------------------------------------------------------ */
static int push(orc_sim *s, const particle *q) {
  if (s->n_stack == s->cap_stack) {
    int64_t nc = s->cap_stack * 2;
    particle *ns = (particle *)realloc(s->stack, sizeof(particle) * (size_t)nc);
    if (!ns) return -1;
    s->stack = ns; s->cap_stack = nc;
  }
  s->stack[s->n_stack++] = *q;
  return 0;
}

/* Weight-window check of a particle in its current cell (Sec. 2).
 * kind 0: after an event (lineage slot 4, daughters take e_daughter);
 * kind 1: at the start of the step (lineage slot 5).
 * xi is the roulette variate.  Returns 0 alive, 1 killed, <0 error. */
static int ww_check(orc_sim *s, particle *p, double xi, int kind, uint32_t e_draw, uint32_t e_daughter) {
  if (!s->ww_on) return 0;
  int i = p->cell;
  double ww = s->centre[i];
  if (p->w > s->ceil_[i]) {
    double nd_f = ceil(p->w / ww);
    if (!(nd_f >= 2.0) || nd_f > 1e9) return -3;
    int64_t nd = (int64_t)nd_f;
    uint32_t raw[4];
    draw(s->seed, s->replica, kind == 0 ? SLOT_LIN_EVENT : SLOT_LIN_START, p->src, p->lin, e_draw,
         NULL, NULL, raw);
    uint64_t base = (uint64_t)raw[0] | ((uint64_t)raw[1] << 32);
    p->w = p->w / (double)nd;
    s->counters[ORC_N_SPLITS] += 1;
    s->counters[ORC_N_DAUGHTERS] += (uint64_t)(nd - 1);
    /* Daughters j = 1..nd-1 are pushed in reverse so that they pop in order. */
    for (int64_t j = nd - 1; j >= 1; --j) {
      particle d = *p;
      d.lin = base + (uint64_t)j;
      d.e = e_daughter;
      if (push(s, &d)) return -3;
    }
    return 0;
  }
  if (p->w < s->floor_[i]) {
    if (xi < p->w / ww) {
      p->w = ww;
      s->counters[ORC_N_RR_SURVIVE] += 1;
      return 0;
    }
    s->counters[ORC_N_RR_KILL] += 1;
    return 1;
  }
  return 0;
}

/* Follow one particle until census, leakage, absorption or roulette death. */
static int transport(orc_sim *s, particle *p) {
  const int I = s->I;
  const int b = batch_of(s, p->src);
  nsum *cells = s->cur.cells + (size_t)b * I * 6;
  nsum *bnd = s->cur.bnd + (size_t)b * 2 * 3;
  for (;;) {
    int i = p->cell;
    double ua, ub;
    draw(s->seed, s->replica, SLOT_FLIGHT, p->src, p->lin, p->e, &ua, &ub, NULL);
    /* Exponential flight distance with mean free path 1/sigma_t. */
    double d_coll = -orc_log(1.0 - ua) * s->inv_sig_t[i];
    double xl = s->edges[i], xr = s->edges[i + 1];
    double d_bnd;
    if (p->mu > 0.0) d_bnd = (xr - p->x) / p->mu;
    else if (p->mu < 0.0) d_bnd = (xl - p->x) / p->mu;
    else d_bnd = INFINITY;
    double d_cen = s->v * p->tau;
    int ev; /* 0 census, 1 boundary, 2 collision: ties go to the lower number */
    double l;
    if (d_cen <= d_bnd && d_cen <= d_coll) { ev = 0; l = d_cen; }
    else if (d_bnd <= d_coll) { ev = 1; l = d_bnd; }
    else { ev = 2; l = d_coll; }

    /* Track-length tally (Eq. phi-mc) and its first and second angular moments. */
    double wl = p->w * l;
    double t1 = wl * p->mu;
    nadd(&cells[i * 6 + ORC_T_PHI], wl);
    if (s->track_moments == 3) nadd(&cells[i * 6 + ORC_T_J], t1);
    if (s->track_moments >= 2) nadd(&cells[i * 6 + ORC_T_K], t1 * p->mu);
    s->tracks[i] += 1;
    s->counters[ORC_N_SEGMENTS] += 1;
    uint32_t e = p->e;
    p->e = e + 1;

    if (ev == 0) {
      double xn = p->x + p->mu * l;
      if (xn < xl) xn = xl;
      if (xn > xr) xn = xr;
      p->x = xn;
      p->tau = s->dt;
      /* The flight draw's second variate is not used at census: it picks
       * the chunk of the next step. */
      p->chunk = chunk_from(s, ub);
      census_tally(s, &s->cur, p);
      s->counters[ORC_N_CENSUS] += 1;
      if (s->n_census >= s->cap) return -3;
      s->census[s->n_census++] = *p;
      nadd(&s->w_chunk_next[p->chunk], p->w);
      return 0;
    }
    p->tau = p->tau - l * s->inv_v;
    if (ev == 1) {
      int leave_left = (i == 0 && p->mu < 0.0);
      int leave_right = (i == I - 1 && p->mu > 0.0);
      if (leave_left || leave_right) {
        /* Edge-crossing estimators at the domain faces: w f(mu)/|mu|. */
        double am = fabs(p->mu);
        nsum *f = bnd + (leave_left ? 0 : 3);
        nadd(&f[ORC_B_PHI], p->w / am);
        nadd(&f[ORC_B_P], p->w * (0.5 - am) / am);
        nadd(&f[ORC_B_F], p->w * (1.0 / 3.0 - p->mu * p->mu) / am);
        s->counters[ORC_N_LEAKS] += 1;
        return 0;
      }
      if (p->mu > 0.0) { p->x = xr; p->cell = i + 1; }
      else { p->x = xl; p->cell = i - 1; }
      s->counters[ORC_N_CROSSINGS] += 1;
      double xi;
      draw(s->seed, s->replica, SLOT_EVENT, p->src, p->lin, e, NULL, &xi, NULL);
      int r = ww_check(s, p, xi, 0, e, p->e);
      if (r < 0) return r;
      if (r == 1) return 0;
      continue;
    }
    /* Collision: analog scattering or absorption. */
    double xn = p->x + p->mu * l;
    if (xn < xl) xn = xl;
    if (xn > xr) xn = xr;
    p->x = xn;
    s->counters[ORC_N_COLLISIONS] += 1;
    if (ub < s->cratio[i]) {
      double ua1, xi;
      draw(s->seed, s->replica, SLOT_EVENT, p->src, p->lin, e, &ua1, &xi, NULL);
      p->mu = 2.0 * ua1 - 1.0;
      s->counters[ORC_N_SCATTERS] += 1;
      int r = ww_check(s, p, xi, 0, e, p->e);
      if (r < 0) return r;
      if (r == 1) return 0;
      continue;
    }
    if (s->fission && ub < s->cfis[i]) {
      /* Fission (Eq. HO_transport, nu_f Sigma_f term): floor(nu_f + xi)
       * neutrons of the parent's weight, isotropic.  The first continues
       * the parent's history with the direction of slot 1; the others are
       * daughters with lineage base + j (base from slot 4) and directions
       * from slot 6 at their own lineage. */
      double ua1, xi;
      draw(s->seed, s->replica, SLOT_EVENT, p->src, p->lin, e, &ua1, &xi, NULL);
      const int64_t nf = (int64_t)floor(s->nu_f + xi);
      s->counters[ORC_N_FISSIONS] += 1;
      s->counters[ORC_N_FISSION_BIRTHS] += (uint64_t)nf;
      if (nf == 0) return 0;
      p->mu = 2.0 * ua1 - 1.0;
      if (nf >= 2) {
        uint32_t raw[4];
        draw(s->seed, s->replica, SLOT_LIN_EVENT, p->src, p->lin, e, NULL, NULL, raw);
        const uint64_t base = (uint64_t)raw[0] | ((uint64_t)raw[1] << 32);
        for (int64_t j = nf - 1; j >= 1; --j) {
          particle d = *p;
          d.lin = base + (uint64_t)j;
          d.e = p->e;
          double ud;
          draw(s->seed, s->replica, SLOT_FISSION_DIR, d.src, d.lin, d.e, &ud, NULL, NULL);
          d.mu = 2.0 * ud - 1.0;
          if (push(s, &d)) return -3;
        }
      }
      continue;
    }
    s->counters[ORC_N_ABSORPTIONS] += 1;
    return 0;
  }
}

static void begin_step(orc_sim *s) {
  /* The census of the finished step becomes the start bank of the next. */
  particle *t = s->start;
  s->start = s->census;
  s->census = t;
  s->n_start = s->n_census;
  s->n_census = 0;
  tally_set tt = s->prev;
  s->prev = s->cur;
  s->cur = tt;
  tally_zero(&s->cur, s->B, s->I);
  memset(s->tracks, 0, sizeof(uint64_t) * s->I);
  memset(s->counters, 0, sizeof s->counters);
  for (int c = 0; c < s->n_chunks; ++c) {
    s->w_chunk_start[c] = s->w_chunk_next[c];
    s->w_chunk_next[c].s = 0.0;
    s->w_chunk_next[c].c = 0.0;
  }
}

int orc_sweep_chunk(orc_sim *s, int32_t step, int32_t chunk) {
  if (!s) return -1;
  if (chunk < 0 || chunk >= s->n_chunks) return -1;
  if (chunk == 0) {
    if (s->next_chunk != s->n_chunks || step != s->step + 1 || step > s->n_steps) return -2;
    begin_step(s);
    s->step = step;
    s->next_chunk = 0;
  } else if (step != s->step || chunk != s->next_chunk) {
    return -2;
  }
  for (int64_t k = 0; k < s->n_start; ++k) {
    particle p = s->start[k];
    if (p.chunk != chunk) continue;
    if (!s->batch_on[batch_of(s, p.src)]) continue;
    s->counters[ORC_N_HISTORIES] += 1;
    s->n_stack = 0;
    /* Start-of-step window check with the current windows. */
    double xi;
    draw(s->seed, s->replica, SLOT_START, p.src, p.lin, p.e, NULL, &xi, NULL);
    int r = ww_check(s, &p, xi, 1, p.e, p.e);
    if (r < 0) return r;
    if (r == 0) {
      r = transport(s, &p);
      if (r < 0) return r;
    }
    while (s->n_stack > 0) {
      particle d = s->stack[--s->n_stack];
      r = transport(s, &d);
      if (r < 0) return r;
    }
  }
  s->next_chunk = chunk + 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Uniform combing                                                           */
/* ------------------------------------------------------------------------ */

/* Canonical order of a bank: source history, then lineage, then event index
 * (particles of equal keys share their whole random stream from there on). */
static int canon_cmp(const void *a, const void *b) {
  const particle *p = (const particle *)a, *q = (const particle *)b;
  if (p->src != q->src) return p->src < q->src ? -1 : 1;
  if (p->lin != q->lin) return p->lin < q->lin ? -1 : 1;
  if (p->e != q->e) return p->e < q->e ? -1 : 1;
  return 0;
}

/* Uniform comb (population control of Sec. 5.1): lay the census particles
 * end to end in canonical order, each an interval as long as its weight, and
 * put n_target teeth at (k + xi) W / n_target, k = 0 .. n_target-1, with one
 * uniform xi per comb (slot 7, counter (step, 0, 0, 0)).  Every tooth makes
 * a copy of the particle whose interval it hits, of weight W / n_target.
 * The weights are laid out as integers in units of 2^eu, eu chosen so that
 * n max(w) < 2^(53 + eu): every prefix sum is then exact both as an integer
 * and as a double, and so is each comparison with a tooth.  Copy k becomes
 * history k of lineage `step` (event index 0) in batch k mod B and chunk
 * (k / B) mod n_chunks. */
int orc_set_comb_mode(orc_sim *s, int32_t mode) {
  if (!s || mode < 0 || mode > 1) return -1;
  s->comb_mode = mode;
  return 0;
}

/* Comb with the teeth spaced in particle index (the other reading of Sec.
 * 5.1's uniform combing, Sec. 5's remark that it thins the particles of
 * weight near 1 at the source): tooth k = 0..n_target-1 takes the particle at
 * canonical position floor((k + xi) n / n_target), with its weight times
 * n / n_target, so every census particle is kept with the same expected
 * number of copies and its expected weight is unchanged.  The weight is
 * taken in the comb's integer unit 2^eu (q: inclusive prefix sums of the
 * integer weights), and the chunk weights from exact integer sums, so that
 * a change of a weight far below the unit changes nothing after the comb. */
static int comb_by_index(orc_sim *s, int64_t n_target, const uint64_t *q, int eu, double *w_total) {
  const int64_t n = s->n_census;
  double xi;
  draw(s->seed, s->replica, SLOT_COMB, (uint32_t)s->step, 0, 0, &xi, NULL, NULL);
  const double delta = (double)n / (double)n_target;
  uint64_t chunk_sum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  particle *dst = s->start;
  for (int64_t k = 0; k < n_target; ++k) {
    int64_t j = (int64_t)(((double)k + xi) * delta);
    if (j >= n) j = n - 1;
    const uint64_t wi = q[j] - (j > 0 ? q[j - 1] : 0);
    particle c = s->census[j];
    c.w = ldexp((double)wi, eu) * delta;
    c.src = (uint32_t)k;
    c.lin = (uint64_t)s->step;
    c.e = 0;
    c.chunk = (int32_t)((k / s->B) % s->n_chunks);
    chunk_sum[c.chunk] += wi;
    dst[k] = c;
  }
  for (int c = 0; c < s->n_chunks; ++c) {
    s->w_chunk_next[c].s = ldexp((double)chunk_sum[c], eu) * delta;
    s->w_chunk_next[c].c = 0.0;
  }
  s->start = s->census;
  s->census = dst;
  s->n_census = n_target;
  if (w_total) *w_total = ldexp((double)q[n - 1], eu);
  return 0;
}

int orc_comb(orc_sim *s, int64_t n_target, int64_t *n_before, double *w_total) {
  if (!s || n_target < 1 || n_target > s->cap || n_target > 0xFFFFFFFFll) return -1;
  if (s->next_chunk != s->n_chunks || s->step < 1) return -2;
  for (int b = 0; b < s->B; ++b)
    if (!s->batch_on[b]) return -2;
  const int64_t n = s->n_census;
  if (n_before) *n_before = n;
  if (w_total) *w_total = 0.0;
  if (n == 0) return 0;
  qsort(s->census, (size_t)n, sizeof(particle), canon_cmp);
  double m = 0.0;
  for (int64_t j = 0; j < n; ++j)
    if (s->census[j].w > m) m = s->census[j].w;
  if (!(m > 0.0) || !isfinite(m)) return -5;
  int em;
  frexp(m, &em); /* m < 2^em */
  int ln = 0;
  while (((int64_t)1 << ln) < n) ++ln;
  const int eu = em + ln - 53;
  uint64_t *q = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
  if (!q) return -3;
  uint64_t acc = 0;
  for (int64_t j = 0; j < n; ++j) {
    acc += (uint64_t)rint(ldexp(s->census[j].w, -eu));
    q[j] = acc; /* inclusive prefix sum */
  }
  const double W = (double)acc;
  if (s->comb_mode == 1) {
    const int rc = comb_by_index(s, n_target, q, eu, w_total);
    free(q);
    return rc;
  }
  double xi;
  draw(s->seed, s->replica, SLOT_COMB, (uint32_t)s->step, 0, 0, &xi, NULL, NULL);
  const double delta = W / (double)n_target;
  const double w_out = ldexp(W, eu) / (double)n_target;
  int64_t *per_chunk = (int64_t *)calloc((size_t)s->n_chunks, sizeof(int64_t));
  if (!per_chunk) { free(q); return -3; }
  particle *dst = s->start;
  for (int64_t k = 0; k < n_target; ++k) {
    double t = ((double)k + xi) * delta;
    if (t >= W) t = W - 1.0;
    /* First particle whose interval ends beyond the tooth. */
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if ((double)q[mid] > t) hi = mid; else lo = mid + 1;
    }
    particle c = s->census[lo];
    c.w = w_out;
    c.src = (uint32_t)k;
    c.lin = (uint64_t)s->step;
    c.e = 0;
    c.chunk = (int32_t)((k / s->B) % s->n_chunks);
    per_chunk[c.chunk] += 1;
    dst[k] = c;
  }
  s->start = s->census;
  s->census = dst;
  s->n_census = n_target;
  for (int c = 0; c < s->n_chunks; ++c) {
    s->w_chunk_next[c].s = (double)per_chunk[c] * w_out;
    s->w_chunk_next[c].c = 0.0;
  }
  if (w_total) *w_total = ldexp(W, eu);
  free(per_chunk);
  free(q);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Deterministic pieces                                                      */
/* ------------------------------------------------------------------------ */

/* Thomas algorithm (no pivoting): a = sub-diagonal (a[0] unused),
 * b = diagonal, c = super-diagonal (c[n-1] unused). */
int orc_thomas(int32_t n, const double *a, const double *b, const double *c, const double *d, double *x) {
  if (n < 1) return -1;
  double *cp = (double *)malloc(sizeof(double) * n);
  double *dp = (double *)malloc(sizeof(double) * n);
  if (!cp || !dp) { free(cp); free(dp); return -1; }
  int rc = 0;
  double den = b[0];
  if (den == 0.0 || !isfinite(den)) rc = -5;
  cp[0] = (n > 1) ? c[0] / den : 0.0;
  dp[0] = d[0] / den;
  for (int i = 1; i < n && rc == 0; ++i) {
    den = b[i] - a[i] * cp[i - 1];
    if (den == 0.0 || !isfinite(den)) { rc = -5; break; }
    cp[i] = (i < n - 1) ? c[i] / den : 0.0;
    dp[i] = (d[i] - a[i] * dp[i - 1]) / den;
  }
  if (rc == 0) {
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
  }
  free(cp); free(dp);
  return rc;
}

/* Moving-average filter (Sec. 4, Eq. moving_average) on chi_1..chi_M with the
 * base shrunk symmetrically near the ends: k_m = min(k, m-1, M-m). */
void orc_ma_filter(const double *in, int32_t M, int32_t k, double *out) {
  for (int m = 1; m <= M; ++m) {
    int km = k;
    if (m - 1 < km) km = m - 1;
    if (M - m < km) km = M - m;
    double acc = 0.0;
    for (int l = -km; l <= km; ++l) acc += in[m - l - 1];
    out[m - 1] = acc / (double)(2 * km + 1);
  }
}

/* Fourier filter (Sec. 4, Eqs. fft and ifft) on chi_1..chi_M: the discrete
 * Fourier transform X_j = sum_m chi_m exp(-i 2 pi j m / M), the modes with
 * frequency |j| <= kappa kept (j and M - j: the real low pass), the others
 * zeroed, and the inverse transform (1/M) sum_j X_j exp(i 2 pi j m / M).
 * Written as the definition, O(M^2). */
void orc_fourier_filter(const double *in, int32_t M, int32_t kappa, double *out) {
  const double two_pi = 6.283185307179586476925286766559;
  double *xr = (double *)calloc((size_t)M, sizeof(double));
  double *xi = (double *)calloc((size_t)M, sizeof(double));
  if (!xr || !xi) { free(xr); free(xi); return; }
  for (int j = 0; j < M; ++j) {
    int f = j <= M - j ? j : M - j;            /* |frequency| of mode j */
    if (f > kappa) continue;
    double re = 0.0, im = 0.0;
    for (int m = 1; m <= M; ++m) {
      double a = two_pi * (double)(((int64_t)j * m) % M) / (double)M;
      re += in[m - 1] * cos(a);
      im -= in[m - 1] * sin(a);
    }
    xr[j] = re; xi[j] = im;
  }
  for (int m = 1; m <= M; ++m) {
    double acc = 0.0;
    for (int j = 0; j < M; ++j) {
      int f = j <= M - j ? j : M - j;
      if (f > kappa) continue;
      double a = two_pi * (double)(((int64_t)j * m) % M) / (double)M;
      acc += xr[j] * cos(a) - xi[j] * sin(a);  /* Re(X_j e^{i a}) */
    }
    out[m - 1] = acc / (double)M;
  }
  free(xr); free(xi);
}

/* Window centres (Sec. 2, Eq. ww-center) from the auxiliary flux, with
 * negative values clamped to zero, times the weight scale of the step. */
int orc_ww_centres(int32_t I, const double *phi, double eps_min, double scale, double *ww) {
  double mx = -INFINITY;
  for (int i = 0; i < I; ++i) {
    if (!isfinite(phi[i])) return -5;
    if (phi[i] > mx) mx = phi[i];
  }
  if (!(mx > 0.0) || !(scale > 0.0)) return -5;
  for (int i = 0; i < I; ++i) {
    double r = phi[i] > 0.0 ? phi[i] / mx : 0.0;
    ww[i] = scale * (r * (1.0 - eps_min) + eps_min);
  }
  return 0;
}

/* One step of the theta-scheme second-order finite-volume LOSM equations
 * (Sec. 3, Eqs. losm-0, losm-1, losm-disc-bc).  Unknowns ordered
 * [phi_0, J_0, phi_1, J_1, ..., phi_I, J_I, phi_{I+1}]:
 *   row 0        : phi_0/2 + J_0                     = 2 J_L + P_L
 *   row 2i       : balance over cell i = [x_{i-1}, x_i], i = 1..I
 *   row 2i+1     : first moment over the two half cells at edge x_i, i = 0..I
 *   row 2I+2     : J_I - phi_{I+1}/2                 = 2 J_R - P_R
 * Readings: the half-cell cross section at edge i averages the two cells that
 * touch x_i (cells i and i+1); the old-time phi difference in the first
 * moment equation is (phi_{i+1} - phi_i), consistent with the continuous
 * theta scheme; the source enters the balance row times the cell width. */
int orc_losm_step(int32_t I, const double *edges, const double *sig_t, const double *sig_s,
                  double v, double dt, double th,
                  const double *phi_o, const double *J_o, const double *F_o, const double *F_n,
                  double PL, double PR, double JL, double JR,
                  const double *q_o, const double *q_n, double *phi_n, double *J_n) {
  int n = 2 * I + 3;
  double *a = (double *)calloc(n, sizeof(double));
  double *b = (double *)calloc(n, sizeof(double));
  double *c = (double *)calloc(n, sizeof(double));
  double *d = (double *)calloc(n, sizeof(double));
  double *u = (double *)calloc(n, sizeof(double));
  double *dx = (double *)calloc(I + 2, sizeof(double)); /* dx[0] = dx[I+1] = 0 */
  double *st = (double *)calloc(I + 2, sizeof(double));
  if (!a || !b || !c || !d || !u || !dx || !st) {
    free(a); free(b); free(c); free(d); free(u); free(dx); free(st);
    return -1;
  }
  for (int i = 1; i <= I; ++i) { dx[i] = edges[i] - edges[i - 1]; st[i] = sig_t[i - 1]; }
  const double inv_vdt = 1.0 / (v * dt);

  b[0] = 0.5; c[0] = 1.0; d[0] = 2.0 * JL + PL;
  for (int i = 1; i <= I; ++i) {
    int r = 2 * i;
    double sa = sig_t[i - 1] - sig_s[i - 1];
    double qn = q_n ? q_n[i - 1] : 0.0;
    double qo = q_o ? q_o[i - 1] : 0.0;
    a[r] = -th;
    b[r] = dx[i] * inv_vdt + th * sa * dx[i];
    c[r] = th;
    d[r] = dx[i] * inv_vdt * phi_o[i] + th * qn * dx[i]
         + (th - 1.0) * (J_o[i] - J_o[i - 1] + sa * dx[i] * phi_o[i] - qo * dx[i]);
  }
  for (int i = 0; i <= I; ++i) {
    int r = 2 * i + 1;
    double dxh = 0.5 * (dx[i + 1] + dx[i]);
    double sh = (st[i] * dx[i] + st[i + 1] * dx[i + 1]) / (dx[i] + dx[i + 1]);
    a[r] = -th / 3.0;
    b[r] = dxh * inv_vdt + th * sh * dxh;
    c[r] = th / 3.0;
    d[r] = dxh * inv_vdt * J_o[i] + th * (F_n[i + 1] - F_n[i])
         + (th - 1.0) * ((phi_o[i + 1] - phi_o[i]) / 3.0 + sh * dxh * J_o[i] - (F_o[i + 1] - F_o[i]));
  }
  a[n - 1] = 1.0; b[n - 1] = -0.5; d[n - 1] = 2.0 * JR - PR;
  int rc = orc_thomas(n, a, b, c, d, u);
  if (rc == 0) {
    for (int i = 0; i <= I + 1; ++i) phi_n[i] = u[2 * i];
    for (int i = 0; i <= I; ++i) J_n[i] = u[2 * i + 1];
  }
  free(a); free(b); free(c); free(d); free(u); free(dx); free(st);
  return rc;
}

/* Grid functions of one tally set, summed over batches and normalised per
 * source particle: cell values phi, J, K (census or track), face values. */
typedef struct {
  double *phi, *J, *K;    /* [I] */
  double fphi[2], fP[2], fF[2];
} grid_fns;

static void grid_from(const orc_sim *s, const tally_set *t, int track, double scale, grid_fns *g) {
  const int I = s->I;
  const double N = (double)s->n_src;
  int k0 = track ? ORC_T_PHI : ORC_C_PHI;
  for (int i = 0; i < I; ++i) {
    nsum a = {0, 0}, bj = {0, 0}, bk = {0, 0};
    for (int b = 0; b < s->B; ++b) {
      const nsum *c = t->cells + ((size_t)b * I + i) * 6;
      nadd(&a, nval(&c[k0])); nadd(&bj, nval(&c[k0 + 1])); nadd(&bk, nval(&c[k0 + 2]));
    }
    double dxi = s->edges[i + 1] - s->edges[i];
    double norm = track ? (N * dxi * s->dt) : (N * dxi);
    g->phi[i] = scale * nval(&a) / norm;
    g->J[i] = scale * nval(&bj) / norm;
    g->K[i] = scale * nval(&bk) / norm;
  }
  for (int f = 0; f < 2; ++f) {
    nsum a = {0, 0}, p = {0, 0}, q = {0, 0};
    for (int b = 0; b < s->B; ++b) {
      const nsum *c = t->bnd + ((size_t)b * 2 + f) * 3;
      nadd(&a, nval(&c[ORC_B_PHI])); nadd(&p, nval(&c[ORC_B_P])); nadd(&q, nval(&c[ORC_B_F]));
    }
    g->fphi[f] = scale * nval(&a) / (N * s->dt);
    g->fP[f] = scale * nval(&p) / (N * s->dt);
    g->fF[f] = scale * nval(&q) / (N * s->dt);
  }
}

/* Start weight of the bank that a solve's windows act on: at the start of
 * a step (semi-implicit) the census of the finished step, inside a step
 * (fully implicit) the start bank of the step. */
static double bank_weight(const orc_sim *s, int implicit) {
  nsum wtot = {0, 0};
  for (int c = 0; c < s->n_chunks; ++c)
    nadd(&wtot, nval(implicit ? &s->w_chunk_start[c] : &s->w_chunk_next[c]));
  return nval(&wtot);
}

/* Initial condition and closures of an HLOSM solve (Sec. 3), before any
 * filter, from the tallies.
 *  - Initial condition at the old time level: cell averages phi_i of the
 *    time-layer tally (Eq. ct-mc), face values phi_0, phi_{I+1} from the
 *    edge-crossing tallies (reading: step averages at the faces stand for
 *    the point values); interior edge currents by linear interpolation of
 *    the two neighbouring cell averages, weighted by the opposite cell's
 *    width; J_0 and J_I from the vacuum boundary relations of Eq.
 *    losm-disc-bc, J_0 = -phi_0/2 + P_L and J_I = phi_{I+1}/2 - P_R.
 *  - Closures F = phi/3 - K (Eq. F) in every cell, face values of F and
 *    P_L, P_R from the edge-crossing tallies (Eq. F_i-n, losm-disc-bc).
 * implicit = 0 (start of the next step, Eq. losm-disc-semi): everything
 * from the finished step; the new-time closures are the lagged ones, so
 * F_n = F_o.  implicit = 1 (inside a step, Eq. losm-disc): the initial
 * condition from the previous step's time layer, the new-time closures
 * from the chunks swept so far (time-layer or, with closure_track, track-
 * length moments), scaled by W_start / W_done, the start weight of the
 * step over the start weight swept.
 * Returns 0; 1 when no start weight has been swept yet (no closures exist,
 * outputs untouched); -2 in the wrong state. */
int orc_losm_inputs(const orc_sim *s, int32_t implicit, int32_t closure_track, double *phi_o, double *J_o,
                    double *F_o, double *F_n, double *P) {
  if (!s || !phi_o || !J_o || !F_o || !F_n || !P) return -1;
  const int I = s->I;
  const tally_set *ic, *cl;
  double scale = 1.0;
  if (!implicit) {
    if (s->next_chunk != s->n_chunks) return -2;
    ic = &s->cur; cl = &s->cur;
  } else {
    if (s->step < 1 || s->next_chunk < 1 || s->next_chunk >= s->n_chunks) return -2;
    ic = &s->prev; cl = &s->cur;
    nsum done = {0, 0};
    for (int c = 0; c < s->next_chunk; ++c) nadd(&done, nval(&s->w_chunk_start[c]));
    if (!(nval(&done) > 0.0)) return 1;
    scale = bank_weight(s, 1) / nval(&done);
  }
  double *buf = (double *)calloc((size_t)6 * I, sizeof(double));
  if (!buf) return -1;
  grid_fns gi = {buf, buf + I, buf + 2 * I, {0}, {0}, {0}};
  grid_fns gc = {buf + 3 * I, buf + 4 * I, buf + 5 * I, {0}, {0}, {0}};

  grid_from(s, ic, 0, 1.0, &gi);
  phi_o[0] = gi.fphi[0];
  phi_o[I + 1] = gi.fphi[1];
  for (int i = 1; i <= I; ++i) phi_o[i] = gi.phi[i - 1];
  for (int i = 1; i <= I - 1; ++i) {
    double dl = s->edges[i] - s->edges[i - 1], dr = s->edges[i + 1] - s->edges[i];
    J_o[i] = (dr * gi.J[i - 1] + dl * gi.J[i]) / (dl + dr);
  }
  J_o[0] = -0.5 * phi_o[0] + gi.fP[0];
  J_o[I] = 0.5 * phi_o[I + 1] - gi.fP[1];
  F_o[0] = gi.fF[0];
  F_o[I + 1] = gi.fF[1];
  for (int i = 1; i <= I; ++i) F_o[i] = gi.phi[i - 1] / 3.0 - gi.K[i - 1];

  if (!implicit) {
    memcpy(F_n, F_o, sizeof(double) * (I + 2));
    P[0] = gi.fP[0]; P[1] = gi.fP[1];
  } else {
    grid_from(s, cl, closure_track, scale, &gc);
    F_n[0] = gc.fF[0];
    F_n[I + 1] = gc.fF[1];
    for (int i = 1; i <= I; ++i) F_n[i] = gc.phi[i - 1] / 3.0 - gc.K[i - 1];
    P[0] = gc.fP[0]; P[1] = gc.fP[1];
  }
  free(buf);
  return 0;
}

int orc_solve_losm(orc_sim *s, const orc_losm_opts *o, double *phi_out, double *J_out) {
  if (!s || !o) return -1;
  if (!(o->theta > 0.0 && o->theta <= 1.0) || o->ma_k < 0 || o->kappa < 0) return -1;
  if (o->apply_windows && (!(o->rho >= 1.0) || !(o->eps_min > 0.0 && o->eps_min <= 1.0))) return -1;
  if (o->closure_track && !o->lagged && s->track_moments < 2) return -1; /* track closures need K */
  if (o->lagged && (o->implicit || !o->apply_windows)) return -1;
  const int I = s->I;
  if (!o->implicit && s->step >= s->n_steps) return -2;
  /* The windows scale with the weight of the bank they act on. */
  const double sc = bank_weight(s, o->implicit) / (double)s->n_src;

  if (o->lagged) {
    /* Lagged weight windows (Sec. 5): the window shape is the Monte Carlo
     * track-length flux of the finished step; no LOSM solve.  A step without
     * track flux (the source) leaves the windows as they are. */
    if (s->next_chunk != s->n_chunks) return -2;
    double *buf = (double *)calloc((size_t)4 * I, sizeof(double));
    if (!buf) return -1;
    grid_fns g = {buf, buf + I, buf + 2 * I, {0}, {0}, {0}};
    grid_from(s, &s->cur, 1, 1.0, &g);
    if (phi_out) {
      phi_out[0] = phi_out[I + 1] = 0.0;
      memcpy(phi_out + 1, g.phi, sizeof(double) * I);
    }
    if (J_out) memset(J_out, 0, sizeof(double) * (I + 1));
    double mx = 0.0;
    for (int i = 0; i < I; ++i) mx = g.phi[i] > mx ? g.phi[i] : mx;
    int rc = 0;
    if (mx > 0.0 && sc > 0.0) {
      rc = orc_ww_centres(I, g.phi, o->eps_min, o->window_scale ? 1.0 : sc, buf + 3 * I);
      if (rc == 0) rc = orc_set_windows(s, buf + 3 * I, o->rho);
    }
    free(buf);
    return rc;
  }

  double *buf = (double *)calloc((size_t)8 * (I + 2), sizeof(double));
  if (!buf) return -1;
  double *phi_o = buf, *J_o = buf + (I + 2), *F_o = buf + 2 * (I + 2);
  double *F_n = buf + 3 * (I + 2), *phi_n = buf + 4 * (I + 2), *J_n = buf + 5 * (I + 2);
  double *tmp = buf + 6 * (I + 2), *tmp2 = buf + 7 * (I + 2);
  double P[2];
  int rc = orc_losm_inputs(s, o->implicit, o->closure_track, phi_o, J_o, F_o, F_n, P);
  if (rc == 1) {
    /* No start weight swept yet: no closures exist, the update is skipped. */
    if (phi_out) memset(phi_out, 0, sizeof(double) * (I + 2));
    if (J_out) memset(J_out, 0, sizeof(double) * (I + 1));
    free(buf);
    return 0;
  }
  if (rc != 0) { free(buf); return rc; }
  /* The filter of Sec. 4 acts on the cell values of F at both time levels
   * and on the initial condition (phi in the cells, J at every edge). */
  if (o->filter == 1) {
    orc_ma_filter(F_n + 1, I, o->ma_k, tmp); memcpy(F_n + 1, tmp, sizeof(double) * I);
    orc_ma_filter(F_o + 1, I, o->ma_k, tmp); memcpy(F_o + 1, tmp, sizeof(double) * I);
    orc_ma_filter(phi_o + 1, I, o->ma_k, tmp); memcpy(phi_o + 1, tmp, sizeof(double) * I);
    orc_ma_filter(J_o, I + 1, o->ma_k, tmp2); memcpy(J_o, tmp2, sizeof(double) * (I + 1));
  } else if (o->filter == 2) {
    orc_fourier_filter(F_n + 1, I, o->kappa, tmp); memcpy(F_n + 1, tmp, sizeof(double) * I);
    orc_fourier_filter(F_o + 1, I, o->kappa, tmp); memcpy(F_o + 1, tmp, sizeof(double) * I);
    orc_fourier_filter(phi_o + 1, I, o->kappa, tmp); memcpy(phi_o + 1, tmp, sizeof(double) * I);
    orc_fourier_filter(J_o, I + 1, o->kappa, tmp2); memcpy(J_o, tmp2, sizeof(double) * (I + 1));
  } else if (o->filter != 0) {
    free(buf);
    return -1;
  }
  rc = orc_losm_step(I, s->edges, s->sig_t, s->sig_s_lo, s->v, s->dt, o->theta,
                     phi_o, J_o, F_o, F_n, P[0], P[1], 0.0, 0.0, NULL, NULL, phi_n, J_n);
  if (rc == 0) {
    if (phi_out) memcpy(phi_out, phi_n, sizeof(double) * (I + 2));
    if (J_out) memcpy(J_out, J_n, sizeof(double) * (I + 1));
    /* An empty bank has nothing to window: the windows stay as they are. */
    if (o->apply_windows && sc > 0.0) {
      /* Eq. ww-center as printed has its largest centre at 1; window_scale 0
       * multiplies it by the bank's mean weight per source particle. */
      rc = orc_ww_centres(I, phi_n + 1, o->eps_min, o->window_scale ? 1.0 : sc, tmp);
      if (rc == 0) rc = orc_set_windows(s, tmp, o->rho);
    }
  }
  free(buf);
  return rc;
}

/* Closures and initial condition that the finished step hands to the next
 * (Sec. 3): the unfiltered inputs of the next step's semi-implicit solve. */
int orc_get_closures(const orc_sim *s, double *F, double *P, double *phi, double *J) {
  if (!s || !F || !P || !phi || !J) return -1;
  double *Fn = (double *)calloc((size_t)s->I + 2, sizeof(double));
  if (!Fn) return -1;
  int rc = orc_losm_inputs(s, 0, 0, phi, J, F, Fn, P);
  free(Fn);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Accessors                                                                 */
/* ------------------------------------------------------------------------ */
int orc_get_tallies(const orc_sim *s, int32_t cur, double *cells, double *bnd) {
  if (!s) return -1;
  const tally_set *t = cur ? &s->cur : &s->prev;
  size_t nc = (size_t)s->B * s->I * 6;
  if (cells) for (size_t k = 0; k < nc; ++k) cells[k] = nval(&t->cells[k]);
  if (bnd) for (size_t k = 0; k < (size_t)s->B * 6; ++k) bnd[k] = nval(&t->bnd[k]);
  return 0;
}

int orc_get_counters(const orc_sim *s, uint64_t *out) {
  if (!s || !out) return -1;
  memcpy(out, s->counters, sizeof s->counters);
  return 0;
}

int orc_get_tracks(const orc_sim *s, uint64_t *out) {
  if (!s || !out) return -1;
  memcpy(out, s->tracks, sizeof(uint64_t) * s->I);
  return 0;
}

int orc_get_windows(const orc_sim *s, double *centre, double *ceil_, double *floor_) {
  if (!s) return -1;
  if (!s->ww_on) return 1;
  if (centre) memcpy(centre, s->centre, sizeof(double) * s->I);
  if (ceil_) memcpy(ceil_, s->ceil_, sizeof(double) * s->I);
  if (floor_) memcpy(floor_, s->floor_, sizeof(double) * s->I);
  return 0;
}

int orc_get_state(const orc_sim *s, int32_t *step, int32_t *next_chunk, double *w_start, double *w_next) {
  if (!s) return -1;
  if (step) *step = s->step;
  if (next_chunk) *next_chunk = s->next_chunk;
  for (int c = 0; c < s->n_chunks; ++c) {
    if (w_start) w_start[c] = nval(&s->w_chunk_start[c]);
    if (w_next) w_next[c] = nval(&s->w_chunk_next[c]);
  }
  return 0;
}

int64_t orc_bank_size(const orc_sim *s, int32_t which) {
  if (!s) return -1;
  return which == 0 ? s->n_start : s->n_census;
}

int orc_get_bank(const orc_sim *s, int32_t which, double *x, double *mu, double *w,
                 uint32_t *src, uint64_t *lin, uint32_t *e, int32_t *cell, int32_t *chunk) {
  if (!s) return -1;
  const particle *bk = which == 0 ? s->start : s->census;
  int64_t n = which == 0 ? s->n_start : s->n_census;
  for (int64_t k = 0; k < n; ++k) {
    if (x) x[k] = bk[k].x;
    if (mu) mu[k] = bk[k].mu;
    if (w) w[k] = bk[k].w;
    if (src) src[k] = bk[k].src;
    if (lin) lin[k] = bk[k].lin;
    if (e) e[k] = bk[k].e;
    if (cell) cell[k] = bk[k].cell;
    if (chunk) chunk[k] = bk[k].chunk;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Deterministic LOSM march with frozen closures and its adjoint             */
/* ------------------------------------------------------------------------ */

/* Matrix coefficients of one LOSM step (rows as in orc_losm_step) for given
 * cross sections: sub-diagonal a, diagonal b, super-diagonal c.  Also the
 * coefficients of the old-time unknowns in the right-hand side: row r of
 * the right-hand side is ba[r] u_{r-1} + bb[r] u_r + bc[r] u_{r+1} plus the
 * closure terms. */
static void losm_coeffs(int I, const double *edges, const double *sig_t, const double *sig_s, double v,
                        double dt, double th, double *a, double *b, double *c, double *ba, double *bb,
                        double *bc) {
  const int n = 2 * I + 3;
  const double inv_vdt = 1.0 / (v * dt);
  for (int r = 0; r < n; ++r) { a[r] = b[r] = c[r] = ba[r] = bb[r] = bc[r] = 0.0; }
  b[0] = 0.5; c[0] = 1.0;
  a[n - 1] = 1.0; b[n - 1] = -0.5;
  for (int i = 1; i <= I; ++i) {
    const int r = 2 * i;
    const double dx = edges[i] - edges[i - 1];
    const double sa = sig_t[i - 1] - sig_s[i - 1];
    a[r] = -th; b[r] = dx * inv_vdt + th * sa * dx; c[r] = th;
    /* dx/(v dt) phi_i + (th-1)(J_i - J_{i-1} + sa dx phi_i) */
    ba[r] = -(th - 1.0); bb[r] = dx * inv_vdt + (th - 1.0) * sa * dx; bc[r] = (th - 1.0);
  }
  for (int j = 0; j <= I; ++j) {
    const int r = 2 * j + 1;
    const double dxl = j >= 1 ? edges[j] - edges[j - 1] : 0.0;
    const double dxr = j <= I - 1 ? edges[j + 1] - edges[j] : 0.0;
    const double stl = j >= 1 ? sig_t[j - 1] : 0.0;
    const double str = j <= I - 1 ? sig_t[j] : 0.0;
    const double dxh = 0.5 * (dxr + dxl);
    const double sh = (stl * dxl + str * dxr) / (dxl + dxr);
    a[r] = -th / 3.0; b[r] = dxh * inv_vdt + th * sh * dxh; c[r] = th / 3.0;
    /* dxh/(v dt) J_j + (th-1)((phi_{j+1} - phi_j)/3 + sh dxh J_j) */
    ba[r] = -(th - 1.0) / 3.0; bb[r] = dxh * inv_vdt + (th - 1.0) * sh * dxh; bc[r] = (th - 1.0) / 3.0;
  }
}

int orc_losm_march(int32_t I, const double *edges, const double *sig_t, const double *sig_s, double v,
                   double dt, double th, int32_t n_steps, const double *F, const double *P,
                   const double *phi0, const double *J0, double *phi_hist, double *J_hist) {
  const int M = I + 2;
  memcpy(phi_hist, phi0, sizeof(double) * M);
  memcpy(J_hist, J0, sizeof(double) * (I + 1));
  for (int n = 1; n <= n_steps; ++n) {
    int rc = orc_losm_step(I, edges, sig_t, sig_s, v, dt, th, phi_hist + (size_t)(n - 1) * M,
                           J_hist + (size_t)(n - 1) * (I + 1), F + (size_t)(n - 1) * M, F + (size_t)n * M,
                           P[2 * n], P[2 * n + 1], 0.0, 0.0, NULL, NULL, phi_hist + (size_t)n * M,
                           J_hist + (size_t)n * (I + 1));
    if (rc) return rc;
  }
  return 0;
}

/* Gradient of G = sum_n sum_i w[n][i] phi_i^n with respect to sigma_t and
 * sigma_s of every cell, for the march above (adjoint method):
 *   A lambda^n = ... is replaced by A^T lambda^n = dG/du^n + B^T lambda^{n+1},
 *   dG/dp = - sum_n lambda^n . (dA/dp u^n - dB/dp u^{n-1}).
 * A depends on sigma through the balance diagonal (theta Sigma_a dx) and the
 * first-moment diagonal (theta Sigma_hat dx_hat, where Sigma_hat dx_hat =
 * (sigma_t,left dx_left + sigma_t,right dx_right)/2); B through the same
 * terms times (theta - 1). */
int orc_losm_adjoint(int32_t I, const double *edges, const double *sig_t, const double *sig_s, double v,
                     double dt, double th, int32_t n_steps, const double *phi_hist, const double *J_hist,
                     const double *w, double *g_t, double *g_s) {
  const int n = 2 * I + 3, M = I + 2;
  double *a = calloc(n, sizeof(double)), *b = calloc(n, sizeof(double)), *c = calloc(n, sizeof(double));
  double *ba = calloc(n, sizeof(double)), *bb = calloc(n, sizeof(double)), *bc = calloc(n, sizeof(double));
  double *at = calloc(n, sizeof(double)), *ct = calloc(n, sizeof(double));
  double *rhs = calloc(n, sizeof(double)), *lam = calloc(n, sizeof(double)), *lam_next = calloc(n, sizeof(double));
  double *u = calloc(n, sizeof(double)), *uo = calloc(n, sizeof(double));
  int rc = 0;
  if (!a || !b || !c || !ba || !bb || !bc || !at || !ct || !rhs || !lam || !lam_next || !u || !uo) { rc = -1; goto done; }
  losm_coeffs(I, edges, sig_t, sig_s, v, dt, th, a, b, c, ba, bb, bc);
  /* A^T: sub-diagonal of row r is c[r-1], super-diagonal is a[r+1]. */
  for (int r = 0; r < n; ++r) {
    at[r] = r > 0 ? c[r - 1] : 0.0;
    ct[r] = r < n - 1 ? a[r + 1] : 0.0;
  }
  for (int i = 0; i < I; ++i) { g_t[i] = 0.0; g_s[i] = 0.0; }
  for (int r = 0; r < n; ++r) lam_next[r] = 0.0;
  for (int s = n_steps; s >= 1; --s) {
    /* dG/du^s: weights on the phi entries. */
    for (int r = 0; r < n; ++r) rhs[r] = 0.0;
    for (int i = 0; i < M; ++i) rhs[2 * i] = w[(size_t)s * M + i];
    /* + B^T lambda^{s+1}: column q of B collects rows q-1, q, q+1. */
    if (s < n_steps) {
      for (int q = 0; q < n; ++q) {
        double acc = bb[q] * lam_next[q];
        if (q + 1 < n) acc += ba[q + 1] * lam_next[q + 1];
        if (q - 1 >= 0) acc += bc[q - 1] * lam_next[q - 1];
        rhs[q] += acc;
      }
    }
    rc = orc_thomas(n, at, b, ct, rhs, lam);
    if (rc) goto done;
    /* u^s and u^{s-1} in interleaved order. */
    for (int i = 0; i < M; ++i) { u[2 * i] = phi_hist[(size_t)s * M + i]; uo[2 * i] = phi_hist[(size_t)(s - 1) * M + i]; }
    for (int j = 0; j <= I; ++j) { u[2 * j + 1] = J_hist[(size_t)s * (I + 1) + j]; uo[2 * j + 1] = J_hist[(size_t)(s - 1) * (I + 1) + j]; }
    for (int i = 1; i <= I; ++i) {
      const double dx = edges[i] - edges[i - 1];
      /* balance row 2i: d/d sigma_a of (A u - B u_old) = th dx phi_i - (th-1) dx phi_i^old */
      const double db = th * dx * u[2 * i] - (th - 1.0) * dx * uo[2 * i];
      g_t[i - 1] -= lam[2 * i] * db;
      g_s[i - 1] += lam[2 * i] * db;
      /* first-moment rows of the edges i-1 and i: d(Sigma_hat dx_hat)/d sigma_t,i = dx/2 */
      for (int e = i - 1; e <= i; ++e) {
        const int r = 2 * e + 1;
        const double dm = th * 0.5 * dx * u[r] - (th - 1.0) * 0.5 * dx * uo[r];
        g_t[i - 1] -= lam[r] * dm;
      }
    }
    for (int r = 0; r < n; ++r) lam_next[r] = lam[r];
  }
done:
  free(a); free(b); free(c); free(ba); free(bb); free(bc); free(at); free(ct);
  free(rhs); free(lam); free(lam_next); free(u); free(uo);
  return rc;
}
