/*
 * hww.h -- C ABI of the MI355X (gfx950) hybrid weight-window sweep library.
 *
 * The library runs one time step of the hybrid weight-window (HWW) Monte
 * Carlo method of Shaw & Anistratov (arXiv 2512.19925) on the GPU: flight,
 * collision and census of a 1D monoenergetic slab particle bank, track-length
 * and time-crossing tallies of the scalar flux, current and second angular
 * moment, split/roulette against weight windows, and the hybrid low-order
 * second-moment (HLOSM) solve that sets the window centres.
 *
 * Conventions shared by every entry point:
 *  - Return value: HWW_OK (0) or a negative HWW_E_* code.  hww_last_error()
 *    gives a text for the last failure of a handle.
 *  - Host arrays passed in are borrowed for the duration of the call and
 *    copied; output arrays are caller-allocated host memory.
 *  - Device memory: the caller allocates one workspace of
 *    hww_workspace_bytes() bytes (any device allocation, 256-byte aligned)
 *    and keeps it alive until hww_destroy(); the library allocates no device
 *    memory of its own.  All device work is queued on the HIP stream given
 *    at init.  A handle is not thread-safe.
 *  - Calls queue work asynchronously.  Errors raised on the device (bank
 *    overflow, a non-finite or non-positive window, a zero pivot) are
 *    reported by the next call that synchronises the stream:
 *    hww_sweep_step() with a non-NULL stats pointer, hww_solve_losm() with a
 *    non-NULL output, hww_read_tallies() and hww_sync().
 *
 * Mesh: cell i (0-based) is [edges[i], edges[i+1]].  A particle exactly on an
 * interior edge belongs to the cell it moves into.  Boundaries are vacuum:
 * leaving particles are scored by the face estimators and die.
 */
#ifndef HWW_H
#define HWW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HWW_OK 0
#define HWW_E_INVALID_ARG (-1) /* bad sizes, sigma_s > sigma_t, non-ascending edges, NULL pointers */
#define HWW_E_STATE (-2)       /* step or chunk out of order                                      */
#define HWW_E_CAPACITY (-3)    /* a bank or daughter queue overflowed; the step's tallies are void */
#define HWW_E_DEVICE (-4)      /* a HIP call failed                                               */
#define HWW_E_NUMERIC (-5)     /* non-finite / non-positive window, zero pivot in the LOSM solve  */

#define HWW_FP64 0 /* FP64 flight arithmetic                                         */
#define HWW_FP32 1 /* FP32 position/direction/flight arithmetic, FP64 weights/tallies */

/* Problem of one replica (Sec. 3 Eqs. HO_transport, t-eq-bc, t-eq-ic with
 * q = 0, vacuum boundaries and an isotropic unit-weight pulse at src_x, t = 0). */
typedef struct hww_problem {
  int32_t n_cells;        /* 1 <= I <= 3136 (3137 with one chunk): the work-group's
                             LDS histogram of the sweep holds [I][6] doubles       */
  const double *edges;    /* I+1 ascending cell edges (host)                      */
  const double *sigma_t;  /* I total cross sections, > 0 (host)                   */
  const double *sigma_s;  /* I scattering cross sections, 0 <= sigma_s <= sigma_t */
  double speed;           /* v > 0                                                */
  double dt;              /* uniform time step > 0                                */
  int32_t n_steps;        /* number of time steps                                 */
  double src_x;           /* pulse position, inside [edges[0], edges[I]]          */
  int64_t n_src;          /* source particles (weight 1 each), < 2^32             */
  int64_t bank_capacity;  /* max particles in a census bank (>= n_src)            */
  uint32_t seed;          /* Philox key word 0                                    */
  uint32_t replica;       /* Philox key word 1 = (replica << 4) | slot, < 2^28    */
  int32_t n_batches;      /* statistical batches B (history src mod B), 1..64     */
  int32_t precision;      /* HWW_FP64 or HWW_FP32                                 */
  int32_t n_chunks;       /* u_ww + 1 window-update chunks per step, 1..8         */
  const double *sigma_f;  /* I fission cross sections (host), or NULL: no fission;
                             0 <= sigma_f, sigma_s + sigma_f <= sigma_t (Eq. HO_transport) */
  double nu_f;            /* mean neutrons per fission, 0 <= nu_f < 1e6 (with sigma_f) */
  int32_t comb;           /* reserve the workspace hww_comb needs and pick its reading of
                             uniform combing (Sec. 5.1): 0 no combing; 1 teeth spaced in
                             cumulative weight, every copy of weight W / n_target; 2 teeth
                             spaced in particle index, each copy keeping its particle's
                             weight times n / n_target (Sec. 5: the comb thins the many
                             particles of weight near 1 at the source)           */
  int32_t track_moments;  /* track-length moments scored per segment (Eq. phi-mc and its mu, mu^2
                             moments): 0 or 3 phi, J and K; 2 phi and K (enough for track-length
                             closures); 1 phi only (census closures need no more); the
                             tallies not scored read as zero                      */
} hww_problem;

typedef struct hww_handle hww_handle;

/* Counters of the current time step so far (all chunks swept in the step up
 * to and including the call that fills the struct, with their daughters). */
typedef struct hww_step_stats {
  uint64_t segments, collisions, scatters, absorptions, crossings, leaks, census;
  uint64_t splits, daughters, rr_kill, rr_survive, histories;
  uint64_t generations;   /* most daughter rounds (barrier-separated passes over a daughter
                             buffer) of any work-group in one launch, + 1            */
  uint64_t launches;      /* sweep-kernel launches of the step so far                   */
  double kernel_ms;       /* summed sweep-kernel time of those launches made with timing
                             on (HIP events; see hww_set_timing)                       */
  uint64_t bytes_moved;   /* algorithmic bank bytes read + written by those launches    */
  uint64_t fissions;      /* collisions that were fissions                              */
  uint64_t fission_births;/* neutrons those fissions produced (the continuing one included) */
} hww_step_stats;

/* Options of an HLOSM solve (Sec. 3 Eqs. losm-disc / losm-disc-semi, Sec. 4). */
typedef struct hww_losm_opts {
  double theta;           /* 1/2 Crank-Nicolson, 1 backward Euler                 */
  int32_t implicit;       /* 0: semi-implicit at step start (lagged closures F^{n-1}, P^{n-1});
                             1: fully implicit inside the step with the closures of the chunks
                                already swept, scaled by W_start / W_done          */
  int32_t filter;         /* 0: none, 1: moving average (Eq. moving_average),
                             2: Fourier low pass (Eqs. fft, ifft): of the discrete Fourier
                                transform of each grid function of M values keep the
                                frequencies 0..kappa and their negatives (real output) */
  int32_t ma_k;           /* moving-average half width k                          */
  double eps_min;         /* window floor of Eq. ww-center, 0 < eps_min <= 1      */
  double rho;             /* window width rho >= 1 (Eq. ww-c&f)                   */
  int32_t closure_track;  /* 0: closures from time-layer (census) tallies;
                             1: from track-length tallies of the step            */
  int32_t apply_windows;  /* 1: set the window centres from the solution         */
  int32_t kappa;          /* Fourier cutoff (filter 2), >= 0                     */
  int32_t lagged;         /* 1: lagged weight windows (Sec. 5): no LOSM solve; the window
                             shape is the Monte Carlo track-length flux of the previous step
                             (semi-implicit calls only; a step with no track flux, such as
                             the source, leaves the windows as they are)          */
  int32_t window_scale;   /* 0: centres of Eq. ww-center times s^n, the start (semi-implicit: census)
                                weight of the step per source particle;
                             1: Eq. ww-center as printed, largest centre 1      */
} hww_losm_opts;

/* Tally kinds for hww_read_tallies. */
#define HWW_TALLY_CELLS 0    /* double [B][I][6]: track phi, J, K; census phi, J, K   */
#define HWW_TALLY_BOUNDARY 1 /* double [B][2][3]: faces (left, right) x (phi, P, F)   */
#define HWW_TALLY_TRACKS 2   /* uint64 [I]: segments per cell                          */
#define HWW_TALLY_PREV_CELLS 3    /* HWW_TALLY_CELLS of the previous step              */
#define HWW_TALLY_PREV_BOUNDARY 4 /* HWW_TALLY_BOUNDARY of the previous step           */
#define HWW_TALLY_WINDOWS 5  /* double [3][I]: centre, ceiling, floor (zeros if analog) */
#define HWW_TALLY_BANK_COUNTS 6   /* uint64 [2]: start-bank and census-bank sizes      */

/* Bytes of device workspace the problem needs. Returns < 0 on invalid input. */
int64_t hww_workspace_bytes(const hww_problem *problem);

/* Validate and copy the problem, lay the workspace out, and build the source
 * bank at t^0 (isotropic directions from Philox slot 3) with its census
 * tallies, which are the initial condition of step 1.  dev_workspace must
 * hold ws_bytes >= hww_workspace_bytes() bytes of device memory.
 * hip_stream is a hipStream_t (NULL = default stream).  On success *out
 * receives a handle owned by the caller (release with hww_destroy). */
int hww_init_problem(const hww_problem *problem, void *dev_workspace, int64_t ws_bytes,
                     void *hip_stream, hww_handle **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): hww_init_problem
 * with the library's own fixed workspace in place of dev_workspace.  Each
 * GPU the library runs on holds one static array of
 * HWW_STATIC_WORKSPACE_BYTES bytes until the process ends; the handle works
 * in the copy of the device that is current at this call (hip_stream, if not
 * NULL, must belong to that device).  The call allocates no device memory.
 * Every handle made this way on one GPU shares that GPU's array, so at most
 * one may be live per GPU at a time: a second call before hww_destroy of the
 * first returns HWW_E_STATE (two processes, or handles that overlap in any
 * other way, would race).  The array keeps the last handle's contents; this
 * call clears every accumulator the sweep and the solves start from.
 * Errors: as hww_init_problem; HWW_E_INVALID_ARG also when the problem needs
 * more than HWW_STATIC_WORKSPACE_BYTES (hww_workspace_bytes tells), or the
 * stream belongs to another device; HWW_E_DEVICE when the array's address
 * cannot be looked up. */
#define HWW_STATIC_WORKSPACE_BYTES (160ll << 20)
int hww_init_problem_static(const hww_problem *problem, void *hip_stream, hww_handle **out);

/* Set absolute window centres ww_i (Sec. 2): ceiling = ww*rho, floor = ww/rho.
 * centre: I positive finite host doubles, or NULL for analog (no windows).
 * Errors: HWW_E_INVALID_ARG (rho < 1), HWW_E_NUMERIC (a centre <= 0 or not finite). */
int hww_set_windows(hww_handle *h, const double *centre, double rho);

/* Sweep chunk `chunk` of time step `step` (1-based): every particle of the
 * start-of-step bank in that chunk gets the start-of-step window check and is
 * transported to census, leakage, absorption or roulette death, together with
 * all daughters split off on the way (Sec. 2, Sec. 3).  Chunks of a step run
 * in order 0..n_chunks-1; chunk 0 of step n needs step n-1 complete and turns
 * its census bank into the start bank.  With stats == NULL the call only
 * queues one kernel launch; with stats it waits for the GPU and fills the
 * step's counters so far.  Errors: HWW_E_STATE, HWW_E_CAPACITY, HWW_E_DEVICE. */
int hww_sweep_step(hww_handle *h, int32_t step, int32_t chunk, hww_step_stats *stats);

/* Uniform combing (the population control of the supercritical test problem,
 * Sec. 5.1) of the census bank of the finished step into n_target particles
 * of equal weight W / n_target, W the census weight.  The census particles
 * are laid end to end in (src, lineage, event) order, each as long as its
 * weight taken as an integer multiple of 2^eu (eu chosen so that
 * count * max weight < 2^(53 + eu), which keeps every prefix sum exact), and
 * n_target teeth are placed at (k + xi) W / n_target with one uniform xi per
 * comb (Philox slot 7, counter (step, 0, 0, 0)).  Tooth k copies the
 * position, direction and cell of the particle it hits; the copy becomes
 * history k (lineage = step, event index 0) of batch k mod B and next-step
 * chunk (k / B) mod n_chunks.  Census tallies are unchanged; the per-chunk
 * census weights become count * W / n_target.  With comb = 2 in the problem
 * the teeth are spaced in particle index instead: tooth k copies the
 * particle at position floor((k + xi) n / n_target) of the n census
 * particles in that order, with that particle's weight times n / n_target,
 * and the per-chunk census weights are the sums of the copies' weights.
 * Call after the last chunk of
 * a step and before the next step's semi-implicit solve.  n_before and
 * w_total (nullable host pointers) receive the census size and W; an empty
 * census stays empty (both 0).  With either pointer given the call
 * synchronises the stream once; with both NULL it only queues the comb and
 * returns: an empty census then leaves an empty combed bank, and a weight
 * that is not positive and finite leaves an empty bank and an error that
 * the next synchronising call reports (HWW_E_NUMERIC, fatal).  Single
 * problems initialised with comb = 1 or 2 only.
 * Errors: HWW_E_INVALID_ARG (n_target outside 1..bank_capacity or > 2^32-1),
 * HWW_E_STATE (step not finished, no comb workspace, a batch or a view),
 * HWW_E_CAPACITY (a region of the new bank overflows), HWW_E_NUMERIC (a
 * census weight not positive and finite; the census is left as it was),
 * HWW_E_DEVICE. */
int hww_comb(hww_handle *h, int64_t n_target, int64_t *n_before, double *w_total);

/* Counters, kernel time and bank bytes of every sweep since init (same
 * fields as hww_step_stats, summed over all steps; generations is the
 * maximum; kernel_ms covers the launches made with timing on, launches
 * counts all).  Synchronises the stream. */
int hww_read_run_stats(hww_handle *h, hww_step_stats *stats);

/* Turn the timing of sweep launches on (default, on != 0) or off.  With
 * timing on, every hww_sweep_step records a HIP event on the handle's
 * stream before and after its launch, which hww_step_stats.kernel_ms sums;
 * each record adds a few microseconds between the launches.  With timing
 * off nothing is recorded and kernel_ms stays at the sum of the timed
 * launches. */
int hww_set_timing(hww_handle *h, int32_t on);

/* Solve the HLOSM equations (Sec. 3) from the tallies on the device:
 * semi-implicit (needs the previous step complete; sets windows for the next
 * step) or fully implicit (inside a step after chunk p < n_chunks-1).  With
 * apply_windows the window centres become s * [(max(phi,0)/max phi)(1-eps)+eps]
 * where s = (start-bank weight of the step) / n_src.
 * phi_out: I+2 host doubles (phi_0, cell averages, phi_{I+1}) or NULL;
 * J_out: I+1 host doubles (edge currents) or NULL. */
int hww_solve_losm(hww_handle *h, const hww_losm_opts *opts, double *phi_out, double *J_out);

/* Closures and initial condition that the finished step hands to the next
 * (Sec. 3): F (I+2: face values and cell averages of F = phi/3 - K at the
 * time layer), P (2: P_L, P_R of the step, from the face tallies), phi (I+2)
 * and J (I+1: edge currents by linear interpolation of the cell averages).
 * Unfiltered, normalised per source particle.  Needs a finished step (or
 * step 0: the source).  Synchronises the stream. */
int hww_read_closures(hww_handle *h, double *F, double *P, double *phi, double *J);

/* Deterministic LOSM march (Sec. 3 Eqs. losm-disc, fully implicit theta
 * scheme) of n_steps <= problem n_steps steps with frozen closures F[n]
 * ((n_steps+1) x (I+2)) and P[n] ((n_steps+1) x 2), from phi0 (I+2), J0
 * (I+1), with the per-cell cross sections sigma_t, sigma_s (I each, any
 * positive values; they need not equal the problem's).  Returns
 * G = sum_{n,i} weights[n][i] phi_i^n in *G and, if the pointers are not
 * NULL, the histories phi_hist ((n_steps+1) x (I+2)) and J_hist
 * ((n_steps+1) x (I+1)).  The march state stays in the workspace for
 * hww_losm_adjoint.  All arrays are host memory.  Synchronises. */
int hww_losm_march(hww_handle *h, const double *sigma_t, const double *sigma_s, double theta, int32_t n_steps,
                   const double *F, const double *P, const double *phi0, const double *J0, const double *weights,
                   double *phi_hist, double *J_hist, double *G);

/* Gradient, with respect to sigma_t and sigma_s of every cell (I host
 * doubles each), of a functional of the last hww_losm_march's flux history,
 * by the adjoint of the discretised march (Sec. 3 Eq. losm-disc): transposed
 * solves backward in time, A^T lambda^n = dG/dphi^n + B^T lambda^{n+1}, then
 * dG/dp = -sum_n lambda^n . (dA/dp u^n - dB/dp u^{n-1}).  dG_dphi gives
 * dG/dphi_i^n ((n_steps+1) x (I+2) host doubles, rows n = 0..n_steps of the
 * march); NULL takes the march's weights, i.e. the gradient of its G.  The
 * entry for n = 0 is not used (phi^0 is an input).  I <= 4096.
 * Errors: HWW_E_STATE without a preceding march.  Synchronises. */
int hww_losm_adjoint(hww_handle *h, const double *dG_dphi, double *grad_sigma_t, double *grad_sigma_s);

/* Copy a tally array of the current step to host memory.  raw = 1: per-batch
 * sums as scored (track sums w*l, time-layer sums v*w, face sums
 * w f(mu)/|mu|).  raw = 0: the same per-batch arrays normalised per source
 * particle, so that their sum over batches is the estimate: track-length
 * moments over N_src dx_i dt (Eq. phi-mc, step average), time-layer moments
 * over N_src dx_i (Eq. ct-mc, at t^n), face tallies over N_src dt (step
 * averages at the faces); the other kinds (tracks, windows, bank counts)
 * are the same either way.  out_bytes must equal the size of the kind.
 * Synchronises the stream. */
int hww_read_tallies(hww_handle *h, int32_t kind, int32_t raw, void *out, int64_t out_bytes);

/* Copy one bank to host memory (for checks): which = 0 start bank of the
 * current step, 1 census bank.  After hww_comb, 1 is the combed bank and 0
 * the census as it was before the comb.  Arrays hold up to `cap` particles;
 * *count receives the number of particles.  Any array pointer may be NULL. */
int hww_read_bank(hww_handle *h, int32_t which, int64_t cap, int64_t *count, double *x, double *mu,
                  double *w, uint32_t *src, uint64_t *lin, uint32_t *e, int32_t *cell, int32_t *chunk);

/* ---------------------------------------------------------------------------
 * Batches of replicas.  Many independent problems of uneven size (mesh,
 * cross sections, particle count, batch count) run as one handle: every
 * sweep_step is one persistent launch over the work units (replica, batch,
 * segment) of all replicas, biggest replicas first, and every solve_losm is
 * one batched launch with one work-group per replica.  Each replica keeps
 * the keying of its own problem (seed, replica), so its results equal those
 * of a handle of its own up to the summation order of the tallies.
 *
 * On a batch handle:
 *  - hww_set_windows takes the replicas' centres concatenated in replica
 *    order (sum of I_r values), or NULL for analog;
 *  - hww_solve_losm writes phi_out (sum of I_r+2) and J_out (sum of I_r+1)
 *    concatenated in replica order;
 *  - hww_read_tallies writes each replica's array of the kind, concatenated
 *    in replica order (out_bytes = the sum of their sizes);
 *  - hww_sweep_step / hww_read_run_stats sum the counters over replicas;
 *  - hww_read_bank, hww_read_closures, hww_losm_march and hww_losm_adjoint
 *    return an error: read one replica through hww_batch_replica.
 * ------------------------------------------------------------------------- */

/* Bytes of device workspace of a batch of n problems (< 0 on invalid input).
 * All problems must share precision, n_chunks and n_steps; 1 <= n <= 65535. */
int64_t hww_batch_workspace_bytes(const hww_problem *problems, int32_t n);

/* Like hww_init_problem for n problems at once (each validated as there);
 * builds every replica's source bank.  The handle is released with
 * hww_destroy. */
int hww_init_batch(const hww_problem *problems, int32_t n, void *dev_workspace, int64_t ws_bytes,
                   void *hip_stream, hww_handle **out);

/* Read-only view of replica r of a batch, owned by the batch (hww_destroy on
 * it does nothing).  The read calls (hww_read_tallies, hww_read_bank,
 * hww_read_closures, hww_sync, hww_last_error) act on that replica alone;
 * the others return HWW_E_STATE. */
int hww_batch_replica(hww_handle *batch, int32_t r, hww_handle **view);

/* Launch shape of the sweep picked by hww_autotune.  A batch sweeps its
 * replicas in up to three persistent launches per chunk, one per LDS class
 * (replicas whose sweep histogram needs at most a quarter of a compute
 * unit's LDS, at most half, more), each tuned on its own; the shape reported
 * is that of the class with the most source particles. */
typedef struct hww_tune_result {
  int32_t block;   /* threads per work-group: 256, 512 or 1024                  */
  int32_t tile;    /* particles a wavefront claims per refill: 64 .. 512        */
  int32_t grid;    /* work-groups of a launch (batches: compute units x 1..4)   */
  int32_t trials;  /* shapes measured (over all classes of a batch)             */
  double ms;       /* best measured sweep time of the trial chunk (batches: the
                      sum of the classes' best)                                 */
} hww_tune_result;

/* Measure the sweep of chunk 0 of step 1 under every launch shape (block
 * size, tile size and, for batches, the persistent grid of each LDS class)
 * twice, keep the fastest for every later sweep, and restore the state of
 * step 0.  The shapes found are kept for the life of the process: a later
 * problem of the same kind on the same device (same precision, fission,
 * chunk and batch counts, work-groups per batch and cell-record placement,
 * and the same power-of-two buckets of cell count and source particles; for
 * a batch, per LDS class: replica count, largest cell count and start
 * particles of the class) takes the stored shape without measuring, and
 * trials counts only the shapes measured by this call (0 when every shape
 * came from the store).  Must run before the first hww_sweep_step (windows
 * may already be set).  The shape changes no result beyond the summation
 * order of the tallies.
 * Errors: HWW_E_STATE after the first sweep, HWW_E_CAPACITY if a trial
 * overflows.  Synchronises. */
int hww_autotune(hww_handle *h, hww_tune_result *best);

/* Wait for the stream and report any pending device error. */
int hww_sync(hww_handle *h);

/* Text of the last error of the handle (or of the last failed init if h is NULL). */
const char *hww_last_error(const hww_handle *h);

/* Release the host state of the handle (the workspace stays the caller's). */
void hww_destroy(hww_handle *h);

#ifdef __cplusplus
}
#endif
#endif
