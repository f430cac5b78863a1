/*
 * pthr.h -- C ABI of the MI355X (gfx950) PTHR library: Parallel Tempering with
 * Houdayer all-cluster moves and an entropic Reservoir for the 3D
 * Edwards-Anderson Ising spin glass with Gaussian couplings.
 *
 * The method is the one of the paper (arXiv 2605.25872), Sec. 3 "Description
 * of the algorithm": one elementary Monte Carlo step (EMCS) of a sample is
 *   (i)   sweeps_per_emcs Metropolis sweeps of every PT clone at its own
 *         temperature, while every entropic-reservoir (ER) clone does
 *         er_sweeps_per_emcs sweeps at T_max            -> pthr_sweep
 *   (ii)  one Houdayer step on every replica pair (2p, 2p+1) at every
 *         temperature T_k < t_acu (all-cluster update by default)
 *                                                        -> pthr_houdayer
 *   (iii) one parallel-tempering step in every replica group, then
 *   (iv)  one ER step: the configuration at T_max and the oldest reservoir
 *         configuration of the group trade places       -> pthr_pt_swap
 *   and observables are accumulated                      -> pthr_measure
 * pthr_run performs whole EMCS (one launch per phase, samples batched).
 *
 * Problem statement (paper Sec. 2, Eq. 1; App. A.2): L^3 simple-cubic lattice
 * with periodic boundaries, couplings J_ij ~ N(0,1) per sample, N_T
 * temperatures (strictly increasing), N_r replica groups of N_T clones.
 *
 * Conventions
 *   site i = x + L*(y + L*z); J[s][d][i] (d = 0,1,2 for x,y,z) is the bond
 *   between i and i + e_d.  A PT clone id is r*N_T + k for the clone that
 *   starts at temperature k of group r; ER clone ids follow, N_r*N_T +
 *   r*n_reservoir + e.  Spins read back as int8 +1/-1.
 *
 * Numerics (PTHR_FP64): bit-exact with the independent CPU reference built
 * from the same definitions: Philox4x32-10 counter-based random numbers keyed
 * by (seed, sample, clone, EMCS, sweep, site) -- a Metropolis block serves 2
 * (FP64) or 4 (FP32) consecutive clone indices, reservoir clones counted from
 * the first multiple of 4 at or above N_r*N_T -- a specified double-precision
 * exp, checkerboard sweeps (sites with even x+y+z, then odd), energies summed
 * by a fixed pairwise tree.  PTHR_FP32: couplings, local fields and the
 * Metropolis exponent in float (couplings rounded to float once, also for the
 * energies); PT exponents, energies and all observable sums stay double.
 *
 * Local update (pthr_params.local_update): PTHR_METROPOLIS, the paper's
 * choice, accepts a flip with probability min{1, exp(-beta dE)}; PTHR_HEAT_BATH,
 * the alternative Sec. 3 names, draws the spin from its conditional Boltzmann
 * weight, i.e. flips with probability 1 / (1 + exp(beta dE)), tested as
 * fma(u, a, u) < a (dE > 0) or < 1 (dE <= 0) with a = exp(-beta |dE|) from the
 * same exp routine and the same random numbers.  PTHR_MICSA (PTHR*, the
 * paper's update for its longest runs; App. A.1 energy-LUT paragraph and
 * App. A.2): every PT clone carries a walker holding an energy W >= 0; a spin
 * flips iff W >= dE, and the walker then gives up dE.  The walker is redrawn
 * from its Boltzmann law at the clone's temperature, W = T_k (-ln u), at the
 * start of every PT sweep whose index m in the EMCS is a multiple of
 * micsa_refresh (u from 53 random bits, ln by a specified double routine;
 * the FP32 form rounds W to float and tests and subtracts in float); the
 * reservoir clones keep Metropolis.  All are bit-exact with the reference.
 *
 * Memory and ownership
 *   The library never allocates device memory.  The caller allocates the state
 *   buffer (pthr_state_bytes) and observable buffers (pthr_obs_bytes) on the
 *   device, e.g. as torch tensors, and passes raw device pointers and a HIP
 *   stream (hipStream_t passed as void*, NULL = default stream).  Host arrays
 *   passed in are copied before the call returns; the caller keeps them.
 *   All device work is enqueued on the given stream; functions that return
 *   host data synchronize that stream first.
 *
 * Errors: every function returns PTHR_OK (0) or a negative code; the message
 * of the last failure on a context is available from pthr_last_error.  No
 * function aborts the process.
 */
#ifndef PTHR_H
#define PTHR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PTHR_OK = 0,
  PTHR_EINVAL = -1,      /* bad argument or parameter                        */
  PTHR_EUNSUPPORTED = -2,/* valid but not supported here (odd L, LDS too small) */
  PTHR_EHIP = -3,        /* a HIP runtime call failed                         */
  PTHR_ESTATE = -4,      /* call out of order (not initialised, counters full) */
  PTHR_EDEVICE = -5      /* a kernel reported an internal bound violation     */
};
enum { PTHR_FP64 = 0, PTHR_FP32 = 1 };
enum { PTHR_ACU = 0, PTHR_SINGLE_NEG = 1 };
enum { PTHR_METROPOLIS = 0, PTHR_HEAT_BATH = 1, PTHR_MICSA = 2 };
enum { PTHR_NOBS = 6 }; /* per (sample, T): sum e, sum e^2, sum q^2, sum q^4, sum q_l, sum S */

typedef struct pthr_params {
  int32_t L;                  /* even, 2..32                                   */
  int32_t n_samples;          /* >= 1                                          */
  int32_t n_replicas;         /* N_r: even, 2..32 (pairs (0,1), (2,3), ...)    */
  int32_t n_temps;            /* N_T: 2..1024                                  */
  int32_t n_reservoir;        /* ER clones per replica group (paper: 4); 0 = no ER */
  int32_t sweeps_per_emcs;    /* PT sweeps per EMCS (paper: 10), 0..256        */
  int32_t er_sweeps_per_emcs; /* ER sweeps per EMCS (paper: 960/4 = 240), 0..256 */
  int32_t precision;          /* PTHR_FP64 or PTHR_FP32                        */
  int32_t houdayer_mode;      /* PTHR_ACU (paper) or PTHR_SINGLE_NEG (Houdayer's original) */
  int32_t local_update;       /* PTHR_METROPOLIS (paper), PTHR_HEAT_BATH or PTHR_MICSA (PTHR*) */
  double t_acu;               /* Houdayer moves at T_k < t_acu (paper: 1.0)    */
  uint64_t seed;              /* Philox key                                    */
  int32_t micsa_refresh;      /* PTHR_MICSA: PT sweeps between walker refreshes, 0..256
                                 (0 = sweeps_per_emcs: once per EMCS)          */
} pthr_params;

typedef struct pthr_ctx pthr_ctx;

/* Opaque context.  pthr_create validates the parameters (PTHR_EINVAL /
 * PTHR_EUNSUPPORTED with no context created) and picks a default launch
 * shape; it enqueues nothing.  *out is set to NULL on failure. */
int pthr_create(const pthr_params *p, pthr_ctx **out);
int pthr_destroy(pthr_ctx *ctx);
const char *pthr_last_error(const pthr_ctx *ctx); /* "" if none; valid until the next call */
/* Message of the last pthr_create failure on this thread. */
const char *pthr_create_error(void);

/* Bytes of device memory the caller must provide (0 if p is invalid).  For
 * PTHR_FP32 with PTHR_MICSA at 4 <= L <= 16 where LDS holds two samples' PT
 * spin words (every lattice of the paper's grids), this includes a second
 * copy of the couplings in the spin words' site order, written by
 * pthr_init_samples and carried by pthr_get_state/pthr_set_state. */
size_t pthr_state_bytes(const pthr_params *p);
/* Observable buffer: uint64 n_meas at offset 0; double acc[S][N_T][PTHR_NOBS]
 * at offset 256; then uint64 hist[N_T][V+1], hist[k][(Q+V)/2] counting the
 * overlaps Q of every replica pair a < b at temperature k, pooled over
 * samples (paper Sec. 2, Eqs. 2-5). */
size_t pthr_obs_bytes(const pthr_params *p);
size_t pthr_obs_acc_offset(const pthr_params *p);
size_t pthr_obs_hist_offset(const pthr_params *p);

/* Binds the state buffer d_state (pthr_state_bytes, device, 256-byte aligned,
 * owned by the caller, must outlive its use) and initialises it: copies J_host
 * [S][3][V] (double; rounded to float for PTHR_FP32) and T_host [N_T] (double,
 * strictly increasing, > 0; beta_k = 1/T_k), draws the initial spins, sets
 * every clone at its starting temperature and every reservoir FIFO to slot 0,
 * and resets the EMCS counter t and the sweep counters.  PTHR_EINVAL on
 * non-finite J or a bad grid, and for PTHR_FP32 when the Metropolis exponent
 * could leave the range its float rounding is exact in:
 * (1/T_0) log2(e) 12 max|J| must stay below 2^22 (T_0 above about 1e-4 for
 * Gaussian couplings). */
int pthr_init_samples(pthr_ctx *ctx, const double *J_host, const double *T_host, void *d_state,
                      void *stream);

/* Step (i), one launch: n_pt sweeps of every PT clone at its temperature and
 * n_er sweeps of every ER clone at T_max (paper Sec. 3: 10 and 960/4 per EMCS),
 * each class continuing its own sweep counter inside the current EMCS
 * (PTHR_ESTATE if a counter would pass 256). */
int pthr_sweep(pthr_ctx *ctx, int n_pt, int n_er, void *stream);
/* Step (ii): one Houdayer move for every pair p and every k with T_k < t_acu:
 * clusters of equal site overlap q_i = s_i^a s_i^b (paper Eq. 2) joined over
 * nearest-neighbour links; ACU flips each cluster in both replicas with
 * probability 1/2; SINGLE_NEG flips the q = -1 cluster of a uniformly chosen
 * q = -1 site. */
int pthr_houdayer(pthr_ctx *ctx, void *stream);
/* Steps (iii)+(iv): energies, PT swaps for k = 0..N_T-2 ascending, each
 * accepted with probability min{1, exp((b_k - b_{k+1})(E_k - E_{k+1}))},
 * round-trip bookkeeping, then the ER exchange if do_reservoir and
 * n_reservoir > 0.  Closes the EMCS: t += 1, sweep counters reset. */
int pthr_pt_swap(pthr_ctx *ctx, int do_reservoir, void *stream);
/* Adds the current observables to d_obs (device, pthr_obs_bytes). */
int pthr_measure(pthr_ctx *ctx, void *d_obs, void *stream);
/* Zero-fills d_obs with a kernel. */
int pthr_obs_clear(pthr_ctx *ctx, void *d_obs, void *stream);
/* n_emcs complete EMCS (sweeps, Houdayer, PT, ER, and measure if d_obs is not
 * NULL), bit-identical to the step-wise calls.  Requires the sweep counters
 * at 0 (PTHR_ESTATE otherwise). */
int pthr_run(pthr_ctx *ctx, int64_t n_emcs, void *d_obs, void *stream);

/* Canonical cluster labels of every Houdayer pair at the current state:
 * d_labels int32 [S][N_r/2][K][V] with K = #{k : T_k < t_acu}; each site holds
 * the smallest site index of its cluster. */
int pthr_cluster_labels(pthr_ctx *ctx, void *d_labels, void *stream);

/* Cluster statistics of the Houdayer graphs at the current state (paper
 * Sec. 1, Fig. 1: the largest clusters of the majority and the minority):
 * d_sizes int32 [S][N_r/2][K][2][6]; for every pair and T_k < t_acu, entry
 * [..][0][r] is the size of the (r+1)-th largest cluster of the majority (the
 * clusters whose overlap sign is that of the whole pair, q >= 0 counting as
 * positive) and [..][1][r] the same for the minority; 0 where there are fewer
 * clusters.  No spin changes.  PTHR_EUNSUPPORTED if the labels and sizes of
 * one move do not fit in LDS. */
int pthr_cluster_stats(pthr_ctx *ctx, void *d_sizes, void *stream);

/* Read-back into host arrays (NULL pointers are skipped); synchronizes. */
int pthr_read_spins(pthr_ctx *ctx, int8_t *spins /* [S][C][V] */, void *stream);
/* Replaces every clone's spins (PT and ER) with spins [S][C][V] (host, int8
 * +1/-1, same layout as pthr_read_spins; PTHR_EINVAL on any other value),
 * e.g. to continue from configurations made elsewhere or to set up a chosen
 * overlap between replicas; permutations, FIFOs and counters are kept.
 * Synchronizes. */
int pthr_write_spins(pthr_ctx *ctx, const int8_t *spins, void *stream);
int pthr_read_pt(pthr_ctx *ctx, int32_t *clone_at /* [S][N_r][N_T] */,
                 int32_t *er_head /* [S][N_r] */, uint8_t *pt_last /* [S][N_r][N_T-1] */,
                 uint32_t *pt_count /* [S][N_r][N_T-1] */, double *pt_energy /* [S][N_r*N_T] */,
                 uint8_t *rt_state /* [S][N_r*N_T] */, uint64_t *rt_count /* [S] */, void *stream);
/* MicSA walker energies [S][N_r*N_T] (host, double; FP32 form: float
 * values) of every PT clone, by clone id; synchronizes. */
int pthr_read_walkers(pthr_ctx *ctx, double *walker, void *stream);
/* EMCS counter and the sweep counters of the current EMCS. */
int pthr_counters(const pthr_ctx *ctx, int64_t *t, int32_t *m_pt, int32_t *m_er);
/* Checks the device-side status words (synchronizes): PTHR_EDEVICE if any
 * kernel hit an internal iteration bound. */
int pthr_check(pthr_ctx *ctx, void *stream);

/* Checkpoint / resume: the blob holds the counters and the whole state
 * buffer; pthr_set_state on a context with the same parameters and a bound
 * state buffer continues bit-identically. */
size_t pthr_blob_bytes(const pthr_ctx *ctx);
int pthr_get_state(pthr_ctx *ctx, void *blob, size_t bytes, void *stream);
int pthr_set_state(pthr_ctx *ctx, const void *blob, size_t bytes, void *stream);

/* Launch schedule.  threads_per_sample: work-items per sample workgroup (each
 * owns V/threads consecutive sites: 2, 4 or 8 of them; the default is the
 * smallest count with a compiled kernel, except that FP32 batches of two or
 * more samples per CU whose reservoir ends in a word of 16 clones take 4
 * sites per work-item when that still gives 256 or more work-items);
 * samples_per_launch:
 * 0 = all samples in one launch, 1 = one sample per launch (the unbatched
 * form); exp_early_out: clones with 1000/T above this value (i.e. colder than
 * T = exp_early_out/1000) decide a Metropolis test from the binade of exp(x)
 * before evaluating the polynomial; 0 = never (the default: the branch-free
 * polynomial is the faster form on gfx950).  Every schedule produces
 * identical bits. */
typedef struct pthr_schedule {
  int32_t threads_per_sample;
  int32_t samples_per_launch;
  int32_t exp_early_out;
  int32_t graph_window; /* pthr_run replays a captured HIP graph of this many EMCS (0 = plain launches) */
  int32_t clone_split;  /* sweeps: 1, 2 or 4 work-items share each chunk of sites, each taking every
                           clone_split-th group of clones of a word (more waves for small lattices);
                           threads_per_sample * clone_split <= 1024 */
  int32_t exp_filter;   /* FP64 Metropolis: 1 (default) decides each test against a float bound on
                           exp first and evaluates the FP64 polynomial only when u lies within
                           2^-20 of it; 0 evaluates the polynomial for every test.  Both give the
                           same decisions. */
  int32_t sample_split; /* sweeps: 1, 2 or 4 workgroups per sample, each taking every
                           sample_split-th group of clones of every word (the clones per
                           workgroup of the sweep); the default fills the compute units when a
                           batch has fewer samples than the GPU has CUs */
  int32_t overlap_reservoir; /* pthr_run as plain launches (graph_window = 0): 0 (default) sweeps
                                PT and reservoir clones in one launch before the Houdayer step; 1
                                runs the reservoir sweeps of each EMCS on a second stream beside
                                the PT sweeps and the Houdayer step, joined before the PT step (the
                                reservoir clones are untouched by both until the exchange, Sec. 3).
                                The library creates that stream and two events once per context.
                                pthr_run with graph_window > 0 and pthr_group_run return
                                PTHR_EUNSUPPORTED for a context with 1. */
} pthr_schedule;
int pthr_get_schedule(const pthr_ctx *ctx, pthr_schedule *out);
int pthr_set_schedule(pthr_ctx *ctx, const pthr_schedule *sch);
/* Times candidate schedules (work-items per sample, clone_split, and for
 * batches of fewer than two samples per compute unit sample_split; early-out
 * off or below T = 0.7 on the unsplit shapes; then the fastest of these with
 * overlap_reservoir = 1, for contexts with a reservoir whose schedule runs
 * plain launches) with pthr_run on a
 * scratch copy of the state (d_scratch: pthr_state_bytes bytes, device):
 * after one untimed EMCS, two timed stretches of n_emcs EMCS each, the
 * faster counting; keeps the fastest candidate (graph_window and exp_filter
 * as they were), restores nothing else.  best_ms (may be NULL) gets its time
 * per EMCS. */
int pthr_autotune(pthr_ctx *ctx, void *d_scratch, int n_emcs, double *best_ms, void *stream);
/* The candidates the last autotuning timed and their ms per EMCS, in the
 * order tried (at most `capacity` of each written; NULL arrays skipped);
 * returns the number of candidates. */
int pthr_autotune_results(const pthr_ctx *ctx, pthr_schedule *schedules, double *ms_per_emcs, int capacity);
/* pthr_autotune for callers that cannot allocate (inside stream capture,
 * serving loops, harnesses that forbid allocation): the same candidates and
 * choice except overlap_reservoir = 1 (which needs a second stream), with the
 * scratch copy of the state in a static device workspace of
 * 64 MiB (PTHR_EINVAL if pthr_state_bytes exceeds it), the trial EMCS run as
 * plain launches (no graph is instantiated) and timed with the host clock
 * (no events are created); nothing is allocated.  The workspace is held on
 * every device the library runs on until the process ends and is shared by
 * every context on that device: calls that overlap on one device race.
 * Synchronizes `stream`. */
int pthr_autotune_noalloc(pthr_ctx *ctx, int n_emcs, double *best_ms, void *stream);

/* Dynamic LDS bytes one sample workgroup needs (0 if invalid). */
size_t pthr_lds_bytes(const pthr_params *p);

/* Groups: several contexts advanced together, e.g. batches of different
 * lattice sizes (the paper simulates L = 6 ... 18 side by side; Table A1).
 * Every context keeps its own state buffer, schedule and counters; a group
 * only owns HIP streams and events (pthr_group_create) and a cached graph.
 * pthr_group_run performs n_emcs complete EMCS of every context, each exactly
 * as pthr_run would (bit-identical), the contexts' chains spread over as many
 * streams as the GPU has hardware queues (GPU_MAX_HW_QUEUES, 4 by default; a
 * further stream would share a queue with another and serialise against
 * it), larger batches first, each stream taking the next context while its
 * load (samples x sites x attempts per site) is the smallest; the streams are
 * forked from and joined back into `stream`, so that the lattices share the
 * GPU.  With graph_window > 0, windows of that many EMCS of all contexts are
 * captured into one graph (one branch per stream) and replayed; the
 * remainder runs as plain launches.  d_obs: NULL (no observables) or an
 * array of n_ctx observable buffers, entries may be NULL.  The contexts must
 * stay alive while the group exists and must not be used from another thread
 * during a run.  PTHR_ESTATE if a context is not initialised or inside an
 * EMCS. */
typedef struct pthr_group pthr_group;
int pthr_group_create(pthr_ctx *const *ctxs, int n_ctx, pthr_group **out); /* 1 <= n_ctx <= 64 */
int pthr_group_destroy(pthr_group *grp);
const char *pthr_group_last_error(const pthr_group *grp);
int pthr_group_run(pthr_group *grp, int64_t n_emcs, void *const *d_obs, int graph_window, void *stream);

#ifdef __cplusplus
}
#endif
#endif
