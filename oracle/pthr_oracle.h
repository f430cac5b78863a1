/*
 * pthr_oracle.h -- plain, sequential CPU reference of one PTHR elementary Monte
 * Carlo step (EMCS) for the 3D Edwards-Anderson spin glass with Gaussian
 * couplings.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against an obviously correct implementation of the method.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load it;
 * the product path never does.  It shares no code, header, table or constant
 * generator with the HIP implementation.
 *
 * Method (paper, Sec. 2 "Model and observables" and Sec. 3 "Description of the
 * algorithm"):
 *   H = -sum_<ij> J_ij s_i s_j on an L^3 simple-cubic lattice with periodic
 *   boundaries (Eq. 1), J_ij ~ N(0,1).  N_r replica groups, each with N_T
 *   clones on a uniform temperature grid.  One EMCS = local Metropolis sweeps,
 *   one all-cluster Houdayer update (ACU) on replica pairs at T < t_acu, one
 *   parallel-tempering (PT) step inside every replica group and one
 *   entropic-reservoir (ER) step.  The ER holds n_reservoir extra clones per
 *   replica group at T_max; they are swept er_sweeps_per_emcs times per EMCS
 *   and the oldest one is exchanged with the PT clone at T_max.
 *
 * Conventions fixed here where the paper is silent (each is listed with its
 * reason in the design notes of the repository):
 *   site i = x + L*(y + L*z); neighbour order +x,-x,+y,-y,+z,-z;
 *   bond J[s][d][i] joins i and i + e_d (d = 0,1,2 for x,y,z);
 *   checkerboard sweep: all sites with (x+y+z) even in increasing i, then odd;
 *   random numbers: Philox4x32-10 (Salmon et al., SC'11) with counter
 *   (site | m<<16 | purpose<<24, t, slot, sample) and key (seed lo, seed hi).
 *
 * Precision: ORACLE_FP64 computes local fields and the Metropolis exponent in
 * double: accept iff dE <= 0 or u < exp(-beta dE).  ORACLE_FP32 computes
 * couplings, local fields and the Metropolis exponent in float, as the FP32
 * form of the GPU path, with the exponent in base 2: t = -(beta log2 e) dE
 * (beta log2 e rounded to float once per temperature), accept iff u <= 2^t
 * (2^t by a float polynomial and 2^k, overflowing to +inf and underflowing to
 * 0), which accepts every dE <= 0.  Energies, the PT exponent and all
 * observable sums stay double in both forms.
 *
 * Local update: Metropolis (the paper's choice) or heat bath (the alternative
 * Sec. 3 names): the spin is drawn from its conditional Boltzmann weight, i.e.
 * flipped with probability 1 / (1 + exp(beta dE)).  With a = exp(-beta |dE|)
 * (the same exponential routine; FP32: a = 2^t, t = -(beta log2 e)|dE|, and
 * a = 0 below t = -124 where 2^t would be subnormal) that
 * is a / (1 + a) for dE > 0 and 1 / (1 + a) for dE <= 0; the test is written
 * without a division, flip iff fma(u, a, u) < a, resp. < 1, with the same
 * random numbers as the Metropolis test.
 *
 * MicSA (App. A.1, energy-LUT paragraph; App. A.2): microcanonical local
 * update of the PT clones.  Every PT clone carries a walker holding an
 * energy W >= 0; a spin flips iff W >= dE, and then W -= dE.  The walker is
 * redrawn from its Boltzmann law at the clone's temperature T_k,
 * W = T_k (-ln u) (density exp(-W/T_k)/T_k), at the start of every PT sweep
 * whose index m in the EMCS is a multiple of micsa_refresh, so at least once
 * per EMCS; u = (b + 1) 2^-53 from 53 bits b of the block (WALKER, site 0,
 * m, t, clone id, sample), ln by the routine oracle_plog below.  FP64 form:
 * W and dE in double; FP32 form: W = (float)(T_k (-ln u)) and the test and
 * subtraction in float with the FP32 form's dE.  Reservoir clones keep
 * Metropolis (the paper's reservoir always used its probability table).
 * The cadence of the refresh is not in the paper (it cites a reference this
 * reading stands in for).
 */
#ifndef PTHR_ORACLE_H
#define PTHR_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_FP64 = 0, ORACLE_FP32 = 1 };
enum { ORACLE_ACU = 0, ORACLE_SINGLE_NEG = 1 };
enum { ORACLE_SWEEP_PT = 1, ORACLE_SWEEP_ER = 2 };
enum { ORACLE_METROPOLIS = 0, ORACLE_HEAT_BATH = 1, ORACLE_MICSA = 2 };
enum { ORACLE_NOBS = 6 }; /* sum e, sum e^2, sum q^2, sum q^4, sum q_l, sum S */

typedef struct oracle_params {
  int32_t L;
  int32_t n_samples;          /* samples held by this context                  */
  int32_t first_sample;       /* global id of sample 0 (Philox counter word 3) */
  int32_t n_replicas;         /* N_r, even, <= 64                              */
  int32_t n_temps;            /* N_T >= 2                                      */
  int32_t n_reservoir;        /* ER clones per replica group (0 = no ER)       */
  int32_t sweeps_per_emcs;    /* PT clones' sweeps per EMCS (paper: 10)        */
  int32_t er_sweeps_per_emcs; /* ER clones' sweeps per EMCS (paper: 960/4)     */
  int32_t precision;          /* ORACLE_FP64 or ORACLE_FP32                    */
  int32_t houdayer_mode;      /* ORACLE_ACU or ORACLE_SINGLE_NEG               */
  double t_acu;               /* Houdayer moves at T_k < t_acu (paper: 1.0)    */
  uint64_t seed;
  int32_t local_update;       /* ORACLE_METROPOLIS (paper), ORACLE_HEAT_BATH or ORACLE_MICSA */
  int32_t micsa_refresh;      /* MicSA: PT sweeps between walker refreshes (0 = sweeps_per_emcs) */
} oracle_params;

typedef struct oracle_ctx oracle_ctx;

/* Returns NULL and writes a message to err (if non-NULL, err_len bytes) when a
 * parameter is out of range.  Odd L is allowed here (sequential sweeps). */
oracle_ctx *oracle_create(const oracle_params *p, char *err, size_t err_len);
void oracle_destroy(oracle_ctx *c);

/* J: [n_samples][3][V] doubles, T: [n_temps] strictly increasing.  Draws the
 * initial spins and resets t, the sweep counters, permutations and ER FIFOs. */
int oracle_init_samples(oracle_ctx *c, const double *J, const double *T);

/* n sweeps of the PT clones (which & 1) and/or the ER clones (which & 2), each
 * class continuing its own sweep counter m inside the current EMCS. */
int oracle_sweep(oracle_ctx *c, int n, int which);
/* One Houdayer step: every pair (2p, 2p+1) at every T_k < t_acu. */
int oracle_houdayer(oracle_ctx *c);
/* Energies, PT swaps, round-trip bookkeeping, then (if do_reservoir and
 * n_reservoir > 0) the ER exchange.  Closes the EMCS: t += 1, m := 0. */
int oracle_pt_swap(oracle_ctx *c, int do_reservoir);
/* Adds this moment's observables into acc [S][N_T][ORACLE_NOBS] and the
 * pooled overlap histogram hist [N_T][V+1]; n_meas += 1. */
int oracle_measure(oracle_ctx *c, double *acc, uint64_t *hist, uint64_t *n_meas);
/* Full EMCS loop: sweeps, Houdayer, PT (+ER), and measure if acc != NULL. */
int oracle_run(oracle_ctx *c, int64_t n_emcs, double *acc, uint64_t *hist, uint64_t *n_meas);

/* Canonical cluster labels (root = minimum site index of the component) of the
 * Houdayer graph of pair p at temperature index k in sample s, current state. */
int oracle_cluster_labels(const oracle_ctx *c, int s, int p, int k, int32_t *labels);

/* State views (owned by the context; valid until oracle_destroy). */
int8_t *oracle_spins(oracle_ctx *c);      /* [S][C][V], +1/-1                */
int32_t *oracle_clone_at(oracle_ctx *c);  /* [S][N_r][N_T]                   */
int32_t *oracle_er_head(oracle_ctx *c);   /* [S][N_r]                        */
uint8_t *oracle_pt_last(oracle_ctx *c);   /* [S][N_r][N_T-1] last EMCS accepts */
uint32_t *oracle_pt_count(oracle_ctx *c); /* [S][N_r][N_T-1] cumulative      */
double *oracle_pt_energy(oracle_ctx *c);  /* [S][N_r*N_T] E per PT clone at the last PT step */
uint8_t *oracle_rt_state(oracle_ctx *c);  /* [S][N_r*N_T] round-trip state    */
uint64_t *oracle_rt_count(oracle_ctx *c); /* [S] completed round trips       */
double *oracle_walker(oracle_ctx *c);     /* [S][N_r*N_T] MicSA walker energy per PT clone */
int64_t oracle_t(const oracle_ctx *c);
int oracle_m(const oracle_ctx *c, int cls);
int oracle_n_clones(const oracle_ctx *c);

/* Building blocks exposed for the pin tests. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double oracle_pexp(double x);
double oracle_uniform53(uint32_t lo, uint32_t hi);
/* ln(u) for 0 < u <= 1 (u normal), the MicSA walker's logarithm. */
double oracle_plog(double u);
float oracle_uniform32(uint32_t w);
float oracle_pexp2_32(float t); /* FP32 form: 2^t (IEEE overflow and gradual underflow) */
float oracle_pexp2_32_coef(int n); /* its polynomial's coefficient c_n, n = 0..6 */
/* Heat-bath flip test given a = exp(-beta |dE|): fma(u, a, u) < (dE > 0 ? a : 1). */
int oracle_heat_bath_flip(double u, double a, double dE);
int oracle_heat_bath_flip32(float u, float a, float dE);
/* Round-trip bookkeeping of one replica group after its PT swaps (at[k]: the
 * clone at temperature k; rt_state indexed by clone); returns the number of
 * round trips completed (0 or 1). */
int oracle_round_trip_step(uint8_t *rt_state, const int32_t *at, int n_temps);
double oracle_energy(const oracle_ctx *c, int s, int clone);
double oracle_delta_e(const oracle_ctx *c, int s, int clone, int site);
int oracle_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
