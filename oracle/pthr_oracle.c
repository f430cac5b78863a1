/*
 * pthr_oracle.c -- plain, sequential CPU reference of PTHR (Parallel Tempering
 * + Houdayer all-cluster moves + entropic Reservoir) for the 3D Gaussian
 * Edwards-Anderson spin glass.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It shares no
 * code with the HIP implementation.  Everything is written for readability:
 * spins are one int8 per site in natural order, every Metropolis attempt draws
 * its own Philox block, clusters are found by breadth-first search.  The only
 * parallelism is an OpenMP loop over independent samples; results do not depend
 * on the thread count.
 *
 * Paper passages followed (section / equation):
 *   Hamiltonian, periodic simple-cubic lattice, Gaussian J ........ Sec. 2, Eq. (1)
 *   site overlap q_i, overlap q, link overlap q_l ................. Sec. 2, Eqs. (2)-(4)
 *   Schwinger-Dyson-Young observable S ............................ Sec. 2, Eq. (5)
 *   EMCS = local sweeps, ACU, PT step, ER step .................... Sec. 3 (item list)
 *   Metropolis min{1, exp(-dE/T)}, dE = 2 sum_j s_i J_ij s_j ...... Sec. 3; App. A.1
 *   ACU: q_i, clusters of equal q, random sign per cluster ....... Sec. 3 (ACU paragraph)
 *   ACU only at T < 1 ............................................. Sec. 3
 *   single negative-overlap cluster (Houdayer's original) ......... Sec. 3 (two key differences)
 *   PT swaps between neighbouring temperatures .................... Sec. 3 (PT step)
 *   ER: oldest reservoir clone exchanged with the PT clone at T_max Sec. 3 (ER step)
 *   round trip T_max -> T_min -> T_max after injection ............ Sec. 5, Eq. (9)
 *
 * Readings where the paper is silent (fixed identically on the GPU side by a
 * separate implementation): checkerboard order inside a sweep; Philox counter
 * layout; the exp routine below; the standard PT acceptance
 * min{1, exp((b_k - b_{k+1})(E_k - E_{k+1}))} applied for k ascending with the
 * updated permutation; the ER exchange moves spin configurations between the
 * PT slot at T_max and the oldest reservoir slot every EMCS; energies are
 * summed by a pairwise tree over sites padded with zeros to a power of two.
 */
#include "pthr_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { PURPOSE_INIT = 1, PURPOSE_METRO = 2, PURPOSE_ACU = 3, PURPOSE_HSEED = 4, PURPOSE_PT = 5, PURPOSE_WALKER = 6 };

struct oracle_ctx {
  oracle_params p;
  int V, C, NPT, NER; /* sites, clones, PT clones (N_r*N_T), ER clones (N_r*n_reservoir) */
  int32_t *nbr;       /* [V][6]: +x,-x,+y,-y,+z,-z                                       */
  uint8_t *parity;    /* [V]: (x+y+z) & 1                                                */
  double *J;          /* [S][3][V]                                                       */
  float *J32;         /* [S][3][V] = (float)J, FP32 form only                            */
  double *T, *beta;   /* [N_T]                                                           */
  float *bl32;        /* [N_T] = (float)(beta log2 e), the FP32 form's Metropolis factor  */
  int8_t *spins;      /* [S][C][V]                                                       */
  int32_t *clone_at;  /* [S][N_r][N_T]: PT clone id at temperature k of group r          */
  int32_t *er_head;   /* [S][N_r]: oldest reservoir slot of group r                      */
  uint8_t *pt_last;   /* [S][N_r][N_T-1]                                                 */
  uint32_t *pt_count; /* [S][N_r][N_T-1]                                                 */
  double *pt_energy;  /* [S][NPT]                                                        */
  uint8_t *rt_state;  /* [S][NPT]: 0 unseen, 1 left T_max, 2 touched T_min since         */
  uint64_t *rt_count; /* [S]                                                             */
  double *walker;     /* [S][NPT]: MicSA walker energy of every PT clone                  */
  int64_t t;
  int m_pt, m_er;
  int ready;
};

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications with the
 * published multipliers, the key bumped by the published Weyl constants
 * between rounds. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * c0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t n0 = (uint32_t)(prod1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)prod1;
    uint32_t n2 = (uint32_t)(prod0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)prod0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* One Philox block for (purpose, site, sweep m, EMCS t, slot, sample s). */
static void draw(const oracle_ctx *c, int purpose, uint32_t site, uint32_t m, uint32_t t,
                 uint32_t slot, int s, uint32_t out[4]) {
  uint32_t ctr[4] = {site | (m << 16) | ((uint32_t)purpose << 24), t, slot,
                     (uint32_t)(c->p.first_sample + s)};
  uint32_t key[2] = {(uint32_t)c->p.seed, (uint32_t)(c->p.seed >> 32)};
  oracle_philox4x32_10(ctr, key, out);
}

/* 53-bit uniform in [0,1) from two words (lo, hi): exact in double. */
double oracle_uniform53(uint32_t lo, uint32_t hi) {
  uint64_t bits = (((uint64_t)hi << 32) | lo) >> 11;
  return (double)bits * 0x1p-53;
}

/* Uniform in [0,1] for the FP32 form: the 32-bit word rounded to float, scaled. */
float oracle_uniform32(uint32_t w) { return (float)w * 0x1p-32f; }

/* ------------------------------------------------------------------------- */
/* exp(x) for x <= 0, written out so both implementations compute the same
 * bits: Cody-Waite reduction x = k ln2 + r with a two-word ln2, then the
 * Taylor polynomial of degree 13 with coefficients 1/n! rounded to double,
 * evaluated by Horner with fused multiply-adds, then scaled by 2^k. */
static const double LOG2E = 0x1.71547652b82fep+0;   /* RN(1/ln 2)                      */
static const double LN2_HI = 0x1.62e42feep-1;       /* ln 2 truncated to 32 bits       */
static const double LN2_LO = 0x1.a39ef35793c76p-33; /* RN(ln 2 - LN2_HI)               */

double oracle_pexp(double x) {
  if (x < -708.0) return 0.0;
  double k = nearbyint(x * LOG2E);
  double r = fma(-k, LN2_HI, x);
  r = fma(-k, LN2_LO, r);
  double fact = 1.0;
  for (int n = 2; n <= 13; ++n) fact *= n; /* 13! is exact in double */
  double p = 1.0 / fact;                   /* RN(1/13!)              */
  for (int n = 12; n >= 0; --n) {
    fact /= (n + 1);                       /* n!, exact              */
    p = fma(p, r, 1.0 / fact);
  }
  return ldexp(p, (int)k);
}

/* ln(u) for 0 < u <= 1 (normal u), written out so both implementations
 * compute the same bits: u = 2^e m with m in [sqrt(1/2), sqrt(2)) (exact),
 * f = m - 1 (exact), s = f / (2 + f), and ln m = 2 atanh(s) =
 * 2 (s + s^3/3 + s^5/5 + ...) summed to s^23 (|s| < 0.172, so the next term
 * is below 2^-60 of the sum) by Horner in z = s^2 with coefficients
 * 2/(2n+1) rounded to double; then ln u = e LN2_HI + (e LN2_LO + ln m)
 * (e LN2_HI is exact: LN2_HI has at most 33 significant bits, |e| <= 1074). */
static const double SQRT_HALF = 0x1.6a09e667f3bcdp-1; /* RN(sqrt(1/2)) */
double oracle_plog(double u) {
  int e;
  double m = frexp(u, &e); /* u = m 2^e, m in [1/2, 1) */
  if (m < SQRT_HALF) {
    m *= 2.0;
    e -= 1;
  }
  double f = m - 1.0;
  double sv = f / (2.0 + f);
  double z = sv * sv;
  double p = 2.0 / 23.0;
  for (int n = 10; n >= 0; --n) p = fma(p, z, 2.0 / (2 * n + 1));
  double lm = sv * p;
  return fma((double)e, LN2_HI, fma((double)e, LN2_LO, lm));
}

/* FP32 form of the Metropolis exponential, in base 2: 2^t for
 * t = -(beta log2(e)) dE.  t = k + f with k = rint(t) and f = t - k (exact,
 * |f| <= 1/2); 2^f by the degree-6 polynomial 1 + c1 f + ... + c6 f^6 whose
 * coefficients minimise the largest relative error on |f| <= 1/2 (fitted by
 * oracle/exp2_fit.py, rounded to float; within 0.952 float ulp of 2^f for
 * every float f there), Horner with fmaf; then 2^k by ldexpf, which
 * overflows to +inf and underflows gradually to 0 (the Metropolis test below
 * decides the same whether a GPU keeps or flushes those subnormals: u is 0 or
 * at least 2^-32). */
static const float EXP2_COEF[7] = {0x1p+0f,        0x1.62e43p-1f,   0x1.ebfbdcp-3f, 0x1.c6aee8p-5f,
                                   0x1.3b2d4cp-7f, 0x1.5f3e54p-10f, 0x1.41fbbcp-13f};
float oracle_pexp2_32_coef(int n) { return n >= 0 && n <= 6 ? EXP2_COEF[n] : 0.0f; }
float oracle_pexp2_32(float t) {
  float k = nearbyintf(t);
  float f = t - k;
  float p = EXP2_COEF[6];
  for (int n = 5; n >= 0; --n) p = fmaf(p, f, EXP2_COEF[n]);
  return ldexpf(p, (int)k);
}

/* ------------------------------------------------------------------------- */
/* Lattice: site i = x + L*(y + L*z), periodic. */
static void build_lattice(oracle_ctx *c) {
  int L = c->p.L;
  for (int z = 0; z < L; ++z)
    for (int y = 0; y < L; ++y)
      for (int x = 0; x < L; ++x) {
        int i = x + L * (y + L * z);
        int32_t *n = c->nbr + 6 * i;
        n[0] = (x + 1) % L + L * (y + L * z);
        n[1] = (x + L - 1) % L + L * (y + L * z);
        n[2] = x + L * ((y + 1) % L + L * z);
        n[3] = x + L * ((y + L - 1) % L + L * z);
        n[4] = x + L * (y + L * ((z + 1) % L));
        n[5] = x + L * (y + L * ((z + L - 1) % L));
        c->parity[i] = (uint8_t)((x + y + z) & 1);
      }
}

/* Coupling on the bond from site i in neighbour direction d (0..5). */
static double bond(const oracle_ctx *c, int s, int i, int d) {
  const double *Js = c->J + (size_t)s * 3 * c->V;
  int axis = d / 2;
  int owner = (d % 2 == 0) ? i : c->nbr[6 * i + d]; /* J[axis][i] joins i and i+e */
  return Js[(size_t)axis * c->V + owner];
}
static float bond32(const oracle_ctx *c, int s, int i, int d) {
  const float *Js = c->J32 + (size_t)s * 3 * c->V;
  int axis = d / 2;
  int owner = (d % 2 == 0) ? i : c->nbr[6 * i + d];
  return Js[(size_t)axis * c->V + owner];
}

static int8_t *clone_spins(const oracle_ctx *c, int s, int clone) {
  return c->spins + ((size_t)s * c->C + clone) * c->V;
}

/* ------------------------------------------------------------------------- */
oracle_ctx *oracle_create(const oracle_params *p, char *err, size_t err_len) {
  const char *msg = NULL;
  if (p->L < 2 || p->L > 40) msg = "L must be in [2, 40]";
  else if (p->n_samples < 1) msg = "n_samples must be >= 1";
  else if (p->first_sample < 0) msg = "first_sample must be >= 0";
  else if (p->n_replicas < 2 || p->n_replicas > 64 || p->n_replicas % 2) msg = "n_replicas must be even and in [2, 64]";
  else if (p->n_temps < 2 || p->n_temps > 65535) msg = "n_temps must be in [2, 65535]";
  else if (p->n_reservoir < 0 || p->n_reservoir > 64) msg = "n_reservoir must be in [0, 64]";
  else if (p->sweeps_per_emcs < 0 || p->sweeps_per_emcs > 256) msg = "sweeps_per_emcs must be in [0, 256]";
  else if (p->er_sweeps_per_emcs < 0 || p->er_sweeps_per_emcs > 256) msg = "er_sweeps_per_emcs must be in [0, 256]";
  else if (p->precision != ORACLE_FP64 && p->precision != ORACLE_FP32) msg = "precision must be FP64 or FP32";
  else if (p->houdayer_mode != ORACLE_ACU && p->houdayer_mode != ORACLE_SINGLE_NEG) msg = "houdayer_mode must be ACU or SINGLE_NEG";
  else if (p->local_update != ORACLE_METROPOLIS && p->local_update != ORACLE_HEAT_BATH && p->local_update != ORACLE_MICSA)
    msg = "local_update must be METROPOLIS, HEAT_BATH or MICSA";
  else if (p->micsa_refresh < 0 || p->micsa_refresh > 256) msg = "micsa_refresh must be in [0, 256]";
  if (msg) {
    if (err && err_len) snprintf(err, err_len, "%s", msg);
    return NULL;
  }
  oracle_ctx *c = (oracle_ctx *)calloc(1, sizeof(oracle_ctx));
  c->p = *p;
  int L = p->L, S = p->n_samples, NR = p->n_replicas, NT = p->n_temps;
  c->V = L * L * L;
  c->NPT = NR * NT;
  c->NER = NR * p->n_reservoir;
  c->C = c->NPT + c->NER;
  c->nbr = (int32_t *)malloc(sizeof(int32_t) * 6 * c->V);
  c->parity = (uint8_t *)malloc(c->V);
  c->J = (double *)calloc((size_t)S * 3 * c->V, sizeof(double));
  c->J32 = (float *)calloc((size_t)S * 3 * c->V, sizeof(float));
  c->T = (double *)calloc(NT, sizeof(double));
  c->beta = (double *)calloc(NT, sizeof(double));
  c->bl32 = (float *)calloc(NT, sizeof(float));
  c->spins = (int8_t *)calloc((size_t)S * c->C * c->V, 1);
  c->clone_at = (int32_t *)calloc((size_t)S * NR * NT, sizeof(int32_t));
  c->er_head = (int32_t *)calloc((size_t)S * NR, sizeof(int32_t));
  c->pt_last = (uint8_t *)calloc((size_t)S * NR * (NT - 1), 1);
  c->pt_count = (uint32_t *)calloc((size_t)S * NR * (NT - 1), sizeof(uint32_t));
  c->pt_energy = (double *)calloc((size_t)S * c->NPT, sizeof(double));
  c->rt_state = (uint8_t *)calloc((size_t)S * c->NPT, 1);
  c->rt_count = (uint64_t *)calloc((size_t)S, sizeof(uint64_t));
  c->walker = (double *)calloc((size_t)S * c->NPT, sizeof(double));
  build_lattice(c);
  return c;
}

void oracle_destroy(oracle_ctx *c) {
  if (!c) return;
  free(c->nbr); free(c->parity); free(c->J); free(c->J32); free(c->T); free(c->beta);
  free(c->bl32); free(c->spins); free(c->clone_at); free(c->er_head); free(c->pt_last);
  free(c->pt_count); free(c->pt_energy); free(c->rt_state); free(c->rt_count); free(c->walker);
  free(c);
}

int oracle_init_samples(oracle_ctx *c, const double *J, const double *T) {
  int S = c->p.n_samples, NR = c->p.n_replicas, NT = c->p.n_temps, V = c->V;
  for (int k = 0; k < NT; ++k) {
    if (!(T[k] > 0.0) || !isfinite(T[k])) return -1;
    if (k > 0 && !(T[k] > T[k - 1])) return -1;
  }
  for (size_t n = 0; n < (size_t)S * 3 * V; ++n)
    if (!isfinite(J[n])) return -1;
  /* The FP32 form simulates the Hamiltonian with couplings rounded to float:
   * its local fields use the float values, and its energies (computed in
   * double) use the same values widened exactly. */
  for (size_t n = 0; n < (size_t)S * 3 * V; ++n) {
    c->J32[n] = (float)J[n];
    c->J[n] = (c->p.precision == ORACLE_FP32) ? (double)c->J32[n] : J[n];
  }
  for (int k = 0; k < NT; ++k) {
    c->T[k] = T[k];
    c->beta[k] = 1.0 / T[k];
    c->bl32[k] = (float)(c->beta[k] * LOG2E); /* FP32 Metropolis: beta log2(e) */
  }
  /* Random initial spins: sign bit of the first word of the INIT block. */
  for (int s = 0; s < S; ++s)
    for (int cl = 0; cl < c->C; ++cl) {
      int8_t *sp = clone_spins(c, s, cl);
      for (int i = 0; i < V; ++i) {
        uint32_t w[4];
        draw(c, PURPOSE_INIT, (uint32_t)i, 0, 0, (uint32_t)cl, s, w);
        sp[i] = (w[0] >> 31) ? -1 : 1;
      }
    }
  for (int s = 0; s < S; ++s)
    for (int r = 0; r < NR; ++r) {
      for (int k = 0; k < NT; ++k) c->clone_at[((size_t)s * NR + r) * NT + k] = r * NT + k;
      c->er_head[(size_t)s * NR + r] = 0;
    }
  memset(c->pt_last, 0, (size_t)S * NR * (NT - 1));
  memset(c->pt_count, 0, sizeof(uint32_t) * (size_t)S * NR * (NT - 1));
  memset(c->pt_energy, 0, sizeof(double) * (size_t)S * c->NPT);
  memset(c->rt_state, 0, (size_t)S * c->NPT);
  memset(c->rt_count, 0, sizeof(uint64_t) * (size_t)S);
  memset(c->walker, 0, sizeof(double) * (size_t)S * c->NPT);
  c->t = 0;
  c->m_pt = c->m_er = 0;
  c->ready = 1;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Local energy change of flipping site i: dE = 2 s_i h with h = sum_j J_ij s_j
 * over the six neighbours, summed axis by axis:
 *   h = ((t[+x] + t[-x]) + (t[+y] + t[-y])) + (t[+z] + t[-z]),  t[d] = J_d s_j(d). */
double oracle_delta_e(const oracle_ctx *c, int s, int clone, int i) {
  const int8_t *sp = clone_spins(c, s, clone);
  double t[6];
  for (int d = 0; d < 6; ++d) t[d] = bond(c, s, i, d) * (double)sp[c->nbr[6 * i + d]];
  double h = ((t[0] + t[1]) + (t[2] + t[3])) + (t[4] + t[5]);
  return 2.0 * (double)sp[i] * h;
}

static float delta_e32(const oracle_ctx *c, int s, int clone, int i) {
  const int8_t *sp = clone_spins(c, s, clone);
  float t[6];
  for (int d = 0; d < 6; ++d) t[d] = bond32(c, s, i, d) * (float)sp[c->nbr[6 * i + d]];
  float h = ((t[0] + t[1]) + (t[2] + t[3])) + (t[4] + t[5]);
  return 2.0f * (float)sp[i] * h;
}

/* Random-number index of a clone in the Metropolis draws: PT clones use their
 * id; reservoir clones follow from the first multiple of 4 at or above N_PT,
 * so that the two classes never share a Philox block. */
static int metro_index(const oracle_ctx *c, int clone) {
  return clone < c->NPT ? clone : (c->NPT + 3) / 4 * 4 + (clone - c->NPT);
}

/* Heat-bath test for a = exp(-beta |dE|): flip with probability a / (1 + a)
 * if dE > 0, else 1 / (1 + a); u (1 + a) is formed as one fused
 * multiply-add u a + u. */
int oracle_heat_bath_flip(double u, double a, double dE) { return fma(u, a, u) < (dE > 0.0 ? a : 1.0); }
int oracle_heat_bath_flip32(float u, float a, float dE) { return fmaf(u, a, u) < (dE > 0.0f ? a : 1.0f); }

/* One local update of site i of a clone at inverse temperature index k.
 * Metropolis (Sec. 3): accept the flip with probability min{1, exp(-beta dE)}.
 * Heat bath (named in Sec. 3 as the alternative): flip with probability
 * 1 / (1 + exp(beta dE)), the conditional Boltzmann probability of the
 * flipped spin; with a = exp(-beta |dE|) it is a / (1 + a) for dE > 0 and
 * 1 / (1 + a) otherwise, tested as u (1 + a) < a (resp. 1) with u (1 + a)
 * rounded once (fma(u, a, u)).  Random numbers, with n = metro_index(clone):
 * FP64: the uniform takes words (0,1) of block n/2 for even n and (2,3) for
 * odd n.  FP32: word n%4 of block n/4. */
static void metropolis_attempt(oracle_ctx *c, int s, int clone, int i, int k, int m) {
  int8_t *sp = clone_spins(c, s, clone);
  const int n = metro_index(c, clone);
  const int heat_bath = c->p.local_update == ORACLE_HEAT_BATH;
  uint32_t w[4];
  int accept;
  if (c->p.precision == ORACLE_FP64) {
    draw(c, PURPOSE_METRO, (uint32_t)i, (uint32_t)m, (uint32_t)c->t, (uint32_t)(n / 2), s, w);
    double u = (n % 2 == 0) ? oracle_uniform53(w[0], w[1]) : oracle_uniform53(w[2], w[3]);
    double dE = oracle_delta_e(c, s, clone, i);
    if (heat_bath) {
      accept = oracle_heat_bath_flip(u, oracle_pexp(-(c->beta[k] * fabs(dE))), dE);
    } else {
      accept = (dE <= 0.0) || (u < oracle_pexp(-(c->beta[k] * dE)));
    }
  } else {
    draw(c, PURPOSE_METRO, (uint32_t)i, (uint32_t)m, (uint32_t)c->t, (uint32_t)(n / 4), s, w);
    float u = oracle_uniform32(w[n % 4]);
    float dE = delta_e32(c, s, clone, i);
    if (heat_bath) {
      /* a = 0 below t = -124, where 2^t would be subnormal and the test
       * would depend on how the hardware treats subnormals */
      float t = -(c->bl32[k] * fabsf(dE));
      accept = oracle_heat_bath_flip32(u, t >= -124.0f ? oracle_pexp2_32(t) : 0.0f, dE);
    } else {
      float t = -(c->bl32[k] * dE);
      accept = u <= oracle_pexp2_32(t);
    }
  }
  if (accept) sp[i] = (int8_t)-sp[i];
}

/* One full sweep: every site of parity 0 in increasing order, then parity 1. */
static void sweep_clone(oracle_ctx *c, int s, int clone, int k, int m) {
  for (int par = 0; par < 2; ++par)
    for (int i = 0; i < c->V; ++i)
      if (c->parity[i] == par) metropolis_attempt(c, s, clone, i, k, m);
}

/* MicSA walker of a PT clone at temperature index k redrawn from its
 * Boltzmann law: W = T_k (-ln u), u = (b + 1) 2^-53 in (0, 1] from the 53
 * bits b of words (0, 1) of the block (WALKER, site 0, sweep m).  The FP32
 * form keeps the value rounded to float. */
static void refresh_walker(oracle_ctx *c, int s, int clone, int k, int m) {
  uint32_t w[4];
  draw(c, PURPOSE_WALKER, 0, (uint32_t)m, (uint32_t)c->t, (uint32_t)clone, s, w);
  uint64_t b = (((uint64_t)w[1] << 32) | w[0]) >> 11;
  double u = (double)(b + 1) * 0x1p-53;
  double W = c->T[k] * -oracle_plog(u);
  if (c->p.precision == ORACLE_FP32) W = (double)(float)W;
  c->walker[(size_t)s * c->NPT + clone] = W;
}

/* One MicSA sweep of a PT clone, in the order of sweep_clone: the spin at i
 * flips iff the walker holds at least dE, which it then gives up. */
static void micsa_sweep_clone(oracle_ctx *c, int s, int clone) {
  int8_t *sp = clone_spins(c, s, clone);
  double *W = c->walker + (size_t)s * c->NPT + clone;
  for (int par = 0; par < 2; ++par)
    for (int i = 0; i < c->V; ++i) {
      if (c->parity[i] != par) continue;
      if (c->p.precision == ORACLE_FP64) {
        double dE = oracle_delta_e(c, s, clone, i);
        if (*W >= dE) {
          sp[i] = (int8_t)-sp[i];
          *W = *W - dE;
        }
      } else {
        float dE = delta_e32(c, s, clone, i);
        float w32 = (float)*W;
        if (w32 >= dE) {
          sp[i] = (int8_t)-sp[i];
          *W = (double)(w32 - dE);
        }
      }
    }
}

/* MicSA's refresh cadence in PT sweeps. */
static int micsa_period(const oracle_ctx *c) {
  if (c->p.micsa_refresh > 0) return c->p.micsa_refresh;
  return c->p.sweeps_per_emcs > 0 ? c->p.sweeps_per_emcs : 1;
}

int oracle_sweep(oracle_ctx *c, int n, int which) {
  if (!c->ready || n < 0 || (which & ~3)) return -1;
  int do_pt = (which & ORACLE_SWEEP_PT) != 0, do_er = (which & ORACLE_SWEEP_ER) != 0 && c->NER > 0;
  if ((do_pt && c->m_pt + n > 256) || (do_er && c->m_er + n > 256)) return -1;
  int S = c->p.n_samples, NR = c->p.n_replicas, NT = c->p.n_temps;
#pragma omp parallel for schedule(dynamic, 1)
  for (int s = 0; s < S; ++s) {
    if (do_pt)
      for (int r = 0; r < NR; ++r)
        for (int k = 0; k < NT; ++k) {
          int clone = c->clone_at[((size_t)s * NR + r) * NT + k];
          for (int mm = 0; mm < n; ++mm) {
            if (c->p.local_update == ORACLE_MICSA) {
              if ((c->m_pt + mm) % micsa_period(c) == 0) refresh_walker(c, s, clone, k, c->m_pt + mm);
              micsa_sweep_clone(c, s, clone);
            } else {
              sweep_clone(c, s, clone, k, c->m_pt + mm);
            }
          }
        }
    if (do_er)
      for (int e = 0; e < c->NER; ++e)
        for (int mm = 0; mm < n; ++mm) sweep_clone(c, s, c->NPT + e, NT - 1, c->m_er + mm);
  }
  if (do_pt) c->m_pt += n;
  if (do_er) c->m_er += n;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Houdayer graph of clones a, b: neighbouring sites are joined iff their site
 * overlaps q_i = s_i^a s_i^b are equal.  Breadth-first search from the
 * smallest unlabelled site, so every label is the minimum site index of its
 * component. */
static void label_clusters(const oracle_ctx *c, int s, int a, int b, int32_t *label, int32_t *queue) {
  const int8_t *sa = clone_spins(c, s, a), *sb = clone_spins(c, s, b);
  int V = c->V;
  for (int i = 0; i < V; ++i) label[i] = -1;
  for (int root = 0; root < V; ++root) {
    if (label[root] >= 0) continue;
    int head = 0, tail = 0;
    label[root] = root;
    queue[tail++] = root;
    while (head < tail) {
      int i = queue[head++];
      int qi = sa[i] * sb[i];
      for (int d = 0; d < 6; ++d) {
        int j = c->nbr[6 * i + d];
        if (label[j] < 0 && sa[j] * sb[j] == qi) {
          label[j] = root;
          queue[tail++] = j;
        }
      }
    }
  }
}

int oracle_cluster_labels(const oracle_ctx *c, int s, int p, int k, int32_t *labels) {
  int NR = c->p.n_replicas, NT = c->p.n_temps;
  if (!c->ready || s < 0 || s >= c->p.n_samples || p < 0 || p >= NR / 2 || k < 0 || k >= NT) return -1;
  int a = c->clone_at[((size_t)s * NR + 2 * p) * NT + k];
  int b = c->clone_at[((size_t)s * NR + 2 * p + 1) * NT + k];
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * c->V);
  label_clusters(c, s, a, b, labels, queue);
  free(queue);
  return 0;
}

/* One Houdayer move on clones a, b (pair p, temperature k).
 * ACU: every cluster c draws a sign eta_c = -1 with probability 1/2 from the
 * block keyed by its root; both replicas are multiplied by eta_c on it.
 * Single: the seed is a uniformly chosen site with q_i = -1 (the j-th one in
 * increasing order, j = floor(w0 * N_minus / 2^32)); its cluster is flipped in
 * both replicas; no-op when no site has q_i = -1. */
static void houdayer_move(oracle_ctx *c, int s, int p, int k, int32_t *label, int32_t *queue) {
  int NR = c->p.n_replicas, NT = c->p.n_temps, V = c->V;
  int a = c->clone_at[((size_t)s * NR + 2 * p) * NT + k];
  int b = c->clone_at[((size_t)s * NR + 2 * p + 1) * NT + k];
  int8_t *sa = clone_spins(c, s, a), *sb = clone_spins(c, s, b);
  uint32_t slot = (uint32_t)(p * NT + k);
  label_clusters(c, s, a, b, label, queue);
  if (c->p.houdayer_mode == ORACLE_ACU) {
    /* queue[] is reused as the per-root sign: 1 = flip */
    for (int i = 0; i < V; ++i) {
      if (label[i] != i) continue;
      uint32_t w[4];
      draw(c, PURPOSE_ACU, (uint32_t)i, 0, (uint32_t)c->t, slot, s, w);
      queue[i] = (int32_t)(w[0] >> 31);
    }
    for (int i = 0; i < V; ++i)
      if (queue[label[i]]) {
        sa[i] = (int8_t)-sa[i];
        sb[i] = (int8_t)-sb[i];
      }
  } else {
    uint32_t n_minus = 0;
    for (int i = 0; i < V; ++i) n_minus += (sa[i] * sb[i] < 0);
    if (n_minus == 0) return;
    uint32_t w[4];
    draw(c, PURPOSE_HSEED, 0, 0, (uint32_t)c->t, slot, s, w);
    uint32_t j = (uint32_t)(((uint64_t)w[0] * n_minus) >> 32);
    int seed = -1;
    for (int i = 0, seen = 0; i < V; ++i)
      if (sa[i] * sb[i] < 0 && (uint32_t)seen++ == j) {
        seed = i;
        break;
      }
    int root = label[seed];
    for (int i = 0; i < V; ++i)
      if (label[i] == root) {
        sa[i] = (int8_t)-sa[i];
        sb[i] = (int8_t)-sb[i];
      }
  }
}

int oracle_houdayer(oracle_ctx *c) {
  if (!c->ready) return -1;
  int S = c->p.n_samples, NR = c->p.n_replicas, NT = c->p.n_temps;
#pragma omp parallel
  {
    int32_t *label = (int32_t *)malloc(sizeof(int32_t) * c->V);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * c->V);
#pragma omp for schedule(dynamic, 1)
    for (int s = 0; s < S; ++s)
      for (int p = 0; p < NR / 2; ++p)
        for (int k = 0; k < NT; ++k)
          if (c->T[k] < c->p.t_acu) houdayer_move(c, s, p, k, label, queue);
    free(label);
    free(queue);
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* E = -sum_<ij> J_ij s_i s_j (Eq. 1).  The 3V bond terms are grouped per site,
 * a_i = (J_x[i] s_i s_{i+x} + J_y[i] s_i s_{i+y}) + J_z[i] s_i s_{i+z}, and the
 * a_i are summed by a pairwise tree over i padded with +0.0 to a power of two. */
double oracle_energy(const oracle_ctx *c, int s, int clone) {
  const int8_t *sp = clone_spins(c, s, clone);
  const double *Js = c->J + (size_t)s * 3 * c->V;
  int V = c->V, P = 1;
  while (P < V) P *= 2;
  double *a = (double *)calloc(P, sizeof(double));
  for (int i = 0; i < V; ++i) {
    double sx = (double)(sp[i] * sp[c->nbr[6 * i + 0]]);
    double sy = (double)(sp[i] * sp[c->nbr[6 * i + 2]]);
    double sz = (double)(sp[i] * sp[c->nbr[6 * i + 4]]);
    a[i] = (Js[i] * sx + Js[V + i] * sy) + Js[2 * V + i] * sz;
  }
  for (int width = P; width > 1; width /= 2)
    for (int j = 0; j < width / 2; ++j) a[j] = a[2 * j] + a[2 * j + 1];
  double E = -a[0];
  free(a);
  return E;
}

/* Round trips (Sec. 5, definition before Eq. 9): a round trip is the stretch
 * in which a clone that starts at T_max reaches T_min and comes back to
 * T_max.  Applied to one replica group after its PT swaps, with at[k] the
 * clone at temperature k: a clone found at T_max is "at the start" (state 1);
 * a clone at the start found at T_min has "touched T_min" (state 2); a clone
 * that touched T_min and is found at T_max again completes one round trip
 * and starts the next.  Clones never seen at T_max (state 0) start nothing.
 * Returns the number of round trips completed (0 or 1). */
int oracle_round_trip_step(uint8_t *rt_state, const int32_t *at, int n_temps) {
  int done = 0;
  if (rt_state[at[0]] == 1) rt_state[at[0]] = 2;
  if (rt_state[at[n_temps - 1]] == 2) done = 1;
  rt_state[at[n_temps - 1]] = 1;
  return done;
}

/* PT step for every replica group, then the ER exchange. */
int oracle_pt_swap(oracle_ctx *c, int do_reservoir) {
  if (!c->ready) return -1;
  int S = c->p.n_samples, NR = c->p.n_replicas, NT = c->p.n_temps, V = c->V;
  int NER_G = c->p.n_reservoir;
#pragma omp parallel for schedule(dynamic, 1)
  for (int s = 0; s < S; ++s) {
    for (int clone = 0; clone < c->NPT; ++clone)
      c->pt_energy[(size_t)s * c->NPT + clone] = oracle_energy(c, s, clone);
    for (int r = 0; r < NR; ++r) {
      int32_t *at = c->clone_at + ((size_t)s * NR + r) * NT;
      const double *E = c->pt_energy + (size_t)s * c->NPT;
      for (int k = 0; k < NT - 1; ++k) {
        double x = (c->beta[k] - c->beta[k + 1]) * (E[at[k]] - E[at[k + 1]]);
        uint32_t w[4];
        draw(c, PURPOSE_PT, (uint32_t)k, 0, (uint32_t)c->t, (uint32_t)r, s, w);
        int accept = (x >= 0.0) || (oracle_uniform53(w[0], w[1]) < oracle_pexp(x));
        size_t idx = ((size_t)s * NR + r) * (NT - 1) + k;
        c->pt_last[idx] = (uint8_t)accept;
        c->pt_count[idx] += (uint32_t)accept;
        if (accept) {
          int32_t tmp = at[k];
          at[k] = at[k + 1];
          at[k + 1] = tmp;
        }
      }
      c->rt_count[s] += (uint64_t)oracle_round_trip_step(c->rt_state + (size_t)s * c->NPT, at, NT);
      /* Entropic reservoir: the configuration of the PT clone at T_max and
       * that of the oldest reservoir clone of this group trade places. */
      if (do_reservoir && NER_G > 0) {
        int32_t *head = c->er_head + (size_t)s * NR + r;
        int er_clone = c->NPT + r * NER_G + *head;
        int8_t *x1 = clone_spins(c, s, at[NT - 1]), *x2 = clone_spins(c, s, er_clone);
        for (int i = 0; i < V; ++i) {
          int8_t tmp = x1[i];
          x1[i] = x2[i];
          x2[i] = tmp;
        }
        *head = (*head + 1) % NER_G;
      }
    }
  }
  c->t += 1;
  c->m_pt = c->m_er = 0;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Observables at every temperature k of every sample (Eqs. 1-5):
 *   e_r = E(clone at k in group r) / V;
 *   for every pair of replica groups a < b: Q = sum_i q_i, Q_l = sum over the
 *   3V bonds of q_i q_j, q = Q/V, q_l = Q_l/(3V),
 *   S_ab = (e_a + e_b)/6 + (1 - q_l) * beta_k   (Eq. 5 averaged over a, b);
 * accumulated as sum_r e_r, sum_r e_r^2, sum q^2, sum q^4, sum q_l, sum S. */
int oracle_measure(oracle_ctx *c, double *acc, uint64_t *hist, uint64_t *n_meas) {
  if (!c->ready) return -1;
  int S = c->p.n_samples, NR = c->p.n_replicas, NT = c->p.n_temps, V = c->V;
  int n_pairs = NR * (NR - 1) / 2;
  int32_t *Qs = (int32_t *)malloc(sizeof(int32_t) * (size_t)S * NT * n_pairs);
#pragma omp parallel for schedule(dynamic, 1)
  for (int s = 0; s < S; ++s)
    for (int k = 0; k < NT; ++k) {
      double e[64];
      for (int r = 0; r < NR; ++r)
        e[r] = oracle_energy(c, s, c->clone_at[((size_t)s * NR + r) * NT + k]) / (double)V;
      double esum = 0.0, e2sum = 0.0, q2sum = 0.0, q4sum = 0.0, qlsum = 0.0, ssum = 0.0;
      for (int r = 0; r < NR; ++r) {
        esum += e[r];
        e2sum += e[r] * e[r];
      }
      int pair = 0;
      for (int a = 0; a < NR; ++a)
        for (int b = a + 1; b < NR; ++b, ++pair) {
          const int8_t *sa = clone_spins(c, s, c->clone_at[((size_t)s * NR + a) * NT + k]);
          const int8_t *sb = clone_spins(c, s, c->clone_at[((size_t)s * NR + b) * NT + k]);
          int32_t Q = 0, QL = 0;
          for (int i = 0; i < V; ++i) {
            int qi = sa[i] * sb[i];
            Q += qi;
            for (int d = 0; d < 6; d += 2) {
              int j = c->nbr[6 * i + d];
              QL += qi * sa[j] * sb[j];
            }
          }
          double q = (double)Q / (double)V;
          double ql = (double)QL / (3.0 * (double)V);
          double q2 = q * q;
          q2sum += q2;
          q4sum += q2 * q2;
          qlsum += ql;
          ssum += (e[a] + e[b]) / 6.0 + (1.0 - ql) * c->beta[k];
          Qs[((size_t)s * NT + k) * n_pairs + pair] = Q;
        }
      double *o = acc + ((size_t)s * NT + k) * ORACLE_NOBS;
      o[0] += esum;
      o[1] += e2sum;
      o[2] += q2sum;
      o[3] += q4sum;
      o[4] += qlsum;
      o[5] += ssum;
    }
  for (int s = 0; s < S; ++s)
    for (int k = 0; k < NT; ++k)
      for (int pair = 0; pair < n_pairs; ++pair)
        hist[(size_t)k * (V + 1) + (Qs[((size_t)s * NT + k) * n_pairs + pair] + V) / 2] += 1;
  free(Qs);
  *n_meas += 1;
  return 0;
}

int oracle_run(oracle_ctx *c, int64_t n_emcs, double *acc, uint64_t *hist, uint64_t *n_meas) {
  for (int64_t e = 0; e < n_emcs; ++e) {
    if (oracle_sweep(c, c->p.sweeps_per_emcs, ORACLE_SWEEP_PT)) return -1;
    if (c->NER > 0 && oracle_sweep(c, c->p.er_sweeps_per_emcs, ORACLE_SWEEP_ER)) return -1;
    if (oracle_houdayer(c)) return -1;
    if (oracle_pt_swap(c, 1)) return -1;
    if (acc && oracle_measure(c, acc, hist, n_meas)) return -1;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
int8_t *oracle_spins(oracle_ctx *c) { return c->spins; }
int32_t *oracle_clone_at(oracle_ctx *c) { return c->clone_at; }
int32_t *oracle_er_head(oracle_ctx *c) { return c->er_head; }
uint8_t *oracle_pt_last(oracle_ctx *c) { return c->pt_last; }
uint32_t *oracle_pt_count(oracle_ctx *c) { return c->pt_count; }
double *oracle_pt_energy(oracle_ctx *c) { return c->pt_energy; }
double *oracle_walker(oracle_ctx *c) { return c->walker; }
uint8_t *oracle_rt_state(oracle_ctx *c) { return c->rt_state; }
uint64_t *oracle_rt_count(oracle_ctx *c) { return c->rt_count; }
int64_t oracle_t(const oracle_ctx *c) { return c->t; }
int oracle_m(const oracle_ctx *c, int cls) { return cls == ORACLE_SWEEP_ER ? c->m_er : c->m_pt; }
int oracle_n_clones(const oracle_ctx *c) { return c->C; }
int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
