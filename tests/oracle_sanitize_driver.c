/*
 * oracle_sanitize_driver.c -- drives every entry point of the CPU oracle
 * (pthr_oracle.c) and the exact enumerator (exact_enum.c) over small
 * lattices, so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer checks their memory accesses and arithmetic.
 * Test infrastructure only; built and run by tests/test_oracle_physics.py.
 * Exits 0 when every call succeeded.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "pthr_oracle.h"

int exact_enumerate(int L, const double *J, int n_beta, const double *beta, double *e_mean, double *e2_mean,
                    double *ql_mean, double *pq);

/* a fixed pseudo-Gaussian coupling table: sum of 12 uniforms minus 6 */
static double gauss(uint64_t *x) {
  double s = 0.0;
  for (int n = 0; n < 12; ++n) {
    *x = *x * 6364136223846793005ull + 1442695040888963407ull;
    s += (double)(*x >> 11) * 0x1p-53;
  }
  return s - 6.0;
}

static int drive(int L, int S, int NR, int NT, int NER, int prec, int mode, int update) {
  oracle_params p = {L, S, 3, NR, NT, NER, 4, 6, prec, mode, 1.0, 0x1234567890abcdefull, update};
  char err[256];
  oracle_ctx *c = oracle_create(&p, err, sizeof err);
  if (!c) {
    fprintf(stderr, "create: %s\n", err);
    return 1;
  }
  int V = L * L * L, rc = 0;
  double *J = malloc(sizeof(double) * (size_t)S * 3 * V);
  double *T = malloc(sizeof(double) * NT);
  uint64_t x = 99u + (uint64_t)L;
  for (int n = 0; n < S * 3 * V; ++n) J[n] = gauss(&x);
  for (int k = 0; k < NT; ++k) T[k] = 0.3 + 1.3 * k / (NT - 1);
  double *acc = calloc((size_t)S * NT * ORACLE_NOBS, sizeof(double));
  uint64_t *hist = calloc((size_t)NT * (V + 1), sizeof(uint64_t));
  uint64_t n_meas = 0;
  int32_t *lab = malloc(sizeof(int32_t) * V);
  rc |= oracle_init_samples(c, J, T);
  for (int e = 0; e < 3; ++e) {
    rc |= oracle_sweep(c, 4, ORACLE_SWEEP_PT);
    rc |= oracle_sweep(c, 6, ORACLE_SWEEP_ER);
    rc |= oracle_houdayer(c);
    rc |= oracle_pt_swap(c, 1);
    rc |= oracle_measure(c, acc, hist, &n_meas);
  }
  rc |= oracle_run(c, 2, acc, hist, &n_meas);
  for (int s = 0; s < S; ++s)
    for (int pr = 0; pr < NR / 2; ++pr)
      for (int k = 0; k < NT; ++k) rc |= oracle_cluster_labels(c, s, pr, k, lab);
  double sink = 0.0;
  for (int s = 0; s < S; ++s)
    for (int cl = 0; cl < oracle_n_clones(c); ++cl) {
      sink += oracle_energy(c, s, cl);
      for (int i = 0; i < V; ++i) sink += oracle_delta_e(c, s, cl, i);
    }
  if (!isfinite(sink) || n_meas != 5) rc |= 1;
  oracle_destroy(c);
  free(J); free(T); free(acc); free(hist); free(lab);
  return rc;
}

int main(void) {
  int rc = 0;
  for (int prec = 0; prec < 2; ++prec)
    for (int mode = 0; mode < 2; ++mode)
      for (int update = 0; update < 2; ++update) {
        rc |= drive(3, 2, 2, 4, 2, prec, mode, update);
        rc |= drive(4, 2, 4, 5, 3, prec, mode, update);
      }
  rc |= drive(2, 3, 2, 2, 0, 0, 0, 0);
  rc |= drive(5, 1, 6, 3, 1, 1, 1, 0);
  double v = 0.0, pe = 0.0;
  for (int n = 0; n < 2000; ++n) {
    double xx = -750.0 + 0.375 * n;
    v += oracle_pexp(xx);
    pe += oracle_pexp2_32((float)(-200.0 + 0.1 * n));
    uint32_t ctr[4] = {(uint32_t)n, 1u, 2u, 3u}, key[2] = {5u, 6u}, out[4];
    oracle_philox4x32_10(ctr, key, out);
    v += oracle_uniform53(out[0], out[1]) + oracle_uniform32(out[2]);
  }
  for (int L = 2; L <= 2; ++L) { /* L = 3 runs the same code over 2^27 states */
    int V = L * L * L;
    double *J = malloc(sizeof(double) * 3 * V), beta[3] = {0.5, 1.0, 2.0};
    double e[3], e2[3], ql[3], *pq = malloc(sizeof(double) * 3 * (V + 1));
    uint64_t x = 7u;
    for (int n = 0; n < 3 * V; ++n) J[n] = gauss(&x);
    rc |= exact_enumerate(L, J, 3, beta, e, e2, ql, pq);
    for (int k = 0; k < 3; ++k) v += e[k] + e2[k] + ql[k];
    free(J);
    free(pq);
  }
  if (!isfinite(v) || !isfinite(pe)) rc |= 1;
  printf("oracle sanitize driver: %s\n", rc ? "FAILED" : "ok");
  return rc ? 1 : 0;
}
