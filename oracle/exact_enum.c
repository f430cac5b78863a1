/*
 * exact_enum.c -- exact equilibrium averages of a small 3D Edwards-Anderson
 * sample by enumerating all 2^V spin configurations.
 *
 * TEST INFRASTRUCTURE ONLY.  It is the brute-force yardstick that pins the
 * Monte Carlo oracle: it shares no code with pthr_oracle.c (its own lattice
 * and Hamiltonian, written again from Eq. (1) of the paper) and none with the
 * GPU library.
 *
 * For every inverse temperature beta it returns, with w(s) = exp(-beta H(s)):
 *   e_mean  = <H>/V and e2_mean = <(H/V)^2>                      (Eq. 1)
 *   ql_mean = <q_l> between two independent replicas              (Eq. 4)
 *           = (1/3V) sum_bonds <s_i s_j>^2
 *   pq[Q]   = probability of the overlap Q = sum_i s_i t_i of two
 *             independent replicas, stored at index (Q+V)/2       (Eqs. 2-3)
 * using the Walsh-Hadamard transform W^(u) = sum_s w(s) (-1)^{u.s}:
 *   <s_i s_j> = W^(e_i + e_j) / W^(0), and the number of differing spins
 *   d = popcount(s xor t) has weight sum_{|x|=n} C(x), where
 *   C(x) = sum_s w(s) w(s xor x) = N^-1 sum_u W^(u)^2 (-1)^{u.x}, so that
 *   sum_{|x|=n} C(x) = N^-1 sum_m K_n(m) sum_{|u|=m} W^(u)^2 with the
 *   Krawtchouk polynomial K_n(m) = sum_j (-1)^j binom(m,j) binom(V-m,n-j).
 * Energies of all states are generated along a Gray code.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int i, j;
  double J;
} enum_bond;

static double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double b = 1.0;
  for (int t = 1; t <= k; ++t) b = b * (n - k + t) / t;
  return nearbyint(b);
}

/* H(s) = -sum_bonds J_b s_i s_j for the configuration with bit i set <=> s_i = -1. */
static double energy_of(uint64_t g, const enum_bond *bonds, int nb) {
  double E = 0.0;
  for (int b = 0; b < nb; ++b) {
    int si = ((g >> bonds[b].i) & 1) ? -1 : 1;
    int sj = ((g >> bonds[b].j) & 1) ? -1 : 1;
    E -= bonds[b].J * si * sj;
  }
  return E;
}

static void fwht(double *w, uint64_t N) {
  const uint64_t BLOCK = (uint64_t)1 << 15;
  uint64_t inner = N < BLOCK ? N : BLOCK;
  /* levels inside cache-sized blocks */
#pragma omp parallel for schedule(static)
  for (int64_t base = 0; base < (int64_t)N; base += (int64_t)inner)
    for (uint64_t h = 1; h < inner; h *= 2)
      for (uint64_t blk = (uint64_t)base; blk < (uint64_t)base + inner; blk += 2 * h)
        for (uint64_t x = blk; x < blk + h; ++x) {
          double a = w[x], b = w[x + h];
          w[x] = a + b;
          w[x + h] = a - b;
        }
  /* remaining levels across blocks */
  for (uint64_t h = inner; h < N; h *= 2) {
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < (int64_t)N; ++x) {
      if ((uint64_t)x & h) continue;
      double a = w[x], b = w[x + h];
      w[x] = a + b;
      w[x + h] = a - b;
    }
  }
}

/* Returns 0 on success, -1 on bad arguments or allocation failure. */
int exact_enumerate(int L, const double *J, int n_beta, const double *beta, double *e_mean,
                    double *e2_mean, double *ql_mean, double *pq) {
  if (L < 2 || L > 3 || n_beta < 1) return -1;
  int V = L * L * L;
  uint64_t N = (uint64_t)1 << V;
  int nb = 3 * V;
  enum_bond *bonds = (enum_bond *)malloc(sizeof(enum_bond) * nb);
  for (int z = 0; z < L; ++z)
    for (int y = 0; y < L; ++y)
      for (int x = 0; x < L; ++x) {
        int i = x + L * y + L * L * z;
        int nx = (x + 1) % L + L * y + L * L * z;
        int ny = x + L * ((y + 1) % L) + L * L * z;
        int nz = x + L * y + L * L * ((z + 1) % L);
        bonds[3 * i + 0] = (enum_bond){i, nx, J[0 * V + i]};
        bonds[3 * i + 1] = (enum_bond){i, ny, J[1 * V + i]};
        bonds[3 * i + 2] = (enum_bond){i, nz, J[2 * V + i]};
      }
  /* per-site incident bonds for the Gray-code energy update */
  int *deg = (int *)calloc(V, sizeof(int));
  int *inc_other = (int *)malloc(sizeof(int) * 2 * nb);
  double *inc_J = (double *)malloc(sizeof(double) * 2 * nb);
  int *start = (int *)calloc(V + 1, sizeof(int));
  for (int b = 0; b < nb; ++b) {
    deg[bonds[b].i]++;
    deg[bonds[b].j]++;
  }
  for (int i = 0; i < V; ++i) start[i + 1] = start[i] + deg[i];
  memset(deg, 0, sizeof(int) * V);
  for (int b = 0; b < nb; ++b) {
    int i = bonds[b].i, j = bonds[b].j;
    inc_other[start[i] + deg[i]] = j;
    inc_J[start[i] + deg[i]++] = bonds[b].J;
    inc_other[start[j] + deg[j]] = i;
    inc_J[start[j] + deg[j]++] = bonds[b].J;
  }
  double *E = (double *)malloc(sizeof(double) * N);
  double *w = (double *)malloc(sizeof(double) * N);
  if (!E || !w) {
    free(E); free(w); free(bonds); free(deg); free(inc_other); free(inc_J); free(start);
    return -1;
  }
  uint64_t g = 0;
  double Ecur = energy_of(0, bonds, nb);
  E[0] = Ecur;
  for (uint64_t n = 1; n < N; ++n) {
    int i = __builtin_ctzll(n);
    int si = ((g >> i) & 1) ? -1 : 1;
    double h = 0.0;
    for (int e = start[i]; e < start[i + 1]; ++e) {
      int sj = ((g >> inc_other[e]) & 1) ? -1 : 1;
      h += inc_J[e] * sj;
    }
    Ecur += 2.0 * si * h; /* H(after) - H(before) */
    g ^= (uint64_t)1 << i;
    if ((n & 4095) == 0) Ecur = energy_of(g, bonds, nb); /* no drift */
    E[g] = Ecur;
  }
  double Emin = E[0];
  for (uint64_t x = 1; x < N; ++x)
    if (E[x] < Emin) Emin = E[x];

  double *Sm = (double *)malloc(sizeof(double) * (V + 1));
  for (int t = 0; t < n_beta; ++t) {
    double bt = beta[t];
    double Z = 0.0, EZ = 0.0, E2Z = 0.0;
#pragma omp parallel for reduction(+ : Z, EZ, E2Z) schedule(static)
    for (int64_t x = 0; x < (int64_t)N; ++x) {
      double wx = exp(-bt * (E[x] - Emin));
      w[x] = wx;
      Z += wx;
      EZ += wx * E[x];
      E2Z += wx * E[x] * E[x];
    }
    e_mean[t] = EZ / Z / V;
    e2_mean[t] = E2Z / Z / ((double)V * V);
    fwht(w, N);
    double W0 = w[0];
    double ql = 0.0;
    for (int b = 0; b < nb; ++b) {
      double corr = w[((uint64_t)1 << bonds[b].i) | ((uint64_t)1 << bonds[b].j)] / W0;
      ql += corr * corr;
    }
    ql_mean[t] = ql / (3.0 * V);
    for (int m = 0; m <= V; ++m) Sm[m] = 0.0;
#pragma omp parallel
    {
      double loc[64];
      for (int m = 0; m <= V; ++m) loc[m] = 0.0;
#pragma omp for schedule(static)
      for (int64_t u = 0; u < (int64_t)N; ++u) loc[__builtin_popcountll((uint64_t)u)] += w[u] * w[u];
#pragma omp critical
      for (int m = 0; m <= V; ++m) Sm[m] += loc[m];
    }
    for (int n = 0; n <= V; ++n) {
      double acc = 0.0;
      for (int m = 0; m <= V; ++m) {
        double K = 0.0;
        for (int j = 0; j <= n; ++j) K += ((j & 1) ? -1.0 : 1.0) * binom(m, j) * binom(V - m, n - j);
        acc += K * Sm[m];
      }
      /* n differing spins <=> Q = V - 2n <=> index (Q+V)/2 = V - n */
      pq[(size_t)t * (V + 1) + (V - n)] = acc / ((double)N * W0 * W0);
    }
  }
  free(Sm); free(E); free(w); free(bonds); free(deg); free(inc_other); free(inc_J); free(start);
  return 0;
}
