/* The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers.py: chains on a random graph and on layered K4,4
 * systems run every path of orc.c (sweeps, swap rounds, the Fig. 7 flip
 * tests, the two-field form, the layer-pair order, the threaded runner), and
 * the running fields, energies and bond sums must equal a recomputation.
 * Prints "oracle_check OK"; a failed check exits non-zero. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "orc.h"

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);   \
      exit(1);                                                          \
    }                                                                   \
  } while (0)

static uint64_t rs = 88172645463325252ull;
static uint32_t rnd(void) { /* xorshift64: inputs only */
  rs ^= rs << 13;
  rs ^= rs >> 7;
  rs ^= rs << 17;
  return (uint32_t)(rs >> 32);
}
static int8_t coupling(void) {
  static const int8_t v[6] = {-3, -2, -1, 1, 2, 3};
  return v[rnd() % 6];
}

typedef struct {
  int32_t N, nE, S, M;
  int32_t *u, *v;
  int8_t *J, *h;
  uint8_t *tau;
} graph;

/* L x L K4,4 cells, M slices in a ring (M >= 3); tau edges last. */
static graph layered(int L, int M) {
  graph g;
  const int S = 8 * L * L, ne_t = 16 * L * L + 8 * L * (L - 1);
  g.S = S;
  g.M = M;
  g.N = S * M;
  g.nE = ne_t * M + S * M;
  g.u = malloc(sizeof(int32_t) * g.nE);
  g.v = malloc(sizeof(int32_t) * g.nE);
  g.J = malloc((size_t)g.nE);
  g.tau = calloc((size_t)g.nE, 1);
  g.h = malloc((size_t)g.N);
  int32_t tu[2048], tv[2048];
  int8_t tj[2048], th[512], tt[512];
  int n = 0;
  for (int y = 0; y < L; y++)
    for (int x = 0; x < L; x++) {
      const int c = (y * L + x) * 8;
      for (int k = 0; k < 4; k++)
        for (int k2 = 4; k2 < 8; k2++) tu[n] = c + k, tv[n] = c + k2, n++;
      if (y + 1 < L)
        for (int k = 0; k < 4; k++) tu[n] = c + k, tv[n] = c + 8 * L + k, n++;
      if (x + 1 < L)
        for (int k = 4; k < 8; k++) tu[n] = c + k, tv[n] = c + 8 + k, n++;
    }
  CHECK(n == ne_t);
  for (int e = 0; e < n; e++) tj[e] = coupling();
  for (int q = 0; q < S; q++) th[q] = coupling(), tt[q] = coupling();
  int e = 0;
  for (int m = 0; m < M; m++)
    for (int t = 0; t < n; t++) g.u[e] = m * S + tu[t], g.v[e] = m * S + tv[t], g.J[e] = tj[t], e++;
  for (int m = 0; m < M; m++)
    for (int q = 0; q < S; q++) {
      g.u[e] = m * S + q, g.v[e] = ((m + 1) % M) * S + q, g.J[e] = tt[q], g.tau[e] = 1, e++;
    }
  for (int m = 0; m < M; m++)
    for (int q = 0; q < S; q++) g.h[m * S + q] = th[q];
  return g;
}

static void free_graph(graph *g) {
  free(g->u);
  free(g->v);
  free(g->J);
  free(g->h);
  free(g->tau);
}

static orc_chain *chain(const graph *g, int K, uint32_t seed0) {
  double beta[64];
  uint32_t seeds[64];
  for (int k = 0; k < K; k++) {
    beta[k] = 0.1 * pow(30.0, K > 1 ? (double)k / (K - 1) : 1.0);
    seeds[k] = seed0 + (uint32_t)k;
  }
  orc_chain *c = orc_new(g->N, g->nE, g->u, g->v, g->J, g->h, K, beta, seeds, seed0 + 1000u);
  CHECK(c != NULL);
  return c;
}

int main(void) {
  /* a random graph of degree <= 8 */
  {
    graph g = {0};
    g.N = 37;
    g.u = malloc(sizeof(int32_t) * 200);
    g.v = malloc(sizeof(int32_t) * 200);
    g.J = malloc(200);
    g.h = malloc(37);
    g.tau = NULL;
    int deg[37] = {0};
    for (int t = 0; t < 5000 && g.nE < 120; t++) {
      int a = (int)(rnd() % 37), b = (int)(rnd() % 37), dup = 0;
      if (a == b || deg[a] >= 8 || deg[b] >= 8) continue;
      for (int e = 0; e < g.nE; e++) dup |= (g.u[e] == a && g.v[e] == b) || (g.u[e] == b && g.v[e] == a);
      if (dup) continue;
      g.u[g.nE] = a, g.v[g.nE] = b, g.J[g.nE] = coupling(), g.nE++, deg[a]++, deg[b]++;
    }
    for (int i = 0; i < 37; i++) g.h[i] = coupling();
    orc_chain *c = chain(&g, 6, 5489);
    orc_sweeps(c, 40, 1, NULL, NULL, NULL);
    orc_set_acceptance(c, ORC_ACCEPT_FAST);
    orc_sweeps(c, 10, 3, NULL, NULL, NULL);
    orc_set_acceptance(c, ORC_ACCEPT_ACCURATE);
    orc_sweeps(c, 10, 2, NULL, NULL, NULL);
    orc_swap_round(c, 1);
    CHECK(orc_check_fields(c) == 0);
    int8_t s[6 * 37];
    orc_get_spins(c, s);
    for (int i = 0; i < 37; i++) s[i] = (int8_t)-s[i];
    orc_set_spins(c, 0, s);
    CHECK(orc_check_fields(c) == 0);
    orc_free(c);
    free(g.u), free(g.v), free(g.J), free(g.h);
  }
  /* layered systems: recorded sweeps, the two-field form, the layer-pair order */
  {
    graph g = layered(2, 4);
    orc_chain *c = chain(&g, 5, 17);
    int32_t *es = malloc(sizeof(int32_t) * 5 * 8);
    int64_t *ss = calloc((size_t)5 * g.N, sizeof(int64_t));
    orc_sweeps(c, 8, 1, es, NULL, ss);
    CHECK(orc_check_fields(c) == 0);
    double a[5], w[5];
    for (int k = 0; k < 5; k++) a[k] = 0.05 * (k + 1), w[k] = 0.3 + 0.1 * k;
    CHECK(orc_set_two_field(c, g.tau, g.nE, a, w) == 0);
    orc_sweeps(c, 12, 1, NULL, NULL, NULL);
    CHECK(orc_check_fields(c) == 0);
    int64_t bond[5];
    orc_get_bond(c, bond);
    for (int k = 0; k < 5; k++) CHECK(bond[k] == orc_bond_of(c, k));
    int32_t *tf = malloc(sizeof(int32_t) * 5 * g.N);
    orc_get_tau_fields(c, tf);
    free(tf);
    free(es);
    free(ss);
    orc_free(c);

    orc_chain *p = chain(&g, 3, 91);
    uint32_t ps[3 * 2];
    for (int i = 0; i < 6; i++) ps[i] = 100000u + (uint32_t)i;
    CHECK(orc_set_pairs(p, g.S, g.M, ps) == 0);
    orc_sweeps(p, 9, 2, NULL, NULL, NULL);
    CHECK(orc_check_fields(p) == 0);
    uint32_t *win = malloc(sizeof(uint32_t) * 6 * 624);
    int64_t used[6];
    orc_get_pair_mt(p, win, used);
    free(win);
    orc_free(p);
    free_graph(&g);
  }
  /* the threaded runner over several chains */
  {
    graph g = layered(1, 3);
    orc_chain *cs[6];
    for (int i = 0; i < 6; i++) cs[i] = chain(&g, 4, 300u + 10u * (uint32_t)i);
    orc_run_many(6, cs, 15, 1, 3);
    for (int i = 0; i < 6; i++) {
      CHECK(orc_check_fields(cs[i]) == 0 && orc_sweeps_done(cs[i]) == 15);
      uint64_t f[4], at[4], ac[4], nr[4];
      orc_get_counters(cs[i], f, at, ac, nr);
      orc_free(cs[i]);
    }
    free_graph(&g);
  }
  for (int kind = 1; kind <= 2; kind++)
    for (int i = -400; i <= 0; i++) { /* the flip test evaluates e^x at x <= 0 */
      const float x = (float)i * 0.25f;
      const float y = orc_exp_approx(x, kind);
      CHECK(y >= 0.0f && isfinite(y));
      (void)orc_approx_threshold(0.5, -i % 64, kind);
      (void)orc_approx_threshold_x(-(double)x, kind);
    }
  printf("oracle_check OK\n");
  return 0;
}
