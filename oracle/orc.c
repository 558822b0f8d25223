/*
 * Oracle for the parallel-tempering Metropolis path -- TEST INFRASTRUCTURE.
 * Loaded only by tests/, the smoke check and the benchmark's CPU baseline.
 *
 * Every step is written the plain way, in the order the paper states it:
 *   - cost function                         Sec. 1 (equation of f)
 *   - Metropolis sweep                      Fig. 1
 *   - neighbour update h_eff[j] -= 2 s_i J  Figs. 3 and 6 (old spin value)
 *   - uniform(0,1) < flip probability       Fig. 1, Sec. 2.4 (exact exp)
 *   - MT19937 recurrence and tempering      Sec. 3, Fig. 8
 *   - parallel tempering                    Sec. 1 (named; details are the
 *                                           standard replica-exchange rule)
 * Points the paper leaves open are settled here as follows: a walker's
 * initial spin i is the top bit of its generator's i-th output; a flip with
 * d = s_i h_eff_i <= 0 is taken without comparing (its draw is still consumed);
 * swap rounds alternate even and odd pairs, each pair consumes one draw of its
 * system's swap generator, and a swap is accepted when Delta >= 0 or
 * u 2^-32 < exp(Delta), Delta = (beta_k - beta_k+1)(E_k - E_k+1).
 * Two-field form (the QMC models' separate in-slice and tau fields): slot k
 * carries weights (a_k, c_k) and a state s the log weight -a_k E_sp + c_k B;
 * a flip is taken when x = a d_sp + c d_t <= 0, else when u 2^-32 < exp(-2x);
 * swaps use the log ratio of the exchanged assignment in the same weights.
 * Layer-pair order (the paper's GPU layout): slices (2t, 2t+1) of a walker
 * share generator t; a sweep runs the even slices, then the odd ones, in index
 * order; the initial spins of slice 2t+j are the top bits of outputs
 * j*S .. j*S+S-1 of generator t.
 */
#include "orc.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* MT19937 (Matsumoto & Nishimura 1998).  Word recurrence                   */
/*   x_{k+624} = x_{k+397} ^ ((upper(x_k) | lower31(x_{k+1})) A)            */
/* with A the twist matrix (shift right, xor 0x9908b0df if the low bit is  */
/* set), output = tempering(x_{k+624}).  Seeding per the 2002 init_genrand. */
/* The last 624 words live in a circular array: word x_k in slot k mod 624. */
/* ------------------------------------------------------------------------ */
void orc_mt_seed(orc_mt *g, uint32_t seed) {
  g->x[0] = seed;
  for (int i = 1; i < 624; i++) g->x[i] = 1812433253u * (g->x[i - 1] ^ (g->x[i - 1] >> 30)) + (uint32_t)i;
  g->n = 0;
}

uint32_t orc_mt_next(orc_mt *g) {
  int k = (int)(g->n % 624); /* slot of x_n, about to become x_{n+624} */
  uint32_t upper = g->x[k] & 0x80000000u;
  uint32_t lower = g->x[(k + 1) % 624] & 0x7fffffffu;
  uint32_t y = upper | lower;
  uint32_t xa = y >> 1;
  if (y & 1u) xa ^= 0x9908b0dfu;
  uint32_t w = g->x[(k + 397) % 624] ^ xa;
  g->x[k] = w;
  g->n++;
  w ^= w >> 11;
  w ^= (w << 7) & 0x9d2c5680u;
  w ^= (w << 15) & 0xefc60000u;
  w ^= w >> 18;
  return w;
}

void orc_mt_window(const orc_mt *g, uint32_t *out624) {
  for (int j = 0; j < 624; j++) out624[j] = g->x[(g->n + j) % 624];
}

void orc_mt_stream(uint32_t seed, int64_t skip, int64_t n, uint32_t *out) {
  orc_mt g;
  orc_mt_seed(&g, seed);
  for (int64_t i = 0; i < skip; i++) (void)orc_mt_next(&g);
  for (int64_t i = 0; i < n; i++) out[i] = orc_mt_next(&g);
}

/* ------------------------------------------------------------------------ */
/* Chain state                                                              */
/* ------------------------------------------------------------------------ */
struct orc_chain {
  int32_t N, K;
  int32_t *rp, *ci; /* adjacency rows (CSR over both directions of each edge) */
  int8_t *cj;
  int8_t *h;
  double *beta; /* [K], slot k */
  int8_t *s;    /* [K][N] */
  int32_t *heff;
  int64_t *E;
  orc_mt *mt;
  orc_mt swap;
  int32_t *temp_of, *walker_at;
  uint64_t *flips, *sw_att, *sw_acc, *sw_near; /* per pair (k, k+1), at slot k */
  int64_t sweeps, rounds;
  int32_t accept_kind; /* ORC_ACCEPT_EXACT / _FAST / _ACCURATE */
  int32_t *ce;         /* input edge of each adjacency entry */
  /* two-field form (off until orc_set_two_field) */
  int32_t two_field;
  uint8_t *ctau;       /* adjacency entry is a tau edge */
  int32_t *htau;       /* [K][N] tau field; heff then holds the in-slice field (with h) */
  int64_t *B;          /* [K] sum over tau edges of J s s' */
  double *wa, *wc;     /* [K] slot weights */
  /* layer-pair order (off until orc_set_pairs) */
  int32_t pairs, pS, pM; /* spins per slice, slices (even) */
  orc_mt *pmt;           /* [K][M/2] one stream per layer pair */
};

static void recompute(orc_chain *c, int32_t w) {
  const int32_t N = c->N;
  int8_t *s = c->s + (size_t)w * N;
  int32_t *he = c->heff + (size_t)w * N;
  for (int32_t i = 0; i < N; i++) {
    int32_t f = c->h[i], ft = 0;
    for (int32_t e = c->rp[i]; e < c->rp[i + 1]; e++) {
      if (c->two_field && c->ctau[e])
        ft += c->cj[e] * s[c->ci[e]];
      else
        f += c->cj[e] * s[c->ci[e]];
    }
    he[i] = f;
    if (c->two_field) c->htau[(size_t)w * N + i] = ft;
  }
  c->E[w] = orc_energy_of(c, w);
  if (c->two_field) c->B[w] = orc_bond_of(c, w);
}

int64_t orc_bond_of(const orc_chain *c, int32_t w) {
  if (!c->two_field) return 0;
  const int32_t N = c->N;
  const int8_t *s = c->s + (size_t)w * N;
  int64_t b = 0;
  for (int32_t i = 0; i < N; i++)
    for (int32_t k = c->rp[i]; k < c->rp[i + 1]; k++) {
      int32_t j = c->ci[k];
      if (j > i && c->ctau[k]) b += (int64_t)c->cj[k] * s[i] * s[j];
    }
  return b;
}

int64_t orc_energy_of(const orc_chain *c, int32_t w) {
  const int32_t N = c->N;
  const int8_t *s = c->s + (size_t)w * N;
  int64_t e = 0;
  for (int32_t i = 0; i < N; i++) {
    e -= (int64_t)c->h[i] * s[i];
    for (int32_t k = c->rp[i]; k < c->rp[i + 1]; k++) {
      int32_t j = c->ci[k];
      if (j > i) e -= (int64_t)c->cj[k] * s[i] * s[j]; /* each undirected edge once */
    }
  }
  return e;
}

orc_chain *orc_new(int32_t N, int32_t nE, const int32_t *u, const int32_t *v, const int8_t *J,
                   const int8_t *h, int32_t K, const double *beta, const uint32_t *walker_seed,
                   uint32_t swap_seed) {
  if (N < 1 || nE < 0 || K < 1) return NULL;
  for (int32_t e = 0; e < nE; e++)
    if (u[e] < 0 || u[e] >= N || v[e] < 0 || v[e] >= N || u[e] == v[e]) return NULL;
  orc_chain *c = (orc_chain *)calloc(1, sizeof(orc_chain));
  c->N = N;
  c->K = K;
  c->rp = (int32_t *)calloc((size_t)N + 1, sizeof(int32_t));
  c->ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * nE + 1));
  c->cj = (int8_t *)malloc((size_t)(2 * nE + 1));
  c->ce = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * nE + 1));
  for (int32_t e = 0; e < nE; e++) {
    c->rp[u[e] + 1]++;
    c->rp[v[e] + 1]++;
  }
  for (int32_t i = 0; i < N; i++) c->rp[i + 1] += c->rp[i];
  int32_t *fill = (int32_t *)calloc((size_t)N, sizeof(int32_t));
  for (int32_t e = 0; e < nE; e++) {
    int32_t a = u[e], b = v[e];
    c->ci[c->rp[a] + fill[a]] = b;
    c->ce[c->rp[a] + fill[a]] = e;
    c->cj[c->rp[a] + fill[a]++] = J[e];
    c->ci[c->rp[b] + fill[b]] = a;
    c->ce[c->rp[b] + fill[b]] = e;
    c->cj[c->rp[b] + fill[b]++] = J[e];
  }
  free(fill);
  c->h = (int8_t *)malloc((size_t)N);
  memcpy(c->h, h, (size_t)N);
  c->beta = (double *)malloc(sizeof(double) * (size_t)K);
  memcpy(c->beta, beta, sizeof(double) * (size_t)K);
  c->s = (int8_t *)malloc((size_t)K * N);
  c->heff = (int32_t *)malloc(sizeof(int32_t) * (size_t)K * N);
  c->E = (int64_t *)calloc((size_t)K, sizeof(int64_t));
  c->mt = (orc_mt *)malloc(sizeof(orc_mt) * (size_t)K);
  c->temp_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
  c->walker_at = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
  c->flips = (uint64_t *)calloc((size_t)K, sizeof(uint64_t));
  c->sw_att = (uint64_t *)calloc((size_t)K, sizeof(uint64_t));
  c->sw_acc = (uint64_t *)calloc((size_t)K, sizeof(uint64_t));
  c->sw_near = (uint64_t *)calloc((size_t)K, sizeof(uint64_t));
  for (int32_t w = 0; w < K; w++) {
    orc_mt_seed(&c->mt[w], walker_seed[w]);
    /* initial spin i: +1 when the top bit of the walker's i-th output is set */
    for (int32_t i = 0; i < N; i++) c->s[(size_t)w * N + i] = (orc_mt_next(&c->mt[w]) >> 31) ? 1 : -1;
    recompute(c, w);
    c->temp_of[w] = w;
    c->walker_at[w] = w;
  }
  orc_mt_seed(&c->swap, swap_seed);
  return c;
}

void orc_free(orc_chain *c) {
  if (!c) return;
  free(c->rp);
  free(c->ci);
  free(c->cj);
  free(c->h);
  free(c->beta);
  free(c->s);
  free(c->heff);
  free(c->E);
  free(c->mt);
  free(c->temp_of);
  free(c->walker_at);
  free(c->flips);
  free(c->sw_att);
  free(c->sw_acc);
  free(c->sw_near);
  free(c->ce);
  free(c->ctau);
  free(c->htau);
  free(c->B);
  free(c->wa);
  free(c->wc);
  free(c->pmt);
  free(c);
}

/* ------------------------------------------------------------------------ */
/* Approximations of e^x (Sec. 2.4, Fig. 7, Appendix), in FP32 as the paper  */
/* states them:                                                             */
/*   fast:     i = round(x * 2^23 log2 e) + 127 * 2^23, read i as a float,  */
/*             times 2 ln^2 2;  valid for -126 ln 2 <= x < 128 ln 2;        */
/*   accurate: the same with 2^25 log2 e (so the float is ~ e^{4x}), then   */
/*             the 4th root; valid for -31.5 ln 2 <= x < 32 ln 2, and 0     */
/*             below that range.                                            */
/* "Convert" is rounding to nearest even; the 4th root is two IEEE square   */
/* roots.  Below the valid range both give 0.                               */
/* ------------------------------------------------------------------------ */
float orc_exp_approx(float x, int32_t kind) {
  const float ln2 = 0.69314718055994531f;
  const float two_ln2_sq = (float)(2.0 * 0.69314718055994531 * 0.69314718055994531);
  if (kind == ORC_ACCEPT_FAST) {
    if (x < -126.0f * ln2) return 0.0f;
    const float scale = (float)(8388608.0 * 1.4426950408889634); /* 2^23 log2 e */
    int32_t i = (int32_t)lrintf(x * scale) + 0x3F800000;
    float f;
    memcpy(&f, &i, sizeof f);
    return f * two_ln2_sq;
  }
  if (x < -31.5f * ln2) return 0.0f;
  const float scale = (float)(33554432.0 * 1.4426950408889634); /* 2^25 log2 e */
  int32_t i = (int32_t)lrintf(x * scale) + 0x3F800000;
  float f;
  memcpy(&f, &i, sizeof f);
  return sqrtf(sqrtf(f * two_ln2_sq));
}

/* Threshold of the approximate flip test for cost increase 2d (d > 0): with
 * p = approx(-2 beta d) the test u * 2^-32 < p, u a 32-bit integer, is
 * u <= ceil(2^32 p) - 1; the threshold is clamped to [0, 2^32 - 1] (so p = 0
 * leaves u = 0, one draw in 2^32). */
uint32_t orc_approx_threshold(double beta, int32_t d, int32_t kind) {
  const float p = orc_exp_approx((float)(-2.0 * beta * (double)d), kind);
  const double t = ceil((double)p * 4294967296.0) - 1.0;
  if (t < 0.0) return 0u;
  if (t > 4294967295.0) return 4294967295u;
  return (uint32_t)t;
}

/* The same for a real cost change 2x (the two-field form): p = approx(-2x). */
uint32_t orc_approx_threshold_x(double x, int32_t kind) {
  const float p = orc_exp_approx((float)(-2.0 * x), kind);
  const double t = ceil((double)p * 4294967296.0) - 1.0;
  if (t < 0.0) return 0u;
  if (t > 4294967295.0) return 4294967295u;
  return (uint32_t)t;
}

void orc_set_acceptance(orc_chain *c, int32_t kind) { c->accept_kind = kind; }

/* ------------------------------------------------------------------------ */
/* Two-field form (Sec. 2.1-2.2: the QMC models keep a field over the       */
/* in-slice edges, h_eff_space, and one over the two tau edges of a spin,   */
/* h_eff_tau, updated by the edge-type switch of Figs. 2 and 3).  Slot k    */
/* weighs a state s by exp(-a_k E_sp(s) + c_k B(s)): E_sp the cost of h and */
/* the in-slice edges, B the sum over tau edges of J s s'.  Flipping spin i */
/* changes the log weight by -2x, x = a d_sp + c d_t, d_sp = s_i             */
/* h_eff_space_i, d_t = s_i h_eff_tau_i.                                     */
/* ------------------------------------------------------------------------ */
int32_t orc_set_two_field(orc_chain *c, const uint8_t *is_tau, int32_t nE, const double *a,
                          const double *cw) {
  if (!is_tau || !a || !cw) return -1;
  const int32_t n_adj = c->rp[c->N];
  for (int32_t e = 0; e < n_adj; e++)
    if (c->ce[e] < 0 || c->ce[e] >= nE) return -1;
  free(c->ctau);
  free(c->htau);
  free(c->B);
  free(c->wa);
  free(c->wc);
  c->ctau = (uint8_t *)malloc((size_t)n_adj + 1);
  for (int32_t e = 0; e < n_adj; e++) c->ctau[e] = is_tau[c->ce[e]] ? 1 : 0;
  c->htau = (int32_t *)calloc((size_t)c->K * c->N, sizeof(int32_t));
  c->B = (int64_t *)calloc((size_t)c->K, sizeof(int64_t));
  c->wa = (double *)malloc(sizeof(double) * (size_t)c->K);
  c->wc = (double *)malloc(sizeof(double) * (size_t)c->K);
  memcpy(c->wa, a, sizeof(double) * (size_t)c->K);
  memcpy(c->wc, cw, sizeof(double) * (size_t)c->K);
  c->two_field = 1;
  for (int32_t w = 0; w < c->K; w++) recompute(c, w);
  return 0;
}

/* Fig. 1 with the two fields: one draw per spin; accept when x <= 0, else
 * when the uniform is below exp(-2x); after a flip, each incident edge
 * updates the neighbour's tau or in-slice field (Figs. 2 and 3). */
static void sweep_walker_two_field(orc_chain *c, int32_t w) {
  const int32_t N = c->N;
  int8_t *s = c->s + (size_t)w * N;
  int32_t *hs = c->heff + (size_t)w * N;
  int32_t *ht = c->htau + (size_t)w * N;
  const int32_t k = c->temp_of[w];
  const double a = c->wa[k], cw = c->wc[k];
  orc_mt *g = &c->mt[w];
  for (int32_t i = 0; i < N; i++) {
    const uint32_t u = orc_mt_next(g); /* one draw per spin */
    int32_t d_sp = s[i] * hs[i];
    int32_t d_t = s[i] * ht[i];
    double x_sp = a * (double)d_sp;
    double x_t = cw * (double)d_t;
    double x = x_sp + x_t; /* the log weight changes by -2x */
    int accept;
    if (x <= 0.0) {
      accept = 1;
    } else if (c->accept_kind == ORC_ACCEPT_EXACT) {
      double uniform = (double)u * 0x1p-32;
      accept = uniform < exp(-2.0 * x);
    } else {
      accept = u <= orc_approx_threshold_x(x, c->accept_kind);
    }
    if (accept) {
      int32_t two_s = 2 * s[i]; /* old spin value */
      for (int32_t e = c->rp[i]; e < c->rp[i + 1]; e++) {
        int32_t *field = c->ctau[e] ? ht : hs;
        field[c->ci[e]] -= two_s * c->cj[e];
      }
      s[i] = (int8_t)-s[i];
      c->E[w] += 2 * (d_sp + d_t);
      c->B[w] -= 2 * d_t;
      c->flips[w]++;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Layer-pair order (Sec. 3.2, Fig. 12c): the M slices of a layered system   */
/* are grouped in pairs (2t, 2t+1), each pair with its own generator; a      */
/* sweep first visits every even slice, each in index order with draws from  */
/* its pair's generator, then every odd slice the same way.  Slices of one   */
/* parity share no edge, so the order among pairs does not matter.           */
/* Spin i = m*S + q.  The walker's initial spin (2t+j, q) is +1 when the top */
/* bit of output j*S + q of pair t's generator is set.                       */
/* ------------------------------------------------------------------------ */
/* One Metropolis step of spin i of walker w with uniform word u (Fig. 1). */
static void metropolis_at(orc_chain *c, int32_t w, int32_t i, uint32_t u, double beta) {
  int8_t *s = c->s + (size_t)w * c->N;
  int32_t *he = c->heff + (size_t)w * c->N;
  int32_t d = s[i] * he[i];    /* flipping changes the cost by 2d */
  int accept;
  if (d <= 0) {
    accept = 1; /* probability min(1, exp(-beta*2d)) = 1 */
  } else if (c->accept_kind == ORC_ACCEPT_EXACT) {
    double p = exp(-2.0 * beta * (double)d);
    double uniform = (double)u * 0x1p-32; /* in [0, 1) */
    accept = uniform < p;
  } else {
    accept = u <= orc_approx_threshold(beta, d, c->accept_kind);
  }
  if (accept) {
    int32_t two_s = 2 * s[i]; /* the old spin value */
    for (int32_t e = c->rp[i]; e < c->rp[i + 1]; e++) he[c->ci[e]] -= two_s * c->cj[e];
    s[i] = (int8_t)-s[i];
    c->E[w] += 2 * d;
    c->flips[w]++;
  }
}

static void sweep_walker_pairs(orc_chain *c, int32_t w) {
  const int32_t S = c->pS, P = c->pM / 2;
  const double beta = c->beta[c->temp_of[w]];
  for (int32_t parity = 0; parity < 2; parity++)
    for (int32_t t = 0; t < P; t++) {
      orc_mt *g = &c->pmt[(size_t)w * P + t];
      const int32_t m = 2 * t + parity;
      for (int32_t q = 0; q < S; q++) metropolis_at(c, w, m * S + q, orc_mt_next(g), beta);
    }
}

int32_t orc_set_pairs(orc_chain *c, int32_t S, int32_t M, const uint32_t *pair_seed) {
  if (!pair_seed || S < 1 || M < 2 || (M & 1) || (int64_t)S * M != c->N || c->two_field) return -1;
  const int32_t P = M / 2;
  free(c->pmt);
  c->pmt = (orc_mt *)malloc(sizeof(orc_mt) * (size_t)c->K * P);
  c->pairs = 1;
  c->pS = S;
  c->pM = M;
  for (int32_t w = 0; w < c->K; w++) {
    int8_t *s = c->s + (size_t)w * c->N;
    for (int32_t t = 0; t < P; t++) {
      orc_mt *g = &c->pmt[(size_t)w * P + t];
      orc_mt_seed(g, pair_seed[(size_t)w * P + t]);
      for (int32_t j = 0; j < 2; j++)
        for (int32_t q = 0; q < S; q++) s[(2 * t + j) * S + q] = (orc_mt_next(g) >> 31) ? 1 : -1;
    }
    recompute(c, w);
  }
  return 0;
}

void orc_get_pair_mt(const orc_chain *c, uint32_t *win, int64_t *used) {
  const int32_t n = c->pairs ? c->K * (c->pM / 2) : 0;
  for (int32_t i = 0; i < n; i++) {
    orc_mt_window(&c->pmt[i], win + (size_t)i * 624);
    used[i] = c->pmt[i].n;
  }
}

/* Fig. 1: for each spin in order, draw a uniform; flip if it is below the
 * flip probability; after a flip update the local fields of the neighbours. */
static void sweep_walker(orc_chain *c, int32_t w) {
  if (c->two_field) {
    sweep_walker_two_field(c, w);
    return;
  }
  if (c->pairs) {
    sweep_walker_pairs(c, w);
    return;
  }
  const int32_t N = c->N;
  const double beta = c->beta[c->temp_of[w]];
  orc_mt *g = &c->mt[w];
  for (int32_t i = 0; i < N; i++) {
    uint32_t u = orc_mt_next(g); /* one draw per spin, also when dE <= 0 */
    metropolis_at(c, w, i, u, beta);
  }
}

/* One round of neighbour exchanges: pairs (k, k+1) with k = parity mod 2.
 * Accept with probability min(1, exp((beta_k - beta_{k+1}) (E_k - E_{k+1})))
 * where E_k is the energy of the walker at slot k; one draw per pair. */
void orc_swap_round(orc_chain *c, int32_t parity) {
  for (int32_t k = parity & 1; k + 1 < c->K; k += 2) {
    int32_t a = c->walker_at[k], b = c->walker_at[k + 1];
    double delta = (c->beta[k] - c->beta[k + 1]) * (double)(c->E[a] - c->E[b]);
    if (c->two_field) {
      /* log ratio of the exchanged to the current assignment:
       * (a_k - a_k+1)(Esp_a - Esp_b) - (c_k - c_k+1)(B_a - B_b), Esp = E + B */
      int64_t esp_a = c->E[a] + c->B[a], esp_b = c->E[b] + c->B[b];
      double d_sp = (c->wa[k] - c->wa[k + 1]) * (double)(esp_a - esp_b);
      double d_t = (c->wc[k] - c->wc[k + 1]) * (double)(c->B[a] - c->B[b]);
      delta = d_sp - d_t;
    }
    uint32_t u = orc_mt_next(&c->swap);
    double uniform = (double)u * 0x1p-32;
    double p = exp(delta);
    int accept = (delta >= 0.0) || (uniform < p);
    if (delta < 0.0 && fabs(uniform - p) < 1e-12) c->sw_near[k]++; /* decided within 1e-12 */
    c->sw_att[k]++;
    if (accept) {
      c->walker_at[k] = b;
      c->walker_at[k + 1] = a;
      c->temp_of[a] = k + 1;
      c->temp_of[b] = k;
      c->sw_acc[k]++;
    }
  }
  c->rounds++;
}

void orc_sweeps(orc_chain *c, int32_t n, int32_t swap_every, int32_t *e_series,
                uint32_t *bits_series, int64_t *slot_spin_sum) {
  const int32_t N = c->N, K = c->K;
  for (int32_t t = 0; t < n; t++) {
    for (int32_t w = 0; w < K; w++) sweep_walker(c, w);
    c->sweeps++;
    if (swap_every > 0 && c->sweeps % swap_every == 0) orc_swap_round(c, (int32_t)(c->rounds & 1));
    for (int32_t k = 0; k < K; k++) {
      int32_t w = c->walker_at[k];
      const int8_t *s = c->s + (size_t)w * N;
      if (e_series) e_series[(size_t)t * K + k] = (int32_t)c->E[w];
      if (bits_series) {
        uint32_t b = 0;
        for (int32_t i = 0; i < N && i < 32; i++)
          if (s[i] > 0) b |= 1u << i;
        bits_series[(size_t)t * K + k] = b;
      }
      if (slot_spin_sum)
        for (int32_t i = 0; i < N; i++) slot_spin_sum[(size_t)k * N + i] += s[i];
    }
  }
}

typedef struct {
  orc_chain **chains;
  int32_t n_chains, n, swap_every;
  int32_t next;
  pthread_mutex_t lock;
} run_job;

static void *run_worker(void *arg) {
  run_job *job = (run_job *)arg;
  for (;;) {
    pthread_mutex_lock(&job->lock);
    int32_t i = job->next++;
    pthread_mutex_unlock(&job->lock);
    if (i >= job->n_chains) break;
    orc_sweeps(job->chains[i], job->n, job->swap_every, NULL, NULL, NULL);
  }
  return NULL;
}

void orc_run_many(int32_t n_chains, orc_chain **chains, int32_t n, int32_t swap_every,
                  int32_t n_threads) {
  if (n_threads < 1) n_threads = 1;
  if (n_threads > n_chains) n_threads = n_chains;
  run_job job = {chains, n_chains, n, swap_every, 0, PTHREAD_MUTEX_INITIALIZER};
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
  for (int32_t t = 0; t < n_threads; t++) pthread_create(&th[t], NULL, run_worker, &job);
  for (int32_t t = 0; t < n_threads; t++) pthread_join(th[t], NULL);
  free(th);
}

int32_t orc_N(const orc_chain *c) { return c->N; }
int32_t orc_K(const orc_chain *c) { return c->K; }
int64_t orc_sweeps_done(const orc_chain *c) { return c->sweeps; }
int64_t orc_rounds_done(const orc_chain *c) { return c->rounds; }

void orc_get_spins(const orc_chain *c, int8_t *out) { memcpy(out, c->s, (size_t)c->K * c->N); }
void orc_get_fields(const orc_chain *c, int32_t *out) {
  memcpy(out, c->heff, sizeof(int32_t) * (size_t)c->K * c->N);
}
void orc_get_energy(const orc_chain *c, int64_t *out) { memcpy(out, c->E, sizeof(int64_t) * (size_t)c->K); }
void orc_get_labels(const orc_chain *c, int32_t *temp_of, int32_t *walker_at) {
  memcpy(temp_of, c->temp_of, sizeof(int32_t) * (size_t)c->K);
  memcpy(walker_at, c->walker_at, sizeof(int32_t) * (size_t)c->K);
}
void orc_get_mt(const orc_chain *c, uint32_t *win, int64_t *used) {
  for (int32_t w = 0; w < c->K; w++) {
    orc_mt_window(&c->mt[w], win + (size_t)w * 624);
    used[w] = c->mt[w].n;
  }
}
void orc_get_swap_mt(const orc_chain *c, uint32_t *win624, int64_t *used) {
  orc_mt_window(&c->swap, win624);
  *used = c->swap.n;
}
void orc_get_counters(const orc_chain *c, uint64_t *flips, uint64_t *sw_att, uint64_t *sw_acc,
                      uint64_t *sw_near) {
  memcpy(flips, c->flips, sizeof(uint64_t) * (size_t)c->K);
  memcpy(sw_att, c->sw_att, sizeof(uint64_t) * (size_t)c->K);
  memcpy(sw_acc, c->sw_acc, sizeof(uint64_t) * (size_t)c->K);
  memcpy(sw_near, c->sw_near, sizeof(uint64_t) * (size_t)c->K);
}

int64_t orc_check_fields(const orc_chain *c) {
  int64_t bad = 0;
  const int32_t N = c->N;
  for (int32_t w = 0; w < c->K; w++) {
    const int8_t *s = c->s + (size_t)w * N;
    const int32_t *he = c->heff + (size_t)w * N;
    for (int32_t i = 0; i < N; i++) {
      int32_t f = c->h[i], ft = 0;
      for (int32_t e = c->rp[i]; e < c->rp[i + 1]; e++) {
        if (c->two_field && c->ctau[e])
          ft += c->cj[e] * s[c->ci[e]];
        else
          f += c->cj[e] * s[c->ci[e]];
      }
      if (f != he[i]) bad++;
      if (c->two_field && ft != c->htau[(size_t)w * N + i]) bad++;
    }
    if (orc_energy_of(c, w) != c->E[w]) bad++;
    if (c->two_field && orc_bond_of(c, w) != c->B[w]) bad++;
  }
  return bad;
}

void orc_set_spins(orc_chain *c, int32_t w, const int8_t *s) {
  memcpy(c->s + (size_t)w * c->N, s, (size_t)c->N);
  recompute(c, w);
}

void orc_get_bond(const orc_chain *c, int64_t *out) {
  for (int32_t w = 0; w < c->K; w++) out[w] = c->two_field ? c->B[w] : 0;
}
void orc_get_tau_fields(const orc_chain *c, int32_t *out) {
  const size_t n = (size_t)c->K * c->N;
  if (c->two_field)
    memcpy(out, c->htau, sizeof(int32_t) * n);
  else
    memset(out, 0, sizeof(int32_t) * n);
}
