/*
 * Oracle for the parallel-tempering Metropolis path -- TEST INFRASTRUCTURE.
 *
 * A plain, slow, obviously correct CPU implementation of what the GPU library
 * computes.  Only the tests, the smoke check and the benchmark's CPU baseline
 * may load it; the product path never does.  It shares no code, header, table
 * or constant generator with the HIP library.
 *
 * Method (Dickson, Karimi & Hamze, "Importance of Explicit Vectorization for
 * CPU and GPU Software Performance", 2010):
 *   - Ising cost f(s) = -sum_i h_i s_i - sum_{edges} J_ij s_i s_j   (Sec. 1)
 *   - Metropolis sweep in ascending spin order, one uniform per spin, flip
 *     when it falls below the flip probability, then update the local data of
 *     the neighbours (Fig. 1; neighbour update as in Figs. 3 and 6)
 *   - MT19937 random numbers (Sec. 3, Fig. 8)
 *   - parallel tempering over a ladder of inverse temperatures (Sec. 1)
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* MT19937 with a circular window of the last 624 generated words. */
typedef struct orc_mt {
  uint32_t x[624];
  int64_t n; /* outputs delivered so far */
} orc_mt;

void orc_mt_seed(orc_mt *g, uint32_t seed);
uint32_t orc_mt_next(orc_mt *g);
/* x_{n} .. x_{n+623}: the 624 most recent words, oldest first. */
void orc_mt_window(const orc_mt *g, uint32_t *out624);
/* outputs [skip, skip+n) of the stream seeded with `seed`. */
void orc_mt_stream(uint32_t seed, int64_t skip, int64_t n, uint32_t *out);

typedef struct orc_chain orc_chain;

/* One system: N spins, nE undirected edges (u[e], v[e], J[e]), fields h[N];
 * K walkers, walker w starts at temperature slot w; walker w's stream is
 * seeded walker_seed[w], the swap stream swap_seed.  Returns NULL on bad input. */
orc_chain *orc_new(int32_t N, int32_t nE, const int32_t *u, const int32_t *v, const int8_t *J,
                   const int8_t *h, int32_t K, const double *beta, const uint32_t *walker_seed,
                   uint32_t swap_seed);
void orc_free(orc_chain *c);

/* n sweeps; after every sweep whose running count is a multiple of
 * swap_every (>0) one round of neighbour swaps, parity = rounds done mod 2.
 * Optional records after each sweep (and its swap round), per slot k:
 *   e_series[t*K + k]      energy of the walker at slot k
 *   bits_series[t*K + k]   its spins as bits (bit i = s_i == +1), N <= 32
 *   slot_spin_sum[k*N + i] += s_i of the walker at slot k                     */
void orc_sweeps(orc_chain *c, int32_t n, int32_t swap_every, int32_t *e_series,
                uint32_t *bits_series, int64_t *slot_spin_sum);
void orc_swap_round(orc_chain *c, int32_t parity);
/* The same n sweeps on many independent chains, spread over threads. */
void orc_run_many(int32_t n_chains, orc_chain **chains, int32_t n, int32_t swap_every,
                  int32_t n_threads);

int32_t orc_N(const orc_chain *c);
int32_t orc_K(const orc_chain *c);
int64_t orc_sweeps_done(const orc_chain *c);
int64_t orc_rounds_done(const orc_chain *c);
void orc_get_spins(const orc_chain *c, int8_t *out);   /* [K][N] +-1 */
void orc_get_fields(const orc_chain *c, int32_t *out); /* [K][N] h_eff */
void orc_get_energy(const orc_chain *c, int64_t *out); /* [K] running energy */
void orc_get_labels(const orc_chain *c, int32_t *temp_of, int32_t *walker_at);
void orc_get_mt(const orc_chain *c, uint32_t *win /*[K][624]*/, int64_t *used /*[K]*/);
void orc_get_swap_mt(const orc_chain *c, uint32_t *win624, int64_t *used);
/* Per walker: accepted flips.  Per pair (k, k+1), at index k: swap attempts,
 * acceptances, and decisions with |u 2^-32 - exp(Delta)| < 1e-12 (Delta < 0). */
void orc_get_counters(const orc_chain *c, uint64_t *flips /*[K]*/, uint64_t *sw_att /*[K]*/,
                      uint64_t *sw_acc /*[K]*/, uint64_t *sw_near /*[K]*/);
/* Energy of walker w's spins by the cost function itself. */
int64_t orc_energy_of(const orc_chain *c, int32_t w);
/* Number of running fields / energies that differ from a recomputation. */
int64_t orc_check_fields(const orc_chain *c);
/* Overwrite a walker's spins (fields and energy are recomputed). */
void orc_set_spins(orc_chain *c, int32_t w, const int8_t *s);

/* Flip-test variants: the exact exp, or the paper's approximations of e^x
 * (Sec. 2.4, Fig. 7).  New chains use the exact one. */
enum { ORC_ACCEPT_EXACT = 0, ORC_ACCEPT_FAST = 1, ORC_ACCEPT_ACCURATE = 2 };
void orc_set_acceptance(orc_chain *c, int32_t kind);
float orc_exp_approx(float x, int32_t kind);
uint32_t orc_approx_threshold(double beta, int32_t d, int32_t kind);

/* Two-field form (Sec. 2.1-2.2): edges flagged in is_tau[nE] (orc_new's edge
 * order) feed a separate tau field; slot k weighs a state by
 * exp(-a[k] E_sp + c[k] B), E_sp = cost of h and the other edges, B = sum
 * over tau edges of J s s'.  Recomputes the fields and B; returns 0, or -1 on
 * bad input.  orc_get_fields then returns the in-slice field (with h). */
int32_t orc_set_two_field(orc_chain *c, const uint8_t *is_tau, int32_t nE, const double *a,
                          const double *cw);
uint32_t orc_approx_threshold_x(double x, int32_t kind);
int64_t orc_bond_of(const orc_chain *c, int32_t w);
void orc_get_bond(const orc_chain *c, int64_t *out);        /* [K] running B */
void orc_get_tau_fields(const orc_chain *c, int32_t *out);  /* [K][N] */

/* Layer-pair order (Sec. 3.2, Fig. 12c): for a layered system of M (even)
 * slices of S spins (spin m*S + q), walker w's pair t = slices (2t, 2t+1)
 * draws from its own generator, seeded pair_seed[w*(M/2) + t]; a sweep visits
 * the even slices, then the odd ones, each in index order.  Redraws the
 * initial spins from the pair generators.  Returns 0, or -1 on bad input. */
int32_t orc_set_pairs(orc_chain *c, int32_t S, int32_t M, const uint32_t *pair_seed);
void orc_get_pair_mt(const orc_chain *c, uint32_t *win /*[K*M/2][624]*/, int64_t *used);

#ifdef __cplusplus
}
#endif
#endif
