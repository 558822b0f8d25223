/*
 * ising.h -- C ABI of the MI355X (gfx950) parallel-tempering Metropolis library.
 *
 * The operation is the Metropolis sweep of Dickson, Karimi & Hamze, "Importance
 * of Explicit Vectorization for CPU and GPU Software Performance" (2010):
 *   - Ising cost f(s) = -sum_i h_i s_i - sum_{i<j} J_ij s_i s_j, s_i = +-1
 *     (Section 1, equation of f; each undirected edge counted once, so
 *     J > 0 favours aligned spins);
 *   - one sweep visits every spin in ascending index order, draws one uniform
 *     number per spin and flips the spin when the number is below the flip
 *     probability min(1, exp(-beta * dE)), dE = 2 s_i h_eff_i, then updates
 *     what its neighbours need (Figure 1; neighbour data as in Figures 3, 6);
 *   - the uniform numbers come from MT19937 (Section 3, Figure 8), one stream
 *     per walker;
 *   - many walkers run at once under parallel tempering (Section 1): after a
 *     sweep, walkers at neighbouring inverse temperatures exchange their
 *     temperature labels with probability min(1, exp((b_k - b_k+1)(E_k - E_k+1))).
 *   - the systems are layered: many identical copies ("slices") of a small
 *     Ising model, corresponding spins of adjacent slices joined, the last
 *     slice optionally wrapping to the first (Section 3.1); every spin has at
 *     most 8 neighbours (Section 1).
 *
 * Conventions
 *   - Spin (m, q) of a system with S spins per slice and M slices has index
 *     i = m*S + q; the sweep order is ascending i.
 *   - Walker r (global, over all systems in load order) uses uniform
 *     u_n * 2^-32 where u_n is the n-th MT19937 output of its stream; its
 *     initial spin i is +1 iff the top bit of output i is set, so sweep t
 *     (0-based) uses outputs (t+1)*N .. (t+2)*N - 1.
 *   - A flip of spin i with d = s_i * h_eff_i is accepted iff d <= 0 or
 *     u < ceil(2^32 * exp(-2.0 * beta * d)) (IEEE double, beta the walker's
 *     current inverse temperature); the integer threshold is exactly the
 *     comparison u * 2^-32 < exp(-2.0 * beta * d).
 *   - Swap rounds are deterministic even/odd: round number n tries the pairs
 *     (k, k+1) with k = n mod 2, 4, ... in ascending k, one draw of the
 *     system's swap stream per pair, accepted iff delta >= 0 or
 *     u * 2^-32 < exp(delta), delta = (beta_k - beta_k+1) * (E_a - E_b) in
 *     IEEE double, a / b the walkers at slots k / k+1.  Decisions with
 *     |u * 2^-32 - exp(delta)| < 1e-12 are counted per pair (swap_near) and in
 *     total (stats[ISING_STAT_NEAR]).
 *
 * Ownership: every device buffer belongs to the caller (e.g. torch tensors);
 * the library never allocates device memory.  Host arrays passed in are read
 * during the call only.  All calls are asynchronous on `stream` (a
 * hipStream_t, NULL for the default stream) unless stated; device-side
 * failures surface as ISING_E_HIP from a later call.  One stream per graph,
 * no internal locking.  Return codes below; no call aborts the process.
 */
#ifndef ISING_H
#define ISING_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ISING_OK = 0,
  ISING_E_INVAL = -1, /* null pointer, negative count, inconsistent description */
  ISING_E_RANGE = -2, /* outside the supported envelope (sizes, degree, field bound) */
  ISING_E_SIZE = -3,  /* a caller buffer is too small */
  ISING_E_HIP = -4,   /* HIP runtime error; see ising_last_error() */
  ISING_E_STATE = -5  /* call out of order (e.g. a sweep before ising_init_state) */
};

/* Supported envelope. */
#define ISING_MAX_S 512     /* spins per slice (threads per walker) */
#define ISING_MAX_DEG 8     /* in-slice neighbours per spin (tau edges extra, total <= 8) */
#define ISING_MAX_D 63      /* |h_i| + sum_j |J_ij| */
#define ISING_MAX_K 256     /* walkers (= temperature slots) per system */
#define ISING_MT_WORDS 624  /* MT19937 state words */

/* One system (host memory, read during ising_graph_bytes / ising_load_graph).
 * Layered form: an S-spin template with `n_edges` in-slice edges, copied into
 * M slices; spin (m, q) is joined to (m+1, q) with coupling J_tau[q] for
 * m = 0 .. M-2, and for a ring (M >= 3) also (M-1, q) to (0, q).
 * M = 1 describes an arbitrary graph on S spins (J_tau ignored).            */
typedef struct {
  int32_t spins_per_slice; /* S, 1 .. ISING_MAX_S */
  int32_t n_slices;        /* M >= 1 */
  int32_t ring;            /* 0 or 1 (1 needs M >= 3) */
  int32_t n_edges;         /* in-slice template edges */
  const int32_t *edge_u;   /* [n_edges], 0 <= u, v < S, u != v, no duplicates */
  const int32_t *edge_v;
  const int8_t *edge_J;    /* [n_edges] */
  const int8_t *h;         /* [S] */
  const int8_t *J_tau;     /* [S]; may be NULL when M == 1 */
  int32_t n_temps;         /* K >= 1: walkers of this system = temperature slots */
  const double *beta;      /* [K] inverse temperatures of the slots, > 0 */
} ising_system_desc;

typedef struct ising_graph ising_graph; /* opaque; owns host metadata only */

/* Bytes of device memory the packed tables of these systems need. */
int32_t ising_graph_bytes(const ising_system_desc *sys, int32_t n_sys, size_t *dev_bytes);

/* Validate and pack the systems (neighbour rows with J inline, Section 2.2,
 * Figures 5-6; integer thresholds per slot, Section 2.3 result caching), copy
 * the tables into the caller's device buffer `dev_tables` (>= the size from
 * ising_graph_bytes, 256-byte aligned, kept alive while the graph is used)
 * and return a handle.  Synchronous with respect to the host arrays.         */
int32_t ising_load_graph(const ising_system_desc *sys, int32_t n_sys, void *dev_tables,
                         size_t bytes, void *stream, ising_graph **out);
void ising_free_graph(ising_graph *g);

/* Totals of a loaded graph, written to out[0..n-1] in this order:
 *   0 n_sys, 1 walkers R, 2 slots (sum K), 3 spin words (uint32) of all walkers,
 *   4 sum over walkers of N (attempts per sweep), 5 max levels per sweep.   */
int32_t ising_graph_info(const ising_graph *g, int64_t *out, int32_t n);
/* Per walker r: first uint32 word of its bit-packed spins; per system s its
 * slice row length in words (row_words[s]).  Bit q of word
 * spin_word[r] + m*row_words[s] + (q >> 5) ... is bit (q & 31): spin (m, q)
 * of walker r is +1 iff that bit is set.  Host arrays [R] and [n_sys].      */
int32_t ising_spin_layout(const ising_graph *g, int64_t *spin_word, int32_t *row_words);

/* Launch shapes.  Systems with the same template size and kernel variant
 * form a bucket, swept by one launch.  A walker's template columns are spread
 * over `tpw` threads (a power of two up to 64, which keeps a walker inside one
 * wavefront, or a count from 65 to 1024, walkers back to back; a thread visits
 * ceil(S/tpw) <= 8 columns per level, at most 2 when tpw above 64 is not a
 * multiple of 64) and a workgroup holds
 * `walkers_per_group` walkers.  Shapes change speed only: the
 * chain is the same for every shape.  bucket_info writes, in this order:
 *   S, systems, walkers, attempts per sweep, tpw, walkers per group, columns
 *   per thread, workgroup threads, LDS bytes per workgroup, workgroups, ladder
 *   (1 when every workgroup holds whole systems, at most 64 threads per walker,
 *   and the swap state fits: then, when every bucket is a ladder bucket,
 *   ising_sweep runs the swap rounds inside the sweep kernel, one launch per
 *   call; the chain is the same), stream (0 = the caller's; see below), work
 *   (attempts per sweep, or nanoseconds per sweep once autotuned).
 * set_launch returns ISING_E_RANGE for a shape that does not fit (threads,
 * LDS, columns per thread) and leaves the bucket unchanged.
 * With several buckets a sweep forks side streams (default priority) from the
 * caller's stream and joins them before it returns: at most as many streams
 * as the process has hardware queues (GPU_MAX_HW_QUEUES, HIP's default 4),
 * since kernels that share a queue run one after another.  The buckets are
 * enqueued largest first, each onto the stream with the least work so far;
 * the work of a bucket is its attempts per sweep, or its time per sweep once
 * ising_autotune has measured it.                                            */
int32_t ising_n_buckets(const ising_graph *g);
int32_t ising_bucket_info(const ising_graph *g, int32_t bucket, int64_t *out, int32_t n);
int32_t ising_set_launch(ising_graph *g, int32_t bucket, int32_t tpw, int32_t walkers_per_group,
                         void *stream);

/* Device buffers of the chain (caller-owned).  Element counts come from
 * ising_state_sizes; walker r of system s is walker r - first(s) there.    */
typedef struct {
  uint32_t *spins;     /* bit-packed spins, layout per ising_spin_layout */
  uint32_t *mt;        /* [R][624]: walker r's 624 most recent MT words, oldest first */
  int32_t *energy;     /* [R] running cost f(s) */
  int32_t *temp_of;    /* [R] temperature slot (0..K-1 within its system) */
  int32_t *walker_at;  /* [slots] walker (index within its system) at each slot */
  uint32_t *swap_mt;   /* [n_sys][624] swap streams, same window convention */
  uint64_t *flips;     /* [R] accepted flips */
  uint64_t *swap_att;  /* [slots] attempts of pair (k, k+1), at slot index k */
  uint64_t *swap_acc;  /* [slots] acceptances */
  uint64_t *stats;     /* [ISING_N_STATS]: see ising_stats */
  uint64_t *wsteps;    /* [R][2] per walker: wavefront steps with an active spin, with a flip */
  int32_t *bond;       /* [R] tau-bond sum B = sum over tau edges of J_tau s s' (kept current by
                          ising_init_state, ising_refresh_energies and two-field sweeps) */
  uint64_t *swap_near; /* [slots] decisions of pair (k, k+1), at slot index k, taken with
                          |u 2^-32 - exp(delta)| < 1e-12 (delta < 0): the FP64 step's
                          near-threshold count, per pair */
  int64_t sweeps;      /* host: sweeps done (set by the library) */
  int64_t rounds;      /* host: swap rounds done */
} ising_state;

enum {
  ISING_STAT_NEAR = 0,       /* swap decisions within 1e-12 of the threshold (sum of swap_near) */
  ISING_STAT_WAVE_STEPS = 1, /* wavefront steps (64 lanes, one level) with an active spin */
  ISING_STAT_WAVE_FLIP = 2,  /* of those, steps in which some lane flipped (the analogue of
                                the paper's probability of waiting for a flip, Section 4) */
  ISING_STAT_ATTEMPTS = 3,   /* spin-flip attempts */
  ISING_STAT_FLIPS = 4,      /* accepted flips */
  ISING_STAT_SWAP_ATT = 5,   /* swap attempts */
  ISING_STAT_SWAP_ACC = 6,   /* accepted swaps */
  ISING_N_STATS = 8
};

/* Element counts: [spins, mt, energy, temp_of, walker_at, swap_mt, flips,
 * swap_att, swap_acc, stats, wsteps, bond, swap_near]. */
#define ISING_STATE_NARRAYS 13
int32_t ising_state_sizes(const ising_graph *g, int64_t *counts);

/* Seed every walker stream (MT19937 init_genrand with walker_seeds[r]) and
 * swap stream (swap_seeds[s]), draw the initial spins, compute energies,
 * put walker j of each system at slot j, clear the counters.  Host arrays. */
int32_t ising_init_state(const ising_graph *g, ising_state *st, const uint32_t *walker_seeds,
                         const uint32_t *swap_seeds, void *stream);

/* n_sweeps sweeps of every walker (Figure 1: spins in ascending index order,
 * one uniform each, a flip when it falls below the flip probability, the
 * neighbours' local fields then current as in Figures 3 and 6); after each
 * sweep whose running count is a multiple of swap_every (> 0; 0 = never) one
 * swap round of every system (replica exchange, Section 1).  Long calls run as
 * several launches whose 32-bit per-launch counters cannot wrap (and of at
 * most n sweeps when the environment sets ISING_LAUNCH_SWEEPS_MAX=n); the
 * chain is the same.  e_series (device, nullable): [n_sweeps][slots] energy of the
 * walker at each slot after each sweep and its swap round.  ISING_E_INVAL for
 * negative counts, ISING_E_STATE before ising_init_state.                    */
int32_t ising_sweep(const ising_graph *g, ising_state *st, int32_t n_sweeps, int32_t swap_every,
                    int32_t *e_series, void *stream);

/* Captured sweep loops.  ising_capture records, on a non-default `stream`,
 * exactly the launches ising_sweep(g, st, n_sweeps, swap_every, e_series)
 * would make from the state's current counters (nothing runs and the state is
 * unchanged) and instantiates them as one HIP graph.  ising_replay_launch
 * enqueues the graph and advances st->sweeps / st->rounds; it returns
 * ISING_E_STATE unless `st` has the captured buffers and the same swap phase
 * (rounds mod 2, sweeps mod swap_every).  e_series, if given, is rewritten by
 * every replay.  The handle owns only the HIP graph objects.                 */
typedef struct ising_replay ising_replay;
int32_t ising_capture(const ising_graph *g, const ising_state *st, int32_t n_sweeps, int32_t swap_every,
                      int32_t *e_series, void *stream, ising_replay **out);
int32_t ising_replay_launch(ising_replay *r, ising_state *st, void *stream);
void ising_replay_free(ising_replay *r);

/* Autotuner: for every bucket, time each admissible launch shape (tpw a power
 * of two from 8 to 1024, or above 64 the template size S, ceil(S/2) and their
 * multiples of 64; walkers per group 1, 2, 4 .. 32) with HIP events over `reps`
 * single-sweep launches on `scratch` (an initialised state of this graph whose
 * chain it advances), then keep the fastest shape.  Optionally writes one row
 * {bucket, tpw, walkers_per_group, nanoseconds per sweep} per trial to
 * report[report_rows][4].  A ladder bucket only tries ladder shapes (its
 * swap rounds stay inside the kernel); when every bucket is one, each timed
 * launch runs 16 sweeps with a swap round after each, as ising_sweep runs
 * them, and the report gives the time per sweep.  The kept shapes' times per
 * sweep then spread the buckets over the sweep's streams.  Returns the number
 * of rows written (>= 0) or an error code.  Synchronous.                     */
int32_t ising_autotune(ising_graph *g, ising_state *scratch, int32_t reps, void *stream, int64_t *report,
                       int32_t report_rows);

/* One swap round of every system with the given parity (0: pairs (0,1),(2,3)..;
 * 1: (1,2),(3,4)..): parallel tempering (Section 1) with the rule and draw
 * order stated at the top of this file, FP64 on the device, near-threshold
 * decisions counted in st->swap_near.  Does not change st->rounds.           */
int32_t pt_swap(const ising_graph *g, ising_state *st, int32_t parity, void *stream);

/* e_row[slots] (device) = running energy of the walker at each slot. */
int32_t ising_record_slots(const ising_graph *g, const ising_state *st, int32_t *e_row, void *stream);

/* Totals over all walkers into host out[ISING_N_STATS] (reduces the per-walker
 * counters on the device; synchronises `stream`).                           */
int32_t ising_stats(const ising_graph *g, const ising_state *st, uint64_t *out, void *stream);

/* Observables per walker into device int32 obs[R][6]: cost recomputed from the
 * spins (the cost function f of Section 1), magnetisation sum_i s_i, running
 * cost, temperature slot, tau-bond sum B recomputed from the spins (the tau
 * edges of the layered models, Section 3.1), running B.  obs is caller-owned,
 * R = walkers of the graph; ISING_E_INVAL for a NULL pointer.                */
int32_t ising_observables(const ising_graph *g, const ising_state *st, int32_t *obs, void *stream);
/* Recompute every walker's running cost and tau-bond sum from its spins. */
int32_t ising_refresh_energies(const ising_graph *g, ising_state *st, void *stream);

/* ---- two-field form --------------------------------------------------------
 * The paper's QMC models keep two local fields per spin (Sections 2.1-2.2,
 * Figures 2, 3 and 6): h_eff_space over the in-slice edges (with h) and
 * h_eff_tau over the two tau edges, and the two are weighted differently.  In
 * this form slot k carries weights (a_k, c_k) and weighs a walker's state s by
 * exp(-a_k E_sp(s) + c_k B(s)), E_sp = -sum h s - sum over in-slice edges of
 * J s s' (all slices), B = sum over tau edges of J_tau s s'; so E = E_sp - B.
 *   - A flip of spin i with d_sp = s_i h_eff_space_i and d_t = s_i h_eff_tau_i
 *     changes the log weight by -2x, x = a d_sp + c d_t (IEEE double, the two
 *     products rounded separately); it is accepted iff x <= 0 or
 *     u < ceil(2^32 exp(-2x)), i.e. u * 2^-32 < exp(-2x).  Under
 *     ISING_ACCEPT_FAST / _ACCURATE the probability is the Figure 7
 *     approximation at -2x rounded to FP32, as for the one-field test.
 *   - Swap rounds: delta = (a_k - a_k+1)(E_sp,a - E_sp,b) - (c_k - c_k+1)(B_a - B_b)
 *     (IEEE double, products rounded separately), accepted iff delta >= 0 or
 *     u * 2^-32 < exp(delta); one draw per pair as before.
 *   - The running cost E stays the full cost f(s); st->bond holds B.
 * Thresholds are precomputed per slot over (d_sp, d_t), so the sweep makes the
 * same integer comparison as the one-field form.  Supported for grids of K4,4
 * cells with rows of (2 ds + 1)(2 dt + 1) <= 1024 words (ds = max |h| +
 * sum |J in-slice| of a spin, dt = max sum |J_tau|); swaps then run in their
 * own kernel; cell moves are refused while the form is on.
 *
 * ising_set_two_field: a[slots], c[slots] (host) switch the graph to the form
 * (both NULL: back to the one-field form).  Needs 2(|a| ds + |c| dt) <= 700 per
 * slot (ISING_E_RANGE otherwise).  Launch shapes return to their defaults.
 * States whose B may be stale (after one-field sweeps or cell moves) need
 * ising_refresh_energies first.  Synchronises `stream`.                      */
int32_t ising_set_two_field(ising_graph *g, const double *a, const double *c, void *stream);
/* Host only: the two-field threshold row of one slot, entry
 * (d_sp + ds)(2 dt + 1) + d_t + dt for |d_sp| <= ds, |d_t| <= dt;
 * 0xffffffff where x <= 0. */
int32_t ising_two_field_row(double a, double c, int32_t ds, int32_t dt, int32_t kind, uint32_t *thr);
/* Host only: Suzuki-Trotter weights of a transverse field gamma over M slices
 * (a reading: the paper does not print them): a_k = beta_k / M and
 * c_k = -1/2 ln tanh(beta_k gamma / M), so that neighbouring copies of a spin
 * carry the transfer factor exp(c s s').                                     */
int32_t ising_trotter_weights(const double *beta, int32_t n, int32_t M, double gamma, double *a, double *c);

/* ---- layer-pair order (the paper's GPU layout) ------------------------------
 * Section 3.2, Figure 12c: the slices of a model are grouped in pairs
 * (2t, 2t+1) that are interlaced over GPU threads; each thread has its own
 * random number generator and first attempts the spins of its even slice,
 * then, after all threads are done, those of its odd slice.  This is a
 * different chain from the sequential sweep above, built as its own mode:
 *   - walker r has M/2 MT19937 generators, lane (pl0(r) + t) for pair t, where
 *     lanes are numbered walker by walker in load order (system s, walker j of
 *     it: lanes sum_{s'<s} K_s' M_s'/2 + j M_s/2 + t); generator lane l is
 *     seeded with init_genrand(pair_seeds[l]);
 *   - initial spin (2t + j, q) is +1 iff the top bit of output j S + q of
 *     generator t is set;
 *   - a sweep visits every even slice, spins in ascending q, one output of the
 *     slice's pair generator per spin, then every odd slice the same way
 *     (slices of one parity share no edge, so they run side by side); the flip
 *     test, thresholds, acceptance variants, energies and swap rounds are those
 *     of the one-field form above;
 *   - after n outputs, word x_{n+i} (i < 624) of a generator is in its slot
 *     k = (n + i) mod 624; slot k of lane l is element
 *     ((k / 4) * lanes + l) * 4 + k % 4 of pair_mt (quads of slots, lanes
 *     side by side: [156][lanes][4]; device, caller owned, 16-byte aligned,
 *     ising_pairs_words elements).
 * Needs every system to be a grid of K4,4 cells (so S is a multiple of 8),
 * with an even number of slices, K * M/2 <= 1024 and its walkers' spins in LDS
 * (ISING_E_RANGE otherwise), and the two-field form off.  One workgroup sweeps a whole system and runs its swap rounds, so one
 * launch (per template class) covers any number of sweeps.  The state's walker
 * streams (st->mt) are not used.                                              */
int32_t ising_pairs_words(const ising_graph *g, int64_t *words);
/* Seed the pair generators (host pair_seeds[lanes]) and swap streams (host
 * swap_seeds[n_sys]), draw the initial spins, compute energies, put walker j
 * of each system at slot j, clear the counters.                              */
int32_t ising_pairs_init(const ising_graph *g, ising_state *st, uint32_t *pair_mt, const uint32_t *pair_seeds,
                         const uint32_t *swap_seeds, void *stream);
/* n_sweeps layer-pair sweeps of every walker, with a swap round after each
 * sweep whose running count is a multiple of swap_every (> 0; 0 = never).   */
int32_t ising_pairs_sweep(const ising_graph *g, ising_state *st, uint32_t *pair_mt, int32_t n_sweeps,
                          int32_t swap_every, void *stream);

/* ---- learned cell proposal --------------------------------------------------
 * An extension of the method (the paper has no learned part): a unit cell of
 * 8 spins of one slice is re-proposed jointly by a 17 -> 128 -> 128 -> 8 ReLU
 * network q(s'|b, beta) given its boundary fields b_k = h_k + sum over
 * neighbours j outside the cell of J_kj s_j, with input
 * [0 x 8, b/8, beta]; outputs are 8 independent Bernoulli logits (spin +1).
 * Moves are accepted with the exact Metropolis-Hastings probability
 * min(1, exp(-beta dE) q(s)/q(s')), dE the integer change of the cost
 * function, so the target distribution is unchanged.  Products run on BF16
 * matrix cores with FP32 sums; the parameters are FP32.
 * Parameter layout (ISING_MLP_PARAMS floats): W1[128][17], b1[128],
 * W2[128][128], b2[128], W3[8][128], b3[8].                                   */
#define ISING_MLP_PARAMS 19848
#define ISING_MLP_PACKED 43008 /* uint16 words of the packed BF16 copies */
#define ISING_MLP_PARTS 128    /* partial gradients of one step (one per workgroup, at most) */
typedef struct {
  float *w;       /* [ISING_MLP_PARAMS] FP32 master weights (device) */
  float *m, *v;   /* [ISING_MLP_PARAMS] Adam moments (device) */
  float *grad;    /* [ISING_MLP_PARAMS] gradient (device, written by ising_mlp_grad) */
  float *part;    /* [ISING_MLP_PARTS][ISING_MLP_PARAMS + 1] scratch of ising_mlp_grad (device) */
  uint16_t *wb;   /* [ISING_MLP_PACKED] BF16 copies read by the kernels (device) */
  int64_t step;   /* host: Adam steps done */
} ising_mlp;

/* Refresh net->wb from net->w (after the caller writes w). */
int32_t ising_mlp_pack(ising_mlp *net, void *stream);
/* logits[n][8] (device) of inputs x[n][17] (device FP32). */
int32_t ising_mlp_forward(const ising_mlp *net, const float *x, int32_t n, float *logits, void *stream);
/* net->grad = gradient of mean_r -log q(y_r | x_r), y[r] (device bytes) bit k
 * set when cell spin k is +1; *loss (device, nullable) = that mean.  Up to
 * ISING_MLP_PARTS workgroups each take every P-th 32-row tile and write a
 * partial gradient to net->part; the partials are then added in order, so the
 * result depends only on the batch (bitwise reproducible). */
int32_t ising_mlp_grad(const ising_mlp *net, const float *x, const uint8_t *y, int32_t n, float *loss,
                       void *stream);
/* The same gradient step for callers that cannot allocate device memory or
 * pass a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): net->part is not used (it may be NULL);
 * the partial gradients go to a fixed array of the library, ISING_MLP_PARTS x
 * (ISING_MLP_PARAMS + 1) floats (10,162,688 bytes) per GPU, held until the
 * process ends.  Every batch size needs at most those rows (ISING_E_SIZE
 * otherwise).  The result equals ising_mlp_grad's bit for bit.  Nothing is
 * allocated; calls that overlap on one GPU share the array and race. */
int32_t ising_mlp_grad_noalloc(const ising_mlp *net, const float *x, const uint8_t *y, int32_t n, float *loss,
                               void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with net->grad, then repack. */
int32_t ising_mlp_adam(ising_mlp *net, float lr, void *stream);

/* Cells: systems whose template is a grid of L x L 8-spin cells (spins
 * (y*L + x)*8 + 0..7 of a slice form cell (y, x), every spin joined to the 4
 * spins of the other half of its cell, and in-slice edges between cells only
 * join grid neighbours).  Cell (m, y, x) of a walker has index (m*L + y)*L + x.
 * Other systems are left out of cell moves.
 *
 * Training rows: row i is cell number (offset + i*stride) mod (all cells of
 * all walkers, walker-major): x[i][17] (device FP32) its network input, y[i]
 * its 8 spins (bit k set when spin k is +1).                                  */
int32_t ising_collect_cells(const ising_graph *g, const ising_state *st, int64_t stride, int64_t offset,
                            int32_t n, float *x, uint8_t *y, void *stream);
/* One pass of cell moves over every walker: the colour classes of cells in
 * order (cells of one class share no edge and move at once); each cell gets a
 * joint proposal from the network and the Metropolis-Hastings test.  Uniforms:
 * Philox4x32-10 with key (key mod 2^32, key div 2^32) and counters (cell,
 * walker, pass_index, j) for blocks j = 0, 1, 2: the eight words of blocks 0
 * and 1 are the proposal uniforms, word 0 of block 2 the acceptance uniform
 * (uniform = word * 2^-32); 0 <= pass_index < 2^32, else ISING_E_RANGE.  Energies
 * are kept exact.  One launch per colour class: boundary fields, network and
 * test run in one kernel, with no device memory besides the state and the
 * network.  moves (device, nullable) [R][2] += proposals, acceptances.      */
int32_t ising_propose_cells(const ising_graph *g, ising_state *st, const ising_mlp *net, uint64_t key,
                            int64_t pass_index, uint64_t *moves, void *stream);

/* One pass of exact heat-bath cell moves (the non-learned control of the
 * learned proposal), same cells and colour classes: each cell is redrawn from
 * its conditional Boltzmann law exp(-beta E_c) given the boundary fields
 * (cost function of Section 1, restricted to the cell).  The cell is
 * bipartite, so the left half (spins 0..3) is drawn from its marginal over 16
 * states, log weight beta sum_k b_k s_k + sum_r log(2 cosh(beta h_r)),
 * h_r = b_r + sum_k J_kr s_k, and then each right spin r is +1 with
 * probability sigmoid(2 beta h_r).  Uniforms: Philox4x32-10 with key (key mod
 * 2^32, key div 2^32), counters (cell, walker, pass_index, j), j = 0, 1: word
 * 0 picks the left state (the first, in index order with bit k = spin k, whose
 * cumulative weight exceeds u * 2^-32 times the total), words 1..4 the right
 * spins (+1 iff u * 2^-32 < the probability).  FP32 weights.  moves (device,
 * nullable) [R][2] += cells visited, cells changed.                          */
int32_t ising_heatbath_cells(const ising_graph *g, ising_state *st, uint64_t key, int64_t pass_index,
                             uint64_t *moves, void *stream);

/* ---- host-only helpers (no device work; usable without a GPU) ------------ */

/* thr[d] = ceil(2^32 * exp(-2.0 * beta * d)) - 1 for d = 1..dmax, thr[0] =
 * 0xffffffff: a flip with d <= 0 or u <= thr[d] is accepted.  ISING_E_RANGE
 * when 2 beta dmax > 700: there exp(-2 beta d) leaves the normal doubles and
 * no uint32 threshold expresses "never" (the same bound as the two-field
 * rows).  ising_load_graph applies it with each system's own largest
 * |h_i| + sum_j |J_ij|, so a ladder whose coldest beta exceeds
 * 350 / that bound is rejected.                                              */
int32_t ising_threshold_row(double beta, int32_t dmax, uint32_t *thr);
/* Level offsets of the exact parallel schedule of one template: f[q] is the
 * length of the longest chain of in-slice edges leading to q in ascending
 * index order; *depth = max f + 1.                                           */
int32_t ising_level_offsets(const ising_system_desc *sys, int32_t *f, int32_t *depth);

/* Flip-test variants.  ISING_ACCEPT_EXACT (the default): thresholds from the
 * exact exp, as above.  ISING_ACCEPT_FAST / ISING_ACCEPT_ACCURATE: the flip
 * probability is the paper's approximation of e^x (Section 2.4, Figure 7), in
 * FP32: x = -2 beta d rounded to FP32, times 2^23 log2 e (fast) or 2^25 log2 e
 * (accurate), rounded to the nearest integer, plus 0x3F800000, read as a
 * float, times 2 ln^2 2; the accurate form then takes the 4th root (two IEEE
 * square roots).  Below the valid range (x < -126 ln 2, resp. -31.5 ln 2) the
 * probability is 0.  Threshold t = ceil(2^32 p) - 1, clamped to
 * [0, 2^32 - 1]: u <= t is u * 2^-32 < p, except that p = 0 still passes u = 0
 * (one draw in 2^32).  These chains sample a slightly different law than the
 * Boltzmann one; they reproduce the paper's optimised variants.           */
enum { ISING_ACCEPT_EXACT = 0, ISING_ACCEPT_FAST = 1, ISING_ACCEPT_ACCURATE = 2 };
/* Host only: the threshold row of one inverse temperature for a variant. */
int32_t ising_acceptance_row(double beta, int32_t dmax, int32_t kind, uint32_t *thr);
/* Rewrite every threshold row of the graph for a variant (host -> device copy
 * on `stream`, then synchronises it); later sweeps use it. */
int32_t ising_set_acceptance(ising_graph *g, int32_t kind, void *stream);

/* Last error message of this thread ("" if none). */
const char *ising_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ISING_H */
