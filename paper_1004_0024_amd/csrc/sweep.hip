// Sweep kernel: the sequential-order Metropolis sweep (Figure 1 of Dickson,
// Karimi & Hamze) run exactly, spin for spin, by many threads per walker.
//
// Exact parallel schedule.  In a sweep spin i reads its neighbours j < i as
// already updated in this sweep and j > i as left by the previous sweep.  For a
// layered system (an S-spin template copied into M slices, tau edges between
// slice m and m+1, Section 3.1) give template spin q the offset f(q): the
// length of the longest chain of in-slice edges q1 < q2 < ... < q in index
// order.  Spin (m, q) then runs at level m + f(q).  Every edge i < j has
// level(i) < level(j) (in-slice: f grows along the edge; tau: m grows; the
// wrap edge (0,q)-(M-1,q) joins levels f and M-1+f), so processing the levels
// in order, each level in parallel, reproduces the sequential sweep bit for
// bit.  A template column q of a walker visits its M spins at levels
// f(q) .. f(q)+M-1; a sweep takes M + F - 1 levels, F = max f + 1.  This is
// the paper's interlacing of layers over threads (Section 3.2, Figure 12c)
// with a skew that keeps the sequential order instead of an even/odd
// reordering.
//
// Work split: a walker has TPW threads; thread t owns the columns at lane
// positions c*TPW + t, c < CPT, and visits them one after another inside a
// level (independent attempts, so their latencies overlap).  Lane positions
// hold the columns in order of their level offset, so the columns of a
// wavefront start (and end) within few levels of each other.  TPW is a power of
// two up to 64, or any count above 64.  When TPW <= 64 a walker lives inside
// one wavefront and a level ends with a wavefront fence instead of a workgroup
// barrier; above 64 the walkers of a workgroup lie back to back, so with TPW
// not a multiple of 64 a wavefront can hold the end of one walker and the
// start of the next (the SHARED instantiations, at most two columns per
// thread).
//
// Data in LDS for the whole launch, per walker:
//  - spins, one bit each, slice rows of RS words (RS odd when > 1, so rows of
//    different slices fall in different LDS banks); on a ring, a halo row in
//    front holds a copy of the last slice and one behind a copy of the first,
//    so the tau neighbours of every slice are the rows just before and after;
//  - the MT19937 generator ring: word n (counted from the launch's first
//    window word) in slot (n + delta) mod Zg, chunks of S words aligned to
//    slot multiples of S, with a copy of the top kMtN slots in front of slot 0
//    so the look-back reads (624, 623 and 227 words back) never wrap;
//  - one uniform queue per template column: chunk g (the uniforms of slice
//    m = g mod M of sweep g / M) is generated one level before its first
//    consumer and each word is also copied to the queue of its column, slot
//    g mod depth, where it waits until the column reaches that slice (slot k
//    of a queue is 64 words after slot k - 1, so a queue sits in one bank and
//    the 64 columns of a wavefront use 64 different banks);
//  - the walker's threshold row, entry kThrZero + d = ceil(2^32 exp(-2 beta d))
//    - 1 (all ones for d <= 0), or in the two-field form the row of its slot
//    over (d_sp, d_t).
// Two-field form (the QMC models' separate fields, Sections 2.1-2.2): the
// in-slice part of the field (with h) and the tau part are kept apart, d_sp =
// s h_sp and d_t = s h_tau, and the threshold is looked up at the pair; the
// walker also tracks its tau-bond sum B, which changes by -2 d_t on a flip.
// The local field of a spin is pulled from its neighbours' bits when the spin
// is visited (no field array, no conflicting neighbour updates).  For cell
// templates (K4,4 unit cells) the four in-cell neighbours are the other nibble
// of the spin's own byte, summed with one 4-way byte dot product.
#include "internal.h"
#include "mt19937.h"
#include "swap_round.h"

namespace ising {

template <bool WS>
__device__ __forceinline__ void level_sync() {
  if (WS) {
    // A walker's threads are one wavefront: its LDS operations execute in
    // order, so only the compiler must not move them across the level.
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

template <int NX, bool CELL, bool RING, int CPT, bool WS, bool LADDER, bool TF, bool SHARED>
__global__ void __launch_bounds__(1024) sweep_kernel(DevTables T, DevState St, int32_t tile0, int32_t G,
                                                     int32_t TPW, int32_t PW, int32_t n_sweeps,
                                                     int32_t init_mode, LadderArgs la) {
  extern __shared__ uint32_t lds[];
  const Tile tile = T.tiles[tile0 + blockIdx.x];
  const SysInfo sy = T.sys[tile.sys];
  const int S = sy.S, M = sy.M, RS = sy.RS, WW = sy.WW, FW = sy.fifo_words;
  const int F = init_mode ? 1 : sy.F;
  const int Zg = gen_ring_words(S);
  const int ZP = Zg + kMtN;
  const int nw = tile.nw;
  const int tid = threadIdx.x, nthr = blockDim.x;

  // walker slot layout: [shadow | generator ring][queues][halo row, spins, halo row][thr][acc]
  auto wbase = [&](int w) { return lds + w * PW; };
  // body(w, j) for every word j < per of every walker w of the tile, spread
  // over the workgroup; a workgroup of one walker needs no division
  auto each_word = [&](int per, auto &&body) {
    if (nw == 1) {
      for (int j = tid; j < per; j += nthr) body(0, j);
    } else {
      for (int i = tid; i < nw * per; i += nthr) {
        const int w = i / per;
        body(w, i - w * per);
      }
    }
  };

  const int delta = (S - (kMtN % S)) % S;  // chunk-aligned slots
  const int kg = Zg / S;
  const int c0 = (kMtN + delta) / S;       // slot chunk of chunk 0 (= kg - 1)
  const int zs = Zg - kMtN;                // slots >= zs also live in the shadow

  // ---- load the walkers' state ----
  each_word(kMtN, [&](int w, int j) {
    const int r = sy.walker0 + tile.w0 + w;
    const uint32_t v = St.mt[(size_t)r * kMtN + j];
    uint32_t *g = wbase(w) + kMtN;
    const int x = j + delta;
    g[x] = v;
    if (x >= zs) g[x - Zg] = v;
  });
  const int SWW = WW + 2 * RS;  // spin rows with the two halo rows
  const int TRW = TF ? T.qrow : kThrRow;  // threshold row words
  constexpr int SG = TF ? 1 : -1;         // sign of the accumulated field
  constexpr int NACC = TF ? 5 : 4;        // reduction words
  each_word(SWW, [&](int w, int j) {
    int src = j - RS;  // halo rows: copies of the last and the first slice (ring), else zero
    if (src < 0) src = RING ? src + WW : -1;
    else if (src >= WW) src = RING ? src - WW : -1;
    wbase(w)[ZP + FW + j] =
        (init_mode || src < 0) ? 0u : St.spins[sy.spin_word0 + (size_t)(tile.w0 + w) * WW + src];
  });
  if (!init_mode) {
    const uint32_t *rows = TF ? T.qthr : T.thr;
    each_word(TRW, [&](int w, int j) {
      const int slot = St.temp_of[sy.walker0 + tile.w0 + w];
      wbase(w)[ZP + FW + SWW + j] = rows[(size_t)(sy.thr0 + slot) * TRW + j];
    });
  }
  // reduction words: running energy (the walker's cost, so a swap round in the
  // launch can read it), flips, wavefront steps, wavefront steps with a flip,
  // and in the two-field form the running tau-bond sum
  for (int i = tid; i < nw * NACC; i += nthr) {
    const int w = i / NACC, j = i - w * NACC;
    const int r = sy.walker0 + tile.w0 + w;
    uint32_t v = 0u;
    if (!init_mode && j == 0) v = (uint32_t)St.energy[r];
    if (TF && !init_mode && j == 4) v = (uint32_t)St.bond[r];
    wbase(w)[ZP + FW + SWW + TRW + j] = v;
  }
  // ladder tiles (the whole system in this workgroup): swap state in LDS,
  // beta of this thread's pair in registers
  const bool ladder = LADDER && la.swap_every > 0 && !init_mode;
  const LadderLds L = ladder_lds(lds + G * PW);
  PairBeta pb{0.0, 0.0, 0.0};
  if (ladder) {
    ladder_load(St, sy, tile.sys, tid, nthr, L);
    pb = pair_beta(T, sy, tid);
  }

  // ---- this thread's walker and columns ----
  const int gw = tid / TPW, t = tid - gw * TPW;
  const bool live = gw < nw;
  uint32_t *wb = wbase(live ? gw : 0);
  uint32_t *gring = wb + kMtN;  // logical slot 0
  uint32_t *fq = wb + ZP;
  uint32_t *sp = fq + FW + RS;  // row 0 (halo rows at sp - RS and sp + WW)
  const uint32_t *thw = sp + WW + RS;
  int32_t *acc = (int32_t *)(thw + TRW);
  const int qwt = TF ? T.qwt : 0, qoff = TF ? T.qoff : 0;

  int qo[CPT], qb[CPT], base[CPT], jt[CPT], f[CPT], jpack[CPT], fb[CPT], fmask[CPT];
  int xoff[CPT][NX > 0 ? NX : 1], xbit[CPT][NX > 0 ? NX : 1], xj2[CPT][NX > 0 ? NX : 1];
  bool col[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int pos = c * TPW + t;
    col[c] = live && pos < S;
    const int qq0 = col[c] ? (int)T.lanes[sy.tmpl0 + pos] : 0;
    qo[c] = qq0 >> 5;
    qb[c] = qq0 & 31;
    const TmplSpin ts = T.tmpl[sy.tmpl0 + qq0];
    int sumJ = 0;
    if (CELL) {
#pragma unroll
      for (int j = 0; j < 4; ++j) sumJ += ts.J[j];
      uint32_t jp = 0;  // the partners' 2J bytes, times SG
#pragma unroll
      for (int j = 0; j < 4; ++j) jp |= (uint32_t)(uint8_t)(int8_t)(SG * (int)(int8_t)(ts.jpack >> (8 * j))) << (8 * j);
      jpack[c] = (int)jp;
    } else {
      jpack[c] = 0;
    }
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const int qq = ts.nbr[(CELL ? 4 : 0) + j];
      xoff[c][j] = (qq >> 5) - qo[c];
      xbit[c][j] = qq & 31;
      xj2[c][j] = SG * 2 * (int)ts.J[(CELL ? 4 : 0) + j];
      sumJ += ts.J[(CELL ? 4 : 0) + j];
    }
    jt[c] = SG * (int)ts.Jtau;
    f[c] = col[c] ? (int)ts.f : (1 << 24);  // a column without a spin is never active
    // h_eff = h + sum_j J_j (2 b_j - 1) + tau terms: the constant part is `base`
    // (in the two-field form without the tau terms, which form h_tau).  The
    // one-field form accumulates -h_eff (every coefficient negated), so that
    // d = s h_eff comes from the spin's bit with one sign extension.
    base[c] = SG * ((int)ts.h - sumJ - (RING && !TF ? 2 * (int)ts.Jtau : 0));
    const uint32_t fw = T.fifo[sy.tmpl0 + qq0];
    fb[c] = (int)(fw >> 8);
    fmask[c] = (1 << (fw & 0xff)) - 1;
  }

  // Range of the level offsets of each column slot over the wavefront: at
  // level lv a lane is on row lv - f, so no lane of the wavefront can be on
  // the first or last slice (whose halo copies a flip must keep) unless lv
  // lies within [fmin, fmax] or [fmin + M - 1, fmax + M - 1].
  int fmin[CPT], fspan[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    int lo = col[c] ? f[c] : (1 << 24), hi = col[c] ? f[c] : -(1 << 24);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      lo = min(lo, __shfl_xor(lo, o));
      hi = max(hi, __shfl_xor(hi, o));
    }
    fmin[c] = __builtin_amdgcn_readfirstlane(lo);
    fspan[c] = __builtin_amdgcn_readfirstlane(hi) - fmin[c];  // negative: no column in the wavefront
  }

  // Generator: chain heads j < min(S, 227) go round-robin to the walker's
  // threads (head h of thread t is j = t + h*TPW; TPW*CPT >= S, so h < CPT);
  // a head makes words j, j+227, j+454 (< S) of each chunk.  The uniform
  // queue of each word's column is resolved once, into registers.
  const int heads = S < kMtLag ? S : kMtLag;
  int gqb[CPT][3], gqm[CPT][3];
#pragma unroll
  for (int h = 0; h < CPT; ++h)
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int o = t + h * TPW + s * kMtLag;
      const bool ok = live && t + h * TPW < heads && o < S;
      const uint32_t fw = ok ? T.fifo[sy.tmpl0 + o] : 0u;
      gqb[h][s] = (int)(fw >> 8);
      gqm[h][s] = (1 << (fw & 0xff)) - 1;
    }
  // The look-back reads of every head run without a guard: for o = j + 227 s
  // < heads + 454 they stay within [-624, Zg) of the ring (its shadow in
  // front included), so only the words with o < S are computed and stored.
  auto gen_chunk = [&](int gslot, int chunk) {
    if (!live) return;
    // the generating wavefronts set the pace of the level's barrier: they
    // issue first while they generate (wave priority, back to 0 after)
    __builtin_amdgcn_s_setprio(3);
#pragma unroll
    for (int h = 0; h < CPT; ++h) {
      const int j = t + h * TPW;
      if (j >= heads) break;
      uint32_t a[3], b[3];
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const int x = gslot + j + s * kMtLag;
        a[s] = gring[x - kMtN];
        b[s] = gring[x - kMtN + 1];
      }
      uint32_t prev = gring[gslot + j - kMtLag];
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const int o = j + s * kMtLag;
        if (o < S) {
          const int x = gslot + o;
          prev = mt_next_word(a[s], b[s], prev);
          gring[x] = prev;
          if (x >= zs) gring[x - Zg] = prev;
          fq[gqb[h][s] + ((chunk & gqm[h][s]) << 6)] = prev;
        }
      }
    }
    __builtin_amdgcn_s_setprio(0);
  };
  auto advance = [Zg, S](int x) {
    x += S;
    return x >= Zg ? x - Zg : x;
  };

  __syncthreads();

  int gslot = c0 * S;  // generator slot of the next chunk
  int dE = 0, nfl = 0;  // per lane: sum of d over flips (the cost changes by 2d), flips
  int dB = 0;           // per lane, two-field form: sum of d_t over flips (B changes by -2 d_t)
  int64_t n_rounds = 0;  // swap rounds run in this launch (ladder tiles)
  uint32_t st_steps = 0, st_flip = 0, nfl_w = 0, nfl_0 = 0;  // per wavefront
  // Flips are counted per lane when a wavefront holds several walkers of at
  // most 64 threads, else per wavefront as popcounts of the flip ballot
  // (scalar work only).  A SHARED wavefront (above 64 threads per walker, not a
  // multiple of 64) holds lanes of at most two walkers: m0 marks those of its
  // first lane's walker, nfl_0 counts their flips and nfl_w all flips.
  const uint64_t m0 = SHARED ? __builtin_amdgcn_ballot_w64(gw == __builtin_amdgcn_readfirstlane(gw)) : ~0ull;

  gen_chunk(gslot, 0);
  gslot = advance(gslot);
  level_sync<WS>();

  if (init_mode) {
    // Initial spins: bit (m, q) = top bit of output m*S + q.
    for (int m = 0; m < M; ++m) {
      if (m + 1 < M) {
        gen_chunk(gslot, m + 1);
        gslot = advance(gslot);
      }
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        if (col[c]) {
          const uint32_t u = mt_temper(fq[fb[c] + ((m & fmask[c]) << 6)]);
          if (u >> 31) atomicOr(sp + m * RS + qo[c], 1u << qb[c]);
        }
      }
      level_sync<WS>();
    }
  } else {
    const int levels = M + F - 1;
    const bool wave_walker = !WS || TPW == 64;  // a wavefront's lanes belong to at most SHARED + 1 walkers
    for (int sw = 0; sw < n_sweeps; ++sw) {
      const int chunk0 = sw * M;
      const int gen_levels = sw + 1 < n_sweeps ? M : M - 1;  // levels that generate a chunk
      for (int lv = 0; lv < levels; ++lv) {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          const int m = lv - f[c];
          const bool active = (unsigned)m < (unsigned)M;
          // Wavefronts with no active lane skip the column; inside, inactive
          // lanes compute on row 0 (in bounds) and their result is dropped.
          const uint64_t act = __builtin_amdgcn_ballot_w64(active);
          if (act != 0ull) {
            ++st_steps;
            const int mm = active ? m : 0;
            const int rc = (int)__umul24((unsigned)mm, (unsigned)RS) + qo[c];
            uint32_t *own_p = sp + rc;
            const uint32_t own = *own_p;
            const uint32_t u0 = fq[fb[c] + (((chunk0 + mm) & fmask[c]) << 6)];
            int hs = base[c];
            if (CELL) {
              const uint32_t nib = __builtin_amdgcn_ubfe(own, (unsigned)((qb[c] & ~3) ^ 4), 4u);
              const uint32_t spread = __umul24(nib, 0x00204081u) & 0x01010101u;  // bit i -> byte i
              hs = __builtin_amdgcn_sdot4((int)spread, jpack[c], hs, false);
            }
#pragma unroll
            for (int j = 0; j < NX; ++j)
              hs += __builtin_amdgcn_sbfe((int)own_p[xoff[c][j]], (unsigned)xbit[c][j], 1u) & xj2[c][j];
            const int bp = (int)__builtin_amdgcn_ubfe(own_p[-RS], (unsigned)qb[c], 1u);
            const int bn = (int)__builtin_amdgcn_ubfe(own_p[RS], (unsigned)qb[c], 1u);
            int ht = 0;  // tau part of the field (two-field form)
            if (RING) {
              if (TF)
                ht = __mul24(2 * jt[c], bp + bn) - 2 * jt[c];
              else
                hs += __mul24(2 * jt[c], bp + bn);
            } else {
              const int jp = mm > 0 ? jt[c] : 0, jn = mm < M - 1 ? jt[c] : 0;
              if (TF)
                ht = __mul24(jp, 2 * bp - 1) + __mul24(jn, 2 * bn - 1);
              else
                hs += __mul24(jp, 2 * bp - 1) + __mul24(jn, 2 * bn - 1);
            }
            // d = s_i * h_eff_i (flipping costs 2d)
            int d, dt = 0;
            uint32_t thv;
            if (TF) {  // with dn = -1 for a spin down and 0 for up, d = (h ^ dn) - dn
              const int dn = __builtin_amdgcn_sbfe((int)~own, (unsigned)qb[c], 1u);
              const int dsp = (hs ^ dn) - dn;
              dt = (ht ^ dn) - dn;
              d = dsp + dt;
              thv = thw[dsp * qwt + dt + qoff];
            } else {  // hs = -h_eff; with up = -1 for a spin up and 0 for down, d = (hs ^ up) - up
              const int up = __builtin_amdgcn_sbfe((int)own, (unsigned)qb[c], 1u);
              d = (hs ^ up) - up;
              thv = thw[d + kThrZero];
            }
            const uint32_t u = mt_temper(u0);
            const bool le = u <= thv;
            const uint64_t fl = __builtin_amdgcn_ballot_w64(le) & act;
            const bool flip = le && active;
            const uint32_t nfl_step = (uint32_t)__builtin_popcountll(fl);
            st_flip += nfl_step != 0u ? 1u : 0u;
            if (wave_walker) {
              nfl_w += nfl_step;
              if (SHARED) nfl_0 += (uint32_t)__builtin_popcountll(fl & m0);
            } else {
              nfl += flip ? 1 : 0;
            }
            dE += flip ? d : 0;
            if (TF) dB += flip ? dt : 0;
            // wavefront-uniform: can any lane be on the first or last slice?
            const bool edge = RING && ((unsigned)(lv - fmin[c]) <= (unsigned)fspan[c] ||
                                       (unsigned)(lv - fmin[c] - (M - 1)) <= (unsigned)fspan[c]);
            if (flip) {
              const uint32_t bit = 1u << qb[c];
              atomicXor(own_p, bit);
              // keep the halo copy of the first / last slice (M >= 3 on a ring)
              if (edge && (mm == 0 || mm == M - 1)) atomicXor(own_p + (mm == 0 ? WW : -WW), bit);
            }
          }
        }
        // the next chunk: slice lv + 1 of this sweep, or slice 0 of the next
        if (lv < gen_levels) {
          gen_chunk(gslot, chunk0 + lv + 1);
          gslot = advance(gslot);
        }
        level_sync<WS>();
      }
      if (ladder && (la.sweeps0 + sw + 1) % la.swap_every == 0) {
        // running energies up to date, then the round; a threshold row belongs
        // to a slot, so the walkers of each accepted pair trade rows
        if (live && dE) atomicAdd(&acc[0], 2 * dE);
        dE = 0;
        __syncthreads();
        const int parity = (int)((la.rounds0 + n_rounds) & 1);
        const int np = ladder_swap_round(sy, parity, tid, L, pb.lo(parity), pb.hi(parity), lds, PW,
                                         ZP + FW + SWW + TRW, (unsigned long long *)St.swap_near + sy.slot0);
        ++n_rounds;
        for (int i = tid; i < np * TRW; i += nthr) {
          const int j = i / TRW, wd = i - j * TRW;
          const int ab = L.moved[j];
          if (ab >= 0) {
            uint32_t *ra = wbase(ab & 0xffff) + ZP + FW + SWW + wd, *rb = wbase(ab >> 16) + ZP + FW + SWW + wd;
            const uint32_t v = *ra;
            *ra = *rb;
            *rb = v;
          }
        }
        __syncthreads();
      }
    }
  }

  // ---- write back ----
  if (live && !init_mode) {
    atomicAdd(&acc[0], 2 * dE);
    if (TF && dB) atomicAdd(&acc[4], -2 * dB);
    if (nfl) atomicAdd(&acc[1], nfl);
    // wavefront statistics and the flips counted per wavefront go to the
    // walker of the wavefront's first lane; in a SHARED wavefront the flips of
    // the second walker's lanes (nfl_w - nfl_0) go to that walker's first lane
    const int lane = tid & 63;
    const uint32_t first = SHARED ? nfl_0 : nfl_w;
    if (lane == 0) {
      atomicAdd(&acc[2], (int)st_steps);
      atomicAdd(&acc[3], (int)st_flip);
      if (first) atomicAdd(&acc[1], (int)first);
    }
    if (SHARED && nfl_w != nfl_0 && lane == __builtin_ctzll(~m0)) atomicAdd(&acc[1], (int)(nfl_w - nfl_0));
  }
  __syncthreads();
  each_word(WW, [&](int w, int j) {
    St.spins[sy.spin_word0 + (size_t)(tile.w0 + w) * WW + j] = wbase(w)[ZP + FW + RS + j];
  });
  // the window's oldest word sits in slot (consumed + delta) mod Zg; j < kMtN < Zg,
  // so one subtraction wraps slot + j
  const long long consumed = init_mode ? (long long)M * S : (long long)n_sweeps * M * S;
  const int wslot = (int)((consumed + delta) % Zg);
  each_word(kMtN, [&](int w, int j) {
    const int r = sy.walker0 + tile.w0 + w;
    int x = wslot + j;
    if (x >= Zg) x -= Zg;
    St.mt[(size_t)r * kMtN + j] = wbase(w)[kMtN + x];
  });
  if (!init_mode && tid < nw) {
    const int r = sy.walker0 + tile.w0 + tid;
    const int32_t *a = (const int32_t *)(wbase(tid) + ZP + FW + SWW + TRW);
    St.energy[r] = a[0];
    if (TF) St.bond[r] = a[4];
    St.flips[r] += (unsigned long long)(uint32_t)a[1];
    St.wsteps[2 * (size_t)r] += (unsigned long long)(uint32_t)a[2];
    St.wsteps[2 * (size_t)r + 1] += (unsigned long long)(uint32_t)a[3];
  }
  if (ladder) ladder_store(St, sy, tile.sys, tid, nthr, L, la.rounds0, n_rounds);
}

template <int NX, bool CELL, bool RING, int CPT, bool WS, bool LADDER, bool TF, bool SHARED = false>
static hipError_t launch_variant(const DevTables &t, const DevState &s, const Bucket &b,
                                 int32_t n_sweeps, int32_t init_mode, hipStream_t st, LadderArgs la) {
  auto kern = sweep_kernel<NX, CELL, RING, CPT, WS, LADDER, TF, SHARED>;
  // Allow the whole LDS once per instantiation and device.
  static std::atomic<uint64_t> lds_limit_set{0};
  if (b.lds > 64 * 1024) {
    hipError_t e = allow_lds(kern, 160 * 1024, lds_limit_set);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(b.ntiles), dim3(b.threads), b.lds, st, t, s, b.tile0, b.G, b.tpw,
                     b.walker_words, n_sweeps, init_mode, la);
  return hipGetLastError();
}

template <int NX, bool CELL, bool RING, bool TF>
static hipError_t launch_cpt(const DevTables &t, const DevState &s, const Bucket &b, int32_t n_sweeps,
                             int32_t init_mode, hipStream_t st, LadderArgs la) {
  const bool ws = b.tpw <= 64;
  if constexpr (!TF) {
    if (b.ladder) {  // whole ladders in one workgroup: walkers of at most one wavefront each
      if (!ws) return hipErrorInvalidValue;
      switch (b.cpt) {
        case 1: return launch_variant<NX, CELL, RING, 1, true, true, false>(t, s, b, n_sweeps, init_mode, st, la);
        case 2: return launch_variant<NX, CELL, RING, 2, true, true, false>(t, s, b, n_sweeps, init_mode, st, la);
        case 4: return launch_variant<NX, CELL, RING, 4, true, true, false>(t, s, b, n_sweeps, init_mode, st, la);
        case 8: return launch_variant<NX, CELL, RING, 8, true, true, false>(t, s, b, n_sweeps, init_mode, st, la);
      }
      return hipErrorInvalidValue;
    }
  } else {
    if (b.ladder) return hipErrorInvalidValue;  // the two-field form swaps in swap_kernel
  }
  // above 64 threads per walker, a count that is not a multiple of 64 lets a
  // wavefront hold two walkers (the host allows it with at most two columns)
  const bool shared = !ws && (b.tpw & 63) != 0;
  if (shared && b.cpt > 2) return hipErrorInvalidValue;
  switch (b.cpt) {
    case 1: return ws       ? launch_variant<NX, CELL, RING, 1, true, false, TF>(t, s, b, n_sweeps, init_mode, st, la)
                   : shared ? launch_variant<NX, CELL, RING, 1, false, false, TF, true>(t, s, b, n_sweeps, init_mode,
                                                                                      st, la)
                            : launch_variant<NX, CELL, RING, 1, false, false, TF>(t, s, b, n_sweeps, init_mode, st, la);
    case 2: return ws       ? launch_variant<NX, CELL, RING, 2, true, false, TF>(t, s, b, n_sweeps, init_mode, st, la)
                   : shared ? launch_variant<NX, CELL, RING, 2, false, false, TF, true>(t, s, b, n_sweeps, init_mode,
                                                                                      st, la)
                            : launch_variant<NX, CELL, RING, 2, false, false, TF>(t, s, b, n_sweeps, init_mode, st, la);
    case 4: return ws ? launch_variant<NX, CELL, RING, 4, true, false, TF>(t, s, b, n_sweeps, init_mode, st, la)
                      : launch_variant<NX, CELL, RING, 4, false, false, TF>(t, s, b, n_sweeps, init_mode, st, la);
    case 8: return ws ? launch_variant<NX, CELL, RING, 8, true, false, TF>(t, s, b, n_sweeps, init_mode, st, la)
                      : launch_variant<NX, CELL, RING, 8, false, false, TF>(t, s, b, n_sweeps, init_mode, st, la);
  }
  return hipErrorInvalidValue;
}

template <bool CELL, bool RING, bool TF>
static hipError_t launch_nx(const DevTables &t, const DevState &s, const Bucket &b, int32_t n_sweeps,
                            int32_t init_mode, hipStream_t st, LadderArgs la) {
  switch (b.nx) {
    case 0: return launch_cpt<0, CELL, RING, TF>(t, s, b, n_sweeps, init_mode, st, la);
    case 2: return launch_cpt<2, CELL, RING, TF>(t, s, b, n_sweeps, init_mode, st, la);
    case 4: return launch_cpt<4, CELL, RING, TF>(t, s, b, n_sweeps, init_mode, st, la);
    case 6: if (!CELL) return launch_cpt<6, CELL, RING, TF>(t, s, b, n_sweeps, init_mode, st, la); break;
    case 8: if (!CELL) return launch_cpt<8, CELL, RING, TF>(t, s, b, n_sweeps, init_mode, st, la); break;
  }
  return hipErrorInvalidValue;
}

// The initial-spins launch (init_mode) reads no thresholds and writes no
// energies, so it always takes the one-field variant.
hipError_t launch_sweep(const DevTables &t, const DevState &s, const Bucket &b, int32_t n_sweeps,
                        int32_t init_mode, hipStream_t st, LadderArgs la) {
  if (b.ntiles == 0) return hipSuccess;
  if (t.two_field && !init_mode) {
    if (!b.cell) return hipErrorInvalidValue;  // the two-field form is built for cell templates
    return b.ring ? launch_nx<true, true, true>(t, s, b, n_sweeps, init_mode, st, la)
                  : launch_nx<true, false, true>(t, s, b, n_sweeps, init_mode, st, la);
  }
  if (b.cell)
    return b.ring ? launch_nx<true, true, false>(t, s, b, n_sweeps, init_mode, st, la)
                  : launch_nx<true, false, false>(t, s, b, n_sweeps, init_mode, st, la);
  return b.ring ? launch_nx<false, true, false>(t, s, b, n_sweeps, init_mode, st, la)
                : launch_nx<false, false, false>(t, s, b, n_sweeps, init_mode, st, la);
}

}  // namespace ising
