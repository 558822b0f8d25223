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
// bit.  One thread owns one template column q of one walker and visits its M
// spins at levels f(q) .. f(q)+M-1; a sweep takes M + F - 1 levels,
// F = max f + 1.  This is the paper's interlacing of layers over threads
// (Section 3.2, Figure 12c) with a skew that keeps the sequential order
// instead of an even/odd reordering.
//
// Data in LDS for the whole launch, per walker:
//  - spins, one bit each, slice rows of RS words (RS odd when > 1, so rows of
//    different slices fall in different LDS banks);
//  - the walker's MT19937 words in a ring of Z words: word n (counted from the
//    launch's first window word) lives in slot (n + delta) mod Z, chunks of S
//    words aligned to slot multiples of S; chunk g holds the uniforms of slice
//    m = g mod M of sweep g / M.  A copy of the last kMtN slots sits in front of
//    slot 0, so the generator's look-back reads (624, 623 and 227 words back)
//    never wrap;
//  - its threshold row thr[d] = ceil(2^32 exp(-2 beta d)) - 1 (d = 0 -> all).
// The local field of a spin is pulled from its neighbours' bits when the spin
// is visited (no field array, no conflicting neighbour updates).  For cell
// templates (K4,4 unit cells) the four in-cell neighbours are the other nibble
// of the spin's own byte and are summed with one 4-way byte dot product.  The
// MT19937 chunk for the next slice is generated cooperatively by the walker's
// threads one level ahead (a generator thread chains the words 227 apart).
#include "internal.h"
#include "mt19937.h"

namespace ising {

template <int NX, bool CELL, bool RING>
__global__ void __launch_bounds__(1024) sweep_kernel(DevTables T, DevState St, int32_t tile0,
                                                     int32_t G, int32_t n_sweeps, int32_t init_mode) {
  extern __shared__ uint32_t lds[];
  const Tile tile = T.tiles[tile0 + blockIdx.x];
  const SysInfo sy = T.sys[tile.sys];
  const int S = sy.S, M = sy.M, RS = sy.RS, WW = sy.WW;
  const int F = init_mode ? 1 : sy.F;
  const int Z = ring_words(S, sy.F);
  const int ZP = Z + kMtN;  // physical ring words per walker (shadow + ring)
  const int nw = tile.nw;
  const int tid = threadIdx.x, nthr = blockDim.x;

  uint32_t *ringp = lds;                          // [G][ZP]
  uint32_t *sp = ringp + G * ZP;                  // [G][WW]
  uint32_t *thr = sp + G * WW;                    // [G][kThrRow]
  int32_t *acc = (int32_t *)(thr + G * kThrRow);  // [G][4]

  const int delta = (S - (kMtN % S)) % S;  // chunk-aligned slots
  const int c0 = (kMtN + delta) / S;       // slot chunk of chunk 0
  const int zs = Z - kMtN;                 // slots >= zs also live in the shadow

  // ---- load the walkers' state ----
  for (int i = tid; i < nw * kMtN; i += nthr) {
    const int w = i / kMtN, j = i - w * kMtN;
    const int r = sy.walker0 + tile.w0 + w;
    const uint32_t v = St.mt[(size_t)r * kMtN + j];
    uint32_t *rb = ringp + w * ZP + kMtN;
    const int x = j + delta;
    rb[x] = v;
    if (x >= zs) rb[x - Z] = v;
  }
  for (int i = tid; i < nw * WW; i += nthr) {
    const int w = i / WW, j = i - w * WW;
    sp[w * WW + j] = init_mode ? 0u : St.spins[sy.spin_word0 + (size_t)(tile.w0 + w) * WW + j];
  }
  if (!init_mode) {
    for (int i = tid; i < nw * kThrRow; i += nthr) {
      const int w = i / kThrRow, j = i - w * kThrRow;
      const int slot = St.temp_of[sy.walker0 + tile.w0 + w];
      thr[w * kThrRow + j] = T.thr[(size_t)(sy.thr0 + slot) * kThrRow + j];
    }
  }
  if (tid < G * 4) acc[tid] = 0;

  // ---- this thread's column ----
  const int gw = tid / S, q = tid - gw * S;
  const bool live = gw < nw;
  const int qo = q >> 5;
  const int qb = q & 31;
  const uint32_t qbit = 1u << qb;
  int xoff[NX > 0 ? NX : 1], xbit[NX > 0 ? NX : 1], xj2[NX > 0 ? NX : 1];
  int base = 0, jt = 0, f = 0, jpack = 0;
  if (live) {
    const TmplSpin ts = T.tmpl[sy.tmpl0 + q];
    int sumJ = 0;
    if (CELL) {
#pragma unroll
      for (int j = 0; j < 4; ++j) sumJ += ts.J[j];
      jpack = ts.jpack;
    }
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const int qq = ts.nbr[(CELL ? 4 : 0) + j];
      xoff[j] = (qq >> 5) - qo;
      xbit[j] = qq & 31;
      xj2[j] = 2 * (int)ts.J[(CELL ? 4 : 0) + j];
      sumJ += ts.J[(CELL ? 4 : 0) + j];
    }
    jt = ts.Jtau;
    f = ts.f;
    // h_eff = h + sum_j J_j (2 b_j - 1) + tau terms: the constant part is `base`.
    base = (int)ts.h - sumJ - (RING ? 2 * jt : 0);
  }
  const int nibpos = (qb & ~3) ^ 4;  // partner nibble inside the own word
  uint32_t *spw = sp + (live ? gw : 0) * WW + qo;  // own word of row 0
  uint32_t *rw = ringp + (live ? gw : 0) * ZP + kMtN;
  const uint32_t *thw = thr + (live ? gw : 0) * kThrRow;

  // Generator role.  S <= 227: thread (gw, q) makes word q of each chunk.
  // S > 227: thread t < G*227 makes words j, j+227, j+454 of walker t/227.
  const bool chained = S > kMtLag;
  const int gen_w = chained ? tid / kMtLag : gw;
  const int gen_j = chained ? tid - gen_w * kMtLag : q;
  const bool gen_live = gen_w < nw && (chained || live);
  uint32_t *grb = ringp + (gen_w < G ? gen_w : 0) * ZP + kMtN;

  auto put = [&](int x, uint32_t v) {
    grb[x] = v;
    if (x >= zs) grb[x - Z] = v;
  };
  auto gen_chunk = [&](int gslot) {  // gslot: ring slot of word 0 of the chunk
    if (!gen_live) return;
    if (!chained) {
      const int x = gslot + gen_j;
      put(x, mt_next_word(grb[x - kMtN], grb[x - kMtN + 1], grb[x - kMtLag]));
    } else {
      uint32_t prev = 0;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int o = gen_j + i * kMtLag;
        if (o < S) {
          const int x = gslot + o;
          const uint32_t c = i == 0 ? grb[x - kMtLag] : prev;
          prev = mt_next_word(grb[x - kMtN], grb[x - kMtN + 1], c);
          put(x, prev);
        }
      }
    }
  };

  __syncthreads();

  int gslot = c0 * S;  // slot of the next chunk to generate
  auto advance = [Z, S](int x) {
    x += S;
    return x >= Z ? x - Z : x;
  };
  int cpos = c0 * S + q;  // slot of this thread's next uniform
  auto cadvance = [Z, S](int x) {
    x += S;
    return x >= Z ? x - Z : x;
  };
  int dE = 0, nfl = 0;
  uint32_t st_steps = 0, st_flip = 0;

  gen_chunk(gslot);
  gslot = advance(gslot);
  __syncthreads();

  if (init_mode) {
    // Initial spins: bit (m, q) = top bit of output m*S + q.
    for (int m = 0; m < M; ++m) {
      if (m + 1 < M) {
        gen_chunk(gslot);
        gslot = advance(gslot);
      }
      if (live) {
        const uint32_t u = mt_temper(rw[cpos]);
        if (u >> 31) atomicOr(spw + m * RS, qbit);
      }
      cpos = cadvance(cpos);
      __syncthreads();
    }
  } else {
    const int levels = M + F - 1;
    const int last_row = (M - 1) * RS;
    for (int t = 0; t < n_sweeps; ++t) {
      for (int lv = 0; lv < levels; ++lv) {
        const int m = lv - f;
        const bool active = live && m >= 0 && m < M;
        bool flip = false;
        if (active) {
          const int rc = (int)__umul24((unsigned)m, (unsigned)RS);
          const int rp = m == 0 ? last_row : rc - RS;
          const int rn = m == M - 1 ? 0 : rc + RS;
          uint32_t *own_p = spw + rc;
          const uint32_t own = *own_p;
          int hs = base;
          if (CELL) {
            const uint32_t nib = __builtin_amdgcn_ubfe(own, (unsigned)nibpos, 4u);
            const uint32_t spread = __umul24(nib, 0x00204081u) & 0x01010101u;  // bit i -> byte i
            hs = __builtin_amdgcn_sdot4((int)spread, jpack, hs, false);
          }
#pragma unroll
          for (int j = 0; j < NX; ++j)
            hs += __builtin_amdgcn_sbfe((int)own_p[xoff[j]], (unsigned)xbit[j], 1u) & xj2[j];
          const int bp = (int)__builtin_amdgcn_ubfe(spw[rp], (unsigned)qb, 1u);
          const int bn = (int)__builtin_amdgcn_ubfe(spw[rn], (unsigned)qb, 1u);
          if (RING) {
            hs += 2 * jt * (bp + bn);
          } else {
            const int jp = m > 0 ? jt : 0, jn = m < M - 1 ? jt : 0;
            hs += jp * (2 * bp - 1) + jn * (2 * bn - 1);
          }
          const int sb = (int)__builtin_amdgcn_ubfe(own, (unsigned)qb, 1u);
          const int d = sb ? hs : -hs;  // s_i * h_eff_i; flipping costs 2d
          const uint32_t u = mt_temper(rw[cpos]);
          flip = u <= thw[d > 0 ? d : 0];
          if (flip) {
            atomicXor(own_p, qbit);
            dE += 2 * d;
            ++nfl;
          }
          cpos = cadvance(cpos);
        }
        st_steps += __ballot(active) != 0ull;
        st_flip += __ballot(flip) != 0ull;
        if (lv + 1 < M || (lv == M - 1 && t + 1 < n_sweeps)) {
          gen_chunk(gslot);
          gslot = advance(gslot);
        }
        __syncthreads();
      }
    }
  }

  // ---- write back ----
  if (live && !init_mode) {
    atomicAdd(&acc[gw * 4 + 0], dE);
    atomicAdd(&acc[gw * 4 + 1], nfl);
  }
  if (!init_mode && (tid & 63) == 0) {
    atomicAdd((unsigned long long *)&St.stats[1], (unsigned long long)st_steps);
    atomicAdd((unsigned long long *)&St.stats[2], (unsigned long long)st_flip);
    if (tid == 0)
      atomicAdd((unsigned long long *)&St.stats[3], (unsigned long long)nw * S * M * n_sweeps);
  }
  __syncthreads();
  for (int i = tid; i < nw * WW; i += nthr) {
    const int w = i / WW, j = i - w * WW;
    St.spins[sy.spin_word0 + (size_t)(tile.w0 + w) * WW + j] = sp[w * WW + j];
  }
  const long long consumed = init_mode ? (long long)M * S : (long long)n_sweeps * M * S;
  for (int i = tid; i < nw * kMtN; i += nthr) {
    const int w = i / kMtN, j = i - w * kMtN;
    const int r = sy.walker0 + tile.w0 + w;
    St.mt[(size_t)r * kMtN + j] = ringp[w * ZP + kMtN + (int)((consumed + j + delta) % Z)];
  }
  if (!init_mode && tid < nw) {
    const int r = sy.walker0 + tile.w0 + tid;
    St.energy[r] += acc[tid * 4 + 0];
    St.flips[r] += (unsigned long long)(uint32_t)acc[tid * 4 + 1];
  }
}

template <int NX, bool CELL, bool RING>
static hipError_t launch_variant(const DevTables &t, const DevState &s, const Bucket &b,
                                 int32_t n_sweeps, int32_t init_mode, hipStream_t st) {
  auto kern = sweep_kernel<NX, CELL, RING>;
  if (b.lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)b.lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(b.ntiles), dim3(b.threads), b.lds, st, t, s, b.tile0, b.G, n_sweeps,
                     init_mode);
  return hipGetLastError();
}

template <bool CELL, bool RING>
static hipError_t launch_nx(const DevTables &t, const DevState &s, const Bucket &b, int32_t n_sweeps,
                            int32_t init_mode, hipStream_t st) {
  switch (b.nx) {
    case 0: return launch_variant<0, CELL, RING>(t, s, b, n_sweeps, init_mode, st);
    case 2: return launch_variant<2, CELL, RING>(t, s, b, n_sweeps, init_mode, st);
    case 4: return launch_variant<4, CELL, RING>(t, s, b, n_sweeps, init_mode, st);
    case 6: return launch_variant<6, CELL, RING>(t, s, b, n_sweeps, init_mode, st);
    case 8: return launch_variant<8, CELL, RING>(t, s, b, n_sweeps, init_mode, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep(const DevTables &t, const DevState &s, const Bucket &b, int32_t n_sweeps,
                        int32_t init_mode, hipStream_t st) {
  if (b.ntiles == 0) return hipSuccess;
  if (b.cell) {
    if (b.nx > 4) return hipErrorInvalidValue;
    return b.ring ? launch_nx<true, true>(t, s, b, n_sweeps, init_mode, st)
                  : launch_nx<true, false>(t, s, b, n_sweeps, init_mode, st);
  }
  return b.ring ? launch_nx<false, true>(t, s, b, n_sweeps, init_mode, st)
                : launch_nx<false, false>(t, s, b, n_sweeps, init_mode, st);
}

}  // namespace ising
