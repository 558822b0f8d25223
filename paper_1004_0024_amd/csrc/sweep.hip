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
//  - spins, one bit each, slice rows of SW = ceil(S/32) words;
//  - the walker's MT19937 words in a ring: word n (counted from the launch's
//    first window word) lives in slot (n + delta) mod Z, chunks of S words
//    aligned to slot multiples of S; chunk g holds the uniforms of slice
//    m = g mod M of sweep g / M;
//  - its threshold row thr[d] = ceil(2^32 exp(-2 beta d)) - 1 (d = 0 -> all).
// The local field of a spin is pulled from its neighbours' bits when the spin
// is visited (no field array, no conflicting neighbour updates), and the
// MT19937 chunk for the next slice is generated cooperatively by the walker's
// threads one level ahead (each generator thread chains the words 227 apart).
#include "internal.h"
#include "mt19937.h"

namespace ising {

template <int NDEG, bool RING>
__global__ void __launch_bounds__(1024) sweep_kernel(DevTables T, DevState St, int32_t tile0,
                                                     int32_t G, int32_t n_sweeps, int32_t init_mode) {
  extern __shared__ uint32_t lds[];
  const Tile tile = T.tiles[tile0 + blockIdx.x];
  const SysInfo sy = T.sys[tile.sys];
  const int S = sy.S, M = sy.M, SW = sy.SW, WW = sy.WW;
  const int F = init_mode ? 1 : sy.F;
  const int Z = ring_words(S, sy.F);
  const int nw = tile.nw;
  const int tid = threadIdx.x, nthr = blockDim.x;

  uint32_t *ring = lds;                    // [G][Z]
  uint32_t *sp = ring + G * Z;             // [G][WW]
  uint32_t *thr = sp + G * WW;             // [G][kThrRow]
  int32_t *acc = (int32_t *)(thr + G * kThrRow);  // [G][4]

  const int delta = (S - (kMtN % S)) % S;  // chunk-aligned slots
  const int c0 = (kMtN + delta) / S;       // slot chunk of chunk 0

  // ---- load the walkers' state ----
  for (int i = tid; i < nw * kMtN; i += nthr) {
    const int w = i / kMtN, j = i - w * kMtN;
    const int r = sy.walker0 + tile.w0 + w;
    ring[w * Z + j + delta] = St.mt[(size_t)r * kMtN + j];
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
  const uint32_t qbit = 1u << (q & 31);
  const int qb = q & 31;
  int nb_word[NDEG > 0 ? NDEG : 1], nb_bit[NDEG > 0 ? NDEG : 1], nb_j2[NDEG > 0 ? NDEG : 1];
  int base = 0, jt = 0, f = 0;
  if (live) {
    const TmplSpin ts = T.tmpl[sy.tmpl0 + q];
    int sumJ = 0;
#pragma unroll
    for (int j = 0; j < NDEG; ++j) {
      const int qq = ts.nbr[j];
      nb_word[j] = qq >> 5;
      nb_bit[j] = qq & 31;
      nb_j2[j] = 2 * (int)ts.J[j];
      sumJ += ts.J[j];
    }
    jt = ts.Jtau;
    f = ts.f;
    // h_eff = h + sum_j J_j (2 b_j - 1) + tau terms: keep the constant part in `base`.
    base = (int)ts.h - sumJ - (RING ? 2 * jt : 0);
  }
  uint32_t *spw = sp + (live ? gw : 0) * WW;
  uint32_t *rw = ring + (live ? gw : 0) * Z;
  const uint32_t *thw = thr + (live ? gw : 0) * kThrRow;

  // Generator role.  S <= 227: thread (gw, q) makes word q of each chunk.
  // S > 227: thread t < G*227 makes words j, j+227, j+454 of walker t/227.
  const bool chained = S > kMtLag;
  const int gen_w = chained ? tid / kMtLag : gw;
  const int gen_j = chained ? tid - gen_w * kMtLag : q;
  const bool gen_live = gen_w < nw && (chained ? true : live);
  uint32_t *gring = ring + (gen_w < G ? gen_w : 0) * Z;

  auto wrapz = [Z](int x) { return x < 0 ? x + Z : x; };
  auto gen_chunk = [&](int gslot) {  // gslot: ring slot of word 0 of the chunk
    if (!gen_live) return;
    uint32_t prev = 0;
    for (int o = gen_j; o < S; o += kMtLag) {
      const int s0 = gslot + o;
      const uint32_t a = gring[wrapz(s0 - kMtN)];
      const uint32_t b = gring[wrapz(s0 - kMtN + 1)];
      const uint32_t c = (o >= kMtLag) ? prev : gring[wrapz(s0 - kMtLag)];
      prev = mt_next_word(a, b, c);
      gring[s0] = prev;
    }
  };

  __syncthreads();

  int gslot = c0 * S;  // slot of the next chunk to generate
  auto advance = [Z, S](int x) {
    x += S;
    return x >= Z ? x - Z : x;
  };
  int cslot = c0 * S;  // slot of this thread's next chunk to consume
  int dE = 0, nfl = 0;
  uint32_t st_steps = 0, st_flip = 0, st_att = 0;

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
        const uint32_t u = mt_temper(rw[cslot + q]);
        if (u >> 31) atomicOr(&spw[m * SW + qo], qbit);
      }
      cslot = advance(cslot);
      __syncthreads();
    }
  } else {
    const int levels = M + F - 1;
    for (int t = 0; t < n_sweeps; ++t) {
      for (int lv = 0; lv < levels; ++lv) {
        const int m = lv - f;
        const bool active = live && m >= 0 && m < M;
        bool flip = false;
        if (active) {
          const int rowm = m * SW;
          const int rowp = (m == 0 ? M - 1 : m - 1) * SW;
          const int rown = (m == M - 1 ? 0 : m + 1) * SW;
          const uint32_t own = spw[rowm + qo];
          const int sb = (own >> qb) & 1;
          int hs = base;
#pragma unroll
          for (int j = 0; j < NDEG; ++j) hs += nb_j2[j] * (int)((spw[rowm + nb_word[j]] >> nb_bit[j]) & 1u);
          const int bp = (spw[rowp + qo] >> qb) & 1;
          const int bn = (spw[rown + qo] >> qb) & 1;
          if (RING) {
            hs += 2 * jt * (bp + bn);
          } else {
            const int jp = m > 0 ? jt : 0, jn = m < M - 1 ? jt : 0;
            hs += jp * (2 * bp - 1) + jn * (2 * bn - 1);
          }
          const int d = sb ? hs : -hs;  // s_i * h_eff_i; flipping costs 2d
          const uint32_t u = mt_temper(rw[cslot + q]);
          flip = u <= thw[d > 0 ? d : 0];
          if (flip) {
            atomicXor(&spw[rowm + qo], qbit);
            dE += 2 * d;
            ++nfl;
          }
          cslot = advance(cslot);
        }
        const unsigned long long act_mask = __ballot(active);
        const unsigned long long flip_mask = __ballot(flip);
        st_steps += act_mask != 0ull;
        st_flip += flip_mask != 0ull;
        st_att += __popcll(act_mask);
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
    atomicAdd((unsigned long long *)&St.stats[3], (unsigned long long)st_att);
  }
  __syncthreads();
  for (int i = tid; i < nw * WW; i += nthr) {
    const int w = i / WW, j = i - w * WW;
    St.spins[sy.spin_word0 + (size_t)(tile.w0 + w) * WW + j] = sp[w * WW + j];
  }
  const int consumed = init_mode ? M * S : n_sweeps * M * S;
  for (int i = tid; i < nw * kMtN; i += nthr) {
    const int w = i / kMtN, j = i - w * kMtN;
    const int r = sy.walker0 + tile.w0 + w;
    St.mt[(size_t)r * kMtN + j] = ring[w * Z + (int)(((long long)consumed + j + delta) % Z)];
  }
  if (!init_mode && tid < nw) {
    const int r = sy.walker0 + tile.w0 + tid;
    St.energy[r] += acc[tid * 4 + 0];
    St.flips[r] += (unsigned long long)(uint32_t)acc[tid * 4 + 1];
  }
}

template <int NDEG, bool RING>
static hipError_t launch_variant(const DevTables &t, const DevState &s, const Bucket &b,
                                 int32_t n_sweeps, int32_t init_mode, hipStream_t st) {
  auto kern = sweep_kernel<NDEG, RING>;
  if (b.lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)b.lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(b.ntiles), dim3(b.threads), b.lds, st, t, s, b.tile0, b.G, n_sweeps,
                     init_mode);
  return hipGetLastError();
}

hipError_t launch_sweep(const DevTables &t, const DevState &s, const Bucket &b, int32_t n_sweeps,
                        int32_t init_mode, hipStream_t st) {
  if (b.ntiles == 0) return hipSuccess;
  const int d = b.deg <= 0 ? 0 : b.deg <= 2 ? 2 : b.deg <= 4 ? 4 : b.deg <= 6 ? 6 : 8;
#define ISING_CASE(D)                                                              \
  case D:                                                                          \
    return b.ring ? launch_variant<D, true>(t, s, b, n_sweeps, init_mode, st)      \
                  : launch_variant<D, false>(t, s, b, n_sweeps, init_mode, st);
  switch (d) {
    ISING_CASE(0)
    ISING_CASE(2)
    ISING_CASE(4)
    ISING_CASE(6)
    ISING_CASE(8)
  }
#undef ISING_CASE
  return hipErrorInvalidValue;
}

}  // namespace ising
