// Layer-pair order: the paper's GPU layout (Section 3.2, Figure 12c) as a
// chain of its own.  The M slices of a walker form M/2 pairs (2t, 2t+1); lane
// t of the walker owns pair t and its MT19937 generator.  A sweep visits every
// even slice (lane t its slice 2t, spins in index order, one draw of its
// generator per spin), then every odd slice.  Slices of one parity share no
// edge, so the lanes of a phase run side by side.  The paper pushes field
// updates to the slice on one side during a phase and to the other side after
// it, so that no two threads write one field at once; here a spin's field is
// pulled from its neighbours' bits when it is visited, which needs neither.
//
// One workgroup holds a whole system (K walkers x M/2 lanes), so swap rounds
// run in the kernel between sweeps.  LDS per walker: the spins (M rows of RS
// words), its slot's threshold row and reduction words; per workgroup the swap
// state and a three-word record per template spin (every lane visits the same
// spin at the same time, so a record is one broadcast read).  A lane keeps the
// word of 32 spins it is sweeping in a register, with the words of the slices
// above and below.  The generators are interlaced in HBM in quads of slots
// ([156][lanes][4]: quad b of every lane side by side, so one 16-byte load per
// lane covers a contiguous 1 KB per wavefront) and updated in place 8 outputs
// (two quads) at a time, the reads of a batch issued while the previous
// batch's spins are attempted: per output one read of slots n and n + 397 and
// one write, the 12 bytes per attempt of the HBM roofline model.  Slices have
// a multiple of 8 spins (K4,4 cells), so every batch is two whole, aligned
// quads.
#include "internal.h"
#include "mt19937.h"
#include "swap_round.h"

namespace ising {

// ---- generator storage: slot k of lane l at ((k / 4) * n_lanes + l) * 4 + k % 4
__host__ __device__ inline int64_t pair_slot(int k, int64_t lane, int64_t n_lanes) {
  return ((int64_t)(k >> 2) * n_lanes + lane) * 4 + (k & 3);
}

// ---- seeding: slot 0 of each lane holds the seed --------------------------
__global__ void pair_seed_kernel(uint32_t *pmt, int64_t n_lanes) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n_lanes) return;
  uint32_t v = pmt[pair_slot(0, l, n_lanes)];
  for (int i = 1; i < kMtN; ++i) {
    v = mt_seed_step(v, (uint32_t)i);
    pmt[pair_slot(i, l, n_lanes)] = v;
  }
}

hipError_t launch_pair_seed(uint32_t *pair_mt, int64_t n_lanes, hipStream_t st) {
  if (n_lanes > 0)
    hipLaunchKernelGGL(pair_seed_kernel, dim3((unsigned)((n_lanes + 255) / 256)), dim3(256), 0, st, pair_mt,
                       n_lanes);
  return hipGetLastError();
}

constexpr int kPairBatch = 8;                 // generator outputs per batch: two quads
constexpr int kPairQuads = kMtN / 4;          // 156

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// A lane's generator is advanced 8 outputs at a time, in place: slot k holds
// x_{n-624} before and x_n after; output i of the batch at slot pos (a
// multiple of 8) reads slots pos+i, pos+i+1 and pos+i+397 (mod 624), none of
// them written earlier in the batch.  pos + 397 = 4 (pos/4 + 99) + 1, so the
// look-back words are words 1..3 of quad pos/4 + 99, all of the next quad and
// word 0 of the one after.  The loads of a batch are issued one batch ahead
// (gen_load), so their latency hides behind the previous batch's attempts; a
// batch's loads touch no slot that the batch before it writes.
struct GenBatch {
  u32x4 a0, a1, m0, m1;  // slots pos..pos+7; look-back quads pos/4 + 99 and + 100
  uint32_t a8, m8;       // slot pos+8; look-back word 0 of quad pos/4 + 101
};

// quad b of this lane: lane0 points at quad 0 of the lane (4 words)
__device__ __forceinline__ const uint32_t *pair_quad(const uint32_t *lane0, int64_t n_lanes, int b) {
  return lane0 + (int64_t)b * n_lanes * 4;
}

__device__ __forceinline__ int quad_add(int b, int d) {
  b += d;
  return b >= kPairQuads ? b - kPairQuads : b;
}

__device__ __forceinline__ void gen_load(const uint32_t *lane0, int64_t n_lanes, int pos, GenBatch &g) {
  const int b = pos >> 2;
  g.a0 = *(const u32x4 *)pair_quad(lane0, n_lanes, b);
  g.a1 = *(const u32x4 *)pair_quad(lane0, n_lanes, quad_add(b, 1));
  g.a8 = pair_quad(lane0, n_lanes, quad_add(b, 2))[0];
  g.m0 = *(const u32x4 *)pair_quad(lane0, n_lanes, quad_add(b, 99));
  g.m1 = *(const u32x4 *)pair_quad(lane0, n_lanes, quad_add(b, 100));
  g.m8 = pair_quad(lane0, n_lanes, quad_add(b, 101))[0];
}

// The 8 outputs of the batch at pos: written back, tempered into u.
__device__ __forceinline__ void gen_finish(uint32_t *lane0, int64_t n_lanes, int pos, const GenBatch &g, uint32_t *u) {
  const uint32_t a[9] = {g.a0.x, g.a0.y, g.a0.z, g.a0.w, g.a1.x, g.a1.y, g.a1.z, g.a1.w, g.a8};
  const uint32_t m[8] = {g.m0.y, g.m0.z, g.m0.w, g.m1.x, g.m1.y, g.m1.z, g.m1.w, g.m8};
  uint32_t x[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    x[i] = mt_next_word(a[i], a[i + 1], m[i]);
    u[i] = mt_temper(x[i]);
  }
  const int b = pos >> 2;
  *(u32x4 *)pair_quad(lane0, n_lanes, b) = u32x4{x[0], x[1], x[2], x[3]};
  *(u32x4 *)pair_quad(lane0, n_lanes, quad_add(b, 1)) = u32x4{x[4], x[5], x[6], x[7]};
}

// Record of template spin q (K4,4 cell templates, at most two neighbours
// outside the cell), three LDS words:
//   [0]  2J to the four partners in the other half of the cell, byte i for
//        partner i (the sdot4 operand);
//   [1]  h - sum of the in-slice J (int8) | J_tau << 8 | 2J_a << 16 | 2J_b << 24;
//   [2]  word offset of outside neighbour a from q's word (int8) | its bit << 8
//        | the same for b << 16 (2J = 0 when the neighbour does not exist).
__device__ __forceinline__ void pair_record(const TmplSpin &ts, int q, uint32_t *r0, uint32_t *r1, uint32_t *r2) {
  int sumJ = 0;
  for (int j = 0; j < ts.deg; ++j) sumJ += ts.J[j];
  uint32_t w1 = (uint32_t)(uint8_t)(int8_t)(ts.h - sumJ) | (uint32_t)(uint8_t)ts.Jtau << 8;
  uint32_t w2 = 0;
  for (int j = 4; j < 6; ++j) {
    const int sh = 16 * (j - 4);
    if (j < ts.deg) {
      const int qq = ts.nbr[j];
      w1 |= (uint32_t)(uint8_t)(int8_t)(2 * ts.J[j]) << (16 + 8 * (j - 4));
      w2 |= ((uint32_t)(uint8_t)(int8_t)((qq >> 5) - (q >> 5)) | (uint32_t)(qq & 31) << 8) << sh;
    }
  }
  *r0 = (uint32_t)ts.jpack;
  *r1 = w1;
  *r2 = w2;
}

template <bool RING>
__global__ void __launch_bounds__(1024) pairs_kernel(DevTables T, DevState St, uint32_t *pmt, int64_t n_lanes,
                                                     int32_t n_sweeps, int32_t init_mode, LadderArgs la) {
  extern __shared__ uint32_t lds[];
  const SysInfo sy = T.sys[blockIdx.x];
  if ((sy.ring != 0) != RING) return;  // the launch of its class takes it
  const int S = sy.S, M = sy.M, RS = sy.RS, WW = sy.WW, K = sy.K, P = M >> 1;
  const int PW = pair_walker_words(WW);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int w = tid / P, t = tid - w * P;
  const bool live = w < K;
  uint32_t *slot = lds + (live ? w : 0) * PW;
  const uint32_t *thw = slot + WW;
  int32_t *acc = (int32_t *)(slot + WW + kPairThrRow);

  // ---- load the walkers' spins, threshold rows and running costs ----
  for (int i = tid; i < K * WW; i += nthr) {
    const int ww = i / WW, j = i - ww * WW;
    lds[ww * PW + j] = init_mode ? 0u : St.spins[sy.spin_word0 + (int64_t)ww * WW + j];
  }
  if (!init_mode)
    for (int i = tid; i < K * kPairThrRow; i += nthr) {  // entries d = 0..63 of the slot's row
      const int ww = i / kPairThrRow, j = i - ww * kPairThrRow;
      const int sl = St.temp_of[sy.walker0 + ww];
      lds[ww * PW + WW + j] = T.thr[(size_t)(sy.thr0 + sl) * kThrRow + kThrZero + j];
    }
  for (int i = tid; i < K * 4; i += nthr)
    lds[(i >> 2) * PW + WW + kPairThrRow + (i & 3)] =
        ((i & 3) == 0 && !init_mode) ? (uint32_t)St.energy[sy.walker0 + (i >> 2)] : 0u;
  const bool ladder = la.swap_every > 0 && !init_mode;
  const LadderLds L = ladder_lds(lds + K * PW);
  uint32_t *prec = lds + K * PW + kLadderWords;  // template records, three arrays of S words
  for (int q = tid; q < S; q += nthr) pair_record(T.tmpl[sy.tmpl0 + q], q, prec + q, prec + S + q, prec + 2 * S + q);
  PairBeta pb{0.0, 0.0, 0.0};
  if (ladder) {
    ladder_load(St, sy, (int)blockIdx.x, tid, nthr, L);
    pb = pair_beta(T, sy, tid);
  }
  __syncthreads();

  // ---- this lane's generator and slices ----
  uint32_t *glane = pmt + ((int64_t)sy.pl0 + (live ? tid : 0)) * 4;  // this lane's quad 0
  int pos = init_mode ? 0 : (int)((2 * (int64_t)S * (1 + la.sweeps0)) % kMtN);
  int dE = 0, nfl = 0;  // sum of d over flips (the cost changes by 2d), flips
  int64_t n_rounds = 0;
  const int nsw = init_mode ? 1 : n_sweeps;
  GenBatch gb;  // the loads of the next batch, issued one batch ahead
  if (live) gen_load(glane, n_lanes, __builtin_amdgcn_readfirstlane(pos), gb);
  for (int sw = 0; sw < nsw; ++sw) {
    for (int par = 0; par < 2; ++par) {
      if (live) {
        const int row = 2 * t + par;
        int ru = row - 1, rd = row + 1;
        if (ru < 0) ru = RING ? M - 1 : -1;
        if (rd >= M) rd = RING ? 0 : -1;
        uint32_t *rp = slot + row * RS;
        const uint32_t *up = slot + (ru < 0 ? row : ru) * RS;
        const uint32_t *dn = slot + (rd < 0 ? row : rd) * RS;
        const uint32_t umask = ru < 0 ? 0u : ~0u, dmask = rd < 0 ? 0u : ~0u;
        const int ntau = (ru >= 0 ? 1 : 0) + (rd >= 0 ? 1 : 0);
        for (int wq = 0; wq * 32 < S; ++wq) {
          // every lane of the workgroup visits the same spin q at the same time:
          // its template record is read once per wavefront, through the scalar cache
          const int wqu = __builtin_amdgcn_readfirstlane(wq);
          const int nq = min(32, S - wqu * 32);
          uint32_t cur = rp[wqu];
          const uint32_t tu = up[wqu] & umask, td = dn[wqu] & dmask;
          // one attempt at bit b of the word, with uniform u
          auto attempt = [&](const int b, const uint32_t u) {
            const int q = wqu * 32 + b;
            const uint32_t r0 = __builtin_amdgcn_readfirstlane(prec[q]);
            const uint32_t r1 = __builtin_amdgcn_readfirstlane(prec[S + q]);
            const uint32_t r2 = __builtin_amdgcn_readfirstlane(prec[2 * S + q]);
            // h_eff = (h - sum J) + sum_j 2 J_j b_j + tau terms
            const uint32_t nib = (cur >> ((b & ~3) ^ 4)) & 15u;  // the other half of the cell
            const uint32_t spread = __umul24(nib, 0x00204081u) & 0x01010101u;
            int hs = __builtin_amdgcn_sdot4((int)spread, (int)r0, (int)(int8_t)r1, false);
            const int wa = (int)(int8_t)r2, wb = (int)(int8_t)(r2 >> 16);
            const uint32_t na = wa == 0 ? cur : rp[wqu + wa];
            const uint32_t nb2 = wb == 0 ? cur : rp[wqu + wb];
            hs += (int)((na >> ((r2 >> 8) & 31u)) & 1u) * (int)(int8_t)(r1 >> 16);
            hs += (int)((nb2 >> ((r2 >> 24) & 31u)) & 1u) * (int)(int8_t)(r1 >> 24);
            const int jt = (int)(int8_t)(r1 >> 8);
            hs += 2 * jt * (int)(((tu >> b) & 1u) + ((td >> b) & 1u)) - jt * ntau;
            const int dn_ = -(int)((~cur >> b) & 1u);  // -1 for a spin down, 0 for up
            const int d = (hs ^ dn_) - dn_;            // s * h_eff
            const bool flip = u <= thw[d > 0 ? d : 0];
            cur ^= flip ? 1u << b : 0u;
            dE += flip ? d : 0;
            nfl += flip ? 1 : 0;
          };
#pragma unroll
          for (int h = 0; h < 32 / kPairBatch; ++h) {
            const int n0 = h * kPairBatch;
            if (nq == 32 || n0 < nq) {  // whole blocks: S is a multiple of 8
              uint32_t u[kPairBatch];
              gen_finish(glane, n_lanes, __builtin_amdgcn_readfirstlane(pos), gb, u);
              pos += kPairBatch;
              if (pos >= kMtN) pos -= kMtN;
              gen_load(glane, n_lanes, __builtin_amdgcn_readfirstlane(pos), gb);
#pragma unroll
              for (int i = 0; i < kPairBatch; ++i) {
                if (init_mode)
                  cur |= (u[i] >> 31) << (n0 + i);  // initial spin: the top bit of the output
                else
                  attempt(n0 + i, u[i]);
              }
            }
          }
          rp[wqu] = cur;
        }
      }
      __syncthreads();  // this parity's slices are final before the other parity reads them
    }
    if (ladder && (la.sweeps0 + sw + 1) % la.swap_every == 0) {
      if (live && dE) atomicAdd(&acc[0], 2 * dE);
      dE = 0;
      __syncthreads();
      // a threshold row belongs to a slot: the walkers of each accepted pair trade rows
      const int parity = (int)((la.rounds0 + n_rounds) & 1);
      const int np = ladder_swap_round(sy, parity, tid, L, pb.lo(parity), pb.hi(parity), lds, PW, WW + kPairThrRow,
                                       (unsigned long long *)St.swap_near + sy.slot0);
      ++n_rounds;
      for (int i = tid; i < np * kPairThrRow; i += nthr) {
        const int j = i / kPairThrRow, wd = i - j * kPairThrRow;
        const int ab = L.moved[j];
        if (ab >= 0) {
          uint32_t *ra = lds + (ab & 0xffff) * PW + WW + wd, *rb = lds + (ab >> 16) * PW + WW + wd;
          const uint32_t v = *ra;
          *ra = *rb;
          *rb = v;
        }
      }
      __syncthreads();
    }
  }

  // ---- write back ----
  if (live && !init_mode) {
    if (dE) atomicAdd(&acc[0], 2 * dE);
    if (nfl) atomicAdd(&acc[1], nfl);
  }
  __syncthreads();
  for (int i = tid; i < K * WW; i += nthr) {
    const int ww = i / WW, j = i - ww * WW;
    St.spins[sy.spin_word0 + (int64_t)ww * WW + j] = lds[ww * PW + j];
  }
  if (!init_mode && tid < K) {
    const int r = sy.walker0 + tid;
    const int32_t *a = (const int32_t *)(lds + tid * PW + WW + kPairThrRow);
    St.energy[r] = a[0];
    St.flips[r] += (unsigned long long)(uint32_t)a[1];
  }
  if (ladder) ladder_store(St, sy, (int)blockIdx.x, tid, nthr, L, la.rounds0, n_rounds);
}

template <bool RING>
static hipError_t launch_pairs_variant(const DevTables &t, const DevState &s, uint32_t *pmt, int64_t n_lanes,
                                       int32_t n_sys, int32_t threads, size_t lds, int32_t n_sweeps,
                                       int32_t init_mode, LadderArgs la, hipStream_t st) {
  auto kern = pairs_kernel<RING>;
  static std::atomic<uint64_t> lds_limit_set{0};
  if (lds > 64 * 1024) {
    hipError_t e = allow_lds(kern, 160 * 1024, lds_limit_set);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(n_sys), dim3(threads), lds, st, t, s, pmt, n_lanes, n_sweeps, init_mode, la);
  return hipGetLastError();
}

// classes: bit 0 set when some system has open slices, bit 1 when some has a
// ring; one launch per class present (systems of the other class return at once).
hipError_t launch_pairs(const DevTables &t, const DevState &s, uint32_t *pair_mt, int64_t n_lanes, int32_t n_sys,
                        int32_t threads, size_t lds, uint32_t classes, int32_t n_sweeps, int32_t init_mode,
                        LadderArgs la, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (classes & 2u) e = launch_pairs_variant<true>(t, s, pair_mt, n_lanes, n_sys, threads, lds, n_sweeps, init_mode, la, st);
  if (e == hipSuccess && (classes & 1u))
    e = launch_pairs_variant<false>(t, s, pair_mt, n_lanes, n_sys, threads, lds, n_sweeps, init_mode, la, st);
  return e;
}

}  // namespace ising
