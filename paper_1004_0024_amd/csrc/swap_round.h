// Parallel-tempering swap rounds run inside a sweep kernel whose workgroup
// holds every walker of the system (the same rule and draw order as
// swap_kernel).
#pragma once
#include "internal.h"
#include "mt19937.h"

namespace ising {

// The swap state in LDS (kLadderWords words): the swap stream's circular
// 624-word window with its head in misc[0], the walker at each slot and the
// slot of each walker, accepted swaps per slot in this launch, and per pair of
// the last round a | b << 16 when the walkers a and b traded slots, else -1.
struct LadderLds {
  uint32_t *swin;
  int32_t *wat, *tof, *misc;
  uint32_t *nacc;
  int32_t *moved;
};

static __device__ __forceinline__ LadderLds ladder_lds(uint32_t *base) {
  LadderLds L;
  L.swin = base;
  L.wat = (int32_t *)(base + kMtN);
  L.tof = L.wat + 256;
  L.misc = L.tof + 256;
  L.nacc = (uint32_t *)(L.misc + 4);
  L.moved = (int32_t *)(L.nacc + 256);
  return L;
}

// One swap round; every thread of the workgroup calls it (it synchronises the
// workgroup).  The round's pairs (k, k + 1), k = parity + 2 j, are disjoint,
// and pair j takes output j of the swap stream in this round, the order in
// which the sequential rule draws them.  Fewer than 227 outputs of MT19937
// never depend on one another, so thread j computes output j from the window
// as it stood before the round.  bk and bk1 are beta of slots k and k + 1 of
// the calling thread's pair; wslots + w * PW + acc_off holds walker w's
// running cost.  A decision within 1e-12 of its threshold is counted in
// near[k], the system's row of the per-pair counts (for a given parity thread
// j always takes the same k, so no other thread writes that entry).  Returns
// the number of pairs.
static __device__ int ladder_swap_round(const SysInfo &sy, int parity, int tid, const LadderLds &L, double bk,
                                        double bk1, const uint32_t *wslots, int PW, int acc_off,
                                        unsigned long long *near) {
#pragma clang fp contract(off)
  const int K = sy.K, p0 = parity & 1, np = (K - p0) / 2;
  const int h = L.misc[0];
  int i = h + tid;
  if (i >= kMtN) i -= kMtN;
  uint32_t x = 0u;
  if (tid < np) {
    const int i1 = i + 1 == kMtN ? 0 : i + 1;
    const int im = i + kMtM < kMtN ? i + kMtM : i + kMtM - kMtN;
    x = mt_next_word(L.swin[i], L.swin[i1], L.swin[im]);
  }
  __syncthreads();  // every output is computed from the old window before any is stored
  if (tid < np) {
    L.swin[i] = x;
    const int k = p0 + 2 * tid;
    const int a = L.wat[k], b = L.wat[k + 1];
    const int ea = (int)wslots[a * PW + acc_off], eb = (int)wslots[b * PW + acc_off];
    const double delta = (bk - bk1) * (double)(ea - eb);
    const double xu = (double)mt_temper(x) * 0x1p-32;
    const double p = exp(delta);
    const bool accept = (delta >= 0.0) || (xu < p);
    if (delta < 0.0 && fabs(xu - p) < 1e-12) near[k] += 1ull;
    L.moved[tid] = accept ? (a | (b << 16)) : -1;
    if (accept) {
      L.wat[k] = b;
      L.wat[k + 1] = a;
      L.tof[a] = k + 1;
      L.tof[b] = k;
      ++L.nacc[k];
    }
  }
  __syncthreads();
  if (tid == 0) L.misc[0] = h + np >= kMtN ? h + np - kMtN : h + np;
  return np;
}

// Beta of the slots a thread's pair may take: thread t holds beta of slots
// 2t, 2t + 1 and 2t + 2 (zero past the ladder); for a round of parity p its
// pair is (2t + p, 2t + p + 1).
struct PairBeta {
  double b0, b1, b2;
  __device__ double lo(int parity) const { return parity & 1 ? b1 : b0; }
  __device__ double hi(int parity) const { return parity & 1 ? b2 : b1; }
};

static __device__ __forceinline__ PairBeta pair_beta(const DevTables &T, const SysInfo &sy, int tid) {
  PairBeta pb{0.0, 0.0, 0.0};
  const int k = 2 * tid;
  if (k < sy.K) pb.b0 = T.beta[sy.slot0 + k];
  if (k + 1 < sy.K) pb.b1 = T.beta[sy.slot0 + k + 1];
  if (k + 2 < sy.K) pb.b2 = T.beta[sy.slot0 + k + 2];
  return pb;
}

// Load the swap state of system tile.sys (stream window, labels) and clear the
// launch's counters.
static __device__ void ladder_load(const DevState &St, const SysInfo &sy, int sys, int tid, int nthr,
                                   const LadderLds &L) {
  for (int j = tid; j < kMtN; j += nthr) L.swin[j] = St.swap_mt[(size_t)sys * kMtN + j];
  for (int k = tid; k < sy.K; k += nthr) {
    L.wat[k] = St.walker_at[sy.slot0 + k];
    L.tof[k] = St.temp_of[sy.walker0 + k];
  }
  for (int k = tid; k < 256; k += nthr) L.nacc[k] = 0u;
  if (tid == 0) L.misc[0] = 0;
}

// Write the swap state back after n_rounds rounds numbered from rounds0: the
// stream window (oldest word first), labels, per-slot attempts (slot k takes
// part in the rounds whose parity is k mod 2) and acceptances.
static __device__ void ladder_store(const DevState &St, const SysInfo &sy, int sys, int tid, int nthr,
                                    const LadderLds &L, int64_t rounds0, int64_t n_rounds) {
  const int h = L.misc[0];
  for (int j = tid; j < kMtN; j += nthr) {
    const int x = h + j;
    St.swap_mt[(size_t)sys * kMtN + j] = L.swin[x >= kMtN ? x - kMtN : x];
  }
  for (int k = tid; k < sy.K; k += nthr) {
    St.walker_at[sy.slot0 + k] = L.wat[k];
    St.temp_of[sy.walker0 + k] = L.tof[k];
    if (k + 1 < sy.K) {
      const int64_t natt = (n_rounds + ((rounds0 & 1) == (k & 1) ? 1 : 0)) / 2;
      if (natt) St.swap_att[sy.slot0 + k] += (unsigned long long)natt;
      if (L.nacc[k]) St.swap_acc[sy.slot0 + k] += (unsigned long long)L.nacc[k];
    }
  }
}

}  // namespace ising
