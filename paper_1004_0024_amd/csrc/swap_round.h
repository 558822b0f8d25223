// One parallel-tempering swap round run inside a sweep kernel whose
// workgroup holds every walker of the system (the same rule and draw order
// as swap_kernel).
#pragma once
#include "internal.h"
#include "mt19937.h"

namespace ising {

// One swap round of a system whose walkers all sit in this workgroup (one
// thread): the same rule and draw order as swap_kernel, on LDS copies of the
// swap stream (circular 624-word window, head *head), the labels and the
// walkers' running energies.
static __device__ void ladder_swap_round(const DevTables &T, const DevState &St, const SysInfo &sy, int parity,
                                  uint32_t *swin, int32_t *wat, int32_t *tof, int32_t *misc,
                                  const uint32_t *wslots, int PW, int acc_off) {
#pragma clang fp contract(off)
  const int K = sy.K, p0 = parity & 1;
  int h = misc[0];
  for (int k = p0; k + 1 < K; k += 2) {
    const int a = wat[k], b = wat[k + 1];
    const int ea = (int)wslots[a * PW + acc_off], eb = (int)wslots[b * PW + acc_off];
    const uint32_t x = mt_next_word(swin[h], swin[h + 1 == kMtN ? 0 : h + 1], swin[h + kMtM < kMtN ? h + kMtM : h + kMtM - kMtN]);
    swin[h] = x;
    h = h + 1 == kMtN ? 0 : h + 1;
    const double delta = (T.beta[sy.slot0 + k] - T.beta[sy.slot0 + k + 1]) * (double)(ea - eb);
    const double xu = (double)mt_temper(x) * 0x1p-32;
    const double p = exp(delta);
    const bool accept = (delta >= 0.0) || (xu < p);
    if (delta < 0.0 && fabs(xu - p) < 1e-12) ++misc[1];
    St.swap_att[sy.slot0 + k] += 1ull;
    if (accept) {
      wat[k] = b;
      wat[k + 1] = a;
      tof[a] = k + 1;
      tof[b] = k;
      St.swap_acc[sy.slot0 + k] += 1ull;
    }
  }
  misc[0] = h;
}

}  // namespace ising
