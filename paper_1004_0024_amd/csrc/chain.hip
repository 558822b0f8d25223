// Chain kernels around the sweep: stream seeding, parallel-tempering swap
// rounds, energy records, observables.
#include "internal.h"
#include "mt19937.h"

namespace ising {

// ---- seeding: word 0 of each 624-word window holds the seed --------------
__global__ void seed_kernel(uint32_t *mt, int32_t n) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  uint32_t *x = mt + (size_t)r * kMtN;
  uint32_t v = x[0];
  for (int i = 1; i < kMtN; ++i) {
    v = mt_seed_step(v, (uint32_t)i);
    x[i] = v;
  }
}

hipError_t launch_seed(const DevState &s, int32_t R, int32_t n_sys, hipStream_t st) {
  if (R > 0) hipLaunchKernelGGL(seed_kernel, dim3((R + 127) / 128), dim3(128), 0, st, s.mt, R);
  if (n_sys > 0)
    hipLaunchKernelGGL(seed_kernel, dim3((n_sys + 127) / 128), dim3(128), 0, st, s.swap_mt, n_sys);
  return hipGetLastError();
}

// ---- totals of the per-walker and per-pair counters -----------------------
// stats[0] near-threshold swaps, [1..2] wavefront steps, [4] flips, [5..6]
// swap attempts / acceptances; one workgroup, fixed-order tree reductions (no
// atomics).
__global__ void __launch_bounds__(256) reduce_stats_kernel(DevState St, int32_t R, int32_t slots) {
  __shared__ unsigned long long red[6][256];
  unsigned long long v[6] = {0, 0, 0, 0, 0, 0};
  for (int r = threadIdx.x; r < R; r += blockDim.x) {
    v[0] += St.wsteps[2 * (size_t)r];
    v[1] += St.wsteps[2 * (size_t)r + 1];
    v[2] += St.flips[r];
  }
  for (int k = threadIdx.x; k < slots; k += blockDim.x) {
    v[3] += St.swap_att[k];
    v[4] += St.swap_acc[k];
    v[5] += St.swap_near[k];
  }
  for (int i = 0; i < 6; ++i) red[i][threadIdx.x] = v[i];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int i = 0; i < 6; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    St.stats[0] = red[5][0];
    St.stats[1] = red[0][0];
    St.stats[2] = red[1][0];
    St.stats[4] = red[2][0];
    St.stats[5] = red[3][0];
    St.stats[6] = red[4][0];
  }
}

hipError_t launch_reduce_stats(const DevState &s, int32_t R, int32_t slots, hipStream_t st) {
  hipLaunchKernelGGL(reduce_stats_kernel, dim3(1), dim3(256), 0, st, s, R, slots);
  return hipGetLastError();
}

// ---- labels: walker j of a system at slot j -------------------------------
__global__ void labels_kernel(DevTables T, DevState St, int32_t R) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const SysInfo sy = T.sys[T.walker_sys[r]];
  const int j = r - sy.walker0;
  St.temp_of[r] = j;
  St.walker_at[sy.slot0 + j] = j;
}

hipError_t launch_labels(const DevTables &t, const DevState &s, int32_t R, int32_t n_sys,
                         hipStream_t st) {
  (void)n_sys;
  if (R > 0) hipLaunchKernelGGL(labels_kernel, dim3((R + 255) / 256), dim3(256), 0, st, t, s, R);
  return hipGetLastError();
}

// ---- parallel-tempering swap round ----------------------------------------
// One workgroup per system.  Pairs (k, k+1), k = parity, parity+2, ..., one
// swap-stream draw each in ascending k; accept iff delta >= 0 or
// u * 2^-32 < exp(delta), delta = (beta_k - beta_k+1)(E_a - E_b) in IEEE
// double (the only floating-point decision of the chain).  In the two-field
// form slot k weighs a state by exp(-a_k E_sp + c_k B) and delta is the log
// ratio of the exchanged to the current assignment,
// (a_k - a_k+1)(E_sp,a - E_sp,b) - (c_k - c_k+1)(B_a - B_b), E_sp = E + B.
// Temperature labels move; spins and streams stay with their walkers.
__global__ void __launch_bounds__(64) swap_kernel(DevTables T, DevState St, int32_t parity,
                                                  int32_t *e_row) {
#pragma clang fp contract(off)
  const int s = blockIdx.x;
  const SysInfo sy = T.sys[s];
  const int K = sy.K;
  const int p0 = parity & 1;
  const int npairs = K >= p0 + 2 ? (K - 2 - p0) / 2 + 1 : 0;
  __shared__ uint32_t buf[kMtN + kMtLag];
  __shared__ int32_t wat[256];
  const int tid = threadIdx.x;
  uint32_t *win = St.swap_mt + (size_t)s * kMtN;
  for (int j = tid; j < kMtN; j += blockDim.x) buf[j] = win[j];
  for (int k = tid; k < K; k += blockDim.x) wat[k] = St.walker_at[sy.slot0 + k];
  __syncthreads();
  for (int j = tid; j < npairs; j += blockDim.x) buf[kMtN + j] = mt_next_word(buf[j], buf[j + 1], buf[j + kMtM]);
  __syncthreads();
  // the round's pairs are disjoint: thread i decides pairs i, i + 64, ... with
  // the stream outputs drawn above in pair order
  for (int i = tid; i < npairs; i += blockDim.x) {
    const int k = p0 + 2 * i;
    const int a = wat[k], b = wat[k + 1];
    const int ea = St.energy[sy.walker0 + a], eb = St.energy[sy.walker0 + b];
    double delta = (T.beta[sy.slot0 + k] - T.beta[sy.slot0 + k + 1]) * (double)(ea - eb);
    if (T.two_field) {
      const int ba = St.bond[sy.walker0 + a], bb = St.bond[sy.walker0 + b];
      const double d_sp = (T.qa[sy.slot0 + k] - T.qa[sy.slot0 + k + 1]) * (double)((ea + ba) - (eb + bb));
      const double d_t = (T.qc[sy.slot0 + k] - T.qc[sy.slot0 + k + 1]) * (double)(ba - bb);
      delta = d_sp - d_t;
    }
    const uint32_t u = mt_temper(buf[kMtN + i]);
    const double x = (double)u * 0x1p-32;
    const double p = exp(delta);
    const bool accept = (delta >= 0.0) || (x < p);
    if (delta < 0.0 && fabs(x - p) < 1e-12) St.swap_near[sy.slot0 + k] += 1ull;
    St.swap_att[sy.slot0 + k] += 1ull;
    if (accept) {
      wat[k] = b;
      wat[k + 1] = a;
      St.temp_of[sy.walker0 + a] = k + 1;
      St.temp_of[sy.walker0 + b] = k;
      St.swap_acc[sy.slot0 + k] += 1ull;
    }
  }
  __syncthreads();
  for (int j = tid; j < kMtN; j += blockDim.x) win[j] = buf[npairs + j];
  for (int k = tid; k < K; k += blockDim.x) {
    St.walker_at[sy.slot0 + k] = wat[k];
    if (e_row) e_row[sy.slot0 + k] = St.energy[sy.walker0 + wat[k]];
  }
}

hipError_t launch_swap(const DevTables &t, const DevState &s, int32_t n_sys, int32_t parity,
                       int32_t *e_row, hipStream_t st) {
  if (n_sys > 0) hipLaunchKernelGGL(swap_kernel, dim3(n_sys), dim3(64), 0, st, t, s, parity, e_row);
  return hipGetLastError();
}

// ---- energy of the walker at each slot -------------------------------------
__global__ void record_kernel(DevTables T, DevState St, int32_t *e_row) {
  const SysInfo sy = T.sys[blockIdx.x];
  for (int k = threadIdx.x; k < sy.K; k += blockDim.x)
    e_row[sy.slot0 + k] = St.energy[sy.walker0 + St.walker_at[sy.slot0 + k]];
}

hipError_t launch_record(const DevTables &t, const DevState &s, int32_t n_sys, int32_t *e_row,
                         hipStream_t st) {
  if (n_sys > 0) hipLaunchKernelGGL(record_kernel, dim3(n_sys), dim3(64), 0, st, t, s, e_row);
  return hipGetLastError();
}

// ---- observables: cost from the spins, magnetisation, tau-bond sum ----------
// f(s) = -sum_i h_i s_i - sum_edges J s s, every edge once: in-slice edges from
// their lower endpoint, tau edges from slice m to m+1 (and M-1 to 0 on a ring);
// B = sum over the tau edges of J_tau s s'.
__global__ void __launch_bounds__(256) observables_kernel(DevTables T, DevState St, int32_t *obs,
                                                          int32_t set_energy) {
  const int r = blockIdx.x;
  const SysInfo sy = T.sys[T.walker_sys[r]];
  const int S = sy.S, M = sy.M, RS = sy.RS;
  const uint32_t *sp = St.spins + sy.spin_word0 + (size_t)(r - sy.walker0) * sy.WW;
  auto spin = [&](int m, int q) { return (int)((sp[m * RS + (q >> 5)] >> (q & 31)) & 1u) * 2 - 1; };
  long long e = 0, mag = 0, bond = 0;
  const int N = S * M;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const int m = i / S, q = i - m * S;
    const TmplSpin ts = T.tmpl[sy.tmpl0 + q];
    const int s = spin(m, q);
    e -= (long long)ts.h * s;
    mag += s;
    for (int j = 0; j < ts.deg; ++j)
      if (ts.nbr[j] > q) e -= (long long)ts.J[j] * s * spin(m, ts.nbr[j]);
    if (M > 1 && (m + 1 < M || sy.ring)) bond += (long long)ts.Jtau * s * spin(m + 1 < M ? m + 1 : 0, q);
  }
  e -= bond;
  __shared__ long long red[3][256];
  red[0][threadIdx.x] = e;
  red[1][threadIdx.x] = mag;
  red[2][threadIdx.x] = bond;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
      red[2][threadIdx.x] += red[2][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int et = (int)red[0][0], bt = (int)red[2][0];
    if (set_energy) {
      St.energy[r] = et;
      St.bond[r] = bt;
    }
    if (obs) {
      int32_t *o = obs + (size_t)r * 6;
      o[0] = et;
      o[1] = (int)red[1][0];
      o[2] = St.energy[r];
      o[3] = St.temp_of[r];
      o[4] = bt;
      o[5] = St.bond[r];
    }
  }
}

hipError_t launch_observables(const DevTables &t, const DevState &s, int32_t R, int32_t *obs,
                              int32_t set_energy, hipStream_t st) {
  if (R > 0) hipLaunchKernelGGL(observables_kernel, dim3(R), dim3(256), 0, st, t, s, obs, set_energy);
  return hipGetLastError();
}

}  // namespace ising
