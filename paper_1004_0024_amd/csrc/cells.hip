// Cell moves of the learned proposal: boundary fields of the 8-spin cells,
// training rows from the chain, and the Metropolis-Hastings acceptance of the
// network's joint proposals.
//
// A phase is one colour class of cells: cells of one colour share no edge, so
// all of them (in every walker) are updated at once; the phases run in order.
// Uniforms come from Philox4x64-10 (Salmon et al., SC'11): key (key, walker),
// counters (pass, cell, 0, 0) and (pass, cell, 1, 0) give eight 64-bit words;
// the high halves are the 8 proposal uniforms, the low half of the first word
// the acceptance uniform.
#include "internal.h"
#include "mlp.h"

namespace ising {

// ---- Philox4x64-10 -----------------------------------------------------------
__device__ __forceinline__ void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t x0 = hi1 ^ c[1] ^ k0, x2 = hi0 ^ c[3] ^ k1;
    c[0] = x0;
    c[1] = lo1;
    c[2] = x2;
    c[3] = lo0;
  }
}

// Last system whose first index (row0 or cell0) is <= v.
template <bool ROWS>
__device__ __forceinline__ int find_system(const SysInfo *sys, int n_sys, int64_t v) {
  int lo = 0, hi = n_sys;  // invariant: answer in [lo, hi)
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    const int64_t first = ROWS ? sys[mid].row0 : sys[mid].cell0;
    if (first <= v) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Boundary fields b_k = h_k + sum_{j outside the cell} J_kj s_j of cell c of slice m.
__device__ __forceinline__ void boundary_fields(const DevTables &T, const SysInfo &sy, const uint32_t *sp, int m,
                                                int c, int b[8]) {
  auto bit = [&](int mm, int q) { return (int)((sp[mm * sy.RS + (q >> 5)] >> (q & 31)) & 1u); };
  const int M = sy.M;
  const int mp = m == 0 ? M - 1 : m - 1, mn = m == M - 1 ? 0 : m + 1;
  const bool has_p = M > 1 && (m > 0 || sy.ring), has_n = M > 1 && (m < M - 1 || sy.ring);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int q = c * 8 + k;
    const TmplSpin ts = T.tmpl[sy.tmpl0 + q];
    int f = ts.h;
    for (int j = 4; j < ts.deg; ++j) f += ts.J[j] * (2 * bit(m, ts.nbr[j]) - 1);  // first 4: in-cell partners
    if (has_p) f += ts.Jtau * (2 * bit(mp, q) - 1);
    if (has_n) f += ts.Jtau * (2 * bit(mn, q) - 1);
    b[k] = f;
  }
}

__device__ __forceinline__ void write_features(float *x, const int b[8], float beta) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    x[k] = 0.f;
    x[8 + k] = (float)b[k] * 0.125f;
  }
  x[16] = beta;
}

// ---- features of the cells of one phase (one row per walker and phase cell) ----
__global__ void cell_features_kernel(DevTables T, DevState St, int32_t n_sys, int64_t rows_total, int32_t phase,
                                     float *X, int8_t *B) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= rows_total) return;
  const SysInfo sy = T.sys[find_system<true>(T.sys, n_sys, row)];
  const int64_t local = row - sy.row0;
  const int w = (int)(local / sy.rows), j = (int)(local % sy.rows);
  float *x = X + row * kIn;
  int8_t *bo = B + row * 8;
  const int count = phase < sy.n_phases ? sy.pc[phase + 1] - sy.pc[phase] : 0;
  if (j >= count) {
    for (int k = 0; k < kIn; ++k) x[k] = 0.f;
    for (int k = 0; k < 8; ++k) bo[k] = 0;
    return;
  }
  const int ci = T.cells[sy.cl0 + sy.pc[phase] + j];
  const int LL = sy.grid_L * sy.grid_L;
  const int m = ci / LL, c = ci - m * LL;
  const uint32_t *sp = St.spins + sy.spin_word0 + (size_t)w * sy.WW;
  int b[8];
  boundary_fields(T, sy, sp, m, c, b);
  write_features(x, b, (float)T.beta[sy.slot0 + St.temp_of[sy.walker0 + w]]);
  for (int k = 0; k < 8; ++k) bo[k] = (int8_t)b[k];
}

hipError_t launch_cell_features(const DevTables &t, const DevState &s, int32_t n_sys, int64_t rows_total,
                                int32_t phase, float *x, int8_t *b, hipStream_t st) {
  if (rows_total <= 0) return hipSuccess;
  hipLaunchKernelGGL(cell_features_kernel, dim3((unsigned)((rows_total + 255) / 256)), dim3(256), 0, st, t, s,
                     n_sys, rows_total, phase, x, b);
  return hipGetLastError();
}

// ---- Metropolis-Hastings acceptance of the proposals of one phase -------------
__device__ __forceinline__ float log_sigmoid_f(float v) { return fminf(v, 0.f) - log1pf(expf(-fabsf(v))); }

// E_c(s) = -sum_k b_k s_k - sum over in-cell edges J s s (bit k of `byte` = spin k is +1).
__device__ __forceinline__ int cell_energy(uint32_t byte, const int b[8], const int jin[16]) {
  int e = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) e -= b[k] * (((byte >> k) & 1u) ? 1 : -1);
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      e -= jin[k * 4 + i] * (((byte >> k) & 1u) ? 1 : -1) * (((byte >> (4 + i)) & 1u) ? 1 : -1);
  return e;
}

__global__ void cell_accept_kernel(DevTables T, DevState St, int32_t n_sys, int64_t rows_total, int32_t phase,
                                   const float *logits, const int8_t *B, uint64_t key, int64_t pass_index,
                                   uint64_t *moves) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool valid = row < rows_total;
  int r = -1, dE = 0;
  bool accept = false;
  if (valid) {
    const SysInfo sy = T.sys[find_system<true>(T.sys, n_sys, row)];
    const int64_t local = row - sy.row0;
    const int w = (int)(local / sy.rows), j = (int)(local % sy.rows);
    const int count = phase < sy.n_phases ? sy.pc[phase + 1] - sy.pc[phase] : 0;
    valid = j < count;
    if (valid) {
      r = sy.walker0 + w;
      const int ci = T.cells[sy.cl0 + sy.pc[phase] + j];
      const int LL = sy.grid_L * sy.grid_L;
      const int m = ci / LL, c = ci - m * LL;
      uint8_t *bytep = (uint8_t *)(St.spins + sy.spin_word0 + (size_t)w * sy.WW + m * sy.RS + ((c * 8) >> 5)) + (c & 3);
      const uint32_t cur = *bytep;
      int b[8], jin[16];
      for (int k = 0; k < 8; ++k) b[k] = B[row * 8 + k];
      for (int k = 0; k < 4; ++k) {
        const int32_t pack = T.tmpl[sy.tmpl0 + c * 8 + k].jpack;  // 2J to partners 4..7
        for (int i = 0; i < 4; ++i) jin[k * 4 + i] = ((int32_t)(int8_t)((pack >> (8 * i)) & 0xff)) / 2;
      }
      float lg[8];
      for (int k = 0; k < 8; ++k) lg[k] = logits[row * kOut + k];
      uint64_t c0[4] = {(uint64_t)pass_index, (uint64_t)ci, 0ull, 0ull};
      uint64_t c1[4] = {(uint64_t)pass_index, (uint64_t)ci, 1ull, 0ull};
      philox4x64(c0, key, (uint64_t)r);
      philox4x64(c1, key, (uint64_t)r);
      const uint64_t wd[8] = {c0[0], c0[1], c0[2], c0[3], c1[0], c1[1], c1[2], c1[3]};
      uint32_t nb = 0;
      float lq_new = 0.f, lq_cur = 0.f;
      for (int k = 0; k < 8; ++k) {
        const float u = (float)(uint32_t)(wd[k] >> 32) * 0x1p-32f;
        const float p = 1.f / (1.f + expf(-lg[k]));
        const bool up = u < p;
        nb |= (up ? 1u : 0u) << k;
        lq_new += log_sigmoid_f(up ? lg[k] : -lg[k]);
        lq_cur += log_sigmoid_f(((cur >> k) & 1u) ? lg[k] : -lg[k]);
      }
      dE = cell_energy(nb, b, jin) - cell_energy(cur, b, jin);
      const float beta = (float)T.beta[sy.slot0 + St.temp_of[r]];
      const float la = -beta * (float)dE + lq_cur - lq_new;
      const float ua = (float)(uint32_t)(wd[0] & 0xffffffffull) * 0x1p-32f;
      accept = la >= 0.f || ua < expf(la);
      if (accept && nb != cur) *bytep = (uint8_t)nb;
      if (!accept) dE = 0;
    }
  }
  // per-walker sums: one atomic per wavefront when its lanes share a walker
  const int r0 = __shfl(r, 0);
  const bool uniform = __all(r == r0);
  if (uniform) {
    if (r0 >= 0) {
      int tot = dE;
      for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
      const unsigned long long na = __popcll(__ballot(valid && accept));
      const unsigned long long nv = __popcll(__ballot(valid));
      if ((threadIdx.x & 63) == 0) {
        if (tot) atomicAdd(&St.energy[r0], tot);
        if (moves) {
          atomicAdd((unsigned long long *)&moves[2 * (size_t)r0], nv);
          atomicAdd((unsigned long long *)&moves[2 * (size_t)r0 + 1], na);
        }
      }
    }
  } else if (valid) {
    if (dE) atomicAdd(&St.energy[r], dE);
    if (moves) {
      atomicAdd((unsigned long long *)&moves[2 * (size_t)r], 1ull);
      if (accept) atomicAdd((unsigned long long *)&moves[2 * (size_t)r + 1], 1ull);
    }
  }
}

hipError_t launch_cell_accept(const DevTables &t, const DevState &s, int32_t n_sys, int64_t rows_total,
                              int32_t phase, const float *logits, const int8_t *b, uint64_t key,
                              int64_t pass_index, uint64_t *moves, hipStream_t st) {
  if (rows_total <= 0) return hipSuccess;
  hipLaunchKernelGGL(cell_accept_kernel, dim3((unsigned)((rows_total + 255) / 256)), dim3(256), 0, st, t, s, n_sys,
                     rows_total, phase, logits, b, key, pass_index, moves);
  return hipGetLastError();
}

// ---- training rows from the current spins ------------------------------------
__global__ void collect_cells_kernel(DevTables T, DevState St, int32_t n_sys, int64_t stride, int64_t offset,
                                     int64_t total_cells, int32_t n, float *X, uint8_t *Y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t g = (offset + (int64_t)i * stride) % total_cells;
  const SysInfo sy = T.sys[find_system<false>(T.sys, n_sys, g)];
  const int LL = sy.grid_L * sy.grid_L;
  const int64_t per_walker = (int64_t)sy.M * LL;
  const int64_t local = g - sy.cell0;
  const int w = (int)(local / per_walker), ci = (int)(local % per_walker);
  const int m = ci / LL, c = ci - m * LL;
  const uint32_t *sp = St.spins + sy.spin_word0 + (size_t)w * sy.WW;
  int b[8];
  boundary_fields(T, sy, sp, m, c, b);
  write_features(X + (int64_t)i * kIn, b, (float)T.beta[sy.slot0 + St.temp_of[sy.walker0 + w]]);
  Y[i] = (uint8_t)((sp[m * sy.RS + ((c * 8) >> 5)] >> ((c * 8) & 31)) & 0xffu);
}

hipError_t launch_collect_cells(const DevTables &t, const DevState &s, int32_t n_sys, int64_t stride,
                                int64_t offset, int64_t total_cells, int32_t n, float *x, uint8_t *y,
                                hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(collect_cells_kernel, dim3((n + 255) / 256), dim3(256), 0, st, t, s, n_sys, stride, offset,
                     total_cells, n, x, y);
  return hipGetLastError();
}

}  // namespace ising
