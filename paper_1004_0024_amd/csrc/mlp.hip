// Learned cell proposal: the 17 -> 128 -> 128 -> 8 ReLU network on BF16 matrix
// cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation), its training step
// (forward + backward in one workgroup, then Adam on FP32 master weights).
//
// Parameter vector (FP32, 19,848 values): W1[128][17], b1[128], W2[128][128],
// b2[128], W3[8][128], b3[8].  The kernels read BF16 copies packed as
//   W1p[128][32] (input padded to 32), W2[128][128], W3p[16][128] (outputs
//   padded to 16), W3T[128][32] (transpose, padded), W2T[128][128].
// Inputs x = [8 zeros, b/8 (8 boundary fields), beta], padded with zeros to 32.
// Every product rounds its operands to BF16 (round to nearest even) and sums
// in FP32; activations are stored as BF16 between layers.
#include "internal.h"
#include "mlp.h"

namespace ising {

// acc[16x16] += A[16 x 32] * B[32 x 16].  A is row-major [i][k] with row stride
// sa, B is given as its transpose Bt [n][k] with row stride sb (both in BF16
// elements, strides multiples of 8).  Lane l supplies A[l%16][8(l/16) .. +8)
// and Bt[l%16][8(l/16) .. +8); element j of the result in lane l is
// D[4(l/16) + j][l%16].
__device__ __forceinline__ f32x4 mma(const uint16_t *A, int sa, const uint16_t *Bt, int sb, f32x4 acc) {
  const int l = threadIdx.x & 63;
  const bf16x8 a = *(const bf16x8 *)(A + (l & 15) * sa + ((l >> 4) << 3));
  const bf16x8 b = *(const bf16x8 *)(Bt + (l & 15) * sb + ((l >> 4) << 3));
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
}

// ---- FP32 master weights -> packed BF16 copies ----------------------------
__global__ void mlp_pack_kernel(const float *w, uint16_t *wb) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kPackEnd; i += gridDim.x * blockDim.x) {
    float v = 0.f;
    if (i < kPW2) {  // W1p[128][32]
      const int r = i / 32, c = i % 32;
      v = c < kIn ? w[kOW1 + r * kIn + c] : 0.f;
    } else if (i < kPW3) {  // W2[128][128]
      v = w[kOW2 + (i - kPW2)];
    } else if (i < kPW3T) {  // W3p[16][128]
      const int r = (i - kPW3) / 128, c = (i - kPW3) % 128;
      v = r < kOut ? w[kOW3 + r * 128 + c] : 0.f;
    } else if (i < kPW2T) {  // W3T[128][32]
      const int r = (i - kPW3T) / 32, c = (i - kPW3T) % 32;
      v = c < kOut ? w[kOW3 + c * 128 + r] : 0.f;
    } else {  // W2T[128][128]
      const int r = (i - kPW2T) / 128, c = (i - kPW2T) % 128;
      v = w[kOW2 + c * 128 + r];
    }
    wb[i] = f2bf(v);
  }
}

hipError_t launch_mlp_pack(const float *w, uint16_t *wb, hipStream_t st) {
  hipLaunchKernelGGL(mlp_pack_kernel, dim3(64), dim3(256), 0, st, w, wb);
  return hipGetLastError();
}

// ---- shared forward pieces --------------------------------------------------
struct alignas(16) FwdLds {
  uint16_t W1[128 * 32], W2[128 * 128], W3[16 * 128];
  float b1[128], b2[128], b3[16];
};

__device__ void load_forward_weights(FwdLds &s, const float *w, const uint16_t *wb) {
  for (int i = threadIdx.x; i < 128 * 32; i += blockDim.x) s.W1[i] = wb[kPW1 + i];
  for (int i = threadIdx.x; i < 128 * 128; i += blockDim.x) s.W2[i] = wb[kPW2 + i];
  for (int i = threadIdx.x; i < 16 * 128; i += blockDim.x) s.W3[i] = wb[kPW3 + i];
  for (int i = threadIdx.x; i < 128; i += blockDim.x) {
    s.b1[i] = w[kOB1 + i];
    s.b2[i] = w[kOB2 + i];
  }
  for (int i = threadIdx.x; i < 16; i += blockDim.x) s.b3[i] = i < kOut ? w[kOB3 + i] : 0.f;
}

// One wavefront: logits of 32 rows whose BF16 inputs sit in X[32][32].
// H1, H2 are [32][128] scratch; out(row, k, value) receives the 8 logits.
template <typename Out>
__device__ void forward_rows(const FwdLds &s, const uint16_t *X, uint16_t *H1, uint16_t *H2, Out out) {
  const int l = threadIdx.x & 63;
  const int col16 = l & 15, row4 = (l >> 4) << 2;
  for (int rg = 0; rg < 2; ++rg)
    for (int ct = 0; ct < 8; ++ct) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mma(X + rg * 16 * 32, 32, s.W1 + ct * 16 * 32, 32, acc);
      const int c = ct * 16 + col16;
#pragma unroll
      for (int j = 0; j < 4; ++j) H1[(rg * 16 + row4 + j) * 128 + c] = f2bf(fmaxf(acc[j] + s.b1[c], 0.f));
    }
  wave_fence();
  for (int rg = 0; rg < 2; ++rg)
    for (int ct = 0; ct < 8; ++ct) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) acc = mma(H1 + rg * 16 * 128 + kk * 32, 128, s.W2 + ct * 16 * 128 + kk * 32, 128, acc);
      const int c = ct * 16 + col16;
#pragma unroll
      for (int j = 0; j < 4; ++j) H2[(rg * 16 + row4 + j) * 128 + c] = f2bf(fmaxf(acc[j] + s.b2[c], 0.f));
    }
  wave_fence();
  for (int rg = 0; rg < 2; ++rg) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) acc = mma(H2 + rg * 16 * 128 + kk * 32, 128, s.W3 + kk * 32, 128, acc);
    if (col16 < kOut) {
#pragma unroll
      for (int j = 0; j < 4; ++j) out(rg * 16 + row4 + j, col16, acc[j] + s.b3[col16]);
    }
  }
  wave_fence();
}

// ---- forward over rows of FP32 inputs x[n][17] ------------------------------
__global__ void __launch_bounds__(256) mlp_forward_kernel(const float *w, const uint16_t *wb, const float *x,
                                                          int32_t n, float *logits) {
  __shared__ FwdLds s;
  __shared__ __attribute__((aligned(16))) uint16_t Xs[4][32 * 32];
  __shared__ __attribute__((aligned(16))) uint16_t H1s[4][32 * 128], H2s[4][32 * 128];
  load_forward_weights(s, w, wb);
  __syncthreads();
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int tiles = (n + 31) / 32;
  for (int tile = blockIdx.x * 4 + wv; tile < tiles; tile += gridDim.x * 4) {
    const int r0 = tile * 32;
    for (int e = l; e < 32 * 32; e += 64) {
      const int r = e >> 5, c = e & 31;
      const float v = (r0 + r < n && c < kIn) ? x[(size_t)(r0 + r) * kIn + c] : 0.f;
      Xs[wv][e] = f2bf(v);
    }
    wave_fence();
    forward_rows(s, Xs[wv], H1s[wv], H2s[wv], [&](int r, int k, float v) {
      if (r0 + r < n) logits[(size_t)(r0 + r) * kOut + k] = v;
    });
  }
}

hipError_t launch_mlp_forward(const float *w, const uint16_t *wb, const float *x, int32_t n, float *logits,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int tiles = (n + 31) / 32;
  const int blocks = std::min(1024, (tiles + 3) / 4);
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(blocks), dim3(256), 0, st, w, wb, x, n, logits);
  return hipGetLastError();
}

// ---- training: forward + backward, partial gradients per workgroup ----------
// Workgroup p of P takes the 32-row tiles p, p + P, p + 2P, ... of the batch and
// writes the gradient of its rows (and its loss sum) to part[p]; a second
// kernel adds the P partials in order.  No atomics: every sum has one owner
// and a fixed order, so the result depends only on the batch.
struct alignas(16) GradLds {
  uint16_t W1[128 * 32], W2[128 * 128], W3[16 * 128], W3T[128 * 32], W2T[128 * 128];
  uint16_t X[32 * 32], XT[32 * 32], H1[32 * 128], H1T[128 * 32], H2[32 * 128], H2T[128 * 32];
  uint16_t DL[32 * 32], DLT[16 * 32], DZ2[32 * 128], DZ2T[128 * 32], DZ1T[128 * 32];
  float b1[128], b2[128], b3[16];
  float db1[128], db2[128], db3w[2][16], lossw[2];
};

__device__ __forceinline__ float log_sigmoid(float v) { return fminf(v, 0.f) - log1pf(expf(-fabsf(v))); }

// Sum over the four 16-lane groups of a wavefront (lanes l, l+16, l+32, l+48).
__device__ __forceinline__ float sum_groups(float v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

__global__ void __launch_bounds__(256) mlp_grad_kernel(const float *w, const uint16_t *wb, const float *x,
                                                       const uint8_t *y, int32_t n, float *part) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds_raw[];
  GradLds &s = *reinterpret_cast<GradLds *>(lds_raw);
  const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
  const int col16 = l & 15, row4 = (l >> 4) << 2;
  for (int i = tid; i < 128 * 32; i += 256) {
    s.W1[i] = wb[kPW1 + i];
    s.W3T[i] = wb[kPW3T + i];
  }
  for (int i = tid; i < 128 * 128; i += 256) {
    s.W2[i] = wb[kPW2 + i];
    s.W2T[i] = wb[kPW2T + i];
  }
  for (int i = tid; i < 16 * 128; i += 256) s.W3[i] = wb[kPW3 + i];
  for (int i = tid; i < 128; i += 256) {
    s.b1[i] = w[kOB1 + i];
    s.b2[i] = w[kOB2 + i];
    s.db1[i] = 0.f;
    s.db2[i] = 0.f;
  }
  if (tid < 16) s.b3[tid] = tid < kOut ? w[kOB3 + tid] : 0.f;
  if (tid < 32) s.db3w[tid >> 4][tid & 15] = 0.f;
  if (tid < 2) s.lossw[tid] = 0.f;
  for (int i = tid; i < 32 * 32; i += 256) s.DL[i] = 0;
  for (int i = tid; i < 16 * 32; i += 256) s.DLT[i] = 0;
  f32x4 gW3[2], gW2[16], gW1[4];
  for (int i = 0; i < 2; ++i) gW3[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < 16; ++i) gW2[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < 4; ++i) gW1[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  const float inv_n = 1.f / (float)n;
  __syncthreads();

  for (int r0 = blockIdx.x * 32; r0 < n; r0 += gridDim.x * 32) {
    // inputs, both layouts
    for (int e = tid; e < 32 * 32; e += 256) {
      const int r = e >> 5, c = e & 31;
      const uint16_t v = f2bf((r0 + r < n && c < kIn) ? x[(size_t)(r0 + r) * kIn + c] : 0.f);
      s.X[e] = v;
      s.XT[c * 32 + r] = v;
    }
    __syncthreads();
    // layer 1: wave wv owns column tiles 2wv, 2wv+1
    for (int rg = 0; rg < 2; ++rg)
      for (int cc = 0; cc < 2; ++cc) {
        const int ct = 2 * wv + cc;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma(s.X + rg * 16 * 32, 32, s.W1 + ct * 16 * 32, 32, acc);
        const int c = ct * 16 + col16;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = rg * 16 + row4 + j;
          const uint16_t v = f2bf(fmaxf(acc[j] + s.b1[c], 0.f));
          s.H1[r * 128 + c] = v;
          s.H1T[c * 32 + r] = v;
        }
      }
    __syncthreads();
    // layer 2
    for (int rg = 0; rg < 2; ++rg)
      for (int cc = 0; cc < 2; ++cc) {
        const int ct = 2 * wv + cc;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc = mma(s.H1 + rg * 16 * 128 + kk * 32, 128, s.W2 + ct * 16 * 128 + kk * 32, 128, acc);
        const int c = ct * 16 + col16;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = rg * 16 + row4 + j;
          const uint16_t v = f2bf(fmaxf(acc[j] + s.b2[c], 0.f));
          s.H2[r * 128 + c] = v;
          s.H2T[c * 32 + r] = v;
        }
      }
    __syncthreads();
    // layer 3 and the loss gradient dl = (sigmoid(l) - y) / n; wave wv < 2 owns rows 16wv ..
    if (wv < 2) {
      const int rg = wv;
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) acc = mma(s.H2 + rg * 16 * 128 + kk * 32, 128, s.W3 + kk * 32, 128, acc);
      float dsum = 0.f, lsum = 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = rg * 16 + row4 + j;
        float dl = 0.f;
        if (col16 < kOut && r0 + r < n) {
          const float lg = acc[j] + s.b3[col16];
          const float yk = (float)((y[r0 + r] >> col16) & 1u);
          dl = (1.f / (1.f + expf(-lg)) - yk) * inv_n;
          lsum -= yk > 0.f ? log_sigmoid(lg) : log_sigmoid(-lg);
          dsum += dl;
        }
        if (col16 < kOut) {
          const uint16_t v = f2bf(dl);
          s.DL[r * 32 + col16] = v;
          s.DLT[col16 * 32 + r] = v;
        }
      }
      dsum = sum_groups(dsum);
      for (int off = 1; off < 16; off <<= 1) lsum += __shfl_xor(lsum, off);
      lsum = sum_groups(lsum);
      if (l < 16) s.db3w[wv][l] += dsum;
      if (l == 0) s.lossw[wv] += lsum;
    }
    __syncthreads();
    // dW3 += dl^T H2 (wave: column tiles 2wv, 2wv+1); dZ2 = (dl W3) * [H2 > 0]
    for (int cc = 0; cc < 2; ++cc) gW3[cc] = mma(s.DLT, 32, s.H2T + (2 * wv + cc) * 16 * 32, 32, gW3[cc]);
    for (int cc = 0; cc < 2; ++cc) {
      const int ct = 2 * wv + cc;
      const int c = ct * 16 + col16;
      float bsum = 0.f;
      for (int rg = 0; rg < 2; ++rg) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma(s.DL + rg * 16 * 32, 32, s.W3T + ct * 16 * 32, 32, acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = rg * 16 + row4 + j;
          const float g = (s.H2[r * 128 + c] & 0x7FFF) != 0 ? acc[j] : 0.f;
          const uint16_t v = f2bf(g);
          s.DZ2[r * 128 + c] = v;
          s.DZ2T[c * 32 + r] = v;
          bsum += bf2f(v);
        }
      }
      bsum = sum_groups(bsum);
      if (l < 16) s.db2[c] += bsum;  // column c belongs to this wavefront only
    }
    __syncthreads();
    // dW2 += dZ2^T H1 (wave: row tiles 2wv, 2wv+1 of dW2); dZ1 = (dZ2 W2) * [H1 > 0]
    for (int rr = 0; rr < 2; ++rr)
      for (int ct = 0; ct < 8; ++ct)
        gW2[rr * 8 + ct] = mma(s.DZ2T + (2 * wv + rr) * 16 * 32, 32, s.H1T + ct * 16 * 32, 32, gW2[rr * 8 + ct]);
    for (int cc = 0; cc < 2; ++cc) {
      const int ct = 2 * wv + cc;
      const int c = ct * 16 + col16;
      float bsum = 0.f;
      for (int rg = 0; rg < 2; ++rg) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
          acc = mma(s.DZ2 + rg * 16 * 128 + kk * 32, 128, s.W2T + ct * 16 * 128 + kk * 32, 128, acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = rg * 16 + row4 + j;
          const float g = (s.H1[r * 128 + c] & 0x7FFF) != 0 ? acc[j] : 0.f;
          const uint16_t v = f2bf(g);
          s.DZ1T[c * 32 + r] = v;
          bsum += bf2f(v);
        }
      }
      bsum = sum_groups(bsum);
      if (l < 16) s.db1[c] += bsum;
    }
    __syncthreads();
    // dW1 += dZ1^T X (wave: row tiles 2wv, 2wv+1 of dW1, both column tiles)
    for (int rr = 0; rr < 2; ++rr)
      for (int ct = 0; ct < 2; ++ct)
        gW1[rr * 2 + ct] = mma(s.DZ1T + (2 * wv + rr) * 16 * 32, 32, s.XT + ct * 16 * 32, 32, gW1[rr * 2 + ct]);
    __syncthreads();
  }
  // ---- this workgroup's partial gradient and loss sum ----
  float *g = part + (size_t)blockIdx.x * (kNParams + 1);
  for (int cc = 0; cc < 2; ++cc) {
    const int c = (2 * wv + cc) * 16 + col16;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = row4 + j;  // output feature of layer 3 (rows 8..15 are padding)
      if (r < kOut) g[kOW3 + r * 128 + c] = gW3[cc][j];
    }
  }
  for (int rr = 0; rr < 2; ++rr)
    for (int ct = 0; ct < 8; ++ct) {
      const int c = ct * 16 + col16;
#pragma unroll
      for (int j = 0; j < 4; ++j) g[kOW2 + ((2 * wv + rr) * 16 + row4 + j) * 128 + c] = gW2[rr * 8 + ct][j];
    }
  for (int rr = 0; rr < 2; ++rr)
    for (int ct = 0; ct < 2; ++ct) {
      const int c = ct * 16 + col16;
      if (c < kIn) {
#pragma unroll
        for (int j = 0; j < 4; ++j) g[kOW1 + ((2 * wv + rr) * 16 + row4 + j) * kIn + c] = gW1[rr * 2 + ct][j];
      }
    }
  __syncthreads();
  for (int i = tid; i < 128; i += 256) {
    g[kOB1 + i] = s.db1[i];
    g[kOB2 + i] = s.db2[i];
  }
  if (tid < kOut) g[kOB3 + tid] = s.db3w[0][tid] + s.db3w[1][tid];
  if (tid == 0) g[kNParams] = s.lossw[0] + s.lossw[1];
}

// grad[i] = sum over p of part[p][i]; loss = (sum of loss sums) / n.  Block:
// 64 entries x 4 lanes; lane group k adds parts p = k, k + 4, ... in order,
// then the four sums are added k = 0..3.  The order depends only on P.
__global__ void __launch_bounds__(256) mlp_reduce_kernel(const float *part, int32_t P, int32_t n, float *grad,
                                                         float *loss) {
  __shared__ float red[4][64];
  const int k = threadIdx.x >> 6, e = threadIdx.x & 63;
  const int i = blockIdx.x * 64 + e;
  float v = 0.f;
  if (i <= kNParams) {
#pragma unroll 8
    for (int p = k; p < P; p += 4) v += part[(size_t)p * (kNParams + 1) + i];
  }
  red[k][e] = v;
  __syncthreads();
  if (k == 0 && i <= kNParams) {
    const float t = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
    if (i < kNParams) grad[i] = t;
    else if (loss) loss[0] = t / (float)n;
  }
}

int mlp_grad_parts(int32_t n) { return std::max(1, std::min(kMlpParts, (n + 31) / 32)); }

hipError_t launch_mlp_grad(const float *w, const uint16_t *wb, const float *x, const uint8_t *y, int32_t n,
                           float *part, float *grad, float *loss, hipStream_t st) {
  static std::atomic<uint64_t> attr{0};
  hipError_t e = allow_lds(mlp_grad_kernel, (int)sizeof(GradLds), attr);
  if (e != hipSuccess) return e;
  const int P = mlp_grad_parts(n);
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(P), dim3(256), sizeof(GradLds), st, w, wb, x, y, n, part);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kNParams + 1 + 63) / 64), dim3(256), 0, st, part, P, n, grad, loss);
  return hipGetLastError();
}

// ---- Adam on the FP32 master weights ------------------------------------------
__global__ void adam_kernel(float *w, float *m, float *v, const float *g, int32_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

hipError_t launch_adam(float *w, float *m, float *v, const float *g, int32_t n, float lr, float b1, float b2,
                       float eps, int64_t t, hipStream_t st) {
  const float c1 = 1.f - (float)pow((double)b1, (double)t);
  const float c2 = 1.f - (float)pow((double)b2, (double)t);
  hipLaunchKernelGGL(adam_kernel, dim3(80), dim3(256), 0, st, w, m, v, g, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

// ---- gradient step without caller scratch ------------------------------------
// The partial gradients of mlp_grad_kernel in a fixed device array, for callers
// that cannot allocate (graph capture, serving loops): kMlpParts rows of
// kNParams + 1 floats, 10,162,688 bytes per GPU, held until the process ends.
// Every launch writes each entry of the rows it uses (its kNParams + 1 floats)
// and the reduction reads only those rows, so nothing needs clearing between
// calls; two calls that overlap on one GPU share the rows and race.
static __device__ __align__(256) float scratch[kMlpParts * (kNParams + 1)];

// Device address of `scratch` on each device, looked up once per device with
// that device current (the array's host-side name is not a device address).
static std::atomic<float *> scratch_ptr[64];

hipError_t mlp_scratch_rows(float **rows) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  float *p = scratch_ptr[dev].load(std::memory_order_acquire);
  if (!p) {
    void *q = nullptr;
    e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    p = (float *)q;
    scratch_ptr[dev].store(p, std::memory_order_release);
  }
  *rows = p;
  return hipSuccess;
}

}  // namespace ising
