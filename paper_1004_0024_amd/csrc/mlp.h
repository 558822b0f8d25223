// Layout constants of the learned cell proposal network.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ising {

constexpr int kIn = 17, kHid = 128, kOut = 8;
// FP32 parameter vector: W1[128][17], b1[128], W2[128][128], b2[128], W3[8][128], b3[8]
constexpr int kOW1 = 0;
constexpr int kOB1 = kOW1 + kHid * kIn;
constexpr int kOW2 = kOB1 + kHid;
constexpr int kOB2 = kOW2 + kHid * kHid;
constexpr int kOW3 = kOB2 + kHid;
constexpr int kOB3 = kOW3 + kOut * kHid;
constexpr int kNParams = kOB3 + kOut;  // 19,848
// Packed BF16 copies: W1p[128][32], W2[128][128], W3p[16][128], W3T[128][32], W2T[128][128]
constexpr int kPW1 = 0;
constexpr int kPW2 = kPW1 + 128 * 32;
constexpr int kPW3 = kPW2 + 128 * 128;
constexpr int kPW3T = kPW3 + 16 * 128;
constexpr int kPW2T = kPW3T + 128 * 32;
constexpr int kPackEnd = kPW2T + 128 * 128;  // 43,008
constexpr int kMlpParts = 128;  // most workgroups of one gradient step (partial gradients)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (finite values).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

hipError_t launch_mlp_pack(const float *w, uint16_t *wb, hipStream_t st);
hipError_t launch_mlp_forward(const float *w, const uint16_t *wb, const float *x, int32_t n, float *logits,
                              hipStream_t st);
int mlp_grad_parts(int32_t n);
hipError_t launch_mlp_grad(const float *w, const uint16_t *wb, const float *x, const uint8_t *y, int32_t n,
                           float *part, float *grad, float *loss, hipStream_t st);
// Device address of the library's own partial-gradient rows (kMlpParts x
// (kNParams + 1) floats) on the current device.
hipError_t mlp_scratch_rows(float **rows);
hipError_t launch_adam(float *w, float *m, float *v, const float *g, int32_t n, float lr, float b1, float b2,
                       float eps, int64_t t, hipStream_t st);

}  // namespace ising
