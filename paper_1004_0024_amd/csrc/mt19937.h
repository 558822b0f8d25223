// MT19937 word recurrence and tempering (Matsumoto & Nishimura 1998), device side.
// The paper generates its uniforms with MT19937 (Section 3, Figure 8).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ising {

// x_n from x_{n-624} (a), x_{n-623} (b) and x_{n-227} (c).
__device__ __forceinline__ uint32_t mt_next_word(uint32_t a, uint32_t b, uint32_t c) {
  const uint32_t y = (a & 0x80000000u) | (b & 0x7fffffffu);
  return c ^ (y >> 1) ^ ((0u - (y & 1u)) & 0x9908b0dfu);
}

// Tempering.  The two masked steps v ^ ((v << s) & C) are one three-input
// bit operation each (truth table 0x78: a ^ (b & c), operand order a, b, c).
__device__ __forceinline__ uint32_t mt_temper(uint32_t v) {
  v ^= v >> 11;
  v = __builtin_amdgcn_bitop3_b32(v, v << 7, 0x9d2c5680u, 0x78);
  v = __builtin_amdgcn_bitop3_b32(v, v << 15, 0xefc60000u, 0x78);
  v ^= v >> 18;
  return v;
}

// init_genrand: word i of the seeded state.
__device__ __forceinline__ uint32_t mt_seed_step(uint32_t prev, uint32_t i) {
  return 1812433253u * (prev ^ (prev >> 30)) + i;
}

}  // namespace ising
