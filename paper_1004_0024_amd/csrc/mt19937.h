// MT19937 word recurrence and tempering (Matsumoto & Nishimura 1998), device side.
// The paper generates its uniforms with MT19937 (Section 3, Figure 8).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ising {

// x_n from x_{n-624} (a), x_{n-623} (b) and x_{n-227} (c).  Two steps are one
// three-input bit operation each: the top bit of a joined to the low 31 bits
// of b (truth table 0xe4: (a & m) | (b & ~m), operand order a, b, m), and
// c ^ (odd ? 0x9908b0df : 0) from the all-ones or zero word of y's low bit
// (truth table 0x6c: (o & k) ^ c, operand order o, c, k).
__device__ __forceinline__ uint32_t mt_next_word(uint32_t a, uint32_t b, uint32_t c) {
  const uint32_t y = __builtin_amdgcn_bitop3_b32(a, b, 0x80000000u, 0xe4);
  const uint32_t odd = (uint32_t)__builtin_amdgcn_sbfe((int)y, 0u, 1u);
  return __builtin_amdgcn_bitop3_b32(odd, c, 0x9908b0dfu, 0x6c) ^ (y >> 1);
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
