// Counter-based random numbers for the Gaussian test blocks Omega_i of the
// randomised SVD (Sec. 2) when a caller gives a seed instead of the blocks.
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC 2011): ten rounds of two 32x32->64-bit products with the
// multipliers 0xD2511F53 / 0xCD9E8D57, the key bumped by 0x9E3779B9 /
// 0xBB67AE85 between rounds.
#pragma once

#include <cstdint>

namespace rng {

void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

// Block Omega of (level, box): s x m_in complex values, row-major (sample t,
// interface node j at t * m_in + j), entries CN(0, 1).  Value v uses counter
// (v, box, level, 0x4f4d4547) and key (seed low, seed high); the four output
// words give two uniforms in (0, 1) of 53 bits, and Box-Muller gives the real
// and imaginary parts, each scaled by 1/sqrt(2).  Interleaved (re, im) doubles.
void omega_block(uint64_t seed, int level, int box, int m_in, int s, double* out);

}  // namespace rng
