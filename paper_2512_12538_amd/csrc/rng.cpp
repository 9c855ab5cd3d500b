// Philox4x32-10 and the Gaussian test blocks; see rng.h.
#include "rng.h"

#include <cmath>

namespace rng {

void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

namespace {
// 53-bit uniform in (0, 1) from two words
double unit(uint32_t hi, uint32_t lo) {
  const uint64_t v = (((uint64_t)hi << 32) | lo) >> 11;
  return ((double)v + 0.5) * (1.0 / 9007199254740992.0);
}
}  // namespace

void omega_block(uint64_t seed, int level, int box, int m_in, int s, double* out) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  const long long n = (long long)m_in * s;
  const double two_pi = 6.283185307179586476925286766559;
  for (long long v = 0; v < n; ++v) {
    const uint32_t ctr[4] = {(uint32_t)v, (uint32_t)box, (uint32_t)level, 0x4f4d4547u};
    uint32_t w[4];
    philox4x32_10(ctr, key, w);
    const double u1 = unit(w[0], w[1]), u2 = unit(w[2], w[3]);
    const double r = std::sqrt(-2.0 * std::log(u1)) * 0.70710678118654752440084436210485;
    out[2 * v] = r * std::cos(two_pi * u2);
    out[2 * v + 1] = r * std::sin(two_pi * u2);
  }
}

}  // namespace rng
