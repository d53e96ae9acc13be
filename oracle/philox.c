/*
 * Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11).
 *
 * The paper draws its random numbers from a per-pixel generator
 * (Sec. 5.1.2, where it picks PCG); here a counter-based generator is keyed
 * by (pixel, sample, bounce, dimension block) so that any single
 * path can be regenerated on its own, by the oracle or by the GPU.
 *
 * One round: with multipliers M0 = 0xD2511F53 and M1 = 0xCD9E8D57, take the
 * 64-bit products M0*c0 and M1*c2 and form
 *   (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)).
 * Between rounds the key advances by the Weyl constants (0x9E3779B9,
 * 0xBB67AE85).  Ten rounds.
 *
 * Dimension layout: dimension k of bounce b comes from block floor(k/4)
 * (counter = (pixel, sample, bounce, block)), output word k mod 4.  The key
 * is (seed low 32 bits, seed high 32 bits).  A 32-bit output x maps to the
 * uniform (x >> 8) * 2^-24, exactly representable in float and double.
 */
#include "oracle_internal.h"

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double ouniform(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t bounce, uint32_t dim) {
  uint32_t ctr[4] = {pixel, sample, bounce, dim / 4u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  oracle_philox4x32_10(ctr, key, out);
  return (double)(out[dim % 4u] >> 8) * (1.0 / 16777216.0);
}

double oracle_uniform(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t bounce, uint32_t dim) {
  return ouniform(seed, pixel, sample, bounce, dim);
}
