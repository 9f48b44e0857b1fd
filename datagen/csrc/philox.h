/* Philox4x32-10 (Salmon et al., SC'11, section 3.2), shared by the host and
 * device twins of the synthetic-input generator.  Pure integer arithmetic:
 * both twins produce identical words for identical (counter, key). */
#ifndef PQRGEN_PHILOX_H
#define PQRGEN_PHILOX_H
#include <stdint.h>

#ifdef __HIPCC__
#define PQRGEN_FN __host__ __device__ static inline
#else
#define PQRGEN_FN static inline
#endif

typedef struct { uint32_t v[4]; } pqrgen_u32x4;

PQRGEN_FN pqrgen_u32x4 pqrgen_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  pqrgen_u32x4 o; o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

/* Genotype entry (i, j): two Bernoulli draws against the integer threshold. */
PQRGEN_FN int8_t pqrgen_dosage(uint32_t i, uint32_t j, uint32_t thr, uint32_t seed, uint32_t tag) {
  pqrgen_u32x4 w = pqrgen_philox(i, j, 2u, 0u, seed, tag);
  return (int8_t)((w.v[0] < thr) + (w.v[1] < thr));
}
#endif
