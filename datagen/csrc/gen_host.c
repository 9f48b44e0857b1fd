/* Host twin of the genotype generator (OpenMP over columns). */
#include <stdint.h>
#include "philox.h"

void pqrgen_philox4x32(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  pqrgen_u32x4 w = pqrgen_philox(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1]);
  for (int k = 0; k < 4; ++k) out[k] = w.v[k];
}

/* Column-major dosages: out[c * ld + i] for rows [0, n) and columns
 * j0 + c, c in [0, ncols); thr[c] is the column's Bernoulli threshold. */
void pqrgen_genotype_i8_host(int8_t* out, int64_t n, int64_t ld, int64_t j0, int64_t ncols,
                             const uint32_t* thr, uint32_t seed, uint32_t tag) {
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < ncols; ++c) {
    const uint32_t t = thr[c];
    const uint32_t j = (uint32_t)(j0 + c);
    int8_t* col = out + c * ld;
    for (int64_t i = 0; i < n; ++i) col[i] = pqrgen_dosage((uint32_t)i, j, t, seed, tag);
  }
}
