/* Device twin of the genotype generator: one thread per entry, column-major
 * output with leading dimension ld (bytes).  Rows in [n, ld) are left as is. */
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "philox.h"

__global__ void pqrgen_genotype_kernel(int8_t* __restrict__ out, int64_t n, int64_t ld, int64_t j0,
                                       int64_t ncols, const uint32_t* __restrict__ thr,
                                       uint32_t seed, uint32_t tag) {
  const int64_t c = blockIdx.y + (int64_t)gridDim.y * blockIdx.z;
  if (c >= ncols) return;
  const uint32_t t = thr[c];
  const uint32_t j = (uint32_t)(j0 + c);
  int8_t* col = out + c * ld;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    col[i] = pqrgen_dosage((uint32_t)i, j, t, seed, tag);
}

extern "C" int pqrgen_genotype_i8_device(int8_t* out, int64_t n, int64_t ld, int64_t j0,
                                         int64_t ncols, const uint32_t* thr, uint32_t seed,
                                         uint32_t tag, void* stream) {
  if (n <= 0 || ncols <= 0) return 0;
  if (ld < n || !out || !thr) return 1;
  const int threads = 256;
  int64_t bx = (n + threads - 1) / threads;
  if (bx > 64) bx = 64;
  const int64_t gy = ncols < 65535 ? ncols : 65535;
  const int64_t gz = (ncols + gy - 1) / gy;
  hipLaunchKernelGGL(pqrgen_genotype_kernel, dim3((unsigned)bx, (unsigned)gy, (unsigned)gz),
                     dim3(threads), 0, (hipStream_t)stream, out, n, ld, j0, ncols, thr, seed, tag);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}
