// Batched FS-QRPPA: K right-hand sides (tau_k, lambda_k) sharing one design
// and one y, iterated together (Algorithm 1 for each k).  The dense part of
// every iteration, V = X~^T Theta (p x K), runs on the int8 matrix cores:
//
//   * X holds the dosage codes (int8, exact);
//   * theta_k is written in fixed point as T_ik = round(theta_ik / c_k * 2^(7S-1))
//     with c_k a power of two >= max_i |theta_ik|, and T is cut into S balanced
//     base-128 digits d_s (|d_s| <= 64), each an int8 "slice" of theta;
//   * v_FIXED = sum_s 128^(S-1-s) * (X^T d_s), every product and sum exact in
//     int32 (|sum| <= n*127*65 < 2^31 for n <= 250k), combined in int64/FP64.
//
// So the only rounding of the batched back-product is the quantisation of
// theta to 7S-1 bits below c_k (S = 3: 2^-20 c_k), instead of FP32 accumulation
// error.  The sparse products X~ B, the prox maps and the dual steps follow the
// single right-hand-side kernels.
#include "pqr_kernels.h"

namespace pqr {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kBS = 3;                  // digit slices of theta
constexpr int kBGroups = 8;             // column groups per workgroup in the GEMM
constexpr int kBRows = 128;             // rows staged in LDS per step
constexpr int kBStride = kBRows + 16;   // padded LDS row stride (bank spread)

// ---------------------------------------------------------------------------
// Digits: T = round(theta / c * 2^(7S-1)), balanced base-128 digits, and the
// exact per-block sums of T (the mean correction uses the same quantised theta).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bdigits(BatchBufs b, int64_t n, int64_t n_pad, int Kp) {
  __shared__ long long red[4];
  const int k = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  long long T = 0;
  if (i < n) {
    const double c = b.scale[k];
    const double t = (double)b.theta[(int64_t)k * n_pad + i] / c * (double)(1 << (7 * kBS - 1));
    T = llrint(t);
    const long long lim = 1ll << (7 * kBS - 1);
    T = T > lim ? lim : (T < -lim ? -lim : T);
  }
  long long rest = T;
  int8_t d[kBS];
#pragma unroll
  for (int s = kBS - 1; s > 0; --s) {
    const long long lo = ((rest + 64) & 127) - 64;
    d[s] = (int8_t)lo;
    rest = (rest - lo) >> 7;
  }
  d[0] = (int8_t)rest;
  if (i < n_pad) {
#pragma unroll
    for (int s = 0; s < kBS; ++s) b.dig[((int64_t)s * Kp + k) * n_pad + i] = d[s];
  }
  // exact block sum of T
  long long v = T;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0)
    b.tpart[(int64_t)blockIdx.x * Kp + k] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_bdsum(BatchBufs b, int nblk, int Kp) {
  const int k = threadIdx.x;
  if (k >= Kp) return;
  long long s = 0;
  for (int q = 0; q < nblk; ++q) s += b.tpart[(int64_t)q * Kp + k];
  b.tsumq[k] = s;
}

// ---------------------------------------------------------------------------
// V = X~^T Theta on the int8 MFMA (16x16x64): one wavefront per 16 right-hand
// sides, kBGroups column groups per workgroup, X staged through LDS; epilogue:
// the weighted soft threshold of eq. beta_update for every (column, k).
// ---------------------------------------------------------------------------
template <int NRT>
__global__ __launch_bounds__(NRT * 64) void k_bgemm(Geom g, BatchBufs b, int Kp) {
  __shared__ __attribute__((aligned(16))) uint8_t xs[kBGroups * kGroup * kBStride];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t grp0 = (int64_t)blockIdx.x * kBGroups;
  const int64_t ng = g.ngroups();
  v4i acc[kBGroups][kBS];
#pragma unroll
  for (int q = 0; q < kBGroups; ++q)
#pragma unroll
    for (int s = 0; s < kBS; ++s) acc[q][s] = v4i{0, 0, 0, 0};
  const int rhs = wv * 16 + (lane & 15);   // B-operand column of this lane
  const int kq = lane >> 4;                // 16-row quarter of a 64-row step
  const int64_t nch = g.nchunks();
  constexpr int kLoads = kBGroups * kGroup * (kBRows / 16);   // uint4 per step
  for (int64_t ch = 0; ch < nch; ++ch) {
    for (int sub = 0; sub < 1024 / kBRows; ++sub) {
      __syncthreads();
      for (int idx = threadIdx.x; idx < kLoads; idx += NRT * 64) {
        const int q = idx / (kGroup * (kBRows / 16));
        const int rem = idx - q * (kGroup * (kBRows / 16));
        const int c = rem / (kBRows / 16), part = rem - c * (kBRows / 16);
        uint4 v = {0u, 0u, 0u, 0u};
        if (grp0 + q < ng)
          v = *reinterpret_cast<const uint4*>(g.seg((grp0 + q) * kGroup + c, ch) + sub * kBRows +
                                              part * 16);
        *reinterpret_cast<uint4*>(&xs[(q * kGroup + c) * kBStride + part * 16]) = v;
      }
      __syncthreads();
      const int64_t rowbase = ch * 1024 + sub * kBRows;
#pragma unroll
      for (int ks = 0; ks < kBRows / 64; ++ks) {
        v4i bf[kBS];
#pragma unroll
        for (int s = 0; s < kBS; ++s) {
          const uint4 t = *reinterpret_cast<const uint4*>(
              b.dig + ((int64_t)s * Kp + rhs) * g.n_pad + rowbase + ks * 64 + kq * 16);
          bf[s] = v4i{(int)t.x, (int)t.y, (int)t.z, (int)t.w};
        }
#pragma unroll
        for (int q = 0; q < kBGroups; ++q) {
          const uint4 t = *reinterpret_cast<const uint4*>(
              &xs[(q * kGroup + (lane & 15)) * kBStride + ks * 64 + kq * 16]);
          const v4i af = v4i{(int)t.x, (int)t.y, (int)t.z, (int)t.w};
#pragma unroll
          for (int s = 0; s < kBS; ++s)
            acc[q][s] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af, bf[s], acc[q][s], 0, 0, 0);
        }
      }
    }
  }
  // epilogue: lane holds columns m = 4*kq + e (e = 0..3) of each group, rhs = this lane's
  const int k = rhs;
  const bool live = k < b.K;
  const double unit = live ? b.scale[k] / (double)(1 << (7 * kBS - 1)) : 0.0;
  const double tq = live ? (double)b.tsumq[k] : 0.0;
  const float lamk = live ? b.lam[k] : 0.f;
#pragma unroll
  for (int q = 0; q < kBGroups; ++q) {
    const int64_t grp = grp0 + q;
    if (grp >= ng) break;
    const float eta = b.geta[grp];
    bool nzany = false;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t j = grp * kGroup + 4 * kq + e;
      long long P = 0;
#pragma unroll
      for (int s = 0; s < kBS; ++s) P = P * 128 + (long long)acc[q][s][e];
      // x~_j^T theta_k = (x_j^T theta_k - m_j sum theta_k) / s_j in the quantised theta
      const double v = ((double)P - (double)b.cm[j] * tq) * unit * (double)b.cinv[j];
      float* bp = b.beta + (int64_t)k * g.p_pad + j;
      if (live) {
        const float bo = *bp;
        const float lj = lamk * b.w[j];
        const float a = eta * bo + (float)v;
        const float bn = (fmaxf(a - lj, 0.f) - fmaxf(-a - lj, 0.f)) / eta;   // eq. beta_update
        *bp = bn;
        nzany |= bn != 0.f;
      }
    }
    const unsigned long long bal = __ballot(nzany);
    if (lane == 0) {
      const uint32_t m16 = (uint32_t)((bal | (bal >> 16) | (bal >> 32) | (bal >> 48)) & 0xffffull);
      b.mask[grp * (Kp / 16) + wv] = m16;
    }
  }
}

// ---------------------------------------------------------------------------
// Union of active groups (any right-hand side), in order; intercepts.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool bflag(const BatchBufs& b, int64_t gi, int nrt) {
  uint32_t m = 0;
  for (int t = 0; t < nrt; ++t) m |= b.mask[gi * nrt + t];
  return m != 0;
}

__global__ __launch_bounds__(1024) void k_bcount(int64_t ngroups, BatchBufs b, int nrt) {
  __shared__ double red[16];
  const int64_t per = (ngroups + kCompactBlocks - 1) / kCompactBlocks;
  const int64_t g0 = (int64_t)blockIdx.x * per, g1 = g0 + per < ngroups ? g0 + per : ngroups;
  double s[1] = {0};
  for (int64_t gi = g0 + threadIdx.x; gi < g1; gi += 1024) s[0] += bflag(b, gi, nrt);
  block_sum<1024, 1, double>(s, red);
  if (threadIdx.x == 0) b.bcnt[blockIdx.x] = (int)s[0];
}

__global__ __launch_bounds__(1024) void k_bscatter(int64_t ngroups, BatchBufs b, int nrt,
                                                   double eta0, int Kp) {
  __shared__ int wcnt[16];
  __shared__ int base_s;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int64_t per = (ngroups + kCompactBlocks - 1) / kCompactBlocks;
  int64_t g0 = (int64_t)blockIdx.x * per;
  const int64_t g1 = g0 + per < ngroups ? g0 + per : ngroups;
  if (g0 > ngroups) g0 = ngroups;
  if (t == 0) {
    int off = 0;
    for (int q = 0; q < (int)blockIdx.x; ++q) off += b.bcnt[q];
    base_s = off;
  }
  __syncthreads();
  int base = base_s;
  for (int64_t tile = g0; tile < g1; tile += 1024) {
    const int64_t gi = tile + t;
    const bool f = gi < g1 && bflag(b, gi, nrt);
    const unsigned long long bal = __ballot(f);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[wid] = __popcll(bal);
    __syncthreads();
    int woff = 0, tot = 0;
    for (int w = 0; w < 16; ++w) { woff += w < wid ? wcnt[w] : 0; tot += wcnt[w]; }
    if (f) b.list[base + woff + before] = (int)gi;
    base += tot;
    __syncthreads();
  }
  if (blockIdx.x == 0) {
    if (t == 0) {
      int total = 0;
      for (int q = 0; q < kCompactBlocks; ++q) total += b.bcnt[q];
      *b.count = total;
    }
    // intercepts (lambda_0 = 0): beta0_k += sum_i theta_ik / eta_0
    for (int k = t; k < b.K; k += 1024) b.beta0[k] += b.tsum[k] / eta0;
  }
}

// ---------------------------------------------------------------------------
// S = X~ B over the union list: one wavefront per row chunk and 4 right-hand
// sides, splits of the list along grid.y, FP64 partials.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int bsplits(int count, int smax, int min_per) {
  const int s = (count + min_per - 1) / min_per;
  return s < 1 ? 1 : (s > smax ? smax : s);
}

__global__ __launch_bounds__(256) void k_baxpy(Geom g, BatchBufs b, int Kp, int smax,
                                               int min_per) {
  const int lane = threadIdx.x & 63;
  const int64_t ch = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int split = blockIdx.y;
  const int k0 = blockIdx.z * 4;
  const int count = *b.count;
  const int seff = bsplits(count, smax, min_per);
  if (split >= seff || ch >= g.nchunks()) return;
  const int per = (count + seff - 1) / seff;
  const int e0 = split * per;
  const int e1 = e0 + per < count ? e0 + per : count;
  const int64_t row0 = ch * 1024 + (int64_t)lane * 16;
  double acc[16][4];
#pragma unroll
  for (int r = 0; r < 16; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[r][q] = 0;
  double off[4] = {0, 0, 0, 0};
  for (int e = e0; e < e1; ++e) {
    const int64_t grp = b.list[e];
    for (int c = 0; c < kGroup; ++c) {
      const int64_t j = grp * kGroup + c;
      double bj[4];
      bool any = false;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        bj[q] = (double)b.beta[(int64_t)(k0 + q) * g.p_pad + j] * (double)b.cinv[j];
        any |= bj[q] != 0.0;
      }
      if (any) {
        double x[16];
        load_rows<I8, 16, double>(g.seg(j, ch), (int64_t)lane * 16, x);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[r][q] = fma(x[r], bj[q], acc[r][q]);
          off[q] = fma((double)b.cm[j], bj[q], off[q]);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double* out = b.partial + ((int64_t)split * Kp + k0 + q) * g.n_pad + row0;
#pragma unroll
    for (int r = 0; r < 16; ++r) out[r] = acc[r][q] - off[q];
  }
}

// ---------------------------------------------------------------------------
// z prox, dual step and per-(block, k) partials; then per-k finalisation.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bupdate(BatchBufs b, int64_t n, int64_t n_pad, int Kp,
                                                 double mu, double sigma, int smax, int min_per) {
  __shared__ double red[8 * 4];
  const int k = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int seff = bsplits(*b.count, smax, min_per);
  double q[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (i < n && k < b.K) {
    double s = b.beta0[k];
    for (int sp = 0; sp < seff; ++sp) s += b.partial[((int64_t)sp * Kp + k) * n_pad + i];
    const int64_t o = (int64_t)k * n_pad + i;
    const float tau = b.tau[k];
    const float muf = (float)mu;
    const float zo = b.z[o], to = b.theta[o], ro = b.r[o];
    const float u = zo + to / muf;
    const float zn = fmaxf(u - (float)(tau / ((double)n * mu)), 0.f) -
                     fmaxf(-u - (float)((1.0 - tau) / ((double)n * mu)), 0.f);   // eq. z_update
    const float rn = (float)(s + (double)zn - (double)b.y[i]);
    const float tn = to - (float)sigma * (2.f * rn - ro);
    b.z[o] = zn;
    b.theta[o] = tn;
    b.r[o] = rn;
    const double dz = (double)zn - zo, dt = (double)tn - to;
    q[0] = (double)tn; q[1] = fabs((double)tn); q[2] = dz * dz; q[3] = dt * dt;
    q[4] = (double)rn * rn;
  }
  // sums for 0, 2, 3, 4 and a max for 1
  double mx = wave_max(q[1]);
  q[1] = 0;
  block_sum<256, 8, double>(q, red);
  __shared__ double mred[4];
  if ((threadIdx.x & 63) == 0) mred[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double* o = b.bpart + ((int64_t)blockIdx.x * Kp + k) * 8;
    o[0] = q[0];
    o[1] = fmax(fmax(mred[0], mred[1]), fmax(mred[2], mred[3]));
    o[2] = q[2]; o[3] = q[3]; o[4] = q[4];
  }
}

__global__ void k_bfinal(BatchBufs b, int nblk, int Kp) {
  const int k = threadIdx.x;
  if (k >= Kp) return;
  double s0 = 0, mx = 0, s2 = 0, s3 = 0, s4 = 0;
  for (int q = 0; q < nblk; ++q) {
    const double* o = b.bpart + ((int64_t)q * Kp + k) * 8;
    s0 += o[0]; mx = fmax(mx, o[1]); s2 += o[2]; s3 += o[3]; s4 += o[4];
  }
  b.tsum[k] = s0;
  // digit scale: the smallest power of two >= max |theta_k| (1 while theta_k = 0)
  int ex = 0;
  const double fr = frexp(mx > 0 ? mx : 1.0, &ex);
  b.scale[k] = ldexp(1.0, fr == 0.5 ? ex - 1 : ex);
  b.norms[k * 4 + 0] = s2;
  b.norms[k * 4 + 1] = s3;
  b.norms[k * 4 + 2] = s4;
}

// ---------------------------------------------------------------------------
hipError_t launch_batch_iteration(const Geom& g, const BatchBufs& b, int Kp, double mu,
                                  double sigma, double eta0, int smax, int min_per,
                                  hipStream_t s) {
  if (g.fmt != I8 || g.rpl != 16 || Kp % 16 || Kp > 128) return hipErrorInvalidValue;
  const unsigned nb = (unsigned)(g.n_pad / 256);
  const int nrt = Kp / 16;
  hipLaunchKernelGGL(k_bdigits, dim3(nb, Kp), dim3(256), 0, s, b, g.n, g.n_pad, Kp);
  hipLaunchKernelGGL(k_bdsum, dim3(1), dim3(128), 0, s, b, (int)nb, Kp);
  const unsigned ngb = (unsigned)((g.ngroups() + kBGroups - 1) / kBGroups);
  switch (nrt) {
    case 1: hipLaunchKernelGGL(k_bgemm<1>, dim3(ngb), dim3(64), 0, s, g, b, Kp); break;
    case 2: hipLaunchKernelGGL(k_bgemm<2>, dim3(ngb), dim3(128), 0, s, g, b, Kp); break;
    case 3: hipLaunchKernelGGL(k_bgemm<3>, dim3(ngb), dim3(192), 0, s, g, b, Kp); break;
    case 4: hipLaunchKernelGGL(k_bgemm<4>, dim3(ngb), dim3(256), 0, s, g, b, Kp); break;
    case 5: hipLaunchKernelGGL(k_bgemm<5>, dim3(ngb), dim3(320), 0, s, g, b, Kp); break;
    case 6: hipLaunchKernelGGL(k_bgemm<6>, dim3(ngb), dim3(384), 0, s, g, b, Kp); break;
    case 7: hipLaunchKernelGGL(k_bgemm<7>, dim3(ngb), dim3(448), 0, s, g, b, Kp); break;
    case 8: hipLaunchKernelGGL(k_bgemm<8>, dim3(ngb), dim3(512), 0, s, g, b, Kp); break;
  }
  hipLaunchKernelGGL(k_bcount, dim3(kCompactBlocks), dim3(1024), 0, s, g.ngroups(), b, nrt);
  hipLaunchKernelGGL(k_bscatter, dim3(kCompactBlocks), dim3(1024), 0, s, g.ngroups(), b, nrt,
                     eta0, Kp);
  hipLaunchKernelGGL(k_baxpy, dim3((unsigned)((g.nchunks() + 3) / 4), smax, Kp / 4), dim3(256), 0,
                     s, g, b, Kp, smax, min_per);
  hipLaunchKernelGGL(k_bupdate, dim3(nb, Kp), dim3(256), 0, s, b, g.n, g.n_pad, Kp, mu, sigma,
                     smax, min_per);
  hipLaunchKernelGGL(k_bfinal, dim3(1), dim3(128), 0, s, b, (int)nb, Kp);
  return hipGetLastError();
}

// Zero start for every right-hand side: beta = 0, z = y, theta = 0, r = 0.
__global__ __launch_bounds__(256) void k_bzero(BatchBufs b, int64_t n_pad, int Kp) {
  const int k = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n_pad; i += (int64_t)gridDim.x * 256) {
    const int64_t o = (int64_t)k * n_pad + i;
    b.z[o] = b.y[i];
    b.theta[o] = 0.f;
    b.r[o] = 0.f;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    b.beta0[k] = 0.0;
    b.tsum[k] = 0.0;
    b.scale[k] = 1.0;
  }
}

hipError_t launch_batch_zero(const Geom& g, const BatchBufs& b, int Kp, hipStream_t s) {
  hipLaunchKernelGGL(k_bzero, dim3(64, Kp), dim3(256), 0, s, b, g.n_pad, Kp);
  return hipGetLastError();
}

}  // namespace pqr
