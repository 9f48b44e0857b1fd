// The per-feature scoring network of the learned warm start: 4 -> 64 -> 64 -> 2
// with SiLU activations.  Parameters are kept in FP32 (for the optimiser) and
// used as BF16 (round to nearest even) in every forward and backward pass;
// activations and all accumulations are FP32, per-workgroup gradient partials
// are reduced in a fixed order (deterministic).
//
// Parameter order (4610 floats): W1[64][4], b1[64], W2[64][64], b2[64],
// W3[2][64], b3[2].  Loss per row: w_reg (o0 - t)^2 + w_pos a softplus(-o1)
// + (1 - a) softplus(o1), averaged over the rows.
#include <cmath>
#include <mutex>

#include "pqr_kernels.h"

namespace pqr {

constexpr int kH = 64;
constexpr int oW1 = 0, oB1 = 256, oW2 = 320, oB2 = 4416, oW3 = 4480, oB3 = 4608, kNP = 4610;

__device__ __forceinline__ float bf16_round(float f) {
  const uint32_t u = __float_as_uint(f);
  return __uint_as_float(((u + 0x7fffu + ((u >> 16) & 1u)) >> 16) << 16);
}
__device__ __forceinline__ float sigm(float x) { return 1.0f / (1.0f + __expf(-x)); }
__device__ __forceinline__ float silu(float x) { return x * sigm(x); }
__device__ __forceinline__ float silu_d(float x) {
  const float s = sigm(x);
  return s * (1.0f + x * (1.0f - s));
}
__device__ __forceinline__ float softplus(float x) {
  return x > 20.f ? x : (x < -20.f ? __expf(x) : log1pf(__expf(x)));
}

__device__ __forceinline__ void load_params(const float* __restrict__ P, float* w) {
  for (int i = threadIdx.x; i < kNP; i += blockDim.x) w[i] = bf16_round(P[i]);
  __syncthreads();
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ P,
                                                     const float* __restrict__ F, int64_t B,
                                                     float* __restrict__ out) {
  __shared__ float w[kNP];
  load_params(P, w);
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < B;
       r += (int64_t)gridDim.x * blockDim.x) {
    const float x0 = F[r * 4 + 0], x1 = F[r * 4 + 1], x2 = F[r * 4 + 2], x3 = F[r * 4 + 3];
    float h1[kH];
#pragma unroll
    for (int u = 0; u < kH; ++u) {
      const float a = w[oB1 + u] + w[oW1 + u * 4 + 0] * x0 + w[oW1 + u * 4 + 1] * x1 +
                      w[oW1 + u * 4 + 2] * x2 + w[oW1 + u * 4 + 3] * x3;
      h1[u] = silu(a);
    }
    float o0 = w[oB3 + 0], o1 = w[oB3 + 1];
    for (int u = 0; u < kH; ++u) {
      float a = w[oB2 + u];
#pragma unroll
      for (int k = 0; k < kH; ++k) a = fmaf(w[oW2 + u * kH + k], h1[k], a);
      const float h2 = silu(a);
      o0 = fmaf(w[oW3 + u], h2, o0);
      o1 = fmaf(w[oW3 + kH + u], h2, o1);
    }
    out[r * 2 + 0] = o0;
    out[r * 2 + 1] = o1;
  }
}

// ---------------------------------------------------------------------------
// Gradient: a 64-thread workgroup handles kGTiles tiles of kGT rows; for each
// tile the first kGT threads run one row each (forward and backward) and leave
// the per-row vectors in LDS, then every thread sums the tile's rows, in order,
// for its share of the parameters and writes the tile's partial gradient.
// ---------------------------------------------------------------------------
constexpr int kGT = 32, kGTiles = 4, kGR = kGT * kGTiles, kGThreads = 64;

__global__ __launch_bounds__(kGThreads) void k_mlp_grad(const float* __restrict__ P,
                                                        const float* __restrict__ F,
                                                        const float* __restrict__ tgt,
                                                        const float* __restrict__ act, int64_t B,
                                                        float w_reg, float w_pos, float* part,
                                                        float* lpart) {
  __shared__ float w[kNP];
  __shared__ float sh1[kGT][kH + 1];
  __shared__ float sd2[kGT][kH + 1];
  __shared__ float sd1[kGT][kH + 1];
  __shared__ float sh2[kGT][kH + 1];
  __shared__ float sx[kGT][4];
  __shared__ float sdo[kGT][2];
  __shared__ float lred[kGT];
  load_params(P, w);
  const int t = threadIdx.x;
  const float invB = 1.0f / (float)B;
  for (int tile = 0; tile < kGTiles; ++tile) {
    if (t < kGT) {
      const int64_t r = (int64_t)blockIdx.x * kGR + tile * kGT + t;
      const bool live = r < B;
      float x[4] = {0, 0, 0, 0};
      if (live)
        for (int i = 0; i < 4; ++i) x[i] = F[r * 4 + i];
      float a1[kH], a2[kH];
#pragma unroll
      for (int u = 0; u < kH; ++u) {
        a1[u] = w[oB1 + u] + w[oW1 + u * 4 + 0] * x[0] + w[oW1 + u * 4 + 1] * x[1] +
                w[oW1 + u * 4 + 2] * x[2] + w[oW1 + u * 4 + 3] * x[3];
        sh1[t][u] = silu(a1[u]);
      }
      float o0 = w[oB3 + 0], o1 = w[oB3 + 1];
      for (int u = 0; u < kH; ++u) {
        float a = w[oB2 + u];
        for (int k = 0; k < kH; ++k) a = fmaf(w[oW2 + u * kH + k], sh1[t][k], a);
        a2[u] = a;
        const float h2 = silu(a);
        sh2[t][u] = h2;
        o0 = fmaf(w[oW3 + u], h2, o0);
        o1 = fmaf(w[oW3 + kH + u], h2, o1);
      }
      float d0 = 0.f, d1 = 0.f, loss = 0.f;
      if (live) {
        const float tt = tgt[r], aa = act[r];
        d0 = 2.f * w_reg * (o0 - tt) * invB;
        d1 = (-w_pos * aa * sigm(-o1) + (1.f - aa) * sigm(o1)) * invB;
        loss = (w_reg * (o0 - tt) * (o0 - tt) + w_pos * aa * softplus(-o1) +
                (1.f - aa) * softplus(o1)) * invB;
      }
      sdo[t][0] = d0;
      sdo[t][1] = d1;
      for (int i = 0; i < 4; ++i) sx[t][i] = x[i];
      lred[t] = loss;
      // d a2 = (W3^T d_o) * silu'(a2);  d a1 = (W2^T d a2) * silu'(a1)
#pragma unroll
      for (int u = 0; u < kH; ++u)
        sd2[t][u] = (w[oW3 + u] * d0 + w[oW3 + kH + u] * d1) * silu_d(a2[u]);
      for (int k = 0; k < kH; ++k) {
        float s = 0.f;
        for (int u = 0; u < kH; ++u) s = fmaf(w[oW2 + u * kH + k], sd2[t][u], s);
        sd1[t][k] = s * silu_d(a1[k]);
      }
    }
    __syncthreads();
    float* out = part + ((int64_t)blockIdx.x * kGTiles + tile) * kNP;
    for (int q = t; q < kNP; q += kGThreads) {
      float acc = 0.f;
      if (q < oB1) {                         // W1[u][i]
        const int u = q / 4, i = q % 4;
        for (int rr = 0; rr < kGT; ++rr) acc = fmaf(sd1[rr][u], sx[rr][i], acc);
      } else if (q < oW2) {                  // b1[u]
        const int u = q - oB1;
        for (int rr = 0; rr < kGT; ++rr) acc += sd1[rr][u];
      } else if (q < oB2) {                  // W2[u][k]
        const int u = (q - oW2) / kH, k = (q - oW2) % kH;
        for (int rr = 0; rr < kGT; ++rr) acc = fmaf(sd2[rr][u], sh1[rr][k], acc);
      } else if (q < oW3) {                  // b2[u]
        const int u = q - oB2;
        for (int rr = 0; rr < kGT; ++rr) acc += sd2[rr][u];
      } else if (q < oB3) {                  // W3[c][u]
        const int c = (q - oW3) / kH, u = (q - oW3) % kH;
        for (int rr = 0; rr < kGT; ++rr) acc = fmaf(sdo[rr][c], sh2[rr][u], acc);
      } else {                               // b3[c]
        const int c = q - oB3;
        for (int rr = 0; rr < kGT; ++rr) acc += sdo[rr][c];
      }
      out[q] = acc;
    }
    if (t == 0) {
      float lt = 0.f;
      for (int rr = 0; rr < kGT; ++rr) lt += lred[rr];
      lpart[(int64_t)blockIdx.x * kGTiles + tile] = lt;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_mlp_grad_reduce(const float* part, const float* lpart,
                                                         int nblk, float* grad, float* loss) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q < kNP) {
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * kNP + q];
    grad[q] = s;
  }
  if (q == 0 && loss) {
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += lpart[b];
    *loss = s;
  }
}

__global__ __launch_bounds__(256) void k_adam(float* P, const float* g, float* m, float* v, int n,
                                              float lr, float b1, float b2, float eps, float c1,
                                              float c2) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + (1.f - b1) * gq;
  const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  P[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// Scale-free per-column features: T_j = sqrt(n) S_j / sqrt(tau (1 - tau)) (the
// score z-statistic), m_j / 2 (the allele frequency of a dosage column), tau,
// log(lambda / lambda_max).  Excluded columns get T_j = 0.
__global__ __launch_bounds__(256) void k_features(const double* __restrict__ score,
                                                  const double* __restrict__ cm,
                                                  const double* __restrict__ cinv, int64_t p,
                                                  double n, double tau, double loglam,
                                                  float* F) {
  const double zs = sqrt(n) / sqrt(tau * (1.0 - tau));
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < p; j += (int64_t)gridDim.x * 256) {
    F[j * 4 + 0] = cinv[j] != 0.0 ? (float)(zs * score[j]) : 0.f;
    F[j * 4 + 1] = (float)(0.5 * cm[j]);
    F[j * 4 + 2] = (float)tau;
    F[j * 4 + 3] = (float)loglam;
  }
}

hipError_t launch_mlp_forward(const float* P, const float* F, int64_t B, float* out,
                              hipStream_t s) {
  const int64_t nb = std::min<int64_t>((B + 255) / 256, 4096);
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)std::max<int64_t>(nb, 1)), dim3(256), 0, s, P, F,
                     B, out);
  return hipGetLastError();
}

int mlp_grad_blocks(int64_t B) { return (int)((B + kGR - 1) / kGR); }
int mlp_grad_partials(int64_t B) { return mlp_grad_blocks(B) * kGTiles; }

hipError_t launch_mlp_grad(const float* P, const float* F, const float* t, const float* a,
                           int64_t B, float w_reg, float w_pos, float* part, float* lpart,
                           float* grad, float* loss, hipStream_t s) {
  const int nb = mlp_grad_blocks(B);
  hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(kGThreads), 0, s, P, F, t, a, B, w_reg, w_pos,
                     part, lpart);
  hipLaunchKernelGGL(k_mlp_grad_reduce, dim3((kNP + 255) / 256), dim3(256), 0, s, part, lpart,
                     nb * kGTiles, grad, loss);
  return hipGetLastError();
}

// Scratch of the allocation-free gradient (pqr_mlp_grad_noalloc): the per-tile
// partial gradients and losses of k_mlp_grad for up to kMlpNoAllocRows rows, in a
// file-scope device array (one copy per GPU, held until the process ends).
// k_mlp_grad writes every partial it covers before k_mlp_grad_reduce reads it, so
// nothing has to be cleared between calls; calls that overlap on one GPU share
// the array and race.
constexpr int64_t kNoAllocPartials = (kMlpNoAllocRows + kGR - 1) / kGR * kGTiles;
static __device__ __align__(256) float scratch[kNoAllocPartials * kNP + kNoAllocPartials];

// Device address of `scratch` on the current device, looked up once per device.
hipError_t mlp_noalloc_scratch(float** part, float** lpart) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static float* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<float*>(ptr);
  }
  *part = addr[dev];
  *lpart = addr[dev] + kNoAllocPartials * kNP;
  return hipSuccess;
}

hipError_t launch_adam(float* P, const float* g, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, P, g, m, v, n, lr, b1, b2, eps,
                     c1, c2);
  return hipGetLastError();
}

hipError_t launch_features(const double* score, const double* cm, const double* cinv, int64_t p,
                           double n, double tau, double loglam, float* F, hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3(1024), dim3(256), 0, s, score, cm, cinv, p, n, tau, loglam, F);
  return hipGetLastError();
}

}  // namespace pqr
