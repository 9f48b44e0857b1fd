// Set-up kernels: encode the design store, column statistics, the Lanczos
// estimate of Lambda_max(X~_g^T X~_g) for all blocks at once, the null-fit
// dual used by lambda_max, and the back-transform of the coefficients.
#include <cmath>

#include "pqr_kernels.h"

namespace pqr {

// ---------------------------------------------------------------------------
// Encode: column-major source (ld elements per column) -> padded store.
// One thread per 4 consecutive rows of one column.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float src_value(const void* src, int src_fmt, int64_t idx) {
  if (src_fmt == F64) return (float)static_cast<const double*>(src)[idx];
  if (src_fmt == F32) return static_cast<const float*>(src)[idx];
  return (float)static_cast<const uint8_t*>(src)[idx];
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__global__ __launch_bounds__(256) void k_encode(const void* __restrict__ src, int src_fmt,
                                                int64_t ld, Geom g, uint8_t* __restrict__ dst) {
  const int64_t quads = g.n_pad / 4;
  const int64_t total = quads * g.p_pad;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * 256) {
    const int64_t j = t / quads, qd = t - j * quads, i0 = qd * 4;
    // point `col` so that col + (bytes of row i0) is row i0's place in its segment
    const int64_t rows_per_seg = (int64_t)kWave * g.rpl;
    const int64_t ch = i0 / rows_per_seg;
    uint8_t* col = dst + (g.seg(j, ch) - g.X) - fmt_col_bytes(g.fmt, ch * rows_per_seg);
    if (g.fmt == F64 && src_fmt == F64) {   // exact copy, no float round trip
      for (int k = 0; k < 4; ++k) {
        const int64_t i = i0 + k;
        reinterpret_cast<double*>(col)[i] =
            (j < g.p && i < g.n) ? static_cast<const double*>(src)[j * ld + i] : 0.0;
      }
      continue;
    }
    float v[4];
    for (int k = 0; k < 4; ++k) {
      const int64_t i = i0 + k;
      v[k] = (j < g.p && i < g.n) ? src_value(src, src_fmt, j * ld + i) : 0.0f;
    }
    switch (g.fmt) {
      case F64:
        for (int k = 0; k < 4; ++k) reinterpret_cast<double*>(col)[i0 + k] = (double)v[k];
        break;
      case F32:
        for (int k = 0; k < 4; ++k) reinterpret_cast<float*>(col)[i0 + k] = v[k];
        break;
      case BF16:
        for (int k = 0; k < 4; ++k) reinterpret_cast<uint16_t*>(col)[i0 + k] = f32_to_bf16_rne(v[k]);
        break;
      case FP8: {
        int w = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], 0, false);
        w = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], w, true);
        reinterpret_cast<uint32_t*>(col)[i0 / 4] = (uint32_t)w;
        break;
      }
      case I8: {
        uint32_t w = 0;
        for (int k = 0; k < 4; ++k) w |= ((uint32_t)(uint8_t)v[k]) << (8 * k);
        reinterpret_cast<uint32_t*>(col)[i0 / 4] = w;
        break;
      }
      case B2: {
        // row i lives in byte i/4 at bits 2*(i%4): byte b of a 32-bit word holds rows 4b..4b+3
        uint32_t c = 0;
        for (int k = 0; k < 4; ++k) {
          uint32_t code = (uint32_t)v[k];
          code = code > 3u ? 3u : code;
          c |= code << (2 * k);
        }
        col[i0 / 4] = (uint8_t)c;
        break;
      }
    }
  }
}

hipError_t launch_encode(const void* src, int src_fmt, int64_t ld, const Geom& g, uint8_t* dst,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_encode, dim3(8192), dim3(256), 0, s, src, src_fmt, ld, g, dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Column sums and sums of squares of the stored values (double; exact for
// integer codes).  One wavefront per 16-column group.
// ---------------------------------------------------------------------------
template <int FMT, int RPL>
__global__ __launch_bounds__(256) void k_colstats(Geom g, double* sum, double* sumsq) {
  const int lane = threadIdx.x & 63;
  const int64_t grp = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (grp >= g.ngroups()) return;
  double a[kGroup], b[kGroup];
#pragma unroll
  for (int c = 0; c < kGroup; ++c) a[c] = b[c] = 0;
  for (int64_t ch = 0; ch < g.nchunks(); ++ch) {
    const uint8_t* base = g.seg(grp * kGroup, ch);
#pragma unroll
    for (int c = 0; c < kGroup; ++c) {
      double x[RPL];
      load_rows<FMT, RPL, double>(base + c * g.seg_bytes, (int64_t)lane * RPL, x);
#pragma unroll
      for (int r = 0; r < RPL; ++r) { a[c] += x[r]; b[c] = fma(x[r], x[r], b[c]); }
    }
  }
  const double sa = reduce16(a, lane), sb = reduce16(b, lane);
  if ((lane & 3) == 0) {
    const int64_t j = grp * kGroup + group_col_of_lane(lane);
    sum[j] = sa;
    sumsq[j] = sb;
  }
}

template <int FMT, int RPL>
static void colstats_fmt(const Geom& g, double* sum, double* sumsq, hipStream_t s) {
  hipLaunchKernelGGL((k_colstats<FMT, RPL>), dim3((unsigned)((g.ngroups() + 3) / 4)), dim3(256), 0,
                     s, g, sum, sumsq);
}

#define PQR_DISPATCH_S(FN, ...)                                          \
  switch (g.fmt * 2 + (g.rpl == 16)) {                                   \
    case F64 * 2: FN<F64, 4>(__VA_ARGS__); break;                        \
    case F64 * 2 + 1: FN<F64, 16>(__VA_ARGS__); break;                   \
    case F32 * 2: FN<F32, 4>(__VA_ARGS__); break;                        \
    case F32 * 2 + 1: FN<F32, 16>(__VA_ARGS__); break;                   \
    case BF16 * 2: FN<BF16, 4>(__VA_ARGS__); break;                      \
    case BF16 * 2 + 1: FN<BF16, 16>(__VA_ARGS__); break;                 \
    case FP8 * 2: FN<FP8, 4>(__VA_ARGS__); break;                        \
    case FP8 * 2 + 1: FN<FP8, 16>(__VA_ARGS__); break;                   \
    case I8 * 2: FN<I8, 4>(__VA_ARGS__); break;                          \
    case I8 * 2 + 1: FN<I8, 16>(__VA_ARGS__); break;                     \
    case B2 * 2 + 1: FN<B2, 16>(__VA_ARGS__); break;                     \
    default: return hipErrorInvalidValue;                                \
  }

hipError_t launch_colstats(const Geom& g, double* sum, double* sumsq, hipStream_t s) {
  PQR_DISPATCH_S(colstats_fmt, g, sum, sumsq, s)
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Lanczos on K_g = X~_g X~_g^T (n x n) for all blocks at once.  Its nonzero
// eigenvalues are those of X~_g^T X~_g; block 0 includes the intercept column.
// ---------------------------------------------------------------------------
template <int FMT, int RPL>
__global__ __launch_bounds__(256) void k_block_dots(Geom g, const float* __restrict__ q,
                                                    int64_t qstride, const int* __restrict__ gblock,
                                                    const float* __restrict__ cm,
                                                    const float* __restrict__ cinv,
                                                    const float* __restrict__ qsum, float* u) {
  const int lane = threadIdx.x & 63;
  const int64_t grp = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (grp >= g.ngroups()) return;
  const int blk = gblock[grp];
  const float* qb = q + (int64_t)blk * qstride;
  float acc[kGroup];
#pragma unroll
  for (int c = 0; c < kGroup; ++c) acc[c] = 0;
  for (int64_t ch = 0; ch < g.nchunks(); ++ch) {
    const int64_t row0 = ch * (kWave * RPL) + (int64_t)lane * RPL;
    const uint8_t* base = g.seg(grp * kGroup, ch);
    float th[RPL];
    load_vec<RPL, float>(qb, row0, th);
#pragma unroll
    for (int c = 0; c < kGroup; ++c) {
      float x[RPL];
      load_rows<FMT, RPL, float>(base + c * g.seg_bytes, (int64_t)lane * RPL, x);
#pragma unroll
      for (int r = 0; r < RPL; ++r) acc[c] = fmaf(x[r], th[r], acc[c]);
    }
  }
  const float dot = reduce16(acc, lane);
  if ((lane & 3) == 0) {
    const int64_t j = grp * kGroup + group_col_of_lane(lane);
    u[j] = (dot - cm[j] * qsum[blk]) * cinv[j];
  }
}

template <int FMT, int RPL>
__global__ __launch_bounds__(256) void k_block_axpy(Geom g, const float* __restrict__ u,
                                                    const float* __restrict__ cm,
                                                    const float* __restrict__ cinv,
                                                    const int* __restrict__ bstart, int splits,
                                                    float* partial) {
  const int lane = threadIdx.x & 63;
  const int64_t ch = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (ch >= g.nchunks()) return;
  const int blk = blockIdx.y / splits, sp = blockIdx.y % splits;
  const int ga = bstart[blk], gb = bstart[blk + 1];   // group range of the block
  const int len = gb - ga, per = (len + splits - 1) / splits;
  const int e0 = ga + sp * per;
  const int e1 = e0 + per < gb ? e0 + per : gb;
  const int64_t row0 = ch * (kWave * RPL) + (int64_t)lane * RPL;
  float acc[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) acc[r] = 0;
  float off = 0;
  for (int grp = e0; grp < e1; ++grp) {
#pragma unroll 4
    for (int c = 0; c < kGroup; ++c) {
      const int64_t j = (int64_t)grp * kGroup + c;
      const float bj = u[j] * cinv[j];
      float x[RPL];
      load_rows<FMT, RPL, float>(g.seg(j, ch), (int64_t)lane * RPL, x);
#pragma unroll
      for (int r = 0; r < RPL; ++r) acc[r] = fmaf(x[r], bj, acc[r]);
      off = fmaf(cm[j], bj, off);
    }
  }
  float* out = partial + (int64_t)blockIdx.y * g.n_pad + row0;
#pragma unroll
  for (int r = 0; r < RPL; ++r) out[r] = acc[r] - off;
}

template <int FMT, int RPL>
static void block_dots_fmt(const Geom& g, const float* q, int64_t qstride, const int* gblock,
                           const float* cm, const float* cinv, const float* qsum, float* u,
                           hipStream_t s) {
  hipLaunchKernelGGL((k_block_dots<FMT, RPL>), dim3((unsigned)((g.ngroups() + 3) / 4)), dim3(256),
                     0, s, g, q, qstride, gblock, cm, cinv, qsum, u);
}
template <int FMT, int RPL>
static void block_axpy_fmt(const Geom& g, const float* u, const float* cm, const float* cinv,
                           const int* bstart, int G, int splits, float* partial, hipStream_t s) {
  hipLaunchKernelGGL((k_block_axpy<FMT, RPL>), dim3((unsigned)((g.nchunks() + 3) / 4), G * splits),
                     dim3(256), 0, s, g, u, cm, cinv, bstart, splits, partial);
}

hipError_t launch_block_dots(const Geom& g, const float* q, int64_t qstride, const int* gblock,
                             const float* cm, const float* cinv, const float* qsum, float* u,
                             hipStream_t s) {
  PQR_DISPATCH_S(block_dots_fmt, g, q, qstride, gblock, cm, cinv, qsum, u, s)
  return hipGetLastError();
}
hipError_t launch_block_axpy(const Geom& g, const float* u, const float* cm, const float* cinv,
                             const int* bstart, int G, int splits, float* partial, hipStream_t s) {
  PQR_DISPATCH_S(block_axpy_fmt, g, u, cm, cinv, bstart, G, splits, partial, s)
  return hipGetLastError();
}

__device__ __forceinline__ float hash_unit(uint32_t a, uint32_t b) {
  uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15; h *= 0x2C1B3C6Du; h ^= h >> 12; h *= 0x297A2D39u; h ^= h >> 15;
  return ((float)(h >> 8) + 0.5f) * (1.0f / 16777216.0f) - 0.5f;
}

// One workgroup per block: start vectors q_g of unit norm, q_prev = 0.
__global__ __launch_bounds__(1024) void k_lanczos_init(int64_t n, int64_t n_pad, float* q,
                                                       float* qprev, float* qsum) {
  __shared__ double red[2 * 16];
  const int blk = blockIdx.x;
  float* qb = q + (int64_t)blk * n_pad;
  double s[2] = {0, 0};
  for (int64_t i = threadIdx.x; i < n_pad; i += 1024) {
    const float v = i < n ? hash_unit((uint32_t)i, (uint32_t)blk) : 0.0f;
    qb[i] = v;
    qprev[(int64_t)blk * n_pad + i] = 0.0f;
    s[0] += (double)v * v;
  }
  block_sum<1024, 2, double>(s, red);
  const float inv = (float)(1.0 / sqrt(s[0]));
  double t[2] = {0, 0};
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    qb[i] *= inv;
    t[0] += qb[i];
  }
  block_sum<1024, 2, double>(t, red);
  if (threadIdx.x == 0) qsum[blk] = (float)t[0];
}

hipError_t launch_lanczos_init(int64_t n, int64_t n_pad, int G, float* q, float* qprev,
                               float* qsum, hipStream_t s) {
  hipLaunchKernelGGL(k_lanczos_init, dim3(G), dim3(1024), 0, s, n, n_pad, q, qprev, qsum);
  return hipGetLastError();
}

// w = K_g q: sum of the block's partials (+ the intercept term for block 0);
// alpha_k = q.w; w -= alpha_k q + beta_{k-1} q_prev; beta_k = |w|; q <- w / beta_k.
__global__ __launch_bounds__(1024) void k_lanczos_step(int64_t n, int64_t n_pad, int splits, int k,
                                                       int T, int icpt_in_block0,
                                                       const float* __restrict__ partial,
                                                       float* q, float* qprev, float* wbuf,
                                                       float* qsum, double* alpha, double* beta) {
  __shared__ double red[2 * 16];
  const int blk = blockIdx.x;
  float* qb = q + (int64_t)blk * n_pad;
  float* pb = qprev + (int64_t)blk * n_pad;
  float* wb = wbuf + (int64_t)blk * n_pad;
  const double u0 = (blk == 0 && icpt_in_block0) ? (double)qsum[0] : 0.0;
  const double bprev = k > 0 ? beta[blk * T + k - 1] : 0.0;
  double s[2] = {0, 0};
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    double acc = u0;
    for (int sp = 0; sp < splits; ++sp) acc += partial[((int64_t)blk * splits + sp) * n_pad + i];
    const float v = (float)acc;
    wb[i] = v;
    s[0] += (double)v * qb[i];
  }
  block_sum<1024, 2, double>(s, red);
  const double a = s[0];
  double t[2] = {0, 0};
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const float v = (float)((double)wb[i] - a * qb[i] - bprev * pb[i]);
    wb[i] = v;
    t[0] += (double)v * v;
  }
  block_sum<1024, 2, double>(t, red);
  const double bnorm = sqrt(t[0]);
  const float inv = bnorm > 1e-30 ? (float)(1.0 / bnorm) : 0.0f;
  double u[2] = {0, 0};
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    pb[i] = qb[i];
    qb[i] = wb[i] * inv;
    u[0] += qb[i];
  }
  block_sum<1024, 2, double>(u, red);
  if (threadIdx.x == 0) {
    alpha[blk * T + k] = a;
    beta[blk * T + k] = bnorm;
    qsum[blk] = (float)u[0];
  }
}

hipError_t launch_lanczos_step(int64_t n, int64_t n_pad, int G, int splits, int k, int T,
                               int icpt_in_block0, const float* partial, float* q, float* qprev,
                               float* wbuf, float* qsum, double* alpha, double* beta,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_lanczos_step, dim3(G), dim3(1024), 0, s, n, n_pad, splits, k, T,
                     icpt_in_block0, partial, q, qprev, wbuf, qsum, alpha, beta);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Null-fit dual: q = the k-th smallest y (radix select on order-preserving
// 64-bit keys), psi_i = tau (y_i > q), tau - 1 (y_i < q), balanced on ties;
// theta_p = psi / n.  out[0] = q.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t okey(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__global__ __launch_bounds__(1024) void k_null_dual(const double* __restrict__ y, int64_t n,
                                                    int64_t n_pad, int64_t kth, double tau,
                                                    double* theta_p, double* out) {
  __shared__ unsigned hist[256];
  __shared__ uint64_t prefix_s;
  __shared__ int64_t rank_s;
  __shared__ double red[3 * 16];
  const int t = threadIdx.x;
  uint64_t prefix = 0;
  int64_t rank = kth;   // 1-based rank among keys matching the prefix so far
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    const uint64_t mask = pass == 0 ? 0ull : (~0ull << (64 - 8 * pass));
    if (t < 256) hist[t] = 0;
    __syncthreads();
    for (int64_t i = t; i < n; i += 1024) {
      const uint64_t kk = okey(y[i]);
      if ((kk & mask) == prefix) atomicAdd(&hist[(kk >> shift) & 0xff], 1u);
    }
    __syncthreads();
    if (t == 0) {
      int64_t acc = 0;
      int d = 0;
      for (; d < 256; ++d) {
        if (acc + hist[d] >= rank) break;
        acc += hist[d];
      }
      prefix_s = prefix | ((uint64_t)d << shift);
      rank_s = rank - acc;
    }
    __syncthreads();
    prefix = prefix_s;
    rank = rank_s;
    __syncthreads();
  }
  // the selected value
  double qv = 0;
  {
    const uint64_t u = (prefix >> 63) ? (prefix & 0x7fffffffffffffffull) : ~prefix;
    qv = __longlong_as_double((long long)u);
  }
  double c[3] = {0, 0, 0};   // above, below, ties
  for (int64_t i = t; i < n; i += 1024) {
    const double v = y[i];
    c[0] += v > qv; c[1] += v < qv; c[2] += v == qv;
  }
  block_sum<1024, 3, double>(c, red);
  const double tie = -(tau * c[0] + (tau - 1.0) * c[1]) / c[2];
  const double inv_n = 1.0 / (double)n;
  for (int64_t i = t; i < n_pad; i += 1024) {
    double v = 0.0;
    if (i < n) {
      const double yi = y[i];
      v = (yi > qv ? tau : (yi < qv ? tau - 1.0 : tie)) * inv_n;
    }
    theta_p[i] = v;
  }
  if (t == 0) { out[0] = qv; out[5] = 0.0; }
}

hipError_t launch_null_dual(const double* y, int64_t n, int64_t n_pad, double tau,
                            double* theta_p, double* out, hipStream_t s) {
  int64_t k = (int64_t)ceil((double)n * tau - 1e-12);
  if (k < 1) k = 1;
  if (k > n) k = n;
  hipLaunchKernelGGL(k_null_dual, dim3(1), dim3(1024), 0, s, y, n, n_pad, k, tau, theta_p, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bt_scale(const double* __restrict__ beta_std, int64_t p,
                                                  const double* __restrict__ cm,
                                                  const double* __restrict__ cinv,
                                                  double* beta_orig, double* mb) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < p; j += (int64_t)gridDim.x * 256) {
    const double b = beta_std[1 + j] * cinv[j];
    beta_orig[1 + j] = b;
    mb[j] = cm[j] * b;
  }
}
__global__ void k_bt_intercept(double beta0, const double* sum_mb, double* beta_orig) {
  if (threadIdx.x == 0 && blockIdx.x == 0) beta_orig[0] = beta0 - sum_mb[0];
}

hipError_t launch_back_transform(const double* beta_std, int64_t p, const double* cm,
                                 const double* cinv, double beta0, double* beta_orig,
                                 double* bpart, hipStream_t s) {
  // bpart must hold p + 512 doubles: p products, 256 stage partials, the total
  double* mb = bpart;
  hipLaunchKernelGGL(k_bt_scale, dim3(1024), dim3(256), 0, s, beta_std, p, cm, cinv, beta_orig, mb);
  (void)launch_reduce_sum(mb, p, bpart + p, bpart + p + 256, s);
  hipLaunchKernelGGL(k_bt_intercept, dim3(1), dim3(64), 0, s, beta0, bpart + p + 256, beta_orig);
  return hipGetLastError();
}

}  // namespace pqr

namespace pqr {

// m_j = sum/n, s_j = sqrt(sumsq/n - m_j^2) (population sd); excluded columns
// (zero variance or padding) get cinv = 0.  Without standardization m = 0, cinv = 1.
__global__ __launch_bounds__(256) void k_colparams(const double* __restrict__ sum,
                                                   const double* __restrict__ sumsq, int64_t n,
                                                   int64_t p, int64_t p_pad, int standardize,
                                                   double* cm_d, double* cinv_d, double* sd_d,
                                                   float* cm_f, float* cinv_f) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < p_pad;
       j += (int64_t)gridDim.x * 256) {
    double m = 0.0, inv = 0.0, sd = 0.0;
    if (j < p) {
      if (standardize) {
        m = sum[j] / (double)n;
        const double var = sumsq[j] / (double)n - m * m;
        sd = var > 1e-24 * (1.0 + m * m) ? sqrt(var) : 0.0;
        inv = sd > 0.0 ? 1.0 / sd : 0.0;
        if (sd == 0.0) m = 0.0;
      } else {
        inv = 1.0;
        sd = 1.0;
      }
    }
    cm_d[j] = m; cinv_d[j] = inv; sd_d[j] = sd;
    cm_f[j] = (float)m; cinv_f[j] = (float)inv;
  }
}

hipError_t launch_colparams(const double* sum, const double* sumsq, int64_t n, int64_t p,
                            int64_t p_pad, int standardize, double* cm_d, double* cinv_d,
                            double* sd_d, float* cm_f, float* cinv_f, hipStream_t s) {
  hipLaunchKernelGGL(k_colparams, dim3(1024), dim3(256), 0, s, sum, sumsq, n, p, p_pad,
                     standardize, cm_d, cinv_d, sd_d, cm_f, cinv_f);
  return hipGetLastError();
}

// y_t = (T) y on the first n rows, 0 on the padding; z = y_t.
template <typename T>
__global__ __launch_bounds__(256) void k_set_y(const double* __restrict__ y, int64_t n,
                                               int64_t n_pad, T* y_t) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n_pad;
       i += (int64_t)gridDim.x * 256)
    y_t[i] = i < n ? (T)y[i] : T(0);
}
template <typename T>
hipError_t launch_set_y(const double* y, int64_t n, int64_t n_pad, T* y_t, hipStream_t s) {
  hipLaunchKernelGGL((k_set_y<T>), dim3(256), dim3(256), 0, s, y, n, n_pad, y_t);
  return hipGetLastError();
}
template hipError_t launch_set_y<float>(const double*, int64_t, int64_t, float*, hipStream_t);
template hipError_t launch_set_y<double>(const double*, int64_t, int64_t, double*, hipStream_t);

}  // namespace pqr

namespace pqr {

// dst column c <- src column cols[c], segment by segment (same geometry of rows);
// padding columns of dst (c >= ncols) are zero.
__global__ __launch_bounds__(256) void k_gather_cols(Geom src, const int64_t* __restrict__ cols,
                                                     int64_t ncols, Geom dst, uint8_t* dbase) {
  const int64_t per = src.seg_bytes / 16;   // uint4 per segment
  const int64_t total = dst.p_pad * dst.nchunks() * per;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * 256) {
    const int64_t c = t / (dst.nchunks() * per);
    const int64_t rem = t - c * dst.nchunks() * per;
    const int64_t ch = rem / per, q = rem - ch * per;
    uint4 v = {0u, 0u, 0u, 0u};
    if (c < ncols) v = reinterpret_cast<const uint4*>(src.seg(cols[c], ch))[q];
    uint8_t* d = dbase + (dst.seg(c, ch) - dst.X);
    reinterpret_cast<uint4*>(d)[q] = v;
  }
}

hipError_t launch_gather_columns(const Geom& src, const int64_t* cols, int64_t ncols,
                                 const Geom& dst, uint8_t* dst_base, hipStream_t s) {
  if (src.seg_bytes % 16 || src.seg_bytes != dst.seg_bytes || src.n_pad != dst.n_pad)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gather_cols, dim3(4096), dim3(256), 0, s, src, cols, ncols, dst, dst_base);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_gather_f64(const double* src, const int64_t* cols,
                                                    int64_t ncols, int64_t npad, double* dst) {
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < npad; c += (int64_t)gridDim.x * 256)
    dst[c] = c < ncols ? src[cols[c]] : 0.0;
}

hipError_t launch_gather_f64(const double* src, const int64_t* cols, int64_t ncols, int64_t npad,
                             double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_f64, dim3(256), dim3(256), 0, s, src, cols, ncols, npad, dst);
  return hipGetLastError();
}

}  // namespace pqr
