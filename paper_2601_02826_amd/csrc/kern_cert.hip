// FP64 optimality certificate and small deterministic reductions.
//
// The dual of the constrained form (eq. reformulated_QR) through its
// Lagrangian (eq. main_lagrangian) is
//     max_theta  y^T theta
//     s.t. (tau-1)/n <= theta_i <= tau/n,  sum_i theta_i = 0 (lambda_0 = 0),
//          |x~_j^T theta| <= lambda_j.
// Any iterate theta is turned into a feasible point by a shift-and-clip
// projection (the shift found by bisection) and a scaling alpha in [0, 1];
// P(beta) - y^T theta~ then bounds the suboptimality of beta (Prop. 1).
#include <cmath>

#include "pqr_kernels.h"

namespace pqr {

template <typename T>
__global__ __launch_bounds__(1024) void k_project(const T* __restrict__ theta, int64_t n,
                                                  int64_t n_pad, double tau,
                                                  const double* __restrict__ y,
                                                  double* __restrict__ tp, double* out) {
  __shared__ double red[3 * 16];
  __shared__ double ab[2];
  const double lo = (tau - 1.0) / (double)n, hi = tau / (double)n;
  const int t = threadIdx.x;
  double mn = INFINITY, mx = -INFINITY;
  for (int64_t i = t; i < n; i += 1024) {
    const double v = (double)theta[i];
    mn = fmin(mn, v);
    mx = fmax(mx, v);
  }
  // block min / max
  mn = -wave_max(-mn);
  mx = wave_max(mx);
  if ((t & 63) == 0) { red[t >> 6] = mn; red[16 + (t >> 6)] = mx; }
  __syncthreads();
  if (t == 0) {
    double a = red[0], b = red[16];
    for (int w = 1; w < 16; ++w) { a = fmin(a, red[w]); b = fmax(b, red[16 + w]); }
    ab[0] = a - hi;   // sum clip(theta - c) = n*hi > 0 here
    ab[1] = b - lo;   // and n*lo < 0 here
  }
  __syncthreads();
  double a = ab[0], b = ab[1];
  for (int it = 0; it < 200; ++it) {
    const double c = 0.5 * (a + b);
    if (c <= a || c >= b) break;
    double s[1] = {0.0};
    for (int64_t i = t; i < n; i += 1024) s[0] += fmin(fmax((double)theta[i] - c, lo), hi);
    block_sum<1024, 1, double>(s, red);
    if (s[0] > 0) a = c; else b = c;
  }
  const double c = 0.5 * (a + b);
  double q[2] = {0.0, 0.0};
  for (int64_t i = t; i < n_pad; i += 1024) {
    double v = 0.0;
    if (i < n) {
      v = fmin(fmax((double)theta[i] - c, lo), hi);
      q[0] += v * y[i];
      q[1] += v;
    }
    tp[i] = v;
  }
  block_sum<1024, 2, double>(q, red);
  if (t == 0) { out[2] = q[0]; out[4] = c; out[5] = q[1]; }
}

template <typename T>
hipError_t launch_project(const T* theta, int64_t n, int64_t n_pad, double tau, const double* y,
                          double* theta_p, double* out, hipStream_t s) {
  hipLaunchKernelGGL((k_project<T>), dim3(1), dim3(1024), 0, s, theta, n, n_pad, tau, y, theta_p,
                     out);
  return hipGetLastError();
}
template hipError_t launch_project<float>(const float*, int64_t, int64_t, double, const double*, double*, double*, hipStream_t);
template hipError_t launch_project<double>(const double*, int64_t, int64_t, double, const double*, double*, double*, hipStream_t);

// ---------------------------------------------------------------------------
template <int FMT, int RPL>
__global__ __launch_bounds__(256) void k_dots64(Geom g, const double* __restrict__ tp,
                                                const double* sum_tp, const double* __restrict__ cm,
                                                const double* __restrict__ cinv,
                                                const double* __restrict__ clam, double* v,
                                                double* gmax) {
  const int lane = threadIdx.x & 63;
  const int64_t grp = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (grp >= g.ngroups()) return;
  double acc[kGroup];
#pragma unroll
  for (int c = 0; c < kGroup; ++c) acc[c] = 0;
  const int64_t nch = g.nchunks();
  for (int64_t ch = 0; ch < nch; ++ch) {
    const int64_t row0 = ch * (kWave * RPL) + (int64_t)lane * RPL;
    const uint8_t* base = g.seg(grp * kGroup, ch);
    double th[RPL];
    load_vec<RPL, double>(tp, row0, th);
#pragma unroll
    for (int c = 0; c < kGroup; ++c) {
      double x[RPL];
      load_rows<FMT, RPL, double>(base + c * g.seg_bytes, (int64_t)lane * RPL, x);
#pragma unroll
      for (int r = 0; r < RPL; ++r) acc[c] = fma(x[r], th[r], acc[c]);
    }
  }
  const double dot = reduce16(acc, lane);
  const int64_t j = grp * kGroup + group_col_of_lane(lane);
  const bool owner = (lane & 3) == 0;
  const double vj = (dot - cm[j] * sum_tp[0]) * cinv[j];
  const double lam = clam[j];
  // lambda_j = 0 (an unpenalized column) is enforced by the projection onto
  // x~_j^T theta = 0 before this pass (launch_unpen_*), not by the ratio
  double ratio = 0.0;
  if (cinv[j] != 0.0 && lam > 0.0) ratio = fabs(vj) / lam;
  if (owner && v) v[j] = vj;
  ratio = wave_max(owner ? ratio : 0.0);
  if (lane == 0) gmax[grp] = ratio;
}

template <int FMT, int RPL>
static void dots64_fmt(const Geom& g, const double* tp, const double* sum_tp, const double* cm,
                       const double* cinv, const double* clam, double* v, double* gmax,
                       hipStream_t s) {
  hipLaunchKernelGGL((k_dots64<FMT, RPL>), dim3((unsigned)((g.ngroups() + 3) / 4)), dim3(256), 0,
                     s, g, tp, sum_tp, cm, cinv, clam, v, gmax);
}

// Up to four certificates at once (int8 store, 16 rows per lane: the batched
// layout): v_kj = x~_j^T theta'_k in FP64 for k < kb (theta'_k at tp + k n_pad,
// sum theta'_k at out + 8k + 5), one pass over X; per group and k the max
// |v_kj| / (lam_k w_j) into gmax[k * ngroups + grp].  A lane keeps the raw bytes
// of its 16 rows of the 16 columns and walks them four rows at a time, with the
// four theta' slices of those rows in registers.
struct Lam4 { double v[4]; };

__global__ __launch_bounds__(256) void k_mdots64(Geom g, const double* __restrict__ tp, int kb,
                                                 const double* out, const double* __restrict__ cm,
                                                 const double* __restrict__ cinv,
                                                 const double* __restrict__ w, Lam4 lam,
                                                 double* gmax) {
  const int lane = threadIdx.x & 63;
  const int64_t grp = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t ng = g.ngroups();
  if (grp >= ng) return;
  double acc[kGroup][4];
#pragma unroll
  for (int c = 0; c < kGroup; ++c)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[c][k] = 0;
  const int64_t nch = g.nchunks();
  for (int64_t ch = 0; ch < nch; ++ch) {
    const int64_t row0 = ch * (kWave * 16) + (int64_t)lane * 16;
    const uint8_t* base = g.seg(grp * kGroup, ch) + lane * 16;
    uint4 raw[kGroup];
#pragma unroll
    for (int c = 0; c < kGroup; ++c) raw[c] = *reinterpret_cast<const uint4*>(base + c * g.seg_bytes);
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4) {
      double th[4][4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          th[k][r] = k < kb ? tp[(int64_t)k * g.n_pad + row0 + 4 * r4 + r] : 0.0;
#pragma unroll
      for (int c = 0; c < kGroup; ++c) {
        const uint32_t wd = r4 == 0 ? raw[c].x : (r4 == 1 ? raw[c].y : (r4 == 2 ? raw[c].z : raw[c].w));
        double x[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = (double)((wd >> (8 * r)) & 0xffu);
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[c][k] = fma(x[r], th[k][r], acc[c][k]);
      }
    }
  }
  const int64_t j = grp * kGroup + group_col_of_lane(lane);
  const bool owner = (lane & 3) == 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k >= kb) break;
    double a[kGroup];
#pragma unroll
    for (int c = 0; c < kGroup; ++c) a[c] = acc[c][k];
    const double dot = reduce16(a, lane);
    const double vj = (dot - cm[j] * out[8 * k + 5]) * cinv[j];
    const double lj = lam.v[k] * w[j];
    double ratio = 0.0;
    if (cinv[j] != 0.0) ratio = lj > 0.0 ? fabs(vj) / lj : (vj != 0.0 ? INFINITY : 0.0);
    ratio = wave_max(owner ? ratio : 0.0);
    if (lane == 0) gmax[(int64_t)k * ng + grp] = ratio;
  }
}

#define PQR_DISPATCH64(FN, ...)                                          \
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

hipError_t launch_mdots64(const Geom& g, const double* tp, int kb, const double* out,
                          const double* cm, const double* cinv, const double* w,
                          const double* lam, double* gmax, hipStream_t s) {
  if (kb < 1 || kb > 4 || g.fmt != I8 || g.rpl != 16) return hipErrorInvalidValue;
  Lam4 l4{{0, 0, 0, 0}};
  for (int k = 0; k < kb; ++k) l4.v[k] = lam[k];
  hipLaunchKernelGGL(k_mdots64, dim3((unsigned)((g.ngroups() + 3) / 4)), dim3(256), 0, s, g, tp, kb,
                     out, cm, cinv, w, l4, gmax);
  return hipGetLastError();
}

hipError_t launch_dots64(const Geom& g, const double* theta_p, const double* sum_tp,
                         const double* cm, const double* cinv, const double* clam, double* v,
                         double* gmax, hipStream_t s) {
  PQR_DISPATCH64(dots64_fmt, g, theta_p, sum_tp, cm, cinv, clam, v, gmax, s)
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sparse s = X~ beta (FP64) over the active list, as in the iteration.
__device__ __forceinline__ int splits_in_use64(int count, int smax, int min_per) {
  const int s = (count + min_per - 1) / min_per;
  return s < 1 ? 1 : (s > smax ? smax : s);
}

template <int FMT, int RPL>
__global__ __launch_bounds__(256) void k_axpy64(Geom g, CertBufs c, int smax, int min_per) {
  const int lane = threadIdx.x & 63;
  const int64_t ch = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int split = blockIdx.y;
  const int count = c.ctl->count;
  const int seff = splits_in_use64(count, smax, min_per);
  if (split >= seff || ch >= g.nchunks()) return;
  const int per = (count + seff - 1) / seff;
  const int e0 = split * per;
  const int e1 = e0 + per < count ? e0 + per : count;
  const int64_t row0 = ch * (kWave * RPL) + (int64_t)lane * RPL;
  double acc[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) acc[r] = 0;
  double off = 0;
  for (int e = e0; e < e1; ++e) {
    const int64_t grp = c.list[e];
    for (int k = 0; k < kGroup; ++k) {
      const int64_t j = grp * kGroup + k;
      const double bj = c.beta_d[j] * c.cinv[j];
      if (bj != 0.0) {
        double x[RPL];
        load_rows<FMT, RPL, double>(g.seg(j, ch), (int64_t)lane * RPL, x);
#pragma unroll
        for (int r = 0; r < RPL; ++r) acc[r] = fma(x[r], bj, acc[r]);
        off = fma(c.cm[j], bj, off);
      }
    }
  }
  double* out = c.partial + (int64_t)split * g.n_pad + row0;
#pragma unroll
  for (int r = 0; r < RPL; ++r) out[r] = acc[r] - off;
}

// Per-row pinball loss of r = y - s - beta0 into block partials.
__global__ __launch_bounds__(256) void k_loss64(CertBufs c, int64_t n, int64_t n_pad, double tau,
                                                int smax, int min_per) {
  __shared__ double red[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int seff = splits_in_use64(c.ctl->count, smax, min_per);
  double q[1] = {0.0};
  if (i < n) {
    const double s = sum_splits(c.partial, seff, n_pad, i, c.ctl->beta0);
    const double r = c.y[i] - s;
    q[0] = (r < 0 ? tau - 1.0 : tau) * r;
  }
  block_sum<256, 1, double>(q, red);
  if (threadIdx.x == 0) c.bpart[blockIdx.x] = q[0];
}

__global__ __launch_bounds__(256) void k_penalty64(const double* __restrict__ beta,
                                                   const double* __restrict__ clam, int64_t p,
                                                   double* bpart) {
  __shared__ double red[4];
  double q[1] = {0.0};
  const int64_t per = (p + gridDim.x - 1) / gridDim.x;
  const int64_t j0 = (int64_t)blockIdx.x * per, j1 = j0 + per < p ? j0 + per : p;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += 256) q[0] += clam[j] * fabs(beta[j]);
  block_sum<256, 1, double>(q, red);
  if (threadIdx.x == 0) bpart[blockIdx.x] = q[0];
}

__global__ __launch_bounds__(256) void k_final_sum(const double* bpart, int64_t m, double scale,
                                                   double* out) {
  __shared__ double red[4];
  double q[1] = {0.0};
  for (int64_t k = threadIdx.x; k < m; k += 256) q[0] += bpart[k];
  block_sum<256, 1, double>(q, red);
  if (threadIdx.x == 0) *out = q[0] * scale;
}

template <int FMT, int RPL>
static void axpy64_fmt(const Geom& g, const CertBufs& c, int smax, int min_per, hipStream_t s) {
  hipLaunchKernelGGL((k_axpy64<FMT, RPL>), dim3((unsigned)((g.nchunks() + 3) / 4), smax),
                     dim3(256), 0, s, g, c, smax, min_per);
}

hipError_t launch_primal64(const Geom& g, const CertBufs& c, double tau, int smax, int min_per,
                           hipStream_t s) {
  PQR_DISPATCH64(axpy64_fmt, g, c, smax, min_per, s)
  const unsigned nb = (unsigned)(g.n_pad / 256);
  hipLaunchKernelGGL(k_loss64, dim3(nb), dim3(256), 0, s, c, g.n, g.n_pad, tau, smax, min_per);
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(256), 0, s, c.bpart, (int64_t)nb,
                     1.0 / (double)g.n, c.out + 0);
  const unsigned np = 512;
  hipLaunchKernelGGL(k_penalty64, dim3(np), dim3(256), 0, s, c.beta_d, c.clam, g.p_pad,
                     c.bpart + nb);
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(256), 0, s, c.bpart + nb, (int64_t)np, 1.0,
                     c.out + 1);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_stage_sum(const double* a, int64_t m, double* bpart) {
  __shared__ double red[4];
  double q[1] = {0.0};
  const int64_t per = (m + gridDim.x - 1) / gridDim.x;
  const int64_t j0 = (int64_t)blockIdx.x * per, j1 = j0 + per < m ? j0 + per : m;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += 256) q[0] += a[j];
  block_sum<256, 1, double>(q, red);
  if (threadIdx.x == 0) bpart[blockIdx.x] = q[0];
}

__global__ __launch_bounds__(256) void k_stage_max(const double* a, int64_t m, double* bpart) {
  double mx = 0.0;
  const int64_t per = (m + gridDim.x - 1) / gridDim.x;
  const int64_t j0 = (int64_t)blockIdx.x * per, j1 = j0 + per < m ? j0 + per : m;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += 256) mx = fmax(mx, a[j]);
  __shared__ double red[4];
  mx = wave_max(mx);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) bpart[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ __launch_bounds__(256) void k_final_max(const double* bpart, int64_t m, double* out) {
  double mx = 0.0;
  for (int64_t k = threadIdx.x; k < m; k += 256) mx = fmax(mx, bpart[k]);
  __shared__ double red[4];
  mx = wave_max(mx);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) *out = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ __launch_bounds__(256) void k_scale(const double* w, double a, int64_t m, double* out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256)
    out[i] = a * w[i];
}

// ---------------------------------------------------------------------------
// Unpenalized columns U (lambda_j = 0) in the dual certificate: the dual point
// must satisfy x~_j^T theta = 0 for j in U, besides sum theta = 0 (the
// intercept).  theta' (box-feasible, sum zero) is projected onto that subspace,
// theta1 = theta' - A c with A = [1, X~_U] and (A^T A) c = A^T theta', then scaled
// toward 0 (strictly inside the box) until the box holds.
// ---------------------------------------------------------------------------
// Dense x~ of the columns cols[0..nu) (nu x n_pad, zero on padding rows); a
// column index -1 stands for the intercept (ones on the n rows).
template <int FMT, int RPL>
__global__ __launch_bounds__(64) void k_dense_cols(Geom g, const int64_t* cols,
                                                   const double* cm, const double* cinv,
                                                   double* xu) {
  const int64_t c = blockIdx.y, ch = blockIdx.x;
  const int64_t j = cols[c];
  const int lane = threadIdx.x;
  const int64_t row0 = ch * (kWave * RPL) + (int64_t)lane * RPL;
  if (j < 0) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) xu[c * g.n_pad + row0 + r] = row0 + r < g.n ? 1.0 : 0.0;
    return;
  }
  double x[RPL];
  load_rows<FMT, RPL, double>(g.seg(j, ch), (int64_t)lane * RPL, x);
#pragma unroll
  for (int r = 0; r < RPL; ++r)
    xu[c * g.n_pad + row0 + r] = row0 + r < g.n ? (x[r] - cm[j]) * cinv[j] : 0.0;
}

template <int FMT, int RPL>
static void dense_cols_fmt(const Geom& g, const int64_t* cols, int64_t nu, const double* cm,
                           const double* cinv, double* xu, hipStream_t s) {
  hipLaunchKernelGGL((k_dense_cols<FMT, RPL>), dim3((unsigned)g.nchunks(), (unsigned)nu), dim3(64),
                     0, s, g, cols, cm, cinv, xu);
}

// out[a * nb + b] = xa^T xb for rows of A (na x m) and B (nb x m), one block per pair.
__global__ __launch_bounds__(256) void k_cross(const double* A, const double* B, int64_t m,
                                               int64_t nb, double* out) {
  __shared__ double red[4];
  const int64_t a = blockIdx.y, b = blockIdx.x;
  double q[1] = {0.0};
  for (int64_t i = threadIdx.x; i < m; i += 256) q[0] += A[a * m + i] * B[b * m + i];
  block_sum<256, 1, double>(q, red);
  if (threadIdx.x == 0) out[a * nb + b] = q[0];
}

// theta1 = theta' - X~_U c in place; per block the largest box scale factor.
__global__ __launch_bounds__(256) void k_unpen_apply(double* tp, const double* xu,
                                                    const double* c, int64_t nu, int64_t n,
                                                    int64_t n_pad, double lo, double hi,
                                                    double* bmin) {
  __shared__ double red[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double sc = 1.0;
  if (i < n) {
    double t = tp[i];
    for (int64_t a = 0; a < nu; ++a) t -= xu[a * n_pad + i] * c[a];
    tp[i] = t;
    if (t > hi) sc = hi / t;
    else if (t < lo) sc = lo / t;
  }
  sc = -wave_max(-sc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sc;
  __syncthreads();
  if (threadIdx.x == 0) bmin[blockIdx.x] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

// theta2 = s theta1 with s the smallest block factor; out[2] = y^T theta2,
// out[5] = sum theta2 (single block, deterministic order).
__global__ __launch_bounds__(1024) void k_unpen_scale(double* tp, const double* y, int64_t n,
                                                      const double* bmin, int64_t nblk, double* out) {
  __shared__ double red[2 * 16];
  __shared__ double s_sh;
  if (threadIdx.x == 0) {
    double s = 1.0;
    for (int64_t b = 0; b < nblk; ++b) s = fmin(s, bmin[b]);
    s_sh = s;
  }
  __syncthreads();
  const double s = s_sh;
  double q[2] = {0.0, 0.0};
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const double t = tp[i] * s;
    tp[i] = t;
    q[0] += t * y[i];
    q[1] += t;
  }
  block_sum<1024, 2, double>(q, red);
  if (threadIdx.x == 0) { out[2] = q[0]; out[5] = q[1]; out[6] = s; }
}

hipError_t launch_dense_cols(const Geom& g, const int64_t* cols, int64_t nu, const double* cm,
                             const double* cinv, double* xu, hipStream_t s) {
  if (nu < 1) return hipSuccess;
  PQR_DISPATCH64(dense_cols_fmt, g, cols, nu, cm, cinv, xu, s)
  return hipGetLastError();
}

hipError_t launch_cross(const double* A, int64_t na, const double* B, int64_t nb, int64_t m,
                        double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_cross, dim3((unsigned)nb, (unsigned)na), dim3(256), 0, s, A, B, m, nb, out);
  return hipGetLastError();
}

hipError_t launch_unpen_project(double* tp, const double* xu, const double* c, int64_t nu,
                                int64_t n, int64_t n_pad, double tau, const double* y,
                                double* bpart, double* out, hipStream_t s) {
  const unsigned nb = (unsigned)(n_pad / 256);
  hipLaunchKernelGGL(k_unpen_apply, dim3(nb), dim3(256), 0, s, tp, xu, c, nu, n, n_pad,
                     (tau - 1.0) / (double)n, tau / (double)n, bpart);
  hipLaunchKernelGGL(k_unpen_scale, dim3(1), dim3(1024), 0, s, tp, y, n, bpart, (int64_t)nb, out);
  return hipGetLastError();
}

// LLA weights (Algorithm 2): w_j = max(p'_lambda(|beta_j|) / lambda, wfloor) with
// p' the SCAD derivative of eq. scad (kind 0) or the MCP derivative of eq. mcp
// (kind 1), beta on the standardized scale; out[0] = 0 (intercept), out[1 + j].
template <typename T>
__global__ __launch_bounds__(256) void k_lla_weights(const T* __restrict__ beta, int64_t p,
                                                     int kind, double a, double lam,
                                                     double wfloor, double* out) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j <= p; j += (int64_t)gridDim.x * 256) {
    if (j == 0) { out[0] = 0.0; continue; }
    const double b = fabs((double)beta[j - 1]);
    double d;
    if (kind == 0)
      d = b <= lam ? lam : (b < a * lam ? (a * lam - b) / (a - 1.0) : 0.0);   // eq. scad
    else
      d = b <= a * lam ? lam - b / a : 0.0;                                   // eq. mcp
    out[j] = fmax(d / lam, wfloor);
  }
}

template <typename T>
hipError_t launch_lla_weights(const T* beta, int64_t p, int kind, double a, double lam,
                              double wfloor, double* out, hipStream_t s) {
  hipLaunchKernelGGL((k_lla_weights<T>), dim3(1024), dim3(256), 0, s, beta, p, kind, a, lam, wfloor,
                     out);
  return hipGetLastError();
}
template hipError_t launch_lla_weights<float>(const float*, int64_t, int, double, double, double, double*, hipStream_t);
template hipError_t launch_lla_weights<double>(const double*, int64_t, int, double, double, double, double*, hipStream_t);

hipError_t launch_scale(const double* w, double a, int64_t m, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(1024), dim3(256), 0, s, w, a, m, out);
  return hipGetLastError();
}

hipError_t launch_reduce_sum(const double* a, int64_t m, double* bpart, double* out,
                             hipStream_t s) {
  const unsigned nb = 256;
  hipLaunchKernelGGL(k_stage_sum, dim3(nb), dim3(256), 0, s, a, m, bpart);
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(256), 0, s, bpart, (int64_t)nb, 1.0, out);
  return hipGetLastError();
}

hipError_t launch_reduce_max(const double* a, int64_t m, double* bpart, double* out,
                             hipStream_t s) {
  const unsigned nb = 256;
  hipLaunchKernelGGL(k_stage_max, dim3(nb), dim3(256), 0, s, a, m, bpart);
  hipLaunchKernelGGL(k_final_max, dim3(1), dim3(256), 0, s, bpart, (int64_t)nb, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <typename S, typename D>
__global__ __launch_bounds__(256) void k_convert(const S* a, int64_t m, D* out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256)
    out[i] = (D)a[i];
}

template <typename T>
hipError_t launch_to_double(const T* a, int64_t m, double* out, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<T, double>), dim3(1024), dim3(256), 0, s, a, m, out);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_from_double(const double* a, int64_t m, T* out, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<double, T>), dim3(1024), dim3(256), 0, s, a, m, out);
  return hipGetLastError();
}
template hipError_t launch_to_double<float>(const float*, int64_t, double*, hipStream_t);
template hipError_t launch_to_double<double>(const double*, int64_t, double*, hipStream_t);
template hipError_t launch_from_double<float>(const double*, int64_t, float*, hipStream_t);
template hipError_t launch_from_double<double>(const double*, int64_t, double*, hipStream_t);

}  // namespace pqr
