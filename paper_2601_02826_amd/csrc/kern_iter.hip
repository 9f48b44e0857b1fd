// One iteration of FS-QRPPA (Algorithm 1) on gfx950, as four kernels:
//
//   k_sweep    v = X~^T theta for every column (one wavefront per 16-column
//              group, the design read once) fused with the per-block
//              weighted soft threshold of eq. beta_update.
//   k_count, k_scatter  the ordered list of column groups holding a nonzero
//              coefficient, the sweep's norm partials, and the intercept
//              (lambda_0 = 0, so its update is a plain step); k_compact1 does
//              the same in one block for designs of at most 8192 groups.
//   k_axpy     s = X~ beta^{k+1} over the nonzero coefficients only: the
//              partial products X_g beta_g of the paper, gathered by column
//              and reduced in a fixed order (no atomics).
//   k_update   the z prox of eq. z_update, the extrapolated dual step of
//              eq. fsppa_update, and the norms of the iteration (including
//              the H-norm successive difference), reduced by the last block.
//
// Each kernel is a thin wrapper around a device body that takes its block
// number explicitly, so that the grouped launches (many independent problems
// per launch, one table of problem descriptors) run the same code.
#include "pqr_kernels.h"

namespace pqr {

template <typename T> __device__ __forceinline__ T tmax(T a, T b) { return a > b ? a : b; }

// Column dot products of one 16-column group with theta.  Each lane sums its
// rows of two chunks in the iterate type and adds that partial to an FP64
// accumulator; the cross-lane reduction is FP64 too, so the FP32 path's
// x~_j^T theta is accurate to the FP32 rounding of theta rather than limited by
// the cancellation of n FP32 products.
template <int FMT, int RPL, typename T>
__device__ __forceinline__ void group_dots(const Geom& g, int64_t grp, const T* __restrict__ theta,
                                           double (&accd)[kGroup]) {
  const int lane = threadIdx.x & 63;
  T acc[kGroup];
#pragma unroll
  for (int c = 0; c < kGroup; ++c) { accd[c] = 0; acc[c] = 0; }
  const int64_t nch = g.nchunks();
  const int64_t lrow = (int64_t)lane * RPL;
  constexpr int B = Batch<FMT, RPL>::value;
  for (int64_t ch = 0; ch < nch; ++ch) {
    const int64_t row0 = ch * (kWave * RPL) + lrow;
    const uint8_t* base = g.seg(grp * kGroup, ch);
#pragma unroll
    for (int cb = 0; cb < kGroup; cb += B) {
      Raw<FMT, RPL> raw[B];
#pragma unroll
      for (int c = 0; c < B; ++c) raw[c] = load_raw<FMT, RPL>(base + (cb + c) * g.seg_bytes, lrow);
      T th[RPL];
      load_vec<RPL, T>(theta, row0, th);
#pragma unroll
      for (int c = 0; c < B; ++c) {
        T x[RPL];
        decode<FMT, RPL, T>(raw[c], x);
#pragma unroll
        for (int r = 0; r < RPL; ++r) acc[cb + c] = fma(x[r], th[r], acc[cb + c]);
      }
    }
    if ((ch & 1) || ch + 1 == nch) {   // flush every two chunks (2*RPL rows per lane)
#pragma unroll
      for (int c = 0; c < kGroup; ++c) { accd[c] += (double)acc[c]; acc[c] = 0; }
    }
  }
}

// ---------------------------------------------------------------------------
template <int FMT, int RPL, typename T>
__device__ __forceinline__ void sweep_body(const Geom& g, const IterBufs<T>& b, int64_t blk) {
  const int lane = threadIdx.x & 63;
  const int64_t grp = blk * 4 + (threadIdx.x >> 6);
  if (grp >= g.ngroups()) return;
  double acc[kGroup];
  group_dots<FMT, RPL, T>(g, grp, b.theta, acc);
  const double dot = reduce16(acc, lane);

  const int64_t j = grp * kGroup + group_col_of_lane(lane);
  const bool owner = (lane & 3) == 0;
  // x~_j^T theta on the standardized scale
  const T v = (T)((dot - (double)b.cm[j] * b.ctl->sum_theta) * (double)b.cinv[j]);
  const T bo = b.beta[j];
  const T eta = b.geta[grp];
  const T lam = b.clam[j];
  const T a = eta * bo + v;
  const T bn = (tmax<T>(a - lam, 0) - tmax<T>(-a - lam, 0)) / eta;   // eq. beta_update
  if (owner) b.beta[j] = bn;
  const T d = bn - bo;
  T q0 = owner ? d * d : T(0);
  T q1 = owner ? bn * bn : T(0);
  T q2 = owner ? eta * d * d : T(0);
  T q3 = owner ? b.cm[j] * b.cinv[j] * bn : T(0);
  const unsigned long long nz = __ballot(owner && bn != T(0));
  q0 = wave_sum(q0); q1 = wave_sum(q1); q2 = wave_sum(q2); q3 = wave_sum(q3);
  if (lane == 0) {
    T* o = b.gnorm + grp * 4;
    o[0] = q0; o[1] = q1; o[2] = q2; o[3] = q3;
    b.gflag[grp] = nz != 0ull;
  }
}

template <int FMT, int RPL, typename T>
__global__ __launch_bounds__(256) void k_sweep(Geom g, IterBufs<T> b) {
  sweep_body<FMT, RPL, T>(g, b, blockIdx.x);
}

// Flags only (for a warm start): group has a nonzero coefficient.
template <typename T>
__global__ __launch_bounds__(256) void k_flags(int64_t ngroups, IterBufs<T> b) {
  const int64_t grp = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (grp >= ngroups) return;
  int f = 0;
  for (int c = 0; c < kGroup; ++c) f |= b.beta[grp * kGroup + c] != T(0);
  b.gflag[grp] = f;
  T* o = b.gnorm + grp * 4;
  o[0] = o[1] = o[2] = o[3] = 0;
}

// ---------------------------------------------------------------------------
// Compaction in two passes over kCompactBlocks contiguous ranges of groups:
// k_count sums each range's flags and norm partials; k_scatter writes each
// range's active groups at its offset (ranges in order, groups in order), and
// its block 0 reduces the norms in a fixed order and steps the intercept.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void compact_range(int64_t ngroups, int blk, int64_t& g0, int64_t& g1) {
  const int64_t per = (ngroups + kCompactBlocks - 1) / kCompactBlocks;
  g0 = (int64_t)blk * per;
  g1 = g0 + per < ngroups ? g0 + per : ngroups;
  if (g0 > ngroups) g0 = ngroups;
}

template <typename T>
__device__ __forceinline__ void count_body(int64_t ngroups, const IterBufs<T>& b, int blk) {
  __shared__ double red[5 * 16];
  int64_t g0, g1;
  compact_range(ngroups, blk, g0, g1);
  double s[5] = {0, 0, 0, 0, 0};
  for (int64_t gi = g0 + threadIdx.x; gi < g1; gi += 1024) {
    s[4] += b.gflag[gi] != 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) s[k] += (double)b.gnorm[gi * 4 + k];
  }
  block_sum<1024, 5, double>(s, red);
  if (threadIdx.x == 0) {
    b.bcnt[blk] = (int)s[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) b.bnrm[blk * 4 + k] = s[k];
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_count(int64_t ngroups, IterBufs<T> b) {
  count_body<T>(ngroups, b, blockIdx.x);
}

template <typename T>
__device__ __forceinline__ void scatter_body(int64_t ngroups, const IterBufs<T>& b, double eta0,
                                             int step_intercept, int blk) {
  __shared__ int wcnt[16];
  __shared__ int base_s;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  int64_t g0, g1;
  compact_range(ngroups, blk, g0, g1);
  if (t == 0) {
    int off = 0;
    for (int k = 0; k < blk; ++k) off += b.bcnt[k];
    base_s = off;
  }
  __syncthreads();
  int base = base_s;
  for (int64_t tile = g0; tile < g1; tile += 1024) {
    const int64_t gi = tile + t;
    const bool f = gi < g1 && b.gflag[gi] != 0;
    const unsigned long long bal = __ballot(f);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[wid] = __popcll(bal);
    __syncthreads();
    int woff = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      woff += w < wid ? wcnt[w] : 0;
      tot += wcnt[w];
    }
    if (f) b.list[base + woff + before] = (int)gi;
    base += tot;
    __syncthreads();
  }
  if (blk == 0 && t == 0) {
    double s[4] = {0, 0, 0, 0};
    int total = 0;
    for (int k = 0; k < kCompactBlocks; ++k) {
      total += b.bcnt[k];
      for (int q = 0; q < 4; ++q) s[q] += b.bnrm[k * 4 + q];
    }
    Ctl* c = b.ctl;
    double b0 = c->beta0, b0n = b0;
    if (step_intercept) b0n = b0 + c->sum_theta / eta0;   // intercept: lambda_0 = 0
    const double d0 = b0n - b0;
    c->beta0 = b0n;
    c->nb[0] = s[0] + d0 * d0;
    c->nb[1] = s[1] + b0n * b0n;
    c->nb[2] = s[2] + eta0 * d0 * d0;
    c->nb[3] = s[3];
    c->count = total;
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_scatter(int64_t ngroups, IterBufs<T> b, double eta0,
                                                  int step_intercept) {
  scatter_body<T>(ngroups, b, eta0, step_intercept, blockIdx.x);
}

// The same compaction in one block for designs of at most kCompactOneBlock groups,
// where two launches of kCompactBlocks blocks cost more than the work: the list (groups
// in order), the count, the intercept step and the norms (summed here by one block's
// tree, so the norms of the monitor can differ in their last bits from the two-kernel
// form; the list, the count and the intercept are identical).
constexpr int64_t kCompactOneBlock = 8192;
template <typename T>
__global__ __launch_bounds__(1024) void k_compact1(int64_t ngroups, IterBufs<T> b, double eta0,
                                                   int step_intercept) {
  __shared__ int wcnt[16];
  __shared__ double red[4 * 16];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  double s[4] = {0, 0, 0, 0};
  int base = 0;
  for (int64_t tile = 0; tile < ngroups; tile += 1024) {
    const int64_t gi = tile + t;
    const bool in = gi < ngroups;
    const bool f = in && b.gflag[gi] != 0;
    if (in)
#pragma unroll
      for (int k = 0; k < 4; ++k) s[k] += (double)b.gnorm[gi * 4 + k];
    const unsigned long long bal = __ballot(f);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[wid] = __popcll(bal);
    __syncthreads();
    int woff = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      woff += w < wid ? wcnt[w] : 0;
      tot += wcnt[w];
    }
    if (f) b.list[base + woff + before] = (int)gi;
    base += tot;
    __syncthreads();
  }
  block_sum<1024, 4, double>(s, red);
  if (t == 0) {
    Ctl* c = b.ctl;
    double b0 = c->beta0, b0n = b0;
    if (step_intercept) b0n = b0 + c->sum_theta / eta0;   // intercept: lambda_0 = 0
    const double d0 = b0n - b0;
    c->beta0 = b0n;
    c->nb[0] = s[0] + d0 * d0;
    c->nb[1] = s[1] + b0n * b0n;
    c->nb[2] = s[2] + eta0 * d0 * d0;
    c->nb[3] = s[3];
    c->count = base;
  }
}

template <typename T>
static void launch_compaction(int64_t ng, const IterBufs<T>& b, double eta0, int step_intercept,
                              hipStream_t s) {
  if (ng <= kCompactOneBlock) {
    hipLaunchKernelGGL((k_compact1<T>), dim3(1), dim3(1024), 0, s, ng, b, eta0, step_intercept);
    return;
  }
  hipLaunchKernelGGL((k_count<T>), dim3(kCompactBlocks), dim3(1024), 0, s, ng, b);
  hipLaunchKernelGGL((k_scatter<T>), dim3(kCompactBlocks), dim3(1024), 0, s, ng, b, eta0,
                     step_intercept);
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ int splits_in_use(int count, int smax, int min_per) {
  const int s = (count + min_per - 1) / min_per;
  return s < 1 ? 1 : (s > smax ? smax : s);
}

template <int FMT, int RPL, typename T>
__device__ __forceinline__ void axpy_body(const Geom& g, const IterBufs<T>& b, int smax,
                                          int min_per, int64_t bx, int split) {
  const int lane = threadIdx.x & 63;
  const int64_t ch = bx * 4 + (threadIdx.x >> 6);
  const int count = b.ctl->count;
  const int seff = splits_in_use(count, smax, min_per);
  if (split >= seff || ch >= g.nchunks()) return;
  const int per = (count + seff - 1) / seff;
  const int e0 = split * per;
  const int e1 = e0 + per < count ? e0 + per : count;
  const int64_t row0 = ch * (kWave * RPL) + (int64_t)lane * RPL;
  double acc[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) acc[r] = 0;
  double off = 0;
  // The group's 16 coefficients first, then the rows of CB columns loaded with no
  // branch between the loads (so that they are in flight together; a column whose
  // coefficient is zero re-reads the rows of the group's first nonzero column, a cache
  // hit, and is skipped below), then the products of the nonzero columns in column
  // order (the same arithmetic as one column at a time).
  constexpr int kRawRegs = (int)(sizeof(Raw<FMT, RPL>) / 4);
  constexpr int CB = kRawRegs <= 4 ? 16 : (kRawRegs <= 8 ? 8 : (kRawRegs <= 16 ? 4 : 2));
  for (int e = e0; e < e1; ++e) {
    const int64_t grp = b.list[e];
    double bj[kGroup], cmj[kGroup];
    uint32_t nzm = 0;   // wave-uniform: bit c = column c has a nonzero coefficient
#pragma unroll
    for (int c = 0; c < kGroup; ++c) {
      const int64_t j = grp * kGroup + c;
      bj[c] = (double)b.beta[j] * (double)b.cinv[j];   // coefficient on the raw column
      cmj[c] = (double)b.cm[j];
      nzm |= (bj[c] != 0.0 ? 1u : 0u) << c;
    }
    if (nzm == 0u) continue;
    const int cfirst = __ffs((int)nzm) - 1;
#pragma unroll
    for (int cb = 0; cb < kGroup; cb += CB) {
      if (((nzm >> cb) & ((1u << CB) - 1u)) == 0u) continue;
      Raw<FMT, RPL> raw[CB];
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const int cc = ((nzm >> (cb + c)) & 1u) ? cb + c : cfirst;
        raw[c] = load_raw<FMT, RPL>(g.seg(grp * kGroup + cc, ch), (int64_t)lane * RPL);
      }
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        if (!((nzm >> (cb + c)) & 1u)) continue;
        double x[RPL];
        decode<FMT, RPL, double>(raw[c], x);
#pragma unroll
        for (int r = 0; r < RPL; ++r) acc[r] = fma(x[r], bj[cb + c], acc[r]);
        off = fma(cmj[cb + c], bj[cb + c], off);
      }
    }
  }
  double* out = b.partial + (int64_t)split * g.n_pad + row0;
#pragma unroll
  for (int r = 0; r < RPL; ++r) out[r] = acc[r] - off;
}

template <int FMT, int RPL, typename T>
__global__ __launch_bounds__(256) void k_axpy(Geom g, IterBufs<T> b, int smax, int min_per) {
  axpy_body<FMT, RPL, T>(g, b, smax, min_per, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void update_body(const IterBufs<T>& b, const IterParams& ip, int64_t n,
                                            int64_t n_pad, int64_t blk, int64_t nblk) {
  __shared__ double red[8 * 4];
  __shared__ int last;
  const int64_t i = blk * 256 + threadIdx.x;
  const int seff = splits_in_use(b.ctl->count, ip.smax, ip.min_per);
  double q[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (i < n) {
    const double s = sum_splits(b.partial, seff, n_pad, i, b.ctl->beta0);
    const T mu = (T)ip.mu;
    const T zo = b.z[i], to = b.theta[i], ro = b.r[i];
    const T u = zo + to / mu;
    const T zn = tmax<T>(u - (T)(ip.tau / ((double)n * ip.mu)), 0) -
                 tmax<T>(-u - (T)((1.0 - ip.tau) / ((double)n * ip.mu)), 0);   // eq. z_update
    const T rn = (T)(s + (double)zn - (double)b.y[i]);
    const T tn = to - (T)ip.sigma * ((T)2 * rn - ro);                         // dual step
    b.z[i] = zn;
    b.theta[i] = tn;
    b.r[i] = rn;
    const double dz = (double)zn - (double)zo, dt = (double)tn - (double)to;
    q[0] = dz * dz; q[1] = (double)zn * zn; q[2] = dt * dt; q[3] = (double)tn * tn;
    q[4] = (double)rn * rn; q[5] = dt * ((double)rn - (double)ro); q[6] = (double)tn;
  }
  block_sum<256, 8, double>(q, red);
  if (threadIdx.x == 0) {
    for (int k = 0; k < 8; ++k) b.bpart[blk * 8 + k] = q[k];
    __threadfence();
    const unsigned prev = atomicAdd(&b.ctl->blocks_done, 1u);
    last = prev == (unsigned)(nblk - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x < 8) {
    double s = 0;
    for (int64_t k = 0; k < nblk; ++k) s += b.bpart[k * 8 + threadIdx.x];
    red[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Ctl* c = b.ctl;
    for (int k = 0; k < 8; ++k) c->nr[k] = red[k];
    c->sum_theta = red[6];
    const double delta = c->nb[2] + ip.mu * red[0] + 2.0 * red[5] + ((ip.G + 1.0) / ip.mu) * red[2];
    c->delta_prev = c->delta;
    c->delta = delta;
    c->n_increase = (c->iter > 0 && delta > c->delta_prev * (1.0 + 1e-6) && delta > 1e-300)
                        ? c->n_increase + 1 : 0;
    c->iter += 1;
    c->blocks_done = 0u;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_update(IterBufs<T> b, IterParams ip, int64_t n,
                                                int64_t n_pad) {
  update_body<T>(b, ip, n, n_pad, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Grouped launches: one grid covers the blocks of every problem of a group.
// off holds three prefix arrays of nprob + 1 block offsets (sweep, axpy,
// update); the compaction gives every problem kCompactBlocks blocks.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_problem(const int* off, int nprob, int64_t blk) {
  int lo = 0, hi = nprob - 1;   // largest i with off[i] <= blk
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int64_t)off[mid] <= blk) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int FMT, int RPL, typename T>
__global__ __launch_bounds__(256) void k_gsweep(const GroupDesc<T>* d, const int* off, int nprob) {
  const int i = find_problem(off, nprob, blockIdx.x);
  const Geom g = d[i].g;
  const IterBufs<T> b = d[i].b;
  sweep_body<FMT, RPL, T>(g, b, (int64_t)blockIdx.x - off[i]);
}

template <typename T>
__global__ __launch_bounds__(1024) void k_gcount(const GroupDesc<T>* d) {
  const int i = blockIdx.x / kCompactBlocks;
  const IterBufs<T> b = d[i].b;
  count_body<T>(d[i].g.ngroups(), b, blockIdx.x % kCompactBlocks);
}

template <typename T>
__global__ __launch_bounds__(1024) void k_gscatter(const GroupDesc<T>* d) {
  const int i = blockIdx.x / kCompactBlocks;
  const IterBufs<T> b = d[i].b;
  scatter_body<T>(d[i].g.ngroups(), b, d[i].ip.eta0, 1, blockIdx.x % kCompactBlocks);
}

template <int FMT, int RPL, typename T>
__global__ __launch_bounds__(256) void k_gaxpy(const GroupDesc<T>* d, const int* off, int nprob) {
  const int* o = off + (nprob + 1);
  const int i = find_problem(o, nprob, blockIdx.x);
  const Geom g = d[i].g;
  const IterBufs<T> b = d[i].b;
  const int64_t local = (int64_t)blockIdx.x - o[i];
  const int64_t nx = (g.nchunks() + 3) / 4;
  axpy_body<FMT, RPL, T>(g, b, d[i].ip.smax, d[i].ip.min_per, local % nx, (int)(local / nx));
}

template <typename T>
__global__ __launch_bounds__(256) void k_gupdate(const GroupDesc<T>* d, const int* off, int nprob) {
  const int* o = off + 2 * (nprob + 1);
  const int i = find_problem(o, nprob, blockIdx.x);
  const IterBufs<T> b = d[i].b;
  const IterParams ip = d[i].ip;
  const int64_t n_pad = d[i].g.n_pad;
  update_body<T>(b, ip, d[i].g.n, n_pad, (int64_t)blockIdx.x - o[i], n_pad / 256);
}

// r = X~beta + beta0 + z - y and sum(theta) for a given state.
template <typename T>
__global__ __launch_bounds__(256) void k_init_r(IterBufs<T> b, IterParams ip, int64_t n,
                                                int64_t n_pad) {
  __shared__ double red[8 * 4];
  __shared__ int last;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int seff = splits_in_use(b.ctl->count, ip.smax, ip.min_per);
  double q[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (i < n) {
    const double s = sum_splits(b.partial, seff, n_pad, i, b.ctl->beta0);
    if (ip.fit & 1) b.z[i] = (T)((double)b.y[i] - s);
    b.r[i] = (T)(s + (double)b.z[i] - (double)b.y[i]);
    if (ip.fit & 2) b.theta[i] = (T)((ip.tau - ((double)b.z[i] < 0.0 ? 1.0 : 0.0)) / (double)n);
    q[6] = (double)b.theta[i];
  }
  block_sum<256, 8, double>(q, red);
  if (threadIdx.x == 0) {
    b.bpart[(int64_t)blockIdx.x * 8 + 6] = q[6];
    __threadfence();
    const unsigned prev = atomicAdd(&b.ctl->blocks_done, 1u);
    last = prev == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x == 0) {
    double s = 0;
    for (unsigned blk = 0; blk < gridDim.x; ++blk) s += b.bpart[blk * 8 + 6];
    b.ctl->sum_theta = s;
    b.ctl->blocks_done = 0u;
    b.ctl->delta = 0;
    b.ctl->delta_prev = 0;
    b.ctl->n_increase = 0;
  }
}

// theta_i -= sum(theta) / n on the n real rows (after k_init_r with ip.fit bit 1).
template <typename T>
__global__ __launch_bounds__(256) void k_center_theta(IterBufs<T> b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const double shift = b.ctl->sum_theta / (double)n;
  if (i < n) b.theta[i] = (T)((double)b.theta[i] - shift);
}

template <typename T>
__global__ void k_zero_sum_theta(IterBufs<T> b) {
  if (threadIdx.x == 0) b.ctl->sum_theta = 0.0;
}

// ---------------------------------------------------------------------------
template <int FMT, int RPL, typename T>
static void launch_fmt(const Geom& g, const IterBufs<T>& b, const IterParams& ip, hipStream_t s,
                       hipEvent_t ev0, hipEvent_t ev1) {
  const int64_t ng = g.ngroups();
  if (ev0) (void)hipEventRecord(ev0, s);
  hipLaunchKernelGGL((k_sweep<FMT, RPL, T>), dim3((unsigned)((ng + 3) / 4)), dim3(256), 0, s, g, b);
  if (ev1) (void)hipEventRecord(ev1, s);
  launch_compaction<T>(ng, b, ip.eta0, 1, s);
  hipLaunchKernelGGL((k_axpy<FMT, RPL, T>), dim3((unsigned)((g.nchunks() + 3) / 4), ip.smax),
                     dim3(256), 0, s, g, b, ip.smax, ip.min_per);
  hipLaunchKernelGGL((k_update<T>), dim3((unsigned)(g.n_pad / 256)), dim3(256), 0, s, b, ip, g.n,
                     g.n_pad);
}

template <int FMT, int RPL, typename T>
static void grouped_fmt(const GroupDesc<T>* d, const int* off, int nprob, const int64_t tot[3],
                        hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (ev0) (void)hipEventRecord(ev0, s);
  hipLaunchKernelGGL((k_gsweep<FMT, RPL, T>), dim3((unsigned)tot[0]), dim3(256), 0, s, d, off, nprob);
  if (ev1) (void)hipEventRecord(ev1, s);
  hipLaunchKernelGGL((k_gcount<T>), dim3((unsigned)(nprob * kCompactBlocks)), dim3(1024), 0, s, d);
  hipLaunchKernelGGL((k_gscatter<T>), dim3((unsigned)(nprob * kCompactBlocks)), dim3(1024), 0, s, d);
  hipLaunchKernelGGL((k_gaxpy<FMT, RPL, T>), dim3((unsigned)tot[1]), dim3(256), 0, s, d, off, nprob);
  hipLaunchKernelGGL((k_gupdate<T>), dim3((unsigned)tot[2]), dim3(256), 0, s, d, off, nprob);
}

template <int FMT, int RPL, typename T>
static void prepare_fmt(const Geom& g, const IterBufs<T>& b, const IterParams& ip, hipStream_t s) {
  const int64_t ng = g.ngroups();
  hipLaunchKernelGGL((k_flags<T>), dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, ng, b);
  launch_compaction<T>(ng, b, ip.eta0, 0, s);
  hipLaunchKernelGGL((k_axpy<FMT, RPL, T>), dim3((unsigned)((g.nchunks() + 3) / 4), ip.smax),
                     dim3(256), 0, s, g, b, ip.smax, ip.min_per);
  hipLaunchKernelGGL((k_init_r<T>), dim3((unsigned)(g.n_pad / 256)), dim3(256), 0, s, b, ip, g.n,
                     g.n_pad);
  if (ip.fit & 2) {
    hipLaunchKernelGGL((k_center_theta<T>), dim3((unsigned)(g.n_pad / 256)), dim3(256), 0, s, b,
                       g.n);
    hipLaunchKernelGGL((k_zero_sum_theta<T>), dim3(1), dim3(64), 0, s, b);
  }
}

#define PQR_DISPATCH(FN, ...)                                                       \
  switch (g.fmt * 2 + (g.rpl == 16)) {                                              \
    case F64 * 2: FN<F64, 4, T>(__VA_ARGS__); break;                                \
    case F64 * 2 + 1: FN<F64, 16, T>(__VA_ARGS__); break;                           \
    case F32 * 2: FN<F32, 4, T>(__VA_ARGS__); break;                                \
    case F32 * 2 + 1: FN<F32, 16, T>(__VA_ARGS__); break;                           \
    case BF16 * 2: FN<BF16, 4, T>(__VA_ARGS__); break;                              \
    case BF16 * 2 + 1: FN<BF16, 16, T>(__VA_ARGS__); break;                         \
    case FP8 * 2: FN<FP8, 4, T>(__VA_ARGS__); break;                                \
    case FP8 * 2 + 1: FN<FP8, 16, T>(__VA_ARGS__); break;                           \
    case I8 * 2: FN<I8, 4, T>(__VA_ARGS__); break;                                  \
    case I8 * 2 + 1: FN<I8, 16, T>(__VA_ARGS__); break;                             \
    case B2 * 2 + 1: FN<B2, 16, T>(__VA_ARGS__); break;                             \
    default: return hipErrorInvalidValue;                                           \
  }

template <typename T>
hipError_t launch_iteration(const Geom& g, const IterBufs<T>& b, const IterParams& ip,
                            hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  PQR_DISPATCH(launch_fmt, g, b, ip, s, ev0, ev1)
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prepare_state(const Geom& g, const IterBufs<T>& b, const IterParams& ip,
                                hipStream_t s) {
  PQR_DISPATCH(prepare_fmt, g, b, ip, s)
  return hipGetLastError();
}

template <typename T>
hipError_t launch_grouped_iteration(const Geom& g, const GroupDesc<T>* d, const int* off,
                                    int nprob, const int64_t tot[3], hipStream_t s,
                                    hipEvent_t ev0, hipEvent_t ev1) {
  if (nprob < 1 || tot[0] < 1 || tot[1] < 1 || tot[2] < 1 || tot[0] > INT32_MAX ||
      tot[1] > INT32_MAX || tot[2] > INT32_MAX || (int64_t)nprob * kCompactBlocks > INT32_MAX)
    return hipErrorInvalidValue;
  PQR_DISPATCH(grouped_fmt, d, off, nprob, tot, s, ev0, ev1)
  return hipGetLastError();
}
template hipError_t launch_grouped_iteration<float>(const Geom&, const GroupDesc<float>*, const int*, int, const int64_t*, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_grouped_iteration<double>(const Geom&, const GroupDesc<double>*, const int*, int, const int64_t*, hipStream_t, hipEvent_t, hipEvent_t);

template <typename T>
hipError_t launch_active_list(const Geom& g, const IterBufs<T>& b, hipStream_t s) {
  const int64_t ng = g.ngroups();
  hipLaunchKernelGGL((k_flags<T>), dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, ng, b);
  launch_compaction<T>(ng, b, 1.0, 0, s);
  return hipGetLastError();
}
template hipError_t launch_active_list<float>(const Geom&, const IterBufs<float>&, hipStream_t);
template hipError_t launch_active_list<double>(const Geom&, const IterBufs<double>&, hipStream_t);

template hipError_t launch_iteration<float>(const Geom&, const IterBufs<float>&, const IterParams&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_iteration<double>(const Geom&, const IterBufs<double>&, const IterParams&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_prepare_state<float>(const Geom&, const IterBufs<float>&, const IterParams&, hipStream_t);
template hipError_t launch_prepare_state<double>(const Geom&, const IterBufs<double>&, const IterParams&, hipStream_t);

}  // namespace pqr
