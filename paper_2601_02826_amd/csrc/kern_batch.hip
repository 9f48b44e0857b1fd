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
#include <atomic>
#include <climits>
#include <utility>


#include "pqr_kernels.h"

namespace pqr {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));

constexpr int kBS = 3;                  // digit slices of theta

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

// one wavefront per right-hand side k (grid Kp): exact integer sums, any order
__global__ __launch_bounds__(64) void k_bdsum(BatchBufs b, int nblk, int Kp) {
  const int k = blockIdx.x, lane = threadIdx.x;
  long long s = 0;
  for (int q = lane; q < nblk; q += 64) s += b.tpart[(int64_t)q * Kp + k];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) b.tsumq[k] = s;
}

// ---------------------------------------------------------------------------
// V = X~^T Theta on the int8 MFMA (16x16x64).  A wavefront owns GW column
// groups over all rows and TW right-hand-side tiles (16 k each): per 64-row
// step it loads one A fragment per group straight from the blocked store (lane:
// column lane % 16, rows 16 (lane / 16) .. +15 of the step, 16 contiguous bytes)
// and one B fragment per (tile, slice) of the digits (staged per block in LDS),
// and issues GW * TW * S MFMAs.  With more than TW tiles, the block's wavefronts
// split the tiles of the same groups (their A loads meet in the caches; HBM
// reads X once).  A fragments are loaded NS - 1 steps ahead of their MFMAs.
// Epilogue: the weighted soft threshold of eq. beta_update for every (column,
// k) and per (group, tile) a 16-bit mask of the columns nonzero for some k.
// ---------------------------------------------------------------------------
// LDS bytes per digit row of a tile of 64 SPT rows (+16: bank spread)
template <int SPT> constexpr int drow_bytes() { return 64 * SPT + 16; }

constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }
// a loop body of L steps never runs past the end: the steps of a column come in
// chunks of 16
template <int L> constexpr bool kStepsDivide() { return 16 % L == 0; }
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F> __device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// SPT = 64-row steps per digit tile (one barrier per tile); WPB = wavefronts per
// block (all of them share each staged digit tile); NS = A fragment sets in flight
// (A from registers); SA = A staged in LDS once per group set and tile.
// S = digit slices; CERT selects the certificate epilogue (per (group set, k)
// maxima of |x~_j^T theta_q| / (lambda_k w_j)) over the iteration's (eq.
// beta_update and the column masks).  The column groups of block bi over all rows.
template <int TW, int GW, int DL, int SPT, int WPB, int NS, int S, bool CERT, bool SA>
__device__ __forceinline__ void bgemm_pass(const Geom& g, const BatchBufs& b, const CertArgs& ca,
                                           int Kp, int wps, int64_t bi, uint8_t* dtile) {
  constexpr int kDRow = drow_bytes<SPT>();
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int nrt = Kp / 16;
  const int64_t ng = g.ngroups();
  // wps wavefronts share one set of GW groups; wavefront wv % wps takes tiles r0..
  // A wavefront past the last group or tile still runs the loop (it takes part in
  // the digit tiles and the barriers) on clamped indices and skips the epilogue.
  const int64_t gw0r = (bi * (WPB / wps) + wv / wps) * GW;
  const int r0r = (wv % wps) * TW;
  const bool wave_live = gw0r < ng && r0r < nrt;
  const int64_t gw0 = gw0r < ng ? gw0r : ng - 1;
  const int r0 = r0r < nrt ? r0r : nrt - 1;
  const int col = lane & 15, kq = lane >> 4;
  v4i acc[GW][TW][S];
#pragma unroll
  for (int q = 0; q < GW; ++q)
#pragma unroll
    for (int r = 0; r < TW; ++r)
#pragma unroll
      for (int s = 0; s < S; ++s) acc[q][r][s] = v4i{0, 0, 0, 0};
  const int64_t nsteps = g.nchunks() * 16;   // 64-row steps (1024-row chunks)
  const int64_t nsup = nsteps / SPT;         // digit tiles of 64 SPT rows
  const bool tile_ok[2] = {true, TW > 1 && r0 + 1 < nrt};
  // Buffer loads: a lane's offset is fixed (one VGPR per fragment), the step's
  // part is a wave-uniform SGPR offset; no per-step address arithmetic.
  // A: segments of the wave's groups, from the first group's chunk 0 (a group
  // past the last one re-reads the last group; the epilogue skips it).
  const int64_t nch = g.nchunks();
  const int64_t cstride = kGroup * g.seg_bytes;   // next chunk of a group
  const int64_t gstride = nch * cstride;           // next group
  const uint8_t* abase = g.X + gw0 * gstride;
  const int64_t arem = g.store_bytes() - gw0 * gstride;
  const __amdgpu_buffer_rsrc_t arsrc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)abase, (short)0, (int)(arem < 0x7fffffffll ? arem : 0x7fffffffll), 0x00020000);
  uint32_t aoff[GW];
#pragma unroll
  for (int q = 0; q < GW; ++q)
    aoff[q] = (uint32_t)((gw0 + q < ng ? q : ng - 1 - gw0) * gstride + col * g.seg_bytes + kq * 16);
  auto load_a = [&](int64_t t, v4i (&af)[GW]) {
    const int so = (int)((t >> 4) * cstride + (t & 15) * 64);
#pragma unroll
    for (int q = 0; q < GW; ++q) {
      const v4u v = __builtin_amdgcn_raw_buffer_load_b128(arsrc, (int)aoff[q], so, 0);
      af[q] = v4i{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
    }
  };
  // B: the digits of every right-hand side for 64 SPT rows are staged once per
  // block in LDS (row s*Kp + k: 64 SPT bytes), double-buffered; a wavefront reads
  // its fragments there (rhs (r0 + r)*16 + col, bytes 64 h + 16 kq of step h).
  constexpr int kParts = 4 * SPT;                  // 16-byte pieces per digit row
  const int drows = S * Kp, total16 = drows * kParts;
  const int64_t dbytes = (int64_t)drows * g.n_pad;
  const __amdgpu_buffer_rsrc_t brsrc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(CERT ? ca.dig : b.dig), (short)0, (int)(dbytes < 0x7fffffffll ? dbytes : 0x7fffffffll), 0x00020000);
  auto load_d = [&](int64_t u, v4u (&dr)[DL]) {
#pragma unroll
    for (int i = 0; i < DL; ++i) {
      const int idx = threadIdx.x + 64 * WPB * i;
      const int row = idx < total16 ? idx / kParts : 0, part = idx % kParts;
      dr[i] = __builtin_amdgcn_raw_buffer_load_b128(brsrc, (int)((int64_t)row * g.n_pad + part * 16),
                                                    (int)(u * 64 * SPT), 0);
    }
  };
  auto store_d = [&](int buf, const v4u (&dr)[DL]) {
#pragma unroll
    for (int i = 0; i < DL; ++i) {
      const int idx = threadIdx.x + 64 * WPB * i;
      if (idx < total16)
        *reinterpret_cast<v4u*>(dtile + ((int64_t)buf * drows + idx / kParts) * kDRow +
                                (idx % kParts) * 16) = dr[i];
    }
  };
  auto read_b = [&](int buf, int h, v4i (&bf)[TW][S]) {
#pragma unroll
    for (int r = 0; r < TW; ++r)
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int row = s * Kp + (r0 + (tile_ok[r] ? r : 0)) * 16 + col;
        bf[r][s] = *reinterpret_cast<const v4i*>(dtile + ((int64_t)buf * drows + row) * kDRow +
                                                 h * 64 + kq * 16);
      }
  };
  auto mma = [&](const v4i (&af)[GW], const v4i (&bf)[TW][S]) {
#pragma unroll
    for (int q = 0; q < GW; ++q)
#pragma unroll
      for (int r = 0; r < TW; ++r)
#pragma unroll
        for (int s = 0; s < S; ++s)
          acc[q][r][s] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[q], bf[r][s], acc[q][r][s], 0, 0, 0);
  };
  v4i bf[TW][S];
  v4u dr[DL];
  if constexpr (!SA) {
    // NS A fragment sets in rotation: step t uses set t % NS, and right after its
    // MFMAs issue the set is reloaded for step t + NS, so NS - 1 steps' loads are in
    // flight while these MFMAs run.  The next digit tile is loaded at the top of a
    // tile and stored to the other LDS buffer at its end; one barrier per tile.
    // Scheduling barriers keep this order; loads past the end re-read the last step
    // or tile (in bounds).  The loop body is L = lcm(NS, SPT) steps, unrolled so that
    // the set and the step within the tile are compile-time constants.
    constexpr int L = NS * SPT / gcd_c(NS, SPT);
    v4i aS[NS][GW];
    load_d(0, dr);
    store_d(0, dr);
    __syncthreads();
    static_for<NS>([&](auto I) {   // each set strictly older than the next on entry
      load_a(I.value < nsteps ? I.value : nsteps - 1, aS[I.value]);
      __builtin_amdgcn_sched_barrier(0);
    });
    for (int64_t t0 = 0; t0 < nsteps; t0 += L) {
      static_for<L>([&](auto I) {
        constexpr int set = I.value % NS, h = I.value % SPT;
        const int64_t t = t0 + I.value;
        const int64_t u = t / SPT;   // digit tile
        const int buf = (int)(u & 1);
        if constexpr (h == 0) {
          load_d(u + 1 < nsup ? u + 1 : nsup - 1, dr);
          __builtin_amdgcn_sched_barrier(0);
        }
        if (kStepsDivide<L>() || t < nsteps) {   // wave-uniform
          read_b(buf, h, bf);
          mma(aS[set], bf);
        }
        __builtin_amdgcn_sched_barrier(0);
        load_a(t + NS < nsteps ? t + NS : nsteps - 1, aS[set]);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (h == SPT - 1) {
          store_d(buf ^ 1, dr);
          __syncthreads();
        }
      });
    }
  } else {
    // Shared A: the wps wavefronts of a group set need the same A fragments, so
    // each tile's GW x SPT fragments of the set are staged once in LDS (behind the
    // digit tiles, double-buffered alongside them) by direct buffer-to-LDS loads
    // (lane l lands at 16 l: the fragment layout), split among the set's wavefronts.
    // Tile u + 1's fragments and digits are loaded at the top of tile u; the
    // barrier at its end (a workgroup fence: every load of the block has landed)
    // makes them visible to the whole block.
    constexpr int NGS = WPB;                 // upper bound of group sets per block
    constexpr int NF = GW * SPT;             // fragments per set and tile
    const int gsl = wv / wps, wi = wv % wps;
    const int ngs_blk = WPB / wps;
    uint8_t* abase = dtile + (size_t)2 * drows * kDRow;
    auto a_slot = [&](int bufA, int f) {
      return abase + ((size_t)(bufA * ngs_blk + gsl) * NF + f) * 1024;
    };
    auto issue_a = [&](int64_t u, int bufA) {
      for (int f = wi; f < NF; f += wps) {   // wave-uniform
        const int h = f / GW, q = f % GW;
        const int64_t t = u * SPT + h;
        const int so = (int)((t >> 4) * cstride + (t & 15) * 64);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            arsrc, (__attribute__((address_space(3))) void*)a_slot(bufA, f), 16, (int)aoff[q],
            so, 0, 0);
      }
    };
    (void)NGS;
    issue_a(0, 0);
    load_d(0, dr);
    store_d(0, dr);
    __syncthreads();
    for (int64_t u = 0; u < nsup; ++u) {
      const int buf = (int)(u & 1);
      const int64_t un = u + 1 < nsup ? u + 1 : nsup - 1;
      issue_a(un, buf ^ 1);
      load_d(un, dr);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int h = 0; h < SPT; ++h) {
        v4i af[GW];
#pragma unroll
        for (int q = 0; q < GW; ++q)
          af[q] = *reinterpret_cast<const v4i*>(a_slot(buf, h * GW + q) + lane * 16);
        read_b(buf, h, bf);
        mma(af, bf);
      }
      __builtin_amdgcn_sched_barrier(0);
      store_d(buf ^ 1, dr);
      __syncthreads();
    }
  }
  if (!wave_live) return;
  if constexpr (CERT) {
    // lane: columns 4 kq + e of each group for k = (r0 + r) 16 + col; exact
    // P = x_j^T T_k (sum T_k = 0, so no mean term), v = P unit_k / s_j
    const int64_t gs = gw0r / GW;
    const int64_t ngs = (ng + GW - 1) / GW;
#pragma unroll
    for (int r = 0; r < TW; ++r) {
      if (!tile_ok[r]) break;
      const int k = (r0 + r) * 16 + col;
      const bool live = k < ca.K;
      const double unit = live ? ca.unit[k] : 0.0;
      const double lamk = live ? ca.lam[k] : 1.0;
      double m = 0.0;
#pragma unroll
      for (int q = 0; q < GW; ++q) {
        const int64_t grp = gw0 + q;
        if (grp >= ng) break;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t j = grp * kGroup + 4 * kq + e;
          if (j >= g.p) continue;
          long long P = 0;
#pragma unroll
          for (int sl = 0; sl < S; ++sl) P = P * 128 + (long long)acc[q][r][sl][e];
          const double v = (double)P * unit * ca.cinv[j];
          m = fmax(m, fabs(v) / (lamk * ca.w[j]));
        }
      }
      // lanes col + 16 h (h = 0..3) hold the same k
      m = fmax(m, __shfl_xor(m, 16));
      m = fmax(m, __shfl_xor(m, 32));
      if (kq == 0 && live) ca.gmax[(int64_t)k * ngs + gs] = m;
    }
  } else {
    // epilogue: lane holds columns 4*kq + e (e = 0..3) of each group for rhs (r0+r)*16 + col
#pragma unroll
    for (int r = 0; r < TW; ++r) {
      if (!tile_ok[r]) break;
      const int k = (r0 + r) * 16 + col;
      const bool live = k < b.K && b.kact[k] != 0;   // frozen: beta kept, out of the union
      const double unit = live ? b.scale[k] / (double)(1 << (7 * S - 1)) : 0.0;
      const double tq = live ? (double)b.tsumq[k] : 0.0;
      const float lamk = live ? b.lam[k] : 0.f;
#pragma unroll
      for (int q = 0; q < GW; ++q) {
        const int64_t grp = gw0 + q;
        if (grp >= ng) break;
        const float eta = b.geta[grp];
        uint32_t cmask = 0;   // bit c: column c of the group is nonzero for some k of the tile
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t j = grp * kGroup + 4 * kq + e;
          long long P = 0;
#pragma unroll
          for (int s = 0; s < S; ++s) P = P * 128 + (long long)acc[q][r][s][e];
          // x~_j^T theta_k = (x_j^T theta_k - m_j sum theta_k) / s_j in the quantised theta
          const double v = ((double)P - (double)b.cm[j] * tq) * unit * (double)b.cinv[j];
          float* bp = b.beta + (int64_t)k * g.p_pad + j;
          if (live) {
            const float bo = *bp;
            const float lj = lamk * b.w[j];
            const float a = eta * bo + (float)v;
            const float bn = (fmaxf(a - lj, 0.f) - fmaxf(-a - lj, 0.f)) / eta;   // eq. beta_update
            *bp = bn;
          }
          // lanes 16 kq .. 16 kq + 15 hold column 4 kq + e for the tile's 16 k
          const unsigned long long bal = __ballot(live && *bp != 0.f);
#pragma unroll
          for (int h = 0; h < 4; ++h)
            cmask |= (((bal >> (16 * h)) & 0xffffull) != 0ull ? 1u : 0u) << (4 * h + e);
        }
        if (lane == 0) b.mask[grp * nrt + r0 + r] = cmask;
      }
    }
  }
}

template <int TW, int GW, int DL, int SPT, int WPB, int NS, int S, bool CERT, bool SA>
__global__ __launch_bounds__(64 * WPB, 2) void k_bgemm(Geom g, BatchBufs b, CertArgs ca, int Kp,
                                                       int wps) {
  // 2 x S*Kp x (64 SPT + 16) digit bytes, then (SA) 2 x (WPB / wps) x GW SPT KB of A
  extern __shared__ __attribute__((aligned(16))) uint8_t dtile[];
  bgemm_pass<TW, GW, DL, SPT, WPB, NS, S, CERT, SA>(g, b, ca, Kp, wps, blockIdx.x, dtile);
}

// ---------------------------------------------------------------------------
// Union of the nonzero columns (any active right-hand side), in increasing
// order, from the per-(group, tile) column masks; intercepts.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t bcols(const BatchBufs& b, int64_t gi, int nrt) {
  uint32_t m = 0;
  for (int t = 0; t < nrt; ++t) m |= b.mask[gi * nrt + t];
  return m;
}

__global__ __launch_bounds__(1024) void k_bcount(int64_t ngroups, BatchBufs b, int nrt) {
  __shared__ double red[16];
  const int64_t per = (ngroups + kCompactBlocks - 1) / kCompactBlocks;
  const int64_t g0 = (int64_t)blockIdx.x * per, g1 = g0 + per < ngroups ? g0 + per : ngroups;
  double s[1] = {0};
  for (int64_t gi = g0 + threadIdx.x; gi < g1; gi += 1024) s[0] += __popc(bcols(b, gi, nrt));
  block_sum<1024, 1, double>(s, red);
  if (threadIdx.x == 0) b.bcnt[blockIdx.x] = (int)s[0];
}

__global__ __launch_bounds__(1024) void k_bscatter(int64_t ngroups, BatchBufs b, int nrt,
                                                   double eta0, int Kp) {
  __shared__ int wsum[16];
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
    const uint32_t m = gi < g1 ? bcols(b, gi, nrt) : 0u;
    const int pc = __popc(m);
    // inclusive scan of the popcounts in the wavefront, then across wavefronts
    int incl = pc;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off);
      if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int woff = 0, tot = 0;
    for (int w = 0; w < 16; ++w) { woff += w < wid ? wsum[w] : 0; tot += wsum[w]; }
    int pos = base + woff + incl - pc;
    for (uint32_t mm = m; mm; mm &= mm - 1) b.list[pos++] = (int)(gi * kGroup + __ffs(mm) - 1);
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
    for (int k = t; k < b.K; k += 1024)
      if (b.kact[k]) b.beta0[k] += b.tsum[k] / eta0;
  }
}

// ---------------------------------------------------------------------------
// S = X~ B over the union list on the int8 MFMA.  The coefficients on the raw
// column scale, b'_kj = beta_kj / s_j, are written in fixed point as
// U_kj = round(b'_kj / d_k * 2^27) with d_k a power of two >= max_j |b'_kj|, cut
// into four balanced base-128 digits (|digit| <= 64); every product and sum of
// a slice is exact in int32 (at most (2^31 - 1) / (64 max_code) columns per split
// of the union), each split's sum_j x_ij U_kj is combined exactly in int64 and the
// splits are added in int64, so S_ik = d_k 2^-27 (sum_j x_ij U_kj - sum_j m_j U_kj)
// is exactly X~ times the quantised coefficients (2^-28 d_k each) up to one final
// FP64 rounding, whatever the number of splits.
// ---------------------------------------------------------------------------
constexpr int kCS = 4;                  // digit slices of the coefficients
constexpr int kDigitBlocks = 256;       // blocks of the coefficient digit kernels
constexpr int kCBits = 7 * kCS - 1;     // fixed-point bits below d_k

__device__ __forceinline__ int bsplits(int count, int smax, int min_per) {
  const int s = (count + min_per - 1) / min_per;
  return s < 1 ? 1 : (s > smax ? smax : s);
}

// The union list is read in "virtual groups" of 16 consecutive entries (entry
// 16 e + c is column c of virtual group e; entries past the count are zero).
//
// Per-block maxima of |b'_kj| over the union (kDigitBlocks blocks; thread t
// takes entry t % 16 of each virtual group and the right-hand sides t / 16 + 16 i).
__global__ __launch_bounds__(256) void k_bbmax(Geom g, BatchBufs b, int Kp) {
  const int t = threadIdx.x, c = t & 15, nrt = Kp / 16;
  const int count = *b.count;
  const int nvg = (count + 15) / 16;
  double mx[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int e = blockIdx.x; e < nvg; e += kDigitBlocks) {
    if (16 * e + c >= count) continue;
    const int64_t j = b.list[16 * e + c];
    const double ci = (double)b.cinv[j];
    for (int r = 0; r < nrt; ++r) {
      const int k = (t >> 4) + 16 * r;
      mx[r] = fmax(mx[r], fabs((double)b.beta[(int64_t)k * g.p_pad + j] * ci));
    }
  }
  for (int r = 0; r < nrt; ++r) {
    double v = mx[r];
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    if (c == 0) b.pmax[(int64_t)blockIdx.x * Kp + (t >> 4) + 16 * r] = v;
  }
}

// Digit slices of the union coefficients (list order, zero past the count) and
// the per-block sums of m_j U_kj; d_k from the maxima of k_bbmax.
__global__ __launch_bounds__(256) void k_bbdigits(Geom g, BatchBufs b, int Kp) {
  __shared__ double dk[128];
  __shared__ double pm[256];
  const int t = threadIdx.x, c = t & 15, nrt = Kp / 16;
  {
    // d_k from the kDigitBlocks partial maxima: 256 / Kp threads per k, then one per k
    const int per = 256 / Kp, kk = t % Kp, part = t / Kp;
    double mx = 0;
    if (part < per)
      for (int q = part; q < kDigitBlocks; q += per) mx = fmax(mx, b.pmax[(int64_t)q * Kp + kk]);
    pm[t] = mx;
    __syncthreads();
    if (t < Kp) {
      for (int u = 1; u < per; ++u) mx = fmax(mx, pm[u * Kp + t]);
      int ex = 0;
      const double fr = frexp(mx > 0 ? mx : 1.0, &ex);
      const double d = ldexp(1.0, fr == 0.5 ? ex - 1 : ex);   // smallest power of two >= mx
      dk[t] = d;
      if (blockIdx.x == 0) b.bscale[t] = d;
    }
  }
  __syncthreads();
  const int count = *b.count;
  const int nvg = (count + 15) / 16;
  double off[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const long long lim = 1ll << kCBits;
  for (int e = blockIdx.x; e < nvg; e += kDigitBlocks) {
    const bool in = 16 * e + c < count;
    const int64_t j = in ? b.list[16 * e + c] : 0;
    const double ci = in ? (double)b.cinv[j] : 0.0, mj = in ? (double)b.cm[j] : 0.0;
    for (int r = 0; r < nrt; ++r) {
      const int k = (t >> 4) + 16 * r;
      const double v = in ? (double)b.beta[(int64_t)k * g.p_pad + j] * ci : 0.0;
      long long U = llrint(v / dk[k] * (double)lim);
      U = U > lim ? lim : (U < -lim ? -lim : U);
      off[r] += mj * (double)U;
      long long rest = U;
      int8_t d[kCS];
#pragma unroll
      for (int sl = kCS - 1; sl > 0; --sl) {
        const long long lo = ((rest + 64) & 127) - 64;
        d[sl] = (int8_t)lo;
        rest = (rest - lo) >> 7;
      }
      d[0] = (int8_t)rest;
      int8_t* o = b.bd + (((int64_t)e * Kp + k) * kCS) * kGroup + c;
#pragma unroll
      for (int sl = 0; sl < kCS; ++sl) o[sl * kGroup] = d[sl];
    }
  }
  for (int r = 0; r < nrt; ++r) {
    double v = off[r];
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    if (c == 0) b.poff[(int64_t)blockIdx.x * Kp + (t >> 4) + 16 * r] = v;
  }
}

// The product itself.  A block of WPB wavefronts owns RB = 16 RT WPB consecutive
// rows (inside one 1024-row chunk) and every right-hand side; wavefront wv owns rows
// 16 RT wv .. +16 RT of them.  Per 64 union columns (one MFMA K step) the block loads
// the RB rows of the 64 columns into one LDS tile (thread t: column t / WPB, 16-byte
// pieces at 16 (t % WPB) + 16 WPB rt, so that the WPB threads of a column read 16 WPB
// contiguous bytes per instruction: whole 128-byte lines at WPB >= 8), each wavefront
// builds its B operand (lane: row l % 16, columns 16 (l / 16) .. +15) from the tile
// with gfx950's transposing LDS reads, and issues RT * NRT * 4 MFMAs with the
// coefficient digits as the A operand, so that the result lands as (right-hand side,
// row) with rows contiguous.  The digits of a step (NRT * 4 KB, the same for every
// row) are staged in LDS beside the tile.  Both are double-buffered (one barrier per
// step).  Splits of the union along grid.y write exact int64 partials.
constexpr int kAxSets = 3;     // union product: loads issued this many 64-column steps ahead
constexpr int kXTilePad = 16;  // LDS bytes after each column of the X tile (bank spread
                               // of the transposing reads; keeps 16-byte alignment)

template <int RT, int NRT, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_baxpy(Geom g, BatchBufs b, int smax, int min_per) {
  constexpr int RB = 16 * RT * WPB;                     // rows of the block
  constexpr int XSB = RB + kXTilePad;                   // LDS bytes per tile column
  constexpr int Kp = NRT * 16;
  constexpr int kDig = NRT * kCS * 64;                  // uint4 digit fragments per step
  constexpr int kDigPer = (kDig + 64 * WPB - 1) / (64 * WPB);
  static_assert(1024 % RB == 0, "a block's rows lie in one 1024-row chunk");
  __shared__ __attribute__((aligned(16))) uint8_t xs[2][64 * XSB];
  __shared__ uint4 dg[2][kDig];                         // [buffer][(r * kCS + sl) * 64 + lane]
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int count = *b.count;
  const int nq = (count + 63) / 64;                     // 64-column K steps of the union
  const int seff = bsplits(nq, smax, min_per);
  const int split = blockIdx.y;
  if (split >= seff) return;                           // uniform per block (an empty
                                                       // union still writes split 0)
  const int per = (nq + seff - 1) / seff;
  const int q0 = split * per, q1 = q0 + per < nq ? q0 + per : nq;
  const int64_t rb = (int64_t)blockIdx.x * RB;          // first row of the block
  const int64_t ch = rb >> 10, roff = rb & 1023;        // its 1024-row chunk
  const int rw = wv * 16 * RT;                          // the wavefront's rows in the tile
  v4i acc[RT][NRT][kCS];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int r = 0; r < NRT; ++r)
#pragma unroll
      for (int sl = 0; sl < kCS; ++sl) acc[rt][r][sl] = v4i{0, 0, 0, 0};
  const int kb = lane >> 4, m = lane & 15;
  const int xc = tid / WPB, xj = tid % WPB;             // this thread's tile column, piece
  const int nvg = (count + 15) / 16;                    // virtual groups with digits
  // The column of union entry 64 qd + xc (past the count it re-reads the last entry;
  // its digits are zero), and this thread's pieces of a column.
  auto fetch_j = [&](int qd) -> int {
    const int il = 64 * qd + xc < count ? 64 * qd + xc : count - 1;
    return b.list[il];
  };
  auto fetch_x = [&](int64_t jl, uint4 (&xv)[RT]) {
    const uint8_t* src = g.seg(jl, ch) + roff + 16 * xj;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
      xv[rt] = *reinterpret_cast<const uint4*>(src + 16 * WPB * rt);
  };
  auto store_x = [&](int buf, const uint4 (&xv)[RT]) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      uint32_t* d = reinterpret_cast<uint32_t*>(&xs[buf][xc * XSB + 16 * xj + 16 * WPB * rt]);
      d[0] = xv[rt].x; d[1] = xv[rt].y; d[2] = xv[rt].z; d[3] = xv[rt].w;
    }
  };
  // This thread's share of the step's digits: fragment f = (r * kCS + sl) * 64 + l
  // holds the A operand of MFMA lane l: digits of (rhs r*16 + l % 16, virtual group
  // 4 qd + l / 16), zero past the last virtual group and for steps past this split
  // (applied when stored, so that no instruction waits for a digit load before the
  // step that stores it).
  auto fetch_d = [&](int qd, uint4 (&dv)[kDigPer]) {
#pragma unroll
    for (int u = 0; u < kDigPer; ++u) {
      const int f = tid + u * 64 * WPB;
      const int fl = f < kDig ? f : 0;
      const int l = fl & 63, sl = (fl >> 6) % kCS, r = (fl >> 6) / kCS;
      const int el = 4 * qd + (l >> 4);
      const int64_t ec = el < nvg ? el : nvg - 1;
      dv[u] = *reinterpret_cast<const uint4*>(
          b.bd + (((int64_t)ec * Kp + r * 16 + (l & 15)) * kCS + sl) * kGroup);
    }
  };
  auto store_d = [&](int buf, const uint4 (&dv)[kDigPer], int qd) {
#pragma unroll
    for (int u = 0; u < kDigPer; ++u) {
      const int f = tid + u * 64 * WPB;
      if (f < kDig)
        dg[buf][f] = qd < q1 && 4 * qd + ((f & 63) >> 4) < nvg ? dv[u] : uint4{0, 0, 0, 0};
    }
  };
  // NS register sets in rotation, the step's set a compile-time index (the loop body
  // is NS steps): at step qd set c = (qd - q0) % NS is free (its step's tile and digits
  // were stored at step qd - 1) and is refilled with step qd + NS, while set (c + 1) %
  // NS is stored into the other LDS buffers for step qd + 1, so that loads run NS - 1
  // steps ahead of their stores with no register moves (a move would wait for its
  // load).  The column index of step qd + NS was loaded at step qd - NS.  Per step the
  // digit loads come first and the index load last, so that the waits (stores of step
  // qd + 1, index of step qd + NS) never cover a later X load.  Every step of the body
  // runs, also past q1 (on the last step's columns with zero digits): a skipped step
  // would leave the compiler's wait counts at zero.
  constexpr int NS = kAxSets;
  uint4 xset[NS][RT];
  uint4 dset[NS][kDigPer];
  int jset[NS];
  auto clampq = [&](int q) { return q < q1 ? q : q1 - 1; };
  if (q0 < q1) {
    // the first NS steps' indices, then per step the loop's own order (digits, X,
    // index of the step NS later), so that the wait counts the compiler derives at
    // the loop's entry are those of its steady state
    int j0[NS];
    static_for<NS>([&](auto I) { j0[I.value] = fetch_j(clampq(q0 + I.value)); });
    static_for<NS>([&](auto I) {
      fetch_d(clampq(q0 + I.value), dset[I.value]);
      fetch_x(j0[I.value], xset[I.value]);
      jset[I.value] = fetch_j(clampq(q0 + NS + I.value));
    });
    store_d(q0 & 1, dset[0], q0);
    store_x(q0 & 1, xset[0]);
  }
  __syncthreads();
  for (int qb = q0; qb < q1; qb += NS) {
    static_for<NS>([&](auto I) __attribute__((always_inline)) {   // inlined: the register
      constexpr int c = I.value;                                   // sets must not escape
      const int qd = qb + c;
      const uint8_t* xb = xs[qd & 1] + rw;
      const uint4* dgb = dg[qd & 1];
      v4i bf[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        // B operand: row rw + 16 rt + m, columns 16 kb + 0..15.  Transposing 8-byte
        // reads (ds_read_b64_tr_b8): in each group of 16 lanes, byte b of the result
        // of lane 16 g + 8 e + j is byte j of what lane 16 g + 2 b + e read.  Lane L
        // reads rows 8 (L & 1) .. +7 of column 16 (L >> 4) + 8 h + ((L >> 1) & 7),
        // so lane (m, kb) receives row m of columns 16 kb + 8 h .. +7 in order.
        v2i r[2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
          r[h] = __builtin_amdgcn_ds_read_tr8_b64_v2i32(
              (__attribute__((address_space(3))) v2i*)(xb +
                  (16 * kb + 8 * h + ((lane >> 1) & 7)) * XSB + 8 * (lane & 1) + 16 * rt));
        bf[rt] = v4i{r[0].x, r[0].y, r[1].x, r[1].y};
      }
#pragma unroll
      for (int r = 0; r < NRT; ++r)
#pragma unroll
        for (int sl = 0; sl < kCS; ++sl) {
          const uint4 a4 = dgb[(r * kCS + sl) * 64 + lane];
          const v4i af = v4i{(int)a4.x, (int)a4.y, (int)a4.z, (int)a4.w};
#pragma unroll
          for (int rt = 0; rt < RT; ++rt)
            acc[rt][r][sl] =
                __builtin_amdgcn_mfma_i32_16x16x64_i8(af, bf[rt], acc[rt][r][sl], 0, 0, 0);
        }
      // every wavefront has finished reading buffers (qd + 1) & 1 (step qd - 1)
      // before the barrier that ended that step, so they can be refilled now
      store_d((qd + 1) & 1, dset[(c + 1) % NS], qd + 1);
      store_x((qd + 1) & 1, xset[(c + 1) % NS]);
      __builtin_amdgcn_sched_barrier(0);
      const int jx = jset[c];
      fetch_d(clampq(qd + NS), dset[c]);
      fetch_x(jx, xset[c]);
      jset[c] = fetch_j(clampq(qd + 2 * NS));
      __builtin_amdgcn_sched_barrier(0);
      __syncthreads();
    });
  }
  // lane holds C[rhs = r*16 + 4 kb + i][row = rb + rw + 16 rt + m]
#pragma unroll
  for (int r = 0; r < NRT; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = r * 16 + 4 * kb + i;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        long long P = 0;
#pragma unroll
        for (int sl = 0; sl < kCS; ++sl) P = P * 128 + (long long)acc[rt][r][sl][i];
        b.partial[((int64_t)split * Kp + k) * g.n_pad + rb + rw + 16 * rt + m] = P;
      }
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
  const int seff = bsplits((*b.count + 63) / 64, smax, min_per);
  double q[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // mean correction of X~ B: d_k 2^-27 sum_j m_j U_kj over the kDigitBlocks (= 256,
  // one per thread) partials, summed by the block's fixed reduction tree
  static_assert(kDigitBlocks == 256, "one digit-block partial per thread");
  double offk;
  {
    double o[1] = {b.poff[(int64_t)threadIdx.x * Kp + k]};
    block_sum<256, 1, double>(o, red);
    offk = o[0] * (b.bscale[k] / (double)(1ll << kCBits));
  }
  if (i < n && k < b.K && b.kact[k]) {
    long long P = 0;   // exact: the splits' integer sums
    for (int sp = 0; sp < seff; ++sp) P += b.partial[((int64_t)sp * Kp + k) * n_pad + i];
    const double s = b.beta0[k] - (*b.count > 0 ? offk : 0.0) +
                     (double)P * (b.bscale[k] / (double)(1ll << kCBits));
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

// one wavefront per right-hand side k (grid Kp): each lane sums the blocks q = lane,
// lane + 64, ... in order, then a fixed butterfly combines the lanes (deterministic)
__global__ __launch_bounds__(64) void k_bfinal(BatchBufs b, int nblk, int Kp) {
  const int k = blockIdx.x, lane = threadIdx.x;
  double s0 = 0, mx = 0, s2 = 0, s3 = 0, s4 = 0;
  for (int q = lane; q < nblk; q += 64) {
    const double* o = b.bpart + ((int64_t)q * Kp + k) * 8;
    s0 += o[0]; mx = fmax(mx, o[1]); s2 += o[2]; s3 += o[3]; s4 += o[4];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    s0 += __shfl_xor(s0, off); mx = fmax(mx, __shfl_xor(mx, off));
    s2 += __shfl_xor(s2, off); s3 += __shfl_xor(s3, off); s4 += __shfl_xor(s4, off);
  }
  if (lane != 0) return;
  b.tsum[k] = s0;
  // digit scale: the smallest power of two >= max |theta_k| (1 while theta_k = 0)
  int ex = 0;
  const double fr = frexp(mx > 0 ? mx : 1.0, &ex);
  b.scale[k] = ldexp(1.0, fr == 0.5 ? ex - 1 : ex);
  b.norms[k * 4 + 0] = s2;
  b.norms[k * 4 + 1] = s3;
  b.norms[k * 4 + 2] = s4;
}

// One k_bgemm launch: groups per block = (WPB / wps) GW, two digit tiles of LDS.
// The block's threads stage every digit row of a tile: 64 WPB DL >= S Kp * 4 SPT.
template <int TW, int GW, int DL, int SPT, int WPB, int NS, int S, bool CERT, bool SA = false>
static hipError_t launch_bgemm(const Geom& g, const BatchBufs& b, const CertArgs& ca, int Kp,
                               int wps, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (64 * WPB * DL < S * Kp * 4 * SPT || WPB % wps || Kp > 16 * TW * wps)
    return hipErrorInvalidValue;
  auto kern = k_bgemm<TW, GW, DL, SPT, WPB, NS, S, CERT, SA>;
  const size_t lds = (size_t)2 * S * Kp * drow_bytes<SPT>() +
                     (SA ? (size_t)2 * (WPB / wps) * GW * SPT * 1024 : 0);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const int64_t per_block = (int64_t)(WPB / wps) * GW;
  const dim3 grid((unsigned)((g.ngroups() + per_block - 1) / per_block));
  // allow more than 64 KB of dynamic LDS for this kernel (a cheap host call)
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (ev0) (void)hipEventRecord(ev0, s);
  hipLaunchKernelGGL(kern, grid, dim3(64 * WPB), lds, s, g, b, ca, Kp, wps);
  if (ev1) (void)hipEventRecord(ev1, s);
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Exact-integer certificate (batched right-hand sides).  The dual point is
// theta_q = unit T, T integer: a point of the dual feasible set of the
// Lagrangian dual (box, zero sum) whose products x~_j^T theta_q the int8 matrix
// cores give exactly, so the only rounding left is in the final FP64 scalings.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_cquant(const double* __restrict__ tp, int64_t n,
                                                 int64_t n_pad, double tau, double unit,
                                                 const double* __restrict__ y, int* tq, int8_t* dig,
                                                 int kc, int Kc, double* out) {
  __shared__ long long rs[16], rmx[16], rmn[16];
  __shared__ int rmxi[16], rmni[16];
  __shared__ double rd[16];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  // box in steps: Tlo = ceil(((tau - 1) / n) / unit), Thi = floor((tau / n) / unit)
  const long long Tlo = (long long)ceil(((tau - 1.0) / (double)n) / unit);
  const long long Thi = (long long)floor((tau / (double)n) / unit);
  long long sum = 0, mx = LLONG_MIN, mn = LLONG_MAX;
  int mxi = 0, mni = 0;
  for (int64_t i = t; i < n; i += 1024) {
    long long T = (long long)(tp[i] / unit);   // truncation toward zero
    T = T > Thi ? Thi : (T < Tlo ? Tlo : T);
    tq[i] = (int)T;
    sum += T;
    if (T > mx) { mx = T; mxi = (int)i; }   // first index of the maximum (i increases)
    if (T < mn) { mn = T; mni = (int)i; }
  }
  // wavefront reductions (ties: smallest index)
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    sum += __shfl_xor(sum, off);
    const long long omx = __shfl_xor(mx, off), omn = __shfl_xor(mn, off);
    const int omxi = __shfl_xor(mxi, off), omni = __shfl_xor(mni, off);
    if (omx > mx || (omx == mx && omxi < mxi)) { mx = omx; mxi = omxi; }
    if (omn < mn || (omn == mn && omni < mni)) { mn = omn; mni = omni; }
  }
  if (lane == 0) { rs[wid] = sum; rmx[wid] = mx; rmn[wid] = mn; rmxi[wid] = mxi; rmni[wid] = mni; }
  __syncthreads();
  if (t == 0) {
    long long S0 = 0, M = LLONG_MIN, N = LLONG_MAX;
    int Mi = 0, Ni = 0;
    for (int w = 0; w < 16; ++w) {
      S0 += rs[w];
      if (rmx[w] > M || (rmx[w] == M && rmxi[w] < Mi)) { M = rmx[w]; Mi = rmxi[w]; }
      if (rmn[w] < N || (rmn[w] == N && rmni[w] < Ni)) { N = rmn[w]; Ni = rmni[w]; }
    }
    double status = 0.0;
    if (S0 > 0) {
      if (M - S0 >= Tlo) tq[Mi] = (int)(M - S0); else status = 1.0;
    } else if (S0 < 0) {
      if (N - S0 <= Thi) tq[Ni] = (int)(N - S0); else status = 1.0;
    }
    out[7] = status;
  }
  __threadfence_block();
  __syncthreads();
  // digits and y^T theta_q
  double q[1] = {0.0};
  for (int64_t i = t; i < n_pad; i += 1024) {
    long long rest = i < n ? (long long)tq[i] : 0;
    if (i < n) q[0] += y[i] * (double)rest;
#pragma unroll
    for (int sl = kCertSlices - 1; sl > 0; --sl) {
      const long long lo = ((rest + 64) & 127) - 64;
      dig[((int64_t)sl * Kc + kc) * n_pad + i] = (int8_t)lo;
      rest = (rest - lo) >> 7;
    }
    dig[(int64_t)kc * n_pad + i] = (int8_t)rest;
  }
  // block sum in a fixed order
  double v = q[0];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  if (lane == 0) rd[wid] = v;
  __syncthreads();
  if (t == 0) {
    double a = 0.0;
    for (int w = 0; w < 16; ++w) a += rd[w];
    out[2] = a * unit;
  }
}

hipError_t launch_cert_quantize(const double* theta_p, int64_t n, int64_t n_pad, double tau,
                                double unit, const double* y, int* tq, int8_t* dig, int kc,
                                int Kc, double* out, hipStream_t s) {
  if (kc < 0 || kc >= Kc || n > 0x7fffffffll || !(unit > 0.0)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cquant, dim3(1), dim3(1024), 0, s, theta_p, n, n_pad, tau, unit, y, tq, dig,
                     kc, Kc, out);
  return hipGetLastError();
}

int64_t cert_group_sets(const Geom& g) { return (g.ngroups() + 3) / 4; }

// GW = 4 groups per wavefront (the group sets of c.gmax); 8-wavefront blocks;
// 4 slices hold 32 accumulator registers more than an iteration's 3, so the
// digit tiles are shorter (at most 5 staging loads per thread, no spills); shared
// A from 3 tiles on, as in the iteration.
hipError_t launch_cert_pass(const Geom& g, const CertArgs& c, int Kc, hipStream_t s) {
  if (g.fmt != I8 || g.rpl != 16 || Kc % 16 || Kc < 16 || Kc > 128 || c.K > Kc)
    return hipErrorInvalidValue;
  const BatchBufs b{};
  constexpr int S = kCertSlices;
  switch (Kc / 16) {   // DL = ceil(16 SPT Kc / (64 WPB))
    case 1: return launch_bgemm<1, 4, 1, 2, 8, 2, S, true>(g, b, c, Kc, 1, s, nullptr, nullptr);
    case 2: return launch_bgemm<2, 4, 2, 2, 8, 2, S, true>(g, b, c, Kc, 1, s, nullptr, nullptr);
    case 3: return launch_bgemm<2, 4, 4, 2, 8, 2, S, true, true>(g, b, c, Kc, 2, s, nullptr, nullptr);
    case 4: return launch_bgemm<2, 4, 4, 2, 8, 2, S, true, true>(g, b, c, Kc, 2, s, nullptr, nullptr);
    case 5: return launch_bgemm<2, 4, 5, 2, 8, 2, S, true, true>(g, b, c, Kc, 4, s, nullptr, nullptr);
    case 6: return launch_bgemm<2, 4, 4, 1, 8, 2, S, true, true>(g, b, c, Kc, 4, s, nullptr, nullptr);
    case 7: return launch_bgemm<2, 4, 4, 1, 8, 2, S, true, true>(g, b, c, Kc, 4, s, nullptr, nullptr);
    case 8: return launch_bgemm<2, 4, 4, 1, 8, 2, S, true, true>(g, b, c, Kc, 4, s, nullptr, nullptr);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Launch variants the batched solve's autotuner times per batch width.  Back-
// product: variant 0 is the configuration chosen per tile count (one or two tiles
// per wavefront, GW = 4 groups, GW * TW * S * 4 <= 96 accumulators; wps = wavefronts
// sharing a set of groups; blocks of 8 wavefronts, so that at about 200 VGPRs one
// block fills a CU and a staged digit tile serves 8 GW / wps groups; with 3 to 8
// tiles the set's A fragments are staged once in LDS too), variant 1 the same with
// GW = 2 (half the accumulators, twice the blocks), variant 2 for 1 or 2 tiles a
// longer digit tile (SPT 4, one barrier per 256 rows) or the shared-A form; variant
// 3 for 1 or 2 tiles takes 3 groups per wavefront in blocks of 12 wavefronts (about
// 150 VGPRs, three wavefronts per SIMD: a 1M-column design is 6.8 rounds of blocks on
// 256 CUs instead of 7.6, and a CU holds 12 wavefronts instead of 8).
// DL = ceil(12 SPT Kp / (64 WPB)) digit loads per thread and tile.

hipError_t launch_bgemm_variant(const Geom& g, const BatchBufs& b, int Kp, int v, hipStream_t s,
                                hipEvent_t ev0, hipEvent_t ev1) {
  const CertArgs c{};
  const int nrt = Kp / 16;
  if (v < 0 || v >= bgemm_variants()) return hipErrorInvalidValue;
  if (v == 3) {   // 12-wavefront blocks, 3 groups per wavefront (1 or 2 tiles; else variant 0)
    if (nrt == 1) return launch_bgemm<1, 3, 1, 2, 12, 2, kBS, false>(g, b, c, Kp, 1, s, ev0, ev1);
    if (nrt == 2) return launch_bgemm<2, 3, 1, 2, 12, 2, kBS, false>(g, b, c, Kp, 1, s, ev0, ev1);
    v = 0;
  }
  switch (nrt) {
    case 1:
      if (v == 0) return launch_bgemm<1, 4, 1, 2, 8, 2, kBS, false>(g, b, c, Kp, 1, s, ev0, ev1);
      if (v == 1) return launch_bgemm<1, 2, 1, 2, 8, 2, kBS, false>(g, b, c, Kp, 1, s, ev0, ev1);
      return launch_bgemm<1, 4, 2, 4, 8, 2, kBS, false>(g, b, c, Kp, 1, s, ev0, ev1);
    case 2:
      if (v == 0) return launch_bgemm<2, 4, 2, 2, 8, 2, kBS, false>(g, b, c, Kp, 1, s, ev0, ev1);
      if (v == 1) return launch_bgemm<2, 2, 2, 2, 8, 2, kBS, false>(g, b, c, Kp, 1, s, ev0, ev1);
      return launch_bgemm<1, 4, 2, 2, 8, 2, kBS, false, true>(g, b, c, Kp, 2, s, ev0, ev1);
    case 3:
    case 4:
      if (v == 1) return launch_bgemm<2, 2, 3, 2, 8, 2, kBS, false, true>(g, b, c, Kp, 2, s, ev0, ev1);
      return launch_bgemm<2, 4, 3, 2, 8, 2, kBS, false, true>(g, b, c, Kp, 2, s, ev0, ev1);
    case 5:
      if (v == 1) return launch_bgemm<2, 2, 4, 2, 8, 2, kBS, false, true>(g, b, c, Kp, 4, s, ev0, ev1);
      return launch_bgemm<2, 4, 4, 2, 8, 2, kBS, false, true>(g, b, c, Kp, 4, s, ev0, ev1);
    case 6:
    case 7:
    case 8:
      if (v == 1) return launch_bgemm<2, 2, 6, 2, 8, 2, kBS, false, true>(g, b, c, Kp, 4, s, ev0, ev1);
      return launch_bgemm<2, 4, 6, 2, 8, 2, kBS, false, true>(g, b, c, Kp, 4, s, ev0, ev1);
  }
  return hipErrorInvalidValue;
}

// Union product: rows per wavefront 16 RT with RT * NRT * 16 <= 128 accumulator
// registers; variants 0, 1, 2 = blocks of 8, 4 and 16 wavefronts sharing the staged
// tile and digits (n_pad is a multiple of 1024 >= 16 W RT rows); splits of the union
// along y.
// The split count (the results do not depend on it: exact integer split sums) is
// the largest that lets every block of the grid be resident at once, so that a
// large union runs as one round of blocks instead of ending in a partly empty
// round; never fewer than smin (the int32 limit on columns per split), never more
// than kBaxpySplits (the partial buffer).
static int device_cus() {
  static std::atomic<int> cus[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int c = cus[dev].load(std::memory_order_relaxed);
  if (c <= 0) {
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1)
      c = 256;
    cus[dev].store(c, std::memory_order_relaxed);
  }
  return c;
}

template <int RT, int NRT, int W>
static hipError_t launch_baxpy_k(const Geom& g, const BatchBufs& b, int smin, int min_per,
                                 hipStream_t s, int* splits) {
  if (smin > kBaxpySplits) return hipErrorInvalidValue;
  auto kern = k_baxpy<RT, NRT, W>;
  static std::atomic<int> per_cu{0};   // resident blocks per CU (one code object: gfx950)
  int bpc = per_cu.load(std::memory_order_relaxed);
  if (bpc <= 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, reinterpret_cast<const void*>(kern),
                                                     64 * W, 0) != hipSuccess || bpc < 1)
      bpc = 1;
    per_cu.store(bpc, std::memory_order_relaxed);
  }
  const int64_t rowblocks = g.n_pad / (16 * W * RT);
  int64_t sp = (int64_t)device_cus() * bpc / (rowblocks > 0 ? rowblocks : 1);
  sp = sp < smin ? smin : sp;
  sp = sp < 1 ? 1 : (sp > kBaxpySplits ? kBaxpySplits : sp);
  hipLaunchKernelGGL(kern, dim3((unsigned)rowblocks, (unsigned)sp), dim3(64 * W), 0, s, g, b,
                     (int)sp, min_per);
  if (splits) *splits = (int)sp;
  return hipGetLastError();
}

template <int W>
static hipError_t launch_baxpy_w(const Geom& g, const BatchBufs& b, int nrt, int smin, int min_per,
                                 hipStream_t s, int* splits) {
  switch (nrt) {
    case 1: return launch_baxpy_k<4, 1, W>(g, b, smin, min_per, s, splits);
    case 2: return launch_baxpy_k<2, 2, W>(g, b, smin, min_per, s, splits);
    case 3: return launch_baxpy_k<1, 3, W>(g, b, smin, min_per, s, splits);
    case 4: return launch_baxpy_k<1, 4, W>(g, b, smin, min_per, s, splits);
    case 5: return launch_baxpy_k<1, 5, W>(g, b, smin, min_per, s, splits);
    case 6: return launch_baxpy_k<1, 6, W>(g, b, smin, min_per, s, splits);
    case 7: return launch_baxpy_k<1, 7, W>(g, b, smin, min_per, s, splits);
    case 8: return launch_baxpy_k<1, 8, W>(g, b, smin, min_per, s, splits);
  }
  return hipErrorInvalidValue;
}

// 16-wavefront blocks cap a wavefront at 128 VGPRs, which from 5 tiles on would spill
// the accumulators (there variant 2 is the 8-wavefront block) and at one tile the
// three X register sets of 64 rows (so one tile takes 32 rows per wavefront).
template <>
hipError_t launch_baxpy_w<16>(const Geom& g, const BatchBufs& b, int nrt, int smin, int min_per,
                              hipStream_t s, int* splits) {
  switch (nrt) {
    case 1: return launch_baxpy_k<2, 1, 16>(g, b, smin, min_per, s, splits);
    case 2: return launch_baxpy_k<2, 2, 16>(g, b, smin, min_per, s, splits);
    case 3: return launch_baxpy_k<1, 3, 16>(g, b, smin, min_per, s, splits);
    case 4: return launch_baxpy_k<1, 4, 16>(g, b, smin, min_per, s, splits);
  }
  return launch_baxpy_w<8>(g, b, nrt, smin, min_per, s, splits);
}

hipError_t launch_baxpy_variant(const Geom& g, const BatchBufs& b, int Kp, int smin, int min_per,
                                int v, hipStream_t s, int* splits) {
  if (g.n_pad % 1024) return hipErrorInvalidValue;
  const int nrt = Kp / 16;
  if (v == 0) return launch_baxpy_w<8>(g, b, nrt, smin, min_per, s, splits);
  if (v == 1) return launch_baxpy_w<4>(g, b, nrt, smin, min_per, s, splits);
  if (v == 2) return launch_baxpy_w<16>(g, b, nrt, smin, min_per, s, splits);
  return hipErrorInvalidValue;
}

hipError_t launch_batch_iteration(const Geom& g, const BatchBufs& b, int Kp, double mu,
                                  double sigma, double eta0, int smin, int min_per,
                                  const BatchTiles& tiles, hipStream_t s, hipEvent_t ev0,
                                  hipEvent_t ev1) {
  if (g.fmt != I8 || g.rpl != 16 || Kp % 16 || Kp > 128) return hipErrorInvalidValue;
  const unsigned nb = (unsigned)(g.n_pad / 256);
  const int nrt = Kp / 16;
  hipLaunchKernelGGL(k_bdigits, dim3(nb, Kp), dim3(256), 0, s, b, g.n, g.n_pad, Kp);
  hipLaunchKernelGGL(k_bdsum, dim3(Kp), dim3(64), 0, s, b, (int)nb, Kp);
  hipError_t e = launch_bgemm_variant(g, b, Kp, tiles.bgemm, s, ev0, ev1);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bcount, dim3(kCompactBlocks), dim3(1024), 0, s, g.ngroups(), b, nrt);
  hipLaunchKernelGGL(k_bscatter, dim3(kCompactBlocks), dim3(1024), 0, s, g.ngroups(), b, nrt,
                     eta0, Kp);
  hipLaunchKernelGGL(k_bbmax, dim3(kDigitBlocks), dim3(256), 0, s, g, b, Kp);
  hipLaunchKernelGGL(k_bbdigits, dim3(kDigitBlocks), dim3(256), 0, s, g, b, Kp);
  int smax = 0;
  e = launch_baxpy_variant(g, b, Kp, smin, min_per, tiles.baxpy, s, &smax);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bupdate, dim3(nb, Kp), dim3(256), 0, s, b, g.n, g.n_pad, Kp, mu, sigma,
                     smax, min_per);
  hipLaunchKernelGGL(k_bfinal, dim3(Kp), dim3(64), 0, s, b, (int)nb, Kp);
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

__global__ void k_zero_int(int* p) {
  if (threadIdx.x == 0) p[0] = 0;
}

// Largest byte of the store (the matrix cores read int8 codes as signed).
__global__ __launch_bounds__(256) void k_max_code(const uint4* __restrict__ x, int64_t n16, int* out) {
  uint32_t mx = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (int64_t)gridDim.x * 256) {
    const uint4 v = x[i];
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int k = 0; k < 4; ++k) mx = max(mx, (w[q] >> (8 * k)) & 0xffu);
  }
  for (int off = 32; off >= 1; off >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, off));
  if ((threadIdx.x & 63) == 0) atomicMax(out, (int)mx);
}

hipError_t launch_max_code(const Geom& g, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, out);
  hipLaunchKernelGGL(k_max_code, dim3(4096), dim3(256), 0, s,
                     reinterpret_cast<const uint4*>(g.X), g.store_bytes() / 16, out);
  return hipGetLastError();
}

}  // namespace pqr
