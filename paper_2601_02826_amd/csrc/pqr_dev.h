// Device-side building blocks of libpqr (gfx950, wave64).
//
// Layout of the design store: rows padded with zeros to n_pad, a multiple of
// 64*RPL, and cut into chunks of 64*RPL rows; a wavefront reads one column's
// chunk (a "segment") with each lane holding RPL consecutive rows, so every
// read is contiguous and fully coalesced, and the lane's RPL values of theta
// are loaded once and reused across the 16 columns of a column group.  The
// segments of one group and chunk are adjacent in memory (see Geom::seg).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pqr {

constexpr int kWave = 64;
constexpr int kGroup = 16;  // columns per group: one wavefront per group in the sweep

enum Fmt : int { F64 = 0, F32 = 1, BF16 = 2, FP8 = 3, I8 = 4, B2 = 5 };

// Bytes of one column holding `rows` rows.
__host__ __device__ constexpr int64_t fmt_col_bytes(int fmt, int64_t rows) {
  return fmt == F64 ? rows * 8 : fmt == F32 ? rows * 4 : fmt == BF16 ? rows * 2
       : fmt == B2 ? rows / 4 : rows;
}

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

// ---------------------------------------------------------------------------
// Raw loads and decoding of RPL consecutive rows of one column, starting at
// row offset `row0` inside a segment.  The split lets a wavefront issue the loads of several columns before
// it decodes any of them (more bytes in flight per wavefront).
// ---------------------------------------------------------------------------
// s + sum_k p[k n_pad + i] over the splits k = 0 .. seff-1, added in that order
// (deterministic) with eight loads in flight: the split partials of one row are
// n_pad apart, and a row's sum is one thread's work.
__device__ __forceinline__ double sum_splits(const double* __restrict__ p, int seff,
                                             int64_t n_pad, int64_t i, double s) {
  int k = 0;
  for (; k + 8 <= seff; k += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(k + u) * n_pad + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; k < seff; ++k) s += p[(int64_t)k * n_pad + i];
  return s;
}

__device__ __forceinline__ float ubyte(uint32_t w, int b) { return (float)((w >> (8 * b)) & 0xffu); }

template <int FMT, int RPL> struct Raw;
template <> struct Raw<I8, 16> { uint4 v; };
template <> struct Raw<I8, 4> { uint32_t v; };
template <> struct Raw<FP8, 16> { uint4 v; };
template <> struct Raw<FP8, 4> { uint32_t v; };
template <> struct Raw<BF16, 16> { uint4 v[2]; };
template <> struct Raw<BF16, 4> { uint2 v; };
template <> struct Raw<F32, 16> { float4 v[4]; };
template <> struct Raw<F32, 4> { float4 v; };
template <> struct Raw<F64, 16> { double2 v[8]; };
template <> struct Raw<F64, 4> { double2 v[2]; };
template <> struct Raw<B2, 16> { uint32_t v; };

// columns whose raw loads are kept in flight together (VGPR budget ~64 per lane)
template <int FMT, int RPL> struct Batch { static constexpr int value = 16; };
template <> struct Batch<BF16, 16> { static constexpr int value = 8; };
template <> struct Batch<F32, 16> { static constexpr int value = 4; };
template <> struct Batch<F64, 16> { static constexpr int value = 2; };
template <> struct Batch<F32, 4> { static constexpr int value = 16; };
template <> struct Batch<F64, 4> { static constexpr int value = 8; };

template <int FMT, int RPL>
__device__ __forceinline__ Raw<FMT, RPL> load_raw(const uint8_t* __restrict__ col, int64_t row0) {
  Raw<FMT, RPL> r;
  if constexpr (FMT == I8 || FMT == FP8) {
    if constexpr (RPL == 16) r.v = *reinterpret_cast<const uint4*>(col + row0);
    else r.v = *reinterpret_cast<const uint32_t*>(col + row0);
  } else if constexpr (FMT == BF16) {
    if constexpr (RPL == 16) {
      const uint4* p = reinterpret_cast<const uint4*>(col + row0 * 2);
      r.v[0] = p[0]; r.v[1] = p[1];
    } else {
      r.v = *reinterpret_cast<const uint2*>(col + row0 * 2);
    }
  } else if constexpr (FMT == F32) {
    const float4* p = reinterpret_cast<const float4*>(col + row0 * 4);
    if constexpr (RPL == 16) { r.v[0] = p[0]; r.v[1] = p[1]; r.v[2] = p[2]; r.v[3] = p[3]; }
    else r.v = p[0];
  } else if constexpr (FMT == F64) {
    const double2* p = reinterpret_cast<const double2*>(col + row0 * 8);
#pragma unroll
    for (int q = 0; q < RPL / 2; ++q) r.v[q] = p[q];
  } else {
    static_assert(FMT == B2 && RPL == 16, "2-bit codes need 16 rows per lane");
    r.v = *reinterpret_cast<const uint32_t*>(col + row0 / 4);
  }
  return r;
}

template <int FMT, int RPL, typename T>
__device__ __forceinline__ void decode(const Raw<FMT, RPL>& r, T (&x)[RPL]) {
  if constexpr (FMT == I8) {
    if constexpr (RPL == 16) {
      const uint32_t w[4] = {r.v.x, r.v.y, r.v.z, r.v.w};
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) x[4 * q + b] = (T)ubyte(w[q], b);
    } else {
#pragma unroll
      for (int b = 0; b < 4; ++b) x[b] = (T)ubyte(r.v, b);
    }
  } else if constexpr (FMT == FP8) {
    uint32_t w[RPL / 4];
    if constexpr (RPL == 16) { w[0] = r.v.x; w[1] = r.v.y; w[2] = r.v.z; w[3] = r.v.w; }
    else w[0] = r.v;
#pragma unroll
    for (int q = 0; q < RPL / 4; ++q) {
      const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[q], false);
      const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[q], true);
      x[4 * q + 0] = (T)lo[0]; x[4 * q + 1] = (T)lo[1];
      x[4 * q + 2] = (T)hi[0]; x[4 * q + 3] = (T)hi[1];
    }
  } else if constexpr (FMT == BF16) {
    uint32_t w[RPL / 2];
    if constexpr (RPL == 16) {
      w[0] = r.v[0].x; w[1] = r.v[0].y; w[2] = r.v[0].z; w[3] = r.v[0].w;
      w[4] = r.v[1].x; w[5] = r.v[1].y; w[6] = r.v[1].z; w[7] = r.v[1].w;
    } else {
      w[0] = r.v.x; w[1] = r.v.y;
    }
#pragma unroll
    for (int q = 0; q < RPL / 2; ++q) {
      x[2 * q + 0] = (T)__uint_as_float(w[q] << 16);
      x[2 * q + 1] = (T)__uint_as_float(w[q] & 0xffff0000u);
    }
  } else if constexpr (FMT == F32) {
    if constexpr (RPL == 16) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        x[4 * q + 0] = (T)r.v[q].x; x[4 * q + 1] = (T)r.v[q].y;
        x[4 * q + 2] = (T)r.v[q].z; x[4 * q + 3] = (T)r.v[q].w;
      }
    } else {
      x[0] = (T)r.v.x; x[1] = (T)r.v.y; x[2] = (T)r.v.z; x[3] = (T)r.v.w;
    }
  } else if constexpr (FMT == F64) {
#pragma unroll
    for (int q = 0; q < RPL / 2; ++q) { x[2 * q] = (T)r.v[q].x; x[2 * q + 1] = (T)r.v[q].y; }
  } else {
    // one 32-bit word = 16 rows; byte b holds rows 4b..4b+3, row 4b+k in bits 2k..2k+1
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t t = (r.v >> (2 * k)) & 0x03030303u;
#pragma unroll
      for (int b = 0; b < 4; ++b) x[4 * b + k] = (T)ubyte(t, b);
    }
  }
}

template <int FMT, int RPL, typename T>
__device__ __forceinline__ void load_rows(const uint8_t* __restrict__ col, int64_t row0, T (&x)[RPL]) {
  decode<FMT, RPL, T>(load_raw<FMT, RPL>(col, row0), x);
}

template <int RPL, typename T>
__device__ __forceinline__ void load_vec(const T* __restrict__ v, int64_t row0, T (&x)[RPL]) {
  using V4 = typename Vec4<T>::type;
  const V4* p = reinterpret_cast<const V4*>(v + row0);
#pragma unroll
  for (int q = 0; q < RPL / 4; ++q) {
    const V4 a = p[q];
    x[4 * q + 0] = a.x; x[4 * q + 1] = a.y; x[4 * q + 2] = a.z; x[4 * q + 3] = a.w;
  }
}

// ---------------------------------------------------------------------------
// Wavefront reductions
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// Reduce 16 per-lane partial sums over the 64 lanes by halving exchanges.
// On return every lane holds the total of column group_col_of_lane(lane);
// the four lanes of a quad hold the same column.
template <typename T>
__device__ __forceinline__ T reduce16(const T (&v)[16], int lane) {
  T w8[8];
  {
    const bool up = lane & 32;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const T send = up ? v[k] : v[k + 8];
      const T keep = up ? v[k + 8] : v[k];
      w8[k] = keep + __shfl_xor(send, 32);
    }
  }
  T w4[4];
  {
    const bool up = lane & 16;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const T send = up ? w8[k] : w8[k + 4];
      const T keep = up ? w8[k + 4] : w8[k];
      w4[k] = keep + __shfl_xor(send, 16);
    }
  }
  T w2[2];
  {
    const bool up = lane & 8;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const T send = up ? w4[k] : w4[k + 2];
      const T keep = up ? w4[k + 2] : w4[k];
      w2[k] = keep + __shfl_xor(send, 8);
    }
  }
  T w1;
  {
    const bool up = lane & 4;
    const T send = up ? w2[0] : w2[1];
    const T keep = up ? w2[1] : w2[0];
    w1 = keep + __shfl_xor(send, 4);
  }
  w1 += __shfl_xor(w1, 2);
  w1 += __shfl_xor(w1, 1);
  return w1;
}

__device__ __forceinline__ int group_col_of_lane(int lane) {
  return ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
}

// Deterministic block reduction of NV values (block size BS, a multiple of 64).
template <int BS, int NV, typename T>
__device__ __forceinline__ void block_sum(T (&v)[NV], T* smem /* NV * BS/64 */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  constexpr int NWV = BS / 64;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) smem[k * NWV + wid] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    T s = 0;
    for (int w = 0; w < NWV; ++w) s += smem[k * NWV + w];
    v[k] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Control block shared by the kernels of one iteration (device memory).
// ---------------------------------------------------------------------------
struct Ctl {
  int64_t iter;          // iterations completed
  int count;             // active column groups after the last sweep
  unsigned blocks_done;  // arrival counter of the update kernel (reset by the last block)
  double beta0;          // intercept (solver scale)
  double sum_theta;      // sum_i theta_i of the current theta
  double nb[4];          // from the sweep: |dbeta|^2, |beta|^2, sum eta |dbeta|^2, -
  double nr[8];          // from the update: |dz|^2, |z|^2, |dtheta|^2, |theta|^2, |r|^2,
                         //   dtheta.(dr), sum theta, -
  double delta;          // ||w^{k+1} - w^k||_H^2 of the last iteration
  double delta_prev;
  int n_increase;        // consecutive iterations with delta growing
  int pad;
};

}  // namespace pqr
