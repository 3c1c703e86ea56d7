// Device helpers shared by the gfx950 kernels: MFMA operand layout, Philox
// draws, block reductions and a coherent double max.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double v4d __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4_f64 (CDNA3/CDNA4).  For a wave of 64 lanes:
//   A operand (16 x 4):  lane l holds A[l % 16][l / 16]
//   B operand (4 x 16):  lane l holds B[l / 16][l % 16]
//   C/D (16 x 16):       lane l, register r holds C[l / 16 + 4 r][l % 16]
// (checked on gfx950 with an in-bounds probe of known operands).
__device__ __forceinline__ v4d mfma_f64_16x16x4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- Philox ----
// Philox4x64-10 of Salmon, Moraes, Dror and Shaw (SC'11): ten rounds, each two
// 64x64->128-bit products with the multipliers M0, M1; the key is bumped by the
// Weyl constants W0, W1 between rounds.
struct Philox4 { uint64_t w[4]; };

__device__ __forceinline__ Philox4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                 uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += W0; k1 += W1;
  }
  Philox4 out;
  out.w[0] = c0; out.w[1] = c1; out.w[2] = c2; out.w[3] = c3;
  return out;
}

// Stream tags of the counter (tag, sweep, (tau << 1) | direction, site).
enum { TAG_INIT = 0, TAG_FLIP = 1, TAG_GAUSS = 2, TAG_LANGEVIN = 3 };

__device__ __forceinline__ double unit_double(uint64_t w) {
  return (double)(w >> 11) * 0x1.0p-53;
}

// ------------------------------------------------------------ reductions ----
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  // red: LDS scratch of NT/64 doubles
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) s = fmax(s, red[i]);
  return s;
}

// Both halves of a double read from one lane (uniform lane index).
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ------------------------------------------------- DPP wave reductions ----
// Whole-wave reductions on VALU data-parallel moves instead of LDS permutes:
// xor-1 and xor-2 quad permutes, the half-row and row mirrors (max/sum over
// 8 and 16 lanes), then row_bcast15 / row_bcast31 carry the row results up;
// lane 63 ends with the wave's result, read with readlane.  OLD is what a
// lane outside the row mask receives (the identity of the operation).
template <int CTRL, int RM>
__device__ __forceinline__ double dpp_d(double v, double old) {
  const long long b = __double_as_longlong(v), o = __double_as_longlong(old);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)b, CTRL, RM, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, RM, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_max_d(double v) {
  const double ni = -INFINITY;
  v = fmax(v, dpp_d<0xB1, 0xF>(v, ni));
  v = fmax(v, dpp_d<0x4E, 0xF>(v, ni));
  v = fmax(v, dpp_d<0x141, 0xF>(v, ni));
  v = fmax(v, dpp_d<0x140, 0xF>(v, ni));
  v = fmax(v, dpp_d<0x142, 0xA>(v, ni));
  v = fmax(v, dpp_d<0x143, 0xC>(v, ni));
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_sum_d(double v) {
  v += dpp_d<0xB1, 0xF>(v, 0.0);
  v += dpp_d<0x4E, 0xF>(v, 0.0);
  v += dpp_d<0x141, 0xF>(v, 0.0);
  v += dpp_d<0x140, 0xF>(v, 0.0);
  v += dpp_d<0x142, 0xA>(v, 0.0);
  v += dpp_d<0x143, 0xC>(v, 0.0);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// K independent wave sums, each DPP round applied to all K values before the
// next, so their latencies overlap; every lane gets the K totals.
template <int K>
__device__ __forceinline__ void wave_sum_d_n(double (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_d<0xB1, 0xF>(v[k], 0.0);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_d<0x4E, 0xF>(v[k], 0.0);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_d<0x141, 0xF>(v[k], 0.0);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_d<0x140, 0xF>(v[k], 0.0);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_d<0x142, 0xA>(v[k], 0.0);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_d<0x143, 0xC>(v[k], 0.0);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = readlane_d(v[k], 63);
}

// ------------------------------------------- several sums in one pass ----
// Lane exchanges that write every lane: DPP quad permutes (xor 1, xor 2), the
// half-row mirror (lane i of 8 <-> 7 - i), a row rotation by 8 (xor 8), and the
// gfx950 permlane swaps across rows (xor 16) and halves (xor 32).
template <int CTRL>
__device__ __forceinline__ double dpp_all(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int CTRL>
__device__ __forceinline__ int dpp_all_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}

// lane S of each quad to the whole quad
template <int S>
__device__ __forceinline__ double quad_bcast_d(double v) {
  return dpp_all<S * 0x55>(v);
}

// the same for a lane index known only after unrolling
__device__ __forceinline__ double quad_bcast_d(double v, int s) {
  switch (s & 3) {
    case 0: return quad_bcast_d<0>(v);
    case 1: return quad_bcast_d<1>(v);
    case 2: return quad_bcast_d<2>(v);
    default: return quad_bcast_d<3>(v);
  }
}

// The pair (v of this lane, v of the lane 16 / 32 away) in some order:
// permlane16_swap of v with itself leaves the even-row data in one result and
// the odd-row data in the other; permlane32_swap does the same for the halves.
__device__ __forceinline__ void pair_xor16(double v, double& x, double& y) {
  const long long b = __double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
  x = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
  y = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}

__device__ __forceinline__ void pair_xor32(double v, double& x, double& y) {
  const long long b = __double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
  x = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
  y = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}

__device__ __forceinline__ double add_xor16(double v) {
  double x, y;
  pair_xor16(v, x, y);
  return x + y;
}

__device__ __forceinline__ double add_xor32(double v) {
  double x, y;
  pair_xor32(v, x, y);
  return x + y;
}

// Whole-wave max / min with the result in every lane (no readlane): xor 1,
// xor 2, the half-row mirror, xor 8, then the permlane swaps.
__device__ __forceinline__ double wave_max_all(double v) {
  v = fmax(v, dpp_all<0xB1>(v));
  v = fmax(v, dpp_all<0x4E>(v));
  v = fmax(v, dpp_all<0x141>(v));
  v = fmax(v, dpp_all<0x128>(v));
  double x, y;
  pair_xor16(v, x, y);
  v = fmax(x, y);
  pair_xor32(v, x, y);
  return fmax(x, y);
}

__device__ __forceinline__ int wave_min_all_i(int v) {
  v = min(v, dpp_all_i<0xB1>(v));
  v = min(v, dpp_all_i<0x4E>(v));
  v = min(v, dpp_all_i<0x141>(v));
  v = min(v, dpp_all_i<0x128>(v));
  const auto a = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
  v = min((int)a[0], (int)a[1]);
  const auto b = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
  return min((int)b[0], (int)b[1]);
}

// One halving step of a multi-sum: lanes whose BIT is 0 keep the first half of
// the values, the others the second half, and each adds its partner's copy of
// the kept half (the partner of CTRL differs in BIT and in no earlier one).
template <int CTRL, int BIT, int N>
__device__ __forceinline__ void split_half(double* x, int lane) {
  const bool up = (lane >> BIT) & 1;
#pragma unroll
  for (int k = 0; k < N / 2; ++k) {
    const double lo = x[k], hi = x[k + N / 2];
    const double send = up ? lo : hi;
    const double keep = up ? hi : lo;
    x[k] = keep + dpp_all<CTRL>(send);
  }
}

// K (2, 4 or 8) wave sums at once by recursive halving: the split steps leave
// one value per lane, value wave_sums_index<K>(lane) (lane bits 2, 0, 1 spell
// it from the top); the remaining lanes are summed by exchanges.  Returns the
// lane's total; every lane also reads all K totals into v.  About 10
// exchanges for K = 8 where K separate reductions take 6 K.
template <int K>
__device__ __forceinline__ int wave_sums_index(int lane) {
  int j = ((lane >> 2) & 1) * (K / 2);
  if constexpr (K >= 4) j += (lane & 1) * (K / 4);
  if constexpr (K >= 8) j += (lane >> 1) & 1;
  return j;
}

// true for exactly one lane per value: lanes 0..7 with the unused bits clear
template <int K>
__device__ __forceinline__ bool wave_sums_holder(int lane) {
  constexpr int unused = (K == 8) ? 0 : (K == 4 ? 2 : 3);
  return lane < 8 && (lane & unused) == 0;
}

template <int K>
__device__ __forceinline__ double wave_sums(double (&v)[K]) {
  static_assert(K == 2 || K == 4 || K == 8, "K must be 2, 4 or 8");
  const int lane = threadIdx.x & 63;
  double x[K];
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] = v[k];
  split_half<0x141, 2, K>(x, lane);                       // half-row mirror: bit 2
  if constexpr (K >= 4) split_half<0xB1, 0, K / 2>(x, lane);   // xor 1: bit 0
  if constexpr (K >= 8) split_half<0x4E, 1, K / 4>(x, lane);   // xor 2: bit 1
  double t = x[0];
  if constexpr (K < 4) t += dpp_all<0xB1>(t);      // xor 1
  if constexpr (K < 8) t += dpp_all<0x4E>(t);      // xor 2
  t += dpp_all<0x128>(t);                           // row rotate by 8: xor 8
  t = add_xor16(t);
  t = add_xor32(t);
#pragma unroll
  for (int j = 0; j < K; ++j) {
    int l = ((j / (K / 2)) & 1) << 2;
    if constexpr (K >= 4) l |= (j / (K / 4)) & 1;
    if constexpr (K >= 8) l |= (j & 1) << 1;
    v[j] = readlane_d(t, l);
  }
  return t;
}

__device__ __forceinline__ int wave_min_i(int v) {
  const int big = 0x7fffffff;
  v = min(v, __builtin_amdgcn_update_dpp(big, v, 0xB1, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(big, v, 0x4E, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(big, v, 0x141, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(big, v, 0x140, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(big, v, 0x142, 0xA, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(big, v, 0x143, 0xC, 0xF, false));
  return __builtin_amdgcn_readlane(v, 63);
}

// max of non-negative doubles through their ordered bit patterns
__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
  if (!(v >= 0.0)) v = __longlong_as_double(0x7ff8000000000000ll);  // NaN propagates as the largest
  atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

// Scale modes of the GEMM epilogue and loaders.
enum { SC_NONE = 0, SC_VAL = 1, SC_EXP = 2, SC_INV_BIG = 3, SC_SMALL = 4, SC_INV = 5 };

__device__ __forceinline__ double scale_of(int mode, const double* v, double coef, int i) {
  switch (mode) {
    case SC_VAL: return v[i];
    case SC_EXP: return exp(coef * v[i]);
    case SC_INV_BIG: return 1.0 / fmax(v[i], 1.0);
    case SC_SMALL: return fmin(v[i], 1.0);
    case SC_INV: return 1.0 / v[i];
    default: return 1.0;
  }
}
