// Blocked Householder QR with column pre-pivoting and blocked LU with partial
// pivoting, the two factorisations of the stabilisation (section
// "Stabilization - a peculiarity of the BSS algorithm").
//
// Both are right-looking with panels of nb <= 32 columns: the panel is
// factorised by one workgroup entirely in LDS (BLAS-2 work, latency bound),
// and the trailing matrix is updated with the MFMA GEMM of gemm.h (BLAS-3).
//
// QR: the columns are first ordered by decreasing 2-norm (the paper's
// "manual pivoting" variant of the stabilisation), then factorised without
// further pivoting.  Each panel produces its Householder vectors V (unit lower
// trapezoidal, stored explicitly) and the compact-WY factor VT = V T with
// H_1 ... H_nb = I - V T V^T, so that Q^T A = A - V (VT^T A) and
// Q X = X - VT (V^T X).
#pragma once
#include <utility>
#include "device_common.h"

// ------------------------------------------------------------ utilities ----
__global__ void k_set_identity(double* A, int n, int ld, size_t cs) {
  A += (size_t)blockIdx.y * cs;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  A[(size_t)i * ld + j] = (i == j) ? 1.0 : 0.0;
}

__global__ void k_fill(double* A, size_t count, double v, size_t cs) {
  A += (size_t)blockIdx.y * cs;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) A[e] = v;
}

__global__ void k_copy(double* dst, const double* src, size_t count, size_t cs) {
  dst += (size_t)blockIdx.y * cs;
  src += (size_t)blockIdx.y * cs;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) dst[e] = src[e];
}

// Batched gathers: dst[chain][0..count) <-> src[chain * cs + 0..count)
__global__ void k_gather(double* dst, const double* src, int count, size_t cs) {
  const int t = threadIdx.x;
  if (t < count) dst[(size_t)blockIdx.y * count + t] = src[(size_t)blockIdx.y * cs + t];
}

__global__ void k_scatter(double* dst, const double* src, int count, size_t cs) {
  const int t = threadIdx.x;
  if (t < count) dst[(size_t)blockIdx.y * cs + t] = src[(size_t)blockIdx.y * count + t];
}

// dst[i][j] = src[j][i] * scale(i)
__global__ void k_transpose_scale(double* dst, int ldd, const double* src, int n, const double* d, int mode,
                                  size_t cs_dst, size_t cs_src) {
  __shared__ double tile[32][33];
  dst += (size_t)blockIdx.z * cs_dst;
  src += (size_t)blockIdx.z * cs_src;
  d += (size_t)blockIdx.z * cs_src;
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int i = by + r, j = bx + tx;                       // read src[i][j]
    tile[r][tx] = (i < n && j < n) ? src[(size_t)i * n + j] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = bx + r, j = by + tx;                       // write dst[i][j] = src[j][i]
    if (i < n && j < n) dst[(size_t)i * ldd + j] = tile[tx][r] * scale_of(mode, d, 0.0, i);
  }
}

// -------------------------------------------------------- QR pre-pivoting ----
// Column norms in two steps: k_colnorm_part sums the squares of kColRows rows
// per workgroup (threads over columns, coalesced), k_colnorm_order adds the
// partial rows in a fixed order and ranks the columns.
constexpr int kColRows = 16;

__global__ __launch_bounds__(256) void k_colnorm_part(const double* M, int n, double* part, size_t cs) {
  M += (size_t)blockIdx.y * cs;
  part += (size_t)blockIdx.y * cs;
  const int r0 = blockIdx.x * kColRows;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double x[kColRows];   // every row's load in flight before the sum
#pragma unroll
    for (int r = 0; r < kColRows; ++r) x[r] = M[(size_t)min(r0 + r, n - 1) * n + j];
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < kColRows; ++r)
      if (r0 + r < n) s += x[r] * x[r];
    part[(size_t)blockIdx.x * n + j] = s;
  }
}

// piv[p] = index of the column with the p-th largest 2-norm (ties: lower
// index): the partial sums added in row-block order, then a bitonic sort of
// (norm descending, index ascending) pairs in LDS, one per thread (n <= 1024;
// the padding sorts last).  The order is total, so the result is the unique
// sorted permutation.
__global__ __launch_bounds__(1024) void k_colnorm_order(const double* part, int nblk, int n, double* norms, int* piv,
                                                        size_t cs) {
  __shared__ double sk[1024];
  __shared__ int si[1024];
  part += (size_t)blockIdx.y * cs;
  norms += (size_t)blockIdx.y * cs;
  piv = reinterpret_cast<int*>(reinterpret_cast<double*>(piv) + (size_t)blockIdx.y * cs);
  const int t = threadIdx.x;
  double s = -1.0;
  if (t < n) {
    s = 0.0;
    constexpr int U = 8;
    for (int b0 = 0; b0 < nblk; b0 += U) {
      double x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = part[(size_t)min(b0 + u, nblk - 1) * n + t];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (b0 + u < nblk) s += x[u];
    }
    s = (s == s) ? s : INFINITY;   // a NaN column sorts first; the order stays a permutation
    norms[t] = s;
  }
  sk[t] = s;
  si[t] = t;
  __syncthreads();
  for (int k = 2; k <= 1024; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int p = t ^ j;
      if (p > t) {
        const double ka = sk[t], kb = sk[p];
        const int ia = si[t], ib = si[p];
        const bool b_first = (kb > ka) || (kb == ka && ib < ia);
        if (b_first == ((t & k) == 0)) {
          sk[t] = kb; sk[p] = ka;
          si[t] = ib; si[p] = ia;
        }
      }
      __syncthreads();
    }
  }
  if (t < n) piv[t] = si[t];
}

__global__ void k_permute_cols(double* dst, const double* src, const int* piv, int n, size_t cs) {
  dst += (size_t)blockIdx.y * cs;
  src += (size_t)blockIdx.y * cs;
  piv = reinterpret_cast<const int*>(reinterpret_cast<const double*>(piv) + (size_t)blockIdx.y * cs);
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  dst[e] = src[(size_t)i * n + piv[j]];
}

// Block reflector applied to one 16-column slab: C <- C - P (S^T C) for the
// columns 16 bx .. 16 bx + 15 of an h x ncol block C (ld ldc) and the h x nbw
// factors P, S (ld ldps, nbw <= 32): with (P, S) = (V, VT) it is Q^T C for the
// trailing matrix of a QR panel, with (VT, V) it is Q C for the accumulation
// of Q.  The four waves split the rows for Z = S^T C (two 16 x 16 MFMA tiles
// each, summed through LDS), then split the 16-row tiles of C for C - P Z
// (the accumulator starts from C and P enters negated).  Operands are read
// from clamped addresses and masked, so the loads issue back to back.  C may
// live in global memory or in LDS (generic addressing).  Every wave of the
// workgroup calls it; zp and Zs are the workgroup's LDS scratch.
__device__ __forceinline__ void apply_wy_slab(const double* P, const double* S, int ldps, double* C, int ldc, int h,
                                              int ncol, int nbw, int bx, double (*zp)[2][4][64],
                                              double (*Zs)[17]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m16 = lane & 15, kk = lane >> 4;
  const int c0 = bx * 16, col = c0 + m16, colc = min(col, ncol - 1);
  const bool cin = col < ncol;
  // Z = S^T C over this wave's quarter of the rows, k-steps of 4
  const int kq = ((h + 15) / 16) * 4;
  const int kb = w * kq, ke = min(h, kb + kq);
  v4d z[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
  constexpr int U = 6;   // k-steps whose loads are issued together
  for (int kc = kb; kc < ke; kc += 4 * U) {
    double a[U][2], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int rc = min(kc + 4 * u + kk, h - 1);
#pragma unroll
      for (int t = 0; t < 2; ++t) a[u][t] = S[(size_t)rc * ldps + min(t * 16 + m16, nbw - 1)];
      b[u] = C[(size_t)rc * ldc + colc];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool rin = kc + 4 * u + kk < ke;
#pragma unroll
      for (int t = 0; t < 2; ++t) a[u][t] = (rin && t * 16 + m16 < nbw) ? a[u][t] : 0.0;
      b[u] = (rin && cin) ? b[u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < 2; ++t) z[t] = mfma_f64_16x16x4(a[u][t], b[u], z[t]);
  }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) zp[w][t][rr][lane] = z[t][rr];
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const double v = (zp[0][t][rr][lane] + zp[1][t][rr][lane]) + (zp[2][t][rr][lane] + zp[3][t][rr][lane]);
        Zs[t * 16 + kk + 4 * rr][m16] = v;   // D layout: row kk + 4 rr, column m16 of tile t
      }
  }
  __syncthreads();
  // C tile - P Z, 16-row tiles over the waves; K = nbw in steps of 4 (Z rows past nbw are zero)
  double zb[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) zb[k] = (4 * k + kk < nbw) ? Zs[4 * k + kk][m16] : 0.0;
  const int nrt = (h + 15) / 16;
  for (int tr0 = w; tr0 < nrt; tr0 += 8) {   // two row tiles per round, their loads together
    v4d acc[2];
    double pa[2][8];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int r0 = (tr0 + 4 * q) * 16, pr = min(r0 + m16, h - 1);
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) acc[q][rr] = C[(size_t)min(r0 + kk + 4 * rr, h - 1) * ldc + colc];
#pragma unroll
      for (int k = 0; k < 8; ++k) pa[q][k] = P[(size_t)pr * ldps + min(4 * k + kk, nbw - 1)];
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int k = 0; k < 8; ++k) pa[q][k] = (4 * k + kk < nbw) ? -pa[q][k] : 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[q] = mfma_f64_16x16x4(pa[q][k], zb[k], acc[q]);
    if (cin) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (tr0 + 4 * q >= nrt) break;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int r = (tr0 + 4 * q) * 16 + kk + 4 * rr;
          if (r < h) C[(size_t)r * ldc + col] = acc[q][rr];
        }
      }
    }
  }
}

// C <- C - P (S^T C) for one 16-column slab C (h rows, leading dimension
// ldc, columns >= ncol inert) and P, S: h x nbw (leading dimension ldps,
// nbw <= 16 KT), by a workgroup of NW waves.  Each wave takes an NW-th of
// the rows for S^T C and every NW-th 16-row tile for the update; every load
// of a phase is issued in one round (UZ k-steps, UC row tiles) while
// h <= 4 NW UZ, so a phase costs one memory latency.  zp: NW x KT x 4 x 64 doubles
// of LDS for the per-wave partial products; Zs: the reduced S^T C.  The
// caller puts a barrier between two calls on the same slab.
template <int NW, int KT, int UZ, int UC>
__device__ __forceinline__ void apply_wy_wide(const double* P, const double* S, int ldps, double* C, int ldc, int h,
                                              int ncol, int nbw, double* zp, double (*Zs)[17]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m16 = lane & 15, kk = lane >> 4;
  const int colc = min(m16, ncol - 1);
  const bool cin = m16 < ncol;
  const int kq = ((h + 4 * NW - 1) / (4 * NW)) * 4;
  const int kb = w * kq, ke = min(h, kb + kq);
  v4d z[KT];
#pragma unroll
  for (int t = 0; t < KT; ++t) z[t] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int kc = kb; kc < ke; kc += 4 * UZ) {
    double a[UZ][KT], b[UZ];
#pragma unroll
    for (int u = 0; u < UZ; ++u) {
      const int rc = min(kc + 4 * u + kk, h - 1);
#pragma unroll
      for (int t = 0; t < KT; ++t) a[u][t] = S[(size_t)rc * ldps + min(t * 16 + m16, nbw - 1)];
      b[u] = C[(size_t)rc * ldc + colc];
    }
#pragma unroll
    for (int u = 0; u < UZ; ++u) {
      const bool rin = kc + 4 * u + kk < ke;
#pragma unroll
      for (int t = 0; t < KT; ++t) a[u][t] = (rin && t * 16 + m16 < nbw) ? a[u][t] : 0.0;
      b[u] = (rin && cin) ? b[u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UZ; ++u)
#pragma unroll
      for (int t = 0; t < KT; ++t) z[t] = mfma_f64_16x16x4(a[u][t], b[u], z[t]);
  }
#pragma unroll
  for (int t = 0; t < KT; ++t)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) zp[((w * KT + t) * 4 + rr) * 64 + lane] = z[t][rr];
  __syncthreads();
  for (int p = w; p < 4 * KT; p += NW) {   // wave p sums the NW partials of D register (t, rr) = (p / 4, p % 4)
    const int t = p >> 2, rr = p & 3;
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) v += zp[((q * KT + t) * 4 + rr) * 64 + lane];
    Zs[t * 16 + kk + 4 * rr][m16] = v;   // D layout: row kk + 4 rr, column m16 of tile t
  }
  __syncthreads();
  double zb[4 * KT];
#pragma unroll
  for (int k = 0; k < 4 * KT; ++k) zb[k] = (4 * k + kk < nbw) ? Zs[4 * k + kk][m16] : 0.0;
  const int nrt = (h + 15) / 16;
  for (int tr0 = w; tr0 < nrt; tr0 += NW * UC) {
    v4d acc[UC];
    double pa[UC][4 * KT];
#pragma unroll
    for (int q = 0; q < UC; ++q) {
      const int r0 = (tr0 + NW * q) * 16, pr = min(r0 + m16, h - 1);
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) acc[q][rr] = C[(size_t)min(r0 + kk + 4 * rr, h - 1) * ldc + colc];
#pragma unroll
      for (int k = 0; k < 4 * KT; ++k) pa[q][k] = P[(size_t)pr * ldps + min(4 * k + kk, nbw - 1)];
    }
#pragma unroll
    for (int q = 0; q < UC; ++q)
#pragma unroll
      for (int k = 0; k < 4 * KT; ++k) pa[q][k] = (4 * k + kk < nbw) ? -pa[q][k] : 0.0;
#pragma unroll
    for (int k = 0; k < 4 * KT; ++k)
#pragma unroll
      for (int q = 0; q < UC; ++q) acc[q] = mfma_f64_16x16x4(pa[q][k], zb[k], acc[q]);
    if (cin) {
#pragma unroll
      for (int q = 0; q < UC; ++q) {
        if (tr0 + NW * q >= nrt) break;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int r = (tr0 + NW * q) * 16 + kk + 4 * rr;
          if (r < h) C[(size_t)r * ldc + m16] = acc[q][rr];
        }
      }
    }
  }
}

// Explicit Q of a QR factorisation in one launch: Q = H_0 H_1 ... H_last I
// by backward accumulation, every workgroup one 16-column slab of Q (grid
// (ceil(n / 16), chains)) held in LDS (n x 16 doubles, dynamic) from the
// identity columns to the end.  The block reflector of the panel at column
// j0 acts on rows j0.. of the slab (apply_wy_slab with (VT, V) of that
// panel, stored h x nbw at Vall + j0 n); the slab's columns left of j0 are
// still identity columns then (only later panels in this order touch them)
// and come out unchanged, and panels starting right of the slab are skipped.
__global__ __launch_bounds__(256) void k_accum_q(const double* Vall, const double* VTall, double* Q, int n, int nb,
                                                 size_t cs) {
  extern __shared__ double qs[];
  __shared__ double zp[4][2][4][64];
  __shared__ double Zs[32][17];
  {
    const size_t co = (size_t)blockIdx.y * cs;
    Vall += co; VTall += co; Q += co;
  }
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * 16, ncol = min(16, n - c0);
  for (int e = tid; e < n * 16; e += 256) {
    const int r = e >> 4, c = e & 15;
    qs[e] = (c < ncol && r == c0 + c) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int last = ((n - 1) / nb) * nb;
  for (int j0 = last; j0 >= 0; j0 -= nb) {
    if (j0 > c0 + ncol - 1) continue;   // uniform
    const int nbw = min(nb, n - j0), h = n - j0;
    apply_wy_slab(VTall + (size_t)j0 * n, Vall + (size_t)j0 * n, nbw, qs + (size_t)j0 * 16, 16, h, ncol, nbw, 0,
                  zp, Zs);
    __syncthreads();
  }
  for (int e = tid; e < n * 16; e += 256) {
    const int r = e >> 4, c = e & 15;
    if (c < ncol) Q[(size_t)r * n + c0 + c] = qs[e];
  }
}

// k_accum_q with 16 waves per slab (blockDim 1024) and apply_wy_wide: the
// panels' applications stay sequential per slab, but each costs about two
// memory latencies instead of one per 6 k-steps and per 2 row tiles.
// Dynamic LDS: the slab (n x 16) and the per-wave partials (16 KT x 4 x 64).
constexpr int kAccumWaves = 16;
constexpr int kAccumWideMaxN = 960;   // the slab and the partials within the LDS of one workgroup
constexpr int kAccumPairMaxN = 728;   // likewise with 32-column blocks (KT = 2)
template <int KT>
__host__ __device__ inline size_t accum_q_lds(int n) {
  return sizeof(double) * (16 * (size_t)n + (size_t)kAccumWaves * KT * 4 * 64);
}

template <int KT>
__global__ __launch_bounds__(1024) void k_accum_q_wide(const double* Vall, const double* VTall, double* Q, int n,
                                                       int nb, size_t cs) {
  extern __shared__ double qs[];
  __shared__ double Zs[32][17];
  double* zp = qs + 16 * (size_t)n;
  {
    const size_t co = (size_t)blockIdx.y * cs;
    Vall += co; VTall += co; Q += co;
  }
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * 16, ncol = min(16, n - c0);
  for (int e = tid; e < n * 16; e += 1024) {
    const int r = e >> 4, c = e & 15;
    qs[e] = (c < ncol && r == c0 + c) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int last = ((n - 1) / nb) * nb;
  for (int j0 = last; j0 >= 0; j0 -= nb) {
    if (j0 > c0 + ncol - 1) continue;   // uniform
    const int nbw = min(nb, n - j0), h = n - j0;
    apply_wy_wide<kAccumWaves, KT, 16 / KT, 4 / KT>(VTall + (size_t)j0 * n, Vall + (size_t)j0 * n, nbw, qs + (size_t)j0 * 16, 16,
                                          h, ncol, nbw, zp, Zs);
    __syncthreads();
  }
  for (int e = tid; e < n * 16; e += 1024) {
    const int r = e >> 4, c = e & 15;
    if (c < ncol) Q[(size_t)r * n + c0 + c] = qs[e];
  }
}

// Two consecutive block reflectors of 16-column panels as one block of up to
// 32 columns, so that the backward accumulation of Q takes half the dependent
// steps.  With H_a = I - P_a S_a^T, H_b = I - P_b S_b^T (P = V T, S = V;
// panel b starts 16 rows below panel a):
//   H_a H_b = I - [P_a, P_b - P_a (S_a^T P_b)] [S_a, S_b]^T.
// Block k is written at column j0 = 32 k in the panels' own layout (height
// n - j0, leading dimension its width min(32, n - j0)); a lone last panel is
// copied.  Grid (ceil(n / 32), chains), 1024 threads: M = S_a^T P_b with
// every wave's loads issued in one round (rows up to 16 x 4 x kPairUZ), then
// the new columns P_b - P_a M by MFMA, 16 rows per tile.
constexpr int kPairWaves = 16, kPairUZ = 12;
__global__ __launch_bounds__(1024) void k_wy_pair(const double* Vall, const double* VTall, double* Sout, double* Pout,
                                                  int n, size_t cs) {
  __shared__ double Mz[kPairWaves][4][64];   // per-wave partials of M in the MFMA D layout
  __shared__ double Ms[16][17];
  {
    const size_t co = (size_t)blockIdx.y * cs;
    Vall += co; VTall += co; Sout += co; Pout += co;
  }
  const int j0 = 32 * blockIdx.x, ha = n - j0, wc = min(32, ha);
  const int nbwa = min(16, ha), nbwb = wc - nbwa, hb = ha - 16;
  const double* Va = Vall + (size_t)j0 * n;
  const double* Pa = VTall + (size_t)j0 * n;
  double* S = Sout + (size_t)j0 * n;
  double* P = Pout + (size_t)j0 * n;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (nbwb <= 0) {   // uniform: a lone panel keeps its layout (width nbwa)
    for (int e = tid; e < ha * nbwa; e += 1024) {
      S[e] = Va[e];
      P[e] = Pa[e];
    }
    return;
  }
  const double* Vb = Vall + (size_t)(j0 + 16) * n;
  const double* Pb = VTall + (size_t)(j0 + 16) * n;
  const int m16 = lane & 15, kk = lane >> 4, cb = min(m16, nbwb - 1);
  // M = S_a^T P_b over the rows of panel b (row r of b is row r + 16 of a)
  {
    const int kq = ((hb + 4 * kPairWaves - 1) / (4 * kPairWaves)) * 4;
    const int kb = w * kq, ke = min(hb, kb + kq);
    v4d z = {0.0, 0.0, 0.0, 0.0};
    for (int kc = kb; kc < ke; kc += 4 * kPairUZ) {   // uniform; one round while hb <= 16 * 4 * kPairUZ
      double a[kPairUZ], bv[kPairUZ];
#pragma unroll
      for (int u = 0; u < kPairUZ; ++u) {
        const int rc = min(kc + 4 * u + kk, hb - 1);
        a[u] = Va[(size_t)(rc + 16) * 16 + m16];
        bv[u] = Pb[(size_t)rc * nbwb + cb];
      }
#pragma unroll
      for (int u = 0; u < kPairUZ; ++u) {
        const bool rin = kc + 4 * u + kk < ke;
        z = mfma_f64_16x16x4(rin ? a[u] : 0.0, (rin && m16 < nbwb) ? bv[u] : 0.0, z);
      }
    }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) Mz[w][rr][lane] = z[rr];
  }
  // meanwhile-independent copies: S = [S_a, S_b shifted down 16 rows], P's first 16 columns
  for (int e = tid; e < ha * 16; e += 1024) {
    const int r = e >> 4, q = e & 15;
    S[(size_t)r * wc + q] = Va[e];
    P[(size_t)r * wc + q] = Pa[e];
    if (q < nbwb) S[(size_t)r * wc + 16 + q] = r >= 16 ? Vb[(size_t)(r - 16) * nbwb + q] : 0.0;
  }
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < kPairWaves; ++q) v += Mz[q][rr][lane];
      Ms[kk + 4 * rr][m16] = v;
    }
  }
  __syncthreads();
  // P's last columns: P_b (shifted) - P_a M, one 16-row tile per wave and step
  double mb[4];
#pragma unroll
  for (int k4 = 0; k4 < 4; ++k4) mb[k4] = -Ms[4 * k4 + kk][m16];
  const int nrt = (ha + 15) / 16;
  for (int t = w; t < nrt; t += kPairWaves) {   // uniform
    v4d acc;
    double pa[4];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int r = 16 * t + kk + 4 * rr, rb = min(max(r - 16, 0), hb - 1);
      const double v = Pb[(size_t)rb * nbwb + cb];
      acc[rr] = (r >= 16 && r < ha && m16 < nbwb) ? v : 0.0;
    }
    const int ra = min(16 * t + m16, ha - 1);
#pragma unroll
    for (int k4 = 0; k4 < 4; ++k4) pa[k4] = Pa[(size_t)ra * 16 + 4 * k4 + kk];
#pragma unroll
    for (int k4 = 0; k4 < 4; ++k4) acc = mfma_f64_16x16x4(pa[k4], mb[k4], acc);
    if (m16 < nbwb) {
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int r = 16 * t + kk + 4 * rr;
        if (r < ha) P[(size_t)r * wc + 16 + m16] = acc[rr];
      }
    }
  }
}

// One launch of apply_wy_slab per 16 columns of C (grid (slabs, chains)).
__global__ __launch_bounds__(256) void k_apply_wy(const double* P, const double* S, int ldps, double* C, int ldc,
                                                  int h, int ncol, int nbw, size_t cs_ps, size_t cs_c) {
  __shared__ double zp[4][2][4][64];   // per-wave partial Z tiles in the MFMA D layout
  __shared__ double Zs[32][17];        // Z: nbw x 16
  P += (size_t)blockIdx.y * cs_ps;
  S += (size_t)blockIdx.y * cs_ps;
  C += (size_t)blockIdx.y * cs_c;
  apply_wy_slab(P, S, ldps, C, ldc, h, ncol, nbw, blockIdx.x, zp, Zs);
}

// ---------------------------------------------------------- QR panel ----
// Householder QR of one panel (columns j0..j0+nbw-1, rows j0..n-1 of A, ld n)
// by one workgroup, with the compact-WY output V (h x nbw, ld nbw, unit lower
// trapezoidal), VT = V T (T upper triangular, forward column-wise, the dlarft
// convention) and the R entries on and above the diagonal in place (entries
// below it are left as they are: nothing reads them).  Householder convention
// of LAPACK's dlarfg: for x = (x0, x'), beta = -sign(x0) |x|,
// tau = (beta - x0)/beta, v = (1, x' / (x0 - beta)); tau = 0 when x' = 0.
//
// Layout: the panel comes in by coalesced loads through LDS (vsh, 64 MAXR
// rows of NBW+1, zero below row h); wave w owns the columns
// w*NBW/4 .. (w+1)*NBW/4 - 1 and lane l the rows l, l + 64, ... (MAXR of
// them), in registers.  The column loop runs over the owning wave and,
// unrolled, over its columns, so the owner addresses its column without
// selects; as NBW <= 32, only the first row group holds rows at or above the
// diagonal.  Per column c: the owner forms the reflector from its registers
// (norm and x0 in one two-value wave sum), keeps v in its registers and writes
// it to column c of vsh, where it stays as column c of V; one barrier; every
// wave takes the dot products of v_c with all its own columns in one
// multi-value wave sum and applies the reflector to the columns right of c
// (a zero multiplier for the others, so no branches), and the lanes that hold
// the sums for columns left of c (v_q below their diagonal) record v_q^T v_c
// in Y.  After the loop: the T recurrence
// T[t][i] = -tau_i sum_{k<i} T[t][k] Y[k][i] row by row (each lane one row,
// the two halves of the wave splitting k), and VT = V T by MFMA.
// Dynamic LDS of k_qr_panel: NBW rows above the panel (the previous panel's
// rows), the panel's rows, Y, T, tau and the diagonal of R.
template <int NBW>
__host__ __device__ inline size_t qr_panel_lds(int rows) {
  return (size_t)(rows + NBW) * (NBW + 1) + 2 * (size_t)NBW * (NBW + 1) + 2 * NBW;
}

// One step of the blocked QR in one launch.  Workgroup 0 factorises the panel
// j0 .. j0 + nbw - 1; when the previous panel's reflector block (Vp, VTp,
// rows j0 - NBW .. n-1, ld NBW) is given, it first applies that block to its
// own columns in LDS (rows j0 - NBW onward) and writes the previous panel's
// rows of them (entries of R) back.  The other workgroups apply the same
// previous block to the columns right of this panel (At: rows j0 - NBW ..,
// columns j0 + nbw .., ntr of them, 16 per workgroup), which this panel does
// not touch, so the two roles never wait for each other.
template <int NBW, int MAXR>
__global__ __launch_bounds__(256) void k_qr_panel(double* A, int n, int j0, int nbw, double* Vout,
                                                  double* VTout, const double* Vp, const double* VTp, double* At,
                                                  int ntr, size_t cs) {
  extern __shared__ double smem[];
  __shared__ double zp[4][2][4][64];   // apply_wy_slab scratch (either role)
  __shared__ double Zs[32][17];
  constexpr int CPW = NBW / 4, PV = NBW + 1, PY = NBW + 1, NE = MAXR * NBW / 4, HR = 64 * MAXR;
  static_assert(NBW <= 32, "rows at or above the diagonal must sit in the first row group");
  {
    const size_t co = (size_t)blockIdx.y * cs;
    A += co; Vout += co; VTout += co;
    if (Vp) { Vp += co; VTp += co; At += co; }
  }
  const int h = n - j0, tid = threadIdx.x, lane = tid & 63;
  if (blockIdx.x > 0) {   // trailing columns: the previous panel's block reflector
    if constexpr (NBW > 16) {
      apply_wy_slab(Vp, VTp, NBW, At, n, h + NBW, ntr, NBW, blockIdx.x - 1, zp, Zs);
    } else {
      const int c0 = 16 * ((int)blockIdx.x - 1);
      apply_wy_wide<4, (NBW + 15) / 16, 12 / ((NBW + 15) / 16), 3>(Vp, VTp, NBW, At + c0, n, h + NBW, ntr - c0, NBW,
                                                                  &zp[0][0][0][0], Zs);
    }
    return;
  }
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  double* top = smem;                       // NBW x PV: rows j0 - NBW .. j0 - 1 of the panel's columns
  double* vsh = top + NBW * PV;             // HR x PV: the panel, then V
  double* Ym = vsh + HR * PV;               // NBW x PY: strictly upper V^T V
  double* Tm = Ym + NBW * PY;               // NBW x PY: T
  double* tau = Tm + NBW * PY;              // NBW
  double* bet = tau + NBW;                  // NBW: diagonal of R
  {
    double t[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = tid + 256 * u, r = e / NBW, q = e % NBW;
      t[u] = (r < h && q < nbw) ? A[(size_t)(j0 + r) * n + j0 + q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = tid + 256 * u, r = e / NBW, q = e % NBW;
      vsh[r * PV + q] = t[u];
    }
  }
  if (Vp) {
    // the previous panel's rows of these columns, then that panel's block
    // reflector on [top; vsh] (h + NBW rows) in LDS, NBW / 16 slabs
    for (int e = tid; e < NBW * NBW; e += 256) {
      const int r = e / NBW, q = e % NBW;
      top[r * PV + q] = (q < nbw) ? A[(size_t)(j0 - NBW + r) * n + j0 + q] : 0.0;
    }
    __syncthreads();
    if constexpr (NBW > 16) {
      for (int bx = 0; bx * 16 < NBW; ++bx) apply_wy_slab(Vp, VTp, NBW, top, PV, h + NBW, nbw, NBW, bx, zp, Zs);
    } else {
      for (int c0 = 0; c0 < nbw; c0 += 16)   // uniform
        apply_wy_wide<4, (NBW + 15) / 16, 12 / ((NBW + 15) / 16), 3>(Vp, VTp, NBW, top + c0, PV, h + NBW, nbw - c0,
                                                                    NBW, &zp[0][0][0][0], Zs);
    }
    __syncthreads();
    for (int e = tid; e < NBW * NBW; e += 256) {
      const int r = e / NBW, q = e % NBW;
      if (q < nbw) A[(size_t)(j0 - NBW + r) * n + j0 + q] = top[r * PV + q];
    }
  }
  for (int e = tid; e < NBW * PY; e += 256) Ym[e] = 0.0;
  if (tid < NBW) { tau[tid] = 0.0; bet[tid] = 0.0; }   // columns >= nbw stay inert
  __syncthreads();
  double a[MAXR][CPW];
#pragma unroll
  for (int i = 0; i < MAXR; ++i)
#pragma unroll
    for (int j = 0; j < CPW; ++j) a[i][j] = vsh[(lane + 64 * i) * PV + w * CPW + j];
  const int ncol = min(nbw, h);
  for (int cw = 0; cw < 4; ++cw) {
#pragma unroll
    for (int cj = 0; cj < CPW; ++cj) {
      const int c = cw * CPW + cj;
      if (c >= ncol) break;
      double vr[MAXR], tc;   // the owner keeps v and tau in registers
      if (w == cw) {
        // sum of squares below c, x0 (rows at or above c are in group 0)
        double sx[2] = {0.0, (lane == c) ? a[0][cj] : 0.0};
        sx[0] = (lane > c) ? a[0][cj] * a[0][cj] : 0.0;
#pragma unroll
        for (int i = 1; i < MAXR; ++i) sx[0] = fma(a[i][cj], a[i][cj], sx[0]);
        wave_sums<2>(sx);
        const double s = sx[0], x0 = sx[1];
        double beta, scal;
        if (s == 0.0) { tc = 0.0; beta = x0; scal = 0.0; }
        else {
          const double nrm = sqrt(x0 * x0 + s);
          beta = (x0 >= 0.0) ? -nrm : nrm;
          tc = (beta - x0) / beta;
          scal = 1.0 / (x0 - beta);
        }
        {
          const double x = a[0][cj];
          vr[0] = (lane > c) ? x * scal : (lane == c ? 1.0 : 0.0);
          a[0][cj] = (lane > c) ? vr[0] : (lane == c ? beta : x);
        }
#pragma unroll
        for (int i = 1; i < MAXR; ++i) {
          vr[i] = a[i][cj] * scal;
          a[i][cj] = vr[i];
        }
#pragma unroll
        for (int i = 0; i < MAXR; ++i) vsh[(lane + 64 * i) * PV + c] = vr[i];
        if (lane == 0) { tau[c] = tc; bet[c] = beta; }
      }
      __syncthreads();
      if (w != cw) {
        tc = tau[c];
#pragma unroll
        for (int i = 0; i < MAXR; ++i) vr[i] = vsh[(lane + 64 * i) * PV + c];
      }
      double p[CPW];
#pragma unroll
      for (int j = 0; j < CPW; ++j) {
        p[j] = 0.0;
#pragma unroll
        for (int i = 0; i < MAXR; ++i) p[j] = fma(vr[i], a[i][j], p[j]);
      }
      const double tl = wave_sums<CPW>(p);
      {
        // one holder lane per sum: v_q^T v_c for the columns left of c
        const int q = w * CPW + wave_sums_index<CPW>(lane);
        if (wave_sums_holder<CPW>(lane) && q < c) Ym[q * PY + c] = tl;
      }
      double tv[MAXR];
#pragma unroll
      for (int i = 0; i < MAXR; ++i) tv[i] = tc * vr[i];
#pragma unroll
      for (int j = 0; j < CPW; ++j) {
        const int q = w * CPW + j;
        const double pj = (q > c && q < nbw) ? p[j] : 0.0;   // uniform
#pragma unroll
        for (int i = 0; i < MAXR; ++i) a[i][j] = fma(-tv[i], pj, a[i][j]);
      }
    }
  }
  // R on and above the diagonal (rows < nbw <= 32 live in the first row group)
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int q = w * CPW + j;
    if (q < nbw && lane <= q) A[(size_t)(j0 + lane) * n + j0 + q] = a[0][j];
  }
  __syncthreads();
  // T rows: lane (t, half) holds T[t][2 m + half] in ts[m]
  if (w == 0) {
    const int t = lane & 31, half = lane >> 5;
    double ts[NBW / 2];
#pragma unroll
    for (int m = 0; m < NBW / 2; ++m) ts[m] = 0.0;
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < (i + 1) / 2; ++m) acc = fma(ts[m], Ym[(2 * m + half) * PY + i], acc);
      const double tot = add_xor32(acc);
      const double ti = tau[i];
      const double val = (i > t) ? -ti * tot : (i == t ? ti : 0.0);
      if (half == (i & 1)) ts[i / 2] = val;
    }
    if (t < NBW) {
#pragma unroll
      for (int m = 0; m < NBW / 2; ++m) Tm[t * PY + 2 * m + half] = ts[m];
    }
  } else {
    // V to global, coalesced, by the other three waves
    const int t3 = tid - 64;
#pragma unroll
    for (int u = 0; u < (NE * 4 + 2) / 3; ++u) {
      const int e = t3 + 192 * u, r = e / NBW, q = e % NBW;
      if (r < h && q < nbw) Vout[(size_t)r * nbw + q] = vsh[r * PV + q];
    }
  }
  __syncthreads();
  // VT = V T (h x nbw): wave w takes the 16-row tiles w, w + 4, ...; the T
  // operands of all column tiles stay in registers
  constexpr int NT = (NBW + 15) / 16, KS = NBW / 4;
  const int m16 = lane & 15, kk = lane >> 4;
  double tb[KS][NT];
#pragma unroll
  for (int k = 0; k < KS; ++k)
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) {
      const int col = tc * 16 + m16;
      tb[k][tc] = (col < NBW) ? Tm[(4 * k + kk) * PY + col] : 0.0;
    }
  const int nrt = (h + 15) >> 4;
  for (int tr = w; tr < nrt; tr += 4) {
    const int row = tr * 16 + m16;
    double av[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) av[k] = vsh[row * PV + 4 * k + kk];
    v4d acc[NT];
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) acc[tc] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < KS; ++k)
#pragma unroll
      for (int tc = 0; tc < NT; ++tc) acc[tc] = mfma_f64_16x16x4(av[k], tb[k][tc], acc[tc]);
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) {
      const int col = tc * 16 + m16;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int orow = tr * 16 + kk + 4 * rr;
        if (orow < h && col < nbw) VTout[(size_t)orow * nbw + col] = acc[tc][rr];
      }
    }
  }
}

// Rt[i][piv[j]] = R[i][j] / |R[i][i]| for j >= i; D[i] = |R[i][i]|
__global__ void k_build_rt(const double* R, const int* piv, int n, double* Rt, double* D, int* err, size_t cs) {
  {
    const size_t co = (size_t)blockIdx.y * cs;
    R += co; Rt += co; D += co;
    piv = reinterpret_cast<const int*>(reinterpret_cast<const double*>(piv) + co);
    err = reinterpret_cast<int*>(reinterpret_cast<double*>(err) + co);
  }
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  const double d = fabs(R[(size_t)i * n + i]);
  if (j == 0) {
    D[i] = d;
    if (!(d > 1e-300)) atomicOr(err, 2);
  }
  Rt[(size_t)i * n + piv[j]] = (j >= i) ? R[(size_t)i * n + j] / d : 0.0;
}

// ------------------------------------------------- blocked LU solve ----
// X Y = R for the bounded merge matrix X (n x n) and nrhs right-hand sides,
// stored side by side as XA = [X | R] (n x (n + nrhs), leading dimension ld),
// by LU with partial pivoting with the forward substitution carried along as
// extra columns.  For each panel of nb columns j0..j0+nbw-1 (pivot: the
// largest |a| among rows j0..n-1, ties to the lowest position):
//   the panel factorisation (lu_panel_factor) gives L11 U11 (diagonal block
//                  of XA), the multipliers L21 (rows below, into M) and the
//                  list of the composed row interchanges;
//   the panel's step on every later column (lu_prev_slab) applies the
//                  interchanges, replaces the panel rows by
//                  U12 = L11^-1 (P XA)[panel rows] and takes L21 U12 from the
//                  rows below.
// k_lu_step runs a panel's factorisation together with the previous panel's
// step (on the panel's own columns first, in the same workgroup, and on the
// other later columns in the launch's other workgroups), so each panel costs
// one launch.  Then R holds L^-1 P R, and the back substitution (below) runs
// block by block from the last.  sum log|U_ii| is log|det X|.  Columns left
// of a panel are never read again and are not updated.
constexpr int kLuMoves = 1 + 2 * 64;   // ints of the move list (count + pairs)

// z <- U^-1 z for a 32 x 32 upper triangular U given by columns in LDS
// (tt[k][r] = U[r][k]), backward and right-looking: z[k] is finished (times
// dinv[k], unless UNIT) and taken out of the rows above; column k - 1 is
// fetched while column k is applied, and scheduling fences bound the live
// registers.  A lower triangular solve runs through it with both index
// orders reversed (the forward form of this loop spills on gfx950).
template <bool UNIT>
__device__ __forceinline__ void tri_solve_back(double (&z)[32], const double (*tt)[34], const double* dinv) {
  double cur[32], nxt[32];
#pragma unroll
  for (int r = 0; r < 31; ++r) cur[r] = tt[31][r];
#pragma unroll
  for (int k = 31; k >= 0; --k) {
    if (k > 0) {
#pragma unroll
      for (int r = 0; r < k - 1; ++r) nxt[r] = tt[k - 1][r];
    }
    __builtin_amdgcn_sched_barrier(0);
    if (!UNIT) z[k] *= dinv[k];
#pragma unroll
    for (int r = 0; r < k; ++r) z[r] = fma(-cur[r], z[k], z[r]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < k - 1; ++r) cur[r] = nxt[r];
  }
}

// Panel factorisation (partial pivoting) of columns j0..j0+nbw-1, rows
// j0..n-1 of XA.  Layout: thread t holds the rows 256 i + t (i < MR) of the
// panel, all nbw columns, in registers, so column c of the unrolled column
// loop is a compile-time register index.  Pivoting is virtual: each held row
// carries its current position, a pivot step swaps two positions (every
// thread applies the same swap), and the rows are written to their final
// places at the end.  Per column c:
//   - each thread forms a key for its candidate rows (position >= c): the bits
//     of |a| (non-negative, so ordered like the value) with the low 11
//     mantissa bits replaced by 2047 - position, so one maximum gives the
//     largest value and, among values equal in the upper bits, the lowest
//     position (a NaN entry never wins, as in a comparison-based search);
//   - a wave maximum of the keys; the winning lane stores its key and its row
//     (columns >= c) in LDS, one slot per wave, two alternating buffers;
//   - one barrier; every thread reads the four keys, takes the largest, reads
//     that wave's row as the pivot row, swaps the positions, and eliminates
//     the rows that end below the pivot.
// The move list (moves[0] = count K <= 2 nbw, then K pairs (destination,
// source), absolute rows, in any order) is written for the next step.
template <int NBW, int MR>
struct LuShared {
  double key[2][4];
  int reg[2][4];
  __attribute__((aligned(16))) double row[2][4][MR][NBW];
};

// Column C of the panel (a template parameter, so every register index is a
// compile-time constant whatever the unroller decides).
template <int NBW, int MR, int C>
__device__ __forceinline__ void lu_column(double (&a)[MR][NBW], int (&pos)[MR], int h, int ncol, LuShared<NBW, MR>& sh,
                                          int* err) {
  if (C >= ncol) return;   // uniform
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int buf = C & 1;
  // candidate key of this thread (0 when it holds no row at or below C)
  double best = 0.0;
  int bi = 0;
#pragma unroll
  for (int i = 0; i < MR; ++i) {
    const bool cand = pos[i] >= C && pos[i] < h;
    const unsigned long long bits =
        ((unsigned long long)__double_as_longlong(fabs(a[i][C])) & ~0x7ffull) | (unsigned long long)(0x7ff - pos[i]);
    const double key = cand ? __longlong_as_double((long long)bits) : 0.0;
    if (key > best) { best = key; bi = i; }
  }
  const double wmax = wave_max_all(best);
  const unsigned long long win = __ballot(best == wmax);
  const int wl = __ffsll((long long)win) - 1;
  if (lane == wl) {
    // all rows of the winning lane (no register selection), and which one won
    sh.key[buf][w] = wmax;
    sh.reg[buf][w] = bi;
#pragma unroll
    for (int i = 0; i < MR; ++i)
#pragma unroll
      for (int q = C; q < NBW; ++q) sh.row[buf][w][i][q] = a[i][q];
  }
  __syncthreads();
  const double k0 = sh.key[buf][0], k1 = sh.key[buf][1], k2 = sh.key[buf][2], k3 = sh.key[buf][3];
  const int w01 = (k1 > k0) ? 1 : 0, w23 = (k3 > k2) ? 3 : 2;
  const double m01 = fmax(k0, k1), m23 = fmax(k2, k3);
  const int ww = __builtin_amdgcn_readfirstlane((m23 > m01) ? w23 : w01);
  const int wr = __builtin_amdgcn_readfirstlane(sh.reg[buf][ww]);
  const double gk = fmax(m01, m23);
  int pp = 0x7ff - (int)((unsigned long long)__double_as_longlong(gk) & 0x7ffull);
  // no finite candidate (a NaN column): keep the row and flag the failure
  if (!(gk > 0.0) || pp < C || pp >= h) {
    pp = C;
    if (tid == 0) atomicOr(err, 4);
  }
  double u[NBW];
#pragma unroll
  for (int q = C; q < NBW; ++q) u[q] = sh.row[buf][ww][wr][q];
  if (tid == 0 && !(fabs(u[C]) > 0.0)) atomicOr(err, 4);
  const double inv = 1.0 / u[C];
#pragma unroll
  for (int i = 0; i < MR; ++i) {
    pos[i] = (pos[i] == pp) ? C : (pos[i] == C ? pp : pos[i]);
    const bool below = pos[i] > C && pos[i] < h;
    const double l = below ? a[i][C] * inv : 0.0;
    a[i][C] = below ? l : a[i][C];
#pragma unroll
    for (int q = C + 1; q < NBW; ++q) a[i][q] = fma(-l, u[q], a[i][q]);
  }
}

template <int NBW, int MR, int... C>
__device__ __forceinline__ void lu_columns(std::integer_sequence<int, C...>, double (&a)[MR][NBW], int (&pos)[MR],
                                           int h, int ncol, LuShared<NBW, MR>& sh, int* err) {
  (lu_column<NBW, MR, C>(a, pos, h, ncol, sh, err), ...);
}

// The factorisation of a staged panel (rows j0 .. n-1 of its columns in
// stage, row stride NBW + 1), as described above; every thread calls it.
template <int NBW, int MR>
__device__ __forceinline__ void lu_panel_factor(double* XA, int n, int ld, int j0, int nbw, double* M, int ldm,
                                                int* moves, int* err, LuShared<NBW, MR>& sh, int& cnt_s,
                                                double* stage) {
  const int h = n - j0, tid = threadIdx.x;
  constexpr int PS = NBW + 1, NL = MR * NBW;
  double a[MR][NBW];
  int pos[MR];
#pragma unroll
  for (int i = 0; i < MR; ++i) {
    const int r = 256 * i + tid;
    pos[i] = (r < h) ? r : 0x7fffffff;
#pragma unroll
    for (int q = 0; q < NBW; ++q) a[i][q] = (r < h) ? stage[r * PS + q] : 0.0;
  }
  if (tid == 0) cnt_s = 0;
  lu_columns<NBW, MR>(std::make_integer_sequence<int, NBW>{}, a, pos, h, min(nbw, h), sh, err);
  // every row to its final place in the stage (the stage rows were last read
  // before the first column's barrier), and the moved rows into the list
#pragma unroll
  for (int i = 0; i < MR; ++i) {
    const int r = 256 * i + tid;
    if (pos[i] < h) {
#pragma unroll
      for (int q = 0; q < NBW; ++q) stage[pos[i] * PS + q] = a[i][q];
      if (pos[i] != r) {
        const int at = atomicAdd(&cnt_s, 1);
        moves[1 + 2 * at] = j0 + pos[i];
        moves[2 + 2 * at] = j0 + r;
      }
    }
  }
  __syncthreads();
  // diagonal block (L11 below, U11 on and above the diagonal) into XA,
  // multipliers of the rows below into M, coalesced
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int e = 256 * u + tid, r = e / NBW, q = e % NBW;
    if (r < h && q < nbw) {
      const double v = stage[r * PS + q];
      if (r < nbw) XA[(size_t)(j0 + r) * ld + j0 + q] = v;
      else M[(size_t)(j0 + r) * ldm + q] = v;
    }
  }
  __syncthreads();
  if (tid == 0) moves[0] = cnt_s;
}


// ---- one launch per LU step ----
// The previous panel's work on a 16-column slab of columns c0 .. c0+15 (only
// those < ncols): its row interchanges, U12 = L11^-1 (P XA)[its rows, slab]
// written to its rows, and the rows below it (from jb = j0p + nbp on) minus
// L21 U12, with the multipliers L21 at Mp (absolute rows, ld 32) and the
// interchanges as lu_panel_factor lists them (movesp).  The updated rows below go
// back to XA, or, for the panel of this launch, to its LDS stage (row r at
// stage + (r - jb) PS, column c - c0 + scol; zero past ncols).  Every thread
// of the workgroup calls it.  NBWP: the panel width of the launch (it sets how
// many row tiles a wave loads at once).
struct LuPrevShared {
  __attribute__((aligned(16))) double lr[32][34];   // lr[k][r] = L11[31 - r][31 - k]
  double u12[32][17];                                // U12 of the slab
  double mv[32][17];                                 // new values of the rows moved out of the panel
  int srcrow[32], od[32], os[32], nout;
};

template <bool TO_STAGE, int NBWP>
__device__ __forceinline__ void lu_prev_slab(double* XA, int n, int ld, int j0p, int nbp, int c0, int ncols,
                                             const double* Mp, const int* movesp, LuPrevShared& sh, short* odmap,
                                             double* stage, int PS, int scol, int scols) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m16 = lane & 15, kk = lane >> 4;
  const int jb = j0p + nbp, hb = n - jb;   // rows below the previous panel
  for (int e = tid; e < 32 * 32; e += 256) {
    const int r = e >> 5, k = e & 31;
    sh.lr[31 - k][31 - r] = (k < r && r < nbp) ? XA[(size_t)(j0p + r) * ld + j0p + k] : (r == k ? 1.0 : 0.0);
  }
  for (int e = tid; e < hb; e += 256) odmap[e] = -1;
  if (tid < 64) {
    const int K = min(movesp[0], 64);
    int dest = -1, src = -1;
    if (tid < K) { dest = movesp[1 + 2 * tid]; src = movesp[2 + 2 * tid]; }
    if (tid < 32) sh.srcrow[tid] = j0p + min(tid, nbp - 1);   // rows past nbp: any valid row
    __builtin_amdgcn_wave_barrier();   // the defaults land before the moves overwrite them
    const bool inpanel = tid < K && dest < jb;
    if (inpanel) sh.srcrow[dest - j0p] = src;
    const bool outside = tid < K && !inpanel;
    const unsigned long long m = __ballot(outside);
    const int at = __popcll(m & ((1ull << tid) - 1ull));
    if (outside && at < 32) { sh.od[at] = dest; sh.os[at] = src; }
    if (tid == 0) sh.nout = min(__popcll(m), 32);
  }
  __syncthreads();
  if (tid < sh.nout) odmap[sh.od[tid] - jb] = (short)tid;
  // the rows moved out of the panel, every thread one entry (all in flight)
  for (int e = tid; e < sh.nout * 16; e += 256) {
    const int i = e >> 4, q = e & 15;
    sh.mv[i][q] = XA[(size_t)sh.os[i] * ld + min(c0 + q, ncols - 1)];
  }
  if (tid < 16) {
    // the slab's panel rows (reversed: x[31 - k] is row j0p + k), solved with L11
    const int col = c0 + tid, colc = min(col, ncols - 1);
    double x[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) x[31 - k] = XA[(size_t)sh.srcrow[k] * ld + colc];
#pragma unroll
    for (int k = 0; k < 32; ++k) x[31 - k] = (k < nbp) ? x[31 - k] : 0.0;
    tri_solve_back<true>(x, sh.lr, nullptr);
#pragma unroll
    for (int k = 0; k < 32; ++k) sh.u12[31 - k][tid] = x[k];
  }
  __syncthreads();
  // rows below: A22 - L21 U12, 16-row tiles over the waves, K = nbp
  const int col = c0 + m16, colc = min(col, ncols - 1);
  const bool cin = col < ncols;
  double ub[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) ub[q] = (4 * q + kk < nbp) ? sh.u12[4 * q + kk][m16] : 0.0;
  // UT row tiles of a wave per round, all their loads issued together: four
  // for the tall 16-wide panels of large N, where one workgroup's latency
  // sets the pace; one for 32-wide panels (batches of small lattices), where
  // the registers of four cost more occupancy than they save
  constexpr int UT = NBWP == 16 ? 4 : 1;
  const int nrt = (hb + 15) / 16;
  for (int t0 = w; t0 < nrt; t0 += 4 * UT) {
    v4d acc[UT];
    double av[UT][8];
#pragma unroll
    for (int u = 0; u < UT; ++u) {
      const int r0 = jb + 16 * (t0 + 4 * u);
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int rowc = min(r0 + kk + 4 * rr, n - 1);
        acc[u][rr] = XA[(size_t)rowc * ld + colc];
      }
      const double* Mrow = Mp + (size_t)min(r0 + m16, n - 1) * 32;
#pragma unroll
      for (int q = 0; q < 8; ++q) av[u][q] = (4 * q < nbp) ? Mrow[4 * q + kk] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UT; ++u) {
      const int r0 = jb + 16 * (t0 + 4 * u);
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int rowc = min(r0 + kk + 4 * rr, n - 1);
        const int mi = odmap[rowc - jb];
        acc[u][rr] = (mi >= 0) ? sh.mv[mi][m16] : acc[u][rr];
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (4 * q >= nbp) break;   // uniform
#pragma unroll
      for (int u = 0; u < UT; ++u) acc[u] = mfma_f64_16x16x4((4 * q + kk < nbp) ? -av[u][q] : 0.0, ub[q], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < UT; ++u) {
      if (t0 + 4 * u >= nrt) break;   // uniform
      const int r0 = jb + 16 * (t0 + 4 * u);
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int row = r0 + kk + 4 * rr;
        if (row >= n) continue;
        if (TO_STAGE) {
          if (scol + m16 < scols) stage[(row - jb) * PS + scol + m16] = cin ? acc[u][rr] : 0.0;
        }
        else if (cin) XA[(size_t)row * ld + col] = acc[u][rr];
      }
    }
  }
  // U12 over the previous panel's rows
  for (int e = tid; e < 32 * 16; e += 256) {
    const int k = e >> 4, q = e & 15;
    if (k < nbp && c0 + q < ncols) XA[(size_t)(j0p + k) * ld + c0 + q] = sh.u12[k][q];
  }
  __syncthreads();
}

// One step of the blocked LU solve in one launch.  With has_panel, workgroup
// 0 factorises the panel j0 .. j0 + nbw - 1 (lu_panel_factor); when
// a previous panel exists (j0p, width nbp, its multipliers Mp and moves
// movesp), that workgroup first applies the previous panel's step to its own
// columns (lu_prev_slab into the stage), and the launch's other workgroups
// apply it to the columns from tstart to ncols - 1, 16 per workgroup.  The
// panel writes its multipliers to M and its moves to moves (the other buffer
// of the pair the next launch reads).  Without has_panel (after the last
// panel) every workgroup is a trailing one.
template <int NBW, int MR>
__global__ __launch_bounds__(256) void k_lu_step(double* XA, int n, int ld, int j0, int nbw, double* M, int* moves,
                                                 int has_panel, int j0p, int nbp, const double* Mp,
                                                 const int* movesp, int tstart, int ncols, int* err, size_t cs) {
  __shared__ LuShared<NBW, MR> sh;
  __shared__ LuPrevShared ps;
  __shared__ short odmap[1024];
  __shared__ int cnt_s;
  extern __shared__ double stage[];   // h rows of NBW + 1: the panel in, then the factors out
  {
    const size_t co = (size_t)blockIdx.y * cs;
    XA += co; M += co;
    moves = reinterpret_cast<int*>(reinterpret_cast<double*>(moves) + co);
    err = reinterpret_cast<int*>(reinterpret_cast<double*>(err) + co);
    if (Mp) {
      Mp += co;
      movesp = reinterpret_cast<const int*>(reinterpret_cast<const double*>(movesp) + co);
    }
  }
  const int tslab = (int)blockIdx.x - (has_panel ? 1 : 0);
  if (tslab >= 0) {   // trailing columns: the previous panel's step
    lu_prev_slab<false, NBW>(XA, n, ld, j0p, nbp, tstart + 16 * tslab, ncols, Mp, movesp, ps, odmap, nullptr, 0, 0,
                             0);
    return;
  }
  const int h = n - j0, tid = threadIdx.x;
  constexpr int PS = NBW + 1, NL = MR * NBW;   // stage row stride; loads per thread
  if (Mp) {
    // the previous panel's step on this panel's columns, straight into the stage
    for (int c0 = 0; c0 < NBW; c0 += 16)
      lu_prev_slab<true, NBW>(XA, n, ld, j0p, nbp, j0 + c0, j0 + nbw, Mp, movesp, ps, odmap, stage, PS, c0, NBW);
  } else {
    // the panel through LDS: coalesced loads (consecutive threads along a row),
    // all issued before the stores, zeros outside the panel
    double t[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int e = 256 * u + tid, r = e / NBW, q = e % NBW;
      t[u] = XA[(size_t)(j0 + min(r, h - 1)) * ld + j0 + min(q, nbw - 1)];
    }
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int e = 256 * u + tid, r = e / NBW, q = e % NBW;
      if (r < h) stage[r * PS + q] = (q < nbw) ? t[u] : 0.0;
    }
    __syncthreads();
  }
  lu_panel_factor<NBW, MR>(XA, n, ld, j0, nbw, M, 32, moves, err, sh, cnt_s, stage);
}

// Back substitution of all right-hand sides in two launches, instead of one
// diagonal solve and one product per block row:
//   k_lu_diag_inv  inverts every diagonal block U_bb of U (grid (blocks,
//                  chains), one workgroup each, the 32 columns of the inverse
//                  by the backward triangular solve on unit vectors); block
//                  b is stored as a 32 x 32 row-major matrix at Uinv + 1024 b,
//                  the identity beyond a ragged last block;
//   k_lu_back      gives every workgroup 16 right-hand-side columns and runs
//                  the whole backward block recursion on them, bottom block
//                  first: Y_b = U_bb^-1 R_b (one 32 x 32 x 16 MFMA product,
//                  written in place of R_b), then R[rows above] -= U[rows
//                  above, b] Y_b (16-row MFMA tiles over the four waves).  The
//                  column slabs are independent, so no workgroup waits for
//                  another.
constexpr int kBackCols = 16;

__global__ __launch_bounds__(256) void k_lu_diag_inv(const double* XA, int n, int ld, int nb, double* Uinv,
                                                     size_t cs) {
  __shared__ __attribute__((aligned(16))) double tt[32][34];   // tt[k][r] = U[r][k]
  __shared__ double dinv[32];
  XA += (size_t)blockIdx.y * cs;
  Uinv += (size_t)blockIdx.y * cs;
  const int r0 = blockIdx.x * nb, nrow = min(nb, n - r0);
  const double* U = XA + (size_t)r0 * ld + r0;
  for (int e = threadIdx.x; e < 32 * 32; e += 256) {
    const int r = e >> 5, k = e & 31;
    tt[k][r] = (r < nrow && k < nrow && k >= r) ? U[(size_t)r * ld + k] : (r == k ? 1.0 : 0.0);
  }
  __syncthreads();
  if (threadIdx.x < 32) dinv[threadIdx.x] = 1.0 / tt[threadIdx.x][threadIdx.x];
  __syncthreads();
  if (threadIdx.x >= 32) return;
  const int col = threadIdx.x;
  double z[32];
#pragma unroll
  for (int r = 0; r < 32; ++r) z[r] = (r == col) ? 1.0 : 0.0;
  tri_solve_back<false>(z, tt, dinv);
  double* out = Uinv + (size_t)blockIdx.x * 1024;
#pragma unroll
  for (int r = 0; r < 32; ++r) out[r * 32 + col] = z[r];
}

__global__ __launch_bounds__(256) void k_lu_back(double* XA, int n, int ld, int nb, int nrhs, const double* Uinv,
                                                 size_t cs) {
  __shared__ double Rb[32][kBackCols + 1];   // R_b of this slab
  __shared__ double Yb[32][kBackCols + 1];   // Y_b = U_bb^-1 R_b
  XA += (size_t)blockIdx.y * cs;
  Uinv += (size_t)blockIdx.y * cs;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m16 = lane & 15, kk = lane >> 4;
  const int c0 = blockIdx.x * kBackCols;             // first right-hand side of the slab
  const int col = c0 + m16, colc = min(col, nrhs - 1);
  const bool cin = col < nrhs;
  double* R = XA + n;                                  // right-hand sides: R[r][j] at R[r * ld + j]
  const int nblk = (n + nb - 1) / nb;
  for (int b = nblk - 1; b >= 0; --b) {
    const int j0 = b * nb, nbw = min(nb, n - j0);
    for (int e = tid; e < 32 * kBackCols; e += 256) {
      const int r = e / kBackCols, q = e % kBackCols;
      const double v = R[(size_t)(j0 + min(r, nbw - 1)) * ld + min(c0 + q, nrhs - 1)];
      Rb[r][q] = (r < nbw && c0 + q < nrhs) ? v : 0.0;
    }
    __syncthreads();
    if (w < 2) {
      // rows w*16 .. w*16+15 of Y_b (K = 32; Uinv is the identity past nbw)
      const double* Ui = Uinv + (size_t)b * 1024;
      v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k0 = 0; k0 < 32; k0 += 4)
        acc = mfma_f64_16x16x4(Ui[(w * 16 + m16) * 32 + k0 + kk], Rb[k0 + kk][m16], acc);
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int row = w * 16 + kk + 4 * rr;
        Yb[row][m16] = acc[rr];
        if (row < nbw && cin) R[(size_t)(j0 + row) * ld + col] = acc[rr];
      }
    }
    __syncthreads();
    // R[0:j0, slab] -= U[0:j0, j0:j0+nbw] Y_b in 16-row tiles; with 8-column
    // panels the last tile may reach past j0, and those rows are left alone
    for (int t = w; t * 16 < j0; t += 4) {
      v4d acc;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) acc[rr] = R[(size_t)min(t * 16 + kk + 4 * rr, n - 1) * ld + colc];
      const int ra = t * 16 + m16;
      const double* Urow = XA + (size_t)min(ra, n - 1) * ld + j0;
#pragma unroll
      for (int k0 = 0; k0 < 32; k0 += 4) {
        if (k0 >= nbw) break;   // uniform
        const int k = k0 + kk;
        const double a = (k < nbw && ra < j0) ? -Urow[min(k, nbw - 1)] : 0.0;
        acc = mfma_f64_16x16x4(a, Yb[k][m16], acc);
      }
      if (cin) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int row = t * 16 + kk + 4 * rr;
          if (row < j0) R[(size_t)row * ld + col] = acc[rr];
        }
      }
    }
    __syncthreads();
  }
}

// k_lu_back for n <= kBackWideMaxN with eight waves and the slab of right-
// hand sides held in LDS (n x 16, rows of 17) from start to end: each block
// step issues its loads of U's columns above the block and of U_bb^-1 before
// Y_b is formed (they do not depend on it), so a step costs one global
// latency and two barriers.  The products and their order are those of
// k_lu_back.  Dynamic LDS: back_wide_lds(n).
constexpr int kBackWaves = 16, kBackWideMaxN = 768, kBackRS = kBackCols + 1;
__host__ __device__ inline size_t back_wide_lds(int n) { return sizeof(double) * (size_t)n * kBackRS; }

__global__ __launch_bounds__(64 * kBackWaves) void k_lu_back_wide(double* XA, int n, int ld, int nb, int nrhs,
                                                                  const double* Uinv, size_t cs) {
  extern __shared__ double Rs[];               // Rs[r * kBackRS + q] = R[r][c0 + q]
  __shared__ double Yb[32][kBackCols + 1];     // Y_b = U_bb^-1 R_b
  constexpr int UT = (kBackWideMaxN / 16 + kBackWaves - 1) / kBackWaves;   // row tiles above a block per wave
  XA += (size_t)blockIdx.y * cs;
  Uinv += (size_t)blockIdx.y * cs;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m16 = lane & 15, kk = lane >> 4;
  const int c0 = blockIdx.x * kBackCols, col = c0 + m16;
  const bool cin = col < nrhs;
  double* R = XA + n;
  for (int e = tid; e < n * kBackCols; e += 64 * kBackWaves) {
    const int r = e / kBackCols, q = e % kBackCols;
    Rs[r * kBackRS + q] = (c0 + q < nrhs) ? R[(size_t)r * ld + c0 + q] : 0.0;
  }
  __syncthreads();
  const int nblk = (n + nb - 1) / nb;
  for (int b = nblk - 1; b >= 0; --b) {
    const int j0 = b * nb, nbw = min(nb, n - j0);
    // loads that do not depend on Y_b: U[rows above, block] and U_bb^-1
    double ua[UT][8];
#pragma unroll
    for (int u = 0; u < UT; ++u) {
      const int ra = (w + kBackWaves * u) * 16 + m16;
      const double* Urow = XA + (size_t)min(ra, n - 1) * ld + j0;
#pragma unroll
      for (int q = 0; q < 8; ++q) ua[u][q] = Urow[min(4 * q + kk, nbw - 1)];
    }
    if (w < 2) {
      const double* Ui = Uinv + (size_t)b * 1024;
      double ui[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) ui[q] = Ui[(w * 16 + m16) * 32 + 4 * q + kk];
      v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = 4 * q + kk;
        acc = mfma_f64_16x16x4(ui[q], k < nbw ? Rs[(j0 + k) * kBackRS + m16] : 0.0, acc);
      }
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) Yb[w * 16 + kk + 4 * rr][m16] = acc[rr];
    }
    __syncthreads();
    // R[0:j0, slab] -= U[0:j0, block] Y_b in 16-row tiles (rows past j0 of
    // the last tile, with 8-column panels, are left alone); Y_b into its rows
#pragma unroll
    for (int u = 0; u < UT; ++u) {
      const int t = w + kBackWaves * u;
      if (t * 16 >= j0) break;   // uniform
      const int ra = t * 16 + m16;
      v4d acc;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) acc[rr] = Rs[min(t * 16 + kk + 4 * rr, n - 1) * kBackRS + m16];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (4 * q >= nbw) break;   // uniform
        const int k = 4 * q + kk;
        const double a = (k < nbw && ra < j0) ? -ua[u][q] : 0.0;
        acc = mfma_f64_16x16x4(a, Yb[k][m16], acc);
      }
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int row = t * 16 + kk + 4 * rr;
        if (row < j0) Rs[row * kBackRS + m16] = acc[rr];
      }
    }
    for (int e = tid; e < nbw * kBackCols; e += 64 * kBackWaves) {
      const int r = e / kBackCols, q = e % kBackCols;
      Rs[(j0 + r) * kBackRS + q] = Yb[r][q];
    }
    __syncthreads();
  }
  for (int e = tid; e < n * kBackCols; e += 64 * kBackWaves) {
    const int r = e / kBackCols, q = e % kBackCols;
    if (c0 + q < nrhs) R[(size_t)r * ld + c0 + q] = Rs[r * kBackRS + q];
  }
  (void)cin;
}

// out += sum_i log|U_ii| (one workgroup)
__global__ __launch_bounds__(256) void k_logabs_diag(const double* U, int n, int ld, double* out, size_t cs) {
  __shared__ double red[8];
  U += (size_t)blockIdx.y * cs;
  out += (size_t)blockIdx.y * cs;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += log(fabs(U[(size_t)i * ld + i]));
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) *out += s;
}

// out = sum_i log max(d_i, 1)
__global__ __launch_bounds__(256) void k_logbig_sum(const double* d, int n, double* out, int accumulate,
                                                    size_t cs_d, size_t cs_out) {
  __shared__ double red[8];
  d += (size_t)blockIdx.y * cs_d;
  out += (size_t)blockIdx.y * cs_out;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += log(fmax(d[i], 1.0));
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) *out = accumulate ? (*out + s) : s;
}
