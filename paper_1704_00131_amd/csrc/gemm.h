// FP64 MFMA GEMM with fused diagonal scalings, used for every dense product of
// the sweep: wraps, chunk products of the stabilisation, WY trailing updates,
// merges, rank-k Green's-function updates and the matrix exponential.
//
//   C = alpha * diag(rs) * op(A) * diag(ks) * op(B) * diag(cs) + beta * C + diag_add * I
//
// op(X) is X or X^T (row-major storage).  Each scale vector is optional and
// may be evaluated from its source with one of the SC_* modes (for example
// exp(coupling * field) for the interaction exponential), so no separate
// scaling pass over HBM is needed.
//
// Tiling: one workgroup of WV waves (4, or 8 for long K on one chain)
// computes a TILE x TILE tile of C (TILE = 16 or 32, chosen per launch so that
// small products still spread over many CUs); the waves split K and their
// partial accumulators are summed through LDS.  Operands are read straight from
// global memory in the v_mfma_f64_16x16x4 lane layout: the 16 lanes feeding
// one MFMA row share a 128-byte line across four k-steps, so the L1 serves
// most loads and no LDS staging is needed for these L2-resident matrices.
#pragma once
#include "device_common.h"

struct GemmArgs {
  int M, N, K;
  const double* A; int lda; int transA;
  const double* B; int ldb; int transB;
  double* C; int ldc;
  double alpha, beta, diag_add;
  const double* rs; double rs_coef; int rs_mode;
  const double* cs; double cs_coef; int cs_mode;
  const double* ks; double ks_coef; int ks_mode;
  // batching: chain = blockIdx.y; operands flagged in `pc` are offset by
  // chain * cstride doubles (the others are shared by all chains)
  size_t cstride; int pc; int nch; int tile;
};
enum { PC_A = 1, PC_B = 2, PC_C = 4, PC_RS = 8, PC_CS = 16, PC_KS = 32 };

// TA, TB, KS: the transposes and whether the k scaling is present, fixed at
// compile time (0 or 1) or read from g (-1); the fixed forms keep the runtime
// selects out of the K loop (a 648^3 product: 24.8 against 25.9 us on 32 x 32
// tiles, 36.0 against 39.4 us on 16 x 16 tiles).  With KS = 1 each wave first
// evaluates the k scaling of its K range once into LDS (an exponential of the
// field for the downward wrap and the left chunk products), instead of every
// lane evaluating it at every step.
template <int TILE, int UNR, int WV, int TA = -1, int TB = -1, int KS = -1>
__device__ __forceinline__ void gemm_tile(GemmArgs g) {
  constexpr int NB = TILE / 16;
  const bool ta = TA < 0 ? g.transA != 0 : TA != 0;
  const bool tb = TB < 0 ? g.transB != 0 : TB != 0;
  const bool ksm = KS < 0 ? g.ks_mode != 0 : KS != 0;
  if (g.cstride) {
    const size_t co = (size_t)blockIdx.y * g.cstride;
    if (g.pc & PC_A) g.A += co;
    if (g.pc & PC_B) g.B += co;
    if (g.pc & PC_C) g.C += co;
    if (g.pc & PC_RS) g.rs += co;
    if (g.pc & PC_CS) g.cs += co;
    if (g.pc & PC_KS) g.ks += co;
  }
  __shared__ double red[WV - 1][NB * NB][4][64];
  const int tilesN = (g.N + TILE - 1) / TILE;
  const int i0 = (blockIdx.x / tilesN) * TILE, j0 = (blockIdx.x % tilesN) * TILE;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  // contiguous K range of this wave, a multiple of 4 long
  const int kq = ((g.K + 4 * WV - 1) / (4 * WV)) * 4;
  const int kb = w * kq, ke = min(g.K, kb + kq);
  const double* kst = nullptr;   // the k scaling of this wave's range, when staged
  if constexpr (KS == 1) {
    constexpr int KSMAX = 1024 / WV;
    __shared__ double ksh[WV][KSMAX];
    if (kq <= KSMAX) {   // uniform
      for (int e = lane; e < kq; e += 64)
        ksh[w][e] = (kb + e < ke) ? scale_of(g.ks_mode, g.ks, g.ks_coef, kb + e) : 1.0;
      kst = ksh[w];
    }
    __syncthreads();
  }
  v4d acc[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  // K in chunks of UNR steps of 4: all loads of a chunk are issued before its
  // MFMAs, so their latencies overlap (UNR = 1 keeps the register count low
  // for launches whose many workgroups already hide the latency)
  for (int kc = kb; kc < ke; kc += 4 * UNR) {
    double av[UNR][NB], bv[UNR][NB];
    // unconditional loads from clamped addresses, masked afterwards, so the
    // loads of the chunk issue back to back
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int k = kc + 4 * u + lk, kk = min(k, g.K - 1);
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        const int row = min(i0 + a * 16 + l16, g.M - 1);
        av[u][a] = ta ? g.A[(size_t)kk * g.lda + row] : g.A[(size_t)row * g.lda + kk];
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int col = min(j0 + b * 16 + l16, g.N - 1);
        bv[u][b] = tb ? g.B[(size_t)col * g.ldb + kk] : g.B[(size_t)kk * g.ldb + col];
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int k = kc + 4 * u + lk;
      const bool kin = k < ke;
      const double ksc =
          (kin && ksm) ? (kst ? kst[k - kb] : scale_of(g.ks_mode, g.ks, g.ks_coef, k)) : 1.0;
#pragma unroll
      for (int a = 0; a < NB; ++a) av[u][a] = (kin && i0 + a * 16 + l16 < g.M) ? av[u][a] * ksc : 0.0;
#pragma unroll
      for (int b = 0; b < NB; ++b) bv[u][b] = (kin && j0 + b * 16 + l16 < g.N) ? bv[u][b] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      if (kc + 4 * u >= ke) break;   // uniform: short K ranges skip the empty steps
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = mfma_f64_16x16x4(av[u][a], bv[u][b], acc[a][b]);
    }
  }
  if (w > 0) {
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[w - 1][a * NB + b][r][lane] = acc[a][b][r];
  }
  __syncthreads();
  if (w != 0) return;
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int col = j0 + b * 16 + l16;
      if (col >= g.N) continue;
      const double cf = g.cs_mode ? scale_of(g.cs_mode, g.cs, g.cs_coef, col) : 1.0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + a * 16 + lk + 4 * r;
        if (row >= g.M) continue;
        double sum = acc[a][b][r];
#pragma unroll
        for (int q = 0; q < WV - 1; ++q) sum += red[q][a * NB + b][r][lane];
        const double rf = g.rs_mode ? scale_of(g.rs_mode, g.rs, g.rs_coef, row) : 1.0;
        double v = g.alpha * (rf * sum * cf);
        double* cp = g.C + (size_t)row * g.ldc + col;
        if (g.beta != 0.0) v += g.beta * (*cp);
        if (row == col) v += g.diag_add;
        *cp = v;
      }
    }
}

template <int TILE, int UNR, int WV, int TA, int TB, int KS>
__global__ __launch_bounds__(64 * WV) void k_gemm(GemmArgs g) {
  gemm_tile<TILE, UNR, WV, TA, TB, KS>(g);
}

// k_gemm with the transposes and the k scaling of g fixed at compile time.
template <int TILE, int UNR, int WV>
static inline void launch_direct(const GemmArgs& g, dim3 grid, hipStream_t s) {
  const dim3 block(64 * WV);
  switch ((g.transA ? 1 : 0) | (g.transB ? 2 : 0) | (g.ks_mode ? 4 : 0)) {
    case 0: hipLaunchKernelGGL((k_gemm<TILE, UNR, WV, 0, 0, 0>), grid, block, 0, s, g); break;
    case 1: hipLaunchKernelGGL((k_gemm<TILE, UNR, WV, 1, 0, 0>), grid, block, 0, s, g); break;
    case 2: hipLaunchKernelGGL((k_gemm<TILE, UNR, WV, 0, 1, 0>), grid, block, 0, s, g); break;
    case 3: hipLaunchKernelGGL((k_gemm<TILE, UNR, WV, 1, 1, 0>), grid, block, 0, s, g); break;
    case 4: hipLaunchKernelGGL((k_gemm<TILE, UNR, WV, 0, 0, 1>), grid, block, 0, s, g); break;
    case 5: hipLaunchKernelGGL((k_gemm<TILE, UNR, WV, 1, 0, 1>), grid, block, 0, s, g); break;
    case 6: hipLaunchKernelGGL((k_gemm<TILE, UNR, WV, 0, 1, 1>), grid, block, 0, s, g); break;
    default: hipLaunchKernelGGL((k_gemm<TILE, UNR, WV, 1, 1, 1>), grid, block, 0, s, g); break;
  }
}

// Up to three independent products of the same M x N shape in one launch
// (blockIdx.z picks the product), so small products fill more of the chip.
struct GemmGroup { GemmArgs g[3]; };

template <int TILE, int UNR, int WV, int TA, int TB, int KS>
__global__ __launch_bounds__(64 * WV) void k_gemm_group(GemmGroup gg) {
  gemm_tile<TILE, UNR, WV, TA, TB, KS>(gg.g[blockIdx.z]);
}

// k_gemm_group with the transposes and the k scaling fixed at compile time
// when all products of the group agree on them, else read per product.
template <int TILE, int UNR, int WV>
static inline void launch_group_direct(const GemmGroup& gg, int count, dim3 grid, hipStream_t s) {
  const dim3 block(64 * WV);
  auto code_of = [](const GemmArgs& g) { return (g.transA ? 1 : 0) | (g.transB ? 2 : 0) | (g.ks_mode ? 4 : 0); };
  int code = code_of(gg.g[0]);
  for (int i = 1; i < count; ++i)
    if (code_of(gg.g[i]) != code) code = 8;
  switch (code) {
    case 0: hipLaunchKernelGGL((k_gemm_group<TILE, UNR, WV, 0, 0, 0>), grid, block, 0, s, gg); break;
    case 1: hipLaunchKernelGGL((k_gemm_group<TILE, UNR, WV, 1, 0, 0>), grid, block, 0, s, gg); break;
    case 2: hipLaunchKernelGGL((k_gemm_group<TILE, UNR, WV, 0, 1, 0>), grid, block, 0, s, gg); break;
    case 3: hipLaunchKernelGGL((k_gemm_group<TILE, UNR, WV, 1, 1, 0>), grid, block, 0, s, gg); break;
    case 4: hipLaunchKernelGGL((k_gemm_group<TILE, UNR, WV, 0, 0, 1>), grid, block, 0, s, gg); break;
    case 5: hipLaunchKernelGGL((k_gemm_group<TILE, UNR, WV, 1, 0, 1>), grid, block, 0, s, gg); break;
    case 6: hipLaunchKernelGGL((k_gemm_group<TILE, UNR, WV, 0, 1, 1>), grid, block, 0, s, gg); break;
    case 7: hipLaunchKernelGGL((k_gemm_group<TILE, UNR, WV, 1, 1, 1>), grid, block, 0, s, gg); break;
    default: hipLaunchKernelGGL((k_gemm_group<TILE, UNR, WV, -1, -1, -1>), grid, block, 0, s, gg); break;
  }
}

// Large products: a 64 x 64 tile per workgroup, K in steps of 32 staged
// through LDS with double buffering (the loads of step t+1 are in flight while
// the four waves run the MFMAs of step t).  Wave (wr, wc) owns the 32 x 32
// quarter (wr, wc) and computes it with v_mfma_f64_4x4x4f64, which on gfx950
// runs at twice the FP64 rate of the 16 x 16 x 4 form.  Its lane layout (4
// blocks b of 4 x 4, checked on gfx950 with an in-bounds probe):
//   A(m, k) of block b in lane m + 4b + 16k,  B(k, n) in lane n + 4b + 16k,
//   D(m, n) in lane n + 4b + 16m,
// so with the same A in all four blocks one instruction yields the 4 x 16
// strip D[m0 + l/16][n0 + l%16] from A[m0 + l%4][k + l/16] and
// B[k + l/16][n0 + l%16]: 8 x 2 strips per wave and 4-step of K.
// LDS layouts are chosen per transpose so that both the coalesced stores and
// the operand reads are free of (or at worst two-way) bank conflicts.
// Tiles are placed XCD-aware: workgroups are dealt round-robin to the eight
// XCDs, so consecutive logical tiles (sharing rows of A) go to workgroups on
// the same XCD and its L2 keeps those rows.  Same operand conventions,
// scalings and batching as k_gemm.  Dynamic LDS: gemm64_lds().
constexpr int kG64 = 64, kGBK = 32, kGXcd = 8;
// strides (doubles) and sizes of the four layouts
constexpr int kSA = kGBK + 4;    // A row-major [i][k]
constexpr int kSAt = kG64 + 8;   // A^T        [k][i]
constexpr int kSB = kG64 + 16;   // B row-major [k][j]
constexpr int kSBt = kGBK + 4;   // B^T        [j][k]
constexpr int kGAsz = (kG64 * kSA > kGBK * kSAt) ? kG64 * kSA : kGBK * kSAt;
constexpr int kGBsz = (kGBK * kSB > kG64 * kSBt) ? kGBK * kSB : kG64 * kSBt;
__host__ __device__ inline size_t gemm64_lds() { return sizeof(double) * 2 * (kGAsz + kGBsz); }
template <int TA, int TB>
__global__ void k_gemm64(GemmArgs g, int ntiles);

// Unconditional loads from clamped addresses (so all sixteen issue back to
// back), masked and scaled afterwards.
template <int TA, int TB>
__device__ __forceinline__ void gemm64_load(const GemmArgs& g, int m0, int n0, int k0, double (&ra)[8],
                                            double (&rb)[8]) {
  const int t = threadIdx.x;
  if (!TA) {          // A[row][k]: 32 k contiguous per row, 8 rows per pass
    const int k = k0 + (t & 31), kk = min(k, g.K - 1);
#pragma unroll
    for (int q = 0; q < 8; ++q) ra[q] = g.A[(size_t)min(m0 + (t >> 5) + 8 * q, g.M - 1) * g.lda + kk];
  } else {                  // element (row, k) at A[k][row]: 64 rows contiguous, 4 k per pass
    const int row = min(m0 + (t & 63), g.M - 1);
#pragma unroll
    for (int q = 0; q < 8; ++q) ra[q] = g.A[(size_t)min(k0 + (t >> 6) + 4 * q, g.K - 1) * g.lda + row];
  }
  if (!TB) {          // B[k][col]: 64 cols contiguous, 4 k per pass
    const int col = min(n0 + (t & 63), g.N - 1);
#pragma unroll
    for (int q = 0; q < 8; ++q) rb[q] = g.B[(size_t)min(k0 + (t >> 6) + 4 * q, g.K - 1) * g.ldb + col];
  } else {                  // element (k, col) at B[col][k]: 32 k contiguous, 8 cols per pass
    const int kk = min(k0 + (t & 31), g.K - 1);
#pragma unroll
    for (int q = 0; q < 8; ++q) rb[q] = g.B[(size_t)min(n0 + (t >> 5) + 8 * q, g.N - 1) * g.ldb + kk];
  }
}

// Zero outside the matrices and apply the k scaling (after the loads landed).
template <int TA, int TB>
__device__ __forceinline__ void gemm64_mask(const GemmArgs& g, int m0, int n0, int k0, double (&ra)[8],
                                            double (&rb)[8]) {
  const int t = threadIdx.x;
  if (!TA) {
    const int k = k0 + (t & 31);
    const double ksc = (g.ks_mode && k < g.K) ? scale_of(g.ks_mode, g.ks, g.ks_coef, k) : 1.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) ra[q] = (m0 + (t >> 5) + 8 * q < g.M && k < g.K) ? ra[q] * ksc : 0.0;
  } else {
    const bool rin = m0 + (t & 63) < g.M;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = k0 + (t >> 6) + 4 * q;
      const double ksc = (g.ks_mode && k < g.K) ? scale_of(g.ks_mode, g.ks, g.ks_coef, k) : 1.0;
      ra[q] = (rin && k < g.K) ? ra[q] * ksc : 0.0;
    }
  }
  if (!TB) {
    const bool cin = n0 + (t & 63) < g.N;
#pragma unroll
    for (int q = 0; q < 8; ++q) rb[q] = (cin && k0 + (t >> 6) + 4 * q < g.K) ? rb[q] : 0.0;
  } else {
    const bool kin = k0 + (t & 31) < g.K;
#pragma unroll
    for (int q = 0; q < 8; ++q) rb[q] = (kin && n0 + (t >> 5) + 8 * q < g.N) ? rb[q] : 0.0;
  }
}

template <int TA, int TB>
__device__ __forceinline__ void gemm64_store(double* As, double* Bs, const double (&ra)[8], const double (&rb)[8]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if (!TA) As[((t >> 5) + 8 * q) * kSA + (t & 31)] = ra[q];
    else As[((t >> 6) + 4 * q) * kSAt + (t & 63)] = ra[q];
    if (!TB) Bs[((t >> 6) + 4 * q) * kSB + (t & 63)] = rb[q];
    else Bs[((t >> 5) + 8 * q) * kSBt + (t & 31)] = rb[q];
  }
}

template <int TA, int TB>
__device__ __forceinline__ void gemm64_tile(GemmArgs g, int ntiles) {
  // physical workgroup -> logical tile: each XCD (physical id mod 8) gets a
  // contiguous range of tiles
  const int per = (ntiles + kGXcd - 1) / kGXcd;
  const int tile = (blockIdx.x % kGXcd) * per + blockIdx.x / kGXcd;
  if (tile >= ntiles) return;
  if (g.cstride) {
    const size_t co = (size_t)blockIdx.y * g.cstride;
    if (g.pc & PC_A) g.A += co;
    if (g.pc & PC_B) g.B += co;
    if (g.pc & PC_C) g.C += co;
    if (g.pc & PC_RS) g.rs += co;
    if (g.pc & PC_CS) g.cs += co;
    if (g.pc & PC_KS) g.ks += co;
  }
  extern __shared__ double sm64[];   // buffer b: A at sm64 + b (kGAsz + kGBsz), B right after it
  const int tilesN = (g.N + kG64 - 1) / kG64;
  const int m0 = (tile / tilesN) * kG64, n0 = (tile % tilesN) * kG64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1, l4 = lane & 3, l16 = lane & 15, lk = lane >> 4;
  // operand offsets within a buffer (k added per step)
  const int ia = wr * 32 + l4;        // A row of strip 0
  const int jb = wc * 32 + l16;       // B column of strip 0
  double acc[8][2];
#pragma unroll
  for (int r = 0; r < 8; ++r) { acc[r][0] = 0.0; acc[r][1] = 0.0; }
  const int nt = (g.K + kGBK - 1) / kGBK;
  double ra[8], rb[8];
  gemm64_load<TA, TB>(g, m0, n0, 0, ra, rb);
  gemm64_mask<TA, TB>(g, m0, n0, 0, ra, rb);
  gemm64_store<TA, TB>(sm64, sm64 + kGAsz, ra, rb);
  __syncthreads();
  for (int t = 0; t < nt; ++t) {
    const int cur = t & 1;
    if (t + 1 < nt) gemm64_load<TA, TB>(g, m0, n0, (t + 1) * kGBK, ra, rb);
    const double* A_ = sm64 + cur * (kGAsz + kGBsz);
    const double* B_ = A_ + kGAsz;
#pragma unroll
    for (int k4 = 0; k4 < kGBK; k4 += 4) {
      const int k = k4 + lk;
      double bv[2], av[8];
#pragma unroll
      for (int c = 0; c < 2; ++c)
        bv[c] = TB ? B_[(jb + 16 * c) * kSBt + k] : B_[k * kSB + jb + 16 * c];
#pragma unroll
      for (int r = 0; r < 8; ++r)
        av[r] = TA ? A_[k * kSAt + ia + 4 * r] : A_[(ia + 4 * r) * kSA + k];
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[r][c] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[r], bv[c], acc[r][c], 0, 0, 0);
    }
    if (t + 1 < nt) {
      double* An = sm64 + (cur ^ 1) * (kGAsz + kGBsz);
      gemm64_mask<TA, TB>(g, m0, n0, (t + 1) * kGBK, ra, rb);
      gemm64_store<TA, TB>(An, An + kGAsz, ra, rb);
    }
    __syncthreads();
  }
  // acc[r][c] in lane l is D[m0 + wr*32 + 4r + l/16][n0 + wc*32 + 16c + l%16]
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int col = n0 + wc * 32 + 16 * c + l16;
    if (col >= g.N) continue;
    const double cf = g.cs_mode ? scale_of(g.cs_mode, g.cs, g.cs_coef, col) : 1.0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int row = m0 + wr * 32 + 4 * r + lk;
      if (row >= g.M) continue;
      const double rf = g.rs_mode ? scale_of(g.rs_mode, g.rs, g.rs_coef, row) : 1.0;
      double v = g.alpha * (rf * acc[r][c] * cf);
      double* cp = g.C + (size_t)row * g.ldc + col;
      if (g.beta != 0.0) v += g.beta * (*cp);
      if (row == col) v += g.diag_add;
      *cp = v;
    }
  }
}

template <int TA, int TB>
__global__ __launch_bounds__(256) void k_gemm64(GemmArgs g, int ntiles) {
  gemm64_tile<TA, TB>(g, ntiles);
}

// Grouped products (blockIdx.z picks one) on the LDS-staged 64 x 64 tiles.
template <int TA, int TB>
__global__ __launch_bounds__(256) void k_gemm64_group(GemmGroup gg, int ntiles) {
  gemm64_tile<TA, TB>(gg.g[blockIdx.z], ntiles);
}

// 32 x 32 tiles staged through LDS like the 64 x 64 kernel (K in steps of
// 32), on v_mfma_f64_4x4x4f64, with the operands of K-step t + 2 loaded while
// the MFMAs of step t run (two register sets, two LDS buffers).  Wave (wr, wc)
// owns the 16 x 16 quarter (wr, wc): four 4 x 16 strips, acc[r] in lane l is
// D[m0 + 16 wr + 4 r + l / 16][n0 + 16 wc + l % 16].  LDS strides as for the
// 64 x 64 kernel: rows of 32 k padded by 4; the column-contiguous layouts by 8
// or 16, so that the four k rows a wave reads fall on different banks.
constexpr int kL32 = 32, kL32K = 32;
constexpr int kL32SA = kL32K + 4;    // A row-major [i][k]
constexpr int kL32SAt = kL32 + 8;    // A^T        [k][i]
constexpr int kL32SB = kL32 + 16;    // B row-major [k][j]
constexpr int kL32SBt = kL32K + 4;   // B^T        [j][k]
constexpr int kL32Asz = (kL32 * kL32SA > kL32K * kL32SAt) ? kL32 * kL32SA : kL32K * kL32SAt;
constexpr int kL32Bsz = (kL32K * kL32SB > kL32 * kL32SBt) ? kL32K * kL32SB : kL32 * kL32SBt;

// Unconditional loads of one K-step from clamped addresses (four of A and four
// of B per thread, coalesced along the contiguous index).
template <int TA, int TB>
__device__ __forceinline__ void gemm32l_load(const GemmArgs& g, int m0, int n0, int k0, double (&ra)[4],
                                             double (&rb)[4]) {
  const int t = threadIdx.x, a = t >> 5, b = t & 31;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ra[q] = TA ? g.A[(size_t)min(k0 + a + 8 * q, g.K - 1) * g.lda + min(m0 + b, g.M - 1)]
               : g.A[(size_t)min(m0 + a + 8 * q, g.M - 1) * g.lda + min(k0 + b, g.K - 1)];
    rb[q] = TB ? g.B[(size_t)min(n0 + a + 8 * q, g.N - 1) * g.ldb + min(k0 + b, g.K - 1)]
               : g.B[(size_t)min(k0 + a + 8 * q, g.K - 1) * g.ldb + min(n0 + b, g.N - 1)];
  }
}

// Zero outside the matrices, apply the k scaling (from ksl when staged),
// store into one LDS buffer.
template <int TA, int TB>
__device__ __forceinline__ void gemm32l_store(const GemmArgs& g, int m0, int n0, int k0, double (&ra)[4],
                                              double (&rb)[4], double* As, double* Bs, const double* ksl) {
  const int t = threadIdx.x, a = t >> 5, b = t & 31;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ai = TA ? m0 + b : m0 + a + 8 * q, ak = TA ? k0 + a + 8 * q : k0 + b;
    const double ksc =
        (g.ks_mode && ak < g.K) ? (ksl ? ksl[ak] : scale_of(g.ks_mode, g.ks, g.ks_coef, ak)) : 1.0;
    const double av = (ai < g.M && ak < g.K) ? ra[q] * ksc : 0.0;
    const int bj = TB ? n0 + a + 8 * q : n0 + b, bk = TB ? k0 + b : k0 + a + 8 * q;
    const double bv = (bj < g.N && bk < g.K) ? rb[q] : 0.0;
    if (TA) As[(a + 8 * q) * kL32SAt + b] = av;    // [k][i]
    else As[(a + 8 * q) * kL32SA + b] = av;        // [i][k]
    if (TB) Bs[(a + 8 * q) * kL32SBt + b] = bv;    // [j][k]
    else Bs[(a + 8 * q) * kL32SB + b] = bv;        // [k][j]
  }
}

template <int TA, int TB>
__device__ __forceinline__ void gemm32l_tile(GemmArgs g, int ntiles) {
  // physical workgroup -> logical tile: each XCD gets a contiguous range
  const int per = (ntiles + kGXcd - 1) / kGXcd;
  const int tile = (blockIdx.x % kGXcd) * per + blockIdx.x / kGXcd;
  if (tile >= ntiles) return;
  if (g.cstride) {
    const size_t co = (size_t)blockIdx.y * g.cstride;
    if (g.pc & PC_A) g.A += co;
    if (g.pc & PC_B) g.B += co;
    if (g.pc & PC_C) g.C += co;
    if (g.pc & PC_RS) g.rs += co;
    if (g.pc & PC_CS) g.cs += co;
    if (g.pc & PC_KS) g.ks += co;
  }
  __shared__ double sl[2][kL32Asz + kL32Bsz];
  // the k scaling, evaluated once per workgroup (K <= 512, keeping four
  // workgroups per CU in LDS), not once per staged element
  __shared__ double ksl[512];
  const double* ks_staged = nullptr;
  if (g.ks_mode && g.K <= 512) {   // uniform
    for (int e = threadIdx.x; e < g.K; e += 256) ksl[e] = scale_of(g.ks_mode, g.ks, g.ks_coef, e);
    __syncthreads();
    ks_staged = ksl;
  }
  const int tilesN = (g.N + kL32 - 1) / kL32;
  const int m0 = (tile / tilesN) * kL32, n0 = (tile % tilesN) * kL32;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1, lk = lane >> 4;
  const int ia = wr * 16 + (lane & 3);   // A row of strip 0
  const int jb = wc * 16 + (lane & 15);  // B column
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int nt = (g.K + kL32K - 1) / kL32K;
  auto mfmas = [&](const double* A_) {
    const double* B_ = A_ + kL32Asz;
#pragma unroll
    for (int k4 = 0; k4 < kL32K; k4 += 4) {
      const int k = k4 + lk;
      const double bv = TB ? B_[jb * kL32SBt + k] : B_[k * kL32SB + jb];
      double av[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) av[r] = TA ? A_[k * kL32SAt + ia + 4 * r] : A_[(ia + 4 * r) * kL32SA + k];
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[r], bv, acc[r], 0, 0, 0);
    }
  };
  // step t lives in buffer t % 2; register set 0 carries the even steps
  double ra0[4], rb0[4], ra1[4], rb1[4];
  gemm32l_load<TA, TB>(g, m0, n0, 0, ra0, rb0);
  if (nt > 1) gemm32l_load<TA, TB>(g, m0, n0, kL32K, ra1, rb1);
  gemm32l_store<TA, TB>(g, m0, n0, 0, ra0, rb0, sl[0], sl[0] + kL32Asz, ks_staged);
  __syncthreads();
  for (int t = 0; t < nt; t += 2) {
    if (t + 2 < nt) gemm32l_load<TA, TB>(g, m0, n0, (t + 2) * kL32K, ra0, rb0);
    mfmas(sl[0]);
    if (t + 1 < nt) gemm32l_store<TA, TB>(g, m0, n0, (t + 1) * kL32K, ra1, rb1, sl[1], sl[1] + kL32Asz, ks_staged);
    __syncthreads();
    if (t + 1 >= nt) break;
    if (t + 3 < nt) gemm32l_load<TA, TB>(g, m0, n0, (t + 3) * kL32K, ra1, rb1);
    mfmas(sl[1]);
    if (t + 2 < nt) gemm32l_store<TA, TB>(g, m0, n0, (t + 2) * kL32K, ra0, rb0, sl[0], sl[0] + kL32Asz, ks_staged);
    __syncthreads();
  }
  const int col = n0 + jb;
  if (col >= g.N) return;
  const double cf = g.cs_mode ? scale_of(g.cs_mode, g.cs, g.cs_coef, col) : 1.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = m0 + wr * 16 + 4 * r + lk;
    if (row >= g.M) continue;
    const double rf = g.rs_mode ? scale_of(g.rs_mode, g.rs, g.rs_coef, row) : 1.0;
    double v = g.alpha * (rf * acc[r] * cf);
    double* cp = g.C + (size_t)row * g.ldc + col;
    if (g.beta != 0.0) v += g.beta * (*cp);
    if (row == col) v += g.diag_add;
    *cp = v;
  }
}

template <int TA, int TB>
__global__ __launch_bounds__(256) void k_gemm32l(GemmArgs g, int ntiles) {
  gemm32l_tile<TA, TB>(g, ntiles);
}

__host__ __device__ inline GemmArgs gemm_args(int M, int N, int K, const double* A, int lda, int transA,
                                            const double* B, int ldb, int transB, double* C, int ldc,
                                            double alpha = 1.0, double beta = 0.0) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.transA = transA;
  g.B = B; g.ldb = ldb; g.transB = transB;
  g.C = C; g.ldc = ldc;
  g.alpha = alpha; g.beta = beta; g.diag_add = 0.0;
  g.rs = nullptr; g.rs_coef = 0.0; g.rs_mode = SC_NONE;
  g.cs = nullptr; g.cs_coef = 0.0; g.cs_mode = SC_NONE;
  g.ks = nullptr; g.ks_coef = 0.0; g.ks_mode = SC_NONE;
  g.cstride = 0; g.pc = 0; g.nch = 1; g.tile = 0;
  return g;
}

// Raise the dynamic LDS limit of the four k_gemm64 instances (once per device).
static inline hipError_t gemm64_set_lds() {
  const void* fns[] = {reinterpret_cast<const void*>(k_gemm64<0, 0>), reinterpret_cast<const void*>(k_gemm64<0, 1>),
                       reinterpret_cast<const void*>(k_gemm64<1, 0>), reinterpret_cast<const void*>(k_gemm64<1, 1>),
                       reinterpret_cast<const void*>(k_gemm64_group<0, 0>)};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm64_lds());
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// A group of products (same M, N and chain count; count <= 3) with the direct
// kernel; tiles as launch_gemm picks them for the whole group.
static inline hipError_t launch_gemm_group(const GemmGroup& gg, int count, hipStream_t s) {
  const GemmArgs& g = gg.g[0];
  if (g.M <= 0 || g.N <= 0 || count < 1 || count > 3) return hipSuccess;
  const int nch = g.nch > 0 ? g.nch : 1;
  // a single chain with enough 64 x 64 tiles over the group to cover the
  // chip: the LDS-staged kernel (over many chains of small lattices the direct
  // tiles are faster: 12.9 against 43.5 us for one product over 256 chains of
  // N = 64)
  bool plain = true;
  for (int i = 0; i < count; ++i) plain = plain && !gg.g[i].transA && !gg.g[i].transB;
  const int t64 = ((g.M + 63) / 64) * ((g.N + 63) / 64);
  if (plain && (g.tile == 64 || (g.tile == 0 && nch == 1 && (long long)t64 * count >= 240))) {
    const unsigned blocks = (unsigned)(((t64 + kGXcd - 1) / kGXcd) * kGXcd);
    hipLaunchKernelGGL((k_gemm64_group<0, 0>), dim3(blocks, nch, count), dim3(256), gemm64_lds(), s, gg, t64);
    return hipGetLastError();
  }
  const int t32 = ((g.M + 31) / 32) * ((g.N + 31) / 32);
  const bool use32 = g.tile == 32 || (g.tile != 16 && (long long)t32 * nch * count >= 192);
  const bool deep = nch == 1 && g.K >= 128;
  if (use32) {
    if (deep) launch_group_direct<32, 2, 8>(gg, count, dim3(t32, nch, count), s);
    else launch_group_direct<32, 1, 4>(gg, count, dim3(t32, nch, count), s);
  } else {
    const int t16 = ((g.M + 15) / 16) * ((g.N + 15) / 16);
    if (deep) launch_group_direct<16, 1, 8>(gg, count, dim3(t16, nch, count), s);
    else launch_group_direct<16, 1, 4>(gg, count, dim3(t16, nch, count), s);
  }
  return hipGetLastError();
}

// Tile choice: g.tile = 16, 32, 33 or 64 forces it (33: the LDS-staged
// 32 x 32 kernel, 64: the LDS-staged 64 x 64 kernel, both autotuner
// candidates); 0 picks the LDS-staged 32 x 32 kernel for batched products
// with M, N and K of at least 96 (14.6 against 17.1 us for the direct 32 x 32
// kernel and 15.2 us for 16 x 16 tiles over 64 chains of N = 100; at N = 64
// and below the direct kernels are faster), else 32 x 32 direct tiles once
// there are enough of them (over all chains) to cover the chip, else 16 x 16.
static inline hipError_t launch_gemm(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const int nch = g.nch > 0 ? g.nch : 1;
  if (g.tile == 33 || (g.tile == 0 && nch > 1 && g.M >= 96 && g.N >= 96 && g.K >= 96)) {
    const int t = ((g.M + 31) / 32) * ((g.N + 31) / 32);
    const dim3 grid((unsigned)(((t + kGXcd - 1) / kGXcd) * kGXcd), nch);
    if (!g.transA && !g.transB) hipLaunchKernelGGL((k_gemm32l<0, 0>), grid, dim3(256), 0, s, g, t);
    else if (!g.transA) hipLaunchKernelGGL((k_gemm32l<0, 1>), grid, dim3(256), 0, s, g, t);
    else if (!g.transB) hipLaunchKernelGGL((k_gemm32l<1, 0>), grid, dim3(256), 0, s, g, t);
    else hipLaunchKernelGGL((k_gemm32l<1, 1>), grid, dim3(256), 0, s, g, t);
    return hipGetLastError();
  }
  const int t64 = ((g.M + 63) / 64) * ((g.N + 63) / 64);
  if (g.tile == 64) {
    const unsigned blocks = (unsigned)(((t64 + kGXcd - 1) / kGXcd) * kGXcd);
    const dim3 grid(blocks, nch);
    if (!g.transA && !g.transB) hipLaunchKernelGGL((k_gemm64<0, 0>), grid, dim3(256), gemm64_lds(), s, g, t64);
    else if (!g.transA) hipLaunchKernelGGL((k_gemm64<0, 1>), grid, dim3(256), gemm64_lds(), s, g, t64);
    else if (!g.transB) hipLaunchKernelGGL((k_gemm64<1, 0>), grid, dim3(256), gemm64_lds(), s, g, t64);
    else hipLaunchKernelGGL((k_gemm64<1, 1>), grid, dim3(256), gemm64_lds(), s, g, t64);
    return hipGetLastError();
  }
  const int t32 = ((g.M + 31) / 32) * ((g.N + 31) / 32);
  const int t16 = ((g.M + 15) / 16) * ((g.N + 15) / 16);
  // over many chains 16 x 16 tiles where they pad much less (4.7 against
  // 7.0 us over 128 chains of N = 36, which 32 x 32 tiles pad to 64)
  const bool pad16 = nch > 1 && 4 * (long long)t16 <= 3 * (long long)t32 * 4 && (long long)t16 * nch >= 192;
  const bool use32 = g.tile == 32 || (g.tile == 0 && !pad16 && (long long)t32 * nch >= 192);
  // long K on few workgroups: eight waves split K, which measured 10-25%
  // faster than four at N = 288 and 648; one K-step per load round (27.0
  // against 27.9 us for two at N = 648)
  const bool deep = nch == 1 && g.K >= 128;
  if (use32) {
    if (deep) launch_direct<32, 1, 8>(g, dim3(t32, nch), s);
    else launch_direct<32, 1, 4>(g, dim3(t32, nch), s);
  } else {
    if (deep) launch_direct<16, 1, 8>(g, dim3(t16, nch), s);
    else launch_direct<16, 1, 4>(g, dim3(t16, nch), s);
  }
  return hipGetLastError();
}
