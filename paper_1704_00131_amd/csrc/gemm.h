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
// Tiling: one workgroup of 256 threads (4 waves) computes a TILE x TILE tile
// of C (TILE = 16 or 32, chosen per launch so that small products still
// spread over many CUs); the four waves split K and their partial
// accumulators are summed through LDS.  Operands are read straight from
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

template <int TILE>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  constexpr int NB = TILE / 16;
  if (g.cstride) {
    const size_t co = (size_t)blockIdx.y * g.cstride;
    if (g.pc & PC_A) g.A += co;
    if (g.pc & PC_B) g.B += co;
    if (g.pc & PC_C) g.C += co;
    if (g.pc & PC_RS) g.rs += co;
    if (g.pc & PC_CS) g.cs += co;
    if (g.pc & PC_KS) g.ks += co;
  }
  __shared__ double red[3][NB * NB][4][64];
  const int tilesN = (g.N + TILE - 1) / TILE;
  const int i0 = (blockIdx.x / tilesN) * TILE, j0 = (blockIdx.x % tilesN) * TILE;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  // contiguous K range of this wave, a multiple of 4 long
  const int kq = ((g.K + 15) / 16) * 4;
  const int kb = w * kq, ke = min(g.K, kb + kq);
  v4d acc[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  for (int k0 = kb; k0 < ke; k0 += 4) {
    const int k = k0 + lk;
    const bool kin = k < ke;
    const double ksc = (kin && g.ks_mode) ? scale_of(g.ks_mode, g.ks, g.ks_coef, k) : 1.0;
    double av[NB], bv[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      const int row = i0 + a * 16 + l16;
      double v = 0.0;
      if (kin && row < g.M) v = g.transA ? g.A[(size_t)k * g.lda + row] : g.A[(size_t)row * g.lda + k];
      av[a] = v * ksc;
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int col = j0 + b * 16 + l16;
      double v = 0.0;
      if (kin && col < g.N) v = g.transB ? g.B[(size_t)col * g.ldb + k] : g.B[(size_t)k * g.ldb + col];
      bv[b] = v;
    }
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[a][b] = mfma_f64_16x16x4(av[a], bv[b], acc[a][b]);
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
        const double sum = acc[a][b][r] + red[0][a * NB + b][r][lane] + red[1][a * NB + b][r][lane] +
                           red[2][a * NB + b][r][lane];
        const double rf = g.rs_mode ? scale_of(g.rs_mode, g.rs, g.rs_coef, row) : 1.0;
        double v = g.alpha * (rf * sum * cf);
        double* cp = g.C + (size_t)row * g.ldc + col;
        if (g.beta != 0.0) v += g.beta * (*cp);
        if (row == col) v += g.diag_add;
        *cp = v;
      }
    }
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

// Tile choice: g.tile = 16 or 32 forces it; 0 picks 32 x 32 tiles once there
// are enough of them (over all chains) to cover the chip.
static inline hipError_t launch_gemm(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const int nch = g.nch > 0 ? g.nch : 1;
  const int t32 = ((g.M + 31) / 32) * ((g.N + 31) / 32);
  const bool use32 = g.tile == 32 || (g.tile == 0 && (long long)t32 * nch >= 192);
  if (use32) {
    hipLaunchKernelGGL(k_gemm<32>, dim3(t32, nch), dim3(256), 0, s, g);
  } else {
    const int t16 = ((g.M + 15) / 16) * ((g.N + 15) / 16);
    hipLaunchKernelGGL(k_gemm<16>, dim3(t16, nch), dim3(256), 0, s, g);
  }
  return hipGetLastError();
}
