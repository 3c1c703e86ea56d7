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
// Tiling: one workgroup of 256 threads (4 waves) computes a 32 x 32 tile of C;
// each wave owns a 16 x 16 quadrant held in one v_mfma_f64_16x16x4 accumulator.
// K is walked in chunks of 16, staged through LDS (both operands stored
// k-major so that the 16 lanes feeding one MFMA row read consecutive
// addresses), with the next chunk prefetched into registers while the current
// one is multiplied.
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
};

namespace gemm_cfg {
constexpr int TM = 32, TN = 32, TK = 16, NT = 256;
constexpr int PAD = 1;
}

__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  using namespace gemm_cfg;
  __shared__ double As[2][TK][TM + PAD];
  __shared__ double Bs[2][TK][TN + PAD];

  const int tilesN = (g.N + TN - 1) / TN;
  const int bi = blockIdx.x / tilesN, bj = blockIdx.x % tilesN;
  const int i0 = bi * TM, j0 = bj * TN;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;

  // each thread moves 2 elements of each operand per chunk (32*16 = 512)
  double ra[2], rb[2];
  int ai[2], ak[2], bk[2], bj_[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = t + NT * q;
    if (!g.transA) { ai[q] = e / TK; ak[q] = e % TK; } else { ak[q] = e / TM; ai[q] = e % TM; }
    if (!g.transB) { bk[q] = e / TN; bj_[q] = e % TN; } else { bj_[q] = e / TK; bk[q] = e % TK; }
  }

  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int i = i0 + ai[q], k = k0 + ak[q];
      double v = 0.0;
      if (i < g.M && k < g.K) {
        v = g.transA ? g.A[(size_t)k * g.lda + i] : g.A[(size_t)i * g.lda + k];
        if (g.ks_mode) v *= scale_of(g.ks_mode, g.ks, g.ks_coef, k);
      }
      ra[q] = v;
      const int kb = k0 + bk[q], j = j0 + bj_[q];
      double u = 0.0;
      if (kb < g.K && j < g.N) u = g.transB ? g.B[(size_t)j * g.ldb + kb] : g.B[(size_t)kb * g.ldb + j];
      rb[q] = u;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      As[buf][ak[q]][ai[q]] = ra[q];
      Bs[buf][bk[q]][bj_[q]] = rb[q];
    }
  };

  v4d acc = {0.0, 0.0, 0.0, 0.0};
  const int nchunks = (g.K + TK - 1) / TK;
  if (nchunks > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  int cur = 0;
  for (int c = 0; c < nchunks; ++c) {
    const bool more = (c + 1) < nchunks;
    if (more) load((c + 1) * TK);
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const double a = As[cur][kk + (lane >> 4)][wr * 16 + (lane & 15)];
      const double b = Bs[cur][kk + (lane >> 4)][wc * 16 + (lane & 15)];
      acc = mfma_f64_16x16x4(a, b, acc);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }

  const int col = j0 + wc * 16 + (lane & 15);
  if (col >= g.N) return;
  const double cf = g.cs_mode ? scale_of(g.cs_mode, g.cs, g.cs_coef, col) : 1.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = i0 + wr * 16 + (lane >> 4) + 4 * r;
    if (row >= g.M) continue;
    const double rf = g.rs_mode ? scale_of(g.rs_mode, g.rs, g.rs_coef, row) : 1.0;
    double v = g.alpha * (rf * acc[r] * cf);
    double* cp = g.C + (size_t)row * g.ldc + col;
    if (g.beta != 0.0) v += g.beta * (*cp);
    if (row == col) v += g.diag_add;
    *cp = v;
  }
}

static inline GemmArgs gemm_args(int M, int N, int K, const double* A, int lda, int transA,
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
  return g;
}

static inline hipError_t launch_gemm(const GemmArgs& g, hipStream_t s) {
  using namespace gemm_cfg;
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const int tiles = ((g.M + TM - 1) / TM) * ((g.N + TN - 1) / TN);
  hipLaunchKernelGGL(k_gemm, dim3(tiles), dim3(NT), 0, s, g);
  return hipGetLastError();
}
