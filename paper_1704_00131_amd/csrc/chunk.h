// The slices between two stabilisations of a small lattice in one launch per
// chain (Algorithm 1 of the section "Pseudo code description": per slice the
// wrap, the sequential single flips of the section "The default: sequential
// single spin flips", and the equal-time estimators), with G resident in LDS.
//
// For n <= kChunkMaxN a chain's G and the exponentials exp(-+dtau K) (and
// exp(-dtau K/2) for the symmetric split), padded to NP = 16 ceil(n / 16) rows
// and columns with the padding kept zero, fit one workgroup's LDS, so a chunk
// of slices costs one launch per chain instead of a wrap GEMM pair, the block
// updates and a measurement launch per slice, and every product operand comes
// from LDS; the stabilisation step that follows each chunk is unchanged.  Arithmetic, per slice tau (B_tau =
// diag(v) E, v = exp(coupling s_tau)):
//   upward:   G <- diag(v) (E G) Einv diag(1/v), then the flips of the slice,
//             then the estimators (not after the chunk's last slice, which
//             the caller measures after the stabilisation);
//   downward: the flips, the estimators, then G <- Einv diag(1/v) G diag(v) E.
// A flip of site i: with the draws and ratio constants of the slice computed
// at its start from Philox counter (TAG_FLIP, sweep, (tau << 1) | dir, i), as
// in the blocked path, r = 1 + Delta (1 - G_ii), R = prefactor r^n_col,
// accept iff u < R, and then G <- G - (Delta / r) G[:,i] (e_i - G[i,:]).
#pragma once
#include "device_common.h"
#include "update.h"

constexpr int kChunkMaxN = 64;                   // 4 tiles of 16 per side
constexpr int kChunkMaxNT = kChunkMaxN / 16;

struct ChunkArgs {
  double* G;                       // N x N (ld N), per chain
  double* field;                   // [L][N], per chain, updated in place
  const double* E;                 // exp(-dtau K), exp(+dtau K): shared by the group
  const double* Einv;
  const double* Eh;                // exp(-dtau K / 2), exp(+dtau K / 2): symmetric split only
  const double* Ehinv;
  const double* K;                 // hopping matrix (E_kin)
  unsigned long long* counters;    // [0] proposals, [1] accepted, [2] sweep, [3] Philox key (per chain)
  double* bins;                    // per chain
  int* err;                        // per chain
  int N, tau0, ntau, dir;          // slices tau0, tau0 + 1, ... (dir 0) or tau0, tau0 - 1, ... (dir 1)
  int measure, skip_last, sym, kind, n_col;
  double coupling, alpha, prop_width, trK, u_int;
  Field4 f4;
  size_t cs;                       // per-chain stride (doubles); chain = blockIdx.y
};

__host__ __device__ inline int chunk_np(int n) { return (n + 15) / 16 * 16; }
// dynamic LDS: G, exp(-dtau K), exp(+dtau K) and, for the symmetric split,
// exp(-dtau K/2), each padded to NP rows of NP + 1 doubles
__host__ __device__ inline size_t chunk_lds(int n, int sym) {
  return sizeof(double) * (size_t)(3 + sym) * chunk_np(n) * (chunk_np(n) + 1);
}

struct ChunkShared {
  double du[kChunkMaxN], ddel[kChunkMaxN], dpre[kChunkMaxN], dsn[kChunkMaxN];   // the slice's draws
  double fld[kChunkMaxN];                                                      // the slice's field
  double diag[kChunkMaxN];                                                     // the diagonal of G (flips)
  double colv[kChunkMaxN], rowv[kChunkMaxN];                                   // an accepted flip's vectors
  double rsc[kChunkMaxN], csc[kChunkMaxN];                                     // row / column scales (0 past N)
  double part[kChunkMaxN][kChunkMaxNT];                                        // diagonal partials (symmetric split)
  double red[4][4];
};

// Gs <- diag(rsc) op diag(csc), op = Xs Gs (LEFT) or Gs Xs, both padded NP x
// NP matrices in LDS (row stride P), products on v_mfma_f64_16x16x4 with the
// wave's output tiles (tile t = w + 4 j of the NT x NT grid) in registers,
// written back in place after a barrier.
template <int NT, bool LEFT>
__device__ __forceinline__ void chunk_product(double* Gs, const double* Xs, int P, const ChunkShared& sh) {
  constexpr int NP = 16 * NT, MAXT = (NT * NT + 3) / 4;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  const int ntile = (NT * NT - w + 3) / 4;   // tiles of this wave (uniform)
  v4d acc[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) acc[t] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k0 = 0; k0 < NP; k0 += 4) {
    const int k = k0 + lk;
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      const int tile = min(w + 4 * t, NT * NT - 1), ti = tile / NT, tj = tile - ti * NT;
      if (t < ntile) {   // uniform
        const int row = ti * 16 + l16, col = tj * 16 + l16;
        if (LEFT) acc[t] = mfma_f64_16x16x4(Xs[row * P + k], Gs[k * P + col], acc[t]);
        else acc[t] = mfma_f64_16x16x4(Gs[row * P + k], Xs[k * P + col], acc[t]);
      }
    }
  }
  __syncthreads();   // every read of Gs is done
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    const int tile = min(w + 4 * t, NT * NT - 1), ti = tile / NT, tj = tile - ti * NT;
    if (t < ntile) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = ti * 16 + lk + 4 * r, col = tj * 16 + l16;
        Gs[row * P + col] = acc[t][r] * sh.rsc[row] * sh.csc[col];
      }
    }
  }
  __syncthreads();
}

// Equal-time estimators of the LDS-resident G into the chain's bins, in the
// sums and order of k_measure_part's bins update (D from the diagonal of
// G~ = G, or exp(-dtau K/2) G exp(+dtau K/2) for the symmetric split).
template <int NT>
__device__ __forceinline__ void chunk_measure(const double* Gs, const double* Ehs, int P, const ChunkArgs& a,
                                              double* bins, int* err, ChunkShared& sh) {
  constexpr int MAXT = (NT * NT + 3) / 4;
  const int N = a.N, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // sum of K o G: lane b of wave w takes column b, rows w + 4 k
  double skg = 0.0, bad = 0.0;
  if (lane < N) {
#pragma unroll
    for (int k = 0; k < 4 * NT; ++k) {
      const int i = w + 4 * k;
      if (i < N) {
        const double g = Gs[i * P + lane];
        skg = fma(a.K[(size_t)i * N + lane], g, skg);
        if (!isfinite(g)) bad = 1.0;
      }
    }
  }
  if (a.sym) {
    // T1 = Eh G by tiles in registers; d_i = sum_b T1[i][b] Ehinv[i][b]
    // (Ehinv symmetric): 16-lane sums per tile row, then the tiles of a row
    // in a fixed order
    const int l16 = lane & 15, lk = lane >> 4;
    v4d acc[MAXT];
#pragma unroll
    for (int t = 0; t < MAXT; ++t) acc[t] = (v4d){0.0, 0.0, 0.0, 0.0};
    const int ntile = (NT * NT - w + 3) / 4;
#pragma unroll 4
    for (int k0 = 0; k0 < 16 * NT; k0 += 4) {
      const int k = k0 + lk;
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        const int tile = min(w + 4 * t, NT * NT - 1), ti = tile / NT, tj = tile - ti * NT;
        if (t < ntile) acc[t] = mfma_f64_16x16x4(Ehs[(ti * 16 + l16) * P + k], Gs[k * P + tj * 16 + l16], acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      const int tile = min(w + 4 * t, NT * NT - 1), ti = tile / NT, tj = tile - ti * NT;
      if (t < ntile) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = ti * 16 + lk + 4 * r, col = tj * 16 + l16;
          const double eh = a.Ehinv[(size_t)min(row, N - 1) * N + min(col, N - 1)];
          double v = (row < N && col < N) ? acc[t][r] * eh : 0.0;
          v += __shfl_xor(v, 1, 64);
          v += __shfl_xor(v, 2, 64);
          v += __shfl_xor(v, 4, 64);
          v += __shfl_xor(v, 8, 64);
          if (l16 == 0) sh.part[row][tj] = v;
        }
      }
    }
    __syncthreads();
  }
  double sd = 0.0;
  if (tid < N) {
    double d;
    if (a.sym) {
      d = 0.0;
      for (int j = 0; j < NT; ++j) d += sh.part[tid][j];
    } else {
      d = Gs[tid * P + tid];
    }
    sd = d * (1.0 - d);
  }
  // fixed-order block sums (deterministic)
  for (int o = 32; o > 0; o >>= 1) {
    sd += __shfl_xor(sd, o, 64);
    skg += __shfl_xor(skg, o, 64);
    bad = fmax(bad, __shfl_xor(bad, o, 64));
  }
  if (lane == 0) { sh.red[w][0] = sd; sh.red[w][1] = skg; sh.red[w][2] = bad; }
  __syncthreads();
  if (tid == 0) {
    const double s0 = (sh.red[0][0] + sh.red[1][0]) + (sh.red[2][0] + sh.red[3][0]);
    const double s1 = (sh.red[0][1] + sh.red[1][1]) + (sh.red[2][1] + sh.red[3][1]);
    const double s2 = fmax(fmax(sh.red[0][2], sh.red[1][2]), fmax(sh.red[2][2], sh.red[3][2]));
    measure_bins(s0, s1, s2, N, a.trK, (double)a.n_col, a.u_int, bins, err);
  }
  __syncthreads();
}

template <int NT>
__global__ __launch_bounds__(256) void k_chunk(ChunkArgs a) {
  extern __shared__ double gsm[];
  __shared__ ChunkShared sh;
  constexpr int NP = 16 * NT;
  constexpr int P = NP + 1;
  double* G = a.G;
  double* field = a.field;
  double* bins = a.bins;
  int* err = a.err;
  unsigned long long* counters = a.counters;
  {
    const size_t co = (size_t)blockIdx.y * a.cs;
    G += co; field += co; bins += co;
    err = reinterpret_cast<int*>(reinterpret_cast<double*>(err) + co);
    counters = reinterpret_cast<unsigned long long*>(reinterpret_cast<double*>(counters) + co);
  }
  const int N = a.N, tid = threadIdx.x;
  double* Gs = gsm;
  double* Es = gsm + NP * P;
  double* Eis = Es + NP * P;
  double* Ehs = Eis + NP * P;   // symmetric split only
  for (int e = tid; e < NP * P; e += 256) {
    const int i = e / P, j = e - i * P;
    const bool in = i < N && j < N;
    const size_t src = in ? (size_t)i * N + j : 0;
    Gs[e] = in ? G[src] : 0.0;
    Es[e] = in ? a.E[src] : 0.0;
    Eis[e] = in ? a.Einv[src] : 0.0;
    if (a.sym) Ehs[e] = in ? a.Eh[src] : 0.0;
  }
  __syncthreads();
  // the rank-1 updates: lane b of wave w takes column b, rows w + 4 k (a
  // compile-time count, so the loads of a step issue together)
  constexpr int RPT = NP / 4;
  const int bcol = tid & 63, rg = tid >> 6;
  unsigned long long nacc = 0;
  for (int q = 0; q < a.ntau; ++q) {
    const int tau = a.dir == 0 ? a.tau0 + q : a.tau0 - q;
    double* frow = field + (size_t)(tau - 1) * N;
    if (a.dir == 0) {
      // wrap up: G <- diag(v) (E G) Einv diag(1/v)
      if (tid < NP) {
        const double v = tid < N ? exp(a.coupling * frow[tid]) : 0.0;
        sh.rsc[tid] = tid < N ? 1.0 : 0.0;
        sh.csc[tid] = tid < N ? 1.0 : 0.0;
        sh.colv[tid] = v;   // v kept for the second product's scales
      }
      __syncthreads();
      chunk_product<NT, true>(Gs, Es, P, sh);
      if (tid < NP) {
        const double v = sh.colv[tid];
        sh.rsc[tid] = v;
        sh.csc[tid] = tid < N ? 1.0 / v : 0.0;
      }
      __syncthreads();
      chunk_product<NT, false>(Gs, Eis, P, sh);
    }
    // the slice's draws (each site's field is unchanged before its own decision)
    if (tid < N) {
      const Philox4 r = philox4x64_10(TAG_FLIP, counters[2], ((unsigned long long)tau << 1) | (unsigned long long)a.dir,
                                      (unsigned long long)tid, counters[3], 0ull);
      const double u0 = unit_double(r.w[0]), u1 = unit_double(r.w[1]);
      const double s = frow[tid];
      double sn, extra;
      if (a.kind == FK_GAUSS) { sn = s + a.prop_width * (2.0 * u1 - 1.0); extra = -0.5 * (sn * sn - s * s); }
      else if (a.kind == FK_ISING4) {
        const int k = field4_index(a.f4, s);
        const int j = min((int)(3.0 * u1), 2);
        const int kn = (j < k) ? j : j + 1;
        sn = field4_pick(a.f4.eta, kn);
        extra = field4_pick(a.f4.lg, kn) - field4_pick(a.f4.lg, k);
      } else { sn = -s; extra = 0.0; }
      sh.du[tid] = u0;
      sh.ddel[tid] = exp(a.coupling * (sn - s)) - 1.0;
      sh.dpre[tid] = exp(a.n_col * a.coupling * a.alpha * (sn - s) + extra);
      sh.dsn[tid] = sn;
      sh.fld[tid] = s;
    }
    __syncthreads();
    // The flips with this thread's part of G in registers: lane b of wave w
    // holds G[w + 4k][b], k < RPT; the diagonal is mirrored in sh.diag.  An
    // accepted flip stages column i (its four owners) and e_i - row i (the
    // owning wave) in LDS, then every thread updates its registers.
    double g[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) g[k] = Gs[min(rg + 4 * k, NP - 1) * P + min(bcol, NP - 1)];
    if (bcol < N && (bcol & 3) == rg) {
      double d = g[0];
#pragma unroll
      for (int k = 1; k < RPT; ++k) d = (k == (bcol >> 2)) ? g[k] : d;
      sh.diag[bcol] = d;
    }
    __syncthreads();
    for (int i = 0; i < N; ++i) {
      const double del = sh.ddel[i];
      const double r = 1.0 + del * (1.0 - sh.diag[i]);
      const double R = sh.dpre[i] * ipow(r, a.n_col);
      if (sh.du[i] < R) {   // uniform: every thread computes the same R
        ++nacc;
        const double gam = del / r;
        if (bcol == i) {
#pragma unroll
          for (int k = 0; k < RPT; ++k) sh.colv[rg + 4 * k] = g[k];
        }
        if (rg == (i & 3) && bcol < N) {
          double gi = g[0];
#pragma unroll
          for (int k = 1; k < RPT; ++k) gi = (k == (i >> 2)) ? g[k] : gi;
          sh.rowv[bcol] = (bcol == i ? 1.0 : 0.0) - gi;
        }
        __syncthreads();
        // rows past N hold zeros and stay zero (their column entries are zero)
        const double rb = bcol < N ? gam * sh.rowv[bcol] : 0.0;
#pragma unroll
        for (int k = 0; k < RPT; ++k) g[k] = fma(-sh.colv[rg + 4 * k], rb, g[k]);
        if (bcol < N && (bcol & 3) == rg) {
          double d = g[0];
#pragma unroll
          for (int k = 1; k < RPT; ++k) d = (k == (bcol >> 2)) ? g[k] : d;
          sh.diag[bcol] = d;
        }
        if (tid == 0) sh.fld[i] = sh.dsn[i];
        __syncthreads();
      }
    }
    if (bcol < NP) {
#pragma unroll
      for (int k = 0; k < RPT; ++k) Gs[(rg + 4 * k) * P + bcol] = g[k];
    }
    if (tid < N) frow[tid] = sh.fld[tid];
    __syncthreads();   // the new field values in sh.fld
    if (a.measure && !(a.skip_last && q == a.ntau - 1)) chunk_measure<NT>(Gs, Ehs, P, a, bins, err, sh);
    if (a.dir == 1) {
      // wrap down: G <- Einv (diag(1/v) G diag(v)) E, with the slice's new field
      if (tid < NP) {
        const double v = tid < N ? exp(a.coupling * sh.fld[tid]) : 0.0;
        sh.colv[tid] = tid < N ? 1.0 / v : 0.0;
        sh.rowv[tid] = v;
        sh.rsc[tid] = tid < N ? 1.0 : 0.0;
        sh.csc[tid] = tid < N ? 1.0 : 0.0;
      }
      __syncthreads();
      if (bcol < N) {
        const double vb = sh.rowv[bcol];
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int r0 = rg + 4 * k;
          if (r0 < N) Gs[r0 * P + bcol] *= sh.colv[r0] * vb;
        }
      }
      __syncthreads();
      chunk_product<NT, false>(Gs, Es, P, sh);
      chunk_product<NT, true>(Gs, Eis, P, sh);
    }
  }
  for (int e = tid; e < N * N; e += 256) {
    const int i = e / N, j = e - i * N;
    G[e] = Gs[i * P + j];
  }
  if (tid == 0) {
    counters[0] += (unsigned long long)a.ntau * N;
    counters[1] += nacc;
  }
}
