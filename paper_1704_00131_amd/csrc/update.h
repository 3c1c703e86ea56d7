// Sequential single-flip updates of one slice, in blocks of up to 32 sites
// (section "Updating schemes", "The default: sequential single spin flips").
//
// Flip at site p of slice tau (from Eq. (Green_eq) and the matrix determinant
// lemma; the paper states the fast update's O(N^2) cost):
//   Delta = exp(coupling (s' - s)) - 1,  r = 1 + Delta (1 - G_pp),
//   R = exp(N_col coupling alpha (s' - s)) r^N_col  (x exp(-(s'^2 - s^2)/2) for
//   a Gaussian field),  accept iff u < R,
//   G <- G - (Delta/r) G[:,p] (e_p - G[p,:])      (Sherman-Morrison).
//
// Blocking (a regrouping of the same arithmetic, exact up to rounding): the
// decisions of a block S of consecutive sites only read G[S,S], so the
// sequential Sherman-Morrison steps run on the |S| x |S| block in LDS, while
// the full matrix is carried as
//   G_cur = G - G[:,S] Phi (E_S^T - G[S,:]),
// where each accepted step adds gamma a b^T to Phi with
//   a = e_j - Phi (e_j - G[S,p]),  b = e_j + Phi^T G[p,S]^T,  gamma = Delta/r.
// After the block, G <- G - G[:,S] W with W = Phi (E_S^T - G[S,:]): one
// rank-|S| MFMA update of G instead of |S| rank-1 passes over it.
#pragma once
#include "device_common.h"

struct BlockArgs {
  const double* Gin;                 // G before the block (N x N)
  double* Gout;                      // G after the block (N x N, distinct from Gin)
  int N; int s0; int bb;
  const double* field_in;            // field of slice tau before the block (N values)
  double* field_out;                 // field of slice tau after the block (may equal field_in only for
                                     // sites outside this block; distinct buffer otherwise)
  const double* draws;               // slice tau of k_pass_draws' output: (u, Delta, prefactor, s_new) per site
  unsigned long long* counters;      // [0] proposals, [1] accepted, [2] sweep, [3] Philox key
  size_t cs;                         // per-chain stride (doubles) of every pointer above; chain = blockIdx.y
};

// The four-valued field of Eq. (HS_squares): eta(l) and log gamma(l) in the
// order l = -2, -1, +1, +2 (the field stores eta; the host fills the table).
// Field kinds: 0 Ising (+-1), 1 Gaussian, 2 four-valued.
struct Field4 { double eta[4]; double lg[4]; };
enum { FK_ISING = 0, FK_GAUSS = 1, FK_ISING4 = 2 };

// index 0..3 of a stored four-valued field value (the values are distinct)
__device__ __forceinline__ int field4_index(const Field4& t, double s) {
  return (s > t.eta[0] ? 1 : 0) + (s > t.eta[1] ? 1 : 0) + (s > t.eta[2] ? 1 : 0);
}
__device__ __forceinline__ double field4_pick(const double (&v)[4], int k) {
  return k == 0 ? v[0] : (k == 1 ? v[1] : (k == 2 ? v[2] : v[3]));
}

// Draws and ratio constants of every site of one pass (upward or downward
// half of a sweep), computed before the pass: each site is visited once per
// pass, so they depend only on the field at the start of the pass.  For site
// i of slice tau, from Philox counter (TAG_FLIP, sweep, (tau << 1) | dir, i):
//   u = u0; s_new = -s (Ising), s + width (2 u1 - 1) (Gaussian), or the value of
//   index floor(3 u1) among the three others in increasing order (four-valued);
//   Delta = exp(coupling (s_new - s)) - 1;
//   prefactor = exp(n_col coupling alpha (s_new - s) + extra), extra =
//   -(s_new^2 - s^2)/2 (Gaussian), log gamma(l') - log gamma(l) (four-valued), 0.
// out[(tau-1) N + i][0..3] = (u, Delta, prefactor, s_new); grid (ceil(L N / 256), chains).
__global__ __launch_bounds__(256) void k_pass_draws(const double* field, int L, int N, unsigned long long dir,
                                                    double coupling, double alpha, int n_col, int kind,
                                                    double prop_width, Field4 f4, const unsigned long long* counters,
                                                    double* out, size_t cs) {
  const size_t co = (size_t)blockIdx.y * cs;
  field += co;
  out += co;
  counters = reinterpret_cast<const unsigned long long*>(reinterpret_cast<const double*>(counters) + co);
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= L * N) return;
  const int tau = e / N + 1, i = e % N;
  const Philox4 r = philox4x64_10(TAG_FLIP, counters[2], ((unsigned long long)tau << 1) | dir, (unsigned long long)i,
                                  counters[3], 0ull);
  const double u0 = unit_double(r.w[0]), u1 = unit_double(r.w[1]);
  const double s = field[e];
  double sn, extra;
  if (kind == FK_GAUSS) { sn = s + prop_width * (2.0 * u1 - 1.0); extra = -0.5 * (sn * sn - s * s); }
  else if (kind == FK_ISING4) {
    const int k = field4_index(f4, s);
    const int j = min((int)(3.0 * u1), 2);
    const int kn = (j < k) ? j : j + 1;
    sn = field4_pick(f4.eta, kn);
    extra = field4_pick(f4.lg, kn) - field4_pick(f4.lg, k);
  } else { sn = -s; extra = 0.0; }
  out[4 * (size_t)e] = u0;
  out[4 * (size_t)e + 1] = exp(coupling * (sn - s)) - 1.0;
  out[4 * (size_t)e + 2] = exp(n_col * coupling * alpha * (sn - s) + extra);
  out[4 * (size_t)e + 3] = sn;
}

__device__ __forceinline__ double ipow(double r, int n) {
  double p = 1.0;
  for (int k = 0; k < n; ++k) p *= r;
  return p;
}


// One workgroup of four waves per 32 x 32 tile (I, J) of G.  Every workgroup
// takes the same sequential decisions of block S (identical arithmetic,
// identical results), then writes
//   Gout[I,J] = Gin[I,J] - Gin[I,S] Phi (E_S^T[:,J] - Gin[S,J]).
//
// Decisions (wave 0 alone): lane x keeps row x of the current c = G_cur[S,S]
// in registers and the draws of site x.  Site i reads c_ii from lane i; an
// accepted flip updates only the trailing block,
//   c[x][y] += gamma c[x][i] c[i][y]   (x, y > i; row i broadcast by readlane),
// since later decisions read only entries past i.  So column i is final
// before site i (only earlier sites touch it) and row i after it, and the
// records of the Phi recursion are
//   T_A[m][k] = -gamma_m c[m][k],  T_B[m][k] = -gamma_m c[k][m]   (k > m).
//
// With the vectors of the Phi recursion in the header, U_i = c a_i and
// V_i = (1 - c_0)^T b_i, so the recursions for a and b become triangular:
//   A (1 + T_A) = 1,  B (1 + T_B) = 1,  Phi = A diag(gamma) B^T.
// The tile needs Phi only inside X diag(gamma) Z with X = Gin[I,S] A and
// Z = B^T (E_S^T[:,J] - Gin[S,J]), that is
//   X[r][k]   = Gin[I+r][S+k] + sum_{m<k} gamma_m X[r][m] c[m][k],
//   Z^T[y][k] = (E_S^T[:,J] - Gin[S,J])[k][y] + sum_{m<k} gamma_m Z^T[y][m] c[k][m].
// Both read c by columns only.  Wave 0 therefore stores each column of c in
// LDS as soon as it is final (one store per lane) and gamma of each site once
// decided, and waves 1 and 2 solve the two systems while the decisions go on:
// wave 1 the rows of X, left-looking (entry k is one dot product with column
// k), wave 2 the rows of Z^T, right-looking (a final entry m is taken out of
// the later ones with column m).  Two lanes share a row, lane sub holding the
// entries k = sub mod 2.  An LDS counter, stored by wave 0 with workgroup-scope
// release one site behind its own stores (so the release finds them done and
// wave 0 does not wait), tells the solving waves how far columns and gammas
// are visible; they read it with acquire.  One MFMA product on all four waves
// finishes the tile.  Workgroup 0 also writes the block's field values and
// the counters.
//
// TR = 64 or 128: tiles of TR rows and 32 columns on TR / 8 waves, the odd
// waves 1, 3, 5, 7 solving the rows of X in groups of 32 (so that a single
// chain of N = 648 needs 231 workgroups, one per CU, instead of 441, which put
// two on most CUs; and a batch repeats each block's decisions in fewer
// workgroups).
template <int NCOL, int TR = 32>
__global__ __launch_bounds__(8 * TR) void k_block_update(BlockArgs a) {
  // rows of X for row group 0 in AB[0], of Z^T in AB[1], of X for row group
  // g >= 1 in AB[g + 1]
  __shared__ double AB[TR / 32 + 1][32][33];
  // columns of c, each split by row parity: colc[i][(x & 1) * 16 + (x >> 1)] = c[x][i]
  __shared__ __attribute__((aligned(16))) double colc[32][32];
  __shared__ double gam[32];
  // vis = v: columns 0..v-1 and gamma_0..gamma_{v-2} are visible
  __shared__ int nacc_s, vis;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int bb = a.bb, s0 = a.s0, N = a.N;
  const int tilesN = (N + 31) >> 5;
  if (a.cs) {
    const size_t co = (size_t)blockIdx.y * a.cs;
    a.Gin += co; a.Gout += co; a.field_in += co; a.field_out += co; a.draws += co;
    a.counters = reinterpret_cast<unsigned long long*>(reinterpret_cast<double*>(a.counters) + co);
  }
  const int I0 = (blockIdx.x / tilesN) * TR, J0 = (blockIdx.x % tilesN) << 5;
  const int wr = w >> 1, wc = w & 1;
  // this thread's four output elements of Gin, fetched early
  const int col = J0 + wc * 16 + (lane & 15);
  double gin[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = I0 + wr * 16 + (lane >> 4) + 4 * r;
    gin[r] = (row < N && col < N) ? a.Gin[(size_t)row * N + col] : 0.0;
  }
  if (tid == 0) vis = 0;
  const int x = lane & 31;               // wave 0: row of c (lanes x and x + 32 alike)
  const int fr = lane >> 1, sub = lane & 1;   // waves 1, 2: row of X or Z^T, entry parity
  double c[32];
  double u = 2.0, dl = 0.0, pr = 0.0, sold = 0.0, snew = 0.0;
  double R[16];                          // waves 1, 2: entries k = 2 j + sub of the row
  if (w == 0) {
    // G[S,S] through LDS (AB[1] is free until the product): two rows per
    // load, zero outside the block
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int e = 64 * j + lane, rr = e >> 5, cc = e & 31;
      c[j] = a.Gin[(size_t)(s0 + min(rr, bb - 1)) * N + s0 + min(cc, bb - 1)];
    }
    // draws and ratio constants of site x (from k_pass_draws)
    {
      const double* d = a.draws + 4 * (size_t)(s0 + min(x, bb - 1));
      u = d[0]; dl = d[1]; pr = d[2]; snew = d[3];
      sold = a.field_in[s0 + min(x, bb - 1)];
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int e = 64 * j + lane, rr = e >> 5, cc = e & 31;
      AB[1][rr][cc] = (rr < bb && cc < bb) ? c[j] : 0.0;
    }
  } else if ((w & 1) && (w >> 1) < TR / 32) {
    // right-hand side of X, Gin[r0+r][s0+k], through LDS: two rows per load
    const int xg = w >> 1, r0 = I0 + 32 * xg;
    double (*st)[33] = AB[xg == 0 ? 0 : xg + 1];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int e = 64 * j + lane, rr = e >> 5, cc = e & 31;
      R[j] = a.Gin[(size_t)min(r0 + rr, N - 1) * N + s0 + min(cc, bb - 1)];
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int e = 64 * j + lane, rr = e >> 5, cc = e & 31;
      st[rr][cc] = (r0 + rr < N && cc < bb) ? R[j] : 0.0;
    }
  } else if (w == 2) {
    // right-hand side of Z^T: delta - Gin[s0+k][J0+fr]
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int k = 2 * j + sub;
      R[j] = a.Gin[(size_t)(s0 + min(k, bb - 1)) * N + min(J0 + fr, N - 1)];
    }
  }
  __syncthreads();   // vis initialised (the loads above may still be in flight)
  if (w == 0) {
#pragma unroll
    for (int y = 0; y < 32; ++y) c[y] = AB[1][x][y];
    const int q = (x & 1) * 16 + (x >> 1);
    colc[0][q] = c[0];                     // lanes x and x + 32 store the same value
    gam[x] = 0.0;
    int nacc = 0, myacc = 0;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      __builtin_amdgcn_sched_barrier(0);   // keeps the per-site scalars from piling up in SGPRs
      if (i < bb) {
        const double cii = readlane_d(c[i], i);
        const double dli = readlane_d(dl, i);
        const double r = 1.0 + dli * (1.0 - cii);
        const double Rt = readlane_d(pr, i) * (NCOL == 2 ? r * r : r);
        // columns 0..i and gammas 0..i-1 were stored at the end of the last site
        __hip_atomic_store(&vis, i + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        double gs = 0.0;
        if (readlane_d(u, i) < Rt) {           // uniform across the wave
          const double gi = dli / r;
          gs = gi;
          ++nacc;
          if (x == i) myacc = 1;
          // row i broadcast, then the rank-1 update of the rows below i (a
          // zero factor keeps the frozen rows as they are)
          const double f = (x > i) ? gi * c[i] : 0.0;
#pragma unroll
          for (int y0 = i + 1; y0 < 32; y0 += 8) {
            double ci[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) if (y0 + t < 32) ci[t] = readlane_d(c[y0 + t], i);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < 8; ++t) if (y0 + t < 32) c[y0 + t] = fma(f, ci[t], c[y0 + t]);
          }
        }
        if (i + 1 < 32) colc[i + 1][q] = c[i + 1];   // column i + 1 is final now
        gam[i] = gs;                         // gs is the same in every lane
      }
    }
    // gamma of the last site; also ends every wait when the block is empty
    __hip_atomic_store(&vis, bb + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (lane == 0) nacc_s = nacc;
    if (blockIdx.x == 0 && lane < bb) a.field_out[s0 + lane] = myacc ? snew : sold;
  } else if ((w & 1) && (w >> 1) < TR / 32) {
    // X, left-looking: step k needs column k and gamma_m for m < k (vis > k).
    // P[j] = gamma_m X[fr][m] for the final entries m = 2 j + sub, else 0.
    const int xg = w >> 1;
    double (*st)[33] = AB[xg == 0 ? 0 : xg + 1];
#pragma unroll
    for (int j = 0; j < 16; ++j) R[j] = st[fr][2 * j + sub];
    double P[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) P[j] = 0.0;
    int seen = 0;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      if (k < bb) {
        while (seen < k + 1) seen = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&vis, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
        if (k > 0 && sub == ((k - 1) & 1)) P[(k - 1) >> 1] = gam[k - 1] * R[(k - 1) >> 1];
        // sum over m < k of P[m] c[m][k]
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int j = 0; 2 * j < k; ++j) s4[j & 3] = fma(P[j], colc[k][sub * 16 + j], s4[j & 3]);
        double part = (s4[0] + s4[1]) + (s4[2] + s4[3]);
        part += dpp_all<0xB1>(part);           // both lanes of the row
        if (sub == (k & 1)) R[k >> 1] += part;
      }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) st[fr][2 * j + sub] = R[j];
  } else if (w == 2) {
    // Z^T, right-looking: step m needs column m and gamma_m (vis > m + 1),
    // fetched together; the last step would only touch entries past the
    // block, which stay as they are
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int k = 2 * j + sub;
      R[j] = ((s0 + k == J0 + fr) ? 1.0 : 0.0) - ((k < bb && J0 + fr < N) ? R[j] : 0.0);
    }
    int seen = 0;
#pragma unroll
    for (int m = 0; m < 31; ++m) {
      if (m + 1 < bb) {
        const int jm = m >> 1;
        while (seen < m + 2) seen = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&vis, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
        const double g = gam[m];
        double cur[16];
#pragma unroll
        for (int j = jm; j < 16; ++j) cur[j] = colc[m][sub * 16 + j];
        // Z^T[fr][m] from its owner lane (DPP quad permutes [0,0,2,2] / [1,1,3,3])
        const double val = (m & 1) ? dpp_all<0xF5>(R[jm]) : dpp_all<0xA0>(R[jm]);
        const double t = g * val;
        R[jm] = fma(sub > (m & 1) ? t : 0.0, cur[jm], R[jm]);
#pragma unroll
        for (int j = jm + 1; j < 16; ++j) R[j] = fma(t, cur[j], R[j]);
      }
    }
    // AB[1] held G[S,S] for wave 0 until its first release
    while (seen < 1) seen = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(&vis, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
#pragma unroll
    for (int j = 0; j < 16; ++j) AB[1][fr][2 * j + sub] = R[j];
  }
  __syncthreads();
  // Gout tile = Gin - X diag(gamma) Z  (32 x 32 x 32 on MFMA)
  v4d acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < 32; k0 += 4) {
    const int k = k0 + (lane >> 4);
    const double av_ = AB[(wr >> 1) == 0 ? 0 : (wr >> 1) + 1][(wr & 1) * 16 + (lane & 15)][k] * gam[k];
    const double bv_ = AB[1][wc * 16 + (lane & 15)][k];
    acc2 = mfma_f64_16x16x4(av_, bv_, acc2);
  }
  if (col < N) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = I0 + wr * 16 + (lane >> 4) + 4 * r;
      if (row < N) a.Gout[(size_t)row * N + col] = gin[r] - acc2[r];
    }
  }
  if (blockIdx.x == 0 && tid == 0) {
    atomicAdd(&a.counters[0], (unsigned long long)bb);
    atomicAdd(&a.counters[1], (unsigned long long)nacc_s);
  }
}

// --------------------------------------------------------- measurements ----
// Equal-time estimators per site (section "Observables"): with d_i the
// diagonal of the measured Green's function,
//   D = (1/N) sum_i d_i (1 - d_i),  E_kin = (n_col/N)(Tr K - Tr(K G)),  E_pot = U D.
// For a symmetric split d_i = sum_b T1[i][b] Ehinv[b][i] with
// T1 = exp(-dtau K/2) G (Ehinv is symmetric, so the sum runs along row i of
// both).  K is symmetric, so Tr(K G) = sum_e K[e] G[e].
//
// k_measure_part gives each workgroup `rows` rows (wave w takes rows
// r0 + w, r0 + w + 4, ...; one row at a time across the wave, coalesced, with
// the row's loads unconditional so they overlap) and writes the partial sums
// (sum d (1 - d), sum K.G, non-finite flag); the workgroup that finishes last
// (a counter after the partials, taken with a device-scope atomic behind a
// release fence, and reset by that workgroup) adds the partials with one wave
// and updates the bins.  For small N a single workgroup covers all rows
// (nblk == 1).  SYM: d_i from T1 and Ehinv as above, else the diagonal of G.
constexpr int kMeasRows = 4, kMeasSmallN = 128;

__device__ __forceinline__ void measure_bins(double sd, double skg, double bad, int N, double trK, double n_col,
                                             double u_int, double* bins, int* err) {
  const double D = sd / N;
  bins[0] += D;
  bins[1] += n_col / N * (trK - skg);
  bins[2] += u_int * D;
  bins[3] += 1.0;
  if (bad > 0.0) atomicOr(err, 1);
}

template <bool SYM>
__global__ __launch_bounds__(256) void k_measure_part(const double* G, const double* T1, const double* Ehinv,
                                                      const double* K, int N, int rows, double* part, double trK,
                                                      double n_col, double u_int, double* bins, int* err, size_t cs) {
  __shared__ double red[4][3];
  __shared__ int last_s;
  {
    const size_t co = (size_t)blockIdx.y * cs;
    G += co;
    if (SYM) T1 += co;
    part += co;
    bins += co;
    err = reinterpret_cast<int*>(reinterpret_cast<double*>(err) + co);
  }
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r0 = blockIdx.x * rows, r1 = min(N, r0 + rows);
  double sd = 0.0, skg = 0.0, bad = 0.0;   // this wave's rows (same in every lane)
  for (int i = r0 + w; i < r1; i += 4) {
    const double* gi = G + (size_t)i * N;
    const double* ki = K + (size_t)i * N;
    double v[4] = {0.0, 0.0, 0.0, 0.0};    // K.G, T1.Ehinv, non-finite
#pragma unroll 4
    for (int b = lane; b < N; b += 64) {
      const double gv = gi[b];
      v[0] = fma(ki[b], gv, v[0]);
      if (!isfinite(gv)) v[2] = 1.0;
      if (SYM) v[1] = fma(T1[(size_t)i * N + b], Ehinv[(size_t)i * N + b], v[1]);
    }
    wave_sums<4>(v);
    const double d = SYM ? v[1] : gi[i];
    sd += d * (1.0 - d);
    skg += v[0];
    bad += v[2];
  }
  if (lane == 0) { red[w][0] = sd; red[w][1] = skg; red[w][2] = bad; }
  __syncthreads();
  const int nblk = gridDim.x;
  unsigned int* counter = reinterpret_cast<unsigned int*>(part + 4 * (size_t)nblk);
  if (tid == 0) {
    part[4 * blockIdx.x] = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
    part[4 * blockIdx.x + 1] = (red[0][1] + red[1][1]) + (red[2][1] + red[3][1]);
    part[4 * blockIdx.x + 2] = (red[0][2] + red[1][2]) + (red[2][2] + red[3][2]);
    __threadfence();
    last_s = (atomicAdd(counter, 1u) == (unsigned)nblk - 1u);
  }
  __syncthreads();
  if (!last_s || w != 0) return;
  __threadfence();
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = lane; b < nblk; b += 64) {
    v[0] += __builtin_nontemporal_load(part + 4 * b);
    v[1] += __builtin_nontemporal_load(part + 4 * b + 1);
    v[2] += __builtin_nontemporal_load(part + 4 * b + 2);
  }
  wave_sums<4>(v);
  if (lane == 0) {
    measure_bins(v[0], v[1], v[2], N, trK, n_col, u_int, bins, err);
    *counter = 0u;   // ready for the next measurement (kernel boundaries order it)
  }
}

// Weight ratio of one proposed change s -> s_new at a site, from G(tau) (the
// same formulas as the sweep's decisions); one thread.
__global__ void k_ratio(const double* G, int N, int site, const double* field_row, double s_new, double coupling,
                        double alpha, int n_col, int kind, Field4 f4, double* out) {
  if (threadIdx.x != 0) return;
  const double s = field_row[site];
  const double extra = kind == FK_GAUSS    ? -0.5 * (s_new * s_new - s * s)
                       : kind == FK_ISING4 ? field4_pick(f4.lg, field4_index(f4, s_new)) -
                                                 field4_pick(f4.lg, field4_index(f4, s))
                                           : 0.0;
  const double dl = exp(coupling * (s_new - s)) - 1.0;
  const double r = 1.0 + dl * (1.0 - G[(size_t)site * N + site]);
  out[0] = exp(n_col * coupling * alpha * (s_new - s) + extra) * ipow(r, n_col);
}

// max |Gw - Gs| into prec_slot (zero on entry), G <- Gs, NaN/Inf check.
// Each workgroup takes kPrecPer x 256 consecutive elements per round (all of
// a thread's loads in flight together), so that few workgroups, and few
// atomics on the one slot, cover the matrix: prec_grid(count) of them.
constexpr int kPrecPer = 8;
inline unsigned prec_grid(size_t count) {
  const size_t g = (count + 256 * kPrecPer - 1) / (256 * kPrecPer);
  return (unsigned)(g < 1024 ? (g > 0 ? g : 1) : 1024);
}
__global__ __launch_bounds__(256) void k_prec_replace(const double* Gw, double* G, const double* Gs, size_t count,
                                                      double* prec_slot, int* err, size_t cs) {
  __shared__ double red[8];
  {
    const size_t co = (size_t)blockIdx.y * cs;
    Gw += co; G += co; Gs += co; prec_slot += co;
    err = reinterpret_cast<int*>(reinterpret_cast<double*>(err) + co);
  }
  double m = 0.0, bad = 0.0;
  for (size_t e0 = (size_t)blockIdx.x * 256 * kPrecPer + threadIdx.x; e0 < count;
       e0 += (size_t)gridDim.x * 256 * kPrecPer) {
    double gs[kPrecPer], gw[kPrecPer];
#pragma unroll
    for (int u = 0; u < kPrecPer; ++u) {
      const size_t e = e0 + 256 * (size_t)u;
      gs[u] = e < count ? Gs[e] : 0.0;
      gw[u] = e < count ? Gw[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kPrecPer; ++u) {
      const size_t e = e0 + 256 * (size_t)u;
      m = fmax(m, fabs(gw[u] - gs[u]));
      if (!isfinite(gs[u])) bad = 1.0;
      if (e < count) G[e] = gs[u];
    }
  }
  m = block_max<256>(m, red);
  bad = block_max<256>(bad, red);
  if (threadIdx.x == 0) {
    atomic_max_nonneg(prec_slot, m);
    if (bad > 0.0) atomicOr(err, 1);
  }
}

// End of a sweep: fold the per-stabilisation precision values into the
// running totals, check the threshold, advance the sweep counter.
__global__ void k_finish_sweep(double* prec_hist, int n_hist, double* prec_tot, double threshold,
                               unsigned long long* counters, int* err, size_t cs) {
  if (threadIdx.x != 0) return;
  {
    const size_t co = (size_t)blockIdx.y * cs;
    prec_hist += co; prec_tot += co;
    counters = reinterpret_cast<unsigned long long*>(reinterpret_cast<double*>(counters) + co);
    err = reinterpret_cast<int*>(reinterpret_cast<double*>(err) + co);
  }
  double s = prec_tot[0], mx = prec_tot[1], cnt = prec_tot[2];
  for (int k = 0; k < n_hist; ++k) {
    const double p = prec_hist[k];
    s += p;
    mx = fmax(mx, p);
    cnt += 1.0;
    if (!(p == p)) atomicOr(err, 1);
    if (threshold > 0.0 && p > threshold) atomicOr(err, 8);
    prec_hist[k] = 0.0;
  }
  prec_tot[0] = s;
  prec_tot[1] = mx;
  prec_tot[2] = cnt;
  counters[2] += 1ull;
}

// Random start of the field (s = +1 iff u < 1/2; eta(l) of index floor(4 u)
// for the four-valued field; or phi ~ N(0,1) by Box-Muller on (1 - u0, u1),
// cosine branch); draws (INIT, 0, tau << 1, site).
__global__ void k_random_field(double* field, int L, int N, const unsigned long long* counters, int kind, Field4 f4,
                               size_t cs) {
  field += (size_t)blockIdx.y * cs;
  counters = reinterpret_cast<const unsigned long long*>(reinterpret_cast<const double*>(counters) +
                                                         (size_t)blockIdx.y * cs);
  const unsigned long long seed = counters[3];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= L * N) return;
  const int tau = e / N + 1, i = e % N;
  const Philox4 w = philox4x64_10(TAG_INIT, 0ull, (unsigned long long)tau << 1, (unsigned long long)i, seed, 0ull);
  const double u0 = unit_double(w.w[0]);
  if (kind == FK_ISING) {
    field[e] = (u0 < 0.5) ? 1.0 : -1.0;
  } else if (kind == FK_ISING4) {
    field[e] = field4_pick(f4.eta, min((int)(4.0 * u0), 3));
  } else {
    const double u1 = unit_double(w.w[1]);
    field[e] = sqrt(-2.0 * log(1.0 - u0)) * cos(2.0 * M_PI * u1);
  }
}
