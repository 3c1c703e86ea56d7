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
  const unsigned long long* sweep_ctr;   // unused: the counters carry the sweep number and the key
  unsigned long long seed, slot;     // slot = counter word 2 = (tau << 1) | dir
  double coupling, alpha; int n_col; int gauss; double prop_width;
  unsigned long long* counters;      // [0] proposals, [1] accepted, [2] sweep, [3] Philox key
  size_t cs;                         // per-chain stride (doubles) of every pointer above; chain = blockIdx.y
};

__device__ __forceinline__ double ipow(double r, int n) {
  double p = 1.0;
  for (int k = 0; k < n; ++k) p *= r;
  return p;
}

// One workgroup per 32 x 32 tile (I, J) of G.  Every workgroup runs the same
// sequential decisions of block S on G[S,S] (identical arithmetic, identical
// results), then writes
//   Gout[I,J] = Gin[I,J] - Gin[I,S] Phi (E_S^T[:,J] - Gin[S,J]).
// Workgroup 0 also writes the block's field values and the counters.
__global__ __launch_bounds__(256) void k_block_update(BlockArgs a) {
  __shared__ double g[32][33], c[32][33], Ph[32][33], GIS[32][33], GSJ[32][33], Wt[32][33];
  __shared__ double dlt[32], pre[32], snew[32], sold[32], uu[32], av[32], bv[32], colj[32], rowj[32];
  __shared__ int accf[32];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int bb = a.bb, s0 = a.s0, N = a.N;
  const int tilesN = (N + 31) >> 5;
  if (a.cs) {
    const size_t co = (size_t)blockIdx.y * a.cs;
    a.Gin += co; a.Gout += co; a.field_in += co; a.field_out += co;
    a.sweep_ctr = reinterpret_cast<const unsigned long long*>(reinterpret_cast<const double*>(a.sweep_ctr) + co);
    a.counters = reinterpret_cast<unsigned long long*>(reinterpret_cast<double*>(a.counters) + co);
  }
  const int I0 = (blockIdx.x / tilesN) << 5, J0 = (blockIdx.x % tilesN) << 5;
  for (int e = tid; e < 1024; e += 256) {
    const int x = e >> 5, y = e & 31;
    const double v = (x < bb && y < bb) ? a.Gin[(size_t)(s0 + x) * N + s0 + y] : 0.0;
    g[x][y] = v;
    c[x][y] = v;
    Ph[x][y] = 0.0;
    GIS[x][y] = (I0 + x < N && y < bb) ? a.Gin[(size_t)(I0 + x) * N + s0 + y] : 0.0;
    GSJ[x][y] = (x < bb && J0 + y < N) ? a.Gin[(size_t)(s0 + x) * N + J0 + y] : 0.0;
  }
  if (tid < 32) {
    accf[tid] = 0;
    if (tid < bb) {
      const Philox4 r = philox4x64_10(TAG_FLIP, a.counters[2], a.slot, (unsigned long long)(s0 + tid), a.counters[3],
                                      0ull);
      const double u0 = unit_double(r.w[0]), u1 = unit_double(r.w[1]);
      const double s = a.field_in[s0 + tid];
      double sn, extra;
      if (a.gauss) { sn = s + a.prop_width * (2.0 * u1 - 1.0); extra = -0.5 * (sn * sn - s * s); }
      else { sn = -s; extra = 0.0; }
      uu[tid] = u0;
      sold[tid] = s;
      snew[tid] = sn;
      dlt[tid] = exp(a.coupling * (sn - s)) - 1.0;
      pre[tid] = exp(a.n_col * a.coupling * a.alpha * (sn - s) + extra);
    }
  }
  __syncthreads();
  int nacc = 0;
  for (int j = 0; j < bb; ++j) {
    const double r = 1.0 + dlt[j] * (1.0 - c[j][j]);
    const double R = pre[j] * ipow(r, a.n_col);
    if (!(uu[j] < R)) continue;          // uniform across the workgroup
    const double gam = dlt[j] / r;
    {
      // a = e_j - Phi (e_j - g[:,j]),  b = e_j + Phi^T g[j,:]^T: thread (x, q)
      // sums 4 of the 32 terms, 8 threads per x reduce by shuffles
      const int x = tid >> 3, q = tid & 7;
      double pa = 0.0, pb = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int y = 4 * q + k;
        pa += Ph[x][y] * ((y == j ? 1.0 : 0.0) - g[y][j]);
        pb += Ph[y][x] * g[j][y];
      }
      pa += __shfl_xor(pa, 1, 64); pb += __shfl_xor(pb, 1, 64);
      pa += __shfl_xor(pa, 2, 64); pb += __shfl_xor(pb, 2, 64);
      pa += __shfl_xor(pa, 4, 64); pb += __shfl_xor(pb, 4, 64);
      if (q == 0) {
        av[x] = (x == j ? 1.0 : 0.0) - pa;
        bv[x] = (x == j ? 1.0 : 0.0) + pb;
        colj[x] = c[x][j];
        rowj[x] = (x == j ? 1.0 : 0.0) - c[j][x];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = tid + 256 * k;
      const int x = e >> 5, y = e & 31;
      Ph[x][y] += gam * av[x] * bv[y];
      c[x][y] -= gam * colj[x] * rowj[y];
    }
    if (tid == 0) accf[j] = 1;
    ++nacc;
    __syncthreads();
  }
  // W tile = Phi (E_S^T[:, J] - G[S, J])  (32 x 32 x 32 on MFMA)
  const int wr = w >> 1, wc = w & 1;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < 32; k0 += 4) {
    const int z = k0 + (lane >> 4), y = wc * 16 + (lane & 15);
    const double av_ = Ph[wr * 16 + (lane & 15)][z];
    const double bz = ((s0 + z == J0 + y) ? 1.0 : 0.0) - GSJ[z][y];
    acc = mfma_f64_16x16x4(av_, bz, acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) Wt[wr * 16 + (lane >> 4) + 4 * r][wc * 16 + (lane & 15)] = acc[r];
  __syncthreads();
  v4d acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < 32; k0 += 4) {
    const double av_ = GIS[wr * 16 + (lane & 15)][k0 + (lane >> 4)];
    const double bw = Wt[k0 + (lane >> 4)][wc * 16 + (lane & 15)];
    acc2 = mfma_f64_16x16x4(av_, bw, acc2);
  }
  const int col = J0 + wc * 16 + (lane & 15);
  if (col < N) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = I0 + wr * 16 + (lane >> 4) + 4 * r;
      if (row < N) a.Gout[(size_t)row * N + col] = a.Gin[(size_t)row * N + col] - acc2[r];
    }
  }
  if (blockIdx.x == 0) {
    if (tid < bb) a.field_out[s0 + tid] = accf[tid] ? snew[tid] : sold[tid];
    if (tid == 0) {
      atomicAdd(&a.counters[0], (unsigned long long)bb);
      atomicAdd(&a.counters[1], (unsigned long long)nacc);
    }
  }
}

// --------------------------------------------------------- measurements ----
// Equal-time estimators per site (section "Observables"): with d_i the
// diagonal of the measured Green's function,
//   D = (1/N) sum_i d_i (1 - d_i),  E_kin = (n_col/N)(Tr K - Tr(K G)),  E_pot = U D.
// For a symmetric split d_i = sum_b T1[i][b] Ehinv[b][i] with
// T1 = exp(-dtau K/2) G (Ehinv is symmetric, so the sum runs along row i of
// both).  K is symmetric, so Tr(K G) = sum_e K[e] G[e].  One workgroup; each
// wave walks rows with coalesced loads.
__global__ __launch_bounds__(1024) void k_measure(const double* G, const double* T1, const double* Ehinv,
                                                  const double* K, int N, double trK, double n_col, double u_int,
                                                  double* bins, int* err, size_t cs) {
  __shared__ double red[16];
  {
    const size_t co = (size_t)blockIdx.y * cs;
    G += co;
    if (T1) T1 += co;
    bins += co;
    err = reinterpret_cast<int*>(reinterpret_cast<double*>(err) + co);
  }
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double sd = 0.0, skg = 0.0, bad = 0.0;
  for (int i = w; i < N; i += 16) {
    double d;
    if (T1) {
      double p = 0.0;
      for (int b = lane; b < N; b += 64) p += T1[(size_t)i * N + b] * Ehinv[(size_t)i * N + b];
      for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o, 64);
      d = p;
    } else {
      d = G[(size_t)i * N + i];
    }
    if (lane == 0) sd += d * (1.0 - d);
  }
  for (size_t e = tid; e < (size_t)N * N; e += 1024) {
    const double gv = G[e];
    skg += K[e] * gv;
    if (!isfinite(gv)) bad = 1.0;
  }
  sd = block_sum<1024>(sd, red);
  skg = block_sum<1024>(skg, red);
  bad = block_sum<1024>(bad, red);
  if (tid == 0) {
    const double D = sd / N;
    bins[0] += D;
    bins[1] += n_col / N * (trK - skg);
    bins[2] += u_int * D;
    bins[3] += 1.0;
    if (bad > 0.0) atomicOr(err, 1);
  }
}

// max |Gw - Gs| into prec_slot (zero on entry), G <- Gs, NaN/Inf check.
__global__ __launch_bounds__(256) void k_prec_replace(const double* Gw, double* G, const double* Gs, size_t count,
                                                      double* prec_slot, int* err, size_t cs) {
  __shared__ double red[8];
  {
    const size_t co = (size_t)blockIdx.y * cs;
    Gw += co; G += co; Gs += co; prec_slot += co;
    err = reinterpret_cast<int*>(reinterpret_cast<double*>(err) + co);
  }
  double m = 0.0, bad = 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (size_t)gridDim.x * 256) {
    const double gs = Gs[e];
    const double d = fabs(Gw[e] - gs);
    m = fmax(m, d);
    if (!isfinite(gs)) bad = 1.0;
    G[e] = gs;
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

// Random start of the field (s = +1 iff u < 1/2, or phi ~ N(0,1) by
// Box-Muller on (1 - u0, u1), cosine branch); draws (INIT, 0, tau << 1, site).
__global__ void k_random_field(double* field, int L, int N, const unsigned long long* counters, int gauss, size_t cs) {
  field += (size_t)blockIdx.y * cs;
  counters = reinterpret_cast<const unsigned long long*>(reinterpret_cast<const double*>(counters) +
                                                         (size_t)blockIdx.y * cs);
  const unsigned long long seed = counters[3];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= L * N) return;
  const int tau = e / N + 1, i = e % N;
  const Philox4 w = philox4x64_10(TAG_INIT, 0ull, (unsigned long long)tau << 1, (unsigned long long)i, seed, 0ull);
  const double u0 = unit_double(w.w[0]);
  if (!gauss) {
    field[e] = (u0 < 0.5) ? 1.0 : -1.0;
  } else {
    const double u1 = unit_double(w.w[1]);
    field[e] = sqrt(-2.0 * log(1.0 - u0)) * cos(2.0 * M_PI * u1);
  }
}
