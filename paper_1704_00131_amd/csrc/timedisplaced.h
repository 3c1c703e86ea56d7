// Time-displaced Green's functions and the S^z-S^z correlation at one
// momentum (section "Measuring time displaced observables"; Eq. (s_corr)).
//
// Propagation between checkpoints, with B_tau = diag(v_tau) E:
//   GT0(tau) = B_tau GT0(tau-1),
//   H(tau)   = G0T(tau)^T = B_tau^-T H(tau-1) = diag(1/v_tau) E^-1 H(tau-1),
// so both are left products on the MFMA GEMM and H keeps G0T transposed,
// which makes the estimator below a coalesced elementwise product.
//
// Estimator per configuration (two sampling-frame colours; S^z maps to
// (n_1 + n_2 - 1)/2 under the partial particle-hole map):
//   4 <S^z_x(tau) S^z_y(0)> = (1 - 2 GTT_xx)(1 - 2 G00_yy) - 2 G0T_yx GT0_xy,
//   S_ab(K,tau) = (1/N_cells) sum_{x in a, y in b} p_x conj(p_y) <S^z_x(tau) S^z_y(0)>,
// p_x = exp(-i K.R_x).  With A_a(tau) = sum_{x in a} p_x (1 - 2 GTT_xx) and
// C_ab = sum_{x in a, y in b} p_x conj(p_y) H_xy GT0_xy:
//   S_ab = (0.25 A_a(tau) conj(A_b(0)) - 0.5 C_ab) / N_cells.
#pragma once
#include "device_common.h"

constexpr int kTdMaxOrb = 4;          // orbitals per unit cell
constexpr int kTdRows = 4;            // rows of the product per workgroup
constexpr int kTdSmallN = 128;        // up to this n one workgroup takes all rows
constexpr int kTdPart = 2 * kTdMaxOrb * kTdMaxOrb + 2 * kTdMaxOrb;   // doubles per partial record
constexpr int kTdStride = 2 * kTdMaxOrb * kTdMaxOrb;                 // doubles per tau of S

// GT0 = G, H = G^T - 1 (tau = 0); 32 x 32 tiles through LDS, grid (t, t, chains).
__global__ __launch_bounds__(256) void k_td_init(const double* G, double* GT0, double* H, int n, size_t cs) {
  __shared__ double tile[32][33];
  const size_t co = (size_t)blockIdx.z * cs;
  G += co; GT0 += co; H += co;
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int i = by + r, j = bx + tx;
    double v = 0.0;
    if (i < n && j < n) {
      v = G[(size_t)i * n + j];
      GT0[(size_t)i * n + j] = v;
    }
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = bx + r, j = by + tx;   // H[i][j] = G[j][i] - delta_ij
    if (i < n && j < n) H[(size_t)i * n + j] = tile[tx][r] - (i == j ? 1.0 : 0.0);
  }
}

// Right-hand sides of the re-anchoring solve, n x 2n with leading dimension ld:
//   [ D_b^-1 Q^T | D_s T ],  D_b = max(D, 1), D_s = min(D, 1).
// Grid (t, t, chains); cs_src = 0 when the right form is the shared identity.
__global__ __launch_bounds__(256) void k_td_rhs(double* R2, int ld_r, const double* Q, const double* T,
                                                const double* D, int n, size_t cs_dst, size_t cs_src) {
  __shared__ double tile[32][33];
  R2 += (size_t)blockIdx.z * cs_dst;
  Q += (size_t)blockIdx.z * cs_src;
  T += (size_t)blockIdx.z * cs_src;
  D += (size_t)blockIdx.z * cs_src;
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const size_t ld = (size_t)ld_r;
  for (int r = ty; r < 32; r += 8) {
    const int i = by + r, j = bx + tx;
    tile[r][tx] = (i < n && j < n) ? Q[(size_t)i * n + j] : 0.0;
    if (i < n && j < n) R2[(size_t)i * ld + n + j] = fmin(D[i], 1.0) * T[(size_t)i * n + j];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = bx + r, j = by + tx;   // left half [i][j] = Q[j][i] / D_b[i]
    if (i < n && j < n) R2[(size_t)i * ld + j] = tile[tx][r] / fmax(D[i], 1.0);
  }
}

// S_ab(K, tau) in one launch: every workgroup sums C_ab and A_a over its
// `rows` rows (wave w every fourth, its lanes the columns) and stores its
// partial record; the workgroup that finishes last (a device-scope counter
// after the records, taken behind a release fence by the writing wave and
// reset by that workgroup) adds the records in a fixed order and forms
// S_ab(K, tau): out[0 .. kTdStride) (entry (a * kTdMaxOrb + b) * 2 +
// {re, im}), also added to bins.  With one workgroup per chain (rows = n)
// there is no record exchange.  At tau = 0 it first stores A_a(0) in a00
// (and counts one pass in *count).  Grid (ceil(n / rows), chains), 256
// threads.  phase: [n][2] (re, im) of exp(-i K.R_x); orb: [n] orbital of each
// site (< norb <= kTdMaxOrb); part: the records, then the counter.
__global__ __launch_bounds__(256) void k_td_measure(const double* GT0, const double* H, const double* GTT,
                                                    const double* phase, const int* orb, int n, int rows,
                                                    double* part, double inv_cells, double* a00, double* out,
                                                    double* bins, double* count, int first, size_t cs) {
  constexpr int kGroups = 256 / kTdPart;   // threads per record entry in the final sum
  __shared__ double red[4][kTdPart];
  __shared__ double gsum[kGroups][kTdPart];
  __shared__ double tot[kTdPart];
  __shared__ int last_s;
  {
    const size_t co = (size_t)blockIdx.y * cs;
    GT0 += co; H += co; GTT += co; part += co; a00 += co; out += co; bins += co; count += co;
  }
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nblk = gridDim.x;
  double acc[kTdPart];
#pragma unroll
  for (int k = 0; k < kTdPart; ++k) acc[k] = 0.0;
  // wave w takes rows x0 + w, x0 + w + 4, ... of the workgroup's rows, its
  // lanes the columns y = lane, lane + 64, ...
  const int x0 = blockIdx.x * rows, x1 = min(n, x0 + rows);
  for (int x = x0 + w; x < x1; x += 4) {
    // row sum over y of conj(p_y) H_xy GT0_xy, split by the orbital of y
    double rr[kTdMaxOrb], ri[kTdMaxOrb];
#pragma unroll
    for (int b = 0; b < kTdMaxOrb; ++b) { rr[b] = 0.0; ri[b] = 0.0; }
    const double* hx = H + (size_t)x * n;
    const double* gx = GT0 + (size_t)x * n;
    for (int y = lane; y < n; y += 64) {
      const double p = hx[y] * gx[y];
      const double cr = phase[2 * y], ci = -phase[2 * y + 1];
      const int ob = orb[y];
#pragma unroll
      for (int b = 0; b < kTdMaxOrb; ++b) {
        const double m = (ob == b) ? p : 0.0;
        rr[b] += m * cr;
        ri[b] += m * ci;
      }
    }
    const double pr = phase[2 * x], pi = phase[2 * x + 1];
    const int oa = orb[x];
#pragma unroll
    for (int a = 0; a < kTdMaxOrb; ++a) {
      const double s = (oa == a) ? 1.0 : 0.0;
#pragma unroll
      for (int b = 0; b < kTdMaxOrb; ++b) {
        acc[2 * (a * kTdMaxOrb + b)] += s * (pr * rr[b] - pi * ri[b]);
        acc[2 * (a * kTdMaxOrb + b) + 1] += s * (pr * ri[b] + pi * rr[b]);
      }
    }
    if (lane == 0) {
      const double d = 1.0 - 2.0 * GTT[(size_t)x * n + x];
#pragma unroll
      for (int a = 0; a < kTdMaxOrb; ++a) {
        const double s = (oa == a) ? d : 0.0;
        acc[2 * kTdMaxOrb * kTdMaxOrb + 2 * a] += s * pr;
        acc[2 * kTdMaxOrb * kTdMaxOrb + 2 * a + 1] += s * pi;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kTdPart; ++k) {
    double v = acc[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) red[w][k] = v;
  }
  __syncthreads();
  unsigned int* counter = reinterpret_cast<unsigned int*>(part + (size_t)nblk * kTdPart);
  if (nblk == 1) {
    if (tid < kTdPart) tot[tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
    __syncthreads();
  } else {
    if (tid < kTdPart) part[(size_t)blockIdx.x * kTdPart + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
    // the record's writers (wave 0) release it, then one lane counts; the
    // device-scope fences stay on one wave per workgroup
    if (w == 0) {
      __threadfence();
      if (lane == 0) last_s = (atomicAdd(counter, 1u) == (unsigned)nblk - 1u);
    }
    __syncthreads();
    if (!last_s) return;
    __threadfence();
    // the records in a fixed order: group g adds records g, g + kGroups, ...,
    // four loads in flight (four partial sums, combined in a fixed order)
    if (tid < kGroups * kTdPart) {
      const int k = tid % kTdPart, g = tid / kTdPart;
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
      int b = g;
      for (; b + 3 * kGroups < nblk; b += 4 * kGroups) {
        double v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = __builtin_nontemporal_load(part + (size_t)(b + q * kGroups) * kTdPart + k);
#pragma unroll
        for (int q = 0; q < 4; ++q) s4[q] += v[q];
      }
      for (; b < nblk; b += kGroups) s4[0] += __builtin_nontemporal_load(part + (size_t)b * kTdPart + k);
      gsum[g][k] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    }
    __syncthreads();
    if (tid < kTdPart) {
      double sg = 0.0;
#pragma unroll
      for (int g = 0; g < kGroups; ++g) sg += gsum[g][tid];
      tot[tid] = sg;
    }
    __syncthreads();
  }
  const double* A = tot + 2 * kTdMaxOrb * kTdMaxOrb;
  if (first && tid < 2 * kTdMaxOrb) a00[tid] = A[tid];
  if (first && tid == 0) count[0] += 1.0;
  const double* A0 = first ? A : a00;   // a00 of an earlier launch when tau > 0
  if (tid < kTdMaxOrb * kTdMaxOrb) {
    const int a = tid / kTdMaxOrb, b = tid % kTdMaxOrb;
    const double ar = A[2 * a], ai = A[2 * a + 1];
    const double br = A0[2 * b], bi = -A0[2 * b + 1];   // conj(A_b(0))
    const double dr = ar * br - ai * bi, di = ar * bi + ai * br;
    const double sr = (0.25 * dr - 0.5 * tot[2 * tid]) * inv_cells;
    const double si = (0.25 * di - 0.5 * tot[2 * tid + 1]) * inv_cells;
    out[2 * tid] = sr;
    out[2 * tid + 1] = si;
    bins[2 * tid] += sr;
    bins[2 * tid + 1] += si;
  }
  if (tid == 0 && nblk > 1) *counter = 0u;   // ready for the next tau (kernel boundaries order it)
}
