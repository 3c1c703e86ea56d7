// Lattice-resolved correlation functions: equal-time and time-displaced bins
// by displacement and orbital pair.
#pragma once
#include "device_common.h"

// Lattice-resolved correlations (section "Observables": correlation functions
// summed over unit cells and stored by the displacement R between them),
// accumulated per measurement:
//   bins[o][R][a][b] += 1/N_cells sum_I <O_i(tau) O_j(0)>,  i = site(I, a), j = site(I + R, b),
// o = Green, SpinZ, SpinXY, Den.  Both particle-hole species carry the same
// Green's functions and s is the sublattice sign of the down-spin map; with
// h = G0T_ji = H_ij (H = G0T^T) and g = GT0_ij, Wick's theorem gives
//   Green  = 1/2 (-h + s_i s_j g)
//   SpinZ  = 1/4 ((1 - 2 GTT_ii)(1 - 2 G00_jj) - 2 h g)
//   SpinXY = 1/4 s_i s_j (h^2 + g^2)      (half of S^x S^x + S^y S^y)
//   Den    = 1 - 2 h g.
// Equal time (TD = false, A = the measured G~): GT0 = G~, G0T = G~ - 1, so
// g = G~_ij, h = G~_ji - d_ij and GTT_ii = G00_jj are diagonal entries of G~.
// Time-displaced (TD = true): A = GT0(tau), H, GTT(tau) and g00 the diagonal
// of G00, all N x N row-major except g00.
// One wavefront per (R, a, b): its lanes take the cells I = lane, lane + 64, ...
// and a butterfly reduction sums them (four waves per workgroup, so N_cells
// norb^2 / 4 workgroups); the wave past the last entry adds 1 to *count when
// count is non-null and, for equal time, the per-orbital <S^z> to
// bins[4 nb + 1 + a].  site[I * norb + a] is the orbital index of orbital a of
// cell I (a permutation of 0..N-1, checked on the host); cells are I = i1 + L1 i2.
template <bool TD>
__global__ __launch_bounds__(256) void k_corr(const double* A, const double* H, const double* GTT, const double* g00,
                                              int N, int L1, int L2, int norb, const int* site, const double* sgn,
                                              double* bins, double* count, size_t cs) {
  {
    const size_t co = (size_t)blockIdx.y * cs;
    A += co;
    bins += co;
    if (count) count += co;
    if (TD) { H += co; GTT += co; g00 += co; }
  }
  const int nc = L1 * L2, nb = nc * norb * norb;
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e > nb) return;
  if (e == nb) {
    if (!TD) {
      // one-point function: bins[4 nb + 1 + a] += 1/N_cells sum_I <S^z_{site(I, a)}>,
      // <S^z_i> = 1/2 (1 - 2 G~_ii) (n_up = n_1, n_dn = 1 - n_2)
      for (int oa = 0; oa < norb; ++oa) {
        double m = 0.0;
        for (int I = lane; I < nc; I += 64) {
          const int i = site[I * norb + oa];
          m += 0.5 * (1.0 - 2.0 * A[(size_t)i * N + i]);
        }
        for (int off = 32; off > 0; off >>= 1) m += __shfl_xor(m, off, 64);
        if (lane == 0) bins[4 * (size_t)nb + 1 + oa] += m / nc;
      }
    }
    if (lane == 0 && count) *count += 1.0;
    return;
  }
  const int R = e / (norb * norb), a = (e / norb) % norb, b = e % norb;
  const int r1 = R % L1, r2 = R / L1;
  double gr = 0.0, z = 0.0, xy = 0.0, dn = 0.0;
  for (int I = lane; I < nc; I += 64) {
    const int i1 = I % L1, i2 = I / L1;
    const int J = (i1 + r1) % L1 + L1 * ((i2 + r2) % L2);
    const int i = site[I * norb + a], j = site[J * norb + b];
    const double g = A[(size_t)i * N + j];
    double h, gtt, gzz;
    if (TD) {
      h = H[(size_t)i * N + j];
      gtt = GTT[(size_t)i * N + i];
      gzz = g00[j];
    } else {
      h = A[(size_t)j * N + i] - ((i == j) ? 1.0 : 0.0);
      gtt = A[(size_t)i * N + i];
      gzz = A[(size_t)j * N + j];
    }
    const double ss = sgn[i] * sgn[j];
    gr += 0.5 * (ss * g - h);
    z += 0.25 * ((1.0 - 2.0 * gtt) * (1.0 - 2.0 * gzz) - 2.0 * h * g);
    xy += 0.25 * ss * (h * h + g * g);
    dn += 1.0 - 2.0 * h * g;
  }
  for (int off = 32; off > 0; off >>= 1) {
    gr += __shfl_xor(gr, off, 64);
    z += __shfl_xor(z, off, 64);
    xy += __shfl_xor(xy, off, 64);
    dn += __shfl_xor(dn, off, 64);
  }
  if (lane == 0) {
    bins[e] += gr / nc;
    bins[(size_t)nb + e] += z / nc;
    bins[2 * (size_t)nb + e] += xy / nc;
    bins[3 * (size_t)nb + e] += dn / nc;
  }
}

// Diagonal of a per-chain N x N matrix into a vector.
__global__ __launch_bounds__(256) void k_diag(const double* M, int N, double* d, size_t cs) {
  const size_t co = (size_t)blockIdx.y * cs;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) d[co + i] = M[co + (size_t)i * N + i];
}
