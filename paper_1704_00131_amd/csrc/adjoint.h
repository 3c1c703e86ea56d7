// Gradient of log det(1 + B(beta,0)) with respect to a continuous HS field and
// the unadjusted Langevin step built on it.
//
// With B_tau = diag(exp(c phi_tau)) exp(-dtau K) (Eq. (partition_2)), the only
// phi_{i,tau} dependence of B(beta,0) is the factor e_i e_i^T of B_tau, so by
// the cyclic trace and Eq. (Green_eq)
//   d log det(1 + B(beta,0)) / d phi_{i,tau} = c (1 - G(tau))_ii,
// i.e. one diagonal per slice of the equal-time Green's functions that the
// upward pass already produces.  The paper's code has no continuous fields
// (section "Definition of the Hamiltonian"; future directions), so this is a
// reading built on those two equations.
#pragma once
#include "device_common.h"

// grad_row[i] = coupling (1 - G_ii); grid (ceil(N/256), chains).
__global__ __launch_bounds__(256) void k_grad_diag(const double* G, int N, double coupling, double* grad_row,
                                                   size_t cs) {
  G += (size_t)blockIdx.y * cs;
  grad_row += (size_t)blockIdx.y * cs;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < N) grad_row[i] = coupling * (1.0 - G[(size_t)i * N + i]);
}

// One Langevin step on the whole field [L][N]:
//   d log W = -phi + n_col c alpha + n_col grad,
//   phi <- phi + eps d log W + sqrt(2 eps) xi,
// xi by Box-Muller (cosine branch) from Philox counter
// (TAG_LANGEVIN, step, tau << 1, site) under the chain's key, where step is
// the chain's Langevin step counter (counters[4]); k_next_langevin_step
// advances it once every workgroup of this launch has read it.
__global__ __launch_bounds__(256) void k_langevin(double* field, const double* grad, int L, int N, double eps,
                                                  double coupling, double alpha, double n_col,
                                                  const unsigned long long* counters, size_t cs) {
  const size_t co = (size_t)blockIdx.y * cs;
  field += co;
  grad += co;
  counters = reinterpret_cast<const unsigned long long*>(reinterpret_cast<const double*>(counters) + co);
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= L * N) return;
  const int tau = e / N + 1, i = e % N;
  const Philox4 w = philox4x64_10(TAG_LANGEVIN, counters[4], (unsigned long long)tau << 1, (unsigned long long)i,
                                  counters[3], 0ull);
  const double u0 = unit_double(w.w[0]), u1 = unit_double(w.w[1]);
  const double xi = sqrt(-2.0 * log1p(-u0)) * cos(2.0 * M_PI * u1);
  const double phi = field[e];
  const double dlw = -phi + n_col * coupling * alpha + n_col * grad[e];
  field[e] = phi + eps * dlw + sqrt(2.0 * eps) * xi;
}

// counters[4] += 1 for every chain (one thread per chain, grid (1, chains)),
// after the step that used it.
__global__ void k_next_langevin_step(unsigned long long* counters, size_t cs) {
  if (threadIdx.x != 0) return;
  counters = reinterpret_cast<unsigned long long*>(reinterpret_cast<double*>(counters) + (size_t)blockIdx.y * cs);
  counters[4] += 1ull;
}
