// The M_z form with two flavours and two Green's functions (section "The
// M_z-Hubbard model on a square lattice": N_fl = 2, one vertex per site coupled
// to n_up - n_dn, alpha = 0, N_col = 1, flavour-dependent hopping).
//
// The two flavours are carried as one 2n x 2n block-diagonal system,
// G = diag(G_up, G_dn), K = diag(K_up, K_dn), with the field of site i acting
// as +s on orbital i and -s on orbital n + i (an expanded field row of 2n
// values), so the wraps, the QR/UDV stabilisation and the merge run unchanged
// on the FP64 MFMA kernels at dimension 2n.  The flips need both flavours'
// blocks: one workgroup per chain holds them in LDS for the whole slice.
//
// A flip of site i from s to s': Delta_up = exp(c (s' - s)) - 1,
// Delta_dn = exp(-c (s' - s)) - 1, r_f = 1 + Delta_f (1 - G_f,ii),
// R = (vertex factor ratio) r_up r_dn, accepted iff u < |R| (the chain samples
// |W|); then each flavour's G_f <- G_f - (Delta_f / r_f) G_f[:,i] (e_i - G_f[i,:]),
// and the configuration's sign (relative to the start) is multiplied by sign(R).
#pragma once
#include "device_common.h"
#include "update.h"

constexpr int kFl2MaxN = 64;   // sites per chain of the two-flavour flips (both blocks in LDS)

// dynamic LDS of k_fl2_update_slice: the two diagonal blocks, rows of n + 1
__host__ __device__ inline size_t fl2_update_lds(int n) { return sizeof(double) * 2 * (size_t)n * (n + 1); }

// field_x[t][i] = field[t][i], field_x[t][n + i] = -field[t][i]; grid
// (ceil(L n / 256), chains).
__global__ __launch_bounds__(256) void k_expand_field(const double* field, double* field_x, int L, int n, size_t cs) {
  field += (size_t)blockIdx.y * cs;
  field_x += (size_t)blockIdx.y * cs;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= L * n) return;
  const int t = e / n, i = e - t * n;
  const double s = field[e];
  field_x[(size_t)t * 2 * n + i] = s;
  field_x[(size_t)t * 2 * n + n + i] = -s;
}

// The sequential flips of one slice, one workgroup per chain: G the 2n x 2n
// block-diagonal image (its diagonal blocks loaded, updated in LDS, written
// back; the off-diagonal blocks are not read and are written as zeros), eta the slice's field row and
// eta_x its expanded row (both updated), draws from Philox counter
// (TAG_FLIP, sweep, (tau << 1) | dir, site) with the proposals of the real
// field kinds.  sign: [sign, 0, 2 once the sign was negative, else 0] of the
// chain, carried along.
__global__ __launch_bounds__(256) void k_fl2_update_slice(double* G, int n, double* eta, double* eta_x, int tau,
                                                          unsigned long long dir, double coupling, int kind,
                                                          double prop_width, Field4 f4,
                                                          unsigned long long* counters, double* sign, size_t cs) {
  extern __shared__ double fsm[];
  const int P = n + 1;
  double* Gu = fsm;                  // G_up[a][b] at Gu[a * P + b]
  double* Gd = fsm + (size_t)n * P;  // G_dn
  __shared__ double cu[kFl2MaxN], cd[kFl2MaxN], ru[kFl2MaxN], rd[kFl2MaxN];   // columns and (e_i - rows)
  __shared__ double du[kFl2MaxN], dsn[kFl2MaxN], ddu[kFl2MaxN], ddd[kFl2MaxN], dpre[kFl2MaxN];
  {
    const size_t co = (size_t)blockIdx.y * cs;
    G += co; eta += co; eta_x += co; sign += co;
    counters = reinterpret_cast<unsigned long long*>(reinterpret_cast<double*>(counters) + co);
  }
  const int tid = threadIdx.x, ld = 2 * n;
  for (int e = tid; e < n * n; e += 256) {
    const int a = e / n, b = e - a * n;
    Gu[a * P + b] = G[(size_t)a * ld + b];
    Gd[a * P + b] = G[(size_t)(a + n) * ld + n + b];
  }
  if (tid < n) {
    const Philox4 w = philox4x64_10(TAG_FLIP, counters[2], ((unsigned long long)tau << 1) | dir,
                                    (unsigned long long)tid, counters[3], 0ull);
    const double u0 = unit_double(w.w[0]), u1 = unit_double(w.w[1]);
    const double s = eta[tid];
    double sn, extra;
    if (kind == FK_GAUSS) { sn = s + prop_width * (2.0 * u1 - 1.0); extra = -0.5 * (sn * sn - s * s); }
    else if (kind == FK_ISING4) {
      const int k = field4_index(f4, s);
      const int j = min((int)(3.0 * u1), 2);
      const int kn = (j < k) ? j : j + 1;
      sn = field4_pick(f4.eta, kn);
      extra = field4_pick(f4.lg, kn) - field4_pick(f4.lg, k);
    } else { sn = -s; extra = 0.0; }
    du[tid] = u0;
    dsn[tid] = sn;
    ddu[tid] = exp(coupling * (sn - s)) - 1.0;
    ddd[tid] = exp(-coupling * (sn - s)) - 1.0;
    dpre[tid] = exp(extra);
  }
  __syncthreads();
  double sg = sign[0], seen = 0.0;
  int nacc = 0;
  for (int i = 0; i < n; ++i) {
    const double r_u = 1.0 + ddu[i] * (1.0 - Gu[i * P + i]);
    const double r_d = 1.0 + ddd[i] * (1.0 - Gd[i * P + i]);
    const double R = dpre[i] * r_u * r_d;
    if (du[i] < fabs(R)) {   // uniform: every thread computes the same R
      ++nacc;
      const double gu = ddu[i] / r_u, gd = ddd[i] / r_d;
      if (tid < n) {
        cu[tid] = Gu[tid * P + i];
        ru[tid] = (tid == i ? 1.0 : 0.0) - Gu[i * P + tid];
        cd[tid] = Gd[tid * P + i];
        rd[tid] = (tid == i ? 1.0 : 0.0) - Gd[i * P + tid];
      }
      __syncthreads();
      for (int e = tid; e < n * n; e += 256) {
        const int a = e / n, b = e - a * n;
        Gu[a * P + b] = fma(-gu * cu[a], ru[b], Gu[a * P + b]);
        Gd[a * P + b] = fma(-gd * cd[a], rd[b], Gd[a * P + b]);
      }
      __syncthreads();
      if (tid == 0) {
        eta[i] = dsn[i];
        eta_x[i] = dsn[i];
        eta_x[n + i] = -dsn[i];
      }
      if (R < 0.0) {
        sg = -sg;
        if (sg < 0.0) seen = 2.0;
      }
    }
  }
  // the off-diagonal blocks, zero in exact arithmetic, are set to zero: the
  // merge leaves rounding there, which the wraps (not similarity transforms
  // between the flavours) would amplify slice by slice
  for (int e = tid; e < n * n; e += 256) {
    const int a = e / n, b = e - a * n;
    G[(size_t)a * ld + b] = Gu[a * P + b];
    G[(size_t)(a + n) * ld + n + b] = Gd[a * P + b];
    G[(size_t)a * ld + n + b] = 0.0;
    G[(size_t)(a + n) * ld + b] = 0.0;
  }
  if (tid == 0) {
    sign[0] = sg;
    sign[2] = fmax(sign[2], seen);
    counters[0] += (unsigned long long)n;
    counters[1] += (unsigned long long)nacc;
  }
}

// Equal-time estimators of the two-flavour chain (original frame,
// n_f,i = 1 - G~_f,ii), weighted by the chain's sign:
//   D = (1/n) sum_i n_up,i n_dn,i,
//   E_kin = (1/n)(Tr K_up + Tr K_dn - Tr(K G)),
//   E_pot = (U/2)(1/n) sum_i (1 - n_up,i - n_dn,i + 2 n_up,i n_dn,i),
// bins += sign (D, E_kin, E_pot, 1).  G~ = G (asymmetric split) or, with T1 the
// image of exp(-dtau K/2) G, the diagonal of T1 exp(+dtau K/2) (symmetric
// split; Ehinv symmetric).  K: the 2n x 2n block-diagonal hopping.  One
// workgroup per chain.
__global__ __launch_bounds__(256) void k_fl2_measure(const double* G, const double* T1, const double* Ehinv,
                                                     const double* K, int n, int sym, double trK, double u_int,
                                                     const double* sign, double* bins, int* err, size_t cs) {
  __shared__ double red[8];
  {
    const size_t co = (size_t)blockIdx.y * cs;
    G += co; bins += co; sign += co;
    if (sym) T1 += co;
    err = reinterpret_cast<int*>(reinterpret_cast<double*>(err) + co);
  }
  const int tid = threadIdx.x, ld = 2 * n;
  double dsum = 0.0, psum = 0.0, bad = 0.0;
  for (int i = tid; i < n; i += 256) {
    double gu = G[(size_t)i * ld + i], gd = G[(size_t)(i + n) * ld + i + n];
    if (sym) {
      gu = 0.0; gd = 0.0;
      for (int b = 0; b < ld; ++b) {
        gu = fma(T1[(size_t)i * ld + b], Ehinv[(size_t)i * ld + b], gu);
        gd = fma(T1[(size_t)(i + n) * ld + b], Ehinv[(size_t)(i + n) * ld + b], gd);
      }
    }
    const double nu = 1.0 - gu, nd = 1.0 - gd;
    dsum += nu * nd;
    psum += 1.0 - nu - nd + 2.0 * nu * nd;
    if (!isfinite(gu) || !isfinite(gd)) bad = 1.0;
  }
  double kg = 0.0;
  for (int e = tid; e < ld * ld; e += 256) kg = fma(K[e], G[e], kg);   // Tr(K G), K symmetric
  dsum = block_sum<256>(dsum, red);
  psum = block_sum<256>(psum, red);
  kg = block_sum<256>(kg, red);
  bad = block_max<256>(bad, red);
  if (tid == 0) {
    const double sg = sign[0];
    bins[0] += sg * dsum / n;
    bins[1] += sg * (trK - kg) / n;
    bins[2] += sg * 0.5 * u_int * psum / n;
    bins[3] += sg;
    if (bad > 0.0) atomicOr(err, 1);
  }
}
