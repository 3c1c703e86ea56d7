// The complex (imaginary-coupling) formulation of the SU(2) Hubbard model
// (section "The SU(2)-Hubbard model on a square lattice": the four-valued field
// of Eq. (HS_squares) at lambda = -U/2 couples to the density with the
// imaginary coupling i c, c = sqrt(dtau U / 2); Eq. (partition_2); the phase
// of Eq. (phase)).
//
// Complex n x n matrices X = X_r + i X_i are carried as their real 2n x 2n
// images [[X_r, -X_i], [X_i, X_r]], which multiply, add and invert like the
// complex matrices.  So the wraps, the QR/UDV stabilisation, the merge and its
// LU solve run unchanged on the FP64 MFMA kernels at dimension 2n; the
// hopping exponential is the block-diagonal image of exp(-dtau T), and
// diag(exp(i c eta)) is a rotation of every pair (row i, row i + n) that these
// kernels apply.  The flips need the complex G itself: one workgroup per
// chain holds it in LDS for the whole slice.
//
// A flip of site i from eta to eta' (the fast formula of the real frame with
// complex numbers): Delta = exp(i c (eta' - eta)) - 1, r = 1 + Delta (1 - G_ii),
// R = gamma(l') / gamma(l) exp(N_col i c alpha (eta' - eta)) r^N_col, accepted
// iff u < |R| (the chain samples |W|), then G <- G - (Delta / r) G[:,i] (e_i - G[i,:])
// and the configuration's phase W / |W| is multiplied by R / |R|.
#pragma once
#include "device_common.h"
#include "update.h"

// dst <- rotations of src (may be the same buffer), for a 2n x 2n image with
// leading dimension ld: with theta_i = coef * eta_i and
// rot(x, y) = (cos theta x - sin theta y, sin theta x + cos theta y),
// rows (i, i + n) by rot with coef_row when rows != 0, then columns
// (j, j + n) by rot with coef_col when cols != 0.  Rows by rot(+c eta) is
// diag(exp(i c eta)) X; columns by rot(+c eta) is X diag(exp(-i c eta)).
// One thread per 2 x 2 block (i, j), i, j < n; grid (ceil(n^2 / 256), chains).
__global__ __launch_bounds__(256) void k_crot(double* dst, const double* src, int n, int ld, const double* eta,
                                              double coef_row, double coef_col, int rows, int cols, size_t cs) {
  dst += (size_t)blockIdx.y * cs;
  src += (size_t)blockIdx.y * cs;
  eta += (size_t)blockIdx.y * cs;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  const int i = e / n, j = e % n;
  double a = src[(size_t)i * ld + j], b = src[(size_t)i * ld + j + n];
  double p = src[(size_t)(i + n) * ld + j], q = src[(size_t)(i + n) * ld + j + n];
  if (rows) {
    double s, c;
    sincos(coef_row * eta[i], &s, &c);
    const double a2 = c * a - s * p, p2 = s * a + c * p;
    const double b2 = c * b - s * q, q2 = s * b + c * q;
    a = a2; p = p2; b = b2; q = q2;
  }
  if (cols) {
    double s, c;
    sincos(coef_col * eta[j], &s, &c);
    const double a2 = c * a - s * b, b2 = s * a + c * b;
    const double p2 = c * p - s * q, q2 = s * p + c * q;
    a = a2; b = b2; p = p2; q = q2;
  }
  dst[(size_t)i * ld + j] = a;
  dst[(size_t)i * ld + j + n] = b;
  dst[(size_t)(i + n) * ld + j] = p;
  dst[(size_t)(i + n) * ld + j + n] = q;
}

constexpr int kCMaxN = 64;   // sites per chain of the complex flips (G in LDS)

// dynamic LDS of k_cupdate_slice: the real and imaginary parts of G, rows of n + 1
__host__ __device__ inline size_t cupdate_lds(int n) { return sizeof(double) * 2 * (size_t)n * (n + 1); }

// The sequential flips of one slice, one workgroup per chain, the complex G
// (n <= kCMaxN) in LDS: loaded from the image G (ld 2n), updated in place,
// written back as the image.  eta: the slice's field row (updated in place);
// draws from Philox counter (TAG_FLIP, sweep, (tau << 1) | dir, site) as in the
// real frame.  phase: [re, im, max |phase - 1|] of the chain, carried along.
__global__ __launch_bounds__(256) void k_cupdate_slice(double* G, int n, double* eta, int tau, unsigned long long dir,
                                                       double coupling, double alpha, int n_col, Field4 f4,
                                                       unsigned long long* counters, double* phase, size_t cs) {
  extern __shared__ double csm[];
  const int P = n + 1;
  double* Gr = csm;                  // Re G[a][b] at Gr[a * P + b]
  double* Gi = csm + (size_t)n * P;  // Im G
  __shared__ double cr[kCMaxN], ci[kCMaxN], rr[kCMaxN], ri[kCMaxN];   // column i and (e_i - row i)
  __shared__ double du[kCMaxN], dsn[kCMaxN], ddr[kCMaxN], ddi[kCMaxN], dpr[kCMaxN], dpi[kCMaxN];
  {
    const size_t co = (size_t)blockIdx.y * cs;
    G += co; eta += co; phase += co;
    counters = reinterpret_cast<unsigned long long*>(reinterpret_cast<double*>(counters) + co);
  }
  const int tid = threadIdx.x, ld = 2 * n;
  for (int e = tid; e < n * n; e += 256) {
    const int a = e / n, b = e % n;
    Gr[a * P + b] = G[(size_t)a * ld + b];
    Gi[a * P + b] = G[(size_t)(a + n) * ld + b];
  }
  if (tid < n) {
    // site tid's draw and the constants of its flip (the field row does not
    // change before the site's own decision)
    const Philox4 w = philox4x64_10(TAG_FLIP, counters[2], ((unsigned long long)tau << 1) | dir,
                                    (unsigned long long)tid, counters[3], 0ull);
    const double u0 = unit_double(w.w[0]), u1 = unit_double(w.w[1]);
    const double s = eta[tid];
    const int k = field4_index(f4, s);
    const int j = min((int)(3.0 * u1), 2);
    const int kn = (j < k) ? j : j + 1;
    const double sn = field4_pick(f4.eta, kn);
    double sd, cd, sp, cp;
    sincos(coupling * (sn - s), &sd, &cd);
    sincos(n_col * coupling * alpha * (sn - s), &sp, &cp);
    const double mag = exp(field4_pick(f4.lg, kn) - field4_pick(f4.lg, k));
    du[tid] = u0; dsn[tid] = sn;
    ddr[tid] = cd - 1.0; ddi[tid] = sd;
    dpr[tid] = mag * cp; dpi[tid] = mag * sp;
  }
  __syncthreads();
  double phr = phase[0], phi = phase[1], pdev = phase[2];
  int nacc = 0;
  for (int i = 0; i < n; ++i) {
    // r = 1 + Delta (1 - G_ii), R = prefactor r^n_col (the same in every thread)
    const double omr = 1.0 - Gr[i * P + i], omi = -Gi[i * P + i];
    const double dr = ddr[i], di = ddi[i];
    const double r_r = 1.0 + (dr * omr - di * omi), r_i = dr * omi + di * omr;
    double pr = r_r, pi = r_i;
    if (n_col == 2) { pr = r_r * r_r - r_i * r_i; pi = 2.0 * r_r * r_i; }
    const double Rr = dpr[i] * pr - dpi[i] * pi, Ri = dpr[i] * pi + dpi[i] * pr;
    const double absR = hypot(Rr, Ri);
    if (du[i] < absR) {   // uniform
      ++nacc;
      // gamma = Delta / r
      const double den = r_r * r_r + r_i * r_i;
      const double gr = (dr * r_r + di * r_i) / den, gi = (di * r_r - dr * r_i) / den;
      if (tid < n) {
        cr[tid] = Gr[tid * P + i]; ci[tid] = Gi[tid * P + i];
        rr[tid] = (tid == i ? 1.0 : 0.0) - Gr[i * P + tid]; ri[tid] = -Gi[i * P + tid];
      }
      __syncthreads();
      for (int e = tid; e < n * n; e += 256) {
        const int a = e / n, b = e % n;
        // gamma * col_a * row_b
        const double xr = gr * cr[a] - gi * ci[a], xi = gr * ci[a] + gi * cr[a];
        Gr[a * P + b] -= xr * rr[b] - xi * ri[b];
        Gi[a * P + b] -= xr * ri[b] + xi * rr[b];
      }
      __syncthreads();
      if (tid == i) eta[i] = dsn[i];
      const double qr = Rr / absR, qi = Ri / absR;
      const double nr = phr * qr - phi * qi, ni = phr * qi + phi * qr;
      phr = nr; phi = ni;
      pdev = fmax(pdev, hypot(phr - 1.0, phi));
    }
  }
  for (int e = tid; e < n * n; e += 256) {
    const int a = e / n, b = e % n;
    G[(size_t)a * ld + b] = Gr[a * P + b];
    G[(size_t)a * ld + b + n] = -Gi[a * P + b];
    G[(size_t)(a + n) * ld + b] = Gi[a * P + b];
    G[(size_t)(a + n) * ld + b + n] = Gr[a * P + b];
  }
  if (tid == 0) {
    phase[0] = phr; phase[1] = phi; phase[2] = pdev;
    counters[0] += (unsigned long long)n;
    counters[1] += (unsigned long long)nacc;
  }
}

// Equal-time estimators of the complex chain (original frame, per colour
// n_i = 1 - G~_ii, both colours the same G), real parts:
//   D = (1/n) sum_i (1 - G~_ii)^2,  E_kin = (n_col / n)(Tr T - Re Tr(T G)),  E_pot = U D,
// G~ = G (asymmetric split) or, with T1 the image of exp(-dtau T/2) G, the
// diagonal of T1 exp(+dtau T/2) (symmetric split; Ehinv symmetric, so row i
// of both).  K is the image of T (ld 2n, T in its upper-left block).  One
// workgroup per chain.
__global__ __launch_bounds__(256) void k_cmeasure(const double* G, const double* T1, const double* Ehinv,
                                                  const double* K, int n, int sym, double trK, double n_col,
                                                  double u_int, double* bins, int* err, size_t cs) {
  __shared__ double red[8];
  {
    const size_t co = (size_t)blockIdx.y * cs;
    G += co; bins += co;
    if (sym) T1 += co;
    err = reinterpret_cast<int*>(reinterpret_cast<double*>(err) + co);
  }
  const int tid = threadIdx.x, ld = 2 * n;
  double dsum = 0.0, bad = 0.0;
  for (int i = tid; i < n; i += 256) {
    double gr = G[(size_t)i * ld + i], gi = G[(size_t)(i + n) * ld + i];
    if (sym) {
      gr = 0.0; gi = 0.0;
      for (int b = 0; b < ld; ++b) {
        gr = fma(T1[(size_t)i * ld + b], Ehinv[(size_t)i * ld + b], gr);
        gi = fma(T1[(size_t)(i + n) * ld + b], Ehinv[(size_t)i * ld + b], gi);
      }
    }
    const double xr = 1.0 - gr, xi = -gi;
    dsum += xr * xr - xi * xi;
    if (!isfinite(gr) || !isfinite(gi)) bad = 1.0;
  }
  double kg = 0.0;
  for (int e = tid; e < n * n; e += 256) {
    const int a = e / n, b = e % n;
    kg = fma(K[(size_t)a * ld + b], G[(size_t)a * ld + b], kg);   // Re Tr(T G) = sum T_ab Re G_ab (T symmetric)
  }
  dsum = block_sum<256>(dsum, red);
  kg = block_sum<256>(kg, red);
  bad = block_max<256>(bad, red);
  if (tid == 0) {
    const double D = dsum / n;
    bins[0] += D;
    bins[1] += n_col / n * (trK - kg);
    bins[2] += u_int * D;
    bins[3] += 1.0;
    if (bad > 0.0) atomicOr(err, 1);
  }
}
