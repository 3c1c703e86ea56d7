// General operator vertices and Ising spins with their own action (section
// "Definition of the Hamiltonian", Eqs. (general_ham_v) and (general_ham_i);
// table "operator"; section "Sampling of e^{-S_{0,I}}").
//
// Vertex k acts on |P_k| <= 2 orbitals: X_k = P^T O_k P, E_k = exp(g_k s X_k)
// = P^T exp(g_k s O_k) P + (1 - P^T P); the slice propagator of the sampling
// frame is B'_tau = E_0 E_1 ... E_{M-1} exp(-dtau K).  A flip of vertex k is
// taken in the frame where E_k is the leftmost factor of B'(tau, 0): in the
// upward pass vertices M-1, ..., 0, each after G <- E_k G E_k^-1 (starting from
// exp(-dtau K) G(tau-1) exp(+dtau K), ending at G(tau)); in the downward pass
// vertices 0, ..., M-1, each followed by G <- E_k^-1 G E_k (starting from
// G(tau)).  With delta = exp(g (s' - s) O) - 1 (|P| x |P|, s' = -s),
//   R_P = 1 + delta (1 - G)_PP,  R = det(R_P)^n_col exp(n_col g alpha (s' - s)) r_S0,
// accepted iff u < R, then G <- G - G[:,P] (R_P^-1 delta) (1 - G)[P,:].  For an
// Ising spin r_S0 = exp(-2 s (Kt (s_{k,tau-1} + s_{k,tau+1}) + dtJ sum s_{k',tau}))
// over the spins k' paired with k (current values), else 1.
#pragma once
#include "device_common.h"

constexpr int kVxMaxN = 64;      // orbitals of a vertex chain (G in one workgroup's LDS)
constexpr int kVxRec = 12;       // doubles per vertex record
constexpr int kVxMaxM = 512;     // vertices of a vertex chain
constexpr int kVxMaxNbr = 2048;  // entries of the Ising partner lists (twice the pairs)
constexpr int kVxPre = 12;       // doubles of per-vertex values computed before a slice's flips
constexpr int kVxInt = 8;        // ints per vertex in LDS: orbitals, kind, partner range, starting sign

// vertex record: [np, p0, p1, ising, g, alpha, o00, o01, o10, o11, first partner, partner count]
// dynamic LDS of k_vx_rows: the n x n matrix (rows of n + 1), the M vertex
// factors and the vertices' orbitals
__host__ __device__ inline size_t vx_rows_lds(int n, int M) {
  return sizeof(double) * ((size_t)n * (n + 1) + 3 * (size_t)M) + sizeof(int) * 3 * (size_t)M;
}
// dynamic LDS of k_vx_slice: G (rows of n + 1), the per-vertex values, the
// slice's field row and the partners' sums, the S0 factors by partner sum,
// the vertices' orbitals and partner ranges, the partner lists
__host__ __device__ inline size_t vx_slice_lds(int n, int M, int nnb) {
  return sizeof(double) * ((size_t)n * (n + 1) + (size_t)(kVxPre + 3) * M + (size_t)nnb) +
         sizeof(int) * ((size_t)kVxInt * M + (size_t)nnb);
}

struct VxRec {
  int np, p0, p1, ising, nb0, nbc;
  double g, alpha, o00, o01, o11;
};

__device__ __forceinline__ VxRec vx_load(const double* tab, int k) {
  const double* r = tab + (size_t)k * kVxRec;
  VxRec v;
  v.np = (int)r[0]; v.p0 = (int)r[1]; v.p1 = (int)r[2]; v.ising = (int)r[3];
  v.g = r[4]; v.alpha = r[5]; v.o00 = r[6]; v.o01 = r[7]; v.o11 = r[9];
  v.nb0 = (int)r[10]; v.nbc = (int)r[11];
  return v;
}

// exp(x O) of a symmetric 2 x 2 O = [[a, b], [b, d]]: with m = (a + d)/2 and
// r = sqrt(((a - d)/2)^2 + b^2), exp(x O) = e^{x m} (cosh(x r) 1 + sinh(x r)/r (O - m 1)).
__device__ __forceinline__ void vx_exp2(double a, double b, double d, double x, double& e00, double& e01,
                                        double& e11) {
  const double m = 0.5 * (a + d), h = 0.5 * (a - d);
  const double r = sqrt(h * h + b * b);
  const double em = exp(x * m);
  const double ch = cosh(x * r);
  const double sr = r > 0.0 ? sinh(x * r) / r : x;
  e00 = em * (ch + sr * h);
  e11 = em * (ch - sr * h);
  e01 = em * sr * b;
}

// Yout <- E Yin for a product E of vertex exponentials applied to the rows of
// the n x n matrix Yin (row-major, leading dimension n; Yout may be Yin):
// order 0 gives exp(V) Y = E_0 (E_1 (... (E_{M-1} Y))), order 1 gives
// exp(V)^T Y = E_{M-1} (... (E_0 Y)) (every E_k is symmetric).  frow: the
// slice's M field values.  One workgroup per chain, Y staged in LDS: the
// vertices' factors are evaluated in parallel (thread k, vertex k), then
// thread j applies them in sequence to column j (no barrier between vertices).
__global__ __launch_bounds__(256) void k_vx_rows(const double* Yin, double* Yout, int n, const double* tab, int M,
                                                 const double* frow, int order, size_t cs) {
  extern __shared__ double ysm[];
  const int P = n + 1, tid = threadIdx.x;
  double* fac = ysm + (size_t)n * P;                    // [M][3]: e00, e01, e11 (e00 alone for one orbital)
  int* orb = reinterpret_cast<int*>(fac + 3 * (size_t)M);   // [M][3]: np, p0, p1
  {
    const size_t co = (size_t)blockIdx.y * cs;
    Yin += co; Yout += co; frow += co;
  }
  for (int e = tid; e < n * n; e += 256) {
    const int a = e / n, b = e - a * n;
    ysm[a * P + b] = Yin[e];
  }
  for (int k = tid; k < M; k += 256) {
    const VxRec v = vx_load(tab, k);
    const double x = v.g * frow[k];
    double e00, e01 = 0.0, e11 = 0.0;
    if (v.np == 1) e00 = exp(x * v.o00);
    else vx_exp2(v.o00, v.o01, v.o11, x, e00, e01, e11);
    fac[3 * k] = e00; fac[3 * k + 1] = e01; fac[3 * k + 2] = e11;
    orb[3 * k] = v.np; orb[3 * k + 1] = v.p0; orb[3 * k + 2] = v.p1;
  }
  __syncthreads();
  if (tid < n) {
    // the next vertex's orbitals and factors are read ahead of this vertex's
    // update (they are never written here), so only the column's own entries
    // form the dependent chain
    int k = order == 0 ? M - 1 : 0;
    int np = orb[3 * k], p0 = orb[3 * k + 1], p1 = orb[3 * k + 2];
    double e00 = fac[3 * k], e01 = fac[3 * k + 1], e11 = fac[3 * k + 2];
    for (int q = 0; q < M; ++q) {
      const int kn = order == 0 ? M - 2 - q : q + 1;
      const int kc = (q + 1 < M) ? kn : k;
      const int np_n = orb[3 * kc], p0_n = orb[3 * kc + 1], p1_n = orb[3 * kc + 2];
      const double e00_n = fac[3 * kc], e01_n = fac[3 * kc + 1], e11_n = fac[3 * kc + 2];
      if (np == 1) {
        ysm[p0 * P + tid] *= e00;
      } else {
        const double y0 = ysm[p0 * P + tid], y1 = ysm[p1 * P + tid];
        ysm[p0 * P + tid] = e00 * y0 + e01 * y1;
        ysm[p1 * P + tid] = e01 * y0 + e11 * y1;
      }
      k = kc; np = np_n; p0 = p0_n; p1 = p1_n; e00 = e00_n; e01 = e01_n; e11 = e11_n;
    }
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += 256) {
    const int a = e / n, b = e - a * n;
    Yout[e] = ysm[a * P + b];
  }
}

// G <- A G A^-1 for A acting on the orbitals P of one vertex (A = [[a00, a01],
// [a01, a11]] on (p0, p1), or a00 on p0 alone), B = A^-1 given as well, in
// one pass: thread t < n takes row-P entries of column t and column-P entries
// of row t; the P x P corner is taken by thread p0 as (A G_PP) B, the order of
// a product of the rows first.  With stage, the new columns G[:,P] and rows
// e_P - G[P,:] are written to cv and rv.  The caller puts a barrier after it.
__device__ __forceinline__ void vx_move(double* gsm, int P, int n, int np, int p0, int p1, double a00, double a01,
                                        double a11, double b00, double b01, double b11, bool stage,
                                        double (*cv)[kVxMaxN], double (*rv)[kVxMaxN]) {
  const int t = threadIdx.x;
  if (t >= n) return;
  if (np == 1) {
    if (t != p0) {
      const double r = a00 * gsm[p0 * P + t], c = gsm[t * P + p0] * b00;
      gsm[p0 * P + t] = r;
      gsm[t * P + p0] = c;
      if (stage) { cv[0][t] = c; rv[0][t] = -r; }
    } else {
      const double g = (a00 * gsm[p0 * P + p0]) * b00;
      gsm[p0 * P + p0] = g;
      if (stage) { cv[0][p0] = g; rv[0][p0] = 1.0 - g; }
    }
    return;
  }
  if (t != p0 && t != p1) {
    const double y0 = gsm[p0 * P + t], y1 = gsm[p1 * P + t];
    const double r0 = a00 * y0 + a01 * y1, r1 = a01 * y0 + a11 * y1;
    const double z0 = gsm[t * P + p0], z1 = gsm[t * P + p1];
    const double c0 = z0 * b00 + z1 * b01, c1 = z0 * b01 + z1 * b11;
    gsm[p0 * P + t] = r0; gsm[p1 * P + t] = r1;
    gsm[t * P + p0] = c0; gsm[t * P + p1] = c1;
    if (stage) { cv[0][t] = c0; cv[1][t] = c1; rv[0][t] = -r0; rv[1][t] = -r1; }
  } else if (t == p0) {
    const double g00 = gsm[p0 * P + p0], g01 = gsm[p0 * P + p1], g10 = gsm[p1 * P + p0], g11 = gsm[p1 * P + p1];
    // rows: H = A G_PP
    const double h00 = a00 * g00 + a01 * g10, h01 = a00 * g01 + a01 * g11;
    const double h10 = a01 * g00 + a11 * g10, h11 = a01 * g01 + a11 * g11;
    // columns: C = H B
    const double c00 = h00 * b00 + h01 * b01, c01 = h00 * b01 + h01 * b11;
    const double c10 = h10 * b00 + h11 * b01, c11 = h10 * b01 + h11 * b11;
    gsm[p0 * P + p0] = c00; gsm[p0 * P + p1] = c01; gsm[p1 * P + p0] = c10; gsm[p1 * P + p1] = c11;
    if (stage) {
      cv[0][p0] = c00; cv[0][p1] = c10; cv[1][p0] = c01; cv[1][p1] = c11;
      rv[0][p0] = 1.0 - c00; rv[0][p1] = -c01; rv[1][p0] = -c10; rv[1][p1] = 1.0 - c11;
    }
  }
}

// The flips of one slice with the partial wraps, one workgroup per chain, G
// (n x n) in LDS.  field: [L][M] (slice tau's row updated in place); nbr: the
// Ising partners (vertex indices, as doubles) of the records' ranges, nnb
// entries.  Everything about a vertex that does not depend on G or on the
// other flips (its exponentials at the slice's current value and their
// inverses, delta of the flip, the alpha factor and the temporal part of the
// S0 ratio, its Philox draw) is evaluated in parallel before the sequential
// loop, and each Ising vertex keeps the sum of its partners' current values
// (updated by the partners' accepted flips); per vertex the loop then costs
// one barrier (two if accepted) upward and two (three) downward.
__global__ __launch_bounds__(256) void k_vx_slice(double* G, int n, double* field, int L, int tau,
                                                  unsigned long long dir, const double* tab, const double* nbr, int nnb,
                                                  int M, double Kt, double dtJ, int n_col,
                                                  unsigned long long* counters, size_t cs) {
  extern __shared__ double gsm[];
  __shared__ double cv[2][2][kVxMaxN], rv[2][2][kVxMaxN];   // staged columns and e_P - rows, by vertex parity
  const int P = n + 1, tid = threadIdx.x;
  double* pre = gsm + (size_t)n * P;            // [M][kVxPre]
  double* fr = pre + (size_t)kVxPre * M;        // slice tau's field, current values
  double* hs = fr + M;                          // Ising vertices: the sum of the partners' current values
  // Ising vertex k with c partners: its S0 factors for the partner sums -c, -c + 2, ..., c
  // at [first partner + k, ... + c]
  double* tb = hs + M;
  // [M][kVxInt]: np, p0, p1, ising, first partner, partner count, the value at the start of the pass
  int* vi = reinterpret_cast<int*>(tb + M + nnb);
  int* nb = vi + (size_t)kVxInt * M;            // partner lists
  {
    const size_t co = (size_t)blockIdx.y * cs;
    G += co; field += co;
    counters = reinterpret_cast<unsigned long long*>(reinterpret_cast<double*>(counters) + co);
  }
  double* frow = field + (size_t)(tau - 1) * M;
  const double* fup = field + (size_t)(tau % L) * M;              // slice tau + 1 (periodic)
  const double* fdn = field + (size_t)((tau - 2 + L) % L) * M;     // slice tau - 1
  for (int e = tid; e < n * n; e += 256) {
    const int a = e / n, b = e - a * n;
    gsm[a * P + b] = G[(size_t)a * n + b];
  }
  for (int j = tid; j < nnb; j += 256) nb[j] = (int)nbr[j];
  const unsigned long long sweep = counters[2], key = counters[3];
  for (int k = tid; k < M; k += 256) {
    const VxRec v = vx_load(tab, k);
    const double s = frow[k];
    fr[k] = s;
    double* w = pre + (size_t)kVxPre * k;
    // exp(g s O), exp(-g s O), delta = exp(-2 g s O) - 1
    if (v.np == 1) {
      w[0] = exp(v.g * s * v.o00); w[1] = 0.0; w[2] = 0.0;
      w[3] = exp(-v.g * s * v.o00); w[4] = 0.0; w[5] = 0.0;
      w[6] = exp(v.g * (-2.0 * s) * v.o00) - 1.0; w[7] = 0.0; w[8] = 0.0;
    } else {
      vx_exp2(v.o00, v.o01, v.o11, v.g * s, w[0], w[1], w[2]);
      vx_exp2(v.o00, v.o01, v.o11, -v.g * s, w[3], w[4], w[5]);
      vx_exp2(v.o00, v.o01, v.o11, v.g * (-2.0 * s), w[6], w[7], w[8]);
      w[6] -= 1.0; w[8] -= 1.0;
    }
    w[9] = exp(n_col * v.g * v.alpha * (-2.0 * s));
    // with a single slice the spin's temporal bond is to itself: a constant
    const double tmp = (v.ising && L > 1) ? Kt * (fup[k] + fdn[k]) : 0.0;
    if (v.ising)
      for (int i = 0; i <= v.nbc; ++i) tb[v.nb0 + k + i] = exp(-2.0 * s * (tmp + dtJ * (double)(2 * i - v.nbc)));
    w[10] = 0.0;
    const Philox4 ph = philox4x64_10(TAG_FLIP, sweep, ((unsigned long long)tau << 1) | dir, (unsigned long long)k,
                                     key, 0ull);
    w[11] = unit_double(ph.w[0]);
    int* iv = vi + (size_t)kVxInt * k;
    iv[0] = v.np; iv[1] = v.p0; iv[2] = v.p1; iv[3] = v.ising; iv[4] = v.nb0; iv[5] = v.nbc;
    iv[6] = s > 0.0 ? 1 : -1;
  }
  __syncthreads();
  for (int k = tid; k < M; k += 256) {
    const int* iv = vi + (size_t)kVxInt * k;
    double sum = 0.0;   // a sum of +-1: exact
    for (int j = 0; j < iv[5]; ++j) sum += fr[nb[iv[4] + j]];
    hs[k] = sum;
  }
  __syncthreads();
  int nacc = 0;
  for (int q = 0; q < M; ++q) {
    const int k = dir == 0 ? M - 1 - q : q;
    const int par = q & 1;
    const int* iv = vi + (size_t)kVxInt * k;
    const int np = iv[0], p0 = iv[1], p1 = iv[2];
    const double* w = pre + (size_t)kVxPre * k;
    const double s = fr[k];   // not yet flipped in this pass
    if (dir == 0) {
      // move to the frame of vertex k (G <- E_k G E_k^-1), staging its columns and rows
      vx_move(gsm, P, n, np, p0, p1, w[0], w[1], w[2], w[3], w[4], w[5], true, cv[par], rv[par]);
      __syncthreads();
    } else {
      // leave the frame of vertex k-1 (G <- E^-1 G E with its current value)
      if (q > 0) {
        const int* ip = vi + (size_t)kVxInt * (k - 1);
        const double* wp = pre + (size_t)kVxPre * (k - 1);
        const bool flipped = fr[k - 1] != (double)ip[6];
        // E(s_now)^-1 and E(s_now): the inverse and the exponential at the original value, swapped once flipped
        const double* ei = flipped ? wp : wp + 3;
        const double* ee = flipped ? wp + 3 : wp;
        vx_move(gsm, P, n, ip[0], ip[1], ip[2], ei[0], ei[1], ei[2], ee[0], ee[1], ee[2], false, nullptr, nullptr);
        __syncthreads();
      }
      if (tid < n) {
        cv[par][0][tid] = gsm[tid * P + p0];
        rv[par][0][tid] = (tid == p0 ? 1.0 : 0.0) - gsm[p0 * P + tid];
        if (np == 2) {
          cv[par][1][tid] = gsm[tid * P + p1];
          rv[par][1][tid] = (tid == p1 ? 1.0 : 0.0) - gsm[p1 * P + tid];
        }
      }
      __syncthreads();
    }
    // the proposal s -> -s (uniform across the workgroup)
    const double d00 = w[6], d01 = w[7], d11 = w[8];
    double det, r00, r01, r10, r11;
    {
      const double m00 = 1.0 - cv[par][0][p0];
      if (np == 1) {
        r00 = 1.0 + d00 * m00; r01 = 0.0; r10 = 0.0; r11 = 1.0;
        det = r00;
      } else {
        const double m01 = -cv[par][1][p0], m10 = -cv[par][0][p1], m11 = 1.0 - cv[par][1][p1];
        r00 = 1.0 + d00 * m00 + d01 * m10; r01 = d00 * m01 + d01 * m11;
        r10 = d01 * m00 + d11 * m10;       r11 = 1.0 + d01 * m01 + d11 * m11;
        det = r00 * r11 - r01 * r10;
      }
    }
    double R = det;
    for (int c = 1; c < n_col; ++c) R *= det;
    R *= w[9];
    if (iv[3]) R *= tb[iv[4] + k + (((int)hs[k] + iv[5]) >> 1)];
    if (w[11] < R) {
      ++nacc;
      // W = R_P^-1 delta, then G <- G - G[:,P] W (1 - G)[P,:]
      double w00, w01, w10, w11;
      if (np == 1) { w00 = d00 / r00; w01 = 0.0; w10 = 0.0; w11 = 0.0; }
      else {
        const double i00 = r11 / det, i01 = -r01 / det, i10 = -r10 / det, i11 = r00 / det;
        w00 = i00 * d00 + i01 * d01; w01 = i00 * d01 + i01 * d11;
        w10 = i10 * d00 + i11 * d01; w11 = i10 * d01 + i11 * d11;
      }
      // thread (a0, b): column b, rows a0, a0 + 4, ... (n <= 64); every
      // operand is read into registers before the first write
      const int b = tid & 63, a0 = tid >> 6;
      if (b < n) {
        const double q0 = rv[par][0][b], q1 = rv[par][1][b];
        double g[16], x0[16], x1[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int a = a0 + 4 * i;
          if (a < n) { g[i] = gsm[a * P + b]; x0[i] = cv[par][0][a]; x1[i] = cv[par][1][a]; }
        }
        if (np == 1) {
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int a = a0 + 4 * i;
            if (a < n) gsm[a * P + b] = g[i] - x0[i] * (w00 * q0);
          }
        } else {
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int a = a0 + 4 * i;
            if (a < n) gsm[a * P + b] = g[i] - (x0[i] * (w00 * q0) + (x0[i] * (w01 * q1) + x1[i] * (w10 * q0 + w11 * q1)));
          }
        }
      }
      if (tid == 0) fr[k] = -s;
      // the partners' sums change by -2 s (LDS atomics: a partner may be listed twice)
      if (iv[3])
        for (int j = tid; j < iv[5]; j += 256) atomicAdd(&hs[nb[iv[4] + j]], -2.0 * s);
      __syncthreads();
    }
  }
  if (dir == 1) {
    // leave the frame of the last vertex
    const int k = M - 1;
    const int* ip = vi + (size_t)kVxInt * k;
    const double* wp = pre + (size_t)kVxPre * k;
    const bool flipped = fr[k] != (double)ip[6];
    const double* ei = flipped ? wp : wp + 3;
    const double* ee = flipped ? wp + 3 : wp;
    vx_move(gsm, P, n, ip[0], ip[1], ip[2], ei[0], ei[1], ei[2], ee[0], ee[1], ee[2], false, nullptr, nullptr);
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += 256) {
    const int a = e / n, b = e - a * n;
    G[(size_t)a * n + b] = gsm[a * P + b];
  }
  for (int k = tid; k < M; k += 256) frow[k] = fr[k];
  if (tid == 0) {
    counters[0] += (unsigned long long)M;
    counters[1] += (unsigned long long)nacc;
  }
}
