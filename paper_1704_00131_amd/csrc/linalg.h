// Blocked Householder QR with column pre-pivoting and blocked LU with partial
// pivoting, the two factorisations of the stabilisation (section
// "Stabilization - a peculiarity of the BSS algorithm").
//
// Both are right-looking with panels of nb <= 32 columns: the panel is
// factorised by one workgroup entirely in LDS (BLAS-2 work, latency bound),
// and the trailing matrix is updated with the MFMA GEMM of gemm.h (BLAS-3).
//
// QR: the columns are first ordered by decreasing 2-norm (the paper's
// "manual pivoting" variant of the stabilisation), then factorised without
// further pivoting.  Each panel produces its Householder vectors V (unit lower
// trapezoidal, stored explicitly) and the compact-WY factor VT = V T with
// H_1 ... H_nb = I - V T V^T, so that Q^T A = A - V (VT^T A) and
// Q X = X - VT (V^T X).
#pragma once
#include "device_common.h"

// ------------------------------------------------------------ utilities ----
__global__ void k_set_identity(double* A, int n, int ld) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  A[(size_t)i * ld + j] = (i == j) ? 1.0 : 0.0;
}

__global__ void k_fill(double* A, size_t count, double v) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) A[e] = v;
}

__global__ void k_copy(double* dst, const double* src, size_t count) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) dst[e] = src[e];
}

// dst[i][j] = src[j][i] * scale(i)
__global__ void k_transpose_scale(double* dst, const double* src, int n, const double* d, int mode) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int i = by + r, j = bx + tx;                       // read src[i][j]
    tile[r][tx] = (i < n && j < n) ? src[(size_t)i * n + j] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = bx + r, j = by + tx;                       // write dst[i][j] = src[j][i]
    if (i < n && j < n) dst[(size_t)i * n + j] = tile[tx][r] * scale_of(mode, d, 0.0, i);
  }
}

// -------------------------------------------------------- QR pre-pivoting ----
// piv[p] = index of the column with the p-th largest 2-norm (ties: lower index)
__global__ __launch_bounds__(1024) void k_colnorm_order(const double* M, int n, double* norms, int* piv) {
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < n; ++r) { const double x = M[(size_t)r * n + j]; s += x * x; }
    norms[j] = (s == s) ? s : INFINITY;   // a NaN column sorts first; ranks stay a permutation
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double v = norms[j];
    int rank = 0;
    for (int i = 0; i < n; ++i) {
      const double u = norms[i];
      rank += (u > v) || (u == v && i < j);
    }
    piv[rank] = j;
  }
}

__global__ void k_permute_cols(double* dst, const double* src, const int* piv, int n) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  dst[e] = src[(size_t)i * n + piv[j]];
}

// ---------------------------------------------------------- QR panel ----
// Panel rows j0..n-1, columns j0..j0+nbw-1 of A (ld n).  Writes R back into the
// panel (zeros below the diagonal), V (h x nbw, ld nbw) and VT = V T (h x nbw).
// LDS: h*(nbw+1) + nbw + nbw*nbw + nbw*nbw + 64 doubles.
__global__ __launch_bounds__(256) void k_qr_panel(double* A, int n, int j0, int nbw, double* Vout,
                                                  double* VTout) {
  extern __shared__ double smem[];
  const int h = n - j0, P = nbw + 1, tid = threadIdx.x;
  double* pan = smem;
  double* tau = pan + (size_t)h * P;
  double* T = tau + nbw;
  double* Y = T + nbw * nbw;
  double* red = Y + nbw * nbw;     // 8
  double* wv = red + 8;            // nbw
  for (int e = tid; e < h * nbw; e += 256) {
    const int r = e / nbw, c = e % nbw;
    pan[r * P + c] = A[(size_t)(j0 + r) * n + j0 + c];
  }
  __syncthreads();
  for (int c = 0; c < nbw && c < h; ++c) {
    double s = 0.0;
    for (int r = c + 1 + tid; r < h; r += 256) { const double x = pan[r * P + c]; s += x * x; }
    s = block_sum<256>(s, red);
    const double x0 = pan[c * P + c];
    double beta, tc, scal;
    if (s == 0.0) { tc = 0.0; beta = x0; scal = 0.0; }
    else {
      const double nrm = sqrt(x0 * x0 + s);
      beta = (x0 >= 0.0) ? -nrm : nrm;
      tc = (beta - x0) / beta;
      scal = 1.0 / (x0 - beta);
    }
    for (int r = c + 1 + tid; r < h; r += 256) pan[r * P + c] *= scal;
    __syncthreads();
    if (tid == 0) { pan[c * P + c] = beta; tau[c] = tc; }
    if (tc != 0.0) {
      for (int q = c + 1 + (tid >> 6); q < nbw; q += 4) {
        double acc = 0.0;
        for (int r = c + 1 + (tid & 63); r < h; r += 64) acc += pan[r * P + c] * pan[r * P + q];
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if ((tid & 63) == 0) wv[q] = tc * (pan[c * P + q] + acc);
      }
      __syncthreads();
      const int nq = nbw - c - 1;
      if (nq > 0) {
        for (int e = tid; e < (h - c) * nq; e += 256) {
          const int r = c + e / nq, q = c + 1 + e % nq;
          const double vr = (r == c) ? 1.0 : pan[r * P + c];
          pan[r * P + q] -= vr * wv[q];
        }
      }
    }
    __syncthreads();
  }
  // Gram matrix Y = V^T V (V unit lower trapezoidal)
  for (int e = tid; e < nbw * nbw; e += 256) {
    const int a = e / nbw, b = e % nbw;
    double acc = 0.0;
    const int r0 = a > b ? a : b;
    for (int r = r0; r < h; ++r) {
      const double va = (r == a) ? 1.0 : pan[r * P + a];
      const double vb = (r == b) ? 1.0 : pan[r * P + b];
      acc += va * vb;
    }
    Y[e] = acc;
    T[e] = 0.0;
  }
  __syncthreads();
  // forward column-wise T: T[i][i] = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] Y[0:i, i]
  for (int i = 0; i < nbw; ++i) {
    if (tid < i) {
      double acc = 0.0;
      for (int k = tid; k < i; ++k) acc += T[tid * nbw + k] * Y[k * nbw + i];
      T[tid * nbw + i] = -tau[i] * acc;
    }
    if (tid == 0) T[i * nbw + i] = tau[i];
    __syncthreads();
  }
  // outputs
  for (int e = tid; e < h * nbw; e += 256) {
    const int r = e / nbw, b = e % nbw;
    const double v = (r == b) ? 1.0 : (r > b ? pan[r * P + b] : 0.0);
    Vout[e] = v;
    double acc = 0.0;
    const int amax = r < b ? r : b;       // V[r][a] nonzero for a <= r; T[a][b] for a <= b
    for (int a = 0; a <= amax; ++a) {
      const double va = (r == a) ? 1.0 : pan[r * P + a];
      acc += va * T[a * nbw + b];
    }
    VTout[e] = acc;
    A[(size_t)(j0 + r) * n + j0 + b] = (r <= b) ? pan[r * P + b] : 0.0;
  }
}

// Rt[i][piv[j]] = R[i][j] / |R[i][i]| for j >= i; D[i] = |R[i][i]|
__global__ void k_build_rt(const double* R, const int* piv, int n, double* Rt, double* D, int* err) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  const double d = fabs(R[(size_t)i * n + i]);
  if (j == 0) {
    D[i] = d;
    if (!(d > 1e-300)) atomicOr(err, 2);
  }
  Rt[(size_t)i * n + piv[j]] = (j >= i) ? R[(size_t)i * n + j] / d : 0.0;
}

// ----------------------------------------------------------- LU panel ----
// Partial pivoting over rows j0..n-1 of the panel columns j0..j0+nbw-1 of X
// (ld n); ipiv[j0+c] = global pivot row.  Rows are swapped inside the panel
// only; k_lu_swap applies the interchanges elsewhere.
__global__ __launch_bounds__(256) void k_lu_panel(double* X, int n, int j0, int nbw, int* ipiv, int* err) {
  extern __shared__ double smem[];
  const int h = n - j0, P = nbw + 1, tid = threadIdx.x;
  double* pan = smem;
  double* rv = pan + (size_t)h * P;     // 4 values
  int* ri = reinterpret_cast<int*>(rv + 4);
  __shared__ int piv_s;
  for (int e = tid; e < h * nbw; e += 256) {
    const int r = e / nbw, c = e % nbw;
    pan[r * P + c] = X[(size_t)(j0 + r) * n + j0 + c];
  }
  __syncthreads();
  for (int c = 0; c < nbw && c < h; ++c) {
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int r = c + tid; r < h; r += 256) {
      const double v = fabs(pan[r * P + c]);
      if (v > best || (v == best && r < bi)) { best = v; bi = r; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if ((tid & 63) == 0) { rv[tid >> 6] = best; ri[tid >> 6] = bi; }
    __syncthreads();
    if (tid == 0) {
      double b = rv[0];
      int i = ri[0];
      for (int w = 1; w < 4; ++w)
        if (rv[w] > b || (rv[w] == b && ri[w] < i)) { b = rv[w]; i = ri[w]; }
      piv_s = i;
      ipiv[j0 + c] = j0 + i;
      if (!(b > 0.0)) atomicOr(err, 4);
    }
    __syncthreads();
    const int p = piv_s;
    if (p != c) {
      for (int q = tid; q < nbw; q += 256) {
        const double t = pan[c * P + q];
        pan[c * P + q] = pan[p * P + q];
        pan[p * P + q] = t;
      }
      __syncthreads();
    }
    const double inv = 1.0 / pan[c * P + c];
    for (int r = c + 1 + tid; r < h; r += 256) pan[r * P + c] *= inv;
    __syncthreads();
    const int nq = nbw - c - 1;
    if (nq > 0) {
      for (int e = tid; e < (h - c - 1) * nq; e += 256) {
        const int r = c + 1 + e / nq, q = c + 1 + e % nq;
        pan[r * P + q] -= pan[r * P + c] * pan[c * P + q];
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < h * nbw; e += 256) {
    const int r = e / nbw, c = e % nbw;
    X[(size_t)(j0 + r) * n + j0 + c] = pan[r * P + c];
  }
}

// Apply the interchanges of one panel to the columns of X outside the panel
// and to every column of the right-hand sides B (n x nrhs, ld ldb).
__global__ void k_lu_swap(double* X, int n, int j0, int nbw, const int* ipiv, double* B, int nrhs, int ldb) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int nx = n - nbw;
  if (col >= nx + nrhs) return;
  double* base;
  size_t ld;
  if (col < nx) {
    const int cc = col < j0 ? col : col + nbw;
    base = X + cc;
    ld = n;
  } else {
    base = B + (col - nx);
    ld = ldb;
  }
  for (int c = 0; c < nbw && j0 + c < n; ++c) {
    const int r = j0 + c, p = ipiv[r];
    if (p != r) {
      const double t = base[(size_t)r * ld];
      base[(size_t)r * ld] = base[(size_t)p * ld];
      base[(size_t)p * ld] = t;
    }
  }
}

// Solve Tri * Z = Bm in place for a block of nrow <= 32 rows: Tri is the
// nrow x nrow diagonal block (ld ldt), lower with unit diagonal or upper with
// its own diagonal.  One thread per column of Bm.
__global__ __launch_bounds__(256) void k_trsm_block(const double* Tri, int ldt, double* Bm, int ldb, int nrow,
                                                    int ncol, int upper) {
  __shared__ double t[32][33];
  for (int e = threadIdx.x; e < nrow * nrow; e += 256) t[e / nrow][e % nrow] = Tri[(size_t)(e / nrow) * ldt + e % nrow];
  __syncthreads();
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncol) return;
  double z[32];
  for (int r = 0; r < nrow; ++r) z[r] = Bm[(size_t)r * ldb + col];
  if (!upper) {
    for (int r = 0; r < nrow; ++r) {
      double v = z[r];
      for (int k = 0; k < r; ++k) v -= t[r][k] * z[k];
      z[r] = v;
    }
  } else {
    for (int r = nrow - 1; r >= 0; --r) {
      double v = z[r];
      for (int k = r + 1; k < nrow; ++k) v -= t[r][k] * z[k];
      z[r] = v / t[r][r];
    }
  }
  for (int r = 0; r < nrow; ++r) Bm[(size_t)r * ldb + col] = z[r];
}

// out += sum_i log|U_ii| (one workgroup)
__global__ __launch_bounds__(256) void k_logabs_diag(const double* U, int n, double* out) {
  __shared__ double red[8];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += log(fabs(U[(size_t)i * n + i]));
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) *out += s;
}

// out = sum_i log max(d_i, 1)
__global__ __launch_bounds__(256) void k_logbig_sum(const double* d, int n, double* out, int accumulate) {
  __shared__ double red[8];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += log(fmax(d[i], 1.0));
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) *out = accumulate ? (*out + s) : s;
}
