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
__global__ void k_set_identity(double* A, int n, int ld, size_t cs) {
  A += (size_t)blockIdx.y * cs;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  A[(size_t)i * ld + j] = (i == j) ? 1.0 : 0.0;
}

__global__ void k_fill(double* A, size_t count, double v, size_t cs) {
  A += (size_t)blockIdx.y * cs;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) A[e] = v;
}

__global__ void k_copy(double* dst, const double* src, size_t count, size_t cs) {
  dst += (size_t)blockIdx.y * cs;
  src += (size_t)blockIdx.y * cs;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) dst[e] = src[e];
}

// Batched gathers: dst[chain][0..count) <-> src[chain * cs + 0..count)
__global__ void k_gather(double* dst, const double* src, int count, size_t cs) {
  const int t = threadIdx.x;
  if (t < count) dst[(size_t)blockIdx.y * count + t] = src[(size_t)blockIdx.y * cs + t];
}

__global__ void k_scatter(double* dst, const double* src, int count, size_t cs) {
  const int t = threadIdx.x;
  if (t < count) dst[(size_t)blockIdx.y * cs + t] = src[(size_t)blockIdx.y * count + t];
}

// dst[i][j] = src[j][i] * scale(i)
__global__ void k_transpose_scale(double* dst, const double* src, int n, const double* d, int mode, size_t cs_dst,
                                  size_t cs_src) {
  __shared__ double tile[32][33];
  dst += (size_t)blockIdx.z * cs_dst;
  src += (size_t)blockIdx.z * cs_src;
  d += (size_t)blockIdx.z * cs_src;
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
// Column norms in two steps: k_colnorm_part sums the squares of kColRows rows
// per workgroup (threads over columns, coalesced), k_colnorm_order adds the
// partial rows in a fixed order and ranks the columns.
constexpr int kColRows = 16;

__global__ __launch_bounds__(256) void k_colnorm_part(const double* M, int n, double* part, size_t cs) {
  M += (size_t)blockIdx.y * cs;
  part += (size_t)blockIdx.y * cs;
  const int r0 = blockIdx.x * kColRows, r1 = min(n, r0 + kColRows);
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double s = 0.0;
    for (int r = r0; r < r1; ++r) { const double x = M[(size_t)r * n + j]; s += x * x; }
    part[(size_t)blockIdx.x * n + j] = s;
  }
}

// piv[p] = index of the column with the p-th largest 2-norm (ties: lower index)
__global__ __launch_bounds__(1024) void k_colnorm_order(const double* part, int nblk, int n, double* norms, int* piv,
                                                        size_t cs) {
  part += (size_t)blockIdx.y * cs;
  norms += (size_t)blockIdx.y * cs;
  piv = reinterpret_cast<int*>(reinterpret_cast<double*>(piv) + (size_t)blockIdx.y * cs);
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * n + j];
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

__global__ void k_permute_cols(double* dst, const double* src, const int* piv, int n, size_t cs) {
  dst += (size_t)blockIdx.y * cs;
  src += (size_t)blockIdx.y * cs;
  piv = reinterpret_cast<const int*>(reinterpret_cast<const double*>(piv) + (size_t)blockIdx.y * cs);
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  dst[e] = src[(size_t)i * n + piv[j]];
}

// ---------------------------------------------------------- QR panel ----
// Householder QR of one panel (columns j0..j0+nbw-1, rows j0..n-1 of A, ld n)
// by one workgroup, with the compact-WY output V (h x nbw, ld nbw, unit lower
// trapezoidal), VT = V T (T upper triangular, forward column-wise, the dlarft
// convention) and the R entries on and above the diagonal in place (entries
// below it are left as they are: nothing reads them).  Householder convention
// of LAPACK's dlarfg: for x = (x0, x'), beta = -sign(x0) |x|,
// tau = (beta - x0)/beta, v = (1, x' / (x0 - beta)); tau = 0 when x' = 0.
//
// Layout: the panel comes in by coalesced loads through LDS (vsh, 64 MAXR
// rows of NBW+1, zero below row h); wave w owns the columns
// w*NBW/4 .. (w+1)*NBW/4 - 1 and lane l the rows l, l + 64, ... (MAXR of
// them), in registers.  The column loop runs over the owning wave and,
// unrolled, over its columns, so the owner addresses its column without
// selects; as NBW <= 32, only the first row group holds rows at or above the
// diagonal.  Per column c: the owner forms the reflector from its registers
// (norm and x0 in one two-value wave sum), keeps v in its registers and writes
// it to column c of vsh, where it stays as column c of V; one barrier; every
// wave takes the dot products of v_c with all its own columns in one
// multi-value wave sum and applies the reflector to the columns right of c
// (a zero multiplier for the others, so no branches), and the lanes that hold
// the sums for columns left of c (v_q below their diagonal) record v_q^T v_c
// in Y.  After the loop: the T recurrence
// T[t][i] = -tau_i sum_{k<i} T[t][k] Y[k][i] row by row (each lane one row,
// the two halves of the wave splitting k), and VT = V T by MFMA.
template <int NBW>
__host__ __device__ inline size_t qr_panel_lds(int rows) {
  return (size_t)rows * (NBW + 1) + 2 * (size_t)NBW * (NBW + 1) + 2 * NBW;
}

template <int NBW, int MAXR>
__global__ __launch_bounds__(256) void k_qr_panel(double* A, int n, int j0, int nbw, double* Vout,
                                                  double* VTout, size_t cs) {
  extern __shared__ double smem[];
  constexpr int CPW = NBW / 4, PV = NBW + 1, PY = NBW + 1, NE = MAXR * NBW / 4, HR = 64 * MAXR;
  static_assert(NBW <= 32, "rows at or above the diagonal must sit in the first row group");
  {
    const size_t co = (size_t)blockIdx.y * cs;
    A += co; Vout += co; VTout += co;
  }
  const int h = n - j0, tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  double* vsh = smem;                       // HR x PV: the panel, then V
  double* Ym = vsh + HR * PV;               // NBW x PY: strictly upper V^T V
  double* Tm = Ym + NBW * PY;               // NBW x PY: T
  double* tau = Tm + NBW * PY;              // NBW
  double* bet = tau + NBW;                  // NBW: diagonal of R
  {
    double t[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = tid + 256 * u, r = e / NBW, q = e % NBW;
      t[u] = (r < h && q < nbw) ? A[(size_t)(j0 + r) * n + j0 + q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = tid + 256 * u, r = e / NBW, q = e % NBW;
      vsh[r * PV + q] = t[u];
    }
  }
  for (int e = tid; e < NBW * PY; e += 256) Ym[e] = 0.0;
  if (tid < NBW) { tau[tid] = 0.0; bet[tid] = 0.0; }   // columns >= nbw stay inert
  __syncthreads();
  double a[MAXR][CPW];
#pragma unroll
  for (int i = 0; i < MAXR; ++i)
#pragma unroll
    for (int j = 0; j < CPW; ++j) a[i][j] = vsh[(lane + 64 * i) * PV + w * CPW + j];
  const int ncol = min(nbw, h);
  for (int cw = 0; cw < 4; ++cw) {
#pragma unroll
    for (int cj = 0; cj < CPW; ++cj) {
      const int c = cw * CPW + cj;
      if (c >= ncol) break;
      double vr[MAXR];
      if (w == cw) {
        // sum of squares below c, x0 (rows at or above c are in group 0)
        double sx[2] = {0.0, (lane == c) ? a[0][cj] : 0.0};
        sx[0] = (lane > c) ? a[0][cj] * a[0][cj] : 0.0;
#pragma unroll
        for (int i = 1; i < MAXR; ++i) sx[0] = fma(a[i][cj], a[i][cj], sx[0]);
        wave_sums<2>(sx);
        const double s = sx[0], x0 = sx[1];
        double beta, tc, scal;
        if (s == 0.0) { tc = 0.0; beta = x0; scal = 0.0; }
        else {
          const double nrm = sqrt(x0 * x0 + s);
          beta = (x0 >= 0.0) ? -nrm : nrm;
          tc = (beta - x0) / beta;
          scal = 1.0 / (x0 - beta);
        }
        {
          const double x = a[0][cj];
          vr[0] = (lane > c) ? x * scal : (lane == c ? 1.0 : 0.0);
          a[0][cj] = (lane > c) ? vr[0] : (lane == c ? beta : x);
        }
#pragma unroll
        for (int i = 1; i < MAXR; ++i) {
          vr[i] = a[i][cj] * scal;
          a[i][cj] = vr[i];
        }
#pragma unroll
        for (int i = 0; i < MAXR; ++i) vsh[(lane + 64 * i) * PV + c] = vr[i];
        if (lane == 0) { tau[c] = tc; bet[c] = beta; }
      }
      __syncthreads();
      const double tc = tau[c];
      if (w != cw) {
#pragma unroll
        for (int i = 0; i < MAXR; ++i) vr[i] = vsh[(lane + 64 * i) * PV + c];
      }
      double p[CPW];
#pragma unroll
      for (int j = 0; j < CPW; ++j) {
        p[j] = 0.0;
#pragma unroll
        for (int i = 0; i < MAXR; ++i) p[j] = fma(vr[i], a[i][j], p[j]);
      }
      const double tl = wave_sums<CPW>(p);
      {
        // one holder lane per sum: v_q^T v_c for the columns left of c
        const int q = w * CPW + wave_sums_index<CPW>(lane);
        if (wave_sums_holder<CPW>(lane) && q < c) Ym[q * PY + c] = tl;
      }
      double tv[MAXR];
#pragma unroll
      for (int i = 0; i < MAXR; ++i) tv[i] = tc * vr[i];
#pragma unroll
      for (int j = 0; j < CPW; ++j) {
        const int q = w * CPW + j;
        const double pj = (q > c && q < nbw) ? p[j] : 0.0;   // uniform
#pragma unroll
        for (int i = 0; i < MAXR; ++i) a[i][j] = fma(-tv[i], pj, a[i][j]);
      }
    }
  }
  // R on and above the diagonal (rows < nbw <= 32 live in the first row group)
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int q = w * CPW + j;
    if (q < nbw && lane <= q) A[(size_t)(j0 + lane) * n + j0 + q] = a[0][j];
  }
  __syncthreads();
  // T rows: lane (t, half) holds T[t][2 m + half] in ts[m]
  if (w == 0) {
    const int t = lane & 31, half = lane >> 5;
    double ts[NBW / 2];
#pragma unroll
    for (int m = 0; m < NBW / 2; ++m) ts[m] = 0.0;
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < (i + 1) / 2; ++m) acc = fma(ts[m], Ym[(2 * m + half) * PY + i], acc);
      const double tot = add_xor32(acc);
      const double ti = tau[i];
      const double val = (i > t) ? -ti * tot : (i == t ? ti : 0.0);
      if (half == (i & 1)) ts[i / 2] = val;
    }
    if (t < NBW) {
#pragma unroll
      for (int m = 0; m < NBW / 2; ++m) Tm[t * PY + 2 * m + half] = ts[m];
    }
  } else {
    // V to global, coalesced, by the other three waves
    const int t3 = tid - 64;
#pragma unroll
    for (int u = 0; u < (NE * 4 + 2) / 3; ++u) {
      const int e = t3 + 192 * u, r = e / NBW, q = e % NBW;
      if (r < h && q < nbw) Vout[(size_t)r * nbw + q] = vsh[r * PV + q];
    }
  }
  __syncthreads();
  // VT = V T (h x nbw): wave w takes the 16-row tiles w, w + 4, ...; the T
  // operands of all column tiles stay in registers
  constexpr int NT = (NBW + 15) / 16, KS = NBW / 4;
  const int m16 = lane & 15, kk = lane >> 4;
  double tb[KS][NT];
#pragma unroll
  for (int k = 0; k < KS; ++k)
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) {
      const int col = tc * 16 + m16;
      tb[k][tc] = (col < NBW) ? Tm[(4 * k + kk) * PY + col] : 0.0;
    }
  const int nrt = (h + 15) >> 4;
  for (int tr = w; tr < nrt; tr += 4) {
    const int row = tr * 16 + m16;
    double av[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) av[k] = vsh[row * PV + 4 * k + kk];
    v4d acc[NT];
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) acc[tc] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < KS; ++k)
#pragma unroll
      for (int tc = 0; tc < NT; ++tc) acc[tc] = mfma_f64_16x16x4(av[k], tb[k][tc], acc[tc]);
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) {
      const int col = tc * 16 + m16;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int orow = tr * 16 + kk + 4 * rr;
        if (orow < h && col < nbw) VTout[(size_t)orow * nbw + col] = acc[tc][rr];
      }
    }
  }
}

// Rt[i][piv[j]] = R[i][j] / |R[i][i]| for j >= i; D[i] = |R[i][i]|
__global__ void k_build_rt(const double* R, const int* piv, int n, double* Rt, double* D, int* err, size_t cs) {
  {
    const size_t co = (size_t)blockIdx.y * cs;
    R += co; Rt += co; D += co;
    piv = reinterpret_cast<const int*>(reinterpret_cast<const double*>(piv) + co);
    err = reinterpret_cast<int*>(reinterpret_cast<double*>(err) + co);
  }
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
// Panel LU with partial pivoting of columns j0..j0+nbw-1 of X (ld n) over rows
// j0..n-1: the pivot is the largest |a| among the remaining rows, ties to the
// lowest position; multipliers by the pivot's reciprocal.  The interchanges
// of the panel, composed, are written as a list of row moves (moves[0] = count
// K <= 2 nbw, then K pairs (destination row, source row), absolute rows), which
// k_lu_swap applies outside the panel.
//
// Layout: wave w owns the columns w*NBW/4 .. (w+1)*NBW/4 - 1 and lane l the rows
// l, l + 64, ... (MAXR of them), in registers; every wave holds the same rows
// in the same lanes.  Pivoting is virtual: each held row carries its current
// position, a pivot step swaps two positions (every wave keeps the same copy),
// and the rows are written back to their final positions.  The column loop
// runs over the owning wave and, unrolled, over its columns, so the owner
// addresses its column without selects.  Per column c the owner finds the
// pivot (wave max, then the lowest position holding it, both left in every
// lane), forms the multipliers of its rows and publishes them with the
// pivot's lane and register through LDS (two alternating buffers); after one
// barrier every wave reads the pivot row from its own registers (a uniform
// register index) by readlane and eliminates its columns, with a zero
// multiplier for columns at or left of c, so no branches.
constexpr int kLuMoves = 1 + 2 * 64;   // ints of the move list (count + pairs)

template <int NBW, int MAXR>
__global__ __launch_bounds__(256) void k_lu_panel_reg(double* X, int n, int j0, int nbw, int* moves, int* err,
                                                      size_t cs) {
  extern __shared__ double smem[];   // 2 x 64 MAXR multipliers
  constexpr int CPW = NBW / 4, HR = 64 * MAXR;
  __shared__ int piv_s[2][3];        // pivot position, lane, register
  {
    const size_t co = (size_t)blockIdx.y * cs;
    X += co;
    moves = reinterpret_cast<int*>(reinterpret_cast<double*>(moves) + co);
    err = reinterpret_cast<int*>(reinterpret_cast<double*>(err) + co);
  }
  const int h = n - j0, tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  double a[MAXR][CPW];
  int pos[MAXR];
#pragma unroll
  for (int i = 0; i < MAXR; ++i) {
    const int r = lane + 64 * i;
    pos[i] = (r < h) ? r : 0x7fffffff;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int q = w * CPW + j;
      a[i][j] = (r < h && q < nbw) ? X[(size_t)(j0 + r) * n + j0 + q] : 0.0;
    }
  }
  const int ncol = min(nbw, h);
  for (int cw = 0; cw < 4; ++cw) {
#pragma unroll
    for (int cj = 0; cj < CPW; ++cj) {
      const int c = cw * CPW + cj;
      if (c >= ncol) break;
      double* lb = smem + (c & 1) * HR;
      int* ps = piv_s[c & 1];
      if (w == cw) {
        double best = -1.0;
        int bi = 0x7fffffff;
#pragma unroll
        for (int i = 0; i < MAXR; ++i) {
          if (pos[i] >= c && pos[i] < h) {
            const double av = fabs(a[i][cj]);
            if (av > best || (av == best && pos[i] < bi)) { best = av; bi = pos[i]; }
          }
        }
        const double wm = wave_max_all(best);
        int pp = wave_min_all_i((best == wm && best >= 0.0) ? bi : 0x7fffffff);
        pp = __builtin_amdgcn_readfirstlane(pp);
        // no finite candidate (a NaN column): keep the row and flag the failure
        if (!(wm >= 0.0) || pp < c || pp >= h) pp = c;
        // the lane and register holding position pp, and the pivot value
        int hit = -1;
        double pv = 0.0;
#pragma unroll
        for (int i = 0; i < MAXR; ++i)
          if (pos[i] == pp) { hit = i; pv = a[i][cj]; }
        const unsigned long long mask = __ballot(hit >= 0);
        const int hl = __ffsll((long long)mask) - 1;
        const int hs = __builtin_amdgcn_readlane(hit, hl);
        const double inv = 1.0 / readlane_d(pv, hl);
        // multipliers of the rows that stay below the pivot (position > c after the swap)
#pragma unroll
        for (int i = 0; i < MAXR; ++i) {
          const int np = (pos[i] == pp) ? c : (pos[i] == c ? pp : pos[i]);
          const bool below = np > c && np < h;
          const double l = below ? a[i][cj] * inv : 0.0;
          lb[lane + 64 * i] = l;
          a[i][cj] = below ? l : a[i][cj];
        }
        if (lane == 0) {
          ps[0] = pp; ps[1] = hl; ps[2] = hs;
          if (!(wm > 0.0)) atomicOr(err, 4);
        }
      }
      __syncthreads();
      const int pp = __builtin_amdgcn_readfirstlane(ps[0]);
      const int hl = __builtin_amdgcn_readfirstlane(ps[1]);
      const int hs = __builtin_amdgcn_readfirstlane(ps[2]);
#pragma unroll
      for (int i = 0; i < MAXR; ++i) pos[i] = (pos[i] == pp) ? c : (pos[i] == c ? pp : pos[i]);
      double lr[MAXR];
#pragma unroll
      for (int i = 0; i < MAXR; ++i) lr[i] = lb[lane + 64 * i];   // 0 for rows not below the pivot
#pragma unroll
      for (int j = 0; j < CPW; ++j) {
        const int q = w * CPW + j;
        double pr = 0.0;
#pragma unroll
        for (int i = 0; i < MAXR; ++i) pr = (i == hs) ? a[i][j] : pr;   // uniform index
        const double u = (q > c && q < nbw) ? readlane_d(pr, hl) : 0.0;
#pragma unroll
        for (int i = 0; i < MAXR; ++i) a[i][j] = fma(-lr[i], u, a[i][j]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < MAXR; ++i) {
    if (pos[i] < h) {
#pragma unroll
      for (int j = 0; j < CPW; ++j) {
        const int q = w * CPW + j;
        if (q < nbw) X[(size_t)(j0 + pos[i]) * n + j0 + q] = a[i][j];
      }
    }
  }
  // the composed interchanges: original row r now sits at position pos(r);
  // every wave holds the same positions, wave 0 lists the rows that moved
  if (w == 0) {
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < MAXR; ++i) {
      const int r = lane + 64 * i;
      const bool moved = pos[i] < h && pos[i] != r;
      const unsigned long long m = __ballot(moved);
      const int at = cnt + __popcll(m & ((1ull << lane) - 1ull));
      if (moved) {
        moves[1 + 2 * at] = j0 + pos[i];
        moves[2 + 2 * at] = j0 + r;
      }
      cnt += __popcll(m);
    }
    if (lane == 0) moves[0] = cnt;
  }
}

// Apply the interchanges of one panel (the move list of k_lu_panel_reg) to the
// columns of X outside the panel and to every column of the right-hand sides B
// (n x nrhs, ld ldb): one thread per column loads all moved rows first, so
// their latencies overlap, then stores them at their destinations.
__global__ __launch_bounds__(256) void k_lu_swap(double* X, int n, int j0, int nbw, const int* moves, double* B,
                                                 int nrhs, int ldb, size_t cs) {
  {
    const size_t co = (size_t)blockIdx.y * cs;
    X += co; B += co;
    moves = reinterpret_cast<const int*>(reinterpret_cast<const double*>(moves) + co);
  }
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
  const int K = min(moves[0], 64);
  double v[64];
#pragma unroll
  for (int k = 0; k < 64; ++k)
    if (k < K) v[k] = base[(size_t)moves[2 + 2 * k] * ld];
#pragma unroll
  for (int k = 0; k < 64; ++k)
    if (k < K) base[(size_t)moves[1 + 2 * k] * ld] = v[k];
}

// Solve Tri * Z = Bm in place for a block of nrow <= 32 rows: Tri is the
// nrow x nrow diagonal block (ld ldt), lower with unit diagonal or upper with
// its own diagonal.  One thread per column of Bm; the column stays in
// registers (a 32-row block padded with identity rows).  Right-looking: once
// z[k] is final it is taken out of every later row, so the dependent chain is
// one FMA per row; Tri is kept in LDS by columns (tt[k][r] = Tri[r][k]) for
// 16-byte broadcast reads, and the upper case multiplies by the reciprocal
// diagonal.
__global__ __launch_bounds__(256) void k_trsm_block(const double* Tri, int ldt, double* Bm, int ldb, int nrow,
                                                    int ncol, int upper, size_t cs) {
  __shared__ __attribute__((aligned(16))) double tt[32][34];
  __shared__ double dinv[32];
  Tri += (size_t)blockIdx.y * cs;
  Bm += (size_t)blockIdx.y * cs;
  for (int e = threadIdx.x; e < 32 * 32; e += 256) {
    const int r = e >> 5, k = e & 31;
    tt[k][r] = (r < nrow && k < nrow) ? Tri[(size_t)r * ldt + k] : (r == k ? 1.0 : 0.0);
  }
  __syncthreads();
  if (threadIdx.x < 32) dinv[threadIdx.x] = 1.0 / tt[threadIdx.x][threadIdx.x];
  __syncthreads();
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncol) return;
  double z[32];
#pragma unroll
  for (int r = 0; r < 32; ++r) z[r] = (r < nrow) ? Bm[(size_t)r * ldb + col] : 0.0;
  if (!upper) {
#pragma unroll
    for (int k = 0; k < 31; ++k)
#pragma unroll
      for (int r = k + 1; r < 32; ++r) z[r] = fma(-tt[k][r], z[k], z[r]);
  } else {
#pragma unroll
    for (int k = 31; k >= 0; --k) {
      z[k] *= dinv[k];
#pragma unroll
      for (int r = 0; r < k; ++r) z[r] = fma(-tt[k][r], z[k], z[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < 32; ++r)
    if (r < nrow) Bm[(size_t)r * ldb + col] = z[r];
}

// out += sum_i log|U_ii| (one workgroup)
__global__ __launch_bounds__(256) void k_logabs_diag(const double* U, int n, double* out, size_t cs) {
  __shared__ double red[8];
  U += (size_t)blockIdx.y * cs;
  out += (size_t)blockIdx.y * cs;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += log(fabs(U[(size_t)i * n + i]));
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) *out += s;
}

// out = sum_i log max(d_i, 1)
__global__ __launch_bounds__(256) void k_logbig_sum(const double* d, int n, double* out, int accumulate,
                                                    size_t cs_d, size_t cs_out) {
  __shared__ double red[8];
  d += (size_t)blockIdx.y * cs_d;
  out += (size_t)blockIdx.y * cs_out;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += log(fmax(d[i], 1.0));
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) *out = accumulate ? (*out + s) : s;
}
