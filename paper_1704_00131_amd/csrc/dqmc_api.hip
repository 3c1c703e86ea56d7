// Host side of the C ABI declared in include/dqmc.h: argument checks, the
// device buffer layout, and the order of kernel launches that makes up
// Algorithm 1 (section "Pseudo code description").  No arithmetic of the
// method runs on the host.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/dqmc.h"
#include "device_common.h"
#include "gemm.h"
#include "linalg.h"
#include "update.h"

namespace {

constexpr int kBlock = 32;   // sites per decision block

struct UDVp { double* Q; double* D; double* T; };

struct Layout {
  size_t off = 0;
  size_t take(size_t doubles) {
    size_t o = off;
    off += (doubles + 31) & ~size_t(31);   // 256-byte alignment
    return o;
  }
};

}  // namespace

struct dqmc_ctx {
  dqmc_model m{};
  int N = 0, L = 0, nw = 0, nk = 0, nb = 32;
  std::vector<double> K;
  double trK = 0.0, normK1 = 0.0;
  hipStream_t stream = nullptr;
  bool bound = false, initialized = false, poisoned = false;
  uint64_t sweeps_host = 0;
  std::string err;

  double *G = nullptr, *field = nullptr, *slots = nullptr, *work = nullptr;
  // work layout (device pointers)
  double *E = nullptr, *Einv = nullptr, *Eh = nullptr, *Ehinv = nullptr, *Kd = nullptr;
  double *S[6] = {};                  // N x N scratch matrices
  double *Vall = nullptr, *VTall = nullptr, *Zq = nullptr, *Rt = nullptr;
  double *X = nullptr, *RHS = nullptr, *Gs = nullptr, *T1 = nullptr;
  UDVp cur{}, uid{}, hA{}, hB{};
  double *G2 = nullptr, *Gcur = nullptr;   // second G buffer of the out-of-place block updates
  double *field_alt = nullptr;             // field rows written by the upward pass
  std::vector<unsigned char> row_alt;      // host mirror: row tau currently in field_alt
  double *norms = nullptr;
  int *piv = nullptr, *ipiv = nullptr;
  double *bins = nullptr, *prec_hist = nullptr, *prec_tot = nullptr, *logdet = nullptr;
  unsigned long long* counters = nullptr;   // proposals, accepted, sweep counter
  int* err_flag = nullptr;
  size_t work_doubles = 0;
  // optional per-launch event timing of one kernel
  bool timing = false;
  int timing_kernel = 0;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  double timed_flops = 0.0;
  ~dqmc_ctx() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }

  UDVp slot(int k) const {
    const size_t per = 2 * (size_t)N * N + N;
    double* b = slots + per * k;
    return UDVp{b, b + (size_t)N * N, b + (size_t)N * N + N};
  }
};

// ------------------------------------------------------------------ errors --
namespace {

dqmc_status fail(dqmc_ctx* c, dqmc_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(c, DQMC_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t layout_work(dqmc_ctx* c, bool assign) {
  const size_t N = c->N, NN = N * N;
  Layout l;
  auto P = [&](size_t n) -> double* { size_t o = l.take(n); return assign ? c->work + o : nullptr; };
  c->E = P(NN); c->Einv = P(NN); c->Eh = P(NN); c->Ehinv = P(NN); c->Kd = P(NN);
  for (int i = 0; i < 6; ++i) c->S[i] = P(NN);
  c->Vall = P(NN); c->VTall = P(NN); c->Zq = P(NN); c->Rt = P(NN);
  c->X = P(NN); c->RHS = P(NN); c->Gs = P(NN); c->T1 = P(NN);
  UDVp* us[4] = {&c->cur, &c->uid, &c->hA, &c->hB};
  for (UDVp* u : us) { u->Q = P(NN); u->D = P(N); u->T = P(NN); }
  c->G2 = P(NN);
  c->field_alt = P((size_t)c->L * N);
  c->norms = P(N);
  double* pv = P(N); double* ipv = P(N);
  c->piv = reinterpret_cast<int*>(pv); c->ipiv = reinterpret_cast<int*>(ipv);
  c->bins = P(4);
  c->prec_hist = P(2 * (size_t)c->nk + 2);
  c->prec_tot = P(4);
  c->logdet = P(4);
  double* ctr = P(4); c->counters = reinterpret_cast<unsigned long long*>(ctr);
  double* ef = P(1); c->err_flag = reinterpret_cast<int*>(ef);
  return l.off;
}

inline unsigned grid1(size_t n, unsigned bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------- device steps --
dqmc_status timing_begin(dqmc_ctx* c, int kernel) {
  if (!c->timing || c->timing_kernel != kernel) return DQMC_OK;
  while (c->ev.size() < c->ev_used + 2) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    c->ev.push_back(e);
  }
  HIPCHK(hipEventRecord(c->ev[c->ev_used], c->stream));
  return DQMC_OK;
}

dqmc_status timing_end(dqmc_ctx* c, int kernel) {
  if (!c->timing || c->timing_kernel != kernel) return DQMC_OK;
  HIPCHK(hipEventRecord(c->ev[c->ev_used + 1], c->stream));
  c->ev_used += 2;
  return DQMC_OK;
}

dqmc_status gemm(dqmc_ctx* c, const GemmArgs& g) {
  if (dqmc_status s = timing_begin(c, DQMC_KERNEL_GEMM)) return s;
  HIPCHK(launch_gemm(g, c->stream));
  if (c->timing && c->timing_kernel == DQMC_KERNEL_GEMM) c->timed_flops += 2.0 * g.M * (double)g.N * g.K;
  return timing_end(c, DQMC_KERNEL_GEMM);
}

// exp(x K) by scaling and squaring of a degree-18 Taylor polynomial in Horner
// form (all products on the device).
dqmc_status expm(dqmc_ctx* c, double x, double* out) {
  const int N = c->N;
  const double nrm = std::fabs(x) * c->normK1;
  int sq = 0;
  while (nrm / std::ldexp(1.0, sq) > 0.5) ++sq;
  const double a = x / std::ldexp(1.0, sq);
  double* P0 = c->S[0];
  double* P1 = c->S[1];
  hipLaunchKernelGGL(k_set_identity, dim3(grid1((size_t)N * N)), dim3(256), 0, c->stream, P0, N, N);
  HIPCHK(hipGetLastError());
  for (int k = 18; k >= 1; --k) {   // P <- I + (a K / k) P
    GemmArgs g = gemm_args(N, N, N, c->Kd, N, 0, P0, N, 0, P1, N, a / k, 0.0);
    g.diag_add = 1.0;
    if (dqmc_status s = gemm(c, g)) return s;
    std::swap(P0, P1);
  }
  for (int k = 0; k < sq; ++k) {
    if (dqmc_status s = gemm(c, gemm_args(N, N, N, P0, N, 0, P0, N, 0, P1, N))) return s;
    std::swap(P0, P1);
  }
  hipLaunchKernelGGL(k_copy, dim3(grid1((size_t)N * N)), dim3(256), 0, c->stream, out, P0, (size_t)N * N);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

// Current location of field row tau: the upward pass writes its rows to
// field_alt, the downward pass writes them back to the caller's field buffer
// (so no launch reads and writes the same sites).
inline double* field_row(dqmc_ctx* c, int tau) {
  double* base = (!c->row_alt.empty() && c->row_alt[tau - 1]) ? c->field_alt : c->field;
  return base + (size_t)(tau - 1) * c->N;
}

// G(tau) = B_tau G(tau-1) B_tau^-1 = diag(v) E G Einv diag(1/v), v = exp(coupling s_tau)
dqmc_status wrap_up(dqmc_ctx* c, int tau) {
  const int N = c->N;
  if (dqmc_status s = gemm(c, gemm_args(N, N, N, c->E, N, 0, c->Gcur, N, 0, c->T1, N))) return s;
  GemmArgs g = gemm_args(N, N, N, c->T1, N, 0, c->Einv, N, 0, c->G, N);
  c->Gcur = c->G;
  g.rs = field_row(c, tau); g.rs_mode = SC_EXP; g.rs_coef = c->m.coupling;
  g.cs = field_row(c, tau); g.cs_mode = SC_EXP; g.cs_coef = -c->m.coupling;
  return gemm(c, g);
}

// G(tau-1) = B_tau^-1 G(tau) B_tau = Einv diag(1/v) G diag(v) E, written to dst
dqmc_status wrap_down(dqmc_ctx* c, int tau, double* dst) {
  const int N = c->N;
  GemmArgs g1 = gemm_args(N, N, N, c->Gcur, N, 0, c->E, N, 0, c->T1, N);
  g1.ks = field_row(c, tau); g1.ks_mode = SC_EXP; g1.ks_coef = c->m.coupling;
  if (dqmc_status s = gemm(c, g1)) return s;
  GemmArgs g2 = gemm_args(N, N, N, c->Einv, N, 0, c->T1, N, 0, dst, N);
  g2.ks = field_row(c, tau); g2.ks_mode = SC_EXP; g2.ks_coef = -c->m.coupling;
  if (dqmc_status s = gemm(c, g2)) return s;
  c->Gcur = dst;
  return DQMC_OK;
}

// Sequential flips of slice tau, one fused launch per block of 32 sites; G
// alternates between the two buffers, the field row moves to the other buffer.
dqmc_status update_slice(dqmc_ctx* c, int tau, int dir) {
  const int N = c->N;
  const double* fin = field_row(c, tau);
  c->row_alt[tau - 1] ^= 1;
  double* fout = field_row(c, tau);
  const int tiles = ((N + 31) / 32) * ((N + 31) / 32);
  for (int s0 = 0; s0 < N; s0 += kBlock) {
    BlockArgs a;
    a.Gin = c->Gcur;
    a.Gout = (c->Gcur == c->G) ? c->G2 : c->G;
    a.N = N; a.s0 = s0; a.bb = std::min(kBlock, N - s0);
    a.field_in = fin; a.field_out = fout;
    a.sweep_ctr = c->counters + 2;
    a.seed = c->m.seed; a.slot = ((unsigned long long)tau << 1) | (unsigned long long)dir;
    a.coupling = c->m.coupling; a.alpha = c->m.alpha; a.n_col = c->m.n_col;
    a.gauss = c->m.field == DQMC_FIELD_GAUSS; a.prop_width = c->m.prop_width;
    a.counters = c->counters;
    if (dqmc_status s = timing_begin(c, DQMC_KERNEL_BLOCK_UPDATE)) return s;
    hipLaunchKernelGGL(k_block_update, dim3(tiles), dim3(256), 0, c->stream, a);
    HIPCHK(hipGetLastError());
    if (dqmc_status s = timing_end(c, DQMC_KERNEL_BLOCK_UPDATE)) return s;
    c->Gcur = a.Gout;
  }
  return DQMC_OK;
}

// ---------------------------------------------------- UDV stabilisation --
template <int NBW, int MAXR>
void qr_panel_launch(dqmc_ctx* c, double* Ap, int j0, int nbw, double* V, double* VT) {
  const int h = c->N - j0;
  hipLaunchKernelGGL((k_qr_panel<NBW, MAXR>), dim3(1), dim3(256), sizeof(double) * qr_panel_lds<NBW>(h), c->stream,
                     Ap, c->N, j0, nbw, V, VT);
}

template <int NBW>
void qr_panel_pick(dqmc_ctx* c, double* Ap, int j0, int nbw, double* V, double* VT) {
  const int rows = (c->N - j0 + (256 / NBW) - 1) / (256 / NBW);   // rows per thread
  if (rows <= 8) qr_panel_launch<NBW, 8>(c, Ap, j0, nbw, V, VT);
  else if (rows <= 16) qr_panel_launch<NBW, 16>(c, Ap, j0, nbw, V, VT);
  else if (rows <= 24) qr_panel_launch<NBW, 24>(c, Ap, j0, nbw, V, VT);
  else if (rows <= 32) qr_panel_launch<NBW, 32>(c, Ap, j0, nbw, V, VT);
  else if (rows <= 40) qr_panel_launch<NBW, 40>(c, Ap, j0, nbw, V, VT);
  else qr_panel_launch<NBW, 48>(c, Ap, j0, nbw, V, VT);
}

dqmc_status launch_qr_panel(dqmc_ctx* c, double* Ap, int j0, int nbw, double* V, double* VT) {
  if (c->nb == 32) qr_panel_pick<32>(c, Ap, j0, nbw, V, VT);
  else if (c->nb == 16) qr_panel_pick<16>(c, Ap, j0, nbw, V, VT);
  else qr_panel_pick<8>(c, Ap, j0, nbw, V, VT);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

dqmc_status launch_lu_panel(dqmc_ctx* c, double* X, int j0, int nbw) {
  const int h = c->N - j0;
  hipLaunchKernelGGL(k_lu_panel, dim3(1), dim3(256), sizeof(double) * lu_panel_lds(h, nbw), c->stream, X, c->N, j0,
                     nbw, c->ipiv, c->err_flag);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

template <int NBW>
hipError_t lds_limit_qr() {
  const void* fns[] = {reinterpret_cast<const void*>(k_qr_panel<NBW, 8>), reinterpret_cast<const void*>(k_qr_panel<NBW, 16>),
                       reinterpret_cast<const void*>(k_qr_panel<NBW, 24>), reinterpret_cast<const void*>(k_qr_panel<NBW, 32>),
                       reinterpret_cast<const void*>(k_qr_panel<NBW, 40>), reinterpret_cast<const void*>(k_qr_panel<NBW, 48>)};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 156 * 1024);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

dqmc_status set_lds_limits(dqmc_ctx* c) {
  HIPCHK(lds_limit_qr<32>());
  HIPCHK(lds_limit_qr<16>());
  HIPCHK(lds_limit_qr<8>());
  HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_lu_panel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             156 * 1024));
  return DQMC_OK;
}

// QR of M (N x N, overwritten) with column pre-pivoting: M P = Q R.  Writes
// Q, D = |diag R| and T_out = D^-1 R P^T T_in.
dqmc_status qr_udv(dqmc_ctx* c, double* M, const double* T_in, UDVp out) {
  const int N = c->N, nb = c->nb;
  double* Ap = c->S[4];
  hipLaunchKernelGGL(k_colnorm_order, dim3(1), dim3(1024), 0, c->stream, M, N, c->norms, c->piv);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_permute_cols, dim3(grid1((size_t)N * N)), dim3(256), 0, c->stream, Ap, M, c->piv, N);
  HIPCHK(hipGetLastError());
  for (int j0 = 0; j0 < N; j0 += nb) {
    const int nbw = std::min(nb, N - j0), h = N - j0;
    double* V = c->Vall + (size_t)j0 * N;
    double* VT = c->VTall + (size_t)j0 * N;
    if (dqmc_status s = launch_qr_panel(c, Ap, j0, nbw, V, VT)) return s;
    const int ntr = N - j0 - nbw;
    if (ntr > 0) {
      double* At = Ap + (size_t)j0 * N + j0 + nbw;
      if (dqmc_status s = gemm(c, gemm_args(nbw, ntr, h, VT, nbw, 1, At, N, 0, c->Zq, N))) return s;
      if (dqmc_status s = gemm(c, gemm_args(h, ntr, nbw, V, nbw, 0, c->Zq, N, 0, At, N, -1.0, 1.0))) return s;
    }
  }
  // explicit Q by backward accumulation of the block reflectors
  hipLaunchKernelGGL(k_set_identity, dim3(grid1((size_t)N * N)), dim3(256), 0, c->stream, out.Q, N, N);
  HIPCHK(hipGetLastError());
  const int last = ((N - 1) / nb) * nb;
  for (int j0 = last; j0 >= 0; j0 -= nb) {
    const int nbw = std::min(nb, N - j0), h = N - j0;
    double* V = c->Vall + (size_t)j0 * N;
    double* VT = c->VTall + (size_t)j0 * N;
    double* Qs = out.Q + (size_t)j0 * N + j0;
    if (dqmc_status s = gemm(c, gemm_args(nbw, h, h, V, nbw, 1, Qs, N, 0, c->Zq, N))) return s;
    if (dqmc_status s = gemm(c, gemm_args(h, h, nbw, VT, nbw, 0, c->Zq, N, 0, Qs, N, -1.0, 1.0))) return s;
  }
  hipLaunchKernelGGL(k_build_rt, dim3(grid1((size_t)N * N)), dim3(256), 0, c->stream, Ap, c->piv, N, c->Rt, out.D,
                     c->err_flag);
  HIPCHK(hipGetLastError());
  return gemm(c, gemm_args(N, N, N, c->Rt, N, 0, T_in, N, 0, out.T, N));
}

// Right step: UDV of B(hi,0) from that of B(lo,0): M = (B_hi ... B_lo+1 Q) D.
dqmc_status right_step(dqmc_ctx* c, UDVp in, int lo, int hi, UDVp out) {
  const int N = c->N;
  const double* src = in.Q;
  double* bufs[2] = {c->S[2], c->S[3]};
  int b = 0;
  for (int tau = lo + 1; tau <= hi; ++tau) {
    GemmArgs g = gemm_args(N, N, N, c->E, N, 0, src, N, 0, bufs[b], N);
    g.rs = field_row(c, tau); g.rs_mode = SC_EXP; g.rs_coef = c->m.coupling;
    if (tau == hi) { g.cs = in.D; g.cs_mode = SC_VAL; }
    if (dqmc_status s = gemm(c, g)) return s;
    src = bufs[b];
    b ^= 1;
  }
  return qr_udv(c, const_cast<double*>(src), in.T, out);
}

// Left step on transposes: B(beta,lo)^T = B_lo+1^T ... B_hi^T B(beta,hi)^T,
// B_tau^T = E diag(v_tau).
dqmc_status left_step(dqmc_ctx* c, UDVp in, int lo, int hi, UDVp out) {
  const int N = c->N;
  const double* src = in.Q;
  double* bufs[2] = {c->S[2], c->S[3]};
  int b = 0;
  for (int tau = hi; tau > lo; --tau) {
    GemmArgs g = gemm_args(N, N, N, c->E, N, 0, src, N, 0, bufs[b], N);
    g.ks = field_row(c, tau); g.ks_mode = SC_EXP; g.ks_coef = c->m.coupling;
    if (tau == lo + 1) { g.cs = in.D; g.cs_mode = SC_VAL; }
    if (dqmc_status s = gemm(c, g)) return s;
    src = bufs[b];
    b ^= 1;
  }
  return qr_udv(c, const_cast<double*>(src), in.T, out);
}

// Solve X Y = RHS in place (blocked LU with partial pivoting).  If logdet is
// given, adds log|det X|.
dqmc_status lu_solve(dqmc_ctx* c, double* X, double* RHS, double* logdet) {
  const int N = c->N, nb = c->nb;
  for (int j0 = 0; j0 < N; j0 += nb) {
    const int nbw = std::min(nb, N - j0), h = N - j0;
    if (dqmc_status s = launch_lu_panel(c, X, j0, nbw)) return s;
    hipLaunchKernelGGL(k_lu_swap, dim3(grid1((size_t)(N - nbw) + N)), dim3(256), 0, c->stream, X, N, j0, nbw,
                       c->ipiv, RHS, N, N);
    HIPCHK(hipGetLastError());
    const int ntr = N - j0 - nbw;
    if (ntr > 0) {
      hipLaunchKernelGGL(k_trsm_block, dim3(grid1(ntr)), dim3(256), 0, c->stream, X + (size_t)j0 * N + j0, N,
                         X + (size_t)j0 * N + j0 + nbw, N, nbw, ntr, 0);
      HIPCHK(hipGetLastError());
      if (dqmc_status s = gemm(c, gemm_args(ntr, ntr, nbw, X + (size_t)(j0 + nbw) * N + j0, N, 0,
                                            X + (size_t)j0 * N + j0 + nbw, N, 0, X + (size_t)(j0 + nbw) * N + j0 + nbw,
                                            N, -1.0, 1.0)))
        return s;
    }
  }
  // forward substitution with unit-lower L (right-looking)
  for (int j0 = 0; j0 < N; j0 += nb) {
    const int nbw = std::min(nb, N - j0);
    hipLaunchKernelGGL(k_trsm_block, dim3(grid1(N)), dim3(256), 0, c->stream, X + (size_t)j0 * N + j0, N,
                       RHS + (size_t)j0 * N, N, nbw, N, 0);
    HIPCHK(hipGetLastError());
    const int rest = N - j0 - nbw;
    if (rest > 0)
      if (dqmc_status s = gemm(c, gemm_args(rest, N, nbw, X + (size_t)(j0 + nbw) * N + j0, N, 0,
                                            RHS + (size_t)j0 * N, N, 0, RHS + (size_t)(j0 + nbw) * N, N, -1.0, 1.0)))
        return s;
  }
  // back substitution with U
  const int last = ((N - 1) / nb) * nb;
  for (int j0 = last; j0 >= 0; j0 -= nb) {
    const int nbw = std::min(nb, N - j0);
    hipLaunchKernelGGL(k_trsm_block, dim3(grid1(N)), dim3(256), 0, c->stream, X + (size_t)j0 * N + j0, N,
                       RHS + (size_t)j0 * N, N, nbw, N, 1);
    HIPCHK(hipGetLastError());
    if (j0 > 0)
      if (dqmc_status s = gemm(c, gemm_args(j0, N, nbw, X + j0, N, 0, RHS + (size_t)j0 * N, N, 0, RHS, N, -1.0,
                                            1.0)))
        return s;
  }
  if (logdet) {
    hipLaunchKernelGGL(k_logabs_diag, dim3(1), dim3(256), 0, c->stream, X, N, logdet);
    HIPCHK(hipGetLastError());
  }
  return DQMC_OK;
}

// G = (1 + B(tau,0) B(beta,tau))^-1 from the right form (Q_R D_R T_R of
// B(tau,0)) and the left form (Q_L D_L T_L of B(beta,tau)^T):
//   X = D_Rb^-1 (Q_R^T Q_L) D_Lb^-1 + D_Rs (T_R T_L^T) D_Ls
//   G = Q_L D_Lb^-1 X^-1 D_Rb^-1 Q_R^T
dqmc_status merge(dqmc_ctx* c, UDVp R, UDVp Lf, double* Gout, double* logdet) {
  const int N = c->N;
  GemmArgs g1 = gemm_args(N, N, N, R.Q, N, 1, Lf.Q, N, 0, c->X, N);
  g1.rs = R.D; g1.rs_mode = SC_INV_BIG; g1.cs = Lf.D; g1.cs_mode = SC_INV_BIG;
  if (dqmc_status s = gemm(c, g1)) return s;
  GemmArgs g2 = gemm_args(N, N, N, R.T, N, 0, Lf.T, N, 1, c->X, N, 1.0, 1.0);
  g2.rs = R.D; g2.rs_mode = SC_SMALL; g2.cs = Lf.D; g2.cs_mode = SC_SMALL;
  if (dqmc_status s = gemm(c, g2)) return s;
  const dim3 tg((N + 31) / 32, (N + 31) / 32);
  hipLaunchKernelGGL(k_transpose_scale, tg, dim3(256), 0, c->stream, c->RHS, R.Q, N, R.D, SC_INV_BIG);
  HIPCHK(hipGetLastError());
  if (logdet) {
    hipLaunchKernelGGL(k_logbig_sum, dim3(1), dim3(256), 0, c->stream, R.D, N, logdet, 0);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_logbig_sum, dim3(1), dim3(256), 0, c->stream, Lf.D, N, logdet, 1);
    HIPCHK(hipGetLastError());
  }
  if (dqmc_status s = lu_solve(c, c->X, c->RHS, logdet)) return s;
  GemmArgs g3 = gemm_args(N, N, N, Lf.Q, N, 0, c->RHS, N, 0, Gout, N);
  g3.ks = Lf.D; g3.ks_mode = SC_INV_BIG;
  return gemm(c, g3);
}

dqmc_status copy_udv(dqmc_ctx* c, UDVp dst, UDVp src) {
  const size_t NN = (size_t)c->N * c->N;
  hipLaunchKernelGGL(k_copy, dim3(grid1(NN)), dim3(256), 0, c->stream, dst.Q, src.Q, NN);
  hipLaunchKernelGGL(k_copy, dim3(grid1(c->N)), dim3(256), 0, c->stream, dst.D, src.D, (size_t)c->N);
  hipLaunchKernelGGL(k_copy, dim3(grid1(NN)), dim3(256), 0, c->stream, dst.T, src.T, NN);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

dqmc_status stabilise(dqmc_ctx* c, int hist_index) {
  const size_t NN = (size_t)c->N * c->N;
  hipLaunchKernelGGL(k_prec_replace, dim3(std::min<size_t>(grid1(NN), 1024)), dim3(256), 0, c->stream, c->Gcur,
                     c->G, c->Gs, NN, c->prec_hist + hist_index, c->err_flag);
  HIPCHK(hipGetLastError());
  c->Gcur = c->G;
  return DQMC_OK;
}

dqmc_status measure(dqmc_ctx* c) {
  const int N = c->N;
  const double* T1 = nullptr;
  if (c->m.trotter == DQMC_TROTTER_SYM) {
    if (dqmc_status s = gemm(c, gemm_args(N, N, N, c->Eh, N, 0, c->Gcur, N, 0, c->T1, N))) return s;
    T1 = c->T1;
  }
  hipLaunchKernelGGL(k_measure, dim3(1), dim3(1024), 0, c->stream, c->Gcur, T1, c->Ehinv, c->Kd, N, c->trK,
                     (double)c->m.n_col, c->m.u_int, c->bins, c->err_flag);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

// One sweep (Algorithm 1): upward pass tau = 1..L, downward pass tau = L..1.
dqmc_status sweep_once(dqmc_ctx* c, bool meas) {
  const int L = c->L, nw = c->nw, nk = c->nk;
  int hist = 0;
  c->row_alt.assign(L, 0);
  c->Gcur = c->G;
  for (int tau = 1; tau <= L; ++tau) {
    if (dqmc_status s = wrap_up(c, tau)) return s;
    if (dqmc_status s = update_slice(c, tau, 0)) return s;
    if (tau % nw == 0) {
      const int k = tau / nw;
      UDVp prev = (k == 1) ? c->uid : c->slot(k - 1);
      if (dqmc_status s = right_step(c, prev, tau - nw, tau, c->cur)) return s;
      UDVp left = (k == nk) ? c->uid : c->slot(k);
      if (dqmc_status s = merge(c, c->cur, left, c->Gs, nullptr)) return s;
      if (dqmc_status s = copy_udv(c, c->slot(k), c->cur)) return s;
      if (dqmc_status s = stabilise(c, hist++)) return s;
    }
    if (meas)
      if (dqmc_status s = measure(c)) return s;
  }
  for (int tau = L; tau >= 1; --tau) {
    if (dqmc_status s = update_slice(c, tau, 1)) return s;
    if (meas)
      if (dqmc_status s = measure(c)) return s;
    if ((tau - 1) % nw == 0) {
      const int k = (tau - 1) / nw;
      // wrapped G(tau-1), compared against the recomputed one below
      if (dqmc_status s = wrap_down(c, tau, c->G)) return s;
      UDVp prev = (k + 1 == nk) ? c->uid : c->slot(k + 1);
      if (dqmc_status s = left_step(c, prev, tau - 1, tau - 1 + nw, c->cur)) return s;
      UDVp right = (k == 0) ? c->uid : c->slot(k);
      if (dqmc_status s = merge(c, right, c->cur, c->Gs, nullptr)) return s;
      if (dqmc_status s = copy_udv(c, c->slot(k), c->cur)) return s;
      if (dqmc_status s = stabilise(c, hist++)) return s;
    } else {
      if (dqmc_status s = wrap_down(c, tau, c->G)) return s;
    }
  }
  hipLaunchKernelGGL(k_finish_sweep, dim3(1), dim3(64), 0, c->stream, c->prec_hist, hist, c->prec_tot,
                     c->m.prec_threshold, c->counters, c->err_flag);
  HIPCHK(hipGetLastError());
  c->row_alt.clear();
  return DQMC_OK;
}

dqmc_status fill_small(dqmc_ctx* c, double* p, size_t n, double v) {
  hipLaunchKernelGGL(k_fill, dim3(grid1(n)), dim3(256), 0, c->stream, p, n, v);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

dqmc_status check_model(const dqmc_model* m) {
  if (!m) return DQMC_E_ARG;
  if (m->n < 1 || m->n > 1024 || m->n_slices < 1 || m->n_wrap < 1) return DQMC_E_ARG;
  if (m->n_slices % m->n_wrap != 0) return DQMC_E_ARG;
  if (!(m->beta > 0.0) || !(m->dtau > 0.0)) return DQMC_E_ARG;
  if (std::fabs(m->beta - m->n_slices * m->dtau) > 1e-12 * m->beta) return DQMC_E_ARG;
  if (m->n_col < 1 || m->n_col > 2) return DQMC_E_ARG;
  if (m->field != DQMC_FIELD_ISING && m->field != DQMC_FIELD_GAUSS) return DQMC_E_ARG;
  if (m->trotter != DQMC_TROTTER_ASYM && m->trotter != DQMC_TROTTER_SYM) return DQMC_E_ARG;
  if (!std::isfinite(m->coupling) || !std::isfinite(m->alpha)) return DQMC_E_ARG;
  return DQMC_OK;
}

dqmc_status read_flag(dqmc_ctx* c) {
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, c->err_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (flag) {
    c->poisoned = true;
    std::string why;
    if (flag & 1) why += " non-finite Green's function;";
    if (flag & 2) why += " vanishing scale in the QR step;";
    if (flag & 4) why += " singular pivot in the LU step;";
    if (flag & 8) why += " stabilisation precision above threshold;";
    return fail(c, DQMC_E_NUMERIC, "numerical failure:" + why);
  }
  return DQMC_OK;
}

}  // namespace

// ===================================================================== ABI ==
extern "C" {

dqmc_status dqmc_query_sizes(const dqmc_model* m, dqmc_sizes* out) {
  if (!out || check_model(m) != DQMC_OK) return DQMC_E_ARG;
  dqmc_ctx tmp;
  tmp.N = m->n; tmp.L = m->n_slices; tmp.nw = m->n_wrap; tmp.nk = m->n_slices / m->n_wrap;
  const size_t N = m->n;
  out->G = N * N * sizeof(double);
  out->field = (size_t)m->n_slices * N * sizeof(double);
  out->slots = (size_t)(tmp.nk + 1) * (2 * N * N + N) * sizeof(double);
  out->work = layout_work(&tmp, false) * sizeof(double);
  return DQMC_OK;
}

dqmc_status dqmc_create(const dqmc_model* m, const double* K, const int32_t* vertex_site, dqmc_ctx** out) {
  if (!out) return DQMC_E_ARG;
  *out = nullptr;
  if (check_model(m) != DQMC_OK || !K) return DQMC_E_ARG;
  const int N = m->n;
  if (vertex_site)
    for (int i = 0; i < N; ++i)
      if (vertex_site[i] != i) return DQMC_E_UNSUPPORTED;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const double a = K[(size_t)i * N + j], b = K[(size_t)j * N + i];
      if (!std::isfinite(a) || a != b) return DQMC_E_ARG;
    }
  dqmc_ctx* c = new (std::nothrow) dqmc_ctx();
  if (!c) return DQMC_E_NOMEM;
  c->m = *m;
  c->N = N; c->L = m->n_slices; c->nw = m->n_wrap; c->nk = m->n_slices / m->n_wrap;
  // panel width: the register panels hold up to 48 rows per thread in
  // 256/nb row groups
  c->nb = (N <= 8 * 48) ? 32 : (N <= 16 * 48 ? 16 : 8);
  c->K.assign(K, K + (size_t)N * N);
  double tr = 0.0, n1 = 0.0;
  for (int j = 0; j < N; ++j) {
    double col = 0.0;
    for (int i = 0; i < N; ++i) col += std::fabs(K[(size_t)i * N + j]);
    n1 = std::max(n1, col);
    tr += K[(size_t)j * N + j];
  }
  c->trK = tr; c->normK1 = n1;
  *out = c;
  return DQMC_OK;
}

dqmc_status dqmc_bind(dqmc_ctx* c, const dqmc_buffers* b, void* stream) {
  if (!c || !b || !b->G || !b->field || !b->slots || !b->work) return fail(c, DQMC_E_ARG, "null buffer");
  for (void* p : {b->G, b->field, b->slots, b->work})
    if (reinterpret_cast<uintptr_t>(p) % 256) return fail(c, DQMC_E_ARG, "buffers must be 256-byte aligned");
  c->G = static_cast<double*>(b->G);
  c->field = static_cast<double*>(b->field);
  c->slots = static_cast<double*>(b->slots);
  c->work = static_cast<double*>(b->work);
  c->stream = static_cast<hipStream_t>(stream);
  c->work_doubles = layout_work(c, true);
  const int N = c->N;
  // the panel kernels keep up to ~150 KB of a panel in LDS
  if (dqmc_status s = set_lds_limits(c)) return s;
  HIPCHK(hipMemcpyAsync(c->Kd, c->K.data(), sizeof(double) * N * N, hipMemcpyHostToDevice, c->stream));
  if (dqmc_status s = expm(c, -c->m.dtau, c->E)) return s;
  if (dqmc_status s = expm(c, +c->m.dtau, c->Einv)) return s;
  if (dqmc_status s = expm(c, -0.5 * c->m.dtau, c->Eh)) return s;
  if (dqmc_status s = expm(c, +0.5 * c->m.dtau, c->Ehinv)) return s;
  hipLaunchKernelGGL(k_set_identity, dim3(grid1((size_t)N * N)), dim3(256), 0, c->stream, c->uid.Q, N, N);
  hipLaunchKernelGGL(k_set_identity, dim3(grid1((size_t)N * N)), dim3(256), 0, c->stream, c->uid.T, N, N);
  if (dqmc_status s = fill_small(c, c->uid.D, N, 1.0)) return s;
  if (dqmc_status s = fill_small(c, reinterpret_cast<double*>(c->counters), 4, 0.0)) return s;
  if (dqmc_status s = fill_small(c, reinterpret_cast<double*>(c->err_flag), 1, 0.0)) return s;
  HIPCHK(hipStreamSynchronize(c->stream));
  c->bound = true;
  c->initialized = false;
  return DQMC_OK;
}

dqmc_status dqmc_set_state(dqmc_ctx* c, const double* field_host, uint64_t sweep_counter) {
  if (!c || !field_host) return fail(c, DQMC_E_ARG, "null argument");
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  const size_t n = (size_t)c->L * c->N;
  for (size_t e = 0; e < n; ++e) {
    const double v = field_host[e];
    if (!std::isfinite(v) || (c->m.field == DQMC_FIELD_ISING && v != 1.0 && v != -1.0))
      return fail(c, DQMC_E_ARG, "field values must be +-1 (Ising) or finite (Gaussian)");
  }
  HIPCHK(hipMemcpyAsync(c->field, field_host, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  unsigned long long ctr = sweep_counter;
  HIPCHK(hipMemcpyAsync(c->counters + 2, &ctr, sizeof(ctr), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->sweeps_host = sweep_counter;
  c->initialized = false;
  return DQMC_OK;
}

dqmc_status dqmc_get_state(dqmc_ctx* c, double* field_host, uint64_t* sweep_counter) {
  if (!c) return DQMC_E_ARG;
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  if (field_host)
    HIPCHK(hipMemcpyAsync(field_host, c->field, (size_t)c->L * c->N * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
  unsigned long long ctr = 0;
  HIPCHK(hipMemcpyAsync(&ctr, c->counters + 2, sizeof(ctr), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (sweep_counter) *sweep_counter = ctr;
  return DQMC_OK;
}

dqmc_status dqmc_random_field(dqmc_ctx* c) {
  if (!c) return DQMC_E_ARG;
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  const size_t n = (size_t)c->L * c->N;
  hipLaunchKernelGGL(k_random_field, dim3(grid1(n)), dim3(256), 0, c->stream, c->field, c->L, c->N,
                     (unsigned long long)c->m.seed, c->m.field == DQMC_FIELD_GAUSS ? 1 : 0);
  HIPCHK(hipGetLastError());
  unsigned long long zero = 0;
  HIPCHK(hipMemcpyAsync(c->counters + 2, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->initialized = false;
  return DQMC_OK;
}

dqmc_status dqmc_init(dqmc_ctx* c) {
  if (!c) return DQMC_E_ARG;
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  // statistics, bins, flag
  if (dqmc_status s = fill_small(c, c->bins, 4, 0.0)) return s;
  if (dqmc_status s = fill_small(c, c->prec_hist, 2 * (size_t)c->nk + 2, 0.0)) return s;
  if (dqmc_status s = fill_small(c, c->prec_tot, 4, 0.0)) return s;
  if (dqmc_status s = fill_small(c, reinterpret_cast<double*>(c->counters), 2, 0.0)) return s;
  if (dqmc_status s = fill_small(c, reinterpret_cast<double*>(c->err_flag), 1, 0.0)) return s;
  // left storage: slot k = UDV of B(beta, tau_k)^T, k = nk-1 .. 0
  for (int k = c->nk - 1; k >= 0; --k) {
    UDVp prev = (k + 1 == c->nk) ? c->uid : c->slot(k + 1);
    if (dqmc_status s = left_step(c, prev, k * c->nw, (k + 1) * c->nw, c->slot(k))) return s;
  }
  if (dqmc_status s = merge(c, c->uid, c->slot(0), c->G, nullptr)) return s;
  if (dqmc_status s = read_flag(c)) return s;
  c->poisoned = false;
  c->initialized = true;
  return DQMC_OK;
}

dqmc_status dqmc_sweep(dqmc_ctx* c, int32_t n_sweeps, int32_t meas, dqmc_stats* st) {
  if (!c || n_sweeps < 0) return fail(c, DQMC_E_ARG, "bad arguments");
  if (!c->bound || !c->initialized || c->poisoned) return fail(c, DQMC_E_STATE, "context not initialised");
  const auto t0 = std::chrono::steady_clock::now();
  for (int s = 0; s < n_sweeps; ++s)
    if (dqmc_status r = sweep_once(c, meas != 0)) return r;
  if (dqmc_status r = read_flag(c)) return r;
  const auto t1 = std::chrono::steady_clock::now();
  if (st) {
    unsigned long long ctr[3];
    double pt[3];
    HIPCHK(hipMemcpyAsync(ctr, c->counters, sizeof(ctr), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(pt, c->prec_tot, sizeof(pt), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    st->proposals = ctr[0];
    st->accepted = ctr[1];
    st->n_prec = (uint64_t)pt[2];
    st->prec_mean = pt[2] > 0 ? pt[0] / pt[2] : 0.0;
    st->prec_max = pt[1];
    st->seconds = std::chrono::duration<double>(t1 - t0).count();
  }
  return DQMC_OK;
}

dqmc_status dqmc_read_bins(dqmc_ctx* c, double* sums) {
  if (!c || !sums) return DQMC_E_ARG;
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  HIPCHK(hipMemcpyAsync(sums, c->bins, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return DQMC_OK;
}

dqmc_status dqmc_reset_bins(dqmc_ctx* c) {
  if (!c) return DQMC_E_ARG;
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  if (dqmc_status s = fill_small(c, c->bins, 4, 0.0)) return s;
  HIPCHK(hipStreamSynchronize(c->stream));
  return DQMC_OK;
}

dqmc_status dqmc_green_scratch(dqmc_ctx* c, int32_t tau, double* G_dev) {
  if (!c || !G_dev || tau < 0 || tau > c->L) return fail(c, DQMC_E_ARG, "bad arguments");
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  // right chain 0 -> tau in chunks aligned to n_wrap, ping-pong hA/hB
  UDVp right = c->uid;
  UDVp bufs[2] = {c->hA, c->hB};
  int b = 0;
  for (int lo = 0; lo < tau;) {
    const int hi = std::min(tau, (lo / c->nw + 1) * c->nw);
    if (dqmc_status s = right_step(c, right, lo, hi, bufs[b])) return s;
    right = bufs[b];
    b ^= 1;
    lo = hi;
  }
  // left chain beta -> tau; the right result stays in `right`
  UDVp left = c->uid;
  UDVp lb[2] = {c->cur, (right.Q == c->hA.Q) ? c->hB : c->hA};
  int q = 0;
  std::vector<int> edges;
  for (int e = tau; e < c->L;) { edges.push_back(e); e = (e / c->nw + 1) * c->nw; }
  edges.push_back(c->L);
  for (int i = (int)edges.size() - 2; i >= 0; --i) {
    if (dqmc_status s = left_step(c, left, edges[i], edges[i + 1], lb[q])) return s;
    left = lb[q];
    q ^= 1;
  }
  if (dqmc_status s = merge(c, right, left, G_dev, nullptr)) return s;
  HIPCHK(hipStreamSynchronize(c->stream));
  return read_flag(c);
}

dqmc_status dqmc_logdet(dqmc_ctx* c, double* logdet) {
  if (!c || !logdet) return DQMC_E_ARG;
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  UDVp left = c->uid;
  UDVp lb[2] = {c->hA, c->hB};
  int q = 0;
  for (int k = c->nk - 1; k >= 0; --k) {
    if (dqmc_status s = left_step(c, left, k * c->nw, (k + 1) * c->nw, lb[q])) return s;
    left = lb[q];
    q ^= 1;
  }
  if (dqmc_status s = merge(c, c->uid, left, c->Gs, c->logdet)) return s;
  HIPCHK(hipMemcpyAsync(logdet, c->logdet, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return read_flag(c);
}

dqmc_status dqmc_timing_enable(dqmc_ctx* c, dqmc_kernel kernel, int32_t enable) {
  if (!c || (kernel != DQMC_KERNEL_BLOCK_UPDATE && kernel != DQMC_KERNEL_GEMM)) return DQMC_E_ARG;
  c->timing = enable != 0;
  c->timing_kernel = kernel;
  c->ev_used = 0;
  c->timed_flops = 0.0;
  return DQMC_OK;
}

dqmc_status dqmc_timing_read(dqmc_ctx* c, double* total_ms, uint64_t* launches, double* flops) {
  if (!c || !total_ms || !launches) return DQMC_E_ARG;
  HIPCHK(hipStreamSynchronize(c->stream));
  double tot = 0.0;
  for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
    tot += ms;
  }
  *total_ms = tot;
  *launches = c->ev_used / 2;
  if (flops) *flops = c->timed_flops;
  c->ev_used = 0;
  c->timed_flops = 0.0;
  return DQMC_OK;
}

const char* dqmc_last_error(const dqmc_ctx* c) { return c ? c->err.c_str() : "null context"; }

void dqmc_destroy(dqmc_ctx* c) { delete c; }

dqmc_status dqmc_hubbard_coupling(double U, double dtau, dqmc_field_kind kind, double* coupling) {
  if (!coupling || !(dtau > 0.0) || !std::isfinite(U)) return DQMC_E_ARG;
  if (kind == DQMC_FIELD_ISING) {
    if (U < 0.0) return DQMC_E_ARG;
    *coupling = std::acosh(std::exp(dtau * U / 2.0));
  } else if (kind == DQMC_FIELD_GAUSS) {
    if (U < 0.0) return DQMC_E_ARG;
    *coupling = std::sqrt(dtau * U);
  } else {
    return DQMC_E_ARG;
  }
  return DQMC_OK;
}

}  // extern "C"
