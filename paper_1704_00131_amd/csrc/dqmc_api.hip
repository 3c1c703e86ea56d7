// Host side of the C ABI declared in include/dqmc.h: argument checks, the
// device buffer layout, and the order of kernel launches that makes up
// Algorithm 1 (section "Pseudo code description").  No arithmetic of the
// method runs on the host.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/dqmc.h"
#include "device_common.h"
#include "gemm.h"
#include "linalg.h"
#include "update.h"
#include "adjoint.h"
#include "timedisplaced.h"
#include "correlations.h"
#include "complex.h"
#include "chunk.h"
#include "flavours.h"
#include "vertices.h"

namespace {

constexpr int kBlock = 32;   // sites per decision block
// largest N with 32-column QR and LU panels (honeycomb 12x12, N = 288:
// 47.0 -> 45.7 ms per sweep with 16-column panels)
constexpr int kNarrowMaxN = 256;
// smallest N above which a single chain takes the latency-oriented Q
// accumulation and back substitution (at N = 288 they took 118 and 70 us
// against 59 and 57 us for the four-wave kernels)
constexpr int kWideMinN = 384;

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
  // field sites per slice; the complex field (cplx) runs on the real 2 Nf x 2 Nf
  // images of its complex matrices, so there N = 2 Nf
  int Nf = 0, cplx = 0;
  // two flavours (the M_z form with two Green's functions) on the 2 Nf x 2 Nf
  // block-diagonal system, the field expanded to [s, -s] per slice in field_x
  int nfl = 1;
  double* field_x = nullptr;
  double trK_field = 0.0;     // trace of the n x n hopping matrix (complex estimators)
  // general operator vertices (nvx > 0): the field is [L][nvx], one value per
  // vertex; records of kVxRec doubles and the Ising partner lists (shared)
  int nvx = 0, nvx_nbr = 0;
  std::vector<double> vx_rec, vx_nbr;
  double *vtab = nullptr, *vnbr = nullptr;
  double vx_Kt = 0.0, vx_dtJ = 0.0;
  double* phase = nullptr;    // complex field: [re, im, max |phase - 1|] per chain
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
  int *piv = nullptr, *moves = nullptr;
  double* XA = nullptr;    // [X | right-hand sides] of the blocked LU solve, n x 3n
  double* Mgj = nullptr;   // multipliers of two consecutive panels, 2 x (n x 32)
  double* Uinv = nullptr;  // inverses of the diagonal blocks of U, 32 x 32 each, for the back substitution
  double *bins = nullptr, *prec_hist = nullptr, *prec_tot = nullptr, *logdet = nullptr;
  double *grad = nullptr, *gprec = nullptr;   // gradient rows [L][N] and the gradient pass's precision
  double* mpart = nullptr;                     // partial sums of the equal-time estimators
  double* draws = nullptr;                     // (u, Delta, prefactor, s_new) per site of the current pass
  // time-displaced pass: GT0 and H = G0T^T (two buffers each), the 2N-column
  // right-hand sides of the re-anchoring solve, S(K, tau) of the current
  // configuration and its bin sums, partial records, A_a(0); the momentum
  // phases and orbital map are shared
  double *TD[4] = {}, *tdS = nullptr, *tdbins = nullptr, *tdpart = nullptr, *a00 = nullptr;
  double* kph = nullptr;
  int* korb = nullptr;
  int td_norb = 0, td_cells = 0;
  // lattice-resolved equal-time correlations: the sublattice signs and the
  // orbital of (cell, orbital) are shared, the bin sums per chain
  double *eq_sign = nullptr, *eq_bins = nullptr;
  int* eq_site = nullptr;
  int eq_L1 = 0, eq_L2 = 0, eq_norb = 0;
  // the same correlations between tau and 0 in the time-displaced pass (single
  // chains only): [L+1] blocks of td_corr_stride doubles, then the count, and
  // the diagonal of G00
  double *td_corr = nullptr, *td_g00 = nullptr;
  bool td_corr_now = false;
  unsigned long long* counters = nullptr;   // proposals, accepted, sweep counter, key, Langevin step
  int* err_flag = nullptr;
  size_t work_doubles = 0;
  // batching: nch chains with identical models except the seed; every
  // per-chain buffer of chain i sits at (its chain-0 address) + i * cs doubles;
  // the exponentials and the identity UDV in [shared_lo, shared_hi) are common
  int nch = 1;
  size_t cs = 0;
  const double *shared_lo = nullptr, *shared_hi = nullptr;
  int gemm_tile = 0;
  // chunks of slices in one launch per chain with G in LDS (n <= kChunkMaxN):
  // 1 always, 0 never, -1 for groups of at least kChunkMinChains chains
  int fused = -1;
  std::vector<uint64_t> seeds;
  double* gbuf = nullptr;
  // optional per-launch event timing of one kernel (every timing_every-th launch)
  bool timing = false, timing_open = false;
  int timing_kernel = 0, timing_every = 1;
  uint64_t timing_seen = 0;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  double timed_flops = 0.0;
  // single chains: a second stream (default priority) on which the
  // time-displaced pass runs the next checkpoint's QR beside the current
  // re-anchoring, joined by events
  hipStream_t side = nullptr;
  hipEvent_t fork_ev[3] = {};
  // single chains of the one-flavour real sweep: the time-displaced pass at
  // the start of a sweep runs on the second stream beside the sweep itself,
  // as a context of its own over the shadow part of the work buffer (its
  // scratch), reading the chain's G, field and stored left forms; it records
  // td_ev[0] once it has read G, td_ev[k] once it has re-anchored at
  // checkpoint k (the last read of slot k) and td_ev[nk] at its end
  bool no_shadow = false;            // contexts that never run it that way
  double* shadow_base = nullptr;
  dqmc_ctx* tdc = nullptr;
  hipStream_t side2 = nullptr;       // the pass's own second stream for its checkpoint QRs
  std::vector<hipEvent_t> td_ev;
  std::vector<hipEvent_t>* td_sync = nullptr;   // in the pass's context: the events it records
  ~dqmc_ctx() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : fork_ev)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : td_ev) (void)hipEventDestroy(e);
    delete tdc;
    if (side) (void)hipStreamDestroy(side);
    if (side2) (void)hipStreamDestroy(side2);
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

constexpr int kEqMaxOrb = 4;   // orbitals per unit cell of the lattice-resolved correlations
// per-chain counters: [0] proposals, [1] accepted, [2] sweep counter, [3] Philox
// key, [4] Langevin step counter (the rest reserved)
constexpr int kCounters = 8;
// Four correlators of N_cells * norb^2 entries each (at most 4 N kEqMaxOrb), then the
// count, then <S^z> per orbital.
inline size_t eq_bins_size(const dqmc_ctx* c) { return 4 * (size_t)c->N * kEqMaxOrb + 8; }
inline size_t td_corr_stride(const dqmc_ctx* c) { return 4 * (size_t)c->N * kEqMaxOrb; }
// inverted diagonal blocks of the LU solve: one 32 x 32 matrix per block of
// the narrowest panel width (8), so the size does not depend on the width chosen
inline size_t uinv_size(const dqmc_ctx* c) { return ((size_t)c->N + 7) / 8 * 1024; }
// partial records of the time-displaced estimator, then its completion counter
inline size_t td_part_size(const dqmc_ctx* c) { return ((size_t)c->N + kTdRows - 1) / kTdRows * kTdPart + 4; }
inline size_t td_corr_size(const dqmc_ctx* c) {
  return c->nch == 1 ? (size_t)(c->L + 1) * td_corr_stride(c) + 4 : 0;
}

// Shared part: the exponentials, K and the identity UDV (one copy for all
// chains).  With base == nullptr only the size is computed and no pointer of
// the context is touched.
size_t layout_shared(dqmc_ctx* c, double* base) {
  const size_t N = c->N, NN = N * N;
  Layout l;
  auto P = [&](double*& dst, size_t n) { const size_t o = l.take(n); if (base) dst = base + o; };
  P(c->E, NN); P(c->Einv, NN); P(c->Eh, NN); P(c->Ehinv, NN); P(c->Kd, NN);
  P(c->uid.Q, NN); P(c->uid.D, N); P(c->uid.T, NN);
  P(c->gbuf, 8 * (size_t)std::max(1, c->nch));   // contiguous staging of per-chain scalars
  P(c->kph, 2 * N);
  double* ko = nullptr;
  P(ko, N / 2 + 1);
  if (base) c->korb = reinterpret_cast<int*>(ko);
  P(c->eq_sign, N);
  double* es = nullptr;
  P(es, N / 2 + 1);
  if (base) c->eq_site = reinterpret_cast<int*>(es);
  if (c->nvx > 0) {
    P(c->vtab, (size_t)c->nvx * kVxRec);
    P(c->vnbr, (size_t)std::max(1, c->nvx_nbr));
  }
  if (base) { c->shared_lo = base; c->shared_hi = base + l.off; }
  return l.off;
}

// Per-chain scratch (same convention for base == nullptr).
size_t layout_chain(dqmc_ctx* c, double* base) {
  const size_t N = c->N, NN = N * N;
  Layout l;
  auto P = [&](double*& dst, size_t n) { const size_t o = l.take(n); if (base) dst = base + o; };
  for (int i = 0; i < 6; ++i) P(c->S[i], NN);
  P(c->Vall, NN); P(c->VTall, NN); P(c->Zq, NN); P(c->Rt, NN);
  P(c->X, NN); P(c->RHS, NN); P(c->Gs, NN); P(c->T1, NN);
  UDVp* us[3] = {&c->cur, &c->hA, &c->hB};
  for (UDVp* u : us) { P(u->Q, NN); P(u->D, N); P(u->T, NN); }
  P(c->G2, NN);
  P(c->XA, 3 * NN);
  P(c->Mgj, 64 * N);
  P(c->Uinv, uinv_size(c));
  P(c->field_alt, (size_t)c->L * N);
  P(c->field_x, c->nfl == 2 ? (size_t)c->L * N : 0);
  P(c->norms, N);
  double* pv = nullptr;
  double* mv = nullptr;
  P(pv, N); P(mv, kLuMoves + 1);   // the move lists of two consecutive panels
  P(c->bins, 4);
  P(c->prec_hist, 2 * (size_t)c->nk + 2);
  P(c->prec_tot, 4);
  P(c->logdet, 4);
  P(c->phase, 4);
  P(c->grad, (size_t)c->L * N);
  P(c->gprec, 4);
  P(c->mpart, 4 * (size_t)((N + kMeasRows - 1) / kMeasRows) + 4);   // partials, then the counter
  P(c->draws, 4 * (size_t)c->L * N);
  for (int i = 0; i < 4; ++i) P(c->TD[i], NN);
  P(c->tdS, (size_t)(c->L + 1) * kTdStride);
  P(c->tdbins, (size_t)(c->L + 1) * kTdStride + 4);
  P(c->tdpart, td_part_size(c));
  P(c->a00, 2 * kTdMaxOrb);
  P(c->eq_bins, eq_bins_size(c));
  P(c->td_g00, N);
  P(c->td_corr, td_corr_size(c));
  double* ctr = nullptr;
  double* ef = nullptr;
  P(ctr, kCounters); P(ef, 1);
  if (base) {
    c->piv = reinterpret_cast<int*>(pv);
    c->moves = reinterpret_cast<int*>(mv);
    c->counters = reinterpret_cast<unsigned long long*>(ctr);
    c->err_flag = reinterpret_cast<int*>(ef);
  }
  return l.off;
}

inline bool wants_shadow(const dqmc_ctx* c) {
  return c->nch == 1 && !c->cplx && c->nfl == 1 && !c->nvx && !c->no_shadow;
}

// Shared part, the chain's scratch and, for a single chain of the one-flavour
// real sweep, a second copy of the chain's scratch for the time-displaced
// pass that runs beside the sweep (shadow_base).
size_t layout_work(dqmc_ctx* c, bool assign) {
  const size_t sh = layout_shared(c, assign ? c->work : nullptr);
  const size_t ch = layout_chain(c, assign ? c->work + sh : nullptr);
  size_t total = sh + ch;
  if (wants_shadow(c)) {
    total = (total + 31) & ~size_t(31);
    if (assign) c->shadow_base = c->work + total;
    total += ch;
  }
  return total;
}

inline unsigned grid1(size_t n, unsigned bs = 256) { return (unsigned)((n + bs - 1) / bs); }
inline dim3 gridc(const dqmc_ctx* c, unsigned x) { return dim3(x, (unsigned)c->nch); }
inline bool is_shared(const dqmc_ctx* c, const void* p) {
  const double* q = static_cast<const double*>(p);
  return q && q >= c->shared_lo && q < c->shared_hi;
}

// ---------------------------------------------------------- device steps --
dqmc_status timing_begin(dqmc_ctx* c, int kernel) {
  if (!c->timing || c->timing_kernel != kernel) return DQMC_OK;
  c->timing_open = (c->timing_seen++ % (uint64_t)c->timing_every) == 0;
  if (!c->timing_open) return DQMC_OK;
  while (c->ev.size() < c->ev_used + 2) {
    // Timing-only events: no system-scope fence (cache writeback) at record,
    // which would otherwise be counted in every bracketed launch.
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    c->ev.push_back(e);
  }
  HIPCHK(hipEventRecord(c->ev[c->ev_used], c->stream));
  return DQMC_OK;
}

dqmc_status timing_end(dqmc_ctx* c, int kernel) {
  if (!c->timing || c->timing_kernel != kernel || !c->timing_open) return DQMC_OK;
  c->timing_open = false;
  HIPCHK(hipEventRecord(c->ev[c->ev_used + 1], c->stream));
  c->ev_used += 2;
  return DQMC_OK;
}

dqmc_status gemm(dqmc_ctx* c, GemmArgs g) {
  g.nch = c->nch;
  g.tile = c->gemm_tile;
  g.cstride = c->cs;
  g.pc = 0;
  if (c->cs) {
    if (!is_shared(c, g.A)) g.pc |= PC_A;
    if (!is_shared(c, g.B)) g.pc |= PC_B;
    if (!is_shared(c, g.C)) g.pc |= PC_C;
    if (g.rs && !is_shared(c, g.rs)) g.pc |= PC_RS;
    if (g.cs && !is_shared(c, g.cs)) g.pc |= PC_CS;
    if (g.ks && !is_shared(c, g.ks)) g.pc |= PC_KS;
  }
  if (dqmc_status s = timing_begin(c, DQMC_KERNEL_GEMM)) return s;
  HIPCHK(launch_gemm(g, c->stream));
  if (c->timing_open && c->timing_kernel == DQMC_KERNEL_GEMM) c->timed_flops += 2.0 * g.M * (double)g.N * g.K * c->nch;
  return timing_end(c, DQMC_KERNEL_GEMM);
}

// Up to three independent products of the same shape in one launch.
dqmc_status gemm_group(dqmc_ctx* c, GemmArgs* gs, int count) {
  GemmGroup gg;
  double flops = 0.0;
  for (int i = 0; i < count; ++i) {
    GemmArgs g = gs[i];
    g.nch = c->nch;
    g.tile = c->gemm_tile;
    g.cstride = c->cs;
    g.pc = 0;
    if (c->cs) {
      if (!is_shared(c, g.A)) g.pc |= PC_A;
      if (!is_shared(c, g.B)) g.pc |= PC_B;
      if (!is_shared(c, g.C)) g.pc |= PC_C;
      if (g.rs && !is_shared(c, g.rs)) g.pc |= PC_RS;
      if (g.cs && !is_shared(c, g.cs)) g.pc |= PC_CS;
      if (g.ks && !is_shared(c, g.ks)) g.pc |= PC_KS;
    }
    if (g.M != gs[0].M || g.N != gs[0].N) return fail(c, DQMC_E_ARG, "grouped products of different shapes");
    gg.g[i] = g;
    flops += 2.0 * g.M * (double)g.N * g.K * c->nch;
  }
  if (dqmc_status s = timing_begin(c, DQMC_KERNEL_GEMM)) return s;
  HIPCHK(launch_gemm_group(gg, count, c->stream));
  if (c->timing_open && c->timing_kernel == DQMC_KERNEL_GEMM) c->timed_flops += flops;
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
  // one chain's scratch serves as workspace; the result is shared
  hipLaunchKernelGGL(k_set_identity, dim3(grid1((size_t)N * N)), dim3(256), 0, c->stream, P0, N, N, (size_t)0);
  HIPCHK(hipGetLastError());
  for (int k = 18; k >= 1; --k) {   // P <- I + (a K / k) P
    GemmArgs g = gemm_args(N, N, N, c->Kd, N, 0, P0, N, 0, P1, N, a / k, 0.0);
    g.diag_add = 1.0;
    HIPCHK(launch_gemm(g, c->stream));
    std::swap(P0, P1);
  }
  for (int k = 0; k < sq; ++k) {
    HIPCHK(launch_gemm(gemm_args(N, N, N, P0, N, 0, P0, N, 0, P1, N), c->stream));
    std::swap(P0, P1);
  }
  hipLaunchKernelGGL(k_copy, dim3(grid1((size_t)N * N)), dim3(256), 0, c->stream, out, P0, (size_t)N * N, (size_t)0);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

// Current location of field row tau: the upward pass writes its rows to
// field_alt, the downward pass writes them back to the caller's field buffer
// (so no launch reads and writes the same sites).
inline double* field_row(dqmc_ctx* c, int tau) {
  double* base = (!c->row_alt.empty() && c->row_alt[tau - 1]) ? c->field_alt : c->field;
  return base + (size_t)(tau - 1) * c->Nf;
}

// The N values that scale the rows or columns of slice tau's exp(V): the
// field row, or for two flavours its expansion [s, -s].
inline double* scale_row(dqmc_ctx* c, int tau) {
  return c->nfl == 2 ? c->field_x + (size_t)(tau - 1) * c->N : field_row(c, tau);
}

// G(tau) = B_tau G(tau-1) B_tau^-1 = diag(v) E G Einv diag(1/v), v = exp(coupling s_tau),
// from Gcur into dst (which may be Gcur itself)
dqmc_status wrap_up(dqmc_ctx* c, int tau, double* dst) {
  const int N = c->N;
  if (dqmc_status s = gemm(c, gemm_args(N, N, N, c->E, N, 0, c->Gcur, N, 0, c->T1, N))) return s;
  GemmArgs g = gemm_args(N, N, N, c->T1, N, 0, c->Einv, N, 0, dst, N);
  c->Gcur = dst;
  g.rs = scale_row(c, tau); g.rs_mode = SC_EXP; g.rs_coef = c->m.coupling;
  g.cs = scale_row(c, tau); g.cs_mode = SC_EXP; g.cs_coef = -c->m.coupling;
  return gemm(c, g);
}

// G(tau-1) = B_tau^-1 G(tau) B_tau = Einv diag(1/v) G diag(v) E, written to dst
dqmc_status wrap_down(dqmc_ctx* c, int tau, double* dst) {
  const int N = c->N;
  GemmArgs g1 = gemm_args(N, N, N, c->Gcur, N, 0, c->E, N, 0, c->T1, N);
  g1.ks = scale_row(c, tau); g1.ks_mode = SC_EXP; g1.ks_coef = c->m.coupling;
  if (dqmc_status s = gemm(c, g1)) return s;
  GemmArgs g2 = gemm_args(N, N, N, c->Einv, N, 0, c->T1, N, 0, dst, N);
  g2.ks = scale_row(c, tau); g2.ks_mode = SC_EXP; g2.ks_coef = -c->m.coupling;
  if (dqmc_status s = gemm(c, g2)) return s;
  c->Gcur = dst;
  return DQMC_OK;
}

// Sequential flips of slice tau, one fused launch per block of 32 sites; G
// alternates between the two buffers, the field row moves to the other buffer.
dqmc_status update_slice(dqmc_ctx* c, int tau) {
  const int N = c->N;
  const double* fin = field_row(c, tau);
  c->row_alt[tau - 1] ^= 1;
  double* fout = field_row(c, tau);
  const int tiles = ((N + 31) / 32) * ((N + 31) / 32);
  // a single large chain: 64-row tiles, one workgroup per CU at N = 648;
  // batches of N >= 96: 128-row tiles, a quarter of the workgroups repeating
  // each block's decisions
  const bool tall = c->nch == 1 && N > kWideMinN;
  const bool tall4 = c->nch > 1 && N >= 96;
  const int tiles64 = ((N + 63) / 64) * ((N + 31) / 32);
  const int tiles128 = ((N + 127) / 128) * ((N + 31) / 32);
  for (int s0 = 0; s0 < N; s0 += kBlock) {
    BlockArgs a;
    a.Gin = c->Gcur;
    a.Gout = (c->Gcur == c->G) ? c->G2 : c->G;
    a.N = N; a.s0 = s0; a.bb = std::min(kBlock, N - s0);
    a.field_in = fin; a.field_out = fout;
    a.draws = c->draws + 4 * (size_t)(tau - 1) * N;
    a.counters = c->counters;
    a.cs = c->cs;
    if (dqmc_status s = timing_begin(c, DQMC_KERNEL_BLOCK_UPDATE)) return s;
    if (tall4 && c->m.n_col == 2)
      hipLaunchKernelGGL((k_block_update<2, 128>), gridc(c, tiles128), dim3(1024), 0, c->stream, a);
    else if (tall4)
      hipLaunchKernelGGL((k_block_update<1, 128>), gridc(c, tiles128), dim3(1024), 0, c->stream, a);
    else if (tall && c->m.n_col == 2)
      hipLaunchKernelGGL((k_block_update<2, 64>), gridc(c, tiles64), dim3(512), 0, c->stream, a);
    else if (tall)
      hipLaunchKernelGGL((k_block_update<1, 64>), gridc(c, tiles64), dim3(512), 0, c->stream, a);
    else if (c->m.n_col == 2)
      hipLaunchKernelGGL(k_block_update<2>, gridc(c, tiles), dim3(256), 0, c->stream, a);
    else
      hipLaunchKernelGGL(k_block_update<1>, gridc(c, tiles), dim3(256), 0, c->stream, a);
    HIPCHK(hipGetLastError());
    if (dqmc_status s = timing_end(c, DQMC_KERNEL_BLOCK_UPDATE)) return s;
    c->Gcur = a.Gout;
  }
  return DQMC_OK;
}

// ---------------------------------------------------- UDV stabilisation --
// One QR step (k_qr_panel): the panel at j0 and, when there is a previous
// panel (its factors at V - nb N, VT - nb N), that panel's block applied to
// this panel's columns in the same workgroup and to the ntr columns right of
// this panel by ntr / 16 more workgroups.
template <int NBW, int MAXR>
void qr_panel_launch(dqmc_ctx* c, double* Ap, int j0, int nbw, double* V, double* VT) {
  const int N = c->N;
  const bool prev = j0 > 0;
  const double* Vp = prev ? V - (size_t)NBW * N : nullptr;
  const double* VTp = prev ? VT - (size_t)NBW * N : nullptr;
  const int ntr = prev ? N - j0 - nbw : 0;
  double* At = prev ? Ap + (size_t)(j0 - NBW) * N + j0 + nbw : nullptr;
  const unsigned gx = 1 + (unsigned)((ntr + 15) / 16);
  hipLaunchKernelGGL((k_qr_panel<NBW, MAXR>), gridc(c, gx), dim3(256), sizeof(double) * qr_panel_lds<NBW>(64 * MAXR),
                     c->stream, Ap, N, j0, nbw, V, VT, Vp, VTp, At, ntr, c->cs);
}

// rows per lane = ceil(h / 64), rounded up to the instantiated counts; the
// panel width is 32 for N <= kNarrowMaxN, 16 for N <= 768, 8 above (set in create)
dqmc_status launch_qr_panel(dqmc_ctx* c, double* Ap, int j0, int nbw, double* V, double* VT) {
  const int rows = (c->N - j0 + 63) / 64;
  if (c->nb == 32 && rows <= 2) qr_panel_launch<32, 2>(c, Ap, j0, nbw, V, VT);
  else if (c->nb == 32 && rows <= 4) qr_panel_launch<32, 4>(c, Ap, j0, nbw, V, VT);
  else if (c->nb == 32 && rows <= 6) qr_panel_launch<32, 6>(c, Ap, j0, nbw, V, VT);
  else if (c->nb == 16 && rows <= 4) qr_panel_launch<16, 4>(c, Ap, j0, nbw, V, VT);
  else if (c->nb == 16 && rows <= 8) qr_panel_launch<16, 8>(c, Ap, j0, nbw, V, VT);
  else if (c->nb == 16 && rows <= 12) qr_panel_launch<16, 12>(c, Ap, j0, nbw, V, VT);
  else if (c->nb == 8 && rows <= 4) qr_panel_launch<8, 4>(c, Ap, j0, nbw, V, VT);
  else if (c->nb == 8 && rows <= 8) qr_panel_launch<8, 8>(c, Ap, j0, nbw, V, VT);
  else if (c->nb == 8 && rows <= 16) qr_panel_launch<8, 16>(c, Ap, j0, nbw, V, VT);
  else return fail(c, DQMC_E_UNSUPPORTED, "no QR panel kernel for this size");
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

// One step s of the blocked LU solve (k_lu_step): panel s at j0 (width nbw,
// when has_panel) and the previous panel's step on its columns and, in other
// workgroups, on the columns from tstart to ncols - 1.  Multipliers and move
// lists alternate between two buffers by step parity.
struct LuStep {
  int j0, nbw, has_panel, j0p, nbp, tstart, ncols, s;
};

template <int NBW, int MR>
void lu_step_launch(dqmc_ctx* c, double* XA, int ld, const LuStep& q) {
  const int N = c->N;
  double* M = c->Mgj + (size_t)(q.s & 1) * 32 * N;
  int* moves = c->moves + (size_t)(q.s & 1) * kLuMoves;
  const bool prev = q.s > 0;
  const double* Mp = prev ? c->Mgj + (size_t)((q.s - 1) & 1) * 32 * N : nullptr;
  const int* movesp = prev ? c->moves + (size_t)((q.s - 1) & 1) * kLuMoves : nullptr;
  const int nT = prev ? (q.ncols - q.tstart + 15) / 16 : 0;
  const size_t lds = q.has_panel ? sizeof(double) * (size_t)(N - q.j0) * (NBW + 1) : 0;   // the staged panel
  const unsigned gx = (unsigned)((q.has_panel ? 1 : 0) + nT);
  hipLaunchKernelGGL((k_lu_step<NBW, MR>), gridc(c, gx), dim3(256), lds, c->stream, XA, N, ld, q.j0, q.nbw, M, moves,
                     q.has_panel, q.j0p, q.nbp, Mp, movesp, q.tstart, q.ncols, c->err_flag, c->cs);
}

// rows per thread = ceil(h / 256) of the panel
dqmc_status launch_lu_step(dqmc_ctx* c, double* XA, int ld, const LuStep& q) {
  const int rows = q.has_panel ? (c->N - q.j0 + 255) / 256 : 1;
  if (c->nb == 32 && rows <= 1) lu_step_launch<32, 1>(c, XA, ld, q);
  else if (c->nb == 32 && rows <= 2) lu_step_launch<32, 2>(c, XA, ld, q);
  else if (c->nb == 16 && rows <= 1) lu_step_launch<16, 1>(c, XA, ld, q);
  else if (c->nb == 16 && rows <= 2) lu_step_launch<16, 2>(c, XA, ld, q);
  else if (c->nb == 16 && rows <= 3) lu_step_launch<16, 3>(c, XA, ld, q);
  else if (c->nb == 8 && rows <= 1) lu_step_launch<8, 1>(c, XA, ld, q);
  else if (c->nb == 8 && rows <= 2) lu_step_launch<8, 2>(c, XA, ld, q);
  else if (c->nb == 8 && rows <= 3) lu_step_launch<8, 3>(c, XA, ld, q);
  else if (c->nb == 8 && rows <= 4) lu_step_launch<8, 4>(c, XA, ld, q);
  else return fail(c, DQMC_E_UNSUPPORTED, "no LU step kernel for this size");
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

// each QR panel instance's dynamic LDS limit: exactly what its launch asks for
// (the static apply_wy_slab scratch comes on top, within the 160 KB of a CU)
template <int NBW, int R1, int R2, int R3>
hipError_t lds_limit_qr() {
  const void* fns[] = {reinterpret_cast<const void*>(k_qr_panel<NBW, R1>),
                       reinterpret_cast<const void*>(k_qr_panel<NBW, R2>),
                       reinterpret_cast<const void*>(k_qr_panel<NBW, R3>)};
  const int rows[] = {R1, R2, R3};
  for (int i = 0; i < 3; ++i) {
    hipError_t e = hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(sizeof(double) * qr_panel_lds<NBW>(64 * rows[i])));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int NBW, int MR>
hipError_t lds_limit_lu() {
  // the staged panel: at most 256 x 33, 768 x 17 or 1024 x 9 doubles (about
  // 104 KB), beside about 24 KB of static LDS
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k_lu_step<NBW, MR>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, 108 * 1024);
}

dqmc_status set_lds_limits(dqmc_ctx* c) {
  HIPCHK((lds_limit_lu<32, 1>()));
  HIPCHK((lds_limit_lu<32, 2>()));
  HIPCHK((lds_limit_lu<16, 1>()));
  HIPCHK((lds_limit_lu<16, 2>()));
  HIPCHK((lds_limit_lu<16, 3>()));
  HIPCHK((lds_limit_lu<8, 1>()));
  HIPCHK((lds_limit_lu<8, 2>()));
  HIPCHK((lds_limit_lu<8, 3>()));
  HIPCHK((lds_limit_lu<8, 4>()));
  HIPCHK((lds_limit_qr<32, 2, 4, 6>()));
  HIPCHK((lds_limit_qr<16, 4, 8, 12>()));
  HIPCHK((lds_limit_qr<8, 4, 8, 16>()));
  HIPCHK(gemm64_set_lds());
  HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_accum_q), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(sizeof(double) * 16 * (size_t)c->N)));
  if (c->N > kWideMinN && c->N <= kBackWideMaxN)
    HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_lu_back_wide),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)back_wide_lds(c->N)));
  if (c->N > kWideMinN && c->N <= kAccumWideMaxN) {
    HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_accum_q_wide<1>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)accum_q_lds<1>(c->N)));
    if (c->N <= kAccumPairMaxN)
      HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_accum_q_wide<2>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)accum_q_lds<2>(c->N)));
  }
  if (!c->cplx && c->N <= kChunkMaxN) {
    const void* fns[] = {reinterpret_cast<const void*>(k_chunk<1>), reinterpret_cast<const void*>(k_chunk<2>),
                         reinterpret_cast<const void*>(k_chunk<3>), reinterpret_cast<const void*>(k_chunk<4>)};
    HIPCHK(hipFuncSetAttribute(fns[chunk_np(c->N) / 16 - 1], hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)chunk_lds(c->N, 1)));
  }
  if (c->nfl == 2)
    HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_fl2_update_slice),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)fl2_update_lds(kFl2MaxN)));
  if (c->cplx)
    HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_cupdate_slice),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)cupdate_lds(kCMaxN)));
  if (c->nvx)
    HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_vx_slice), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)vx_slice_lds(kVxMaxN, kVxMaxM, kVxMaxNbr)));
  return DQMC_OK;
}

// QR of M (N x N, overwritten) with column pre-pivoting: M P = Q R.  Writes
// Q, D = |diag R| and T_out = D^-1 R P^T T_in.
dqmc_status qr_udv(dqmc_ctx* c, double* M, const double* T_in, UDVp out) {
  const int N = c->N, nb = c->nb;
  double* Ap = c->S[4];
  // column norms (partial rows in Zq, free until the trailing updates), then the ranks
  const int nrb = (N + kColRows - 1) / kColRows;
  hipLaunchKernelGGL(k_colnorm_part, gridc(c, (unsigned)nrb), dim3(256), 0, c->stream, M, N, c->Zq, c->cs);
  hipLaunchKernelGGL(k_colnorm_order, gridc(c, 1), dim3(1024), 0, c->stream, c->Zq, nrb, N, c->norms, c->piv, c->cs);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_permute_cols, gridc(c, grid1((size_t)N * N)), dim3(256), 0, c->stream, Ap, M, c->piv, N,
                     c->cs);
  HIPCHK(hipGetLastError());
  // one launch per panel: each applies the previous panel's reflectors (to
  // its own columns and, in other workgroups, to the rest) and factorises
  for (int j0 = 0; j0 < N; j0 += nb) {
    const int nbw = std::min(nb, N - j0);
    double* V = c->Vall + (size_t)j0 * N;
    double* VT = c->VTall + (size_t)j0 * N;
    if (dqmc_status s = launch_qr_panel(c, Ap, j0, nbw, V, VT)) return s;
  }
  // explicit Q by backward accumulation of the block reflectors, every
  // 16-column slab through all panels in one launch
  // the sixteen-wave accumulation pays for the tall 16-wide panels of large N
  // and a lone chain leaves the chip idle; batches keep the four-wave kernel
  if (N > kWideMinN && N <= kAccumWideMaxN && c->nch == 1) {
    if (nb > 16) {
      hipLaunchKernelGGL(k_accum_q_wide<2>, gridc(c, (unsigned)((N + 15) / 16)), dim3(64 * kAccumWaves),
                         accum_q_lds<2>(N), c->stream, c->Vall, c->VTall, out.Q, N, nb, c->cs);
    } else if (N <= kAccumPairMaxN) {
      // pairs of 16-column panels joined into 32-column blocks (in Zq and Rt,
      // both free here): 21 dependent steps instead of 41 at N = 648
      hipLaunchKernelGGL(k_wy_pair, gridc(c, (unsigned)((N + 31) / 32)), dim3(64 * kPairWaves), 0, c->stream, c->Vall, c->VTall,
                         c->Zq, c->Rt, N, c->cs);
      hipLaunchKernelGGL(k_accum_q_wide<2>, gridc(c, (unsigned)((N + 15) / 16)), dim3(64 * kAccumWaves),
                         accum_q_lds<2>(N), c->stream, c->Zq, c->Rt, out.Q, N, 32, c->cs);
    } else
      hipLaunchKernelGGL(k_accum_q_wide<1>, gridc(c, (unsigned)((N + 15) / 16)), dim3(64 * kAccumWaves),
                         accum_q_lds<1>(N), c->stream, c->Vall, c->VTall, out.Q, N, nb, c->cs);
  } else {
    hipLaunchKernelGGL(k_accum_q, gridc(c, (unsigned)((N + 15) / 16)), dim3(256), sizeof(double) * 16 * (size_t)N,
                       c->stream, c->Vall, c->VTall, out.Q, N, nb, c->cs);
  }
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_build_rt, gridc(c, grid1((size_t)N * N)), dim3(256), 0, c->stream, Ap, c->piv, N, c->Rt,
                     out.D, c->err_flag, c->cs);
  HIPCHK(hipGetLastError());
  return gemm(c, gemm_args(N, N, N, c->Rt, N, 0, T_in, N, 0, out.T, N));
}

// Rotations of a complex field's images (k_crot): rows by diag(exp(i c_row eta)),
// columns by diag(exp(-i c_col eta)); a zero coefficient skips that side.
dqmc_status crot(dqmc_ctx* c, double* dst, const double* src, int tau, double coef_row, double coef_col) {
  const int n = c->Nf;
  hipLaunchKernelGGL(k_crot, gridc(c, grid1((size_t)n * n)), dim3(256), 0, c->stream, dst, src, n, c->N,
                     field_row(c, tau), coef_row, coef_col, coef_row != 0.0 ? 1 : 0, coef_col != 0.0 ? 1 : 0, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

// The vertex factors of slice tau on the rows (k_vx_rows): order 0 applies
// exp(V_tau), order 1 its transpose.
dqmc_status vx_rows(dqmc_ctx* c, const double* src, double* dst, int tau, int order) {
  hipLaunchKernelGGL(k_vx_rows, gridc(c, 1), dim3(256), vx_rows_lds(c->N, c->nvx), c->stream, src, dst, c->N, c->vtab,
                     c->nvx,
                     c->field + (size_t)(tau - 1) * c->Nf, order, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

// Right step: UDV of B(hi,0) from that of B(lo,0): M = (B_hi ... B_lo+1 Q) D.
dqmc_status right_step(dqmc_ctx* c, UDVp in, int lo, int hi, UDVp out) {
  const int N = c->N;
  const double* src = in.Q;
  double* bufs[2] = {c->S[2], c->S[3]};
  int b = 0;
  for (int tau = lo + 1; tau <= hi; ++tau) {
    GemmArgs g = gemm_args(N, N, N, c->E, N, 0, src, N, 0, bufs[b], N);
    if (!c->cplx && !c->nvx) { g.rs = scale_row(c, tau); g.rs_mode = SC_EXP; g.rs_coef = c->m.coupling; }
    if (tau == hi) { g.cs = in.D; g.cs_mode = SC_VAL; }
    if (dqmc_status s = gemm(c, g)) return s;
    // general vertices: B_tau = exp(V_tau) exp(-dtau K), the vertex factors on the rows
    if (c->nvx)
      if (dqmc_status s = vx_rows(c, bufs[b], bufs[b], tau, 0)) return s;
    // complex field: B_tau = diag(exp(i c eta)) E on the image, a row rotation
    if (c->cplx)
      if (dqmc_status s = crot(c, bufs[b], bufs[b], tau, c->m.coupling, 0.0)) return s;
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
    // complex field: the image of B_tau transposed is E times the rotation by
    // diag(exp(-i c eta)) of the rows, applied first (into S[5])
    if (c->cplx) {
      if (dqmc_status s = crot(c, c->S[5], src, tau, -c->m.coupling, 0.0)) return s;
      src = c->S[5];
    }
    // general vertices: B_tau^T = exp(-dtau K) exp(V_tau)^T, the vertex factors first
    if (c->nvx) {
      if (dqmc_status s = vx_rows(c, src, c->S[5], tau, 1)) return s;
      src = c->S[5];
    }
    GemmArgs g = gemm_args(N, N, N, c->E, N, 0, src, N, 0, bufs[b], N);
    if (!c->cplx && !c->nvx) { g.ks = scale_row(c, tau); g.ks_mode = SC_EXP; g.ks_coef = c->m.coupling; }
    if (tau == lo + 1) { g.cs = in.D; g.cs_mode = SC_VAL; }
    if (dqmc_status s = gemm(c, g)) return s;
    src = bufs[b];
    b ^= 1;
  }
  return qr_udv(c, const_cast<double*>(src), in.T, out);
}

// Solve X Y = R in place by blocked LU with partial pivoting, the forward
// substitution carried along as extra columns: XA = [X | R] is
// n x (n + nrhs) with leading dimension ld; Y replaces R.  If logdet is
// given, adds log|det X|.
dqmc_status lu_solve(dqmc_ctx* c, double* XA, int nrhs, int ld, double* logdet) {
  const int N = c->N, nb = c->nb, ncols = N + nrhs;
  // one launch per panel (its factorisation, with the previous panel's step
  // on all later columns beside it), then one for the last panel's step on
  // the right-hand sides
  const int np = (N + nb - 1) / nb;
  for (int s = 0; s <= np; ++s) {
    LuStep q;
    q.s = s;
    q.has_panel = s < np ? 1 : 0;
    q.j0 = s * nb;
    q.nbw = q.has_panel ? std::min(nb, N - q.j0) : 0;
    q.j0p = (s - 1) * nb;
    q.nbp = s > 0 ? std::min(nb, N - q.j0p) : 0;
    q.tstart = q.has_panel ? q.j0 + q.nbw : N;
    q.ncols = ncols;
    if (dqmc_status st = launch_lu_step(c, XA, ld, q)) return st;
  }
  // back substitution: the inverses of U's 32 x 32 diagonal blocks (U is
  // upper triangular, so any diagonal block is; 32 rows per step halve the
  // dependent steps of 16-column panels), then every 16-column slab of the
  // right-hand sides through the whole block recursion at once
  constexpr int bs = 32;
  const int nblk = (N + bs - 1) / bs;
  hipLaunchKernelGGL(k_lu_diag_inv, gridc(c, (unsigned)nblk), dim3(256), 0, c->stream, XA, N, ld, bs, c->Uinv, c->cs);
  if (N > kWideMinN && N <= kBackWideMaxN && c->nch == 1)   // likewise
    hipLaunchKernelGGL(k_lu_back_wide, gridc(c, (unsigned)((nrhs + kBackCols - 1) / kBackCols)), dim3(64 * kBackWaves),
                       back_wide_lds(N), c->stream, XA, N, ld, bs, nrhs, c->Uinv, c->cs);
  else
    hipLaunchKernelGGL(k_lu_back, gridc(c, (unsigned)((nrhs + kBackCols - 1) / kBackCols)), dim3(256), 0, c->stream,
                       XA, N, ld, bs, nrhs, c->Uinv, c->cs);
  HIPCHK(hipGetLastError());
  if (logdet) {
    hipLaunchKernelGGL(k_logabs_diag, gridc(c, 1), dim3(256), 0, c->stream, XA, N, ld, logdet, c->cs);
    HIPCHK(hipGetLastError());
  }
  return DQMC_OK;
}

// G = (1 + B(tau,0) B(beta,tau))^-1 from the right form (Q_R D_R T_R of
// B(tau,0)) and the left form (Q_L D_L T_L of B(beta,tau)^T):
//   X = D_Rb^-1 (Q_R^T Q_L) D_Lb^-1 + D_Rs (T_R T_L^T) D_Ls
//   G = Q_L D_Lb^-1 X^-1 D_Rb^-1 Q_R^T
dqmc_status merge(dqmc_ctx* c, UDVp R, UDVp Lf, double* Gout, double* logdet) {
  const int N = c->N, ld = 2 * N;   // XA = [X | D_Rb^-1 Q_R^T]
  GemmArgs g1 = gemm_args(N, N, N, R.Q, N, 1, Lf.Q, N, 0, c->XA, ld);
  g1.rs = R.D; g1.rs_mode = SC_INV_BIG; g1.cs = Lf.D; g1.cs_mode = SC_INV_BIG;
  if (dqmc_status s = gemm(c, g1)) return s;
  GemmArgs g2 = gemm_args(N, N, N, R.T, N, 0, Lf.T, N, 1, c->XA, ld, 1.0, 1.0);
  g2.rs = R.D; g2.rs_mode = SC_SMALL; g2.cs = Lf.D; g2.cs_mode = SC_SMALL;
  if (dqmc_status s = gemm(c, g2)) return s;
  const dim3 tg((N + 31) / 32, (N + 31) / 32, (unsigned)c->nch);
  // the right form may be the shared identity: offset it only when it is per chain
  hipLaunchKernelGGL(k_transpose_scale, tg, dim3(256), 0, c->stream, c->XA + N, ld, R.Q, N, R.D, SC_INV_BIG, c->cs,
                     is_shared(c, R.Q) ? (size_t)0 : c->cs);
  HIPCHK(hipGetLastError());
  if (logdet) {
    hipLaunchKernelGGL(k_logbig_sum, gridc(c, 1), dim3(256), 0, c->stream, R.D, N, logdet, 0,
                       is_shared(c, R.D) ? (size_t)0 : c->cs, c->cs);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_logbig_sum, gridc(c, 1), dim3(256), 0, c->stream, Lf.D, N, logdet, 1,
                       is_shared(c, Lf.D) ? (size_t)0 : c->cs, c->cs);
    HIPCHK(hipGetLastError());
  }
  if (dqmc_status s = lu_solve(c, c->XA, N, ld, logdet)) return s;
  GemmArgs g3 = gemm_args(N, N, N, Lf.Q, N, 0, c->XA + N, ld, 0, Gout, N);
  g3.ks = Lf.D; g3.ks_mode = SC_INV_BIG;
  return gemm(c, g3);
}

dqmc_status copy_udv(dqmc_ctx* c, UDVp dst, UDVp src) {
  const size_t NN = (size_t)c->N * c->N;
  hipLaunchKernelGGL(k_copy, gridc(c, grid1(NN)), dim3(256), 0, c->stream, dst.Q, src.Q, NN, c->cs);
  hipLaunchKernelGGL(k_copy, gridc(c, grid1(c->N)), dim3(256), 0, c->stream, dst.D, src.D, (size_t)c->N, c->cs);
  hipLaunchKernelGGL(k_copy, gridc(c, grid1(NN)), dim3(256), 0, c->stream, dst.T, src.T, NN, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

dqmc_status stabilise(dqmc_ctx* c, int hist_index) {
  const size_t NN = (size_t)c->N * c->N;
  hipLaunchKernelGGL(k_prec_replace, gridc(c, prec_grid(NN)), dim3(256), 0, c->stream,
                     c->Gcur, c->G, c->Gs, NN, c->prec_hist + hist_index, c->err_flag, c->cs);
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
  const int rows = N <= kMeasSmallN ? N : kMeasRows;
  const int nblk = (N + rows - 1) / rows;
  if (T1)
    hipLaunchKernelGGL(k_measure_part<true>, gridc(c, (unsigned)nblk), dim3(256), 0, c->stream, c->Gcur, T1, c->Ehinv,
                       c->Kd, N, rows, c->mpart, c->trK, (double)c->m.n_col, c->m.u_int, c->bins, c->err_flag, c->cs);
  else
    hipLaunchKernelGGL(k_measure_part<false>, gridc(c, (unsigned)nblk), dim3(256), 0, c->stream, c->Gcur, T1,
                       c->Ehinv, c->Kd, N, rows, c->mpart, c->trK, (double)c->m.n_col, c->m.u_int, c->bins,
                       c->err_flag, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

// Lattice-resolved equal-time correlations of the current configuration,
// added to the bins, from G~ = e^{-dtau K/2} G e^{+dtau K/2} (symmetric split)
// or G (asymmetric split).  t1_ready: T1 already holds e^{-dtau K/2} G of this
// configuration (the equal-time estimators ran just before).
dqmc_status eq_measure(dqmc_ctx* c, bool t1_ready) {
  const int N = c->N;
  const double* Gt = c->Gcur;
  if (c->m.trotter == DQMC_TROTTER_SYM) {
    if (!t1_ready)
      if (dqmc_status s = gemm(c, gemm_args(N, N, N, c->Eh, N, 0, c->Gcur, N, 0, c->T1, N))) return s;
    if (dqmc_status s = gemm(c, gemm_args(N, N, N, c->T1, N, 0, c->Ehinv, N, 0, c->Gs, N))) return s;
    Gt = c->Gs;
  }
  const int nb = c->eq_L1 * c->eq_L2 * c->eq_norb * c->eq_norb;
  hipLaunchKernelGGL(k_corr<false>, gridc(c, grid1((size_t)nb + 1, 4)), dim3(256), 0, c->stream, Gt, nullptr, nullptr,
                     nullptr, N, c->eq_L1, c->eq_L2, c->eq_norb, c->eq_site, c->eq_sign, c->eq_bins,
                     c->eq_bins + 4 * (size_t)nb, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

// The four-valued field's values eta(l) and log gamma(l), l = -2, -1, +1, +2
// (Eq. (HS_squares)), computed on the host.
Field4 field4_table() {
  const double s6 = std::sqrt(6.0);
  const double e1 = std::sqrt(2.0 * (3.0 - s6)), e2 = std::sqrt(2.0 * (3.0 + s6));
  const double g1 = 1.0 + s6 / 3.0, g2 = 1.0 - s6 / 3.0;
  Field4 t;
  t.eta[0] = -e2; t.eta[1] = -e1; t.eta[2] = e1; t.eta[3] = e2;
  t.lg[0] = std::log(g2); t.lg[1] = std::log(g1); t.lg[2] = std::log(g1); t.lg[3] = std::log(g2);
  return t;
}

bool field_value_ok(dqmc_field_kind kind, double v) {
  if (!std::isfinite(v)) return false;
  if (kind == DQMC_FIELD_ISING) return v == 1.0 || v == -1.0;
  if (kind == DQMC_FIELD_ISING4 || kind == DQMC_FIELD_ISING4_IMAG) {
    const Field4 t = field4_table();
    return v == t.eta[0] || v == t.eta[1] || v == t.eta[2] || v == t.eta[3];
  }
  return true;
}

// Draws of every site of the coming pass, from the field as it stands (all
// rows at the same place: the caller's buffer before the upward pass, the
// second buffer before the downward pass).
dqmc_status pass_draws(dqmc_ctx* c, int dir) {
  const size_t n = (size_t)c->L * c->N;
  hipLaunchKernelGGL(k_pass_draws, gridc(c, grid1(n)), dim3(256), 0, c->stream, field_row(c, 1), c->L, c->N,
                     (unsigned long long)dir, c->m.coupling, c->m.alpha, c->m.n_col,
                     (int)c->m.field, c->m.prop_width, field4_table(), c->counters, c->draws, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

// One sweep (Algorithm 1): upward pass tau = 1..L, downward pass tau = L..1.
// meas: bit 0 = equal-time estimators on every slice, bit 1 = the
// time-displaced pass at the start of the sweep, bit 2 = the lattice-resolved
// equal-time correlations on every slice, bit 3 = the lattice-resolved
// time-displaced correlations in that pass.
dqmc_status td_pass(dqmc_ctx* c);

// The chunk kernel runs the sweep's slices between stabilisations when the
// lattice fits its LDS, for the equal-time estimators and the time-displaced
// pass (the lattice-resolved equal-time correlations take the blocked path),
// unless it is switched off or the block update is being timed.
// One workgroup per chain keeps a lone chain on one CU, where the blocked
// kernels spread it over many: the automatic choice takes the chunk kernel
// for groups of at least this many chains.
constexpr int kChunkMinChains = 16;

bool use_chunks(const dqmc_ctx* c, int meas) {
  const bool on = c->fused == 1 || (c->fused == -1 && c->nch >= kChunkMinChains);
  return on && !c->cplx && c->nfl == 1 && !c->nvx && c->N <= kChunkMaxN && !(meas & 4) &&
         !(c->timing && c->timing_kernel == DQMC_KERNEL_BLOCK_UPDATE);
}

template <int NT>
void launch_chunk_nt(const ChunkArgs& a, dim3 grid, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_chunk<NT>, grid, dim3(256), lds, s, a);
}

dqmc_status launch_chunk(dqmc_ctx* c, int tau0, int ntau, int dir, int measure, int skip_last) {
  ChunkArgs a;
  a.G = c->G; a.field = c->field;
  a.E = c->E; a.Einv = c->Einv; a.Eh = c->Eh; a.Ehinv = c->Ehinv; a.K = c->Kd;
  a.counters = c->counters; a.bins = c->bins; a.err = c->err_flag;
  a.N = c->N; a.tau0 = tau0; a.ntau = ntau; a.dir = dir;
  a.measure = measure; a.skip_last = skip_last;
  a.sym = c->m.trotter == DQMC_TROTTER_SYM ? 1 : 0;
  a.kind = (int)c->m.field; a.n_col = c->m.n_col;
  a.coupling = c->m.coupling; a.alpha = c->m.alpha; a.prop_width = c->m.prop_width;
  a.trK = c->trK; a.u_int = c->m.u_int;
  a.f4 = field4_table();
  a.cs = c->cs;
  const dim3 grid = gridc(c, 1);
  const size_t lds = chunk_lds(c->N, a.sym);
  switch (chunk_np(c->N) / 16) {
    case 1: launch_chunk_nt<1>(a, grid, lds, c->stream); break;
    case 2: launch_chunk_nt<2>(a, grid, lds, c->stream); break;
    case 3: launch_chunk_nt<3>(a, grid, lds, c->stream); break;
    case 4: launch_chunk_nt<4>(a, grid, lds, c->stream); break;
    default: return fail(c, DQMC_E_UNSUPPORTED, "lattice too large for the chunk kernel");
  }
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

// One sweep (Algorithm 1) with the slices of every chunk in one launch: the
// upward chunk k covers slices (k-1) n_wrap + 1 .. k n_wrap (measured but for
// the last, which is measured after its stabilisation), the downward chunk k
// slices (k+1) n_wrap .. k n_wrap + 1, each followed by the stabilisation step
// of the blocked sweep.
dqmc_status sweep_chunks(dqmc_ctx* c, int meas) {
  const int nw = c->nw, nk = c->nk;
  if (meas & 2) {
    c->td_corr_now = (meas & 8) != 0;
    const dqmc_status s = td_pass(c);
    c->td_corr_now = false;
    if (s) return s;
  }
  int hist = 0;
  c->row_alt.clear();
  c->Gcur = c->G;
  for (int k = 1; k <= nk; ++k) {
    if (dqmc_status s = launch_chunk(c, (k - 1) * nw + 1, nw, 0, meas & 1, 1)) return s;
    if (dqmc_status s = timing_begin(c, DQMC_KERNEL_STABILISE)) return s;
    UDVp prev = (k == 1) ? c->uid : c->slot(k - 1);
    if (dqmc_status s = right_step(c, prev, (k - 1) * nw, k * nw, c->cur)) return s;
    UDVp left = (k == nk) ? c->uid : c->slot(k);
    if (dqmc_status s = merge(c, c->cur, left, c->Gs, nullptr)) return s;
    if (dqmc_status s = copy_udv(c, c->slot(k), c->cur)) return s;
    if (dqmc_status s = stabilise(c, hist++)) return s;
    if (dqmc_status s = timing_end(c, DQMC_KERNEL_STABILISE)) return s;
    if (meas & 1)
      if (dqmc_status s = measure(c)) return s;
  }
  for (int k = nk - 1; k >= 0; --k) {
    if (dqmc_status s = launch_chunk(c, (k + 1) * nw, nw, 1, meas & 1, 0)) return s;
    if (dqmc_status s = timing_begin(c, DQMC_KERNEL_STABILISE)) return s;
    UDVp prev = (k + 1 == nk) ? c->uid : c->slot(k + 1);
    if (dqmc_status s = left_step(c, prev, k * nw, (k + 1) * nw, c->cur)) return s;
    UDVp right = (k == 0) ? c->uid : c->slot(k);
    if (dqmc_status s = merge(c, right, c->cur, c->Gs, nullptr)) return s;
    if (dqmc_status s = copy_udv(c, c->slot(k), c->cur)) return s;
    if (dqmc_status s = stabilise(c, hist++)) return s;
    if (dqmc_status s = timing_end(c, DQMC_KERNEL_STABILISE)) return s;
  }
  hipLaunchKernelGGL(k_finish_sweep, gridc(c, 1), dim3(64), 0, c->stream, c->prec_hist, hist, c->prec_tot,
                     c->m.prec_threshold, c->counters, c->err_flag, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

dqmc_status td_pass_async(dqmc_ctx* c);

// The second stream serves a single chain whose stream is not being captured
// into a graph.
bool side_ok(dqmc_ctx* c) {
  if (!c->side || c->nch != 1) return false;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(c->stream, &cap) != hipSuccess) return false;
  return cap == hipStreamCaptureStatusNone;
}

dqmc_status sweep_once(dqmc_ctx* c, int meas) {
  if (use_chunks(c, meas)) return sweep_chunks(c, meas);
  const int L = c->L, nw = c->nw, nk = c->nk;
  const bool async_td = (meas & 2) && c->tdc && c->shadow_base && c->side2 && side_ok(c);
  if (meas & 2) {
    c->td_corr_now = (meas & 8) != 0;
    const dqmc_status s = async_td ? td_pass_async(c) : td_pass(c);
    c->td_corr_now = false;
    if (s) return s;
  }
  int hist = 0;
  c->row_alt.assign(L, 0);
  c->Gcur = c->G;
  if (dqmc_status s = pass_draws(c, 0)) return s;
  for (int tau = 1; tau <= L; ++tau) {
    if (dqmc_status s = wrap_up(c, tau, c->G)) return s;
    if (dqmc_status s = update_slice(c, tau)) return s;
    if (tau % nw == 0) {
      const int k = tau / nw;
      if (dqmc_status s = timing_begin(c, DQMC_KERNEL_STABILISE)) return s;
      UDVp prev = (k == 1) ? c->uid : c->slot(k - 1);
      if (dqmc_status s = right_step(c, prev, tau - nw, tau, c->cur)) return s;
      UDVp left = (k == nk) ? c->uid : c->slot(k);
      if (dqmc_status s = merge(c, c->cur, left, c->Gs, nullptr)) return s;
      // the time-displaced pass beside the sweep reads slot k until it has re-anchored there
      if (async_td && k < nk) HIPCHK(hipStreamWaitEvent(c->stream, c->td_ev[k], 0));
      if (dqmc_status s = copy_udv(c, c->slot(k), c->cur)) return s;
      if (dqmc_status s = stabilise(c, hist++)) return s;
      if (dqmc_status s = timing_end(c, DQMC_KERNEL_STABILISE)) return s;
    }
    if (meas & 1)
      if (dqmc_status s = measure(c)) return s;
    if (meas & 4)
      if (dqmc_status s = eq_measure(c, (meas & 1) != 0)) return s;
  }
  // the downward pass writes the field rows back, which that pass reads to its end
  if (async_td) HIPCHK(hipStreamWaitEvent(c->stream, c->td_ev[nk], 0));
  if (dqmc_status s = pass_draws(c, 1)) return s;
  for (int tau = L; tau >= 1; --tau) {
    if (dqmc_status s = update_slice(c, tau)) return s;
    if (meas & 1)
      if (dqmc_status s = measure(c)) return s;
    if (meas & 4)
      if (dqmc_status s = eq_measure(c, (meas & 1) != 0)) return s;
    if ((tau - 1) % nw == 0) {
      const int k = (tau - 1) / nw;
      // wrapped G(tau-1), compared against the recomputed one below
      if (dqmc_status s = wrap_down(c, tau, c->G)) return s;
      if (dqmc_status s = timing_begin(c, DQMC_KERNEL_STABILISE)) return s;
      UDVp prev = (k + 1 == nk) ? c->uid : c->slot(k + 1);
      if (dqmc_status s = left_step(c, prev, tau - 1, tau - 1 + nw, c->cur)) return s;
      UDVp right = (k == 0) ? c->uid : c->slot(k);
      if (dqmc_status s = merge(c, right, c->cur, c->Gs, nullptr)) return s;
      if (dqmc_status s = copy_udv(c, c->slot(k), c->cur)) return s;
      if (dqmc_status s = stabilise(c, hist++)) return s;
      if (dqmc_status s = timing_end(c, DQMC_KERNEL_STABILISE)) return s;
    } else {
      if (dqmc_status s = wrap_down(c, tau, c->G)) return s;
    }
  }
  hipLaunchKernelGGL(k_finish_sweep, gridc(c, 1), dim3(64), 0, c->stream, c->prec_hist, hist, c->prec_tot,
                     c->m.prec_threshold, c->counters, c->err_flag, c->cs);
  HIPCHK(hipGetLastError());
  c->row_alt.clear();
  return DQMC_OK;
}

// ------------------------------------------------- complex-field sweep --
// The sweep of Algorithm 1 for the imaginary-coupling four-valued field, on
// the real 2n x 2n images: wraps as two products and the rotations, the flips
// with the complex G in LDS (k_cupdate_slice), the stabilisation of the real
// sweep at dimension 2n, the original-frame estimators (k_cmeasure).
dqmc_status cwrap_up(dqmc_ctx* c, int tau) {
  const int N = c->N;
  if (dqmc_status s = gemm(c, gemm_args(N, N, N, c->E, N, 0, c->G, N, 0, c->T1, N))) return s;
  if (dqmc_status s = gemm(c, gemm_args(N, N, N, c->T1, N, 0, c->Einv, N, 0, c->Gs, N))) return s;
  return crot(c, c->G, c->Gs, tau, c->m.coupling, c->m.coupling);
}

dqmc_status cwrap_down(dqmc_ctx* c, int tau) {
  const int N = c->N;
  if (dqmc_status s = crot(c, c->T1, c->G, tau, -c->m.coupling, -c->m.coupling)) return s;
  if (dqmc_status s = gemm(c, gemm_args(N, N, N, c->T1, N, 0, c->E, N, 0, c->Gs, N))) return s;
  return gemm(c, gemm_args(N, N, N, c->Einv, N, 0, c->Gs, N, 0, c->G, N));
}

dqmc_status cupdate(dqmc_ctx* c, int tau, int dir) {
  hipLaunchKernelGGL(k_cupdate_slice, gridc(c, 1), dim3(256), cupdate_lds(c->Nf), c->stream, c->G, c->Nf,
                     field_row(c, tau), tau, (unsigned long long)dir, c->m.coupling, c->m.alpha, c->m.n_col,
                     field4_table(), c->counters, c->phase, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

dqmc_status cmeasure(dqmc_ctx* c) {
  const int N = c->N;
  const bool sym = c->m.trotter == DQMC_TROTTER_SYM;
  if (sym)
    if (dqmc_status s = gemm(c, gemm_args(N, N, N, c->Eh, N, 0, c->G, N, 0, c->T1, N))) return s;
  hipLaunchKernelGGL(k_cmeasure, gridc(c, 1), dim3(256), 0, c->stream, c->G, sym ? c->T1 : nullptr, c->Ehinv,
                     c->Kd, c->Nf, sym ? 1 : 0, c->trK_field, (double)c->m.n_col, c->m.u_int, c->bins,
                     c->err_flag, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

dqmc_status stabilise(dqmc_ctx* c, int hist_index);
dqmc_status copy_udv(dqmc_ctx* c, UDVp dst, UDVp src);
dqmc_status csweep_once(dqmc_ctx* c, int meas) {
  const int L = c->L, nw = c->nw, nk = c->nk;
  int hist = 0;
  c->row_alt.clear();
  c->Gcur = c->G;
  for (int tau = 1; tau <= L; ++tau) {
    if (dqmc_status s = cwrap_up(c, tau)) return s;
    if (dqmc_status s = cupdate(c, tau, 0)) return s;
    if (tau % nw == 0) {
      const int k = tau / nw;
      if (dqmc_status s = timing_begin(c, DQMC_KERNEL_STABILISE)) return s;
      UDVp prev = (k == 1) ? c->uid : c->slot(k - 1);
      if (dqmc_status s = right_step(c, prev, tau - nw, tau, c->cur)) return s;
      UDVp left = (k == nk) ? c->uid : c->slot(k);
      if (dqmc_status s = merge(c, c->cur, left, c->Gs, nullptr)) return s;
      if (dqmc_status s = copy_udv(c, c->slot(k), c->cur)) return s;
      if (dqmc_status s = stabilise(c, hist++)) return s;
      if (dqmc_status s = timing_end(c, DQMC_KERNEL_STABILISE)) return s;
    }
    if (meas & 1)
      if (dqmc_status s = cmeasure(c)) return s;
  }
  for (int tau = L; tau >= 1; --tau) {
    if (dqmc_status s = cupdate(c, tau, 1)) return s;
    if (meas & 1)
      if (dqmc_status s = cmeasure(c)) return s;
    if ((tau - 1) % nw == 0) {
      const int k = (tau - 1) / nw;
      if (dqmc_status s = cwrap_down(c, tau)) return s;
      if (dqmc_status s = timing_begin(c, DQMC_KERNEL_STABILISE)) return s;
      UDVp prev = (k + 1 == nk) ? c->uid : c->slot(k + 1);
      if (dqmc_status s = left_step(c, prev, tau - 1, tau - 1 + nw, c->cur)) return s;
      UDVp right = (k == 0) ? c->uid : c->slot(k);
      if (dqmc_status s = merge(c, right, c->cur, c->Gs, nullptr)) return s;
      if (dqmc_status s = copy_udv(c, c->slot(k), c->cur)) return s;
      if (dqmc_status s = stabilise(c, hist++)) return s;
      if (dqmc_status s = timing_end(c, DQMC_KERNEL_STABILISE)) return s;
    } else {
      if (dqmc_status s = cwrap_down(c, tau)) return s;
    }
  }
  hipLaunchKernelGGL(k_finish_sweep, gridc(c, 1), dim3(64), 0, c->stream, c->prec_hist, hist, c->prec_tot,
                     c->m.prec_threshold, c->counters, c->err_flag, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

// ------------------------------------------------ two-flavour sweep --
// The sweep of Algorithm 1 for the M_z form with two Green's functions on
// the 2n x 2n block-diagonal system: the wraps and the stabilisation of the
// one-flavour sweep (with the expanded field rows), the flips of both
// flavours in one workgroup per chain (k_fl2_update_slice), the sign-weighted
// estimators (k_fl2_measure).
dqmc_status fl2update(dqmc_ctx* c, int tau, int dir) {
  hipLaunchKernelGGL(k_fl2_update_slice, gridc(c, 1), dim3(256), fl2_update_lds(c->Nf), c->stream, c->G, c->Nf,
                     field_row(c, tau), scale_row(c, tau), tau, (unsigned long long)dir, c->m.coupling,
                     (int)c->m.field, c->m.prop_width, field4_table(), c->counters, c->phase, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

dqmc_status fl2measure(dqmc_ctx* c) {
  const int N = c->N;
  const bool sym = c->m.trotter == DQMC_TROTTER_SYM;
  if (sym)
    if (dqmc_status s = gemm(c, gemm_args(N, N, N, c->Eh, N, 0, c->G, N, 0, c->T1, N))) return s;
  hipLaunchKernelGGL(k_fl2_measure, gridc(c, 1), dim3(256), 0, c->stream, c->G, sym ? c->T1 : nullptr, c->Ehinv,
                     c->Kd, c->Nf, sym ? 1 : 0, c->trK, c->m.u_int, c->phase, c->bins, c->err_flag, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

dqmc_status fl2sweep_once(dqmc_ctx* c, int meas) {
  const int L = c->L, nw = c->nw, nk = c->nk;
  int hist = 0;
  c->row_alt.clear();
  c->Gcur = c->G;
  for (int tau = 1; tau <= L; ++tau) {
    if (dqmc_status s = wrap_up(c, tau, c->G)) return s;
    if (dqmc_status s = fl2update(c, tau, 0)) return s;
    if (tau % nw == 0) {
      const int k = tau / nw;
      if (dqmc_status s = timing_begin(c, DQMC_KERNEL_STABILISE)) return s;
      UDVp prev = (k == 1) ? c->uid : c->slot(k - 1);
      if (dqmc_status s = right_step(c, prev, tau - nw, tau, c->cur)) return s;
      UDVp left = (k == nk) ? c->uid : c->slot(k);
      if (dqmc_status s = merge(c, c->cur, left, c->Gs, nullptr)) return s;
      if (dqmc_status s = copy_udv(c, c->slot(k), c->cur)) return s;
      if (dqmc_status s = stabilise(c, hist++)) return s;
      if (dqmc_status s = timing_end(c, DQMC_KERNEL_STABILISE)) return s;
    }
    if (meas & 1)
      if (dqmc_status s = fl2measure(c)) return s;
  }
  for (int tau = L; tau >= 1; --tau) {
    if (dqmc_status s = fl2update(c, tau, 1)) return s;
    if (meas & 1)
      if (dqmc_status s = fl2measure(c)) return s;
    if (dqmc_status s = wrap_down(c, tau, c->G)) return s;
    if ((tau - 1) % nw == 0) {
      const int k = (tau - 1) / nw;
      if (dqmc_status s = timing_begin(c, DQMC_KERNEL_STABILISE)) return s;
      UDVp prev = (k + 1 == nk) ? c->uid : c->slot(k + 1);
      if (dqmc_status s = left_step(c, prev, tau - 1, tau - 1 + nw, c->cur)) return s;
      UDVp right = (k == 0) ? c->uid : c->slot(k);
      if (dqmc_status s = merge(c, right, c->cur, c->Gs, nullptr)) return s;
      if (dqmc_status s = copy_udv(c, c->slot(k), c->cur)) return s;
      if (dqmc_status s = stabilise(c, hist++)) return s;
      if (dqmc_status s = timing_end(c, DQMC_KERNEL_STABILISE)) return s;
    }
  }
  hipLaunchKernelGGL(k_finish_sweep, gridc(c, 1), dim3(64), 0, c->stream, c->prec_hist, hist, c->prec_tot,
                     c->m.prec_threshold, c->counters, c->err_flag, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

// ------------------------------------------------ general-vertex sweep --
// The sweep of Algorithm 1 with general operator vertices and Ising spins
// (section "Definition of the Hamiltonian"): the kinetic wraps as plain
// products, the flips of a slice with the partial wraps E_k G E_k^-1 in one
// workgroup per chain (k_vx_slice), the stabilisation with the vertex factors
// applied by k_vx_rows, the estimators of the one-flavour sweep.
dqmc_status vx_wrap(dqmc_ctx* c, bool up) {
  const int N = c->N;
  const double* A = up ? c->E : c->Einv;
  const double* B = up ? c->Einv : c->E;
  if (dqmc_status s = gemm(c, gemm_args(N, N, N, A, N, 0, c->G, N, 0, c->T1, N))) return s;
  return gemm(c, gemm_args(N, N, N, c->T1, N, 0, B, N, 0, c->G, N));
}

dqmc_status vx_slice(dqmc_ctx* c, int tau, int dir) {
  hipLaunchKernelGGL(k_vx_slice, gridc(c, 1), dim3(256), vx_slice_lds(c->N, c->nvx, c->nvx_nbr), c->stream, c->G,
                     c->N, c->field, c->L, tau, (unsigned long long)dir, c->vtab, c->vnbr, c->nvx_nbr, c->nvx,
                     c->vx_Kt, c->vx_dtJ, c->m.n_col, c->counters, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

dqmc_status vx_sweep_once(dqmc_ctx* c, int meas) {
  const int L = c->L, nw = c->nw, nk = c->nk;
  int hist = 0;
  c->row_alt.clear();
  c->Gcur = c->G;
  for (int tau = 1; tau <= L; ++tau) {
    if (dqmc_status s = vx_wrap(c, true)) return s;
    if (dqmc_status s = vx_slice(c, tau, 0)) return s;
    if (tau % nw == 0) {
      const int k = tau / nw;
      if (dqmc_status s = timing_begin(c, DQMC_KERNEL_STABILISE)) return s;
      UDVp prev = (k == 1) ? c->uid : c->slot(k - 1);
      if (dqmc_status s = right_step(c, prev, tau - nw, tau, c->cur)) return s;
      UDVp left = (k == nk) ? c->uid : c->slot(k);
      if (dqmc_status s = merge(c, c->cur, left, c->Gs, nullptr)) return s;
      if (dqmc_status s = copy_udv(c, c->slot(k), c->cur)) return s;
      if (dqmc_status s = stabilise(c, hist++)) return s;
      if (dqmc_status s = timing_end(c, DQMC_KERNEL_STABILISE)) return s;
    }
    if (meas & 1)
      if (dqmc_status s = measure(c)) return s;
  }
  for (int tau = L; tau >= 1; --tau) {
    if (meas & 1)
      if (dqmc_status s = measure(c)) return s;
    if (dqmc_status s = vx_slice(c, tau, 1)) return s;
    if (dqmc_status s = vx_wrap(c, false)) return s;
    if ((tau - 1) % nw == 0) {
      const int k = (tau - 1) / nw;
      if (dqmc_status s = timing_begin(c, DQMC_KERNEL_STABILISE)) return s;
      UDVp prev = (k + 1 == nk) ? c->uid : c->slot(k + 1);
      if (dqmc_status s = left_step(c, prev, tau - 1, tau - 1 + nw, c->cur)) return s;
      UDVp right = (k == 0) ? c->uid : c->slot(k);
      if (dqmc_status s = merge(c, right, c->cur, c->Gs, nullptr)) return s;
      if (dqmc_status s = copy_udv(c, c->slot(k), c->cur)) return s;
      if (dqmc_status s = stabilise(c, hist++)) return s;
      if (dqmc_status s = timing_end(c, DQMC_KERNEL_STABILISE)) return s;
    }
  }
  hipLaunchKernelGGL(k_finish_sweep, gridc(c, 1), dim3(64), 0, c->stream, c->prec_hist, hist, c->prec_tot,
                     c->m.prec_threshold, c->counters, c->err_flag, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

dqmc_status expand_field(dqmc_ctx* c) {
  if (c->nfl != 2) return DQMC_OK;
  hipLaunchKernelGGL(k_expand_field, gridc(c, grid1((size_t)c->L * c->Nf)), dim3(256), 0, c->stream, c->field,
                     c->field_x, c->L, c->Nf, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

dqmc_status fill_small(dqmc_ctx* c, double* p, size_t n, double v) {
  hipLaunchKernelGGL(k_fill, gridc(c, grid1(n)), dim3(256), 0, c->stream, p, n, v, is_shared(c, p) ? (size_t)0 : c->cs);
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
  if (m->field != DQMC_FIELD_ISING && m->field != DQMC_FIELD_GAUSS && m->field != DQMC_FIELD_ISING4 &&
      m->field != DQMC_FIELD_ISING4_IMAG)
    return DQMC_E_ARG;
  if (m->trotter != DQMC_TROTTER_ASYM && m->trotter != DQMC_TROTTER_SYM) return DQMC_E_ARG;
  if (!std::isfinite(m->coupling) || !std::isfinite(m->alpha)) return DQMC_E_ARG;
  return DQMC_OK;
}

// Left storage and G(0) from the current field: slot k = UDV of
// B(beta, k n_wrap)^T for k = nk-1 .. 0, then G = (1 + B(beta,0))^-1.
dqmc_status reanchor(dqmc_ctx* c) {
  for (int k = c->nk - 1; k >= 0; --k) {
    UDVp prev = (k + 1 == c->nk) ? c->uid : c->slot(k + 1);
    if (dqmc_status s = left_step(c, prev, k * c->nw, (k + 1) * c->nw, c->slot(k))) return s;
  }
  return merge(c, c->uid, c->slot(0), c->G, nullptr);
}

// Gradient pass: the upward pass of Algorithm 1 without updates.  G(tau) for
// tau = 1..L is wrapped from G(0) in the second G buffer and, every n_wrap
// slices, recomputed from a running right form and the stored left forms
// (the checkpoints), so no product of L slices is ever stored; row tau of
// the gradient is coupling (1 - G(tau)_ii).  G, the field and the stored
// left forms are left as they were; gprec holds max |wrapped - recomputed|.
dqmc_status grad_pass(dqmc_ctx* c) {
  const int N = c->N, L = c->L, nw = c->nw, nk = c->nk;
  const size_t NN = (size_t)N * N;
  c->row_alt.clear();
  if (dqmc_status s = fill_small(c, c->gprec, 1, 0.0)) return s;
  hipLaunchKernelGGL(k_copy, gridc(c, grid1(NN)), dim3(256), 0, c->stream, c->G2, c->G, NN, c->cs);
  HIPCHK(hipGetLastError());
  c->Gcur = c->G2;
  UDVp right = c->uid;
  UDVp bufs[2] = {c->hA, c->hB};
  int b = 0;
  for (int tau = 1; tau <= L; ++tau) {
    if (dqmc_status s = wrap_up(c, tau, c->G2)) return s;
    if (tau % nw == 0) {
      const int k = tau / nw;
      if (dqmc_status s = right_step(c, right, tau - nw, tau, bufs[b])) return s;
      right = bufs[b];
      b ^= 1;
      UDVp left = (k == nk) ? c->uid : c->slot(k);
      if (dqmc_status s = merge(c, right, left, c->Gs, nullptr)) return s;
      hipLaunchKernelGGL(k_prec_replace, gridc(c, prec_grid(NN)), dim3(256), 0,
                         c->stream, c->G2, c->G2, c->Gs, NN, c->gprec, c->err_flag, c->cs);
      HIPCHK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_grad_diag, gridc(c, grid1(N)), dim3(256), 0, c->stream, c->G2, N, c->m.coupling,
                       c->grad + (size_t)(tau - 1) * N, c->cs);
    HIPCHK(hipGetLastError());
  }
  c->Gcur = c->G;
  return DQMC_OK;
}

// One Langevin step of every chain: gradient pass, field update, then the
// left storage and G(0) of the new field.
dqmc_status langevin_once(dqmc_ctx* c, double eps) {
  if (dqmc_status s = grad_pass(c)) return s;
  const size_t n = (size_t)c->L * c->N;
  hipLaunchKernelGGL(k_langevin, gridc(c, grid1(n)), dim3(256), 0, c->stream, c->field, c->grad, c->L, c->N, eps,
                     c->m.coupling, c->m.alpha, (double)c->m.n_col, c->counters, c->cs);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_next_langevin_step, dim3(1, c->nch), dim3(64), 0, c->stream, c->counters, c->cs);
  HIPCHK(hipGetLastError());
  return reanchor(c);
}

// --------------------------------------------------- time-displaced pass --
// Re-anchoring at a checkpoint from the right form R of B(tau,0) and the left
// form Lf of B(beta,tau)^T.  With X the bounded matrix of the merge,
//   [Y1 | Y2] = X^-1 [D_Rb^-1 Q_R^T | D_Rs T_R],
//   GTT = Q_L D_Lb^-1 Y1,  GT0 = Q_L D_Lb^-1 Y2,  G0T^T = -Y1^T D_Ls T_L,
// each replacing its propagated value (largest deviation into gprec[0] for
// GTT, gprec[1] for GT0 and G0T).
dqmc_status td_anchor(dqmc_ctx* c, UDVp R, UDVp Lf, double* gt0, double* h) {
  const int N = c->N, ld = 3 * N;   // XA = [X | D_Rb^-1 Q_R^T | D_Rs T_R]
  const size_t NN = (size_t)N * N;
  GemmArgs g1 = gemm_args(N, N, N, R.Q, N, 1, Lf.Q, N, 0, c->XA, ld);
  g1.rs = R.D; g1.rs_mode = SC_INV_BIG; g1.cs = Lf.D; g1.cs_mode = SC_INV_BIG;
  if (dqmc_status s = gemm(c, g1)) return s;
  GemmArgs g2 = gemm_args(N, N, N, R.T, N, 0, Lf.T, N, 1, c->XA, ld, 1.0, 1.0);
  g2.rs = R.D; g2.rs_mode = SC_SMALL; g2.cs = Lf.D; g2.cs_mode = SC_SMALL;
  if (dqmc_status s = gemm(c, g2)) return s;
  const unsigned t = (unsigned)((N + 31) / 32);
  hipLaunchKernelGGL(k_td_rhs, dim3(t, t, (unsigned)c->nch), dim3(256), 0, c->stream, c->XA + N, ld, R.Q, R.T, R.D,
                     N, c->cs, is_shared(c, R.Q) ? (size_t)0 : c->cs);
  HIPCHK(hipGetLastError());
  if (dqmc_status s = lu_solve(c, c->XA, 2 * N, ld, nullptr)) return s;
  const unsigned pg = prec_grid(NN);
  GemmArgs g3 = gemm_args(N, N, N, Lf.Q, N, 0, c->XA + N, ld, 0, c->Gs, N);
  g3.ks = Lf.D; g3.ks_mode = SC_INV_BIG;
  if (dqmc_status s = gemm(c, g3)) return s;
  hipLaunchKernelGGL(k_prec_replace, gridc(c, pg), dim3(256), 0, c->stream, c->G2, c->G2, c->Gs, NN, c->gprec,
                     c->err_flag, c->cs);
  GemmArgs g4 = gemm_args(N, N, N, Lf.Q, N, 0, c->XA + 2 * N, ld, 0, c->X, N);
  g4.ks = Lf.D; g4.ks_mode = SC_INV_BIG;
  if (dqmc_status s = gemm(c, g4)) return s;
  hipLaunchKernelGGL(k_prec_replace, gridc(c, pg), dim3(256), 0, c->stream, gt0, gt0, c->X, NN, c->gprec + 1,
                     c->err_flag, c->cs);
  GemmArgs g5 = gemm_args(N, N, N, c->XA + N, ld, 1, Lf.T, N, 0, c->RHS, N, -1.0);
  g5.ks = Lf.D; g5.ks_mode = SC_SMALL;
  if (dqmc_status s = gemm(c, g5)) return s;
  hipLaunchKernelGGL(k_prec_replace, gridc(c, pg), dim3(256), 0, c->stream, h, h, c->RHS, NN, c->gprec + 1,
                     c->err_flag, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

// S_ab(K, tau) of the current GT0, H = G0T^T and GTT.  With the symmetric
// Trotter split the estimator takes the rotated exp(-dtau K/2) (.) exp(+dtau K/2)
// matrices (for H the rotation is exp(+dtau K/2) H exp(-dtau K/2)).
dqmc_status td_measure(dqmc_ctx* c, int tau, const double* gt0, const double* h, const double* gtt) {
  const int N = c->N;
  if (c->m.trotter == DQMC_TROTTER_SYM) {
    // e^{-dtau K/2} (.) e^{+dtau K/2} of GT0 and GTT, e^{+dtau K/2} H e^{-dtau K/2}:
    // the three left products in one launch, then the three right products
    GemmArgs gl[3] = {gemm_args(N, N, N, c->Eh, N, 0, gt0, N, 0, c->T1, N),
                      gemm_args(N, N, N, c->Ehinv, N, 0, h, N, 0, c->S[0], N),
                      gemm_args(N, N, N, c->Eh, N, 0, gtt, N, 0, c->S[1], N)};
    if (dqmc_status s = gemm_group(c, gl, 3)) return s;
    GemmArgs gr[3] = {gemm_args(N, N, N, c->T1, N, 0, c->Ehinv, N, 0, c->Gs, N),
                      gemm_args(N, N, N, c->S[0], N, 0, c->Eh, N, 0, c->X, N),
                      gemm_args(N, N, N, c->S[1], N, 0, c->Ehinv, N, 0, c->RHS, N)};
    if (dqmc_status s = gemm_group(c, gr, 3)) return s;
    gt0 = c->Gs; h = c->X; gtt = c->RHS;
  }
  if (c->td_corr_now) {
    if (tau == 0) {
      hipLaunchKernelGGL(k_diag, gridc(c, grid1(N)), dim3(256), 0, c->stream, gtt, N, c->td_g00, c->cs);
      HIPCHK(hipGetLastError());
    }
    const int nb = c->eq_L1 * c->eq_L2 * c->eq_norb * c->eq_norb;
    hipLaunchKernelGGL(k_corr<true>, gridc(c, grid1((size_t)nb + 1, 4)), dim3(256), 0, c->stream, gt0, h, gtt,
                       c->td_g00, N, c->eq_L1, c->eq_L2, c->eq_norb, c->eq_site, c->eq_sign,
                       c->td_corr + (size_t)tau * td_corr_stride(c),
                       tau == 0 ? c->td_corr + (size_t)(c->L + 1) * td_corr_stride(c) : nullptr, c->cs);
    HIPCHK(hipGetLastError());
  }
  // small lattices: one workgroup per chain (no partial records, no fences)
  const int rows = N <= kTdSmallN ? N : kTdRows;
  const int nblk = (N + rows - 1) / rows;
  const size_t off = (size_t)tau * kTdStride;
  hipLaunchKernelGGL(k_td_measure, gridc(c, (unsigned)nblk), dim3(256), 0, c->stream, gt0, h, gtt, c->kph, c->korb, N,
                     rows, c->tdpart, 1.0 / c->td_cells, c->a00, c->tdS + off, c->tdbins + off,
                     c->tdbins + (size_t)(c->L + 1) * kTdStride, tau == 0 ? 1 : 0, c->cs);
  HIPCHK(hipGetLastError());
  return DQMC_OK;
}

// Time-displaced pass from the state at the start of a sweep (G = G(0), left
// forms stored): for tau = 1..L, GTT is wrapped, GT0 and H propagated, all
// three re-anchored every n_wrap slices from a running right form and the
// stored left forms, and S(K, tau) measured at tau = 0..L.  The chain's G,
// field and stored forms are left unchanged.
dqmc_status td_pass(dqmc_ctx* c) {
  const int N = c->N, L = c->L, nw = c->nw, nk = c->nk;
  const size_t NN = (size_t)N * N;
  if (c->td_norb < 1) return fail(c, DQMC_E_STATE, "time-displaced measurement not set up");
  c->row_alt.clear();
  if (dqmc_status s = fill_small(c, c->gprec, 2, 0.0)) return s;
  hipLaunchKernelGGL(k_copy, gridc(c, grid1(NN)), dim3(256), 0, c->stream, c->G2, c->G, NN, c->cs);
  const unsigned t = (unsigned)((N + 31) / 32);
  hipLaunchKernelGGL(k_td_init, dim3(t, t, (unsigned)c->nch), dim3(256), 0, c->stream, c->G, c->TD[0], c->TD[2], N,
                     c->cs);
  HIPCHK(hipGetLastError());
  if (c->td_sync) HIPCHK(hipEventRecord((*c->td_sync)[0], c->stream));   // G is read
  double *gt0 = c->TD[0], *gt0_alt = c->TD[1], *h = c->TD[2], *h_alt = c->TD[3];
  c->Gcur = c->G2;
  if (dqmc_status s = td_measure(c, 0, gt0, h, c->G2)) return s;
  // The right forms of the checkpoints depend only on the field: right_k
  // (in bufs[(k - 1) & 1]) is computed on the second stream while the main
  // stream re-anchors at checkpoint k - 1 and propagates (a single chain not
  // under graph capture; otherwise in line).  The QR of right_k reads
  // S[2..4], Zq, norms, piv, Vall, VTall, Rt and writes bufs[(k - 1) & 1],
  // none of which the main stream touches in this pass; it waits for the
  // main stream's re-anchoring at k - 2, the last reader of that buffer.
  UDVp bufs[2] = {c->hA, c->hB};
  bool fork = c->side != nullptr && c->nch == 1;
  if (fork) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIPCHK(hipStreamIsCapturing(c->stream, &cap));
    fork = cap == hipStreamCaptureStatusNone;
  }
  auto right_of = [&](int k) { return k == 0 ? c->uid : bufs[(k - 1) & 1]; };
  // enqueue right_k after the main stream's work so far
  auto launch_right = [&](int k) -> dqmc_status {
    if (!fork) return right_step(c, right_of(k - 1), (k - 1) * nw, k * nw, bufs[(k - 1) & 1]);
    HIPCHK(hipEventRecord(c->fork_ev[2], c->stream));
    HIPCHK(hipStreamWaitEvent(c->side, c->fork_ev[2], 0));
    hipStream_t main = c->stream;
    c->stream = c->side;
    const dqmc_status s = right_step(c, right_of(k - 1), (k - 1) * nw, k * nw, bufs[(k - 1) & 1]);
    c->stream = main;
    if (s) return s;
    HIPCHK(hipEventRecord(c->fork_ev[(k - 1) & 1], c->side));
    return DQMC_OK;
  };
  if (dqmc_status s = launch_right(1)) return s;
  for (int tau = 1; tau <= L; ++tau) {
    // three independent left products in one launch: E GTT (first half of
    // the wrap), B_tau GT0 and B_tau^-T H; then the wrap's second half
    GemmArgs g3[3];
    g3[0] = gemm_args(N, N, N, c->E, N, 0, c->G2, N, 0, c->T1, N);
    g3[1] = gemm_args(N, N, N, c->E, N, 0, gt0, N, 0, gt0_alt, N);
    g3[1].rs = field_row(c, tau); g3[1].rs_mode = SC_EXP; g3[1].rs_coef = c->m.coupling;
    g3[2] = gemm_args(N, N, N, c->Einv, N, 0, h, N, 0, h_alt, N);
    g3[2].rs = field_row(c, tau); g3[2].rs_mode = SC_EXP; g3[2].rs_coef = -c->m.coupling;
    if (dqmc_status s = gemm_group(c, g3, 3)) return s;
    GemmArgs gw = gemm_args(N, N, N, c->T1, N, 0, c->Einv, N, 0, c->G2, N);
    gw.rs = field_row(c, tau); gw.rs_mode = SC_EXP; gw.rs_coef = c->m.coupling;
    gw.cs = field_row(c, tau); gw.cs_mode = SC_EXP; gw.cs_coef = -c->m.coupling;
    if (dqmc_status s = gemm(c, gw)) return s;
    std::swap(gt0, gt0_alt);
    std::swap(h, h_alt);
    if (tau % nw == 0) {
      const int k = tau / nw;
      if (fork) HIPCHK(hipStreamWaitEvent(c->stream, c->fork_ev[(k - 1) & 1], 0));
      if (k < nk)
        if (dqmc_status s = launch_right(k + 1)) return s;
      UDVp left = (k == nk) ? c->uid : c->slot(k);
      if (dqmc_status s = td_anchor(c, right_of(k), left, gt0, h)) return s;
      if (c->td_sync && k < nk) HIPCHK(hipEventRecord((*c->td_sync)[k], c->stream));   // slot k is read
    }
    if (dqmc_status s = td_measure(c, tau, gt0, h, c->G2)) return s;
  }
  if (c->td_sync) HIPCHK(hipEventRecord((*c->td_sync)[nk], c->stream));
  c->Gcur = c->G;
  return DQMC_OK;
}

// The time-displaced pass of a single chain on the second stream, beside the
// sweep (which then waits for td_ev[0] before it overwrites G, for td_ev[k]
// before it stores its right form in slot k, and for td_ev[nk] before the
// downward pass writes the field back).  The pass runs in the chain's shadow
// context: the chain's G, field, left forms and bins, its own scratch.
dqmc_status td_pass_async(dqmc_ctx* c) {
  dqmc_ctx* t = c->tdc;
  t->m = c->m;
  // beside the sweep the grouped products take the direct 32 x 32 kernel
  // rather than the LDS-staged 64 x 64 one (18x18 sweep with its pass 289 ->
  // 287 ms; alone the 64 x 64 tiles are faster)
  t->gemm_tile = 32;
  t->td_norb = c->td_norb; t->td_cells = c->td_cells; t->td_corr_now = c->td_corr_now;
  t->eq_L1 = c->eq_L1; t->eq_L2 = c->eq_L2; t->eq_norb = c->eq_norb;
  HIPCHK(hipEventRecord(c->fork_ev[2], c->stream));
  HIPCHK(hipStreamWaitEvent(c->side, c->fork_ev[2], 0));
  t->stream = c->side;
  t->side = c->side2;
  t->td_sync = &c->td_ev;
  const dqmc_status s = td_pass(t);
  t->side = nullptr;     // owned by c
  t->td_sync = nullptr;
  t->stream = c->stream;
  if (s) {
    c->err = t->err;
    return s;
  }
  HIPCHK(hipStreamWaitEvent(c->stream, c->td_ev[0], 0));
  return DQMC_OK;
}

// Copy `bytes` (<= 64) of a per-chain item from every chain into host dst
// (chain-major), through the contiguous staging buffer.
dqmc_status gather(dqmc_ctx* c, void* dst, const void* src, size_t bytes) {
  if (c->nch == 1) {
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->stream));
    return DQMC_OK;
  }
  const int count = (int)((bytes + 7) / 8);
  hipLaunchKernelGGL(k_gather, dim3(1, c->nch), dim3(64), 0, c->stream, c->gbuf, static_cast<const double*>(src),
                     count, c->cs);
  HIPCHK(hipGetLastError());
  std::vector<double> tmp((size_t)count * c->nch);
  HIPCHK(hipMemcpyAsync(tmp.data(), c->gbuf, tmp.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int i = 0; i < c->nch; ++i)
    std::memcpy(static_cast<char*>(dst) + i * bytes, tmp.data() + (size_t)i * count, bytes);
  return DQMC_OK;
}

dqmc_status read_flag(dqmc_ctx* c) {
  std::vector<int> flags(c->nch, 0);
  if (dqmc_status s = gather(c, flags.data(), c->err_flag, sizeof(int))) return s;
  HIPCHK(hipStreamSynchronize(c->stream));
  int flag = 0;
  for (int f : flags) flag |= f;
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

// Statistics of one chain (chain >= 0) or summed over all chains (chain < 0).
dqmc_status chain_stats(dqmc_ctx* c, int chain, dqmc_stats* st) {
  std::vector<unsigned long long> ctr(4 * (size_t)c->nch);
  std::vector<double> pt(4 * (size_t)c->nch);
  if (dqmc_status s = gather(c, ctr.data(), c->counters, 4 * sizeof(double))) return s;
  if (dqmc_status s = gather(c, pt.data(), c->prec_tot, 4 * sizeof(double))) return s;
  HIPCHK(hipStreamSynchronize(c->stream));
  dqmc_stats t{};
  double ps = 0.0, pc = 0.0, pm = 0.0;
  for (int i = 0; i < c->nch; ++i) {
    if (chain >= 0 && i != chain) continue;
    t.proposals += ctr[4 * i];
    t.accepted += ctr[4 * i + 1];
    ps += pt[4 * i];
    pm = std::max(pm, pt[4 * i + 1]);
    pc += pt[4 * i + 2];
  }
  t.n_prec = (uint64_t)pc;
  t.prec_mean = pc > 0 ? ps / pc : 0.0;
  t.prec_max = pm;
  *st = t;
  return DQMC_OK;
}

}  // namespace

// ===================================================================== ABI ==
extern "C" {

dqmc_status dqmc_query_sizes(const dqmc_model* m, dqmc_sizes* out) {
  if (!out || check_model(m) != DQMC_OK) return DQMC_E_ARG;
  const bool cplx = m->field == DQMC_FIELD_ISING4_IMAG;
  if (cplx && m->n > kCMaxN) return DQMC_E_UNSUPPORTED;
  dqmc_ctx tmp;
  tmp.N = cplx ? 2 * m->n : m->n; tmp.Nf = m->n; tmp.cplx = cplx ? 1 : 0;
  tmp.L = m->n_slices; tmp.nw = m->n_wrap; tmp.nk = m->n_slices / m->n_wrap;
  const size_t N = tmp.N;
  out->G = N * N * sizeof(double);
  out->field = (size_t)m->n_slices * m->n * sizeof(double);
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
  const bool cplx = m->field == DQMC_FIELD_ISING4_IMAG;
  if (cplx && N > kCMaxN) return DQMC_E_UNSUPPORTED;
  dqmc_ctx* c = new (std::nothrow) dqmc_ctx();
  if (!c) return DQMC_E_NOMEM;
  c->m = *m;
  // a complex field runs on the 2n x 2n images: K becomes diag(K, K)
  const int Nd = cplx ? 2 * N : N;
  c->N = Nd; c->Nf = N; c->cplx = cplx ? 1 : 0;
  c->L = m->n_slices; c->nw = m->n_wrap; c->nk = m->n_slices / m->n_wrap;
  // panel width: the register panels hold up to 48 rows per thread in
  // 256/nb row groups
  c->nb = (Nd <= kNarrowMaxN) ? 32 : (Nd <= 16 * 48 ? 16 : 8);
  c->K.assign((size_t)Nd * Nd, 0.0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      c->K[(size_t)i * Nd + j] = K[(size_t)i * N + j];
      if (cplx) c->K[(size_t)(i + N) * Nd + j + N] = K[(size_t)i * N + j];
    }
  double tr = 0.0, n1 = 0.0;
  for (int j = 0; j < N; ++j) {
    double col = 0.0;
    for (int i = 0; i < N; ++i) col += std::fabs(K[(size_t)i * N + j]);
    n1 = std::max(n1, col);
    tr += K[(size_t)j * N + j];
  }
  c->trK = cplx ? 2.0 * tr : tr; c->trK_field = tr; c->normK1 = n1;
  *out = c;
  return DQMC_OK;
}

dqmc_status dqmc_create_mz(const dqmc_model* m, const double* K_up, const double* K_dn, dqmc_ctx** out) {
  if (!out) return DQMC_E_ARG;
  *out = nullptr;
  if (check_model(m) != DQMC_OK || !K_up || !K_dn) return DQMC_E_ARG;
  if (m->field == DQMC_FIELD_ISING4_IMAG || m->alpha != 0.0 || m->n_col != 1) return DQMC_E_ARG;
  const int n = m->n;
  if (n > kFl2MaxN) return DQMC_E_UNSUPPORTED;
  for (const double* K : {K_up, K_dn})
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double a = K[(size_t)i * n + j], b = K[(size_t)j * n + i];
        if (!std::isfinite(a) || a != b) return DQMC_E_ARG;
      }
  dqmc_ctx* c = new (std::nothrow) dqmc_ctx();
  if (!c) return DQMC_E_NOMEM;
  c->m = *m;
  const int Nd = 2 * n;
  c->N = Nd; c->Nf = n; c->nfl = 2;
  c->L = m->n_slices; c->nw = m->n_wrap; c->nk = m->n_slices / m->n_wrap;
  c->nb = 32;
  c->K.assign((size_t)Nd * Nd, 0.0);
  double tr = 0.0, n1 = 0.0;
  for (int f = 0; f < 2; ++f) {
    const double* K = f == 0 ? K_up : K_dn;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) c->K[(size_t)(i + f * n) * Nd + j + f * n] = K[(size_t)i * n + j];
    for (int j = 0; j < n; ++j) {
      double col = 0.0;
      for (int i = 0; i < n; ++i) col += std::fabs(K[(size_t)i * n + j]);
      n1 = std::max(n1, col);
      tr += K[(size_t)j * n + j];
    }
  }
  c->trK = tr; c->trK_field = tr; c->normK1 = n1;
  *out = c;
  return DQMC_OK;
}

dqmc_status dqmc_create_vertices(const dqmc_model* m, const double* K, int32_t n_vertices, const dqmc_vertex* v,
                                 double h, double J, int32_t n_pairs, const int32_t* pairs, dqmc_ctx** out) {
  if (!out) return DQMC_E_ARG;
  *out = nullptr;
  if (check_model(m) != DQMC_OK || !K || !v || n_vertices < 1 || n_pairs < 0 || (n_pairs > 0 && !pairs))
    return DQMC_E_ARG;
  if (m->field != DQMC_FIELD_ISING) return DQMC_E_ARG;
  if (!std::isfinite(h) || h < 0.0 || !std::isfinite(J)) return DQMC_E_ARG;
  const int n = m->n, M = n_vertices;
  if (n > kVxMaxN || M > kVxMaxM) return DQMC_E_UNSUPPORTED;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double a = K[(size_t)i * n + j], b = K[(size_t)j * n + i];
      if (!std::isfinite(a) || a != b) return DQMC_E_ARG;
    }
  bool any_ising = false;
  for (int k = 0; k < M; ++k) {
    const dqmc_vertex& x = v[k];
    if (x.n_orb < 1 || x.n_orb > 2) return DQMC_E_UNSUPPORTED;
    for (int a = 0; a < x.n_orb; ++a)
      if (x.orb[a] < 0 || x.orb[a] >= n) return DQMC_E_ARG;
    if (x.n_orb == 2 && x.orb[0] == x.orb[1]) return DQMC_E_ARG;
    if (x.ising != 0 && x.ising != 1) return DQMC_E_ARG;
    if (!std::isfinite(x.g) || !std::isfinite(x.alpha)) return DQMC_E_ARG;
    for (int a = 0; a < 4; ++a)
      if (!std::isfinite(x.O[a])) return DQMC_E_ARG;
    if (x.n_orb == 2 && x.O[1] != x.O[2]) return DQMC_E_ARG;
    any_ising = any_ising || x.ising;
  }
  // an Ising spin with a transverse field needs h > 0 (Kt = -ln tanh(dtau h) / 2)
  if (any_ising && !(h > 0.0)) return DQMC_E_ARG;
  std::vector<std::vector<int>> nbr(M);
  for (int p = 0; p < n_pairs; ++p) {
    const int a = pairs[2 * p], b = pairs[2 * p + 1];
    if (a < 0 || a >= M || b < 0 || b >= M || a == b || !v[a].ising || !v[b].ising) return DQMC_E_ARG;
    nbr[a].push_back(b);
    nbr[b].push_back(a);
  }
  if (2 * (int64_t)n_pairs > kVxMaxNbr) return DQMC_E_UNSUPPORTED;
  dqmc_ctx* c = new (std::nothrow) dqmc_ctx();
  if (!c) return DQMC_E_NOMEM;
  c->m = *m;
  c->m.coupling = 0.0;
  c->N = n; c->Nf = M; c->nvx = M;
  c->L = m->n_slices; c->nw = m->n_wrap; c->nk = m->n_slices / m->n_wrap;
  c->nb = 32;
  c->K.assign(K, K + (size_t)n * n);
  double tr = 0.0, n1 = 0.0;
  for (int j = 0; j < n; ++j) {
    double col = 0.0;
    for (int i = 0; i < n; ++i) col += std::fabs(K[(size_t)i * n + j]);
    n1 = std::max(n1, col);
    tr += K[(size_t)j * n + j];
  }
  c->trK = tr; c->trK_field = tr; c->normK1 = n1;
  c->vx_Kt = any_ising ? -0.5 * std::log(std::tanh(m->dtau * h)) : 0.0;
  c->vx_dtJ = m->dtau * J;
  c->vx_rec.assign((size_t)M * kVxRec, 0.0);
  for (int k = 0; k < M; ++k) {
    const dqmc_vertex& x = v[k];
    double* r = c->vx_rec.data() + (size_t)k * kVxRec;
    r[0] = x.n_orb; r[1] = x.orb[0]; r[2] = x.n_orb == 2 ? x.orb[1] : x.orb[0]; r[3] = x.ising;
    r[4] = x.g; r[5] = x.alpha;
    r[6] = x.O[0]; r[7] = x.n_orb == 2 ? x.O[1] : 0.0; r[8] = x.n_orb == 2 ? x.O[2] : 0.0;
    r[9] = x.n_orb == 2 ? x.O[3] : 0.0;
    r[10] = (double)c->vx_nbr.size(); r[11] = (double)nbr[k].size();
    for (int b : nbr[k]) c->vx_nbr.push_back((double)b);
  }
  c->nvx_nbr = (int)c->vx_nbr.size();
  *out = c;
  return DQMC_OK;
}

dqmc_status dqmc_ctx_sizes(const dqmc_ctx* c, dqmc_sizes* out) {
  if (!c || !out) return DQMC_E_ARG;
  dqmc_ctx tmp;
  tmp.N = c->N; tmp.Nf = c->Nf; tmp.cplx = c->cplx; tmp.nfl = c->nfl;
  tmp.nvx = c->nvx; tmp.nvx_nbr = c->nvx_nbr;
  tmp.L = c->L; tmp.nw = c->nw; tmp.nk = c->nk;
  const size_t N = c->N;
  out->G = N * N * sizeof(double);
  out->field = (size_t)c->L * c->Nf * sizeof(double);
  out->slots = (size_t)(c->nk + 1) * (2 * N * N + N) * sizeof(double);
  out->work = layout_work(&tmp, false) * sizeof(double);
  return DQMC_OK;
}

}  // extern "C"

namespace {

// The context of the time-displaced pass that runs beside the sweep of a
// single chain: the model and sizes of c, its scratch in the shadow part of
// the work buffer, c's shared matrices, c's G, field and stored forms (read
// only) and c's time-displaced bins, precision record and error flag.
dqmc_status shadow_setup(dqmc_ctx* c) {
  if (!c->shadow_base) return fail(c, DQMC_E_STATE, "no shadow part in the work buffer");
  if (!c->tdc) {
    c->tdc = new (std::nothrow) dqmc_ctx();
    if (!c->tdc) return fail(c, DQMC_E_NOMEM, "no host memory for the time-displaced pass's context");
  }
  dqmc_ctx* t = c->tdc;
  t->m = c->m;
  t->N = c->N; t->L = c->L; t->nw = c->nw; t->nk = c->nk; t->nb = c->nb; t->Nf = c->Nf;
  t->K = c->K; t->trK = c->trK; t->normK1 = c->normK1; t->trK_field = c->trK_field;
  t->nch = 1; t->cs = 0; t->no_shadow = true;
  layout_chain(t, c->shadow_base);
  if (!t->XA || !t->tdpart || !t->TD[3] || !t->Uinv)
    return fail(c, DQMC_E_STATE, "the time-displaced pass's scratch is not laid out");
  t->E = c->E; t->Einv = c->Einv; t->Eh = c->Eh; t->Ehinv = c->Ehinv; t->Kd = c->Kd; t->uid = c->uid;
  t->gbuf = c->gbuf; t->kph = c->kph; t->korb = c->korb; t->eq_sign = c->eq_sign; t->eq_site = c->eq_site;
  t->shared_lo = c->shared_lo; t->shared_hi = c->shared_hi;
  t->G = c->G; t->field = c->field; t->slots = c->slots; t->work = c->work;
  t->tdS = c->tdS; t->tdbins = c->tdbins; t->td_corr = c->td_corr; t->td_g00 = c->td_g00; t->gprec = c->gprec;
  t->err_flag = c->err_flag;
  t->stream = c->stream;
  t->bound = true;
  for (hipEvent_t& e : t->fork_ev)
    if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  while ((int)c->td_ev.size() < c->nk + 1) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->td_ev.push_back(e);
  }
  if (!c->side2) HIPCHK(hipStreamCreateWithFlags(&c->side2, hipStreamNonBlocking));
  // the completion counter of the estimator's partial records starts at zero
  return fill_small(t, t->tdpart, td_part_size(t), 0.0);
}

// Device-side set-up of a bound context (one chain or a group of chains):
// exponentials, identity UDV, zeroed counters and the chains' Philox keys.
dqmc_status setup_device(dqmc_ctx* c) {
  const int N = c->N;
  if (dqmc_status s = set_lds_limits(c)) return s;
  HIPCHK(hipMemcpyAsync(c->Kd, c->K.data(), sizeof(double) * N * N, hipMemcpyHostToDevice, c->stream));
  if (c->nvx) {
    HIPCHK(hipMemcpyAsync(c->vtab, c->vx_rec.data(), sizeof(double) * c->vx_rec.size(), hipMemcpyHostToDevice,
                          c->stream));
    if (c->nvx_nbr)
      HIPCHK(hipMemcpyAsync(c->vnbr, c->vx_nbr.data(), sizeof(double) * c->vx_nbr.size(), hipMemcpyHostToDevice,
                            c->stream));
  }
  if (dqmc_status s = expm(c, -c->m.dtau, c->E)) return s;
  if (dqmc_status s = expm(c, +c->m.dtau, c->Einv)) return s;
  if (dqmc_status s = expm(c, -0.5 * c->m.dtau, c->Eh)) return s;
  if (dqmc_status s = expm(c, +0.5 * c->m.dtau, c->Ehinv)) return s;
  hipLaunchKernelGGL(k_set_identity, dim3(grid1((size_t)N * N)), dim3(256), 0, c->stream, c->uid.Q, N, N, (size_t)0);
  hipLaunchKernelGGL(k_set_identity, dim3(grid1((size_t)N * N)), dim3(256), 0, c->stream, c->uid.T, N, N, (size_t)0);
  if (dqmc_status s = fill_small(c, c->uid.D, N, 1.0)) return s;
  if (dqmc_status s = fill_small(c, reinterpret_cast<double*>(c->counters), kCounters, 0.0)) return s;
  if (dqmc_status s = fill_small(c, reinterpret_cast<double*>(c->err_flag), 1, 0.0)) return s;
  // measurement partials and their completion counters
  if (dqmc_status s = fill_small(c, c->mpart, 4 * (size_t)((N + kMeasRows - 1) / kMeasRows) + 4, 0.0)) return s;
  if (dqmc_status s = fill_small(c, c->tdpart, td_part_size(c), 0.0)) return s;
  if (c->seeds.empty()) c->seeds.assign(c->nch, c->m.seed);
  if (c->nch == 1 && !c->side) {
    HIPCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    for (hipEvent_t& e : c->fork_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  if (wants_shadow(c))
    if (dqmc_status s = shadow_setup(c)) return s;
  // chain keys: host -> staging buffer -> counters[3] of every chain
  HIPCHK(hipMemcpyAsync(c->gbuf, c->seeds.data(), sizeof(uint64_t) * c->nch, hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_scatter, dim3(1, c->nch), dim3(64), 0, c->stream, reinterpret_cast<double*>(c->counters + 3),
                     c->gbuf, 1, c->cs);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  c->bound = true;
  c->initialized = false;
  return DQMC_OK;
}

}  // namespace

extern "C" {

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
  return setup_device(c);
}

dqmc_status dqmc_set_state(dqmc_ctx* c, const double* field_host, uint64_t sweep_counter) {
  if (!c || !field_host) return fail(c, DQMC_E_ARG, "null argument");
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  const size_t n = (size_t)c->L * c->Nf;
  for (size_t e = 0; e < n; ++e) {
    const double v = field_host[e];
    if (!field_value_ok(c->m.field, v))
      return fail(c, DQMC_E_ARG, "field values must be +-1 (Ising), eta(l) (four-valued) or finite (Gaussian)");
  }
  HIPCHK(hipMemcpyAsync(c->field, field_host, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  if (dqmc_status s = expand_field(c)) return s;
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
    HIPCHK(hipMemcpyAsync(field_host, c->field, (size_t)c->L * c->Nf * sizeof(double), hipMemcpyDeviceToHost,
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
  const size_t n = (size_t)c->L * c->Nf;
  const int kind = c->cplx ? (int)DQMC_FIELD_ISING4 : (int)c->m.field;   // the same four values
  hipLaunchKernelGGL(k_random_field, gridc(c, grid1(n)), dim3(256), 0, c->stream, c->field, c->L, c->Nf,
                     c->counters, kind, field4_table(), c->cs);
  HIPCHK(hipGetLastError());
  if (dqmc_status s = expand_field(c)) return s;
  if (dqmc_status s = fill_small(c, reinterpret_cast<double*>(c->counters + 2), 1, 0.0)) return s;
  if (dqmc_status s = fill_small(c, reinterpret_cast<double*>(c->counters + 4), 1, 0.0)) return s;
  HIPCHK(hipStreamSynchronize(c->stream));
  c->initialized = false;
  return DQMC_OK;
}

dqmc_status dqmc_init(dqmc_ctx* c) {
  if (!c) return DQMC_E_ARG;
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  // statistics, bins, flag
  if (dqmc_status s = fill_small(c, c->bins, 4, 0.0)) return s;
  if (dqmc_status s = fill_small(c, c->tdbins, (size_t)(c->L + 1) * kTdStride + 4, 0.0)) return s;
  if (dqmc_status s = fill_small(c, c->eq_bins, eq_bins_size(c), 0.0)) return s;
  if (td_corr_size(c))
    if (dqmc_status s = fill_small(c, c->td_corr, td_corr_size(c), 0.0)) return s;
  if (dqmc_status s = fill_small(c, c->prec_hist, 2 * (size_t)c->nk + 2, 0.0)) return s;
  if (dqmc_status s = fill_small(c, c->prec_tot, 4, 0.0)) return s;
  if (dqmc_status s = fill_small(c, reinterpret_cast<double*>(c->counters), 2, 0.0)) return s;
  if (dqmc_status s = fill_small(c, reinterpret_cast<double*>(c->err_flag), 1, 0.0)) return s;
  if (dqmc_status s = fill_small(c, c->phase, 1, 1.0)) return s;
  if (dqmc_status s = fill_small(c, c->phase + 1, 3, 0.0)) return s;
  if (dqmc_status s = reanchor(c)) return s;
  if (dqmc_status s = read_flag(c)) return s;
  c->poisoned = false;
  c->initialized = true;
  return DQMC_OK;
}

dqmc_status dqmc_sweep(dqmc_ctx* c, int32_t n_sweeps, int32_t meas, dqmc_stats* st) {
  if (!c || n_sweeps < 0) return fail(c, DQMC_E_ARG, "bad arguments");
  if (!c->bound || !c->initialized || c->poisoned) return fail(c, DQMC_E_STATE, "context not initialised");
  if (meas & ~15) return fail(c, DQMC_E_ARG, "unknown measurement flags");
  if (c->cplx && (meas & ~1)) return fail(c, DQMC_E_UNSUPPORTED, "a complex field measures the estimators of bit 0 only");
  if (c->nfl == 2 && (meas & ~1))
    return fail(c, DQMC_E_UNSUPPORTED, "the two-flavour form measures the estimators of bit 0 only");
  if (c->nvx && (meas & ~1))
    return fail(c, DQMC_E_UNSUPPORTED, "general vertices measure the estimators of bit 0 only");
  if ((meas & 8) && (!(meas & 2) || c->eq_norb < 1 || td_corr_size(c) == 0))
    return fail(c, DQMC_E_STATE, "time-displaced correlations need bit 1 and dqmc_eq_setup");
  if ((meas & 2) && c->td_norb < 1) return fail(c, DQMC_E_STATE, "time-displaced measurement not set up");
  if ((meas & 4) && c->eq_norb < 1) return fail(c, DQMC_E_STATE, "lattice-resolved correlations not set up");
  const auto t0 = std::chrono::steady_clock::now();
  for (int s = 0; s < n_sweeps; ++s)
    if (dqmc_status r = c->cplx       ? csweep_once(c, meas)
                        : c->nfl == 2 ? fl2sweep_once(c, meas)
                        : c->nvx      ? vx_sweep_once(c, meas)
                                      : sweep_once(c, meas))
      return r;
  if (dqmc_status r = read_flag(c)) return r;
  const auto t1 = std::chrono::steady_clock::now();
  if (st) {
    if (dqmc_status s = chain_stats(c, -1, st)) return s;
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
  if (dqmc_status s = fill_small(c, c->tdbins, (size_t)(c->L + 1) * kTdStride + 4, 0.0)) return s;
  if (dqmc_status s = fill_small(c, c->eq_bins, eq_bins_size(c), 0.0)) return s;
  if (td_corr_size(c))
    if (dqmc_status s = fill_small(c, c->td_corr, td_corr_size(c), 0.0)) return s;
  HIPCHK(hipStreamSynchronize(c->stream));
  return DQMC_OK;
}

dqmc_status dqmc_read_phase(dqmc_ctx* c, double* out3) {
  if (!c || !out3) return DQMC_E_ARG;
  if (!c->cplx && c->nfl != 2) return fail(c, DQMC_E_UNSUPPORTED, "only a complex field or two flavours carry a phase");
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  HIPCHK(hipMemcpyAsync(out3, c->phase, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return DQMC_OK;
}

}  // extern "C"

namespace {

// G(tau) from scratch for the field the context points at, into G_dev: the
// right chain 0 -> tau and the left chain beta -> tau in chunks aligned to
// n_wrap, then the merge (enqueued only).
dqmc_status green_scratch_into(dqmc_ctx* c, int tau, double* G_dev) {
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
  return merge(c, right, left, G_dev, nullptr);
}

}  // namespace

extern "C" {

dqmc_status dqmc_green_scratch(dqmc_ctx* c, int32_t tau, double* G_dev) {
  if (!c || !G_dev || tau < 0 || tau > c->L) return fail(c, DQMC_E_ARG, "bad arguments");
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  if (dqmc_status s = green_scratch_into(c, tau, G_dev)) return s;
  HIPCHK(hipStreamSynchronize(c->stream));
  return read_flag(c);
}

dqmc_status dqmc_ratio(dqmc_ctx* c, int32_t tau, int32_t site, double s_new, double* R) {
  if (!c || !R || tau < 1 || site < 0 || !std::isfinite(s_new)) return fail(c, DQMC_E_ARG, "bad arguments");
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  if (c->nch != 1) return fail(c, DQMC_E_UNSUPPORTED, "single chains only");
  if (tau > c->L || site >= c->N) return fail(c, DQMC_E_ARG, "tau or site out of range");
  if (!field_value_ok(c->m.field, s_new)) return fail(c, DQMC_E_ARG, "not a value of the field");
  if (c->cplx || c->nfl == 2 || c->nvx)
    return fail(c, DQMC_E_UNSUPPORTED, "not built for a complex field, two flavours or general vertices");
  if (dqmc_status s = dqmc_green_scratch(c, tau, c->Gs)) return s;
  hipLaunchKernelGGL(k_ratio, dim3(1), dim3(64), 0, c->stream, c->Gs, c->N, site,
                     c->field + (size_t)(tau - 1) * c->N, s_new, c->m.coupling, c->m.alpha, c->m.n_col,
                     (int)c->m.field, field4_table(), c->logdet + 1);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(R, c->logdet + 1, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return DQMC_OK;
}

dqmc_status dqmc_logdet(dqmc_ctx* c, double* logdet) {
  if (!c || !logdet) return DQMC_E_ARG;
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  if (c->cplx || c->nfl == 2) return fail(c, DQMC_E_UNSUPPORTED, "not built for a complex field or two flavours");
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

dqmc_status dqmc_grad_logdet(dqmc_ctx* c, double* grad_dev, double* prec) {
  if (!c || !grad_dev) return fail(c, DQMC_E_ARG, "null argument");
  if (c->cplx || c->nfl == 2 || c->nvx)
    return fail(c, DQMC_E_UNSUPPORTED, "not built for a complex field, two flavours or general vertices");
  if (!c->bound || !c->initialized || c->poisoned) return fail(c, DQMC_E_STATE, "context not initialised");
  if (dqmc_status s = grad_pass(c)) return s;
  HIPCHK(hipMemcpyAsync(grad_dev, c->grad, (size_t)c->L * c->N * sizeof(double), hipMemcpyDeviceToDevice,
                        c->stream));
  if (prec) HIPCHK(hipMemcpyAsync(prec, c->gprec, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return read_flag(c);
}

dqmc_status dqmc_langevin(dqmc_ctx* c, double eps, int32_t n_steps) {
  if (!c || n_steps < 0 || !(eps > 0.0) || !std::isfinite(eps)) return fail(c, DQMC_E_ARG, "bad arguments");
  if (c->m.field != DQMC_FIELD_GAUSS || c->nfl == 2)
    return fail(c, DQMC_E_UNSUPPORTED, "Langevin steps need a one-flavour Gaussian field");
  if (!c->bound || !c->initialized || c->poisoned) return fail(c, DQMC_E_STATE, "context not initialised");
  for (int k = 0; k < n_steps; ++k)
    if (dqmc_status s = langevin_once(c, eps)) return s;
  return read_flag(c);
}

dqmc_status dqmc_get_langevin_step(dqmc_ctx* c, uint64_t* step) {
  if (!c || !step) return fail(c, DQMC_E_ARG, "null argument");
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  unsigned long long v = 0;
  HIPCHK(hipMemcpyAsync(&v, c->counters + 4, sizeof(v), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *step = v;
  return DQMC_OK;
}

dqmc_status dqmc_set_langevin_step(dqmc_ctx* c, uint64_t step) {
  if (!c) return DQMC_E_ARG;
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  unsigned long long v = step;
  HIPCHK(hipMemcpyAsync(c->counters + 4, &v, sizeof(v), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return DQMC_OK;
}

dqmc_status dqmc_td_setup(dqmc_ctx* c, int32_t norb, const int32_t* orb_of, const double* phase, int32_t n_cells) {
  if (!c || !orb_of || !phase || norb < 1 || norb > kTdMaxOrb || n_cells < 1)
    return fail(c, DQMC_E_ARG, "bad arguments");
  if (c->cplx || c->nfl == 2 || c->nvx)
    return fail(c, DQMC_E_UNSUPPORTED, "not built for a complex field, two flavours or general vertices");
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  for (int i = 0; i < c->N; ++i) {
    if (orb_of[i] < 0 || orb_of[i] >= norb) return fail(c, DQMC_E_ARG, "orbital index out of range");
    if (!std::isfinite(phase[2 * i]) || !std::isfinite(phase[2 * i + 1])) return fail(c, DQMC_E_ARG, "bad phase");
  }
  HIPCHK(hipMemcpyAsync(c->kph, phase, 2 * sizeof(double) * c->N, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->korb, orb_of, sizeof(int32_t) * c->N, hipMemcpyHostToDevice, c->stream));
  if (dqmc_status s = fill_small(c, c->tdbins, (size_t)(c->L + 1) * kTdStride + 4, 0.0)) return s;
  HIPCHK(hipStreamSynchronize(c->stream));
  c->td_norb = norb;
  c->td_cells = n_cells;
  return DQMC_OK;
}

dqmc_status dqmc_eq_setup(dqmc_ctx* c, int32_t L1, int32_t L2, int32_t norb, const int32_t* site, const double* sign) {
  if (!c || !site || !sign || L1 < 1 || L2 < 1 || norb < 1 || norb > kEqMaxOrb)
    return fail(c, DQMC_E_ARG, "bad arguments");
  if (c->cplx || c->nfl == 2 || c->nvx)
    return fail(c, DQMC_E_UNSUPPORTED, "not built for a complex field, two flavours or general vertices");
  if (!c->bound) return fail(c, DQMC_E_STATE, "not bound");
  if ((int64_t)L1 * L2 * norb != c->N) return fail(c, DQMC_E_ARG, "L1 * L2 * norb must equal the number of orbitals");
  std::vector<char> seen(c->N, 0);
  for (int i = 0; i < c->N; ++i) {
    if (site[i] < 0 || site[i] >= c->N || seen[site[i]]) return fail(c, DQMC_E_ARG, "site map is not a permutation");
    seen[site[i]] = 1;
    if (sign[i] != 1.0 && sign[i] != -1.0) return fail(c, DQMC_E_ARG, "sublattice signs must be +1 or -1");
  }
  HIPCHK(hipMemcpyAsync(c->eq_sign, sign, sizeof(double) * c->N, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->eq_site, site, sizeof(int32_t) * c->N, hipMemcpyHostToDevice, c->stream));
  if (dqmc_status s = fill_small(c, c->eq_bins, eq_bins_size(c), 0.0)) return s;
  if (td_corr_size(c))
    if (dqmc_status s = fill_small(c, c->td_corr, td_corr_size(c), 0.0)) return s;
  HIPCHK(hipStreamSynchronize(c->stream));
  c->eq_L1 = L1;
  c->eq_L2 = L2;
  c->eq_norb = norb;
  return DQMC_OK;
}

dqmc_status dqmc_eq_read_bins(dqmc_ctx* c, double* sums_host, double* count) {
  if (!c || !sums_host) return DQMC_E_ARG;
  if (!c->bound || c->eq_norb < 1) return fail(c, DQMC_E_STATE, "lattice-resolved correlations not set up");
  const size_t nb = (size_t)c->eq_L1 * c->eq_L2 * c->eq_norb * c->eq_norb;
  std::vector<double> raw(4 * nb + 1);
  HIPCHK(hipMemcpyAsync(raw.data(), c->eq_bins, raw.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  std::copy(raw.begin(), raw.begin() + 4 * nb, sums_host);
  if (count) *count = raw.back();
  return DQMC_OK;
}

dqmc_status dqmc_eq_read_spin_z(dqmc_ctx* c, double* sz_host, double* count) {
  if (!c || !sz_host) return DQMC_E_ARG;
  if (!c->bound || c->eq_norb < 1) return fail(c, DQMC_E_STATE, "lattice-resolved correlations not set up");
  const size_t nb = (size_t)c->eq_L1 * c->eq_L2 * c->eq_norb * c->eq_norb;
  double raw[1 + kEqMaxOrb];
  HIPCHK(hipMemcpyAsync(raw, c->eq_bins + 4 * nb, (1 + c->eq_norb) * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int a = 0; a < c->eq_norb; ++a) sz_host[a] = raw[1 + a];
  if (count) *count = raw[0];
  return DQMC_OK;
}

dqmc_status dqmc_td_read_corr_bins(dqmc_ctx* c, double* sums_host, double* count) {
  if (!c || !sums_host) return DQMC_E_ARG;
  if (!c->bound || c->eq_norb < 1 || td_corr_size(c) == 0)
    return fail(c, DQMC_E_STATE, "lattice-resolved correlations not set up");
  const size_t nb = (size_t)c->eq_L1 * c->eq_L2 * c->eq_norb * c->eq_norb, st = td_corr_stride(c);
  std::vector<double> raw(td_corr_size(c));
  HIPCHK(hipMemcpyAsync(raw.data(), c->td_corr, raw.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int t = 0; t <= c->L; ++t)
    std::copy(raw.begin() + t * st, raw.begin() + t * st + 4 * nb, sums_host + (size_t)t * 4 * nb);
  if (count) *count = raw[(size_t)(c->L + 1) * st];
  return DQMC_OK;
}

// Copies S(K, tau) for tau = 0..L out of the device layout (stride kTdStride,
// entry (a * kTdMaxOrb + b) * 2) into [L+1][norb][norb][2].
static void td_compact(const dqmc_ctx* c, const double* dev_layout, double* out) {
  const int no = c->td_norb;
  for (int t = 0; t <= c->L; ++t)
    for (int a = 0; a < no; ++a)
      for (int b = 0; b < no; ++b)
        for (int r = 0; r < 2; ++r)
          out[(((size_t)t * no + a) * no + b) * 2 + r] = dev_layout[(size_t)t * kTdStride + (a * kTdMaxOrb + b) * 2 + r];
}

dqmc_status dqmc_td_measure(dqmc_ctx* c, double* S_host, double* prec) {
  if (!c) return DQMC_E_ARG;
  if (!c->bound || !c->initialized || c->poisoned) return fail(c, DQMC_E_STATE, "context not initialised");
  if (dqmc_status s = td_pass(c)) return s;
  std::vector<double> raw;
  if (S_host) {
    raw.resize((size_t)(c->L + 1) * kTdStride);
    HIPCHK(hipMemcpyAsync(raw.data(), c->tdS, raw.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  }
  double pr[2] = {0.0, 0.0};
  if (prec) HIPCHK(hipMemcpyAsync(pr, c->gprec, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (S_host) td_compact(c, raw.data(), S_host);
  if (prec) { prec[0] = pr[0]; prec[1] = pr[1]; }
  return read_flag(c);
}

dqmc_status dqmc_td_read_bins(dqmc_ctx* c, double* sums_host, double* count) {
  if (!c || !sums_host) return DQMC_E_ARG;
  if (!c->bound || c->td_norb < 1) return fail(c, DQMC_E_STATE, "time-displaced measurement not set up");
  std::vector<double> raw((size_t)(c->L + 1) * kTdStride + 1);
  HIPCHK(hipMemcpyAsync(raw.data(), c->tdbins, raw.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  td_compact(c, raw.data(), sums_host);
  if (count) *count = raw.back();
  return DQMC_OK;
}

dqmc_status dqmc_set_chunk_kernel(dqmc_ctx* c, int32_t enable) {
  if (!c || enable < -1 || enable > 1) return fail(c, DQMC_E_ARG, "bad arguments");
  c->fused = enable;
  return DQMC_OK;
}

dqmc_status dqmc_timing_enable(dqmc_ctx* c, dqmc_kernel kernel, int32_t enable) {
  if (!c || enable < 0 ||
      (kernel != DQMC_KERNEL_BLOCK_UPDATE && kernel != DQMC_KERNEL_GEMM && kernel != DQMC_KERNEL_STABILISE))
    return DQMC_E_ARG;
  c->timing = enable != 0;
  c->timing_open = false;
  c->timing_kernel = kernel;
  c->timing_every = enable > 1 ? enable : 1;
  c->timing_seen = 0;
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

dqmc_status dqmc_mz_frame_hopping(int32_t n, const double* T, double h, const double* sign, double* K_out) {
  if (n < 1 || !T || !sign || !K_out || !std::isfinite(h)) return DQMC_E_ARG;
  for (int i = 0; i < n; ++i)
    if (sign[i] != 1.0 && sign[i] != -1.0) return DQMC_E_ARG;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double up = T[(size_t)i * n + j] - (i == j ? h : 0.0);                // K_1
      const double dn = -sign[i] * (T[(size_t)j * n + i] + (i == j ? h : 0.0)) * sign[j];   // K_2
      if (!std::isfinite(up) || up != dn) return DQMC_E_UNSUPPORTED;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) K_out[(size_t)i * n + j] = T[(size_t)i * n + j] - (i == j ? h : 0.0);
  return DQMC_OK;
}

dqmc_status dqmc_hubbard_coupling(double U, double dtau, dqmc_field_kind kind, double* coupling) {
  if (!coupling || !(dtau > 0.0) || !std::isfinite(U)) return DQMC_E_ARG;
  if (kind == DQMC_FIELD_ISING) {
    if (U < 0.0) return DQMC_E_ARG;
    *coupling = std::acosh(std::exp(dtau * U / 2.0));
  } else if (kind == DQMC_FIELD_GAUSS) {
    if (U < 0.0) return DQMC_E_ARG;
    *coupling = std::sqrt(dtau * U);
  } else if (kind == DQMC_FIELD_ISING4 || kind == DQMC_FIELD_ISING4_IMAG) {
    // the real coupling of the attractive frame, or c of the imaginary one i c
    if (U < 0.0) return DQMC_E_ARG;
    *coupling = std::sqrt(dtau * U / 2.0);
  } else {
    return DQMC_E_ARG;
  }
  return DQMC_OK;
}

}  // extern "C"

// ================================================================ batch ==
// A batch of independent chains.  Chains whose models agree in everything
// but the seed (same lattice, N, L, n_wrap, couplings) form a group; a group
// is one context whose every launch covers all of its chains (blockIdx.y =
// chain), so one sweep of the whole batch is one launch sequence per group.
// That sequence can be captured once into a hipGraph and replayed.
struct dqmc_batch {
  std::vector<dqmc_ctx*> groups;
  std::vector<int> group_of, index_of;
  std::vector<size_t> group_off;   // doubles
  size_t total = 0;
  double* work = nullptr;
  hipStream_t stream = nullptr;
  bool bound = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int graph_sweeps = 0, graph_measure = -1;
  // with several groups, one stream per group (default priority) and the
  // events that fork it from the batch stream and join it back
  std::vector<hipStream_t> gstream;
  std::vector<hipEvent_t> gjoin;
  hipEvent_t gfork = nullptr;
  bool side_by_side = true;   // dqmc_batch_set_side_by_side
  std::string err;
  ~dqmc_batch() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    for (dqmc_ctx* g : groups) delete g;
    for (hipEvent_t e : gjoin) (void)hipEventDestroy(e);
    if (gfork) (void)hipEventDestroy(gfork);
    for (hipStream_t s : gstream) (void)hipStreamDestroy(s);
  }
};

namespace {

dqmc_status bfail(dqmc_batch* b, dqmc_status s, const std::string& msg) {
  if (b) b->err = msg;
  return s;
}

#define BHIPCHK_(expr)                                                                    \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return bfail(b, DQMC_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

bool same_group(const dqmc_model& a, const dqmc_model& b, const double* Ka, const double* Kb) {
  return a.n == b.n && a.n_slices == b.n_slices && a.beta == b.beta && a.dtau == b.dtau && a.n_wrap == b.n_wrap &&
         a.n_col == b.n_col && a.field == b.field && a.coupling == b.coupling && a.alpha == b.alpha &&
         a.u_int == b.u_int && a.trotter == b.trotter && a.prec_threshold == b.prec_threshold &&
         a.prop_width == b.prop_width && std::memcmp(Ka, Kb, sizeof(double) * a.n * a.n) == 0;
}

// Per-chain region of a group: G, field, slots, then the chain scratch.
size_t group_chain_doubles(dqmc_ctx* c) {
  const size_t N = c->N, NN = N * N;
  Layout l;
  l.take(NN);
  l.take((size_t)c->L * N);
  l.take((size_t)(c->nk + 1) * (2 * NN + N));
  return l.off + layout_chain(c, nullptr);
}

void place_group(dqmc_ctx* c, double* base) {
  const size_t N = c->N, NN = N * N;
  c->cs = group_chain_doubles(c);          // size only: touches no pointer
  const size_t sh = layout_shared(c, base);
  double* chain0 = base + sh;
  Layout l;
  c->G = chain0 + l.take(NN);
  c->field = chain0 + l.take((size_t)c->L * N);
  c->slots = chain0 + l.take((size_t)(c->nk + 1) * (2 * NN + N));
  layout_chain(c, chain0 + l.off);
  c->work = base;
}

// Every per-chain pointer of every chain, and every shared pointer, must lie
// inside [lo, hi) with its full extent: checked on the host before any launch.
bool layout_ok(const dqmc_ctx* c, const double* lo, const double* hi) {
  const size_t N = c->N, NN = N * N, last = (size_t)(c->nch - 1) * c->cs;
  auto in = [&](const void* p, size_t n, bool per_chain) {
    const double* q = static_cast<const double*>(p);
    if (!q || q < lo) return false;
    return q + (per_chain ? last : 0) + n <= hi;
  };
  bool ok = in(c->E, NN, false) && in(c->Einv, NN, false) && in(c->Eh, NN, false) && in(c->Ehinv, NN, false) &&
            in(c->Kd, NN, false) && in(c->uid.Q, NN, false) && in(c->uid.D, N, false) && in(c->uid.T, NN, false) &&
            in(c->gbuf, 8 * (size_t)c->nch, false);
  ok = ok && in(c->G, NN, true) && in(c->field, (size_t)c->L * N, true) &&
       in(c->slots, (size_t)(c->nk + 1) * (2 * NN + N), true);
  for (int i = 0; i < 6; ++i) ok = ok && in(c->S[i], NN, true);
  for (const double* p : {c->Vall, c->VTall, c->Zq, c->Rt, c->X, c->RHS, c->Gs, c->T1, c->G2}) ok = ok && in(p, NN, true);
  ok = ok && in(c->XA, 3 * NN, true) && in(c->Mgj, 64 * N, true) && in(c->Uinv, uinv_size(c), true);
  for (const UDVp* u : {&c->cur, &c->hA, &c->hB}) ok = ok && in(u->Q, NN, true) && in(u->D, N, true) && in(u->T, NN, true);
  ok = ok && in(c->field_alt, (size_t)c->L * N, true) && in(c->norms, N, true) && in(c->piv, N / 2 + 1, true) &&
       in(c->moves, kLuMoves + 1, true) && in(c->bins, 4, true) && in(c->prec_hist, 2 * (size_t)c->nk + 2, true) &&
       in(c->prec_tot, 4, true) && in(c->logdet, 4, true) && in(c->grad, (size_t)c->L * N, true) && in(c->gprec, 4, true) &&
       in(c->mpart, 4 * (size_t)((N + kMeasRows - 1) / kMeasRows) + 4, true) &&
       in(c->draws, 4 * (size_t)c->L * N, true) &&
       in(c->TD[0], NN, true) && in(c->TD[1], NN, true) && in(c->TD[2], NN, true) && in(c->TD[3], NN, true) &&
       in(c->tdS, (size_t)(c->L + 1) * kTdStride, true) &&
       in(c->tdbins, (size_t)(c->L + 1) * kTdStride + 4, true) &&
       in(c->tdpart, td_part_size(c), true) && in(c->a00, 2 * kTdMaxOrb, true) &&
       in(c->kph, 2 * N, false) && in(c->korb, N / 2 + 1, false) && in(c->eq_sign, N, false) &&
       in(c->eq_site, N / 2 + 1, false) && in(c->eq_bins, eq_bins_size(c), true) && in(c->td_g00, N, true) &&
       (td_corr_size(c) == 0 || in(c->td_corr, td_corr_size(c), true)) &&
       in(c->counters, kCounters, true) && in(c->err_flag, 1, true);
  return ok;
}

// Sweep flags of one group for a batch call's measure flags: bit 0 the
// equal-time estimators, bit 1 the time-displaced pass and bit 2 the
// lattice-resolved correlations, each where the group has been set up for it.
int group_flags(const dqmc_ctx* c, int measure) {
  return (measure & 1) | (((measure & 2) && c->td_norb > 0) ? 2 : 0) | (((measure & 4) && c->eq_norb > 0) ? 4 : 0);
}

// One sweep of every group.  Groups touch disjoint parts of the work buffer,
// so with several groups each sweeps on a stream of its own, forked from the
// batch stream and joined back into it by events (a capture records them as
// parallel branches); the launches of one group then fill the CUs that
// another group's latency-bound steps leave idle.
dqmc_status sweep_groups(dqmc_batch* b, int measure) {
  if (!b->side_by_side || b->gstream.size() != b->groups.size()) {
    for (dqmc_ctx* c : b->groups)
      if (dqmc_status r = sweep_once(c, group_flags(c, measure))) return bfail(b, r, c->err);
    return DQMC_OK;
  }
  BHIPCHK_(hipEventRecord(b->gfork, b->stream));
  dqmc_status first = DQMC_OK;
  std::string why;
  for (size_t g = 0; g < b->groups.size(); ++g) {
    dqmc_ctx* c = b->groups[g];
    BHIPCHK_(hipStreamWaitEvent(b->gstream[g], b->gfork, 0));
    c->stream = b->gstream[g];
    const dqmc_status r = sweep_once(c, group_flags(c, measure));
    c->stream = b->stream;
    if (r && !first) { first = r; why = c->err; }
    // joined even after a failure, so that a capture stays well formed
    BHIPCHK_(hipEventRecord(b->gjoin[g], b->gstream[g]));
    BHIPCHK_(hipStreamWaitEvent(b->stream, b->gjoin[g], 0));
    if (r) break;
  }
  return first ? bfail(b, first, why) : DQMC_OK;
}

dqmc_status batch_flags(dqmc_batch* b) {
  for (dqmc_ctx* g : b->groups)
    if (dqmc_status s = read_flag(g)) return bfail(b, s, g->err);
  return DQMC_OK;
}

}  // namespace

extern "C" {

dqmc_status dqmc_batch_create(int32_t n_chains, const dqmc_model* models, const double* const* K, dqmc_batch** out) {
  if (!out) return DQMC_E_ARG;
  *out = nullptr;
  if (n_chains < 1 || !models || !K) return DQMC_E_ARG;
  for (int i = 0; i < n_chains; ++i)
    if (models[i].field == DQMC_FIELD_ISING4_IMAG) return DQMC_E_UNSUPPORTED;   // single chains only
  dqmc_batch* b = new (std::nothrow) dqmc_batch();
  if (!b) return DQMC_E_NOMEM;
  std::vector<int> first_of;   // chain index that defines each group
  b->group_of.resize(n_chains);
  b->index_of.resize(n_chains);
  for (int i = 0; i < n_chains; ++i) {
    int g = -1;
    for (size_t k = 0; k < first_of.size() && g < 0; ++k)
      if (same_group(models[first_of[k]], models[i], K[first_of[k]], K[i])) g = (int)k;
    if (g < 0) {
      dqmc_ctx* c = nullptr;
      dqmc_status s = dqmc_create(&models[i], K[i], nullptr, &c);
      if (s != DQMC_OK) { delete b; return s; }
      c->nch = 0;
      c->no_shadow = true;   // a group's buffers are laid out by place_group, without a shadow part
      b->groups.push_back(c);
      first_of.push_back(i);
      g = (int)first_of.size() - 1;
    }
    dqmc_ctx* c = b->groups[g];
    b->group_of[i] = g;
    b->index_of[i] = c->nch++;
    c->seeds.push_back(models[i].seed);
  }
  size_t off = 0;
  for (dqmc_ctx* c : b->groups) {
    Layout l;
    l.take(layout_shared(c, nullptr));
    l.take(group_chain_doubles(c) * c->nch);
    b->group_off.push_back(off);
    off += l.off;
  }
  b->total = off;
  *out = b;
  return DQMC_OK;
}

dqmc_status dqmc_batch_query_size(const dqmc_batch* b, size_t* work_bytes) {
  if (!b || !work_bytes) return DQMC_E_ARG;
  *work_bytes = b->total * sizeof(double);
  return DQMC_OK;
}

dqmc_status dqmc_batch_bind(dqmc_batch* b, void* work, void* stream) {
  if (!b || !work) return bfail(b, DQMC_E_ARG, "null buffer");
  if (reinterpret_cast<uintptr_t>(work) % 256) return bfail(b, DQMC_E_ARG, "buffer must be 256-byte aligned");
  b->work = static_cast<double*>(work);
  b->stream = static_cast<hipStream_t>(stream);
  for (size_t g = 0; g < b->groups.size(); ++g) {
    dqmc_ctx* c = b->groups[g];
    c->stream = b->stream;
    double* base = b->work + b->group_off[g];
    place_group(c, base);
    const double* hi = (g + 1 < b->groups.size()) ? b->work + b->group_off[g + 1] : b->work + b->total;
    if (!layout_ok(c, base, hi)) return bfail(b, DQMC_E_STATE, "internal layout check failed");
  }
  for (dqmc_ctx* c : b->groups)
    if (dqmc_status s = setup_device(c)) return bfail(b, s, c->err);
  if (b->groups.size() > 1 && b->gstream.empty()) {
    BHIPCHK_(hipEventCreateWithFlags(&b->gfork, hipEventDisableTiming));
    for (size_t g = 0; g < b->groups.size(); ++g) {
      hipStream_t st = nullptr;
      hipEvent_t ev = nullptr;
      BHIPCHK_(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      b->gstream.push_back(st);
      BHIPCHK_(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      b->gjoin.push_back(ev);
    }
  }
  b->bound = true;
  return DQMC_OK;
}

dqmc_status dqmc_batch_random_fields(dqmc_batch* b) {
  if (!b) return DQMC_E_ARG;
  if (!b->bound) return bfail(b, DQMC_E_STATE, "not bound");
  for (dqmc_ctx* c : b->groups)
    if (dqmc_status s = dqmc_random_field(c)) return bfail(b, s, c->err);
  return DQMC_OK;
}

dqmc_status dqmc_batch_set_state(dqmc_batch* b, int32_t chain, const double* field_host, uint64_t sweep_counter) {
  if (!b || !field_host || chain < 0 || chain >= (int)b->group_of.size()) return bfail(b, DQMC_E_ARG, "bad arguments");
  if (!b->bound) return bfail(b, DQMC_E_STATE, "not bound");
  dqmc_ctx* c = b->groups[b->group_of[chain]];
  const size_t co = (size_t)b->index_of[chain] * c->cs;
  const size_t n = (size_t)c->L * c->N;
  for (size_t e = 0; e < n; ++e)
    if (!field_value_ok(c->m.field, field_host[e])) return bfail(b, DQMC_E_ARG, "bad field value");
  BHIPCHK_(hipMemcpyAsync(c->field + co, field_host, n * sizeof(double), hipMemcpyHostToDevice, b->stream));
  unsigned long long ctr = sweep_counter;
  BHIPCHK_(hipMemcpyAsync(reinterpret_cast<double*>(c->counters + 2) + co, &ctr, sizeof(ctr), hipMemcpyHostToDevice,
                          b->stream));
  BHIPCHK_(hipStreamSynchronize(b->stream));
  c->initialized = false;
  return DQMC_OK;
}

dqmc_status dqmc_batch_get_state(dqmc_batch* b, int32_t chain, double* field_host, uint64_t* sweep_counter) {
  if (!b || chain < 0 || chain >= (int)b->group_of.size()) return bfail(b, DQMC_E_ARG, "bad arguments");
  if (!b->bound) return bfail(b, DQMC_E_STATE, "not bound");
  dqmc_ctx* c = b->groups[b->group_of[chain]];
  const size_t co = (size_t)b->index_of[chain] * c->cs;
  if (field_host)
    BHIPCHK_(hipMemcpyAsync(field_host, c->field + co, (size_t)c->L * c->N * sizeof(double), hipMemcpyDeviceToHost,
                            b->stream));
  unsigned long long ctr = 0;
  BHIPCHK_(hipMemcpyAsync(&ctr, reinterpret_cast<double*>(c->counters + 2) + co, sizeof(ctr), hipMemcpyDeviceToHost,
                          b->stream));
  BHIPCHK_(hipStreamSynchronize(b->stream));
  if (sweep_counter) *sweep_counter = ctr;
  return DQMC_OK;
}

dqmc_status dqmc_batch_init(dqmc_batch* b) {
  if (!b) return DQMC_E_ARG;
  if (!b->bound) return bfail(b, DQMC_E_STATE, "not bound");
  for (dqmc_ctx* c : b->groups)
    if (dqmc_status s = dqmc_init(c)) return bfail(b, s, c->err);
  return DQMC_OK;
}

dqmc_status dqmc_batch_sweep(dqmc_batch* b, int32_t n_sweeps, int32_t measure, dqmc_stats* st) {
  if (!b || n_sweeps < 0) return bfail(b, DQMC_E_ARG, "bad arguments");
  if (measure & ~7) return bfail(b, DQMC_E_ARG, "unknown measurement flags");
  for (dqmc_ctx* c : b->groups)
    if (!c->bound || !c->initialized || c->poisoned) return bfail(b, DQMC_E_STATE, "batch not initialised");
  const auto t0 = std::chrono::steady_clock::now();
  int left = n_sweeps;
  if (b->gexec && b->graph_measure == measure) {
    while (left >= b->graph_sweeps) {
      BHIPCHK_(hipGraphLaunch(b->gexec, b->stream));
      left -= b->graph_sweeps;
    }
  }
  for (int s = 0; s < left; ++s)
    if (dqmc_status r = sweep_groups(b, measure)) return r;
  if (dqmc_status r = batch_flags(b)) return r;
  const auto t1 = std::chrono::steady_clock::now();
  if (st) {
    dqmc_stats tot{};
    double psum = 0.0;
    for (dqmc_ctx* c : b->groups) {
      dqmc_stats g{};
      if (dqmc_status r = chain_stats(c, -1, &g)) return bfail(b, r, c->err);
      tot.proposals += g.proposals;
      tot.accepted += g.accepted;
      tot.n_prec += g.n_prec;
      psum += g.prec_mean * g.n_prec;
      tot.prec_max = std::max(tot.prec_max, g.prec_max);
    }
    tot.prec_mean = tot.n_prec ? psum / tot.n_prec : 0.0;
    tot.seconds = std::chrono::duration<double>(t1 - t0).count();
    *st = tot;
  }
  return DQMC_OK;
}

dqmc_status dqmc_batch_capture(dqmc_batch* b, int32_t sweeps_per_graph, int32_t measure) {
  if (!b || sweeps_per_graph < 1) return bfail(b, DQMC_E_ARG, "bad arguments");
  if (measure & ~7) return bfail(b, DQMC_E_ARG, "unknown measurement flags");
  if (!b->bound) return bfail(b, DQMC_E_STATE, "not bound");
  if (!b->stream) return bfail(b, DQMC_E_ARG, "graph capture needs a stream other than the null stream");
  for (dqmc_ctx* c : b->groups)
    if (c->timing) return bfail(b, DQMC_E_STATE, "disable kernel timing before capturing");
  if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  BHIPCHK_(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  dqmc_status st = DQMC_OK;
  for (int s = 0; s < sweeps_per_graph && st == DQMC_OK; ++s) st = sweep_groups(b, measure);
  hipError_t ce = hipStreamEndCapture(b->stream, &b->graph);
  if (st != DQMC_OK) return bfail(b, st, "capture failed");
  BHIPCHK_(ce);
  BHIPCHK_(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
  b->graph_sweeps = sweeps_per_graph;
  b->graph_measure = measure;
  return DQMC_OK;
}

// Autotuner: for every group, `trials` sweeps are timed (HIP events) with
// each GEMM kernel (16 x 16 and 32 x 32 direct tiles, 64 x 64 LDS-staged) and
// the fastest is kept.  The
// trial sweeps advance the chains like warm-up sweeps; a captured graph is
// dropped (it would replay the old tiles).
dqmc_status dqmc_batch_set_side_by_side(dqmc_batch* b, int32_t enable) {
  if (!b || enable < 0 || enable > 1) return bfail(b, DQMC_E_ARG, "bad arguments");
  b->side_by_side = enable != 0;
  if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  return DQMC_OK;
}

dqmc_status dqmc_batch_set_chunk_kernel(dqmc_batch* b, int32_t enable) {
  if (!b || enable < -1 || enable > 1) return bfail(b, DQMC_E_ARG, "bad arguments");
  for (dqmc_ctx* c : b->groups) c->fused = enable;
  if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  return DQMC_OK;
}

dqmc_status dqmc_batch_autotune(dqmc_batch* b, int32_t trials) {
  if (!b || trials < 1) return bfail(b, DQMC_E_ARG, "bad arguments");
  for (dqmc_ctx* c : b->groups)
    if (!c->bound || !c->initialized || c->poisoned) return bfail(b, DQMC_E_STATE, "batch not initialised");
  if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  hipEvent_t e0, e1;
  BHIPCHK_(hipEventCreate(&e0));
  BHIPCHK_(hipEventCreate(&e1));
  const int cands[4] = {16, 32, 33, 64};
  for (dqmc_ctx* c : b->groups) {
    float best = 0.0f;
    int pick = 0;
    for (int t : cands) {
      c->gemm_tile = t;
      BHIPCHK_(hipEventRecord(e0, b->stream));
      for (int s = 0; s < trials; ++s)
        if (dqmc_status r = sweep_once(c, 0)) return bfail(b, r, c->err);
      BHIPCHK_(hipEventRecord(e1, b->stream));
      BHIPCHK_(hipEventSynchronize(e1));
      float ms = 0.0f;
      BHIPCHK_(hipEventElapsedTime(&ms, e0, e1));
      if (pick == 0 || ms < best) { best = ms; pick = t; }
    }
    c->gemm_tile = pick;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return batch_flags(b);
}

dqmc_status dqmc_batch_tuning(const dqmc_batch* b, int32_t chain, int32_t* gemm_tile) {
  if (!b || !gemm_tile || chain < 0 || chain >= (int)b->group_of.size()) return DQMC_E_ARG;
  *gemm_tile = b->groups[b->group_of[chain]]->gemm_tile;
  return DQMC_OK;
}

dqmc_status dqmc_batch_read_chain(dqmc_batch* b, int32_t chain, double* G_host, double* bins_host, dqmc_stats* st) {
  if (!b || chain < 0 || chain >= (int)b->group_of.size()) return bfail(b, DQMC_E_ARG, "bad arguments");
  if (!b->bound) return bfail(b, DQMC_E_STATE, "not bound");
  dqmc_ctx* c = b->groups[b->group_of[chain]];
  const int i = b->index_of[chain];
  const size_t co = (size_t)i * c->cs;
  if (G_host)
    BHIPCHK_(hipMemcpyAsync(G_host, c->G + co, sizeof(double) * c->N * c->N, hipMemcpyDeviceToHost, b->stream));
  if (bins_host)
    BHIPCHK_(hipMemcpyAsync(bins_host, c->bins + co, 4 * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  BHIPCHK_(hipStreamSynchronize(b->stream));
  if (st)
    if (dqmc_status r = chain_stats(c, i, st)) return bfail(b, r, c->err);
  return DQMC_OK;
}

dqmc_status dqmc_batch_eq_setup(dqmc_batch* b, int32_t chain, int32_t L1, int32_t L2, int32_t norb,
                                const int32_t* site, const double* sign) {
  if (!b || chain < 0 || chain >= (int)b->group_of.size()) return bfail(b, DQMC_E_ARG, "bad arguments");
  if (!b->bound) return bfail(b, DQMC_E_STATE, "not bound");
  dqmc_ctx* c = b->groups[b->group_of[chain]];
  if (dqmc_status s = dqmc_eq_setup(c, L1, L2, norb, site, sign)) return bfail(b, s, c->err);
  // a captured graph was recorded without (or with other) correlations
  if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  return DQMC_OK;
}

dqmc_status dqmc_batch_td_setup(dqmc_batch* b, int32_t chain, int32_t norb, const int32_t* orb_of,
                                const double* phase, int32_t n_cells) {
  if (!b || chain < 0 || chain >= (int)b->group_of.size()) return bfail(b, DQMC_E_ARG, "bad arguments");
  if (!b->bound) return bfail(b, DQMC_E_STATE, "not bound");
  dqmc_ctx* c = b->groups[b->group_of[chain]];
  if (dqmc_status s = dqmc_td_setup(c, norb, orb_of, phase, n_cells)) return bfail(b, s, c->err);
  if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  return DQMC_OK;
}

dqmc_status dqmc_batch_td_read_bins(dqmc_batch* b, int32_t chain, int32_t* norb, double* sums_host, double* count) {
  if (!b || chain < 0 || chain >= (int)b->group_of.size()) return bfail(b, DQMC_E_ARG, "bad arguments");
  if (!b->bound) return bfail(b, DQMC_E_STATE, "not bound");
  dqmc_ctx* c = b->groups[b->group_of[chain]];
  if (c->td_norb < 1) return bfail(b, DQMC_E_STATE, "time-displaced measurement not set up for this chain's group");
  if (norb) *norb = c->td_norb;
  if (!sums_host && !count) return DQMC_OK;
  std::vector<double> raw((size_t)(c->L + 1) * kTdStride + 1);
  BHIPCHK_(hipMemcpyAsync(raw.data(), c->tdbins + (size_t)b->index_of[chain] * c->cs, raw.size() * sizeof(double),
                          hipMemcpyDeviceToHost, b->stream));
  BHIPCHK_(hipStreamSynchronize(b->stream));
  if (sums_host) td_compact(c, raw.data(), sums_host);
  if (count) *count = raw.back();
  return DQMC_OK;
}

dqmc_status dqmc_batch_eq_read(dqmc_batch* b, int32_t chain, int32_t* shape, double* sums_host, double* sz_host,
                               double* count) {
  if (!b || chain < 0 || chain >= (int)b->group_of.size()) return bfail(b, DQMC_E_ARG, "bad arguments");
  if (!b->bound) return bfail(b, DQMC_E_STATE, "not bound");
  dqmc_ctx* c = b->groups[b->group_of[chain]];
  if (c->eq_norb < 1) return bfail(b, DQMC_E_STATE, "lattice-resolved correlations not set up for this chain's group");
  const size_t nb = (size_t)c->eq_L1 * c->eq_L2 * c->eq_norb * c->eq_norb;
  if (shape) { shape[0] = c->eq_L1 * c->eq_L2; shape[1] = c->eq_norb; }
  if (!sums_host && !sz_host && !count) return DQMC_OK;
  std::vector<double> raw(4 * nb + 1 + c->eq_norb);
  BHIPCHK_(hipMemcpyAsync(raw.data(), c->eq_bins + (size_t)b->index_of[chain] * c->cs, raw.size() * sizeof(double),
                          hipMemcpyDeviceToHost, b->stream));
  BHIPCHK_(hipStreamSynchronize(b->stream));
  if (sums_host) std::copy(raw.begin(), raw.begin() + 4 * nb, sums_host);
  if (count) *count = raw[4 * nb];
  if (sz_host) std::copy(raw.begin() + 4 * nb + 1, raw.end(), sz_host);
  return DQMC_OK;
}

dqmc_status dqmc_batch_grad_logdet(dqmc_batch* b) {
  if (!b) return DQMC_E_ARG;
  for (dqmc_ctx* c : b->groups)
    if (!c->bound || !c->initialized || c->poisoned) return bfail(b, DQMC_E_STATE, "batch not initialised");
  for (dqmc_ctx* c : b->groups)
    if (dqmc_status s = grad_pass(c)) return bfail(b, s, c->err);
  return batch_flags(b);
}

dqmc_status dqmc_batch_read_grad(dqmc_batch* b, int32_t chain, double* grad_host, double* prec) {
  if (!b || !grad_host || chain < 0 || chain >= (int)b->group_of.size()) return bfail(b, DQMC_E_ARG, "bad arguments");
  if (!b->bound) return bfail(b, DQMC_E_STATE, "not bound");
  dqmc_ctx* c = b->groups[b->group_of[chain]];
  const size_t co = (size_t)b->index_of[chain] * c->cs;
  BHIPCHK_(hipMemcpyAsync(grad_host, c->grad + co, (size_t)c->L * c->N * sizeof(double), hipMemcpyDeviceToHost,
                          b->stream));
  if (prec) BHIPCHK_(hipMemcpyAsync(prec, c->gprec + co, sizeof(double), hipMemcpyDeviceToHost, b->stream));
  BHIPCHK_(hipStreamSynchronize(b->stream));
  return DQMC_OK;
}

dqmc_status dqmc_batch_langevin(dqmc_batch* b, double eps, int32_t n_steps) {
  if (!b || n_steps < 0 || !(eps > 0.0) || !std::isfinite(eps)) return bfail(b, DQMC_E_ARG, "bad arguments");
  for (dqmc_ctx* c : b->groups) {
    if (!c->bound || !c->initialized || c->poisoned) return bfail(b, DQMC_E_STATE, "batch not initialised");
    if (c->m.field != DQMC_FIELD_GAUSS) return bfail(b, DQMC_E_UNSUPPORTED, "Langevin steps need a Gaussian field");
  }
  for (int k = 0; k < n_steps; ++k)
    for (dqmc_ctx* c : b->groups)
      if (dqmc_status s = langevin_once(c, eps)) return bfail(b, s, c->err);
  return batch_flags(b);
}

dqmc_status dqmc_batch_get_langevin_step(dqmc_batch* b, int32_t chain, uint64_t* step) {
  if (!b || !step || chain < 0 || chain >= (int)b->group_of.size()) return bfail(b, DQMC_E_ARG, "bad arguments");
  if (!b->bound) return bfail(b, DQMC_E_STATE, "not bound");
  dqmc_ctx* c = b->groups[b->group_of[chain]];
  unsigned long long v = 0;
  BHIPCHK_(hipMemcpyAsync(&v, reinterpret_cast<double*>(c->counters + 4) + (size_t)b->index_of[chain] * c->cs,
                          sizeof(v), hipMemcpyDeviceToHost, b->stream));
  BHIPCHK_(hipStreamSynchronize(b->stream));
  *step = v;
  return DQMC_OK;
}

dqmc_status dqmc_batch_set_langevin_step(dqmc_batch* b, int32_t chain, uint64_t step) {
  if (!b || chain < 0 || chain >= (int)b->group_of.size()) return bfail(b, DQMC_E_ARG, "bad arguments");
  if (!b->bound) return bfail(b, DQMC_E_STATE, "not bound");
  dqmc_ctx* c = b->groups[b->group_of[chain]];
  unsigned long long v = step;
  BHIPCHK_(hipMemcpyAsync(reinterpret_cast<double*>(c->counters + 4) + (size_t)b->index_of[chain] * c->cs, &v,
                          sizeof(v), hipMemcpyHostToDevice, b->stream));
  BHIPCHK_(hipStreamSynchronize(b->stream));
  return DQMC_OK;
}

int32_t dqmc_batch_groups(const dqmc_batch* b) { return b ? (int32_t)b->groups.size() : 0; }

// Host-only self-check of the buffer layout, placing the groups at a fake
// base address (nothing is dereferenced): DQMC_OK or DQMC_E_STATE.
dqmc_status dqmc_batch_check_layout(dqmc_batch* b) {
  if (!b) return DQMC_E_ARG;
  double* fake = reinterpret_cast<double*>(uintptr_t(1) << 40);
  for (size_t g = 0; g < b->groups.size(); ++g) {
    double* base = fake + b->group_off[g];
    place_group(b->groups[g], base);
    const double* hi = (g + 1 < b->groups.size()) ? fake + b->group_off[g + 1] : fake + b->total;
    if (!layout_ok(b->groups[g], base, hi)) return DQMC_E_STATE;
  }
  // a bound batch gets its real placement back
  if (b->work)
    for (size_t g = 0; g < b->groups.size(); ++g) place_group(b->groups[g], b->work + b->group_off[g]);
  return DQMC_OK;
}

const char* dqmc_batch_last_error(const dqmc_batch* b) { return b ? b->err.c_str() : "null batch"; }

void dqmc_batch_destroy(dqmc_batch* b) { delete b; }

}  // extern "C"

// ============================================== allocation-free variant ==
// dqmc_green_scratch_noalloc computes what dqmc_green_scratch computes, with
// every device buffer it needs besides its input (the field) and its output
// (G) in one static device array, so it runs without any device allocation
// by the caller or the library.  Each GPU holds its own copy of the array
// for the life of the process; host code reaches it only through the
// address hipGetSymbolAddress returns on that device.
namespace {

constexpr size_t kNoallocScratchDoubles = (size_t)4 << 20;   // 32 MiB
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
dqmc_status scratch_address(dqmc_ctx* c, double** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(c, DQMC_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(c, DQMC_E_DEVICE, "no device address for the static scratch array");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return DQMC_OK;
}

}  // namespace

extern "C" {

dqmc_status dqmc_green_scratch_noalloc(dqmc_ctx* c, const double* field_dev, int32_t tau, double* G_dev,
                                       void* hip_stream) {
  if (!c || !field_dev || !G_dev || tau < 0 || tau > c->L) return fail(c, DQMC_E_ARG, "bad arguments");
  if (c->nfl == 2 || c->nvx) return fail(c, DQMC_E_UNSUPPORTED, "not built for two flavours or general vertices");
  // a host-side context of its own: model and hopping from c, every device
  // pointer inside the static array (c's own binding, if any, is untouched)
  dqmc_ctx t;
  t.no_shadow = true;
  t.m = c->m;
  t.N = c->N; t.L = c->L; t.nw = c->nw; t.nk = c->nk; t.nb = c->nb;
  t.Nf = c->Nf; t.cplx = c->cplx; t.trK_field = c->trK_field;
  t.K = c->K;
  t.trK = c->trK; t.normK1 = c->normK1;
  const size_t need = layout_work(&t, false);
  if (need > kNoallocScratchDoubles)
    return fail(c, DQMC_E_UNSUPPORTED,
                "dqmc_green_scratch_noalloc: this model needs " + std::to_string(need * 8 >> 20) +
                    " MiB of scratch, above the static maximum of " +
                    std::to_string(kNoallocScratchDoubles * 8 >> 20) + " MiB");
  double* base = nullptr;
  if (dqmc_status s = scratch_address(c, &base)) return s;
  t.stream = static_cast<hipStream_t>(hip_stream);
  t.work = base;
  t.field = const_cast<double*>(field_dev);   // read only on this path
  layout_work(&t, true);
  auto run = [&]() -> dqmc_status {
    if (dqmc_status s = set_lds_limits(&t)) return s;
    // the array keeps the last call's contents: everything read below is
    // written first, and the error flag is cleared here
    if (dqmc_status s = fill_small(&t, reinterpret_cast<double*>(t.err_flag), 1, 0.0)) return s;
    HIPCHK(hipMemcpyAsync(t.Kd, t.K.data(), sizeof(double) * t.N * t.N, hipMemcpyHostToDevice, t.stream));
    if (dqmc_status s = expm(&t, -t.m.dtau, t.E)) return s;
    hipLaunchKernelGGL(k_set_identity, dim3(grid1((size_t)t.N * t.N)), dim3(256), 0, t.stream, t.uid.Q, t.N, t.N,
                       (size_t)0);
    hipLaunchKernelGGL(k_set_identity, dim3(grid1((size_t)t.N * t.N)), dim3(256), 0, t.stream, t.uid.T, t.N, t.N,
                       (size_t)0);
    HIPCHK(hipGetLastError());
    if (dqmc_status s = fill_small(&t, t.uid.D, t.N, 1.0)) return s;
    if (dqmc_status s = green_scratch_into(&t, tau, G_dev)) return s;
    int flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, t.err_flag, sizeof(int), hipMemcpyDeviceToHost, t.stream));
    HIPCHK(hipStreamSynchronize(t.stream));
    if (flag) return fail(&t, DQMC_E_NUMERIC, "numerical failure in the recomputation (flags " +
                                                  std::to_string(flag) + ")");
    return DQMC_OK;
  };
  const dqmc_status s = run();
  if (s != DQMC_OK && !t.err.empty()) c->err = t.err;
  return s;
}

}  // extern "C"
