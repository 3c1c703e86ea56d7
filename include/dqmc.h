/*
 * dqmc.h -- C ABI of the MI355X (gfx950) determinant quantum Monte Carlo sweep.
 *
 * The library runs the Monte Carlo sweep of the finite-temperature
 * auxiliary-field (BSS) method documented in ALF 1.0 (arXiv:1704.00131):
 * weight ratios from the equal-time Green's function, Sherman-Morrison updates
 * of G, wraps G -> B_tau G B_tau^-1, QR/UDV-stabilised recomputation of G every
 * n_wrap slices, and equal-time measurements.  All arithmetic is FP64 on the
 * GPU; the host side only checks arguments and enqueues kernels.
 *
 * Conventions shared by all calls
 * -------------------------------
 *  - Every function returns a dqmc_status and never throws.  On failure the
 *    text of the last error is available from dqmc_last_error().
 *  - Matrices are row-major FP64, n x n, leading dimension n.
 *  - The field is FP64 [n_slices][n]: field[(tau-1)*n + i] is the
 *    Hubbard-Stratonovich field of vertex i on slice tau (the paper's nsigma
 *    array, section "The SU(2)-Hubbard model on a square lattice").  An Ising
 *    field holds +1.0 / -1.0, a Gaussian field any real value.
 *  - Device buffers are allocated and owned by the caller (for example torch
 *    tensors); they must stay alive while they are bound.  The library never
 *    allocates or frees device memory of its own.  Host inputs are copied
 *    during the call that receives them.
 *  - All device work of a context is enqueued on the stream given to
 *    dqmc_bind(); calls that return host data synchronise that stream.
 */
#ifndef DQMC_H
#define DQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DQMC_OK = 0,
  DQMC_E_ARG = 1,          /* invalid argument, detected on the host before any launch      */
  DQMC_E_UNSUPPORTED = 2,  /* valid in the paper's general model but not built here          */
  DQMC_E_DEVICE = 3,       /* a HIP call failed                                              */
  DQMC_E_NUMERIC = 4,      /* NaN/Inf in G, vanishing QR scale, or precision above threshold */
  DQMC_E_NOMEM = 5,        /* host allocation failed                                         */
  DQMC_E_STATE = 6         /* call out of order (not bound / not initialised / poisoned)     */
} dqmc_status;

typedef enum {
  DQMC_FIELD_ISING = 0,
  DQMC_FIELD_GAUSS = 1,
  DQMC_FIELD_ISING4 = 2,
  DQMC_FIELD_ISING4_IMAG = 3
} dqmc_field_kind;
typedef enum { DQMC_TROTTER_ASYM = 0, DQMC_TROTTER_SYM = 1 } dqmc_trotter;

/*
 * Model of one Markov chain (section "Definition of the Hamiltonian",
 * Eqs. (general_ham_t) and (general_ham_v), with M_T = 1, N_fl = 1 and one
 * single-site vertex per orbital, V^(k) = e_k e_k^T).
 *
 * The slice propagator sampled is B_tau = exp(V_tau) exp(-dtau K) with
 * exp(V_tau) = diag(exp(coupling * field[tau])); its determinant product equals
 * that of Eq. (Green_eq) and of a symmetric split.  The configuration weight is
 * exp(n_col * coupling * alpha * sum(field)) det(1 + B(beta,0))^n_col
 * (Eq. (partition_2)), times exp(-sum(field^2)/2) for a Gaussian field.
 * Field kinds: DQMC_FIELD_ISING stores +-1 (the exact two-valued identity);
 * DQMC_FIELD_ISING4 stores eta(l), l = +-1, +-2, of the paper's four-valued
 * identity (Eq. (HS_squares)), and the weight gains prod gamma(l); a flip
 * proposes one of the three other values with probability 1/3 each;
 * DQMC_FIELD_GAUSS stores a real phi (continuous field, Gaussian weight).
 *
 * DQMC_FIELD_ISING4_IMAG is the complex formulation of the section "The
 * SU(2)-Hubbard model on a square lattice": the four-valued field at
 * lambda = -U/2 with the imaginary coupling i c (coupling holds c =
 * sqrt(dtau U / 2)), in the original frame, exp(V_tau) = diag(exp(i c eta)),
 * alpha = -1/2, n_col = 2, G complex.  The weight is complex; the chain
 * samples its modulus (a flip is accepted iff u < |R|) and carries the phase
 * W / |W| of Eq. (phase) (dqmc_read_phase).  Every complex n x n matrix is
 * held as its real 2n x 2n image [[Re X, -Im X], [Im X, Re X]]: G is that
 * image (4 n^2 doubles), the field stays n_slices*n doubles.  n <= 64, single
 * chains; the sweep with measure bit 0 and dqmc_green_scratch are built, every
 * other entry point returns DQMC_E_UNSUPPORTED.  The equal-time estimators
 * are the real parts of D = (1/n) sum_i (1 - G~_ii)^2,
 * E_kin = (n_col / n)(Tr T - Tr(T G)) and E_pot = U D.
 */
typedef struct {
  int32_t n;               /* N_dim, number of orbitals, 1 <= n <= 1024                       */
  int32_t n_slices;        /* L_Trotter; |beta - n_slices*dtau| <= 1e-12*beta                  */
  double beta, dtau;
  int32_t n_wrap;          /* slices between stabilisations; n_slices % n_wrap == 0            */
  int32_t n_col;           /* N_col (N_SUN): weight carries det(...)^n_col, 1 or 2             */
  dqmc_field_kind field;
  double coupling;         /* lambda (Ising) or c (Gaussian)                                  */
  double alpha;            /* the constant of (V + alpha) in Eq. (general_ham_v)              */
  double u_int;            /* U, used only by the potential-energy estimator E_pot = U D     */
  dqmc_trotter trotter;    /* SYM: measure exp(-dtau K/2) G exp(+dtau K/2)                    */
  double prec_threshold;   /* max |G_wrapped - G_scratch| tolerated; <= 0: never trip         */
  double prop_width;       /* Gaussian local move phi' = phi + prop_width*(2u-1)              */
  uint64_t seed;           /* Philox key of the chain                                         */
} dqmc_model;

typedef struct { size_t G, field, slots, work; } dqmc_sizes;     /* bytes of each device buffer */
typedef struct { void *G, *field, *slots, *work; } dqmc_buffers; /* caller-owned device memory  */

typedef struct {
  uint64_t proposals, accepted;  /* cumulative since dqmc_init                               */
  double prec_mean, prec_max;    /* wrapped vs recomputed G over all stabilisations so far   */
  uint64_t n_prec;               /* number of stabilisations counted                         */
  double seconds;                /* host wall time of the last dqmc_sweep call               */
} dqmc_stats;

typedef struct dqmc_ctx dqmc_ctx;

/* Byte sizes of the device buffers for a model.  G: n*n doubles (the 2n x 2n
 * image, 4 n^2 doubles, for DQMC_FIELD_ISING4_IMAG); field:
 * n_slices*n doubles; slots: the UDV storage of Algorithm 1,
 * (n_slices/n_wrap + 1) * (2 n^2 + n) doubles; work: scratch.  DQMC_E_ARG on
 * an inconsistent model. */
dqmc_status dqmc_query_sizes(const dqmc_model* model, dqmc_sizes* out);

/* Create a context.  K: n*n host hopping matrix (Eq. (general_ham_t), the
 * paper's T), must be symmetric (DQMC_E_ARG otherwise) and is copied.
 * vertex_site: NULL or the identity map 0..n-1 (one vertex per orbital);
 * anything else is DQMC_E_UNSUPPORTED.  No device work happens here. */
dqmc_status dqmc_create(const dqmc_model* model, const double* K, const int32_t* vertex_site,
                        dqmc_ctx** out);

/* The M_z form with two flavours and two Green's functions (section "The
 * M_z-Hubbard model on a square lattice", Eq. (hubbard_Mz)): per site one
 * vertex coupled to n_up - n_dn, the field acting with +coupling on the up
 * flavour and -coupling on the down flavour, each flavour with its own
 * hopping matrix (K_up, K_dn: n*n host arrays, symmetric, copied), so a
 * Zeeman field, a chemical potential or spin-dependent hopping.  The weight
 * prod(vertex factors) det(1 + B_up(beta,0)) det(1 + B_dn(beta,0)) is real
 * but may be negative (the sign problem): the chain samples its modulus
 * (a flip is accepted iff u < |R|, R = vertex factor ratio x r_up x r_dn) and
 * carries the sign relative to the starting configuration (dqmc_read_phase:
 * out3_host[0] = the sign, [1] = 0, [2] = 2 once a negative sign was seen,
 * else 0).  The bins hold sign-weighted sums with the sum of the signs in
 * place of the count, of D = <n_up n_dn>, E_kin = (1/n) sum_f (Tr K_f -
 * Tr(K_f G_f)) and E_pot = (U/2)(1/n) sum_i <(n_i - 1)^2> per site (the
 * original frame).  The flavours are held as one 2n x 2n block-diagonal
 * system: G is that image (4 n^2 doubles, G_up in the upper-left block, G_dn
 * in the lower-right), the field stays n_slices*n doubles; take the buffer
 * sizes from dqmc_ctx_sizes.  model: alpha = 0 and n_col = 1 (DQMC_E_ARG
 * otherwise), field kinds Ising (the exact identity, coupling lambda with
 * cosh(lambda) = exp(dtau U / 2)), four-valued or Gaussian; n <= 64
 * (DQMC_E_UNSUPPORTED otherwise).  Single chains; the sweep with measure
 * bit 0 and dqmc_green_scratch are built, every other entry point returns
 * DQMC_E_UNSUPPORTED. */
dqmc_status dqmc_create_mz(const dqmc_model* model, const double* K_up, const double* K_dn, dqmc_ctx** out);

/* One operator vertex (section "Definition of the Hamiltonian", table
 * "operator"): X = P^T O P on n_orb = |P| orbitals orb[0..n_orb-1] (1 or 2,
 * distinct), O a real symmetric n_orb x n_orb matrix (row-major in O[0..3];
 * for n_orb = 1 only O[0] is read), so exp(g s X) = P^T exp(g s O) P +
 * (1 - P^T P).  ising = 0: a two-valued HS field of Eq. (general_ham_v),
 * s = +-1, weight factor exp(n_col g alpha s); ising = 1: an Ising spin
 * Z_k of Eq. (general_ham_i), whose own dynamics enters through S0. */
typedef struct {
  int32_t n_orb;
  int32_t orb[2];
  int32_t ising;
  double g;
  double alpha;
  double O[4];
} dqmc_vertex;

/* General operator vertices and Ising spins with their own action
 * (Eqs. (general_ham_v), (general_ham_i) and (partition_2), section
 * "Sampling of e^{-S_{0,I}}").  The slice propagator sampled is
 * B_tau = E_0 E_1 ... E_{M-1} exp(-dtau K), E_k = exp(g_k s_{k,tau} X_k), the
 * weight exp(-S0) exp(n_col sum g_k alpha_k s_{k,tau}) det(1 + B(beta,0))^n_col
 * with, for the Ising spins (transverse field h > 0 and coupling J between
 * the listed pairs), exp(-S0) = prod exp(Kt s_{k,tau} s_{k,tau+1})
 * prod_pairs exp(dtau J s_{k,tau} s_{k',tau}), Kt = -ln(tanh(dtau h)) / 2,
 * periodic in tau.  The flips of a slice take its vertices in a fixed order:
 * upward M-1 down to 0, downward 0 up to M-1, each in the frame where E_k is
 * the leftmost factor of the slice (G <- E_k G E_k^-1 before it in the
 * upward pass, G <- E_k^-1 G E_k after it in the downward pass); a flip
 * s -> -s with delta = exp(-2 g s O) - 1 has the ratio
 * det(1 + delta (1 - G)_PP)^n_col exp(-2 n_col g alpha s) times the ratio of
 * exp(-S0), is accepted iff u < R, and updates G <- G - G[:,P] (1 + delta
 * (1 - G)_PP)^-1 delta (1 - G)[P,:].  K: n*n host array, symmetric, copied.
 * vertices: n_vertices (= M) host records, copied; pairs: n_pairs pairs of
 * Ising vertex indices (2 n_pairs int32).  The field is [n_slices][M],
 * +-1 per vertex; G is n x n.  model: field kind Ising (DQMC_E_ARG
 * otherwise); coupling and alpha are ignored (per vertex here), u_int enters
 * the estimator E_pot = u_int D only.  n <= 64, M <= 512, n_orb 1 or 2 and
 * n_pairs <= 1024 (DQMC_E_UNSUPPORTED otherwise); an O that is not symmetric, an orbital out
 * of range, a pair that is not two distinct Ising vertices, or h <= 0 with
 * an Ising vertex is DQMC_E_ARG.  Single chains; take the buffer sizes from
 * dqmc_ctx_sizes.  The sweep with measure bit 0 (the estimators of the
 * one-flavour sweep on G(tau)), dqmc_green_scratch and dqmc_logdet are
 * built; dqmc_ratio, the gradient, Langevin, the correlation set-ups and
 * the allocation-free recomputation return DQMC_E_UNSUPPORTED. */
dqmc_status dqmc_create_vertices(const dqmc_model* model, const double* K, int32_t n_vertices,
                                 const dqmc_vertex* vertices, double h, double J, int32_t n_pairs,
                                 const int32_t* pairs, dqmc_ctx** out);

/* Byte sizes of the device buffers of a created context (those of
 * dqmc_query_sizes for the model; the two-flavour and vertex contexts need
 * these). */
dqmc_status dqmc_ctx_sizes(const dqmc_ctx* ctx, dqmc_sizes* out);

/* Bind caller-owned device buffers (sizes from dqmc_query_sizes, 256-byte
 * aligned) and the hipStream_t on which all later work is enqueued (NULL = the
 * null stream).  Computes exp(+-dtau K) and exp(+-dtau K/2) on the device. */
dqmc_status dqmc_bind(dqmc_ctx* ctx, const dqmc_buffers* buf, void* hip_stream);

/* Field configuration in and out (the paper's confin / confout): field_host is
 * n_slices*n doubles; sweep_counter is the chain's position in its random
 * stream.  Setting the state invalidates G until dqmc_init. */
dqmc_status dqmc_set_state(dqmc_ctx* ctx, const double* field_host, uint64_t sweep_counter);
dqmc_status dqmc_get_state(dqmc_ctx* ctx, double* field_host, uint64_t* sweep_counter);

/* Random start of the field from the chain's seed (s = +1 iff u < 1/2, or
 * phi ~ N(0,1)), sweep counter 0. */
dqmc_status dqmc_random_field(dqmc_ctx* ctx);

/* Algorithm 1 set-up: fill the storage with the left UDV forms of
 * B(beta, tau_k) and compute G(0) from scratch (section "Stabilization").
 * Clears the statistics, bins and the error flag. */
dqmc_status dqmc_init(dqmc_ctx* ctx);

/* n_sweeps sweeps (upward then downward pass, every field visited twice,
 * Algorithm 1).  measure: bit 0 accumulates the equal-time estimators on
 * every slice of both passes; bit 1 runs the time-displaced pass
 * (dqmc_td_measure, needs dqmc_td_setup) at the start of every sweep, as the
 * paper does for its time-displaced observables; bit 2 accumulates the
 * lattice-resolved equal-time correlations (needs dqmc_eq_setup) on every
 * slice of both passes; bit 3 adds the lattice-resolved time-displaced
 * correlations to the pass of bit 1 (needs bit 1, dqmc_eq_setup and a single
 * chain, else DQMC_E_STATE).  Other bits: DQMC_E_ARG.  stats may be NULL.
 * DQMC_E_NUMERIC if the device flagged a numerical failure; the context then
 * needs dqmc_init. */
dqmc_status dqmc_sweep(dqmc_ctx* ctx, int32_t n_sweeps, int32_t measure, dqmc_stats* stats);

/* Bin sums: sums_host[0..3] = sum of D, sum of E_kin, sum of E_pot (per site)
 * and the number of measurements.  dqmc_reset_bins zeroes them. */
dqmc_status dqmc_read_bins(dqmc_ctx* ctx, double* sums_host);
/* The configuration's phase W / |W| (Eq. (phase)) carried along by the
 * sweeps of a complex field: out3_host[0..1] = its real and imaginary parts,
 * out3_host[2] = the largest |phase - 1| since dqmc_init (the "precision" of
 * the phase: the weight of a half-filled bipartite lattice is real and
 * positive, so the phase stays 1 up to rounding).  Reset to 1 by dqmc_init.
 * DQMC_E_UNSUPPORTED for a real field. */
dqmc_status dqmc_read_phase(dqmc_ctx* ctx, double* out3_host);
dqmc_status dqmc_reset_bins(dqmc_ctx* ctx);

/* Test hook: G(tau) = (1 + B(tau,0) B(beta,tau))^-1 recomputed from scratch
 * for the current field into the device buffer G_dev (n*n doubles), using the
 * same stabilised products as the sweep.  Does not change the chain. */
dqmc_status dqmc_green_scratch(dqmc_ctx* ctx, int32_t tau, double* G_dev);

/* The same recomputation for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): every device buffer it needs besides its input and its output
 * lives in one static device array of at most 32 MiB that each GPU holds for
 * the life of the process; nothing is allocated or freed.  ctx: a created
 * context (bound or not; its model and hopping matrix are used, its own
 * buffers are not touched).  field_dev: device field of the chain, n_slices*n
 * doubles (read only).  G_dev: device output, n*n doubles.  The work is
 * enqueued on hip_stream, which is synchronised before return.
 * DQMC_E_UNSUPPORTED if the model's scratch exceeds 32 MiB (the 12x12
 * honeycomb chain, N = 288 and L = 100, needs 28.5 MB).  Every call on one GPU
 * uses that GPU's single array, so calls that overlap in time on the same GPU
 * (any contexts, any streams) race and must be serialised by the caller. */
dqmc_status dqmc_green_scratch_noalloc(dqmc_ctx* ctx, const double* field_dev, int32_t tau, double* G_dev,
                                       void* hip_stream);

/* Test hook: the weight ratio R of changing the field of `site` on slice tau
 * (1..L) to s_new, with everything else fixed (section "Updating schemes";
 * Eq. (Green_eq) and the matrix determinant lemma): with Delta =
 * exp(coupling (s_new - s)) - 1 and G(tau) recomputed from scratch,
 *   r = 1 + Delta (1 - G(tau)_ii),
 *   R = exp(n_col coupling alpha (s_new - s)) r^n_col  (x exp(-(s_new^2 - s^2)/2) Gaussian).
 * R: one host double.  Single chains; s_new must be +-1 for an Ising field. */
dqmc_status dqmc_ratio(dqmc_ctx* ctx, int32_t tau, int32_t site, double s_new, double* R);

/* log|det(1 + B(beta,0))| of the current field from scratch. */
dqmc_status dqmc_logdet(dqmc_ctx* ctx, double* logdet);

/* Gradient of log|det(1 + B(beta,0))| (one colour) with respect to the field,
 * read as a continuous variable:
 *   grad[tau-1][i] = d log det / d phi_{i,tau} = coupling (1 - G(tau)_ii),
 * which follows from Eq. (Green_eq) with B_tau of Eq. (partition_2) and the
 * cyclic trace (the paper's code has no continuous fields: a reading).  G(tau)
 * comes from an upward pass without updates that wraps G(0) slice by slice and
 * recomputes it every n_wrap slices from the stored left forms (the
 * checkpoints) and a running right form; no product of all L slices is kept.
 * grad_dev: device buffer of L*n doubles, row-major [L][n], owned by the
 * caller.  prec (host, may be NULL): max |wrapped - recomputed| over the
 * pass.  Needs an initialised chain (after dqmc_init or a sweep); the chain's
 * G, field and stored forms are unchanged. */
dqmc_status dqmc_grad_logdet(dqmc_ctx* ctx, double* grad_dev, double* prec);

/* n_steps unadjusted Langevin steps of a Gaussian field:
 *   phi <- phi + eps (-phi + n_col coupling alpha + n_col grad) + sqrt(2 eps) xi,
 * xi standard normal (Box-Muller, cosine branch) from Philox counter
 * (tag 3, step, tau << 1, site), grad as in dqmc_grad_logdet.  step is the
 * chain's Langevin step counter, kept on the device: it starts at 0
 * (dqmc_random_field, dqmc_bind) and advances by one per step, so successive
 * calls never reuse noise.  After each step the stored forms and G(0) are
 * rebuilt from the new field.  DQMC_E_UNSUPPORTED for an Ising field; eps
 * must be positive and finite. */
dqmc_status dqmc_langevin(dqmc_ctx* ctx, double eps, int32_t n_steps);
/* The Langevin step counter, read and set (part of the chain's state beside
 * the field and the sweep counter, for resuming a run). */
dqmc_status dqmc_get_langevin_step(dqmc_ctx* ctx, uint64_t* step);
dqmc_status dqmc_set_langevin_step(dqmc_ctx* ctx, uint64_t step);

/* ---- time-displaced Green's functions (section "Measuring time displaced
 * observables"; Eq. (s_corr)) ----
 * GT0(tau) = B(tau,0) G(0), G0T(tau) = -(1 - G(0)) B(tau,0)^-1 and
 * GTT(tau) = G(tau) for tau = 0..L, propagated slice by slice from the state at
 * the start of a sweep and re-anchored every n_wrap slices from the stabilised
 * forms through the bounded matrix of the equal-time merge (the paper does not
 * give the stable formulas: a reading).  Measured on them, per tau,
 *   S_ab(K, tau) = (1/n_cells) sum_{x in a, y in b} p_x conj(p_y) <S^z_x(tau) S^z_y(0)>,
 *   4 <S^z_x(tau) S^z_y(0)> = (1 - 2 GTT_xx)(1 - 2 G00_yy) - 2 G0T_yx GT0_xy,
 * with the symmetric split's rotation applied as for the equal-time G.
 *
 * dqmc_td_setup: norb orbitals per cell (1..4); orb_of[n] the orbital of each
 * site; phase[2n] = (cos, sin) of -K.R_cell(x) for each site x; n_cells the
 * number of unit cells.  Host arrays, copied.  Zeroes the time-displaced bins. */
dqmc_status dqmc_td_setup(dqmc_ctx* ctx, int32_t norb, const int32_t* orb_of, const double* phase, int32_t n_cells);
/* One time-displaced pass of the current configuration (an initialised chain
 * at the start of a sweep); adds S to the bins.  S_host (may be NULL):
 * (L+1)*norb*norb*2 doubles [tau][a][b][re, im].  prec (may be NULL): 2 host
 * doubles, the largest |propagated - re-anchored| of GTT and of GT0 / G0T.
 * The chain's G, field and stored forms are unchanged. */
dqmc_status dqmc_td_measure(dqmc_ctx* ctx, double* S_host, double* prec);
/* Bin sums of S in the layout of dqmc_td_measure and the number of passes
 * summed (count, may be NULL).  Zeroed by dqmc_init and dqmc_reset_bins. */
dqmc_status dqmc_td_read_bins(dqmc_ctx* ctx, double* sums_host, double* count);

/* ---- lattice-resolved equal-time correlations (section "Observables":
 * correlation functions summed over unit cells and stored by the displacement
 * R between cells) ----
 * Per measurement, from the measured G~ (G, or e^{-dtau K/2} G e^{+dtau K/2}
 * for the symmetric split), both particle-hole species sharing G and s_i the
 * sublattice sign of the down-spin map,
 *   C_o[R][a][b] += 1/n_cells sum_I O(site(I, a), site(I + R, b)),
 *   Green  = 1/2 (d_ij - G_ji + s_i s_j G_ij)
 *   SpinZ  = 1/4 ((1 - 2 G_ii)(1 - 2 G_jj) + 2 (d_ij - G_ji) G_ij)
 *   SpinXY = 1/4 s_i s_j ((d_ij - G_ji)^2 + G_ij^2)
 *   Den    = 1 + 2 (d_ij - G_ji) G_ij,
 * cells I = i1 + L1 i2 and R = r1 + L1 r2, I + R taken modulo (L1, L2).
 *
 * dqmc_eq_setup: an L1 x L2 lattice of norb orbitals per cell (1..4,
 * L1 L2 norb = n, else DQMC_E_ARG); site[I * norb + a] the orbital index of
 * orbital a of cell I (a permutation of 0..n-1, else DQMC_E_ARG); sign[n] the
 * sublattice signs, each +1 or -1 (else DQMC_E_ARG).  Host arrays, copied.
 * Zeroes these bins. */
dqmc_status dqmc_eq_setup(dqmc_ctx* ctx, int32_t L1, int32_t L2, int32_t norb, const int32_t* site, const double* sign);
/* Bin sums [o][R][a][b] (4 * n_cells * norb * norb host doubles, o = Green,
 * SpinZ, SpinXY, Den) and the number of measurements summed (count, may be
 * NULL).  Zeroed by dqmc_init, dqmc_reset_bins and dqmc_eq_setup. */
dqmc_status dqmc_eq_read_bins(dqmc_ctx* ctx, double* sums_host, double* count);
/* Bin sums of the one-point function <S^z> per orbital of the cell, summed
 * with the correlations of bit 2: 1/n_cells sum_I 1/2 (1 - 2 G~_ii) for
 * i = site(I, a) (n_up = n_1, n_dn = 1 - n_2 in the frame), norb host doubles,
 * and the number of measurements (count, may be NULL).  Zeroed with the
 * correlation bins. */
dqmc_status dqmc_eq_read_spin_z(dqmc_ctx* ctx, double* sz_host, double* count);
/* The same four correlators between tau and 0, from the time-displaced pass
 * (section "Measuring time displaced observables"), per configuration
 *   C_o[tau][R][a][b] += 1/n_cells sum_I <O_i(tau) O_j(0)>,  i = site(I, a), j = site(I + R, b),
 * with h = G0T_ji, g = GT0_ij:
 *   Green  = 1/2 (-h + s_i s_j g)
 *   SpinZ  = 1/4 ((1 - 2 GTT_ii)(1 - 2 G00_jj) - 2 h g)
 *   SpinXY = 1/4 s_i s_j (h^2 + g^2)
 *   Den    = 1 - 2 h g
 * (the equal-time ones at tau = 0).  Accumulated by sweeps with bits 1 and 3.
 * Bin sums [tau][o][R][a][b] ((L+1) * 4 * n_cells * norb * norb host doubles)
 * and the number of passes summed (count, may be NULL).  Zeroed by dqmc_init,
 * dqmc_reset_bins and dqmc_eq_setup.  DQMC_E_STATE without dqmc_eq_setup. */
dqmc_status dqmc_td_read_corr_bins(dqmc_ctx* ctx, double* sums_host, double* count);

/* Per-launch timing of one kernel of the sweep, for roofline reports: while
 * enabled, launches of the selected kernel on the context's stream are
 * bracketed by two HIP events: every launch for enable = 1, every enable-th
 * launch for enable > 1 (a sample that keeps the event markers from slowing
 * the timed work; a period coprime with the launches per slice visits every
 * launch position).  0 disables; negative values are DQMC_E_ARG.
 * dqmc_timing_read synchronises the stream, returns the summed event time (ms)
 * and the number of bracketed launches since the last read (and, for the GEMM,
 * their FLOPs), and clears them.  kernel: DQMC_KERNEL_BLOCK_UPDATE (the fused
 * block update), DQMC_KERNEL_GEMM (the MFMA product) or DQMC_KERNEL_STABILISE
 * (a whole stabilisation step of a sweep: the chunk products, the QR, the
 * merge with its LU solve and the precision check, section "Stabilization";
 * the events bracket the step's launch sequence). */
typedef enum { DQMC_KERNEL_BLOCK_UPDATE = 0, DQMC_KERNEL_GEMM = 1, DQMC_KERNEL_STABILISE = 2 } dqmc_kernel;

/* Kernel choice for the slices between stabilisations (Algorithm 1: the
 * wraps, the sequential single flips and the equal-time estimators).  With
 * enable = 1 a lattice of n <= 64 orbitals runs each chunk of n_wrap slices in
 * one launch per chain, one workgroup per chain with G and the exponentials
 * resident in LDS; 0 selects the blocked kernels (wrap products, 32-site
 * block updates, one measurement launch per slice), which larger lattices
 * always use, as do sweeps with the lattice-resolved equal-time correlations
 * and sweeps whose block update is being timed; -1 (the default) takes the
 * chunk kernel for batch groups of at least 16 chains and the blocked
 * kernels otherwise (a lone chain on one workgroup leaves the chip idle).
 * Both follow the same decisions and random numbers; G agrees up to
 * rounding.  DQMC_E_ARG for other values. */
dqmc_status dqmc_set_chunk_kernel(dqmc_ctx* ctx, int32_t enable);
dqmc_status dqmc_timing_enable(dqmc_ctx* ctx, dqmc_kernel kernel, int32_t enable);
dqmc_status dqmc_timing_read(dqmc_ctx* ctx, double* total_ms, uint64_t* launches, double* flops);

const char* dqmc_last_error(const dqmc_ctx* ctx);
void dqmc_destroy(dqmc_ctx* ctx);

/* ------------------------------------------------------------- batches ----
 * Many independent Markov chains, the paper's one-walker-per-MPI-task
 * parallelism (section "Performance, memory requirements and
 * parallelization") moved onto one GPU.  Chains whose models agree in all but
 * the seed form a group; every kernel of a group's sweep covers all of its
 * chains in one launch (one chain per grid row), so a sweep of the whole batch
 * is one launch sequence per group, which dqmc_batch_capture records once
 * into a hipGraph.  Each chain follows exactly the arithmetic and random
 * numbers of a single-chain context with the same model. */
typedef struct dqmc_batch dqmc_batch;

/* models[i] and K[i] (n_i x n_i host, symmetric) describe chain i; copied. */
dqmc_status dqmc_batch_create(int32_t n_chains, const dqmc_model* models, const double* const* K,
                              dqmc_batch** out);
/* Bytes of the single caller-owned device buffer that holds every chain. */
dqmc_status dqmc_batch_query_size(const dqmc_batch* b, size_t* work_bytes);
/* Bind that buffer (256-byte aligned) and the stream; computes the
 * exponentials once per group.  With more than one group it also creates one
 * stream per group (default priority, owned by the batch and destroyed with
 * it): sweeps and captures run each group on its own stream, forked from the
 * bound stream and joined back into it, so every call still completes in the
 * bound stream's order. */
dqmc_status dqmc_batch_bind(dqmc_batch* b, void* work, void* hip_stream);
dqmc_status dqmc_batch_random_fields(dqmc_batch* b);
dqmc_status dqmc_batch_set_state(dqmc_batch* b, int32_t chain, const double* field_host, uint64_t sweep_counter);
dqmc_status dqmc_batch_get_state(dqmc_batch* b, int32_t chain, double* field_host, uint64_t* sweep_counter);
/* Storage fill and G(0) of every chain. */
dqmc_status dqmc_batch_init(dqmc_batch* b);
/* dqmc_set_chunk_kernel for every group of the batch; drops a captured graph. */
dqmc_status dqmc_batch_set_chunk_kernel(dqmc_batch* b, int32_t enable);
/* With more than one group: 1 (the default) sweeps the groups side by side,
 * each on its own stream; 0 one after the other on the bound stream.  The
 * groups share no memory, so the results are bit-identical either way.  Drops
 * a captured graph.  DQMC_E_ARG for other values. */
dqmc_status dqmc_batch_set_side_by_side(dqmc_batch* b, int32_t enable);
/* Autotuner: per group, times `trials` sweeps with each GEMM kernel (16 x 16
 * and 32 x 32 direct MFMA tiles, 32 x 32 and 64 x 64 LDS-staged tiles) and
 * keeps the fastest (the trial sweeps advance the chains like warm-up sweeps;
 * a captured graph is dropped). */
dqmc_status dqmc_batch_autotune(dqmc_batch* b, int32_t trials);
/* The GEMM kernel chosen for a chain's group: 16 or 32 (direct tiles), 33
 * (32 x 32 LDS-staged), 64 (64 x 64 LDS-staged), 0 = size-based default. */
dqmc_status dqmc_batch_tuning(const dqmc_batch* b, int32_t chain, int32_t* gemm_tile);
/* Record `sweeps_per_graph` sweeps of the whole batch into a hipGraph; later
 * dqmc_batch_sweep calls with the same measure flags replay it.  measure:
 * bit 0 the equal-time estimators, bit 1 the time-displaced pass at the start
 * of each sweep for the groups set up with dqmc_batch_td_setup, bit 2 the
 * lattice-resolved equal-time correlations of the groups set up with
 * dqmc_batch_eq_setup (groups without a set-up skip that part); other bits
 * DQMC_E_ARG. */
dqmc_status dqmc_batch_capture(dqmc_batch* b, int32_t sweeps_per_graph, int32_t measure);
/* n_sweeps sweeps of every chain (measure as for dqmc_batch_capture); stats
 * summed over chains. */
dqmc_status dqmc_batch_sweep(dqmc_batch* b, int32_t n_sweeps, int32_t measure, dqmc_stats* total);
/* G (n*n host doubles), bin sums (4 host doubles) and statistics of one chain. */
dqmc_status dqmc_batch_read_chain(dqmc_batch* b, int32_t chain, double* G_host, double* bins_host,
                                  dqmc_stats* stats);
/* Time-displaced measurement (as dqmc_td_setup) for every chain of `chain`'s
 * group; zeroes their time-displaced bins and drops a captured graph. */
dqmc_status dqmc_batch_td_setup(dqmc_batch* b, int32_t chain, int32_t norb, const int32_t* orb_of,
                                const double* phase, int32_t n_cells);
/* One chain's time-displaced bins: norb (may be NULL) receives the group's
 * orbitals per cell; sums_host (may be NULL) the sums in the layout of
 * dqmc_td_read_bins ((L+1)*norb*norb*2 host doubles); count (may be NULL) the
 * passes summed.  DQMC_E_STATE if the chain's group is not set up. */
dqmc_status dqmc_batch_td_read_bins(dqmc_batch* b, int32_t chain, int32_t* norb, double* sums_host, double* count);
/* Lattice-resolved equal-time correlations (as dqmc_eq_setup) for every chain
 * of `chain`'s group (chains with the same model but the seed share the
 * lattice); zeroes their correlation bins and drops a captured graph.  Each
 * chain keeps its own bins. */
dqmc_status dqmc_batch_eq_setup(dqmc_batch* b, int32_t chain, int32_t L1, int32_t L2, int32_t norb,
                                const int32_t* site, const double* sign);
/* One chain's correlation bins: shape[2] (may be NULL) receives n_cells and
 * norb; sums_host (may be NULL) the 4 * n_cells * norb * norb sums of
 * dqmc_eq_read_bins; sz_host (may be NULL) the norb sums of
 * dqmc_eq_read_spin_z; count (may be NULL) the measurements summed.
 * DQMC_E_STATE if the chain's group is not set up. */
dqmc_status dqmc_batch_eq_read(dqmc_batch* b, int32_t chain, int32_t* shape, double* sums_host, double* sz_host,
                               double* count);
/* Gradient pass (as dqmc_grad_logdet) of every chain, kept on the device. */
dqmc_status dqmc_batch_grad_logdet(dqmc_batch* b);
/* The last gradient of one chain: L*n host doubles [L][n]; prec may be NULL. */
dqmc_status dqmc_batch_read_grad(dqmc_batch* b, int32_t chain, double* grad_host, double* prec);
/* n_steps Langevin steps (as dqmc_langevin) of every chain, each with its own
 * step counter; Gaussian fields only. */
dqmc_status dqmc_batch_langevin(dqmc_batch* b, double eps, int32_t n_steps);
dqmc_status dqmc_batch_get_langevin_step(dqmc_batch* b, int32_t chain, uint64_t* step);
dqmc_status dqmc_batch_set_langevin_step(dqmc_batch* b, int32_t chain, uint64_t step);
int32_t dqmc_batch_groups(const dqmc_batch* b);
/* Host-only self-check of the batch buffer layout (no device access). */
dqmc_status dqmc_batch_check_layout(dqmc_batch* b);
const char* dqmc_batch_last_error(const dqmc_batch* b);
void dqmc_batch_destroy(dqmc_batch* b);

/* Coupling of the exact two-valued Hubbard-Stratonovich identity,
 * cosh(lambda) = exp(dtau U / 2) (DQMC_FIELD_ISING), of the Gaussian
 * identity, c = sqrt(dtau U) (DQMC_FIELD_GAUSS), or of the four-valued
 * identity of Eq. (HS_squares), sqrt(dtau U / 2) (DQMC_FIELD_ISING4, and c of the
 * imaginary coupling i c for DQMC_FIELD_ISING4_IMAG). */
dqmc_status dqmc_hubbard_coupling(double U, double dtau, dqmc_field_kind kind, double* coupling);

/* Hopping matrix of the density frame for the M_z form of the Hubbard model
 * (section "The M_z-Hubbard model on a square lattice": two flavours coupled
 * to n_up - n_dn) with a Zeeman field h, i.e. flavour hopping T_up = T - h and
 * T_dn = T + h.  Under c_{i,dn} = s_i c'^+_i the flavours' matrices become
 * K_1 = T - h 1 and K_2 = -S (T + h 1)^T S, S = diag(sign); when they are equal
 * (T symmetric with zero diagonal, bonds only between opposite signs) the
 * frame's single Green's function serves both and K_out = T - h 1.  T (n*n,
 * row-major), sign (n, each +1 or -1) and K_out (n*n) are host arrays owned by
 * the caller.  DQMC_E_ARG for bad arguments, DQMC_E_UNSUPPORTED when the two
 * flavours differ (a chemical potential, a non-bipartite bond, flavour-
 * dependent hopping beyond the field): those need two Green's functions. */
dqmc_status dqmc_mz_frame_hopping(int32_t n, const double* T, double h, const double* sign, double* K_out);

#ifdef __cplusplus
}
#endif
#endif /* DQMC_H */
