"""Model setup of the oracle: HS constants, exponentials and slice propagators.

Frame (a reading; the paper is inconsistent about the sign of the SU(2)
coupling in its square-lattice example): the repulsive half-filled Hubbard
model is simulated through its image under the partial particle-hole map
c_{i,dn} -> (-1)^i c_{i,dn}^+, exact at mu = 0 on bipartite lattices.  That
image is the paper's SU(2) form with U_k = -U/2, V = one site, alpha = -1/2,
N_col = 2, N_fl = 1, whose density-coupled HS field is real, so the whole
method runs in real FP64.

HS transformation (replaces the paper's four-valued approximate identity of
the section "Formulation of the method" by the exact two-valued one, since
(n - 1)^2 only takes the values 0 and 1):

    exp(dtau U/2 (n-1)^2) = 1/2 sum_{s=+-1} exp(lambda s (n-1)),  cosh(lambda) = exp(dtau U/2)

Four-valued field (the paper's approximate identity for perfect squares,
Eq. (HS_squares), with lambda = U/2 and A = n - 1):
    exp(dtau U/2 A^2) ~ 1/4 sum_{l=+-1,+-2} gamma(l) exp(c4 eta(l) A),  c4 = sqrt(dtau U / 2),
the field storing eta(l) (the paper's type = 2 vertex sets phi = eta) and the
weight carrying gamma(l) per vertex; the 1/4 is a constant and drops out.

Continuous field (outside the paper, which lists continuous HS fields as not
supported): exp(dtau U/2 A^2) = int dphi (2pi)^-1/2 exp(-phi^2/2) exp(c phi A)
with c = sqrt(dtau U).
"""
from dataclasses import dataclass
from typing import Optional

import numpy as np


def ising_coupling(U: float, dtau: float) -> float:
    """lambda with cosh(lambda) = exp(dtau U / 2)."""
    return float(np.arccosh(np.exp(dtau * U / 2.0)))


def gauss_coupling(U: float, dtau: float) -> float:
    """c = sqrt(dtau U) of the Gaussian identity."""
    return float(np.sqrt(dtau * U))


def ising4_coupling(U: float, dtau: float) -> float:
    """sqrt(dtau lambda) of Eq. (HS_squares) with lambda = U / 2."""
    return float(np.sqrt(dtau * U / 2.0))


# values of the four-valued field, in the order l = -2, -1, +1, +2 (Eq. (HS_squares))
_S6 = float(np.sqrt(6.0))
ETA4 = (-float(np.sqrt(2.0 * (3.0 + _S6))), -float(np.sqrt(2.0 * (3.0 - _S6))),
        float(np.sqrt(2.0 * (3.0 - _S6))), float(np.sqrt(2.0 * (3.0 + _S6))))
GAMMA4 = (1.0 - _S6 / 3.0, 1.0 + _S6 / 3.0, 1.0 + _S6 / 3.0, 1.0 - _S6 / 3.0)


def ising4_index(phi) -> np.ndarray:
    """Index (0..3, order l = -2, -1, +1, +2) of stored field values eta(l)."""
    phi = np.asarray(phi, dtype=np.float64)
    return (phi > ETA4[0]).astype(int) + (phi > ETA4[1]).astype(int) + (phi > ETA4[2]).astype(int)


def expm_sym(K: np.ndarray, x: float) -> np.ndarray:
    """exp(x K) for symmetric K from its eigendecomposition, the way the
    paper's Operator type exponentiates a Hermitian matrix (table "operator":
    U and E from diagonalising O)."""
    w, V = np.linalg.eigh(K)
    return (V * np.exp(x * w)[None, :]) @ V.T


@dataclass
class Model:
    """Parameters of one chain.  Field layout: field[tau-1, i] is the field of
    vertex i on slice tau (tau = 1..L), as the paper's nsigma array."""
    K: np.ndarray
    beta: float
    dtau: float
    n_wrap: int
    coupling: float          # lambda (ising), c (gauss) or c4 (ising4)
    U: float = 0.0           # only used by the potential-energy estimator
    alpha: float = -0.5
    n_col: int = 2
    field_kind: str = "ising"
    trotter: str = "sym"
    seed: int = 0
    prop_width: float = 1.0  # width a of the continuous-field local move

    def __post_init__(self):
        self.K = np.asarray(self.K, dtype=np.float64)
        self.N = self.K.shape[0]
        self.L = int(round(self.beta / self.dtau))
        if abs(self.L * self.dtau - self.beta) > 1e-12 * self.beta:
            raise ValueError("beta must be an integer multiple of dtau")
        if self.L % self.n_wrap != 0:
            raise ValueError("L must be a multiple of n_wrap")
        self.expK = expm_sym(self.K, -self.dtau)          # exp(-dtau K)
        self.expK_inv = expm_sym(self.K, +self.dtau)      # exp(+dtau K)
        self.expK_half = expm_sym(self.K, -self.dtau / 2)
        self.expK_half_inv = expm_sym(self.K, +self.dtau / 2)

    @property
    def n_stab(self) -> int:
        return self.L // self.n_wrap

    def vdiag(self, field_slice: np.ndarray) -> np.ndarray:
        """Diagonal of exp(V_tau) for one slice: exp(coupling * field)."""
        return np.exp(self.coupling * np.asarray(field_slice, dtype=np.float64))

    def B(self, field: np.ndarray, tau: int) -> np.ndarray:
        """B'_tau = exp(V_tau) exp(-dtau K), the sampling-frame slice
        propagator (the paper's B_tau of Eq. (Green_eq) with the factors
        cyclically reordered; the determinant is unchanged)."""
        return self.vdiag(field[tau - 1])[:, None] * self.expK

    def B_inv(self, field: np.ndarray, tau: int) -> np.ndarray:
        return self.expK_inv * (1.0 / self.vdiag(field[tau - 1]))[None, :]

    def vertex_log_factor(self, s) -> np.ndarray:
        """log of the factor one vertex's field value carries in the weight
        besides exp(N_col coupling alpha s): the Gaussian measure -phi^2/2 of
        the continuous field, log gamma(l) of the four-valued field of
        Eq. (HS_squares), zero for the two-valued field (elementwise)."""
        s = np.asarray(s, dtype=np.float64)
        if self.field_kind == "gauss":
            return -0.5 * s * s
        if self.field_kind == "ising4":
            return np.log(np.array(GAMMA4))[ising4_index(s)]
        return np.zeros_like(s)

    def prefactor_log(self, field: np.ndarray) -> float:
        """log of the field-dependent prefactor of Eq. (partition_2):
        N_col * coupling * alpha * sum(field) plus the vertex factors above."""
        f = np.asarray(field, dtype=np.float64)
        out = self.n_col * self.coupling * self.alpha * f.sum()
        out += float(np.sum(self.vertex_log_factor(f)))
        return float(out)


def mz_frame_hopping(T, h, sign) -> np.ndarray:
    """Hopping of the sampling frame for the M_z form of the Hubbard model
    (section "The M_z-Hubbard model on a square lattice": two flavours with
    V = +1 and -1 on the site, alpha = 0, flavour hopping T_up, T_dn) with a
    Zeeman field h: T_up = T - h, T_dn = T + h.  The field coupled to
    n_up - n_dn becomes, under c_{i,dn} = s_i c'^+_i, the field coupled to
    n_1 + n_2 - 1 of the density frame, and the flavours' hopping become
    K_1 = T_up and K_2 = -S T_dn^T S (S = diag(s)).  When these agree (T
    symmetric, T_ij = 0 unless s_i s_j = -1, no chemical potential) one
    Green's function serves both and K = T - h 1; otherwise the two flavours
    need two Green's functions, outside this frame (ValueError)."""
    T = np.asarray(T, dtype=np.float64)
    S = np.diag(np.asarray(sign, dtype=np.float64))
    n = T.shape[0]
    K1 = T - h * np.eye(n)
    K2 = -S @ (T + h * np.eye(n)).T @ S
    if not np.array_equal(K1, K2):
        raise ValueError("the two flavours' hopping differ in the density frame")
    return K1


def hubbard_model(K, U, beta, dtau, n_wrap, field_kind="ising", trotter="sym", seed=0) -> Model:
    lam = {"ising": ising_coupling, "gauss": gauss_coupling, "ising4": ising4_coupling}[field_kind](U, dtau)
    return Model(K=K, beta=beta, dtau=dtau, n_wrap=n_wrap, coupling=lam, U=U,
                 field_kind=field_kind, trotter=trotter, seed=seed)


def product_B(model: Model, field: np.ndarray, tau2: int, tau1: int) -> np.ndarray:
    """Unstabilised B'(tau2, tau1) = B'_{tau2} ... B'_{tau1+1} (tiny cases only)."""
    P = np.eye(model.N)
    for tau in range(tau1 + 1, tau2 + 1):
        P = model.B(field, tau) @ P
    return P


def green_naive(model: Model, field: np.ndarray, tau: int = 0) -> np.ndarray:
    """G(tau) = (1 + B'(tau,0) B'(beta,tau))^-1 by a plain inverse (tiny, well
    conditioned cases only; Eq. (Green_eq))."""
    A = product_B(model, field, tau, 0) @ product_B(model, field, model.L, tau)
    return np.linalg.inv(np.eye(model.N) + A)


def init_field(model: Model, seed: Optional[int] = None) -> np.ndarray:
    """Random start (section "Monte Carlo sampling": the run starts from a
    randomly chosen configuration): s = +1 iff u < 1/2 for an Ising field,
    eta(l) with index floor(4 u) for the four-valued field, phi ~ N(0, 1) for a
    Gaussian field; draws addressed by (INIT, 0, tau, site)."""
    from . import philox
    seed = model.seed if seed is None else seed
    f = np.empty((model.L, model.N))
    for tau in range(1, model.L + 1):
        if model.field_kind == "ising":
            u = philox.uniforms(seed, philox.TAG_INIT, 0, tau, 0, model.N)
            f[tau - 1] = np.where(u < 0.5, 1.0, -1.0)
        elif model.field_kind == "ising4":
            u = philox.uniforms(seed, philox.TAG_INIT, 0, tau, 0, model.N)
            f[tau - 1] = np.array(ETA4)[np.floor(4.0 * u).astype(int)]
        else:
            f[tau - 1] = philox.normals(seed, philox.TAG_INIT, 0, tau, 0, model.N)
    return f
