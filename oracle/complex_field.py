"""The paper-literal complex formulation of the SU(2) Hubbard model (oracle
side; test infrastructure: only the tests, the smoke check and the CPU leg of
the benchmark use it).

Section "The SU(2)-Hubbard model on a square lattice": the repulsive model
H = sum_sigma c^+ T c + (U/2) sum_x (n_x - 1)^2, n_x = n_x,up + n_x,dn, with
N_fl = 1, N_col = 2, one vertex V = e_x e_x^T per site and alpha = -1/2.  The
interaction is decoupled with the four-valued field of Eq. (HS_squares) at
lambda = -U/2, so its coupling sqrt(dtau lambda) is imaginary (the example's
g = sqrt(-dtau U / N_SUN)):

    exp(-dtau U/2 A^2) ~ 1/4 sum_l gamma(l) exp(i c eta(l) A),  c = sqrt(dtau U / 2),

in the original frame (no particle-hole map): the field couples to the
total density, both spin colours share one complex Green's function, and the
slice propagator is B_tau = diag(exp(i c eta_tau)) exp(-dtau T) (the factor
order of the real frame).  The identity is exact up to an effective U for the
density, because A^2 = (n - 1)^2 only takes the values 0 and 1:

    1/2 (gamma(1) cos(c eta(1)) + gamma(2) cos(c eta(2))) = exp(-dtau U_eff / 2).

Weight (Eq. (partition_2)):

    W(C) = prod gamma(l) [exp(i c alpha sum eta) det(1 + B(beta,0))]^N_col,

complex in general; its phase W / |W| is Eq. (phase).  At half filling on a
bipartite lattice the bracket is real, so W >= 0 and the phase is 1 up to
rounding (no sign problem, but complex arithmetic throughout).

Readings where the paper is silent:
- the chain samples |W| and carries the phase W / |W| along (the paper's
  reweighting of observables by the phase); a flip is accepted iff u < |R|,
  R = W(C') / W(C) from the fast formula below, and the phase is multiplied
  by R / |R|;
- the flip ratio: Delta = exp(i c (eta' - eta)) - 1, r = 1 + Delta (1 - G_ii),
  R = gamma(l') / gamma(l) exp(N_col i c alpha (eta' - eta)) r^N_col, and the
  Sherman-Morrison update of the complex G as in the real frame;
- estimators in the original frame, per colour n_i = 1 - G~_ii:
  D = (1/N) sum_i (1 - G~_ii)^2 (both colours carry the same G),
  E_kin = (N_col / N)(Tr T - Tr(T G)), E_pot = U D, each as its real part;
- "Precision Phase": the largest |phase - 1| over the run, the recomputed
  phase of this sign-free model being exactly 1.
"""
import numpy as np

from . import hubbard, philox
from .hubbard import ETA4, GAMMA4, ising4_index
from .measure import measured_green
from .stable import left_udv, merge
from .sweep import Chain


def imag_coupling(U: float, dtau: float) -> float:
    """c of the imaginary coupling i c = sqrt(-dtau U / 2)."""
    return float(np.sqrt(dtau * U / 2.0))


def u_eff(U: float, dtau: float) -> float:
    """The density interaction the four-valued imaginary identity reproduces
    exactly on A^2 in {0, 1}."""
    c = imag_coupling(U, dtau)
    v = 0.5 * (GAMMA4[2] * np.cos(c * ETA4[2]) + GAMMA4[3] * np.cos(c * ETA4[3]))
    return float(-2.0 * np.log(v) / dtau)


class ComplexModel(hubbard.Model):
    """A four-valued field with the imaginary coupling i c on every site."""

    def vdiag(self, field_slice):
        return np.exp(1j * self.coupling * np.asarray(field_slice, dtype=np.float64))

    def prefactor_log(self, field) -> complex:
        """log of prod gamma(l) exp(N_col i c alpha sum eta) (complex)."""
        f = np.asarray(field, dtype=np.float64)
        return complex(self.n_col * 1j * self.coupling * self.alpha * f.sum()
                       + np.sum(self.vertex_log_factor(f)))


def complex_model(K, U, beta, dtau, n_wrap, trotter="sym", seed=0) -> ComplexModel:
    return ComplexModel(K=K, beta=beta, dtau=dtau, n_wrap=n_wrap, coupling=imag_coupling(U, dtau), U=U,
                        field_kind="ising4", trotter=trotter, seed=seed)


def logdet_complex(model, field) -> complex:
    """log det(1 + B(beta,0)) with its phase, from the stabilised left form
    B(beta,0)^T = Q D T: 1 + B(beta,0) = [conj(Q) D_b^-1 + T^T D_s] D_b Q^T, so
    det = det(X) prod D_b det(Q) with X the bracket (the merge's matrix with
    the identity as right form)."""
    left = left_udv(model, field, 0)
    Db, Ds = np.maximum(left.D, 1.0), np.minimum(left.D, 1.0)
    X = left.Q.conj() / Db[None, :] + left.T.T * Ds[None, :]
    return complex(np.log(complex(np.linalg.det(X))) + np.sum(np.log(Db)) + np.log(complex(np.linalg.det(left.Q))))


def log_weight_complex(model, field) -> complex:
    """log W(C) of Eq. (partition_2), complex."""
    return model.prefactor_log(field) + model.n_col * logdet_complex(model, field)


def equal_time_complex(model, G):
    """(D, E_kin, E_pot) per site of one configuration, real parts, in the
    original frame (n_i per colour = 1 - G~_ii)."""
    Gt = measured_green(model, G)
    d = 1.0 - np.diag(Gt)
    D = np.mean(d * d)
    ekin = model.n_col / model.N * (np.trace(model.K) - np.trace(model.K @ G))
    return float(D.real), float(ekin.real), float(model.U * D.real)


class ComplexChain(Chain):
    """The sweep of Algorithm 1 for the complex field: the wraps, the
    stabilisation and the merge are those of the real chain (they take complex
    matrices as they are); the flip, the phase and the estimators follow the
    module's description."""

    def __init__(self, model, field, sweep_counter: int = 0):
        super().__init__(model, field, sweep_counter)
        self.phase = 1.0 + 0.0j
        self.phase_dev = 0.0      # largest |phase - 1| seen

    def _propose(self, tau: int, i: int, u: float, u1: float):
        m = self.m
        s = self.field[tau - 1, i]
        k = int(ising4_index(s))
        j = min(int(3.0 * u1), 2)
        kn = j if j < k else j + 1
        s_new = ETA4[kn]
        extra = float(m.vertex_log_factor(s_new)) - float(m.vertex_log_factor(s))
        delta = np.exp(1j * m.coupling * (s_new - s)) - 1.0
        r = 1.0 + delta * (1.0 - self.G[i, i])
        R = np.exp(m.n_col * 1j * m.coupling * m.alpha * (s_new - s) + extra) * r ** m.n_col
        absR = abs(R)
        self.proposals += 1
        self.min_tie = min(self.min_tie, abs(absR - u))
        acc = bool(u < absR)
        if acc:
            G = self.G
            col = G[:, i].copy()
            row = -G[i, :].copy()
            row[i] += 1.0
            self.G = G - (delta / r) * np.outer(col, row)
            self.field[tau - 1, i] = s_new
            self.accepted += 1
            self.phase = self.phase * (R / absR)
            self.phase_dev = max(self.phase_dev, abs(self.phase - 1.0))
        if self.trace is not None:
            self.trace.append(("flip", tau, i, complex(R), float(u), acc))
        return acc

    def _measure(self, measure: bool):
        if measure:
            D, ekin, epot = equal_time_complex(self.m, self.G)
            self.bins += np.array([D, ekin, epot, 1.0])


def init_field(model, seed=None):
    """Random start: eta(l) with index floor(4 u), draws (INIT, 0, tau, site)."""
    return hubbard.init_field(model, seed)


__all__ = ["imag_coupling", "u_eff", "ComplexModel", "complex_model", "logdet_complex", "log_weight_complex",
           "equal_time_complex", "ComplexChain", "init_field", "philox"]
