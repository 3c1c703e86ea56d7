"""General operator vertices and Ising fields with their own dynamics (oracle
side; test infrastructure: only the tests, the smoke check and the CPU leg of
the benchmark use it).

Section "Definition of the Hamiltonian": the interaction is a sum of perfect
squares of one-body operators (Eq. (general_ham_v), decoupled by an HS field)
and of one-body operators coupled to Ising spins Z_k (Eq. (general_ham_i))
whose own dynamics H_{0,I} contributes the action S_{0,I} to the weight
(Eq. (partition_2)).  A vertex is the paper's Operator type (table
"operator"): X = P^T O P with P selecting |P| orbitals and O a real symmetric
|P| x |P| matrix, so exp(g phi X) = P^T exp(g phi O) P + (1 - P^T P).  The
example of the section "The SU(2)-Hubbard model on a square lattice coupled to
a transverse Ising field" (Eq. (hubbard_sun_Ising)) has Ising spins on the
bonds coupled to the bond hopping, O = [[0, 1], [1, 0]], g = -dtau xi, and the
Hubbard interaction on the sites; in the particle-hole frame of
oracle.hubbard the bond hopping of both spins maps to itself on a bipartite
lattice, so both colours share one G.

Slice propagator of the sampling frame and weight:

    B'_tau = E_0 E_1 ... E_{M-1} exp(-dtau K),   E_k = exp(g_k phi_{k,tau} X_k),
    W(C) = exp(-S0(C)) exp(N_col sum g_k alpha_k phi_{k,tau}) det(1 + B'(beta, 0))^N_col.

Ising action (the spins' transverse field h and a coupling J between listed
pairs of Ising vertices, in the Z basis of the Trotterised
exp(dtau h sum X) exp(dtau J sum Z Z), periodic in tau):

    exp(-S0) ~ prod exp(Kt s_{k,tau} s_{k,tau+1}) prod exp(dtau J s_{k,tau} s_{k',tau}),
    Kt = -1/2 ln tanh(dtau h).

Readings where the paper is silent:
- the order of the flips within a slice: in the upward pass, after the wrap
  by exp(-dtau K), vertices M-1, ..., 0, each after moving G to the frame in
  which E_k is the leftmost factor (G <- E_k G E_k^-1), which ends at G(tau);
  in the downward pass, from G(tau), vertices 0, ..., M-1, each followed by
  G <- E_k^-1 G E_k, then the wrap by exp(+dtau K); the equal-time estimators
  are taken on G(tau): after the flips in the upward pass, before them in
  the downward pass (the configuration they see is the chain's either way);
- the flip of a vertex (an Ising spin or a two-valued HS field, s' = -s):
  delta = exp(g (s' - s) O) - 1, R_P = 1 + delta (1 - G)_PP, R = det(R_P)^N_col
  exp(N_col g alpha (s' - s)) times, for an Ising spin, the ratio of exp(-S0),
  exp(-2 s (Kt (s_{k,tau-1} + s_{k,tau+1}) + dtau J sum_{k'} s_{k',tau})),
  accepted iff u < R; then G <- G - G[:,P] R_P^-1 delta (1 - G)[P,:]
  (Woodbury; the rank-1 update of the on-site vertices for |P| = 1);
- draws of vertex k from Philox counter (TAG_FLIP, sweep, (tau << 1) | dir, k).
"""
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

from . import hubbard, philox
from .measure import equal_time
from .stable import left_step, merge, right_step


@dataclass
class Vertex:
    P: Tuple[int, ...]
    O: np.ndarray
    g: float
    alpha: float = 0.0
    ising: bool = False          # an Ising spin with the action S0; else a two-valued HS field

    def __post_init__(self):
        self.P = tuple(int(p) for p in self.P)
        self.O = np.asarray(self.O, dtype=np.float64).reshape(len(self.P), len(self.P))


def _expm_small(O, x):
    w, V = np.linalg.eigh(O)
    return (V * np.exp(x * w)[None, :]) @ V.T


class VertexModel(hubbard.Model):
    """A hopping matrix K and an ordered list of vertices, N_col colours
    sharing one G, the Ising spins' transverse field h and pair coupling J."""

    def setup(self, vertices: Sequence[Vertex], h: float = 0.0, J: float = 0.0,
              pairs: Sequence[Tuple[int, int]] = ()):
        self.vertices = list(vertices)
        self.M = len(self.vertices)
        self.Kt = float(-0.5 * np.log(np.tanh(self.dtau * h))) if h > 0.0 else 0.0
        self.dtJ = float(self.dtau * J)
        self.pairs = [tuple(p) for p in pairs]
        self.nbr = [[] for _ in range(self.M)]
        for a, b in self.pairs:
            self.nbr[a].append(b)
            self.nbr[b].append(a)
        return self

    # -- slice propagators ---------------------------------------------------
    def E_k(self, k: int, s: float) -> np.ndarray:
        """exp(g_k s X_k) as an N x N matrix."""
        v = self.vertices[k]
        E = np.eye(self.N)
        idx = np.array(v.P)
        E[np.ix_(idx, idx)] = _expm_small(v.O, v.g * s)
        return E

    def expV(self, row) -> np.ndarray:
        out = np.eye(self.N)
        for k in range(self.M - 1, -1, -1):
            out = self.E_k(k, row[k]) @ out
        return out

    def expV_inv(self, row) -> np.ndarray:
        out = np.eye(self.N)
        for k in range(self.M):
            out = self.E_k(k, -row[k]) @ out
        return out

    def B(self, field, tau: int) -> np.ndarray:
        return self.expV(field[tau - 1]) @ self.expK

    def B_inv(self, field, tau: int) -> np.ndarray:
        return self.expK_inv @ self.expV_inv(field[tau - 1])

    # -- weight ---------------------------------------------------------------
    def S0(self, field) -> float:
        """S0 of the Ising spins (up to a constant), periodic in tau."""
        f = np.asarray(field, dtype=np.float64)
        s = 0.0
        for k, v in enumerate(self.vertices):
            if v.ising:
                s -= self.Kt * float(np.sum(f[:, k] * np.roll(f[:, k], -1)))
        for a, b in self.pairs:
            s -= self.dtJ * float(np.sum(f[:, a] * f[:, b]))
        return s

    def prefactor_log(self, field) -> float:
        f = np.asarray(field, dtype=np.float64)
        out = -self.S0(f)
        for k, v in enumerate(self.vertices):
            out += self.n_col * v.g * v.alpha * float(np.sum(f[:, k]))
        return out

    def s0_ratio(self, field, tau: int, k: int) -> float:
        """exp(-S0(C')) / exp(-S0(C)) for flipping the Ising spin k at tau."""
        if not self.vertices[k].ising:
            return 1.0
        s = field[tau - 1, k]
        up = field[tau % self.L, k]
        dn = field[(tau - 2) % self.L, k]
        # with a single slice the spin's temporal bond is to itself: a constant
        loc = (self.Kt * (up + dn) if self.L > 1 else 0.0) + self.dtJ * sum(field[tau - 1, j] for j in self.nbr[k])
        return float(np.exp(-2.0 * s * loc))


def vertex_model(K, vertices, beta, dtau, n_wrap, U=0.0, h=0.0, J=0.0, pairs=(), n_col=2, trotter="asym",
                 seed=0) -> VertexModel:
    m = VertexModel(K=K, beta=beta, dtau=dtau, n_wrap=n_wrap, coupling=0.0, U=U, n_col=n_col, trotter=trotter,
                    seed=seed)
    return m.setup(vertices, h=h, J=J, pairs=pairs)


def log_weight(model: VertexModel, field) -> float:
    from .stable import logdet_scratch
    return model.prefactor_log(field) + model.n_col * logdet_scratch(model, field)


def init_field(model: VertexModel, seed=None) -> np.ndarray:
    """s = +1 iff u < 1/2, draws (INIT, 0, tau, vertex)."""
    seed = model.seed if seed is None else seed
    f = np.empty((model.L, model.M))
    for tau in range(1, model.L + 1):
        u = philox.uniforms(seed, philox.TAG_INIT, 0, tau, 0, model.M)
        f[tau - 1] = np.where(u < 0.5, 1.0, -1.0)
    return f


class VertexChain:
    """The sweep of Algorithm 1 with general vertices and the Ising action."""

    def __init__(self, model: VertexModel, field, sweep_counter: int = 0):
        self.m = model
        self.field = np.array(field, dtype=np.float64)
        self.sweep_counter = int(sweep_counter)
        self.G = None
        self.slots = None
        self.bins = np.zeros(4)
        self.proposals = 0
        self.accepted = 0
        self.prec = []
        self.min_tie = np.inf
        self.trace = None

    def init(self):
        m = self.m
        self.slots = [None] * (m.n_stab + 1)
        left = None
        for k in range(m.n_stab - 1, -1, -1):
            left = left_step(m, self.field, left, k * m.n_wrap, (k + 1) * m.n_wrap)
            self.slots[k] = left
        self.G, _ = merge(None, self.slots[0], m.N)
        return self

    def _propose(self, tau: int, k: int, u: float):
        m = self.m
        v = m.vertices[k]
        s = self.field[tau - 1, k]
        sn = -s
        idx = np.array(v.P)
        delta = _expm_small(v.O, v.g * (sn - s)) - np.eye(len(idx))
        one_m_G = np.eye(m.N)[idx][:, idx] - self.G[np.ix_(idx, idx)]
        RP = np.eye(len(idx)) + delta @ one_m_G
        R = np.linalg.det(RP) ** m.n_col * np.exp(m.n_col * v.g * v.alpha * (sn - s)) * m.s0_ratio(self.field, tau, k)
        self.proposals += 1
        self.min_tie = min(self.min_tie, abs(R - u))
        acc = bool(u < R)
        if acc:
            G = self.G
            right = (np.eye(m.N)[idx] - G[idx, :])            # (1 - G)[P, :]
            self.G = G - G[:, idx] @ np.linalg.solve(RP, delta @ right)
            self.field[tau - 1, k] = sn
            self.accepted += 1
        if self.trace is not None:
            self.trace.append(("flip", tau, k, float(R), float(u), acc))
        return acc

    def _draws(self, tau, direction):
        m = self.m
        w = philox.philox4x64_10_vec(np.uint64(philox.TAG_FLIP), np.uint64(self.sweep_counter),
                                     np.uint64(philox.slot(tau, direction)),
                                     np.arange(m.M, dtype=np.uint64), (m.seed, 0))
        return philox.to_unit(w[0])

    def _frame(self, tau, k, forward: bool):
        """G <- E_k G E_k^-1 (forward) or E_k^-1 G E_k, with the current field."""
        m = self.m
        s = self.field[tau - 1, k]
        E, Ei = m.E_k(k, s), m.E_k(k, -s)
        self.G = E @ self.G @ Ei if forward else Ei @ self.G @ E

    def _measure(self, measure):
        if measure:
            D, ekin, epot = equal_time(self.m, self.G)
            self.bins += np.array([D, ekin, epot, 1.0])

    def _stab(self, G_s, G_cmp):
        self.prec.append(float(np.max(np.abs(G_cmp - G_s))))
        self.G = G_s

    def sweep(self, measure=True):
        m = self.m
        nw, nk = m.n_wrap, m.n_stab
        if self.G is None:
            self.init()
        right = None
        for tau in range(1, m.L + 1):
            self.G = m.expK @ self.G @ m.expK_inv
            u = self._draws(tau, philox.DIR_UP)
            for k in range(m.M - 1, -1, -1):
                self._frame(tau, k, True)
                self._propose(tau, k, float(u[k]))
            if tau % nw == 0:
                j = tau // nw
                right = right_step(m, self.field, right, tau - nw, tau)
                left = self.slots[j] if j < nk else None
                G_s, _ = merge(right, left, m.N)
                self.slots[j] = right
                self._stab(G_s, self.G)
            self._measure(measure)
        left = None
        for tau in range(m.L, 0, -1):
            self._measure(measure)
            u = self._draws(tau, philox.DIR_DOWN)
            for k in range(m.M):
                self._propose(tau, k, float(u[k]))
                self._frame(tau, k, False)
            G_w = m.expK_inv @ self.G @ m.expK
            if (tau - 1) % nw == 0:
                j = (tau - 1) // nw
                left = left_step(m, self.field, left, tau - 1, tau - 1 + nw)
                right = self.slots[j] if j > 0 else None
                G_s, _ = merge(right, left, m.N)
                self.slots[j] = left
                self._stab(G_s, G_w)
            else:
                self.G = G_w
        self.sweep_counter += 1
        return self


def bond_ising_model(L_sites: int, bonds, t: float, U: float, xi: float, h: float, J: float, beta: float,
                     dtau: float, n_wrap: int, pairs=(), trotter="asym", seed=0, periodic=False) -> VertexModel:
    """The example of Eq. (hubbard_sun_Ising) on a chain of L_sites sites: Ising
    spins on the given bonds coupled to the bond hopping (g = -dtau xi), then
    the Hubbard interaction on every site through the exact two-valued field of
    the particle-hole frame (coupling lambda, alpha = -1/2), N_col = 2."""
    K = np.zeros((L_sites, L_sites))
    for a in range(L_sites - (0 if periodic else 1)):
        b = (a + 1) % L_sites
        K[a, b] = K[b, a] = -t
    vs: List[Vertex] = [Vertex(P=(a, b), O=[[0.0, 1.0], [1.0, 0.0]], g=-dtau * xi, ising=True) for a, b in bonds]
    lam = hubbard.ising_coupling(U, dtau) if U > 0.0 else 0.0
    if U > 0.0:
        vs += [Vertex(P=(i,), O=[[1.0]], g=lam, alpha=-0.5) for i in range(L_sites)]
    return vertex_model(K, vs, beta, dtau, n_wrap, U=U, h=h, J=J, pairs=pairs, trotter=trotter, seed=seed)


__all__ = ["Vertex", "VertexModel", "vertex_model", "log_weight", "init_field", "VertexChain", "bond_ising_model"]
