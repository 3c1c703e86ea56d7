"""Pins of the oracle's general vertices and Ising fields with their own
action (section "Definition of the Hamiltonian", Eqs. (general_ham_v) and
(general_ham_i); table "operator"; section "Sampling of e^{-S_{0,I}}"; the
example of Eq. (hubbard_sun_Ising): Ising spins on bonds coupled to the bond
hopping, a transverse field h and a coupling J between them, and the Hubbard
interaction on the sites).

Independent of the oracle, the Fock space of the fermions times the Ising
spins is built from Jordan-Wigner fermions and Pauli matrices, and the
Trotter product of one slice,
    S = exp(dtau h sum X) exp(dtau J sum Z Z) F exp(-dtau H_T),
F the product of exp(-dtau xi Z_b O_b) over the bonds and
exp(-dtau U/2 (n_i - 1)^2) over the sites in the vertex order, gives
<O> = Tr(S^L O) / Tr(S^L).  The enumeration of every Ising and HS
configuration with the oracle's weight (S0, N_col = 2 determinants in the
particle-hole frame) must reproduce it; the two bonds share a site, so their
exponentials do not commute and their order is pinned too.  Planted mistakes
(the bond order reversed, S0 of the wrong sign, the Ising spins left without
S0) fail."""
import itertools

import numpy as np
import pytest

from oracle import stable
from oracle import vertices as vx


def _expmh(H, x):
    w, V = np.linalg.eigh(H)
    return (V * np.exp(x * w)[None, :]) @ V.T


class BondIsingFock:
    """Fermions (two spins) on a chain times Ising spins on its bonds."""

    def __init__(self, n_sites, bonds, t, U, xi, h, J, pairs, periodic=False):
        nm = 2 * n_sites
        nb = len(bonds)
        a = np.array([[0.0, 1.0], [0.0, 0.0]])
        Zp, I2 = np.diag([1.0, -1.0]), np.eye(2)
        Xp = np.array([[0.0, 1.0], [1.0, 0.0]])
        c = []
        for m in range(nm):
            op = np.array([[1.0]])
            for j in range(nm):
                op = np.kron(op, Zp if j < m else (a if j == m else I2))
            c.append(op)
        dF, dI = 2 ** nm, 2 ** nb

        def ising(op, b):
            out = np.array([[1.0]])
            for j in range(nb):
                out = np.kron(out, op if j == b else I2)
            return out

        self.IF, self.II = np.eye(dF), np.eye(dI)
        mode = lambda i, s: 2 * i + s  # noqa: E731
        hop = lambda x, y: sum(c[mode(x, s)].T @ c[mode(y, s)] + c[mode(y, s)].T @ c[mode(x, s)]  # noqa: E731
                               for s in range(2))
        HT = np.zeros((dF, dF))
        for x in range(n_sites - (0 if periodic else 1)):
            HT += -t * hop(x, (x + 1) % n_sites)
        self.n = [[c[mode(i, s)].T @ c[mode(i, s)] for s in range(2)] for i in range(n_sites)]
        HU = [0.5 * U * (self.n[i][0] + self.n[i][1] - self.IF) @ (self.n[i][0] + self.n[i][1] - self.IF)
              for i in range(n_sites)]
        self.N = n_sites
        self.HT = HT
        self.parts = dict(HT=HT, HU=HU, hop=[hop(x, y) for x, y in bonds], Z=[ising(Zp, b) for b in range(nb)],
                          X=[ising(Xp, b) for b in range(nb)], pairs=pairs, xi=xi, h=h, J=J)

    def slice_operator(self, dtau, order=None):
        p = self.parts
        nb = len(p["Z"])
        TX = np.eye(self.II.shape[0])
        for b in range(nb):
            TX = _expmh(p["X"][b], dtau * p["h"]) @ TX
        DZ = np.zeros_like(self.II)
        for a, b in p["pairs"]:
            DZ += p["Z"][a] @ p["Z"][b]
        DZ = _expmh(DZ, dtau * p["J"]) if p["pairs"] else self.II
        F = np.eye(self.IF.shape[0] * self.II.shape[0])
        factors = [np.kron(self.IF, self.II)] * 0
        xis = p["xi"] if np.ndim(p["xi"]) else [p["xi"]] * nb
        for b in (order if order is not None else range(nb)):
            factors.append(_expmh(np.kron(p["hop"][b], p["Z"][b]), -dtau * xis[b]))
        for HUi in p["HU"]:
            factors.append(np.kron(_expmh(HUi, -dtau), self.II))
        for f in factors:
            F = F @ f
        return np.kron(self.IF, TX @ DZ) @ F @ np.kron(_expmh(p["HT"], -dtau), self.II)

    def expect(self, S, O, L):
        Sl = np.linalg.matrix_power(S, L)
        Of = np.kron(O, self.II)
        return float(np.trace(Sl @ Of) / np.trace(Sl))

    def double_occ(self):
        return sum(self.n[i][0] @ self.n[i][1] for i in range(self.N)) / self.N

    def kinetic(self):
        return self.HT / self.N


def _fields(m):
    for vals in itertools.product([-1.0, 1.0], repeat=m.L * m.M):
        yield np.array(vals).reshape(m.L, m.M)


def _enumerate(m):
    ws, obs = [], []
    for f in _fields(m):
        ws.append(np.exp(vx.log_weight(m, f)))
        G = stable.green_scratch(m, f, 0)
        D = np.mean(np.diag(G) * (1.0 - np.diag(G)))
        ekin = m.n_col / m.N * (np.trace(m.K) - np.trace(m.K @ G))
        obs.append([D, ekin])
    ws = np.array(ws)
    return np.array(obs).T @ ws / ws.sum()


PARAMS = dict(t=1.0, U=4.0, xi=(0.7, 0.3), h=1.1, J=0.4)


def _model(order=(0, 1), **kw):
    """The 3-site chain with Ising spins on bonds (0,1) and (1,2) of
    different fermion couplings, listed in the given order."""
    p = dict(PARAMS)
    p.update(kw)
    dtau, bonds = 0.25, [(0, 1), (1, 2)]
    m0 = vx.bond_ising_model(3, bonds, p["t"], p["U"], 1.0, p["h"], p["J"], 0.5, dtau, 1, pairs=[(0, 1)])
    vs = list(m0.vertices)
    for b in range(2):
        vs[b] = vx.Vertex(P=bonds[b], O=[[0.0, 1.0], [1.0, 0.0]], g=-dtau * p["xi"][b], ising=True)
    vs = [vs[order[0]], vs[order[1]]] + vs[2:]
    return vx.vertex_model(m0.K, vs, 0.5, dtau, 1, U=p["U"], h=p["h"], J=p["J"], pairs=[(0, 1)])


def _fock(order=None, **kw):
    p = dict(PARAMS)
    p.update(kw)
    F = BondIsingFock(3, [(0, 1), (1, 2)], p["t"], p["U"], p["xi"], p["h"], p["J"], [(0, 1)])
    S = F.slice_operator(0.25, order)
    return np.array([F.expect(S, F.double_occ(), 2), F.expect(S, F.kinetic(), 2)])


def test_bond_ising_enumeration_equals_fock():
    """3-site chain, two bonds with Ising spins (transverse field 1.1, coupling
    0.4 between them, fermion couplings 0.7 and 0.3), U = 4 on the sites, 2
    slices: D and E_kin over all 2^10 configurations equal the Fock-space
    Trotter product to 1e-12."""
    got = _enumerate(_model())
    assert np.max(np.abs(got - _fock())) < 1e-12


def test_bond_order_and_s0_are_pinned():
    """The two bonds share a site: with the other bond order in the oracle
    (or in the Fock product) the averages differ; S0 of the wrong sign, or no
    S0 at all, leave Fock space."""
    ref = _enumerate(_model())
    assert np.max(np.abs(_enumerate(_model(order=(1, 0))) - _fock(order=[1, 0]))) < 1e-12
    assert np.max(np.abs(ref - _fock(order=[1, 0]))) > 1e-6
    m = _model()
    m.Kt, m.dtJ = -m.Kt, -m.dtJ
    assert np.max(np.abs(_enumerate(m) - _fock())) > 1e-4
    m = _model()
    m.Kt, m.dtJ = 0.0, 0.0
    assert np.max(np.abs(_enumerate(m) - _fock())) > 1e-4


@pytest.fixture(scope="module")
def chain6():
    """A ring of 6 sites, Ising spins on all 6 bonds (neighbouring bonds
    coupled), U = 4: a lattice where every site has two bond vertices."""
    bonds = [(i, (i + 1) % 6) for i in range(6)]
    m = vx.bond_ising_model(6, bonds, 1.0, 4.0, 0.6, 0.9, 0.3, 1.0, 0.1, 5,
                            pairs=[(i, (i + 1) % 6) for i in range(6)], periodic=True, seed=4)
    return m, vx.init_field(m)


def test_stable_green_equals_naive_inverse(chain6):
    from oracle import hubbard
    m, f = chain6
    for tau in (0, 3, 7, 10):
        A = hubbard.product_B(m, f, tau, 0) @ hubbard.product_B(m, f, m.L, tau)
        assert np.max(np.abs(stable.green_scratch(m, f, tau) - np.linalg.inv(np.eye(m.N) + A))) < 1e-12


def test_fast_ratio_and_woodbury_update_equal_scratch(chain6):
    """In the frame where vertex k is leftmost, the chain's R equals the
    from-scratch weight ratio (bond vertices with S0 and site vertices), and
    the rank-|P| update equals that frame's scratch G of the new field."""
    m, f = chain6
    rng = np.random.default_rng(8)
    for _ in range(8):
        tau = int(rng.integers(1, m.L + 1))
        k = int(rng.integers(0, m.M))
        ch = vx.VertexChain(m, f.copy())
        # the frame: G(tau) moved by (E_0 ... E_{k-1})^-1
        X = np.eye(m.N)
        for j in range(k):
            X = X @ m.E_k(j, ch.field[tau - 1, j])
        ch.G = np.linalg.solve(X, stable.green_scratch(m, ch.field, tau) @ X)
        ch.trace = []
        old = ch.field.copy()
        assert ch._propose(tau, k, 0.0)
        R = ch.trace[-1][3]
        want = np.exp(vx.log_weight(m, ch.field) - vx.log_weight(m, old))
        assert abs(R - want) < 1e-9 * abs(want)
        X = np.eye(m.N)
        for j in range(k):
            X = X @ m.E_k(j, ch.field[tau - 1, j])
        assert np.max(np.abs(ch.G - np.linalg.solve(X, stable.green_scratch(m, ch.field, tau) @ X))) < 1e-10


def test_sweep_tracks_scratch_green(chain6):
    """Two sweeps: at the end G equals the from-scratch G(0) of the final
    field, and the wrapped-versus-recomputed deviations stay at rounding."""
    m, f = chain6
    ch = vx.VertexChain(m, f.copy()).init()
    for _ in range(2):
        ch.sweep()
    assert np.max(np.abs(ch.G - stable.green_scratch(m, ch.field, 0))) < 1e-10
    assert max(ch.prec) < 1e-9
    assert 0 < ch.accepted < ch.proposals


def test_chain_samples_the_weight():
    """2 sites, one bond spin and two site fields, 2 slices (64 configurations):
    the visited fields follow W / sum W (chi^2); without S0 they do not."""
    m = vx.bond_ising_model(2, [(0, 1)], 1.0, 4.0, 0.8, 0.7, 0.0, 0.5, 0.25, 2, seed=12)
    fields = list(_fields(m))
    p = np.array([np.exp(vx.log_weight(m, f)) for f in fields])
    p /= p.sum()
    index = {tuple(f.ravel()): j for j, f in enumerate(fields)}
    ch = vx.VertexChain(m, vx.init_field(m)).init()
    counts = np.zeros(p.size)
    n = 6000
    for _ in range(n):
        ch.sweep(measure=False)
        counts[index[tuple(ch.field.ravel())]] += 1
    assert np.sum((counts - n * p) ** 2 / (n * p)) / (p.size - 1) < 2.0
    m.Kt = 0.0
    q = np.array([np.exp(vx.log_weight(m, f)) for f in fields])
    q /= q.sum()
    assert np.sum((counts - n * q) ** 2 / (n * q)) / (q.size - 1) > 5.0


@pytest.mark.parametrize("L", [1, 2, 3])
def test_s0_ratio_equals_the_action_difference(L):
    """The local S0 ratio of a flip equals exp(S0(C) - S0(C')) of the whole
    action (periodic in tau) for every spin and slice, also with one slice,
    where the spin's temporal bond joins it to itself and does not change."""
    m = vx.bond_ising_model(4, [(0, 1), (1, 2), (2, 3)], 1.0, 2.0, 0.6, 0.7, 0.45, 0.3 * L, 0.3, 1,
                            pairs=[(0, 1), (1, 2), (0, 2)])
    rng = np.random.default_rng(L)
    f = np.where(rng.random((m.L, m.M)) < 0.5, 1.0, -1.0)
    for tau in range(1, m.L + 1):
        for k in range(m.M):
            g = f.copy()
            g[tau - 1, k] = -g[tau - 1, k]
            want = np.exp(m.S0(f) - m.S0(g))
            assert abs(m.s0_ratio(f, tau, k) - want) < 1e-13 * want
