"""Pins of the oracle's complex (imaginary-coupling) formulation of the SU(2)
Hubbard model (section "The SU(2)-Hubbard model on a square lattice",
Eq. (HS_squares) with lambda = -U/2, Eq. (partition_2), Eq. (phase)).

The four-valued identity is exact at an effective U because (n - 1)^2 is 0 or
1, so an enumeration of every field configuration of a tiny lattice must
reproduce the Fock-space Trotter product of the repulsive Hubbard model at
that U_eff (tests/fock.py, the original frame, no particle-hole map); the
weight of every configuration must be real and positive (the phase is 1 on a
half-filled bipartite lattice); the fast flip ratio must equal the ratio of
from-scratch complex weights; and the chain must sample |W|.  Planted
mistakes (the sign of alpha, the coupling left real) fail these."""
import itertools

import numpy as np
import pytest

from fock import Fock
from inputs import square_lattice
from oracle import complex_field as cf
from oracle import hubbard, stable


def _all_fields(m):
    for vals in itertools.product(hubbard.ETA4, repeat=m.L * m.N):
        yield np.array(vals).reshape(m.L, m.N)


def test_imaginary_four_valued_identity_and_effective_u():
    """1/4 sum_l gamma(l) exp(i c eta(l) A) is 1 at A = 0 and exp(-dtau U_eff/2)
    at A = +-1, with U_eff - U of order dtau^3 (halving dtau divides it by 8)."""
    U = 4.0
    for dtau in (0.1, 0.05):
        c = cf.imag_coupling(U, dtau)
        for A, want in ((0.0, 1.0), (1.0, np.exp(-dtau * cf.u_eff(U, dtau) / 2)),
                        (-1.0, np.exp(-dtau * cf.u_eff(U, dtau) / 2))):
            got = sum(g * np.exp(1j * c * e * A) for g, e in zip(hubbard.GAMMA4, hubbard.ETA4)) / 4.0
            assert abs(got - want) < 1e-14
    e1 = cf.u_eff(U, 0.1) - U
    e2 = cf.u_eff(U, 0.05) - U
    assert abs(e1) < 1e-3 and abs(e1 / e2 - 8.0) < 0.5


@pytest.mark.parametrize("trotter", ["sym", "asym"])
def test_complex_enumeration_equals_fock_trotter(trotter):
    """2 sites x 2 slices, all 4^4 fields: phases 1, and the weighted averages
    of D and E_kin at both slices equal the Fock-space Trotter product of the
    repulsive model at U_eff."""
    K = np.array([[0.0, -1.0], [-1.0, 0.0]])
    U, dtau, L = 4.0, 0.25, 2
    m = cf.complex_model(K, U, L * dtau, dtau, 1, trotter=trotter)
    ws, obs = [], []
    for f in _all_fields(m):
        lw = cf.log_weight_complex(m, f)
        w = np.exp(lw)
        assert abs(w / abs(w) - 1.0) < 1e-10
        ws.append(w.real)
        obs.append([cf.equal_time_complex(m, stable.green_scratch(m, f, t))[:2] for t in (0, 1)])
    ws = np.array(ws)
    res = np.einsum("c,ctk->tk", ws, np.array(obs)) / ws.sum()
    F = Fock(K, cf.u_eff(U, dtau))
    S = F.trotter(dtau) if trotter == "sym" else F.trotter_asym(dtau)
    assert np.max(np.abs(res[:, 0] - F.expect_with(S, F.double_occ(), L))) < 1e-12
    assert np.max(np.abs(res[:, 1] - F.expect_with(S, F.kinetic(), L))) < 1e-12


def test_complex_phase_detects_planted_mistakes():
    """With alpha of the wrong sign the configurations' phases leave 1; with
    the coupling left real (no factor i) the averages leave Fock space."""
    K = np.array([[0.0, -1.0], [-1.0, 0.0]])
    U, dtau, L = 4.0, 0.25, 2
    m = cf.complex_model(K, U, L * dtau, dtau, 1)
    m.alpha = +0.5
    worst = max(abs(np.exp(cf.log_weight_complex(m, f)) / abs(np.exp(cf.log_weight_complex(m, f))) - 1.0)
                for f in _all_fields(m))
    assert worst > 1e-2
    m2 = cf.complex_model(K, U, L * dtau, dtau, 1)
    m2.vdiag = lambda fs: np.exp(m2.coupling * np.asarray(fs, dtype=float))
    ws, ds = [], []
    for f in _all_fields(m2):
        ws.append(np.exp(cf.log_weight_complex(m2, f)))
        ds.append(cf.equal_time_complex(m2, stable.green_scratch(m2, f, 0))[0])
    F = Fock(K, cf.u_eff(U, dtau))
    D = F.expect_with(F.trotter(dtau), F.double_occ(), L)
    got = np.real(np.dot(ws, ds) / np.sum(ws))
    assert abs(got - D) > 1e-3


@pytest.fixture(scope="module")
def c3x3():
    # a bipartite lattice (the phase is 1 only there)
    lat = square_lattice(4, 2)
    m = cf.complex_model(lat.K, 4.0, 1.0, 0.1, 5, seed=2)
    return m, cf.init_field(m)


def test_complex_phase_on_a_frustrated_lattice_is_not_one():
    """On the 3x3 torus (odd cycles, not bipartite) the weight is genuinely
    complex: the phase argument needs the bipartite structure."""
    lat = square_lattice(3, 3)
    m = cf.complex_model(lat.K, 4.0, 1.0, 0.1, 5, seed=2)
    w = np.exp(cf.log_weight_complex(m, cf.init_field(m)))
    assert abs(w / abs(w) - 1.0) > 1e-6


def test_complex_stable_green_equals_naive_inverse(c3x3):
    m, f = c3x3
    for tau in (0, 3, 7, 10):
        A = hubbard.product_B(m, f, tau, 0) @ hubbard.product_B(m, f, m.L, tau)
        G0 = np.linalg.inv(np.eye(m.N) + A)
        assert np.max(np.abs(stable.green_scratch(m, f, tau) - G0)) < 1e-12


def test_complex_flip_ratio_equals_weight_ratio_and_update_equals_scratch(c3x3):
    """The chain's fast ratio R (recorded by its trace) equals W(C')/W(C) of
    the from-scratch complex weights, and the updated G equals the scratch G
    of the new field."""
    m, f = c3x3
    rng = np.random.default_rng(5)
    for _ in range(6):
        tau = int(rng.integers(1, m.L + 1))
        i = int(rng.integers(0, m.N))
        ch = cf.ComplexChain(m, f.copy())
        ch.G = stable.green_scratch(m, ch.field, tau)
        ch.trace = []
        old = ch.field.copy()
        acc = ch._propose(tau, i, 0.0, float(rng.random()))
        assert acc
        R = ch.trace[-1][3]
        want = np.exp(cf.log_weight_complex(m, ch.field) - cf.log_weight_complex(m, old))
        assert abs(R - want) < 1e-10 * abs(want)
        assert np.max(np.abs(ch.G - stable.green_scratch(m, ch.field, tau))) < 1e-11
        assert abs(ch.phase - 1.0) < 1e-12


def test_complex_chain_samples_the_weight():
    """2 sites x 2 slices: the visited configurations follow |W(C)| / Z (chi^2),
    and not the weights with gamma(l) left out (alpha only enters |W| through
    a phase here, which the phase pins above cover)."""
    K = np.array([[0.0, -1.0], [-1.0, 0.0]])
    m = cf.complex_model(K, 4.0, 0.5, 0.25, 2, seed=17)
    fields = list(_all_fields(m))
    w = np.array([abs(np.exp(cf.log_weight_complex(m, f))) for f in fields])
    p = w / w.sum()
    index = {tuple(f.ravel()): j for j, f in enumerate(fields)}
    ch = cf.ComplexChain(m, cf.init_field(m)).init()
    counts = np.zeros(p.size)
    n = 6000
    for _ in range(n):
        ch.sweep(measure=False)
        counts[index[tuple(ch.field.ravel())]] += 1
    chi2 = np.sum((counts - n * p) ** 2 / (n * p)) / (p.size - 1)
    assert chi2 < 2.0
    assert ch.phase_dev < 1e-12
    m2 = cf.complex_model(K, 4.0, 0.5, 0.25, 2)
    m2.vertex_log_factor = lambda fs: np.zeros_like(np.asarray(fs, dtype=float))
    w2 = np.array([abs(np.exp(cf.log_weight_complex(m2, f))) for f in fields])
    p2 = w2 / w2.sum()
    chi2_wrong = np.sum((counts - n * p2) ** 2 / (n * p2)) / (p.size - 1)
    assert chi2_wrong > 5.0
