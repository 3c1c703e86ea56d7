"""Pins of the oracle's two-flavour M_z form (section "The M_z-Hubbard model
on a square lattice", Eq. (hubbard_Mz); N_fl = 2, two Green's functions,
flavour-dependent hopping) and of its sign (section "The sign problem").

The decoupling of (U/2)(n - 1)^2 through the magnetisation is exact at any
filling, so an enumeration of every field configuration, each weighted by
its signed weight, must reproduce the Fock-space Trotter product of the
Hubbard model with the two flavours' hopping matrices (tests/fock.py); on a
frustrated ring with a chemical potential some weights are negative, and
only the sign-weighted average agrees.  Planted mistakes (the down flavour
coupled with the up flavour's sign, the sign dropped) fail these."""
import itertools

import numpy as np
import pytest

from fock import Fock
from oracle import hubbard
from oracle import mz_flavours as mz


def _pair(mu, t_up, t_dn):
    K_up = np.array([[-mu, -t_up], [-t_up, -mu]])
    K_dn = np.array([[-mu, -t_dn], [-t_dn, -mu]])
    return K_up, K_dn


def _ring(n, t, mu):
    K = -mu * np.eye(n)
    for i in range(n):
        K[i, (i + 1) % n] = K[(i + 1) % n, i] = -t
    return K


def _fields(mm):
    for vals in itertools.product([-1.0, 1.0], repeat=mm.L * mm.N):
        yield np.array(vals).reshape(mm.L, mm.N)


def _enumerate(mm, taus, signed=True):
    """Sign-weighted averages of (D, E_kin, E_pot) at the given slices over all
    fields (|W| instead of W when `signed` is False)."""
    ws, obs = [], []
    for f in _fields(mm):
        s, lw = mz.log_weight_signed(mm, f)
        ws.append((s if signed else 1.0) * np.exp(lw))
        obs.append([mz.equal_time_mz(mm, mz.green_scratch_mz(mm, f, t)) for t in taus])
    ws = np.array(ws)
    return np.einsum("c,ctk->tk", ws, np.array(obs)) / ws.sum()


def _fock(K_up, K_dn, U, dtau, L, trotter):
    F = Fock(K_up, U, K_dn=K_dn)
    S = F.trotter(dtau) if trotter == "sym" else F.trotter_asym(dtau)
    return np.array([F.expect_with(S, O, L) for O in (F.double_occ(), F.kinetic(), F.potential())])


def test_signed_weight_equals_naive_determinants():
    """The stabilised signed log-weight equals the product of the two plain
    determinants on a ring where some weights are negative."""
    mm = mz.MzModel(_ring(3, 1.0, 1.5), _ring(3, 0.4, 1.5), 8.0, 1.5, 0.5, 1)
    neg = 0
    for f in _fields(mm):
        s, lw = mz.log_weight_signed(mm, f)
        W = np.exp(np.sum(mm.vertex_log_factor(f)))
        for m in mm.fl:
            W *= np.linalg.det(np.eye(3) + hubbard.product_B(m, f, mm.L, 0))
        assert abs(W - s * np.exp(lw)) < 1e-10 * abs(W)
        neg += s < 0
    assert neg > 0


@pytest.mark.parametrize("trotter", ["sym", "asym"])
def test_two_flavour_enumeration_equals_fock(trotter):
    """2 sites x 2 slices, chemical potential 0.3, t_up = 1, t_dn = 0.6: the
    averages of D, E_kin, E_pot at both slices equal the Fock-space Trotter
    product of the Hubbard model with the two hopping matrices (1e-12)."""
    K_up, K_dn = _pair(0.3, 1.0, 0.6)
    U, dtau, L = 4.0, 0.25, 2
    mm = mz.MzModel(K_up, K_dn, U, L * dtau, dtau, 1, trotter=trotter)
    got = _enumerate(mm, (0, 1))
    want = _fock(K_up, K_dn, U, dtau, L, trotter)
    assert np.max(np.abs(got - want[None, :])) < 1e-12


def test_sign_problem_needs_the_sign():
    """3-site ring, chemical potential 1.5, t_up = 1, t_dn = 0.4, U = 8, three
    slices: some weights are negative; the sign-weighted averages equal Fock
    space, the |W| averages do not."""
    K_up, K_dn = _ring(3, 1.0, 1.5), _ring(3, 0.4, 1.5)
    U, dtau, L = 8.0, 0.5, 3
    mm = mz.MzModel(K_up, K_dn, U, L * dtau, dtau, 1, trotter="asym")
    want = _fock(K_up, K_dn, U, dtau, L, "asym")
    got = _enumerate(mm, (0,))[0]
    assert np.max(np.abs(got - want)) < 1e-11
    wrong = _enumerate(mm, (0,), signed=False)[0]
    assert np.max(np.abs(wrong - want)) > 1e-4


def test_down_flavour_coupling_sign_is_pinned():
    """Coupling the down flavour with +lambda (as the up flavour) leaves Fock
    space."""
    K_up, K_dn = _pair(0.3, 1.0, 0.6)
    U, dtau, L = 4.0, 0.25, 2
    mm = mz.MzModel(K_up, K_dn, U, L * dtau, dtau, 1, trotter="sym")
    mm.fl[1] = hubbard.Model(K=K_dn, beta=L * dtau, dtau=dtau, n_wrap=1, coupling=mm.coupling, U=U, alpha=0.0,
                             n_col=1, trotter="sym")
    got = _enumerate(mm, (0,))[0]
    want = _fock(K_up, K_dn, U, dtau, L, "sym")
    assert np.max(np.abs(got - want)) > 1e-3


@pytest.fixture(scope="module")
def ring4():
    mm = mz.MzModel(_ring(4, 1.0, 0.7), _ring(4, 0.5, 0.7), 6.0, 1.0, 0.1, 5, seed=3)
    return mm, mz.init_field(mm)


def test_stable_green_equals_naive_inverse(ring4):
    mm, f = ring4
    for tau in (0, 3, 7, 10):
        for m, G in zip(mm.fl, mz.green_scratch_mz(mm, f, tau)):
            A = hubbard.product_B(m, f, tau, 0) @ hubbard.product_B(m, f, mm.L, tau)
            assert np.max(np.abs(G - np.linalg.inv(np.eye(mm.N) + A))) < 1e-12


def test_fast_ratio_and_updates_equal_scratch(ring4):
    """The chain's R (product of the two flavours' ratios) equals the ratio of
    the from-scratch signed weights; both updated G's equal their scratch G."""
    mm, f = ring4
    rng = np.random.default_rng(4)
    for _ in range(6):
        tau = int(rng.integers(1, mm.L + 1))
        i = int(rng.integers(0, mm.N))
        ch = mz.MzChain(mm, f.copy())
        ch.G = mz.green_scratch_mz(mm, ch.field, tau)
        ch.trace = []
        old = ch.field.copy()
        assert ch._propose(tau, i, 0.0, float(rng.random()))
        R = ch.trace[-1][3]
        s0, l0 = mz.log_weight_signed(mm, old)
        s1, l1 = mz.log_weight_signed(mm, ch.field)
        want = s0 * s1 * np.exp(l1 - l0)
        assert abs(R - want) < 1e-10 * abs(want)
        for G, Gs in zip(ch.G, mz.green_scratch_mz(mm, ch.field, tau)):
            assert np.max(np.abs(G - Gs)) < 1e-11


def test_chain_samples_abs_weight():
    """2 sites x 2 slices with two hopping matrices: the visited fields follow
    |W| / sum |W| (chi^2); the down flavour coupled with +lambda fails it."""
    K_up, K_dn = _pair(0.3, 1.0, 0.6)
    mm = mz.MzModel(K_up, K_dn, 4.0, 0.5, 0.25, 2, trotter="sym", seed=21)
    fields = list(_fields(mm))
    p = np.array([np.exp(mz.log_weight_signed(mm, f)[1]) for f in fields])
    p /= p.sum()
    index = {tuple(f.ravel()): j for j, f in enumerate(fields)}
    ch = mz.MzChain(mm, mz.init_field(mm)).init()
    counts = np.zeros(p.size)
    n = 6000
    for _ in range(n):
        ch.sweep(measure=False)
        counts[index[tuple(ch.field.ravel())]] += 1
    assert np.sum((counts - n * p) ** 2 / (n * p)) / (p.size - 1) < 2.0
    mw = mz.MzModel(K_up, K_dn, 4.0, 0.5, 0.25, 2)
    mw.fl[1] = hubbard.Model(K=K_dn, beta=0.5, dtau=0.25, n_wrap=2, coupling=mw.coupling, U=4.0, alpha=0.0,
                             n_col=1, trotter="sym")
    q = np.array([np.exp(mz.log_weight_signed(mw, f)[1]) for f in fields])
    q /= q.sum()
    assert np.sum((counts - n * q) ** 2 / (n * q)) / (q.size - 1) > 5.0


def test_chain_carries_the_sign():
    """3-site ring with negative weights, three slices: the carried sign
    (relative to the starting field) equals the sign of the weight recomputed
    from scratch, and negative configurations are visited."""
    K_up, K_dn = _ring(3, 1.0, 1.5), _ring(3, 0.4, 1.5)
    mm = mz.MzModel(K_up, K_dn, 8.0, 1.5, 0.5, 1, trotter="asym", seed=9)
    ch = mz.MzChain(mm, mz.init_field(mm)).init()
    s0 = mz.log_weight_signed(mm, ch.field)[0]
    seen_negative = False
    for k in range(3000):
        ch.sweep(measure=False)
        if k % 10 == 0 or ch.sign * s0 < 0:
            assert ch.sign * s0 == mz.log_weight_signed(mm, ch.field)[0]
        seen_negative = seen_negative or ch.sign * s0 < 0
    assert seen_negative
