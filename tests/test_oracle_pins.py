"""Pins of the oracle against facts that do not come from the oracle itself.

Each test fixes a part of the oracle with something independent: a published
generator, a closed form, an exact enumeration against a Fock-space Trotter
product, a matrix identity, or a 60-digit mpmath evaluation.  A plausible
mistake (a dropped prefactor, a wrong sign of alpha, a transposed product, a
wrong rotation of the measured G, a wrong chunk in the stabilisation) fails at
least one of them.
"""
import itertools

import numpy as np
import pytest

from fock import Fock
from inputs import square_lattice, honeycomb_lattice
from oracle import exact_small, hubbard, measure, philox, stable, sweep


# ---------------------------------------------------------------- generator --
@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)), ((12345, 0), (7, 3, 41, 5)),
                                     ((2**64 - 1, 17), (1, 2**63, 2**40 + 3, 99))])
def test_philox_matches_numpy(key, ctr):
    # numpy's Philox increments its 256-bit counter before producing a block
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
    raw = [int(x) for x in bg.random_raw(8)]
    c1 = list(ctr)
    c1[0] = (c1[0] + 1) % 2**64
    assert list(philox.philox4x64_10(c1, key)) == raw[:4]
    c2 = list(c1)
    c2[0] += 1
    assert list(philox.philox4x64_10(c2, key)) == raw[4:]
    v = philox.philox4x64_10_vec(*[np.array([c], dtype=np.uint64) for c in c1], key)
    assert [int(x[0]) for x in v] == raw[:4]


def test_uniform_and_normal_ranges():
    u = philox.uniforms(3, philox.TAG_FLIP, 5, 7, 1, 4096)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.02
    z = philox.normals(3, philox.TAG_INIT, 0, 1, 0, 20000)
    assert abs(z.mean()) < 0.05 and abs(z.std() - 1.0) < 0.05


# ----------------------------------------------------------- HS identities --
@pytest.mark.parametrize("U,dtau", [(4.0, 0.1), (5.0, 0.1), (8.0, 0.05)])
def test_hs_identities(U, dtau):
    lam = hubbard.ising_coupling(U, dtau)
    for n in (0, 1, 2):
        lhs = np.exp(dtau * U / 2 * (n - 1) ** 2)
        rhs = 0.5 * sum(np.exp(lam * s * (n - 1)) for s in (1, -1))
        assert abs(lhs - rhs) < 1e-14 * lhs
    c = hubbard.gauss_coupling(U, dtau)
    x, w = np.polynomial.hermite_e.hermegauss(80)      # weight exp(-x^2/2)
    for A in (-1.0, 0.0, 1.0, 2.0):
        quad = np.sum(w * np.exp(c * x * A)) / np.sqrt(2 * np.pi)
        assert abs(quad - np.exp(dtau * U / 2 * A * A)) < 1e-13


def test_hs4_identity_is_eighth_order():
    """Eq. (HS_squares): 1/4 sum_l gamma(l) exp(x eta(l)) = exp(x^2) + O(x^8)
    (the paper's O(dtau^4)): the moments sum_l gamma eta^(2k) are 4, 8, 48, 480
    = 4 (2k)! / k!, so the series agrees through x^6, and halving x shrinks the
    error by 2^8."""
    g, e = np.array(hubbard.GAMMA4), np.array(hubbard.ETA4)
    for k, want in enumerate((4.0, 8.0, 48.0, 480.0)):
        assert abs(np.sum(g * e ** (2 * k)) - want) < 1e-12 * want
    assert abs(np.sum(g * e)) < 1e-14 and abs(np.sum(g * e ** 3)) < 1e-12
    err = [0.25 * np.sum(g * np.exp(x * e)) - np.exp(x * x) for x in (0.2, 0.1, 0.05)]
    assert abs(err[0]) < 1e-7
    for a, b in zip(err, err[1:]):
        assert 240.0 < a / b < 275.0


def test_two_site_enumeration_ising4_equals_fock_at_u_eff():
    """With A = n - 1 in {-1, 0, 1}, the four-valued sum of Eq. (HS_squares) is
    exactly exp(dtau U_eff / 2 A^2) with exp(dtau U_eff / 2) = 1/2 (gamma_1
    cosh(c4 eta_1) + gamma_2 cosh(c4 eta_2)); the enumeration over all 4^(N L)
    configurations must reproduce the Fock-space Trotter product at U_eff."""
    K = np.array([[0.0, -1.0], [-1.0, 0.0]])
    U, dtau, L = 4.0, 0.25, 3
    m = hubbard.hubbard_model(K, U, L * dtau, dtau, 3, field_kind="ising4")
    res = exact_small.enumerate_observables(m, taus=(0, 1))
    g, e = hubbard.GAMMA4, hubbard.ETA4
    F1 = 0.5 * (g[2] * np.cosh(m.coupling * e[2]) + g[3] * np.cosh(m.coupling * e[3]))
    U_eff = 2.0 * np.log(F1) / dtau
    assert abs(U_eff - U) < 1e-2 and U_eff != U       # next to exact (dtau^4), not exact
    F = Fock(K, U_eff)
    S = F.trotter(dtau)
    D = F.expect_with(S, F.double_occ(), L)
    E = F.expect_with(S, F.kinetic(), L)
    assert np.max(np.abs(res[:, 0] - D)) < 1e-13
    assert np.max(np.abs(res[:, 1] - E)) < 1e-13
    # a planted mistake (gamma left out of the weight) breaks it
    g_saved = hubbard.GAMMA4
    try:
        hubbard.GAMMA4 = (1.0, 1.0, 1.0, 1.0)
        bad = exact_small.enumerate_observables(m, taus=(0,))
    finally:
        hubbard.GAMMA4 = g_saved
    assert abs(bad[0, 0] - D) > 1e-3


# -------------------------------------------------------- U = 0 closed form --
def _square_u0_green(L1, L2, beta):
    """(1 + exp(-beta K))^-1 on the square lattice from plane waves and the
    dispersion eps_k = -2 (cos kx + cos ky), not from an eigensolver."""
    n = L1 * L2
    xs = np.array([(i % L1, i // L1) for i in range(n)], dtype=float)
    G = np.zeros((n, n), dtype=complex)
    ekin = 0.0
    for a in range(L1):
        for b in range(L2):
            k = np.array([2 * np.pi * a / L1, 2 * np.pi * b / L2])
            eps = -2.0 * (np.cos(k[0]) + np.cos(k[1]))
            ph = np.exp(1j * xs @ k)
            occ_hole = 1.0 / (1.0 + np.exp(-beta * eps))      # 1 - f(eps)
            G += np.outer(ph, ph.conj()) * occ_hole / n
            ekin += 2.0 * eps / (np.exp(beta * eps) + 1.0) / n
    return G.real, ekin


@pytest.mark.parametrize("beta,trotter", [(2.0, "sym"), (40.0, "asym"), (40.0, "sym")])
def test_u0_closed_form(beta, trotter):
    lat = square_lattice(4, 4)
    m = hubbard.hubbard_model(lat.K, 0.0, beta, 0.1, 10, trotter=trotter)
    f = hubbard.init_field(m)
    G0, ekin0 = _square_u0_green(4, 4, beta)
    for tau in (0, 3, 10, m.L // 2 + 7, m.L):
        G = stable.green_scratch(m, f, tau)
        assert np.max(np.abs(G - G0)) < 1e-12
        D, ekin, _ = measure.equal_time(m, G)
        assert abs(ekin - ekin0) < 1e-12


# ------------------------------------------------------------ atomic limit --
def test_atomic_limit_double_occupancy():
    """t = 0: D = 1 / (2 (1 + exp(beta U / 2))) exactly, for any dtau."""
    U, beta = 4.0, 2.0
    m = hubbard.hubbard_model(np.zeros((1, 1)), U, beta, beta / 8, 4)
    res = exact_small.enumerate_observables(m, taus=(0, 5))
    exact = 1.0 / (2.0 * (1.0 + np.exp(beta * U / 2)))
    assert abs(exact - 0.0089931) < 1e-7
    assert np.max(np.abs(res[:, 0] - exact)) < 1e-14
    assert np.max(np.abs(res[:, 2] - U * exact)) < 1e-13


# ------------------------------------------------- 2 sites x 4 slices exact --
@pytest.mark.parametrize("trotter", ["sym", "asym"])
def test_two_site_enumeration_equals_fock_trotter(trotter):
    K = np.array([[0.0, -1.0], [-1.0, 0.0]])
    U, dtau, L = 4.0, 0.25, 4
    m = hubbard.hubbard_model(K, U, L * dtau, dtau, 2, trotter=trotter)
    res = exact_small.enumerate_observables(m, taus=(0, 1, 2, 3))
    F = Fock(K, U)
    S = F.trotter(dtau) if trotter == "sym" else F.trotter_asym(dtau)
    D = F.expect_with(S, F.double_occ(), L)
    E = F.expect_with(S, F.kinetic(), L)
    assert np.max(np.abs(res[:, 0] - D)) < 1e-13
    assert np.max(np.abs(res[:, 1] - E)) < 1e-13


@pytest.mark.parametrize("trotter", ["sym", "asym"])
def test_mz_zeeman_field_enumeration_equals_fock(trotter):
    """The M_z form with a Zeeman field h (flavour hopping T -+ h): the oracle
    in the density frame with K = T - h (one Green's function for both
    flavours) against the Fock-space Trotter product of the original-frame
    Hamiltonian with the field.  Double occupancy, and the frame's kinetic
    energy per site plus h (the constant of the particle-hole map) equal to
    <H_T>/N; the field polarises (<n_up - n_dn> = 1 - 2 G_ii per site, here
    compared with Fock space too)."""
    from oracle.measure import measured_green
    from oracle.stable import green_scratch, log_weight
    K = np.array([[0.0, -1.0], [-1.0, 0.0]])
    U, dtau, L, h = 4.0, 0.25, 4, 0.7
    sign = np.array([1.0, -1.0])
    Kf = hubbard.mz_frame_hopping(K, h, sign)
    m = hubbard.hubbard_model(Kf, U, L * dtau, dtau, 2, trotter=trotter)
    res = exact_small.enumerate_observables(m, taus=(0, 1, 2, 3))
    F = Fock(K, U, h)
    S = F.trotter(dtau) if trotter == "sym" else F.trotter_asym(dtau)
    D = F.expect_with(S, F.double_occ(), L)
    E = F.expect_with(S, F.kinetic(), L)
    assert np.max(np.abs(res[:, 0] - D)) < 1e-13
    assert np.max(np.abs(res[:, 1] + h - E)) < 1e-13
    # magnetisation per site
    mz_fock = F.expect_with(S, sum(F.n[i][0] - F.n[i][1] for i in range(2)) / 2, L)
    logw, mz = [], []
    for f in exact_small.all_fields(m):
        logw.append(log_weight(m, f))
        mz.append(np.mean(1.0 - 2.0 * np.diag(measured_green(m, green_scratch(m, f, 1)))))
    w = np.exp(np.array(logw) - max(logw))
    assert abs(np.dot(w, mz) / w.sum() - mz_fock) < 1e-13
    assert mz_fock > 0.05
    # a chemical potential makes the flavours differ in this frame: refused
    with pytest.raises(ValueError):
        hubbard.mz_frame_hopping(K - 0.3 * np.eye(2), h, sign)


def test_two_site_enumeration_detects_wrong_alpha():
    """Planted mistake on the CPU: flipping the sign of alpha moves D away
    from the Fock-space value, so the pin above is sensitive to it."""
    K = np.array([[0.0, -1.0], [-1.0, 0.0]])
    U, dtau, L = 4.0, 0.25, 4
    m = hubbard.hubbard_model(K, U, L * dtau, dtau, 2)
    m.alpha = +0.5
    res = exact_small.enumerate_observables(m, taus=(0,))
    F = Fock(K, U)
    D = F.expect(F.double_occ(), dtau, L)
    assert abs(res[0, 0] - D) > 1e-3


# ---------------------------------------------------------------- invariants --
@pytest.fixture(scope="module")
def c1_like():
    lat = square_lattice(4, 4)
    m = hubbard.hubbard_model(lat.K, 4.0, 2.0, 0.1, 10, seed=0)
    return m, hubbard.init_field(m)


def test_sm_ratio_equals_determinant_ratio(c1_like):
    m, f = c1_like
    rng = np.random.default_rng(1)
    for _ in range(6):
        tau = int(rng.integers(1, m.L + 1))
        i = int(rng.integers(0, m.N))
        G = stable.green_scratch(m, f, tau)
        s = f[tau - 1, i]
        delta = np.exp(m.coupling * (-2 * s)) - 1.0
        r = 1.0 + delta * (1.0 - G[i, i])
        R = np.exp(m.n_col * m.coupling * m.alpha * (-2 * s)) * r ** m.n_col
        R_full = stable.weight_ratio(m, f, tau, i, -s)
        assert abs(R - R_full) < 1e-11 * max(1.0, abs(R_full))


def test_sm_update_equals_scratch(c1_like):
    m, f = c1_like
    ch = sweep.Chain(m, f.copy())
    tau, i = 7, 5
    ch.G = stable.green_scratch(m, ch.field, tau)
    assert ch._propose(tau, i, u=0.0, u1=0.0)        # u = 0 always accepts
    assert np.max(np.abs(ch.G - stable.green_scratch(m, ch.field, tau))) < 1e-12


def test_wrap_equals_scratch(c1_like):
    m, f = c1_like
    for tau in (1, 5, 11, 20):
        Gm = stable.green_scratch(m, f, tau - 1)
        Gw = m.B(f, tau) @ Gm @ m.B_inv(f, tau)
        assert np.max(np.abs(Gw - stable.green_scratch(m, f, tau))) < 1e-11
        Gd = m.B_inv(f, tau) @ stable.green_scratch(m, f, tau) @ m.B(f, tau)
        assert np.max(np.abs(Gd - Gm)) < 1e-11


def test_green_scratch_independent_of_n_wrap(c1_like):
    m, f = c1_like
    m5 = hubbard.hubbard_model(m.K, 4.0, 2.0, 0.1, 5, seed=0)
    for tau in (0, 4, 13):
        assert np.max(np.abs(stable.green_scratch(m, f, tau) - stable.green_scratch(m5, f, tau))) < 1e-12


def test_stable_green_vs_mpmath():
    """beta = 12, L = 120 on a 2x2 square: cond(1 + B) ~ 1e13; the stabilised
    G agrees with a 60-digit evaluation, the plain inverse does not."""
    import mpmath as mp
    mp.mp.dps = 60
    lat = square_lattice(2, 2)
    m = hubbard.hubbard_model(lat.K, 4.0, 12.0, 0.1, 10, seed=4)
    f = hubbard.init_field(m)
    E = mp.expm(mp.matrix((-m.dtau * lat.K).tolist()))
    lam = mp.acosh(mp.e ** (mp.mpf(m.dtau) * 4 / 2))
    P = mp.eye(m.N)
    for tau in range(1, m.L + 1):
        Dg = mp.diag([mp.e ** (lam * int(s)) for s in f[tau - 1]])
        P = Dg * E * P
    Gmp = (mp.eye(m.N) + P) ** -1
    Gref = np.array(Gmp.tolist(), dtype=float)
    G = stable.green_scratch(m, f, 0)
    assert np.max(np.abs(G - Gref)) < 1e-10
    lin = np.abs(np.linalg.slogdet(np.eye(m.N) + np.array(P.tolist(), dtype=float))[1])
    assert abs(stable.logdet_scratch(m, f) - float(mp.log(abs(mp.det(mp.eye(m.N) + P))))) < 1e-9 * lin


def test_sweep_precision_and_scratch(c1_like):
    m, f = c1_like
    ch = sweep.Chain(m, f.copy()).init()
    for _ in range(3):
        ch.sweep()
    assert np.mean(ch.prec) < 1e-8         # the paper's recommended mean precision
    assert np.max(np.abs(ch.G - stable.green_scratch(m, ch.field, 0))) < 1e-10
    d = ch.bins / ch.bins[3]
    assert 0.0 < d[0] < 0.25 and d[1] < 0


def test_half_filling_density(c1_like):
    m, f = c1_like
    for tau in (0, 9):
        G = stable.green_scratch(m, f, tau)
        # particle-hole symmetry of the sampling frame at mu = 0 is a property of
        # the ensemble, not of one field; check only the range here
        n = measure.density(m, G)
        assert 0.0 < n < 2.0


# ------------------------------------------------------------ MC sampler --
def test_mc_histogram_matches_exact_weights():
    """Stationarity of the sequential single-flip chain (section "The default:
    sequential single spin flips"): the visited configurations of a 2-site x
    4-slice chain follow W(C)/Z."""
    K = np.array([[0.0, -1.0], [-1.0, 0.0]])
    m = hubbard.hubbard_model(K, 4.0, 1.0, 0.25, 2, seed=11)
    p = exact_small.enumerate_weights(m)
    index = {tuple(fl.ravel()): j for j, fl in enumerate(exact_small.all_fields(m))}
    ch = sweep.Chain(m, hubbard.init_field(m)).init()
    counts = np.zeros(p.size)
    n_sweeps = 4000
    for _ in range(n_sweeps):
        ch.sweep(measure=False)
        counts[index[tuple(ch.field.ravel())]] += 1
    # chi^2 per degree of freedom; successive sweeps are mildly correlated, so
    # allow a factor of ~2 over the independent-sample value of 1
    chi2 = np.sum((counts - n_sweeps * p) ** 2 / (n_sweeps * p)) / (p.size - 1)
    assert chi2 < 2.0
    # the same counts against a planted wrong weight (sign of alpha) fail clearly
    m2 = hubbard.hubbard_model(K, 4.0, 1.0, 0.25, 2)
    m2.alpha = 0.5
    p2 = exact_small.enumerate_weights(m2)
    chi2_wrong = np.sum((counts - n_sweeps * p2) ** 2 / (n_sweeps * p2)) / (p.size - 1)
    assert chi2_wrong > 5.0


def test_mc_histogram_ising4_matches_exact_weights():
    """The same stationarity check for the four-valued field: the three-way
    proposal of the other values is symmetric, so the chain must visit the
    4^(N L) configurations of 2 sites x 2 slices with frequency W(C)/Z."""
    K = np.array([[0.0, -1.0], [-1.0, 0.0]])
    m = hubbard.hubbard_model(K, 4.0, 0.5, 0.25, 2, field_kind="ising4", seed=13)
    p = exact_small.enumerate_weights(m)
    index = {tuple(fl.ravel()): j for j, fl in enumerate(exact_small.all_fields(m))}
    ch = sweep.Chain(m, hubbard.init_field(m)).init()
    counts = np.zeros(p.size)
    n_sweeps = 6000
    for _ in range(n_sweeps):
        ch.sweep(measure=False)
        counts[index[tuple(ch.field.ravel())]] += 1
    chi2 = np.sum((counts - n_sweeps * p) ** 2 / (n_sweeps * p)) / (p.size - 1)
    assert chi2 < 2.0
    g_saved = hubbard.GAMMA4
    try:
        hubbard.GAMMA4 = (1.0, 1.0, 1.0, 1.0)
        p2 = exact_small.enumerate_weights(m)
    finally:
        hubbard.GAMMA4 = g_saved
    chi2_wrong = np.sum((counts - n_sweeps * p2) ** 2 / (n_sweeps * p2)) / (p.size - 1)
    assert chi2_wrong > 5.0


# --------------------------------------------------------------- jackknife --
def test_jackknife_reduces_to_mean_and_stderr():
    x = np.random.default_rng(0).normal(size=37)
    mean, err = measure.jackknife(x)
    assert abs(mean - x.mean()) < 1e-14
    assert abs(err - x.std(ddof=1) / np.sqrt(x.size)) < 1e-14


# ---------------------------------------------------------------- lattices --
def test_honeycomb_lattice_structure():
    lat = honeycomb_lattice(3, 3)
    K = lat.K
    assert np.allclose(K, K.T)
    assert np.all(np.sum(K != 0, axis=1) == 3)            # coordination 3
    s = lat.sublattice_sign()
    assert np.all(K * np.outer(s, s) >= 0)                 # hops only between sublattices
    w = np.linalg.eigvalsh(K)
    assert abs(w.min() + 3.0) < 1e-12 and abs(w.max() - 3.0) < 1e-12


# ------------------------------------------------------------------ golden --
def test_oracle_golden_trajectory():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "square4x4_U4_b2_3sweeps.json")
    g = json.load(open(path))
    lat = square_lattice(4, 4)
    m = hubbard.hubbard_model(lat.K, 4.0, 2.0, 0.1, 10, trotter="sym", seed=0)
    ch = sweep.Chain(m, hubbard.init_field(m)).init()
    for _ in range(3):
        ch.sweep()
    assert ch.accepted == g["accepted"] and ch.proposals == g["proposals"]
    assert np.array_equal(ch.field.astype(int), np.array(g["field"]))
    assert np.max(np.abs(ch.G - np.array(g["G0"]))) < 1e-12
    assert np.max(np.abs(ch.bins - np.array(g["bins"]))) < 1e-10


# ------------------------------------------------------------- gradient --
def test_gradient_matches_finite_differences():
    """d log det / d phi = c (1 - G(tau)_ii) against central differences
    (h = 1e-5) of the stabilised log det on a 3x3 square with a Gaussian field."""
    from oracle import gradient
    lat = square_lattice(3, 3)
    m = hubbard.hubbard_model(lat.K, 4.0, 2.0, 0.1, 5, field_kind="gauss", seed=3)
    f = hubbard.init_field(m)
    g = gradient.grad_logdet(m, f)
    rng = np.random.default_rng(0)
    for _ in range(8):
        tau = int(rng.integers(1, m.L + 1))
        i = int(rng.integers(0, m.N))
        fd = gradient.fd_logdet(m, f, tau, i)
        assert abs(fd - g[tau - 1, i]) < 1e-7 * max(1.0, abs(g[tau - 1, i]))


def test_gradient_atomic_closed_form():
    """t = 0, one site: det(1 + B) = 1 + exp(c sum_tau phi_tau), so the
    gradient is c e^x / (1 + e^x) for every slice (x = c sum phi)."""
    from oracle import gradient
    m = hubbard.hubbard_model(np.zeros((1, 1)), 4.0, 1.0, 0.1, 5, field_kind="gauss", seed=1)
    f = hubbard.init_field(m)
    x = m.coupling * f.sum()
    g = gradient.grad_logdet(m, f)
    assert np.max(np.abs(g - m.coupling * np.exp(x) / (1 + np.exp(x)))) < 1e-13


def test_langevin_step_is_the_stated_update():
    from oracle import gradient, philox
    lat = square_lattice(2, 2)
    m = hubbard.hubbard_model(lat.K, 4.0, 1.0, 0.1, 5, field_kind="gauss", seed=5)
    f = hubbard.init_field(m)
    new = gradient.langevin_step(m, f, 1e-3, 7)
    xi = philox.normals(5, philox.TAG_LANGEVIN, 7, 3, 0, m.N)
    dlw = gradient.grad_log_weight(m, f)
    assert np.max(np.abs(new[2] - (f[2] + 1e-3 * dlw[2] + np.sqrt(2e-3) * xi))) < 1e-15


# ------------------------------------------------------ time-displaced G --
def _td_model(trotter="sym", beta=1.0, seed=4):
    lat = square_lattice(3, 3)
    m = hubbard.hubbard_model(lat.K, 4.0, beta, 0.1, 5, trotter=trotter, seed=seed)
    return lat, m, hubbard.init_field(m)


def test_tdgf_stable_forms_equal_definitions():
    """The stabilised GT0 / G0T / GTT against B'(tau,0) G(0),
    -(1 - G(0)) B'(tau,0)^-1 and the plain inverse, on a well conditioned case."""
    from oracle import timedisplaced as td
    lat, m, f = _td_model()
    for tau in (0, 1, 4, 5, 7, 10):
        a = td.tdgf_scratch(m, f, tau)
        b = td.tdgf_naive(m, f, tau)
        for x, y in zip(a, b):
            assert np.max(np.abs(x - y)) < 1e-11


def test_tdgf_boundaries():
    """GT0(0) = G(0), G0T(0) = G(0) - 1, GT0(beta) = 1 - G(0), G0T(beta) = -G(0)."""
    from oracle import timedisplaced as td
    lat, m, f = _td_model(beta=4.0)
    G0 = stable.green_scratch(m, f, 0)
    I = np.eye(m.N)
    GT0, G0T, GTT = td.tdgf_scratch(m, f, 0)
    assert np.max(np.abs(GT0 - G0)) < 1e-12 and np.max(np.abs(G0T - (G0 - I))) < 1e-12
    GT0, G0T, GTT = td.tdgf_scratch(m, f, m.L)
    assert np.max(np.abs(GT0 - (I - G0))) < 1e-10 and np.max(np.abs(G0T + G0)) < 1e-10
    assert np.max(np.abs(GTT - G0)) < 1e-10


@pytest.mark.parametrize("trotter", ["sym", "asym"])
def test_total_sz_correlation_is_conserved(trotter):
    """S^z_tot commutes with every slice propagator, so for one configuration
    sum_ab S_ab(K = 0, tau) does not depend on tau."""
    from oracle import timedisplaced as td
    lat = honeycomb_lattice(2, 2)
    m = hubbard.hubbard_model(lat.K, 4.0, 2.0, 0.1, 5, trotter=trotter, seed=9)
    f = hubbard.init_field(m)
    S = td.tdgf_measure(m, lat, np.zeros(2), f, taus=(0, 3, 10, 11, 20))
    tot = S.sum(axis=(1, 2))
    assert np.max(np.abs(tot - tot[0])) < 1e-10
    assert abs(tot[0].imag) < 1e-12


@pytest.mark.parametrize("trotter", ["sym", "asym"])
def test_szsz_enumeration_equals_fock(trotter):
    """4-site honeycomb ring (2 cells x 2 orbitals) x 2 slices: the exact
    weighted average of the time-displaced estimator at K = g2/2 against
    Tr(S^(L-n) S^z_x S^n S^z_y) / Tr(S^L) in Fock space, Fourier transformed."""
    from oracle import exact_small
    lat = honeycomb_lattice(1, 2)
    U, dtau, L = 4.0, 0.25, 2
    m = hubbard.hubbard_model(lat.K, U, L * dtau, dtau, 1, trotter=trotter)
    g1, g2 = lat.reciprocal()
    kvec = 0.5 * g2
    got = exact_small.enumerate_szsz(m, lat, kvec, taus=(0, 1, 2))
    F = Fock(lat.K, U)
    S = F.trotter(dtau) if trotter == "sym" else F.trotter_asym(dtau)
    R = lat.cell_pos[lat.cell_of]
    ph = np.exp(-1j * (R @ kvec))
    for t, n in enumerate((0, 1, 2)):
        want = np.zeros((2, 2), dtype=complex)
        for x in range(4):
            for y in range(4):
                c = F.expect_tau_with(S, F.sz(x), F.sz(y), L, n)
                want[lat.orb_of[x], lat.orb_of[y]] += ph[x] * np.conj(ph[y]) * c
        want /= lat.n_cells
        assert np.max(np.abs(got[t] - want)) < 1e-12, (trotter, n, got[t], want)


@pytest.mark.parametrize("trotter,h", [("sym", 0.0), ("asym", 0.0), ("sym", 0.6), ("asym", 0.6)])
def test_eq_correlations_enumeration_equals_fock(trotter, h):
    """Lattice-resolved equal-time correlations (Green, SpinZ, SpinXY, Den by
    displacement and orbital pair) of a 4-site honeycomb ring (2 cells x 2
    orbitals) x 2 slices: the exact weighted average of the per-configuration
    estimators against Tr(S^L O_ij) / Tr(S^L) in Fock space, with O_ij built
    from the original-frame fermions (no particle-hole map); h > 0 adds the
    M_z form's Zeeman field (frame hopping K = T - h)."""
    from oracle import exact_small, measure
    from oracle.stable import green_scratch, log_weight
    lat = honeycomb_lattice(1, 2)
    U, dtau, L = 4.0, 0.25, 2
    K = hubbard.mz_frame_hopping(lat.K, h, lat.sublattice_sign())
    m = hubbard.hubbard_model(K, U, L * dtau, dtau, 1, trotter=trotter)
    got = exact_small.enumerate_eq_correlations(m, lat, tau=0)
    F = Fock(lat.K, U, h)
    S = F.trotter(dtau) if trotter == "sym" else F.trotter_asym(dtau)
    c = F.c

    def ops(i, j):
        green = 0.5 * sum(c[2 * i + s].T @ c[2 * j + s] for s in (0, 1))
        spz = F.sz(i) @ F.sz(j)
        sp_i, sp_j = c[2 * i].T @ c[2 * i + 1], c[2 * j].T @ c[2 * j + 1]
        spxy = 0.25 * (sp_i @ sp_j.T + sp_i.T @ sp_j)
        den = (F.n[i][0] + F.n[i][1]) @ (F.n[j][0] + F.n[j][1])
        return (green, spz, spxy, den)

    nc, norb = lat.n_cells, lat.norb
    site = {(int(lat.cell_of[i]), int(lat.orb_of[i])): i for i in range(lat.n)}
    want = np.zeros((4, nc, norb, norb))
    for I in range(nc):
        i1, i2 = I % lat.L1, I // lat.L1
        for R in range(nc):
            J = (i1 + R % lat.L1) % lat.L1 + lat.L1 * ((i2 + R // lat.L1) % lat.L2)
            for a in range(norb):
                for b in range(norb):
                    for o, O in enumerate(ops(site[I, a], site[J, b])):
                        want[o, R, a, b] += F.expect_with(S, O, L) / nc
    assert np.max(np.abs(got - want)) < 1e-12, (trotter, np.max(np.abs(got - want), axis=(1, 2, 3)))
    # <S^z> per orbital, averaged over cells
    logw, sz = [], []
    for f in exact_small.all_fields(m):
        logw.append(log_weight(m, f))
        sz.append(measure.eq_spin_z(m, lat, green_scratch(m, f, 0)))
    w = np.exp(np.array(logw) - max(logw))
    sz_want = np.zeros(norb)
    for I in range(nc):
        for a in range(norb):
            sz_want[a] += F.expect_with(S, F.sz(site[I, a]), L) / nc
    assert np.max(np.abs(w @ np.array(sz) / w.sum() - sz_want)) < 1e-12
    assert (np.min(sz_want) > 1e-3) == (h > 0.0)
    # SU(2): the z and xy spin correlations agree on average (not per
    # configuration); the Zeeman field breaks it
    if h == 0.0:
        assert np.max(np.abs(got[1] - got[2])) < 1e-12
    else:
        assert np.max(np.abs(got[1] - got[2])) > 1e-3
    # a planted mistake (no sublattice sign in the down-spin Green term) fails
    s_saved = lat.sublattice_sign
    try:
        lat.sublattice_sign = lambda: np.ones(lat.n)
        bad = exact_small.enumerate_eq_correlations(m, lat, tau=0)
    finally:
        lat.sublattice_sign = s_saved
    assert np.max(np.abs(bad[0] - want[0])) > 1e-3


@pytest.mark.parametrize("trotter,h", [("sym", 0.0), ("asym", 0.0), ("asym", 0.6)])
def test_td_correlations_enumeration_equals_fock(trotter, h):
    """Time-displaced lattice-resolved correlations (Green, SpinZ, SpinXY, Den
    by displacement and orbital pair) of a 4-site honeycomb ring (2 cells x 2
    orbitals) x 2 slices at tau = 0, 1, 2 slices: the exact weighted average of
    the per-configuration estimators against Tr(S^(L-n) A_i S^n B_j) / Tr(S^L)
    in Fock space, with A, B built from the original-frame fermions; h > 0 adds
    the M_z form's Zeeman field (frame hopping K = T - h)."""
    from oracle import exact_small
    from oracle import timedisplaced as otd
    lat = honeycomb_lattice(1, 2)
    U, dtau, L = 4.0, 0.25, 2
    K = hubbard.mz_frame_hopping(lat.K, h, lat.sublattice_sign())
    m = hubbard.hubbard_model(K, U, L * dtau, dtau, 1, trotter=trotter)
    taus = (0, 1, 2)
    got = exact_small.enumerate_td_correlations(m, lat, taus)
    F = Fock(lat.K, U, h)
    S = F.trotter(dtau) if trotter == "sym" else F.trotter_asym(dtau)
    c = F.c

    def pairs(i, j):
        sp_i, sp_j = c[2 * i].T @ c[2 * i + 1], c[2 * j].T @ c[2 * j + 1]
        n_i, n_j = F.n[i][0] + F.n[i][1], F.n[j][0] + F.n[j][1]
        return ([(0.5, c[2 * i + s].T, c[2 * j + s]) for s in (0, 1)],
                [(1.0, F.sz(i), F.sz(j))],
                [(0.25, sp_i, sp_j.T), (0.25, sp_i.T, sp_j)],
                [(1.0, n_i, n_j)])

    nc, norb = lat.n_cells, lat.norb
    site = {(int(lat.cell_of[i]), int(lat.orb_of[i])): i for i in range(lat.n)}
    want = np.zeros((len(taus), 4, nc, norb, norb))
    for t, n in enumerate(taus):
        for I in range(nc):
            i1, i2 = I % lat.L1, I // lat.L1
            for R in range(nc):
                J = (i1 + R % lat.L1) % lat.L1 + lat.L1 * ((i2 + R // lat.L1) % lat.L2)
                for a in range(norb):
                    for b in range(norb):
                        for o, terms in enumerate(pairs(site[I, a], site[J, b])):
                            for w, A, B in terms:
                                want[t, o, R, a, b] += w * F.expect_tau_with(S, A, B, L, n) / nc
    assert np.max(np.abs(got - want)) < 1e-12, (trotter, np.max(np.abs(got - want), axis=(2, 3, 4)))
    # SU(2) on average (without the Zeeman field); tau = 0 is the equal-time
    # estimator; the Fourier sum of SpinZ at K is the momentum-space estimator
    if h == 0.0:
        assert np.max(np.abs(got[:, 1] - got[:, 2])) < 1e-12
    assert np.max(np.abs(got[0] - exact_small.enumerate_eq_correlations(m, lat, tau=0))) < 1e-12
    g1, g2 = lat.reciprocal()
    kvec = 0.5 * g2
    rpos = np.array([(R % lat.L1) * lat.a1 + (R // lat.L1) * lat.a2 for R in range(nc)])
    sk = np.einsum("r,trab->tab", np.exp(1j * (rpos @ kvec)), got[:, 1])
    assert np.max(np.abs(sk - exact_small.enumerate_szsz(m, lat, kvec, taus))) < 1e-12
    # a planted mistake in the oracle (G0T transposed) fails it
    saved = otd.tdgf_scratch
    try:
        otd.tdgf_scratch = lambda model, f, tau: (lambda r: (r[0], r[1].T, r[2]))(saved(model, f, tau))
        bad = exact_small.enumerate_td_correlations(m, lat, taus)
    finally:
        otd.tdgf_scratch = saved
    assert np.max(np.abs(bad[1:] - want[1:])) > 1e-3


def test_correlation_entry_subsets_equal_the_full_evaluation():
    """The oracle's optional entry lists evaluate exactly the listed entries
    of the full (Fock-pinned) evaluation, equal-time and time-displaced."""
    from oracle import measure
    from oracle import timedisplaced as otd
    lat = honeycomb_lattice(3, 2)
    m = hubbard.hubbard_model(lat.K, 4.0, 0.4, 0.1, 2, trotter="sym")
    f = np.where(np.random.default_rng(5).random((m.L, m.N)) < 0.5, 1.0, -1.0)
    entries = [(0, 0, 0), (0, 1, 0), (4, 0, 1), (5, 1, 1), (2, 1, 0)]
    from oracle.stable import green_scratch
    G = green_scratch(m, f, 2)
    full = measure.eq_correlations(m, lat, G)
    sub = measure.eq_correlations(m, lat, G, entries)
    assert sub.shape == (4, len(entries))
    for e, (R, a, b) in enumerate(entries):
        assert np.array_equal(sub[:, e], full[:, R, a, b])
    full_t = otd.tdgf_correlations(m, lat, f, taus=(1, 3))
    sub_t = otd.tdgf_correlations(m, lat, f, taus=(1, 3), entries=entries)
    for e, (R, a, b) in enumerate(entries):
        assert np.array_equal(sub_t[:, :, e], full_t[:, :, R, a, b])
