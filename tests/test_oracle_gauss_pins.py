"""Pins of the oracle's continuous (Gaussian) field against physics.

The Gaussian identity exp(dtau U/2 A^2) = int dphi (2 pi)^-1/2 exp(-phi^2/2)
exp(c phi A), c = sqrt(dtau U), is exact for every A, so the oracle's weight
of a Gaussian field (the -phi^2/2 measure, the alpha prefactor and the
determinant, Eq. (partition_2)) integrated over phi must reproduce the same
Trotterised expectation values as the two-valued field and as Fock space.
These tests integrate the oracle's own log_weight and estimators with
Gauss-Hermite product rules (no sampling error), check the drift of the
Langevin step against finite differences of that weight, and check that the
local move of the Gaussian field samples the exact one-site marginal.  Each
pin is shown to fail for a planted mistake of the kind it guards against.
"""
import itertools
import math

import numpy as np
import pytest

from fock import Fock
from inputs import square_lattice
from oracle import gradient, hubbard, measure, stable, sweep


def _gh_average(model, n_nodes, taus, obs):
    """Weighted averages of obs(model, G(tau)) over the Gaussian field by a
    product Gauss-Hermite rule in every field value (probabilists' weight
    exp(-x^2/2); the oracle's log_weight carries that factor itself, so it is
    divided out at the nodes)."""
    x, w = np.polynomial.hermite_e.hermegauss(n_nodes)
    L, N = model.L, model.N
    num = np.zeros((len(taus),) + np.shape(obs(model, np.eye(N) * 0.5)))
    den = 0.0
    for idx in itertools.product(range(n_nodes), repeat=L * N):
        f = x[list(idx)].reshape(L, N)
        lw = stable.log_weight(model, f) + 0.5 * float(np.sum(f * f))
        wt = math.exp(lw) * float(np.prod(w[list(idx)]))
        den += wt
        for k, t in enumerate(taus):
            num[k] += wt * np.asarray(obs(model, stable.green_scratch(model, f, t)))
    return num / den


def _double_occ(model, G):
    return measure.equal_time(model, G)[0]


def _d_and_ekin(model, G):
    D, ekin, _ = measure.equal_time(model, G)
    return np.array([D, ekin])


# ------------------------------------------------------------- atomic limit --
def test_gaussian_atomic_limit_double_occupancy():
    """t = 0, one site: D = 1 / (2 (1 + exp(beta U / 2))) exactly for the
    Gaussian field too (the identity is exact on every slice)."""
    U, beta, L = 4.0, 1.0, 2
    m = hubbard.hubbard_model(np.zeros((1, 1)), U, beta, beta / L, L, field_kind="gauss")
    exact = 1.0 / (2.0 * (1.0 + np.exp(beta * U / 2)))
    res = _gh_average(m, 40, (0, 1), _double_occ)
    assert np.max(np.abs(res - exact)) < 1e-13


def test_gaussian_atomic_limit_three_slices():
    U, beta, L = 5.0, 0.9, 3
    m = hubbard.hubbard_model(np.zeros((1, 1)), U, beta, beta / L, L, field_kind="gauss")
    exact = 1.0 / (2.0 * (1.0 + np.exp(beta * U / 2)))
    res = _gh_average(m, 24, (0, 2), _double_occ)
    assert np.max(np.abs(res - exact)) < 1e-12


def test_gaussian_atomic_limit_detects_wrong_measure():
    """Planted mistakes in the Gaussian factor of the weight: -phi^2 in place
    of -phi^2/2, or the measure left out, move D away from the exact value."""
    U, beta, L = 4.0, 1.0, 2
    exact = 1.0 / (2.0 * (1.0 + np.exp(beta * U / 2)))
    for wrong in (lambda s: -np.asarray(s, dtype=float) ** 2, lambda s: np.zeros_like(np.asarray(s, dtype=float))):
        m = hubbard.hubbard_model(np.zeros((1, 1)), U, beta, beta / L, L, field_kind="gauss")
        m.vertex_log_factor = wrong
        res = _gh_average(m, 40, (0,), _double_occ)
        assert abs(res[0] - exact) > 1e-3


# ------------------------------------------------------- 2 sites, Fock space --
@pytest.mark.parametrize("trotter", ["sym", "asym"])
def test_gaussian_two_site_equals_fock_trotter(trotter):
    """2 sites x 2 slices: the Gauss-Hermite average of the oracle's D and
    E_kin over the four field values equals the Fock-space Trotter product of
    the repulsive Hubbard model (tests/fock.py) at every slice."""
    K = np.array([[0.0, -1.0], [-1.0, 0.0]])
    U, dtau, L = 4.0, 0.25, 2
    m = hubbard.hubbard_model(K, U, L * dtau, dtau, 1, field_kind="gauss", trotter=trotter)
    res = _gh_average(m, 12, (0, 1), _d_and_ekin)
    F = Fock(K, U)
    S = F.trotter(dtau) if trotter == "sym" else F.trotter_asym(dtau)
    D = F.expect_with(S, F.double_occ(), L)
    E = F.expect_with(S, F.kinetic(), L)
    assert np.max(np.abs(res[:, 0] - D)) < 1e-12
    assert np.max(np.abs(res[:, 1] - E)) < 1e-12


# --------------------------------------------------- Langevin drift vs weight --
def _drift_error(model, field, drift, points, h=1e-5):
    """Largest |drift - central difference of log W| over the given (tau, i)."""
    err = 0.0
    for tau, i in points:
        fp = np.array(field, dtype=float)
        fm = np.array(field, dtype=float)
        fp[tau - 1, i] += h
        fm[tau - 1, i] -= h
        fd = (stable.log_weight(model, fp) - stable.log_weight(model, fm)) / (2.0 * h)
        err = max(err, abs(fd - drift[tau - 1, i]))
    return err


@pytest.fixture(scope="module")
def gauss_chain():
    lat = square_lattice(3, 3)
    m = hubbard.hubbard_model(lat.K, 4.0, 2.0, 0.1, 5, field_kind="gauss", seed=3)
    f = hubbard.init_field(m)
    rng = np.random.default_rng(7)
    pts = [(int(rng.integers(1, m.L + 1)), int(rng.integers(0, m.N))) for _ in range(8)]
    return m, f, pts


def test_grad_log_weight_matches_fd_of_log_weight(gauss_chain):
    """d log W / d phi_{i,tau} = -phi + N_col c alpha + N_col c (1 - G(tau)_ii),
    the Langevin drift, against central differences (h = 1e-5) of the full
    log weight of Eq. (partition_2) (prefactor and N_col log det)."""
    m, f, pts = gauss_chain
    drift = gradient.grad_log_weight(m, f)
    assert _drift_error(m, f, drift, pts) < 1e-6


def test_grad_log_weight_fd_detects_planted_mistakes(gauss_chain):
    """The same check fails for a drift with N_col dropped from the
    determinant term, with the sign of alpha flipped, or with the Gaussian
    term doubled."""
    m, f, pts = gauss_chain
    g = gradient.grad_logdet(m, f)
    c, a, nc = m.coupling, m.alpha, m.n_col
    wrong = {
        "dropped N_col": -f + nc * c * a + g,
        "flipped alpha": -f - nc * c * a + nc * g,
        "doubled Gaussian term": -2.0 * f + nc * c * a + nc * g,
    }
    for name, d in wrong.items():
        assert _drift_error(m, f, d, pts) > 1e-2, name


# ------------------------------------------------- local move, 1 site x 1 slice --
def _marginal_bin_probs(c, edges):
    """Exact marginal of phi on one site and one slice at t = 0 (N_col = 2,
    alpha = -1/2): W(phi) = exp(-phi^2/2) exp(-c phi) (1 + exp(c phi))^2
    = exp(-phi^2/2) (exp(-c phi) + 2 + exp(c phi)); each term integrates to a
    shifted normal distribution function."""
    def Phi(z):
        return 0.5 * (1.0 + np.array([math.erf(v / math.sqrt(2.0)) for v in z]))
    mass = np.zeros(len(edges) - 1)
    total = 0.0
    for k, coef in ((-c, 1.0), (0.0, 2.0), (c, 1.0)):
        scale = coef * math.exp(0.5 * k * k)
        cdf = Phi(edges - k)
        mass += scale * np.diff(cdf)
        total += scale
    return mass / total


def _local_move_histogram(model, n_sweeps, edges):
    """Histogram of the field after each sweep, or None when the chain runs
    away (a weight that is not normalisable sends phi off to infinity)."""
    ch = sweep.Chain(model, hubbard.init_field(model)).init()
    counts = np.zeros(len(edges) - 1)
    with np.errstate(all="ignore"):
        for _ in range(n_sweeps):
            try:
                ch.sweep(measure=False)
            except (ValueError, FloatingPointError, np.linalg.LinAlgError):
                return None
            phi = ch.field[0, 0]
            if not np.isfinite(phi) or abs(phi) > 1e3:
                return None
            counts[np.searchsorted(edges, phi) - 1] += 1
    return counts


def test_gaussian_local_move_samples_exact_marginal():
    """The local move phi' = phi + a (2 u - 1) with the ratio of Eq. (partition_2)
    (Gaussian factor, alpha prefactor, determinant) must leave the exact
    marginal invariant; chi^2 of the visited values over 12 bins."""
    U, dtau = 4.0, 0.25
    m = hubbard.hubbard_model(np.zeros((1, 1)), U, dtau, dtau, 1, field_kind="gauss", seed=21)
    m.prop_width = 1.5
    edges = np.concatenate([[-np.inf], np.linspace(-2.5, 2.5, 11), [np.inf]])
    p = _marginal_bin_probs(m.coupling, edges)
    n = 6000
    counts = _local_move_histogram(m, n, edges)
    chi2 = np.sum((counts - n * p) ** 2 / (n * p)) / (p.size - 1)
    # successive sweeps are correlated (two moves per sweep); allow about 2.5x
    assert chi2 < 2.5
    # planted mistakes in the move's Gaussian factor
    for wrong in (lambda s: -np.asarray(s, dtype=float) ** 2, lambda s: 0.5 * np.asarray(s, dtype=float) ** 2):
        m2 = hubbard.hubbard_model(np.zeros((1, 1)), U, dtau, dtau, 1, field_kind="gauss", seed=21)
        m2.prop_width = 1.5
        m2.vertex_log_factor = wrong
        c2 = _local_move_histogram(m2, n, edges)
        chi2w = np.inf if c2 is None else np.sum((c2 - n * p) ** 2 / (n * p)) / (p.size - 1)
        assert chi2w > 8.0
