"""The bin analysis (paper_1704_00131_amd.analysis) against closed forms.

- jackknife of f = mean is the sample mean with the bias-corrected standard
  error (the paper's stated special case);
- jackknife of a ratio of means agrees with the delta-method error, and a
  planted mistake (no (n-1)/n factor) does not;
- the autocorrelation of an AR(1) series x_t = rho x_{t-1} + e_t is rho^t;
- rebinning an AR(1) series converges to the known error of its mean,
  sigma sqrt((1 + rho)/(1 - rho) / n), from below;
- the covariance of the means of normal bins with a known covariance C is C/n.
"""
import numpy as np
import pytest

from paper_1704_00131_amd import analysis as an


def _ar1(rho, n, seed):
    rng = np.random.default_rng(seed)
    e = rng.normal(size=n)
    x = np.empty(n)
    x[0] = e[0] / np.sqrt(1.0 - rho * rho)          # stationary start
    for t in range(1, n):
        x[t] = rho * x[t - 1] + e[t]
    return x


def test_jackknife_of_the_mean_is_mean_and_stderr():
    x = np.random.default_rng(1).normal(size=(50, 3))
    m, e = an.jackknife(lambda a: a, x)
    assert np.max(np.abs(m - x.mean(axis=0))) < 1e-14
    assert np.max(np.abs(e - x.std(axis=0, ddof=1) / np.sqrt(50))) < 1e-14


def test_jackknife_ratio_matches_delta_method():
    rng = np.random.default_rng(2)
    n = 4000
    A = 2.0 + 0.3 * rng.normal(size=n)
    B = 5.0 + 0.4 * rng.normal(size=n) + 0.2 * (A - 2.0)
    m, e = an.jackknife(lambda a, b: a / b, A, B)
    ma, mb = A.mean(), B.mean()
    C = np.cov(np.vstack([A, B]))
    grad = np.array([1.0 / mb, -ma / mb ** 2])
    e_delta = np.sqrt(grad @ C @ grad / n)
    assert abs(m - ma / mb) < 1e-6
    assert abs(e / e_delta - 1.0) < 0.01
    # the same resampling without the (n - 1)/n factor is off by sqrt(n)
    assert abs(e / np.sqrt((n - 1) / n) * np.sqrt(1.0 / (n - 1)) / e_delta - 1.0) > 0.5


@pytest.mark.parametrize("rho", [0.5, 0.8])
def test_autocorrelation_of_ar1(rho):
    x = _ar1(rho, 200000, 3)
    a = an.autocorrelation(x, 6)
    assert a[0] == pytest.approx(1.0)
    assert np.max(np.abs(a - rho ** np.arange(7))) < 0.01


def test_rebinning_converges_to_the_ar1_error():
    rho, n = 0.8, 200000
    x = _ar1(rho, n, 4)
    sizes = [1, 4, 16, 64, 256]
    err = an.error_vs_rebin(x, sizes)
    exact = np.sqrt((1.0 + rho) / (1.0 - rho) / (1.0 - rho * rho) / n)   # var(x) = 1/(1 - rho^2)
    assert err[0] < 0.5 * exact                       # single bins underestimate it
    assert np.all(np.diff(err) > -0.05 * exact)       # non-decreasing within noise
    assert abs(err[-1] / exact - 1.0) < 0.1


def test_covariance_of_normal_bins():
    C = np.array([[1.0, 0.6, 0.2], [0.6, 2.0, -0.3], [0.2, -0.3, 0.5]])
    n = 100000
    x = np.random.default_rng(5).multivariate_normal(np.zeros(3), C, size=n)
    cov = an.covariance(x)
    assert np.max(np.abs(cov * n - C)) < 0.03


def test_skip_and_rebin_shapes_and_errors():
    x = np.arange(10.0)
    assert np.array_equal(an.skip(x, 3), np.arange(3.0, 10.0))
    assert np.array_equal(an.rebin(x, 3), np.array([1.0, 4.0, 7.0]))
    with pytest.raises(ValueError):
        an.rebin(x, 11)
    with pytest.raises(ValueError):
        an.skip(x, 10)
    with pytest.raises(ValueError):
        an.autocorrelation(np.ones(5), 2)


def test_momentum_transform_matches_the_site_double_sum():
    """The Fourier transform of the displacement-resolved SpinZ correlation of
    one configuration equals, at every torus momentum, the double sum over
    sites with a phase per site (the time-displaced S(K, tau) estimator); the
    inverse transform over the grid gives C(R) back."""
    from inputs import honeycomb_lattice
    from oracle import hubbard
    from oracle import timedisplaced as otd
    lat = honeycomb_lattice(3, 3)
    m = hubbard.hubbard_model(lat.K, 4.0, 0.4, 0.1, 2, trotter="asym")
    f = np.where(np.random.default_rng(1).random((m.L, m.N)) < 0.5, 1.0, -1.0)
    GT0, G0T, GTT = otd.tdgf_scratch(m, f, 2)
    _, _, G00 = otd.tdgf_scratch(m, f, 0)
    C = otd.td_correlations(m, lat, GT0, G0T, GTT, G00)
    ks = an.momentum_grid(lat)
    Ck = an.to_momentum(C[1], lat, ks)
    assert Ck.shape == (lat.n_cells, 2, 2)
    for k in range(lat.n_cells):
        assert np.max(np.abs(Ck[k] - otd.szsz_k(m, lat, ks[k], GT0, G0T, GTT, G00))) < 1e-12
    back = np.einsum("kr,kab->rab", np.exp(-1j * (ks @ an.displacements(lat).T)), Ck) / lat.n_cells
    assert np.max(np.abs(back - C[1])) < 1e-12
    # every correlator at once: leading axes are kept
    assert an.to_momentum(C, lat, ks[:3]).shape == (4, 3, 2, 2)


def test_spin_total_equals_fock_s_dot_s():
    """(SpinZ + 2 SpinXY)/3 of the exactly enumerated correlation bins equals
    the Fock-space <S_i . S_j>/3 with the Zeeman field on (where SpinZ and
    SpinXY differ, so a wrong weight fails)."""
    from fock import Fock
    from inputs import honeycomb_lattice
    from oracle import exact_small, hubbard
    lat = honeycomb_lattice(1, 2)
    U, dtau, L, h = 4.0, 0.25, 2, 0.6
    m = hubbard.hubbard_model(hubbard.mz_frame_hopping(lat.K, h, lat.sublattice_sign()), U, L * dtau, dtau, 1,
                              trotter="asym")
    C = exact_small.enumerate_eq_correlations(m, lat, tau=0)
    F = Fock(lat.K, U, h)
    S = F.trotter_asym(dtau)
    c = F.c
    site = {(int(lat.cell_of[i]), int(lat.orb_of[i])): i for i in range(lat.n)}
    want = np.zeros((lat.n_cells, 2, 2))
    for I in range(lat.n_cells):
        for R in range(lat.n_cells):
            J = (I % lat.L1 + R % lat.L1) % lat.L1 + lat.L1 * ((I // lat.L1 + R // lat.L1) % lat.L2)
            for a in range(2):
                for b in range(2):
                    i, j = site[I, a], site[J, b]
                    sp_i, sp_j = c[2 * i].T @ c[2 * i + 1], c[2 * j].T @ c[2 * j + 1]
                    sdots = F.sz(i) @ F.sz(j) + 0.5 * (sp_i @ sp_j.T + sp_i.T @ sp_j)
                    want[R, a, b] += F.expect_with(S, sdots, L) / 3.0 / lat.n_cells
    assert np.max(np.abs(an.spin_total(C) - want)) < 1e-12
    assert np.max(np.abs(C[1] - want)) > 1e-3
