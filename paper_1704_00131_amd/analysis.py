"""Error analysis of binned Monte Carlo data (section "Monte Carlo sampling",
its subsections on the jackknife resampling method and on error estimation).

The library accumulates observables into bins on the device; a caller reads
and resets them every few sweeps (dqmc_read_bins / dqmc_reset_bins), which
gives one row per bin.  Everything here works on such host arrays, shape
[n_bins] or [n_bins, n_obs]:

- skip(x, n_skip)       drop warm-up bins (the analysis parameter n_skip);
- rebin(x, n_rebin)     average n_rebin adjacent bins into one (N_rebin);
- jackknife(f, *obs)    delete-1 jackknife mean and error of a function of
                        expectation values;
- autocorrelation(x, n) the normalised autocorrelation function of the bin
                        series for lags 0..n (N_auto);
- covariance(x)         the covariance of the bin means of a vector
                        observable, e.g. S(k, tau) over tau (N_Cov);
- spin_total(C)         the rotation-averaged spin correlation
                        (S^x S^x + S^y S^y + S^z S^z)/3 from the SpinZ and
                        SpinXY bins (the improved estimator of the error
                        analysis section);
- momentum_grid(lat)    the L1 x L2 momenta of the Bravais torus;
- to_momentum(C, lat, k) a correlation stored by displacement R (the
                        lattice-resolved bins) at momenta k:
                        C(k) = sum_R exp(i k.R) C(R).
"""
from typing import Callable, Sequence, Tuple

import numpy as np


def skip(x, n_skip: int) -> np.ndarray:
    """The bins after the first n_skip."""
    x = np.asarray(x, dtype=np.float64)
    if n_skip < 0 or n_skip >= x.shape[0]:
        raise ValueError("n_skip must leave at least one bin")
    return x[n_skip:]


def rebin(x, n_rebin: int) -> np.ndarray:
    """New bins from n_rebin adjacent old ones (a trailing remainder is dropped)."""
    x = np.asarray(x, dtype=np.float64)
    if n_rebin < 1:
        raise ValueError("n_rebin must be positive")
    nb = x.shape[0] // n_rebin
    if nb < 1:
        raise ValueError("fewer bins than n_rebin")
    return x[: nb * n_rebin].reshape((nb, n_rebin) + x.shape[1:]).mean(axis=1)


def jackknife(f: Callable[..., np.ndarray], *obs) -> Tuple[np.ndarray, np.ndarray]:
    """Delete-1 jackknife of f(<A>, <B>, ...) from the bin series A, B, ...
    (each [n_bins] or [n_bins, ...]): with A_(i) the mean without bin i and
    f_(i) = f(A_(i), B_(i), ...), the mean is the average of the f_(i) and the
    squared error (n - 1)/n times the sum of their squared deviations from it."""
    arrs = [np.asarray(a, dtype=np.float64) for a in obs]
    n = arrs[0].shape[0]
    if n < 2 or any(a.shape[0] != n for a in arrs):
        raise ValueError("need at least two bins, the same number for every observable")
    loo = [(a.sum(axis=0)[None, ...] - a) / (n - 1) for a in arrs]
    fi = np.array([np.asarray(f(*[l[i] for l in loo]), dtype=np.float64) for i in range(n)])
    mean = fi.mean(axis=0)
    err = np.sqrt((n - 1) / n * np.sum((fi - mean) ** 2, axis=0))
    return mean, err


def autocorrelation(x, n_auto: int) -> np.ndarray:
    """Auto(t) for t = 0..n_auto: the sum over i of (O_i - m)(O_{i+t} - m),
    divided by the sum over i of (O_i - m)^2, with m the mean over all bins
    (Auto(0) = 1)."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim != 1 or n_auto < 0 or n_auto >= x.shape[0]:
        raise ValueError("a 1-d series longer than n_auto is needed")
    d = x - x.mean()
    den = np.dot(d, d)
    if den == 0.0:
        raise ValueError("constant series")
    return np.array([np.dot(d[: d.size - t], d[t:]) / den for t in range(n_auto + 1)])


def covariance(x) -> np.ndarray:
    """COV[a, b] of the bin means of a vector observable (bins x components):
    1/n times the average over bins of (x_a - <x_a>)(x_b - <x_b>), with the
    unbiased 1/(n - 1) normalisation of that average."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim != 2 or x.shape[0] < 2:
        raise ValueError("bins x components, at least two bins")
    n = x.shape[0]
    d = x - x.mean(axis=0)
    return d.T @ d / (n - 1) / n


def error_vs_rebin(x, sizes: Sequence[int]) -> np.ndarray:
    """Jackknife error of the mean for each rebinning size: it grows while the
    effective bins are shorter than the autocorrelation time and levels off
    beyond it."""
    return np.array([jackknife(lambda a: a, rebin(x, s))[1] for s in sizes])


def displacements(lat) -> np.ndarray:
    """[N_cells, 2] positions R = r1 a1 + r2 a2 of the displacement index
    r1 + L1 r2 used by the lattice-resolved bins."""
    idx = np.arange(lat.L1 * lat.L2)
    return np.outer(idx % lat.L1, lat.a1) + np.outer(idx // lat.L1, lat.a2)


def momentum_grid(lat) -> np.ndarray:
    """[N_cells, 2] momenta k = (m1/L1) g1 + (m2/L2) g2 of the torus, m1 + L1 m2
    ordered like the displacements (g1, g2 the reciprocal vectors)."""
    g1, g2 = lat.reciprocal()
    idx = np.arange(lat.L1 * lat.L2)
    return np.outer((idx % lat.L1) / lat.L1, g1) + np.outer((idx // lat.L1) / lat.L2, g2)


def to_momentum(C, lat, kvecs) -> np.ndarray:
    """C(k)[..., a, b] = sum_R exp(i k.R) C[..., R, a, b] for each k in kvecs
    ([n_k, 2]): the Fourier transform of a correlation stored by displacement,
    C(R) = 1/N_cells sum_I <O_{I,a} O_{I+R,b}>; its sign convention makes C(k)
    at a torus momentum equal to 1/N_cells sum_{I,J} exp(-i k.(R_I - R_J))
    <O_{I,a} O_{J,b}>.  Returns [..., n_k, norb, norb] complex."""
    C = np.asarray(C, dtype=np.float64)
    ph = np.exp(1j * (np.asarray(kvecs, dtype=np.float64).reshape(-1, 2) @ displacements(lat).T))   # [k, R]
    return np.einsum("kr,...rab->...kab", ph, C)


def spin_total(C) -> np.ndarray:
    """(<S^x S^x> + <S^y S^y> + <S^z S^z>)/3 from correlation bins ordered
    Green, SpinZ, SpinXY, Den on the first axis ([4, ...]; for time-displaced
    bins [L+1, 4, ...] pass them with that axis first, e.g. np.moveaxis(C, 1,
    0)).  SpinXY holds half of S^x S^x + S^y S^y, so the sum is
    (SpinZ + 2 SpinXY)/3.  Its average equals SpinZ's where the spin symmetry
    holds, and it fluctuates less between configurations."""
    C = np.asarray(C, dtype=np.float64)
    return (C[1] + 2.0 * C[2]) / 3.0
