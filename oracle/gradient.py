"""Gradient of the fermion determinant and Langevin updates of a continuous
HS field (oracle side).

Continuous fields are outside the paper's code (section "Definition of the
Hamiltonian": continuous HS transformations are not accessible; listed again
among the future directions), so this module is a reading built on
Eq. (Green_eq) and Eq. (partition_2):

    B_tau = diag(exp(c phi_tau)) exp(-dtau K),   dB_tau/dphi_{i,tau} = c e_i e_i^T B_tau,
    d log det(1 + B(beta,0)) / dphi_{i,tau}
        = c [B(tau,0) (1 + B(beta,0))^-1 B(beta,tau)]_ii = c (1 - G(tau))_ii,

with G(tau) = (1 + B(tau,0) B(beta,tau))^-1 (trace identity; B(beta,0) =
B(beta,tau) B(tau,0)).  With the Gaussian prefactor of the weight,

    d log W / dphi_{i,tau} = -phi_{i,tau} + N_col c alpha + N_col c (1 - G(tau)_ii).

Unadjusted Langevin step (reading): phi <- phi + eps d log W + sqrt(2 eps) xi,
xi ~ N(0,1) from Philox (tag LANGEVIN, counter (step, tau << 1, site)).
"""
import numpy as np

from . import philox
from .stable import green_scratch, logdet_scratch


def grad_logdet(model, field, taus=None):
    """[L, N]: d log det(1 + B(beta,0)) / d phi, from scratch G(tau) for every
    tau (or [len(taus), N] for the listed slices only)."""
    taus = range(1, model.L + 1) if taus is None else taus
    g = np.empty((len(taus), model.N))
    for k, tau in enumerate(taus):
        G = green_scratch(model, field, tau)
        g[k] = model.coupling * (1.0 - np.diag(G))
    return g


def grad_log_weight(model, field):
    return -np.asarray(field) + model.n_col * model.coupling * model.alpha \
        + model.n_col * grad_logdet(model, field)


def fd_logdet(model, field, tau, i, h=1e-5):
    """Central finite difference of log det(1 + B(beta,0)) in phi_{i,tau}."""
    fp = np.array(field, dtype=float)
    fm = np.array(field, dtype=float)
    fp[tau - 1, i] += h
    fm[tau - 1, i] -= h
    return (logdet_scratch(model, fp) - logdet_scratch(model, fm)) / (2.0 * h)


def langevin_step(model, field, eps, step):
    xi = np.empty((model.L, model.N))
    for tau in range(1, model.L + 1):
        xi[tau - 1] = philox.normals(model.seed, philox.TAG_LANGEVIN, step, tau, 0, model.N)
    return np.asarray(field) + eps * grad_log_weight(model, field) + np.sqrt(2.0 * eps) * xi
