"""Brute-force enumeration over every field configuration of a tiny system.

Eq. (obs): <O> = sum_C P(C) <<O>>_C with P(C) proportional to the weight of
Eq. (partition_2).  For N L <= ~10 all 2^(N L) Ising configurations are summed
exactly; the result is the Trotterised expectation value with no sampling
error, which the tests compare with a Fock-space evaluation.
"""
import itertools

import numpy as np

from .measure import eq_correlations, equal_time
from .stable import green_scratch, log_weight
from .timedisplaced import tdgf_measure


def all_fields(model):
    """Every configuration: +-1 per vertex, or the four values eta(l) of
    Eq. (HS_squares) for the four-valued field."""
    from .hubbard import ETA4
    values = ETA4 if model.field_kind == "ising4" else (1.0, -1.0)
    for bits in itertools.product(values, repeat=model.L * model.N):
        yield np.array(bits).reshape(model.L, model.N)


def enumerate_observables(model, taus=(0,)):
    """Exact weighted averages of (D, E_kin, E_pot) at each tau in taus."""
    logw = []
    obs = []
    for f in all_fields(model):
        logw.append(log_weight(model, f))
        obs.append([equal_time(model, green_scratch(model, f, t)) for t in taus])
    logw = np.array(logw)
    w = np.exp(logw - logw.max())
    obs = np.array(obs)                                # [configs, taus, 3]
    return np.einsum("c,ctk->tk", w, obs) / w.sum()


def enumerate_weights(model):
    """Normalised P(C) over all configurations (in itertools order)."""
    logw = np.array([log_weight(model, f) for f in all_fields(model)])
    w = np.exp(logw - logw.max())
    return w / w.sum()


def enumerate_szsz(model, lat, kvec, taus):
    """Exact weighted average of S_ab(K, tau) (time-displaced estimator) at
    each tau in taus: [len(taus), norb, norb] complex."""
    logw = []
    obs = []
    for f in all_fields(model):
        logw.append(log_weight(model, f))
        obs.append(tdgf_measure(model, lat, kvec, f, taus))
    logw = np.array(logw)
    w = np.exp(logw - logw.max())
    return np.einsum("c,ctab->tab", w, np.array(obs)) / w.sum()


def enumerate_eq_correlations(model, lat, tau=0):
    """Exact weighted average of the lattice-resolved equal-time correlations
    (measure.eq_correlations) at slice tau: [4, N_cells, norb, norb]."""
    logw = []
    obs = []
    for f in all_fields(model):
        logw.append(log_weight(model, f))
        obs.append(eq_correlations(model, lat, green_scratch(model, f, tau)))
    logw = np.array(logw)
    w = np.exp(logw - logw.max())
    return np.einsum("c,c...->...", w, np.array(obs)) / w.sum()


def enumerate_td_correlations(model, lat, taus):
    """Exact weighted average of the time-displaced lattice-resolved
    correlations (timedisplaced.td_correlations) at each tau in taus:
    [len(taus), 4, N_cells, norb, norb]."""
    from .timedisplaced import tdgf_correlations
    logw = []
    obs = []
    for f in all_fields(model):
        logw.append(log_weight(model, f))
        obs.append(tdgf_correlations(model, lat, f, taus))
    logw = np.array(logw)
    w = np.exp(logw - logw.max())
    return np.einsum("c,c...->...", w, np.array(obs)) / w.sum()
