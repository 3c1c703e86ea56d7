"""Equal-time estimators of the oracle (section "Observables", the potential
energy and GRC listings of the square-lattice example).

In the sampling frame the repulsive double occupancy n_up n_dn becomes
n_up (1 - n_dn); with the two colours independent for a given field (Wick's
theorem, SU(N_col) symmetry of Eq. (partition_2)) its per-configuration value
is Gt_ii (1 - Gt_ii), where Gt is the Green's function of the measured split.
With a symmetric Trotter split the measured G is
Gt = exp(-dtau K/2) G exp(+dtau K/2) (a reading: the paper's B_tau has the
kinetic factor on one side only).  The kinetic energy per site is
(N_col/N) sum_xy K_xy <c_x^+ c_y> = (2/N)(Tr K - Tr(K G)), using
<c_x^+ c_y> = delta_xy - G_yx; it is unchanged by the rotation.  The total
energy per site is E = E_kin + U D (the paper leaves "Ener" to the user).
"""
import numpy as np


def measured_green(model, G: np.ndarray) -> np.ndarray:
    if model.trotter == "sym":
        return model.expK_half @ G @ model.expK_half_inv
    return G


def equal_time(model, G: np.ndarray):
    """Returns (D, E_kin, E_pot) per site for one configuration."""
    Gt = measured_green(model, G)
    d = np.diag(Gt)
    D = float(np.mean(d * (1.0 - d)))
    ekin = float(model.n_col / model.N * (np.trace(model.K) - np.trace(model.K @ G)))
    return D, ekin, model.U * D


def density(model, G: np.ndarray) -> float:
    """Per-site density in the sampling frame, (N_col/N) sum_i (1 - G_ii)."""
    return float(model.n_col / model.N * np.sum(1.0 - np.diag(G)))


def jackknife(values: np.ndarray):
    """Delete-1 jackknife mean and error of the bin means (Eqs. (jack_mean),
    (jack_error)) for f = <A>."""
    v = np.asarray(values, dtype=np.float64)
    n = v.size
    loo = (v.sum() - v) / (n - 1)
    mean = loo.mean()
    err = np.sqrt((n - 1) / n * np.sum((loo - mean) ** 2))
    return float(mean), float(err)
