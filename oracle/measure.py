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


def eq_correlations(model, lat, G: np.ndarray, entries=None) -> np.ndarray:
    """Equal-time correlation functions on the Bravais lattice (section
    "Observables": correlations summed over unit cells and stored by the
    displacement R between them), per configuration, from the measured G~:

        C_o[R, a, b] = 1/N_cells sum_I O(site(I, a), site(I + R, b)),

    o = Green, SpinZ, SpinXY, Den (entries: an optional list of (R, a, b); then
    only those are evaluated and [4, len(entries)] is returned).  In the sampling frame both species carry
    the same G (G_ij = <c_i c_j^+>), the down spin is the particle-hole image
    c_{i,dn} = s_i c'^+_i with s_i the sublattice sign, and Wick's theorem gives
        Green  1/2 <c^+_{i s} c_{j s}> summed over s = 1/2 (d_ij - G_ji + s_i s_j G_ij),
        SpinZ  <S^z_i S^z_j> = 1/4 ((1 - 2 G_ii)(1 - 2 G_jj) + 2 (d_ij - G_ji) G_ij),
        SpinXY 1/2 <S^x_i S^x_j + S^y_i S^y_j> = 1/4 s_i s_j ((d_ij - G_ji)^2 + G_ij^2),
        Den    <n_i n_j> = 1 + 2 (d_ij - G_ji) G_ij.
    Returns [4, N_cells, norb, norb]."""
    Gt = measured_green(model, G)
    n = Gt.shape[0]
    L1, L2, norb = lat.L1, lat.L2, lat.norb
    nc = L1 * L2
    s = lat.sublattice_sign()
    site = -np.ones((nc, norb), dtype=int)
    for i in range(n):
        site[lat.cell_of[i], lat.orb_of[i]] = i
    todo = [(R, a, b) for R in range(nc) for a in range(norb) for b in range(norb)] if entries is None else entries
    vals = np.zeros((4, len(todo)))
    for e, (R, a, b) in enumerate(todo):
        r1, r2 = R % L1, R // L1
        for I in range(nc):
            i1, i2 = I % L1, I // L1
            J = (i1 + r1) % L1 + L1 * ((i2 + r2) % L2)
            i, j = site[I, a], site[J, b]
            d = 1.0 if i == j else 0.0
            gij, gji = Gt[i, j], Gt[j, i]
            vals[0, e] += 0.5 * (d - gji + s[i] * s[j] * gij)
            vals[1, e] += 0.25 * ((1.0 - 2.0 * Gt[i, i]) * (1.0 - 2.0 * Gt[j, j]) + 2.0 * (d - gji) * gij)
            vals[2, e] += 0.25 * s[i] * s[j] * ((d - gji) ** 2 + gij ** 2)
            vals[3, e] += 1.0 + 2.0 * (d - gji) * gij
    vals /= nc
    if entries is not None:
        return vals
    return vals.reshape(4, nc, norb, norb)


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


def eq_spin_z(model, lat, G: np.ndarray) -> np.ndarray:
    """<S^z> per orbital of the unit cell, one configuration (the one-point
    function of the section "Observables", averaged over cells): with the
    down spin the particle-hole image of the second colour, n_up = n_1 and
    n_dn = 1 - n_2, so <S^z_i> = 1/2 (<n_1> - 1 + <n_2>) = 1/2 (1 - 2 G~_ii)
    (both colours carry G).  Returns [norb]: 1/N_cells sum_I <S^z_{site(I,a)}>."""
    Gt = measured_green(model, G)
    out = np.zeros(lat.norb)
    for i in range(model.N):
        out[lat.orb_of[i]] += 0.5 * (1.0 - 2.0 * Gt[i, i])
    return out / (lat.L1 * lat.L2)
