"""The Monte Carlo sweep of the oracle (Algorithm 1 of the section "Pseudo code
description", with the update rules of the section "Updating schemes").

One sweep is an upward pass tau = 1..L followed by a downward pass tau = L..1;
every field is visited twice (section "Monte Carlo sampling").

Upward pass, per slice tau:
    G <- B'_tau G B'_tau^-1                       (wrap; wrapgrup)
    sequential single flips at sites 0..N-1        (wrapgrup)
    at a stabilisation point tau = k n_wrap:       (wrapur, storage, cgr,
        right form B'(tau_k,0) from the previous one and the chunk,
        read the left form of slot k, write the right form to slot k,
        G_s <- merge, precision <- max|G - G_s|, G <- G_s  control_precisionG)
    measure on G(tau)                              (obser)
Downward pass, per slice tau:
    sequential single flips at sites 0..N-1, measure on G(tau)
    G_w <- B'_tau^-1 G B'_tau                      (wrap down to tau - 1)
    if tau - 1 = k n_wrap: left form of B'(beta, tau_k)^T, read the right
        form of slot k, write the left form, G <- merge, precision vs G_w
    else G <- G_w

Readings where the paper is silent: sites are visited in the order 0..N-1 in
both passes; the recomputed G replaces the wrapped one; measurements are taken
on every slice of both passes; Metropolis acceptance is "accept iff u < R"
with R the full weight ratio (min(1, R) implied); the random numbers follow
the Philox addressing of oracle.philox.

Flip of the field on (i, tau) (from Eq. (Green_eq) and the matrix determinant
lemma; the paper only states the O(N^2) cost of the fast update): the leftmost
factor exp(V_tau) of B'(tau, 0) is multiplied by (1 + Delta e_i e_i^T) with
Delta = exp(coupling (s' - s)) - 1, so

    r = 1 + Delta (1 - G_ii),  R = exp(N_col coupling alpha (s' - s)) r^N_col
    G <- G - (Delta / r) G[:, i] (e_i - G[i, :])      (Sherman-Morrison)

For a Gaussian field the move is phi' = phi + a (2 u1 - 1) and R carries the
extra factor exp(-(phi'^2 - phi^2) / 2).  For the four-valued field of
Eq. (HS_squares) the move picks one of the three other values, index
floor(3 u1) among them in increasing order (a symmetric proposal), and R
carries gamma(l') / gamma(l).
"""
import numpy as np

from . import philox
from .measure import equal_time
from .stable import left_step, merge, right_step


class Chain:
    def __init__(self, model, field: np.ndarray, sweep_counter: int = 0):
        self.m = model
        self.field = np.array(field, dtype=np.float64)
        self.sweep_counter = int(sweep_counter)
        self.G = None
        self.slots = None
        self.bins = np.zeros(4)           # sums of D, E_kin, E_pot and the count
        self.proposals = 0
        self.accepted = 0
        self.prec = []                    # max|G_wrapped - G_scratch| per stabilisation
        self.trace = None                 # optional per-event record
        self.min_tie = np.inf             # min |R - u| over all proposals
        self.eq_lat = None                # lattice for the lattice-resolved correlations, if measured
        self.eq_entries = None            # optional list of (R, a, b) to evaluate
        self.eq_bins = None
        self.eq_sz = None

    # -- setup (Algorithm 1: confin, then the wrapul fill) ----------------------
    def init(self):
        m = self.m
        nk = m.n_stab
        self.slots = [None] * (nk + 1)
        left = None
        for k in range(nk - 1, -1, -1):
            left = left_step(m, self.field, left, k * m.n_wrap, (k + 1) * m.n_wrap)
            self.slots[k] = left
        self.G, _ = merge(None, self.slots[0], m.N)
        return self

    # -- one flip (section "The default: sequential single spin flips") --------
    def _propose(self, tau: int, i: int, u: float, u1: float):
        m = self.m
        s = self.field[tau - 1, i]
        if m.field_kind == "ising":
            s_new = -s
        elif m.field_kind == "ising4":
            # one of the three other values of the four-valued field, equally likely
            from .hubbard import ETA4, ising4_index
            k = int(ising4_index(s))
            j = min(int(3.0 * u1), 2)
            kn = j if j < k else j + 1
            s_new = ETA4[kn]
        else:
            s_new = s + m.prop_width * (2.0 * u1 - 1.0)
        # the change of the vertex's own factor in the weight (zero, the
        # Gaussian measure, or gamma(l') / gamma(l))
        extra = float(m.vertex_log_factor(s_new)) - float(m.vertex_log_factor(s))
        delta = np.exp(m.coupling * (s_new - s)) - 1.0
        r = 1.0 + delta * (1.0 - self.G[i, i])
        R = np.exp(m.n_col * m.coupling * m.alpha * (s_new - s) + extra) * r ** m.n_col
        self.proposals += 1
        self.min_tie = min(self.min_tie, abs(R - u))
        acc = bool(u < R)
        if acc:
            G = self.G
            col = G[:, i].copy()
            row = -G[i, :].copy()
            row[i] += 1.0
            self.G = G - (delta / r) * np.outer(col, row)
            self.field[tau - 1, i] = s_new
            self.accepted += 1
        if self.trace is not None:
            self.trace.append(("flip", tau, i, float(R), float(u), acc))
        return acc

    def _update_slice(self, tau: int, direction: int):
        m = self.m
        w = philox.philox4x64_10_vec(np.uint64(philox.TAG_FLIP), np.uint64(self.sweep_counter),
                                     np.uint64(philox.slot(tau, direction)),
                                     np.arange(m.N, dtype=np.uint64), (m.seed, 0))
        u = philox.to_unit(w[0])
        u1 = philox.to_unit(w[1])
        for i in range(m.N):
            self._propose(tau, i, float(u[i]), float(u1[i]))

    def _measure(self, measure: bool):
        if measure:
            D, ekin, epot = equal_time(self.m, self.G)
            self.bins += np.array([D, ekin, epot, 1.0])
            if self.eq_lat is not None:
                from .measure import eq_correlations
                c = eq_correlations(self.m, self.eq_lat, self.G, self.eq_entries)
                self.eq_bins = c if self.eq_bins is None else self.eq_bins + c
                from .measure import eq_spin_z
                mz = eq_spin_z(self.m, self.eq_lat, self.G)
                self.eq_sz = mz if self.eq_sz is None else self.eq_sz + mz

    def _stabilise(self, G_s, G_cmp):
        self.prec.append(float(np.max(np.abs(G_cmp - G_s))))
        if self.trace is not None:
            self.trace.append(("stab", G_s.copy(), self.prec[-1]))
        self.G = G_s

    # -- one sweep -----------------------------------------------------------
    def sweep(self, measure: bool = True, max_slices=None):
        """One sweep.  max_slices (a bounded sample, for timing only): stop
        after that many slices of the upward pass, leaving the sweep
        unfinished and the sweep counter where it was."""
        m = self.m
        nw = m.n_wrap
        nk = m.n_stab
        if self.G is None:
            self.init()
        # upward pass
        right = None
        for tau in range(1, m.L + 1):
            if max_slices is not None and tau > max_slices:
                return self
            self.G = m.B(self.field, tau) @ self.G @ m.B_inv(self.field, tau)
            self._update_slice(tau, philox.DIR_UP)
            if tau % nw == 0:
                k = tau // nw
                right = right_step(m, self.field, right, tau - nw, tau)
                left = self.slots[k] if k < nk else None
                G_s, _ = merge(right, left, m.N)
                self.slots[k] = right
                self._stabilise(G_s, self.G)
            self._measure(measure)
        # downward pass
        left = None
        for tau in range(m.L, 0, -1):
            self._update_slice(tau, philox.DIR_DOWN)
            self._measure(measure)
            G_w = m.B_inv(self.field, tau) @ self.G @ m.B(self.field, tau)
            if (tau - 1) % nw == 0:
                k = (tau - 1) // nw
                left = left_step(m, self.field, left, tau - 1, tau - 1 + nw)
                right = self.slots[k] if k > 0 else None
                G_s, _ = merge(right, left, m.N)
                self.slots[k] = left
                self._stabilise(G_s, G_w)
            else:
                self.G = G_w
        self.sweep_counter += 1
        return self
