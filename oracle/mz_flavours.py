"""The M_z form of the Hubbard model with two flavours and two Green's
functions (oracle side; test infrastructure: only the tests, the smoke check
and the CPU leg of the benchmark use it).

Section "The M_z-Hubbard model on a square lattice" (Eq. (hubbard_Mz)):
N_fl = 2 flavours (the spins), N_col = 1, and per site one vertex coupled to
the magnetisation, V = +1 on the up flavour and -1 on the down flavour, with
alpha = 0.  Each flavour has its own hopping matrix K_sigma (a Zeeman field,
a chemical potential, spin-dependent hopping).  Since (n - 1)^2 = 1 -
(n_up - n_dn)^2 on a site, the interaction (U/2)(n - 1)^2 is decoupled
exactly by the two-valued field,

    exp(-dtau U/2 (n - 1)^2) = exp(-dtau U/2) 1/2 sum_{s = +-1} exp(lambda s (n_up - n_dn)),
    cosh(lambda) = exp(dtau U / 2),

at any filling (the four-valued field of Eq. (HS_squares) and a Gaussian
field apply to the same square with couplings sqrt(dtau U/2) and sqrt(dtau U)).
The slice propagator of flavour sigma (sign +1 up, -1 down) is
B_sigma,tau = diag(exp(sigma lambda s_tau)) exp(-dtau K_sigma), and the
weight (Eq. (partition_2)) is

    W(C) = prod(vertex factors) det(1 + B_up(beta, 0)) det(1 + B_dn(beta, 0)),

real but not of one sign once the flavours differ beyond the particle-hole
symmetric case (a chemical potential): the sign problem of the section
"The sign problem".

Readings where the paper is silent:
- the chain samples |W| and carries the sign of W relative to its starting
  configuration (taken as +1: a constant factor that cancels in every
  average); a flip is accepted iff u < |R| and the sign is multiplied by
  sign(R); the bins hold sign-weighted sums, with the sum of the signs in
  place of the count, so <O> = bins[k] / bins[3] (the paper's reweighting by
  the sign);
- the flip: Delta_sigma = exp(sigma lambda (s' - s)) - 1,
  r_sigma = 1 + Delta_sigma (1 - G_sigma,ii), R = (vertex factor ratio) r_up r_dn,
  and each flavour's Sherman-Morrison update with its own Delta / r;
- estimators in the original frame, n_sigma,i = 1 - G~_sigma,ii:
  D = <n_up n_dn>, E_kin = (1/N) sum_sigma (Tr K_sigma - Tr(K_sigma G_sigma)),
  E_pot = (U/2)(1/N) sum_i <(n_i - 1)^2> = (U/2)(1/N) sum_i (1 - n_up - n_dn + 2 n_up n_dn),
  the last equal to U D at half filling.
"""
import numpy as np

from . import hubbard, philox
from .stable import left_udv, left_step, merge, right_step


def mz_coupling(U: float, dtau: float, field_kind: str = "ising") -> float:
    return {"ising": hubbard.ising_coupling, "gauss": hubbard.gauss_coupling,
            "ising4": hubbard.ising4_coupling}[field_kind](U, dtau)


class MzModel:
    """Two flavour models sharing the field: flavour 0 (up) with +coupling,
    flavour 1 (down) with -coupling, alpha = 0, N_col = 1 each."""

    def __init__(self, K_up, K_dn, U, beta, dtau, n_wrap, field_kind="ising", trotter="sym", seed=0):
        lam = mz_coupling(U, dtau, field_kind)
        self.fl = [hubbard.Model(K=K, beta=beta, dtau=dtau, n_wrap=n_wrap, coupling=sgn * lam, U=U, alpha=0.0,
                                 n_col=1, field_kind=field_kind, trotter=trotter, seed=seed)
                   for K, sgn in ((K_up, 1.0), (K_dn, -1.0))]
        m = self.fl[0]
        self.N, self.L, self.n_wrap, self.n_stab = m.N, m.L, m.n_wrap, m.n_stab
        self.coupling = lam
        self.U = U
        self.field_kind = field_kind
        self.trotter = trotter
        self.seed = seed
        self.prop_width = m.prop_width

    def vertex_log_factor(self, s):
        return self.fl[0].vertex_log_factor(s)


def logdet_signed(model: hubbard.Model, field) -> tuple:
    """(sign, log|det(1 + B(beta, 0))|) from the stabilised left form
    B(beta, 0)^T = Q D T: with D_b = max(D, 1), D_s = min(D, 1) and the
    merge's bounded matrix against the identity right form,
    X = Q D_b^-1 + T^T D_s, one has 1 + B = X D_b Q^T, so
    det(1 + B) = det(X) prod(D_b) det(Q)."""
    left = left_udv(model, field, 0)
    if left is None:
        return 1.0, 0.0
    Db, Ds = np.maximum(left.D, 1.0), np.minimum(left.D, 1.0)
    X = left.Q / Db[None, :] + left.T.T * Ds[None, :]
    sX, lX = np.linalg.slogdet(X)
    sQ, _ = np.linalg.slogdet(left.Q)
    return float(sX * sQ), float(lX + np.sum(np.log(Db)))


def log_weight_signed(mm: MzModel, field) -> tuple:
    """(sign, log|W(C)|) of the two-flavour weight."""
    sign, lw = 1.0, float(np.sum(mm.vertex_log_factor(field)))
    for m in mm.fl:
        s, l = logdet_signed(m, field)
        sign *= s
        lw += l
    return sign, lw


def equal_time_mz(mm: MzModel, Gs) -> np.ndarray:
    """(D, E_kin, E_pot) per site of one configuration from the two flavours'
    G (original frame)."""
    from .measure import measured_green
    n = [1.0 - np.diag(measured_green(m, G)) for m, G in zip(mm.fl, Gs)]
    D = np.mean(n[0] * n[1])
    ekin = sum(np.trace(m.K) - np.trace(m.K @ G) for m, G in zip(mm.fl, Gs)) / mm.N
    epot = 0.5 * mm.U * np.mean(1.0 - n[0] - n[1] + 2.0 * n[0] * n[1])
    return np.array([D, ekin, epot])


def green_scratch_mz(mm: MzModel, field, tau: int = 0):
    from .stable import green_scratch
    return [green_scratch(m, field, tau) for m in mm.fl]


class MzChain:
    """The sweep of Algorithm 1 for two flavours: per slice both G's are
    wrapped, the flips use the product of the flavours' ratios, and every
    n_wrap slices both are recomputed from their own stored UDV forms."""

    def __init__(self, mm: MzModel, field, sweep_counter: int = 0):
        self.mm = mm
        self.field = np.array(field, dtype=np.float64)
        self.sweep_counter = int(sweep_counter)
        self.G = None
        self.slots = None
        self.bins = np.zeros(4)
        self.proposals = 0
        self.accepted = 0
        self.sign = 1.0
        self.prec = []
        self.min_tie = np.inf
        self.trace = None

    def init(self):
        mm = self.mm
        self.slots = []
        self.G = []
        for m in mm.fl:
            sl = [None] * (mm.n_stab + 1)
            left = None
            for k in range(mm.n_stab - 1, -1, -1):
                left = left_step(m, self.field, left, k * m.n_wrap, (k + 1) * m.n_wrap)
                sl[k] = left
            self.slots.append(sl)
            self.G.append(merge(None, sl[0], m.N)[0])
        return self

    def _propose(self, tau, i, u, u1):
        mm = self.mm
        s = self.field[tau - 1, i]
        if mm.field_kind == "ising":
            s_new = -s
        elif mm.field_kind == "ising4":
            k = int(hubbard.ising4_index(s))
            j = min(int(3.0 * u1), 2)
            s_new = hubbard.ETA4[j if j < k else j + 1]
        else:
            s_new = s + mm.prop_width * (2.0 * u1 - 1.0)
        R = np.exp(float(mm.vertex_log_factor(s_new)) - float(mm.vertex_log_factor(s)))
        deltas, rs = [], []
        for m, G in zip(mm.fl, self.G):
            d = np.exp(m.coupling * (s_new - s)) - 1.0
            r = 1.0 + d * (1.0 - G[i, i])
            deltas.append(d)
            rs.append(r)
            R *= r
        self.proposals += 1
        self.min_tie = min(self.min_tie, abs(abs(R) - u))
        acc = bool(u < abs(R))
        if acc:
            for f in range(2):
                G = self.G[f]
                col = G[:, i].copy()
                row = -G[i, :].copy()
                row[i] += 1.0
                self.G[f] = G - (deltas[f] / rs[f]) * np.outer(col, row)
            self.field[tau - 1, i] = s_new
            self.accepted += 1
            self.sign *= np.sign(R)
        if self.trace is not None:
            self.trace.append(("flip", tau, i, float(R), float(u), acc))
        return acc

    def _update_slice(self, tau, direction):
        mm = self.mm
        w = philox.philox4x64_10_vec(np.uint64(philox.TAG_FLIP), np.uint64(self.sweep_counter),
                                     np.uint64(philox.slot(tau, direction)),
                                     np.arange(mm.N, dtype=np.uint64), (mm.seed, 0))
        u = philox.to_unit(w[0])
        u1 = philox.to_unit(w[1])
        for i in range(mm.N):
            self._propose(tau, i, float(u[i]), float(u1[i]))

    def _measure(self, measure):
        if measure:
            o = equal_time_mz(self.mm, self.G)
            self.bins += self.sign * np.array([o[0], o[1], o[2], 1.0])

    def sweep(self, measure=True):
        mm = self.mm
        nw, nk = mm.n_wrap, mm.n_stab
        if self.G is None:
            self.init()
        rights = [None, None]
        for tau in range(1, mm.L + 1):
            self.G = [m.B(self.field, tau) @ G @ m.B_inv(self.field, tau) for m, G in zip(mm.fl, self.G)]
            self._update_slice(tau, philox.DIR_UP)
            if tau % nw == 0:
                k = tau // nw
                news, dev = [], 0.0
                for f, m in enumerate(mm.fl):
                    rights[f] = right_step(m, self.field, rights[f], tau - nw, tau)
                    left = self.slots[f][k] if k < nk else None
                    Gs, _ = merge(rights[f], left, m.N)
                    self.slots[f][k] = rights[f]
                    dev = max(dev, float(np.max(np.abs(self.G[f] - Gs))))
                    news.append(Gs)
                self.prec.append(dev)
                self.G = news
            self._measure(measure)
        lefts = [None, None]
        for tau in range(mm.L, 0, -1):
            self._update_slice(tau, philox.DIR_DOWN)
            self._measure(measure)
            Gw = [m.B_inv(self.field, tau) @ G @ m.B(self.field, tau) for m, G in zip(mm.fl, self.G)]
            if (tau - 1) % nw == 0:
                k = (tau - 1) // nw
                news, dev = [], 0.0
                for f, m in enumerate(mm.fl):
                    lefts[f] = left_step(m, self.field, lefts[f], tau - 1, tau - 1 + nw)
                    right = self.slots[f][k] if k > 0 else None
                    Gs, _ = merge(right, lefts[f], m.N)
                    self.slots[f][k] = lefts[f]
                    dev = max(dev, float(np.max(np.abs(Gw[f] - Gs))))
                    news.append(Gs)
                self.prec.append(dev)
                self.G = news
            else:
                self.G = Gw
        self.sweep_counter += 1
        return self


def init_field(mm: MzModel, seed=None):
    """Random start with the draws of hubbard.init_field."""
    return hubbard.init_field(mm.fl[0], seed)


__all__ = ["MzModel", "mz_coupling", "logdet_signed", "log_weight_signed", "equal_time_mz", "green_scratch_mz",
           "MzChain", "init_field"]
