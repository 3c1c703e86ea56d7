"""Time-displaced Green's functions and the S^z-S^z correlation at one
momentum (oracle side).

Definitions (section "Measuring time displaced observables", with the
sampling-frame propagators B'(tau2, tau1) of Eq. (Green_eq)):

    GT0(tau) = B'(tau,0) G(0)                 = (B'(tau,0)^-1 + B'(beta,tau))^-1
    G0T(tau) = -(1 - G(0)) B'(tau,0)^-1        = -(B'(tau,0) + B'(beta,tau)^-1)^-1
    GTT(tau) = G(tau),  G00 = G(0).

The paper does not say how these are evaluated stably.  Reading taken here:
with the right form B'(tau,0) = Q_R D_R T_R, the left form
B'(beta,tau)^T = Q_L D_L T_L and the same scale split as the equal-time merge
(D^b = max(D,1), D^s = min(D,1)), both inverses reduce to the same bounded
matrix X = D_Rb^-1 (Q_R^T Q_L) D_Lb^-1 + D_Rs (T_R T_L^T) D_Ls:

    GTT = Q_L D_Lb^-1 X^-1 D_Rb^-1 Q_R^T
    GT0 = Q_L D_Lb^-1 X^-1 D_Rs T_R
    G0T = -T_L^T D_Ls X^-1 D_Rb^-1 Q_R^T

(write B'(tau,0)^-1 + B'(beta,tau) = T_R^-1 D_Rs^-1 X D_Lb Q_L^T and
B'(tau,0) + B'(beta,tau)^-1 = Q_R D_Rb X D_Ls^-1 T_L^-T).

Estimator (Wick's theorem per colour; the repulsive S^z maps to
(n_1 + n_2 - 1)/2 of the two sampling-frame colours under the partial
particle-hole map, so the paper's SU(2) result -2 G0T_yx GT0_xy gains the
disconnected term that vanishes only on average):

    4 <S^z_x(tau) S^z_y(0)> = (1 - 2 GTT_xx)(1 - 2 G00_yy) - 2 G0T_yx GT0_xy,

and S_ab(K, tau) = (1/N_uc) sum_{I,J} exp(-i K.(R_I - R_J)) <S^z_{I,a}(tau) S^z_{J,b}(0)>
(Eq. (s_corr) with the factor i that the printed exponent drops).  With the
symmetric Trotter split all four Green's functions are taken after the
rotation exp(-dtau K/2) (.) exp(+dtau K/2), as the equal-time one.
"""
import numpy as np

from .hubbard import green_naive, product_B
from .stable import identity_udv, left_udv, right_udv


def tdgf_scratch(model, field, tau: int):
    """(GT0, G0T, GTT) at slice tau from scratch, by the stabilised forms."""
    n = model.N
    right = right_udv(model, field, tau) or identity_udv(n)
    left = left_udv(model, field, tau) or identity_udv(n)
    DRb, DRs = np.maximum(right.D, 1.0), np.minimum(right.D, 1.0)
    DLb, DLs = np.maximum(left.D, 1.0), np.minimum(left.D, 1.0)
    X = (right.Q.T @ left.Q) / DRb[:, None] / DLb[None, :] \
        + (DRs[:, None] * (right.T @ left.T.T)) * DLs[None, :]
    Y1 = np.linalg.solve(X, right.Q.T / DRb[:, None])
    Y2 = np.linalg.solve(X, DRs[:, None] * right.T)
    GTT = (left.Q / DLb[None, :]) @ Y1
    GT0 = (left.Q / DLb[None, :]) @ Y2
    G0T = -(left.T.T * DLs[None, :]) @ Y1
    return GT0, G0T, GTT


def tdgf_naive(model, field, tau: int):
    """The definitions with plain products and inverses (tiny, well
    conditioned cases only)."""
    G0 = green_naive(model, field, 0)
    Bt = product_B(model, field, tau, 0)
    GT0 = Bt @ G0
    G0T = -(np.eye(model.N) - G0) @ np.linalg.inv(Bt)
    return GT0, G0T, green_naive(model, field, tau)


def _rotate(model, M):
    if model.trotter == "sym":
        return model.expK_half @ M @ model.expK_half_inv
    return M


def szsz_k(model, lat, kvec, GT0, G0T, GTT, G00):
    """[norb, norb] complex S_ab(K, tau) of one configuration."""
    GT0, G0T, GTT, G00 = (_rotate(model, M) for M in (GT0, G0T, GTT, G00))
    n = model.N
    szsz = np.empty((n, n))
    for x in range(n):
        for y in range(n):
            szsz[x, y] = 0.25 * ((1.0 - 2.0 * GTT[x, x]) * (1.0 - 2.0 * G00[y, y]) - 2.0 * G0T[y, x] * GT0[x, y])
    R = lat.cell_pos[lat.cell_of]                      # [N, 2] cell position of each orbital
    ph = np.exp(-1j * (R @ np.asarray(kvec, dtype=float)))
    S = np.zeros((lat.norb, lat.norb), dtype=complex)
    for x in range(n):
        for y in range(n):
            S[lat.orb_of[x], lat.orb_of[y]] += ph[x] * np.conj(ph[y]) * szsz[x, y]
    return S / lat.n_cells


def td_correlations(model, lat, GT0, G0T, GTT, G00, entries=None):
    """Time-displaced correlation functions on the Bravais lattice (section
    "Observables": correlations summed over unit cells and stored by the
    displacement R; section "Measuring time displaced observables" for the
    time-displaced Green's functions), one configuration at one tau:

        C_o[R, a, b] = 1/N_cells sum_I <O_i(tau) O_j(0)>,  i = site(I, a), j = site(I + R, b),

    o = Green, SpinZ, SpinXY, Den.  Wick's theorem per sampling-frame colour,
    both colours carrying the same Green's functions and the down spin the
    particle-hole image c_{i,dn} = s_i c'^+_i (s the sublattice sign), with
    <c^+_i(tau) c_j(0)> = -G0T_ji and <c_i(tau) c^+_j(0)> = GT0_ij:
        Green  1/2 sum_s <c^+_{i s}(tau) c_{j s}(0)>  = 1/2 (-G0T_ji + s_i s_j GT0_ij)
        SpinZ  <S^z_i(tau) S^z_j(0)>                  = 1/4 ((1 - 2 GTT_ii)(1 - 2 G00_jj) - 2 G0T_ji GT0_ij)
        SpinXY 1/2 <S^x_i S^x_j + S^y_i S^y_j>(tau)   = 1/4 s_i s_j (G0T_ji^2 + GT0_ij^2)
        Den    <n_i(tau) n_j(0)>                      = 1 - 2 G0T_ji GT0_ij.
    At tau = 0 (GT0 = G, G0T = G - 1) these are the equal-time estimators.
    With the symmetric split all four are rotated as the equal-time G.
    Returns [4, N_cells, norb, norb], or [4, len(entries)] for an optional list
    of (R, a, b) entries, the only ones then evaluated."""
    GT0, G0T, GTT, G00 = (_rotate(model, M) for M in (GT0, G0T, GTT, G00))
    L1, L2, norb = lat.L1, lat.L2, lat.norb
    nc = L1 * L2
    s = lat.sublattice_sign()
    site = -np.ones((nc, norb), dtype=int)
    for i in range(model.N):
        site[lat.cell_of[i], lat.orb_of[i]] = i
    todo = [(R, a, b) for R in range(nc) for a in range(norb) for b in range(norb)] if entries is None else entries
    vals = np.zeros((4, len(todo)))
    for e, (R, a, b) in enumerate(todo):
        for I in range(nc):
            i1, i2 = I % L1, I // L1
            J = (i1 + R % L1) % L1 + L1 * ((i2 + R // L1) % L2)
            i, j = site[I, a], site[J, b]
            h, g = G0T[j, i], GT0[i, j]
            vals[0, e] += 0.5 * (-h + s[i] * s[j] * g)
            vals[1, e] += 0.25 * ((1.0 - 2.0 * GTT[i, i]) * (1.0 - 2.0 * G00[j, j]) - 2.0 * h * g)
            vals[2, e] += 0.25 * s[i] * s[j] * (h * h + g * g)
            vals[3, e] += 1.0 - 2.0 * h * g
    vals /= nc
    if entries is not None:
        return vals
    return vals.reshape(4, nc, norb, norb)


def tdgf_correlations(model, lat, field, taus=None, entries=None):
    """td_correlations for tau in taus (default 0..L) of one configuration,
    every tau from scratch: [len(taus), 4, N_cells, norb, norb] (or
    [len(taus), 4, len(entries)])."""
    taus = range(model.L + 1) if taus is None else taus
    _, _, G00 = tdgf_scratch(model, field, 0)
    out = []
    for tau in taus:
        GT0, G0T, GTT = tdgf_scratch(model, field, tau)
        out.append(td_correlations(model, lat, GT0, G0T, GTT, G00, entries))
    return np.array(out)


def tdgf_measure(model, lat, kvec, field, taus=None):
    """S_ab(K, tau) for tau in taus (default 0..L) of one configuration, every
    tau evaluated from scratch."""
    taus = range(model.L + 1) if taus is None else taus
    _, _, G00 = tdgf_scratch(model, field, 0)
    out = []
    for tau in taus:
        GT0, G0T, GTT = tdgf_scratch(model, field, tau)
        out.append(szsz_k(model, lat, kvec, GT0, G0T, GTT, G00))
    return np.array(out)
