"""Stabilised products of slice propagators and the from-scratch Green's function.

Follows the section "Stabilization - a peculiarity of the BSS algorithm",
Eqs. (green_stable) and (diagnorm): a product A = Q D T is extended by a chunk
of n_wrap slices in three steps,

    1. M = (B_chunk Q) D            (the parentheses matter)
    2. M = Q' D' R'  by a QR decomposition, D' = |diag R'|
    3. T' = R' T

with column pivoting, the default QR of the paper's code (section "Compiling
and running", the STAB options).  Pivoting: M P = Q R, so R' = D'^-1 R P^T.

The left product B'(beta, tau) is kept as the UDV form of its transpose,
B'(beta, tau)^T = Q_L D_L T_L, built by the same three steps applied to
transposed slices.

The merge of a right form B'(tau,0) = Q_R D_R T_R with a left form into
G(tau) = (1 + B'(tau,0) B'(beta,tau))^-1 is not spelled out in the paper (its
cgr routine is only named).  Reading taken here, written out from
1 + Q_R D_R T_R T_L^T D_L Q_L^T = Q_R D_Rb X D_Lb Q_L^T with the scales split
as D^b = max(D, 1), D^s = min(D, 1):

    X = D_Rb^-1 (Q_R^T Q_L) D_Lb^-1 + D_Rs (T_R T_L^T) D_Ls
    G = Q_L D_Lb^-1 X^-1 D_Rb^-1 Q_R^T

and log|det(1 + B'(beta,0))| = sum log D_Rb + sum log D_Lb + log|det X|.
"""
from dataclasses import dataclass
from typing import Optional

import numpy as np
import scipy.linalg


@dataclass
class UDV:
    Q: np.ndarray
    D: np.ndarray
    T: np.ndarray

    def matrix(self) -> np.ndarray:
        return (self.Q * self.D[None, :]) @ self.T


def identity_udv(n: int) -> UDV:
    return UDV(np.eye(n), np.ones(n), np.eye(n))


def qr_udv(M: np.ndarray):
    """Column-pivoted QR (LAPACK dgeqp3): M P = Q R; returns Q, D = |diag R|,
    Rt = D^-1 R P^T, so that M = Q D Rt (Eq. (diagnorm))."""
    Q, R, piv = scipy.linalg.qr(M, pivoting=True)
    D = np.abs(np.diag(R))
    if np.any(D < 1e-300):
        raise FloatingPointError("vanishing scale in the QR step")
    Rd = R / D[:, None]
    Rt = np.empty_like(Rd)
    Rt[:, piv] = Rd
    return Q, D, Rt


def right_step(model, field, udv: Optional[UDV], tau_lo: int, tau_hi: int) -> UDV:
    """UDV of B'(tau_hi, 0) from that of B'(tau_lo, 0) (None = identity) and the
    chunk B'_{tau_hi} ... B'_{tau_lo+1}."""
    udv = udv or identity_udv(model.N)
    Y = udv.Q.copy()
    for tau in range(tau_lo + 1, tau_hi + 1):
        Y = model.B(field, tau) @ Y
    M = Y * udv.D[None, :]
    Q, D, Rt = qr_udv(M)
    return UDV(Q, D, Rt @ udv.T)


def left_step(model, field, udv: Optional[UDV], tau_lo: int, tau_hi: int) -> UDV:
    """UDV of B'(beta, tau_lo)^T from that of B'(beta, tau_hi)^T (None = identity):
    B'(beta,tau_lo)^T = B'_{tau_lo+1}^T ... B'_{tau_hi}^T B'(beta,tau_hi)^T."""
    udv = udv or identity_udv(model.N)
    Y = udv.Q.copy()
    for tau in range(tau_hi, tau_lo, -1):
        Y = model.B(field, tau).T @ Y
    M = Y * udv.D[None, :]
    Q, D, Rt = qr_udv(M)
    return UDV(Q, D, Rt @ udv.T)


def _split(D):
    return np.maximum(D, 1.0), np.minimum(D, 1.0)


def merge(right: Optional[UDV], left: Optional[UDV], n: int):
    """G(tau) and log|det(1 + B'(tau,0) B'(beta,tau))| from a right and a left
    UDV form (None = identity).  The Q factors are orthogonal (real) or
    unitary (complex), so Q_R^-1 = Q_R^H and (Q_L^T)^-1 = conj(Q_L); for real
    factors the conjugations change nothing."""
    right = right or identity_udv(n)
    left = left or identity_udv(n)
    DRb, DRs = _split(right.D)
    DLb, DLs = _split(left.D)
    QRh = right.Q.conj().T
    QLc = left.Q.conj()
    X = (QRh @ QLc) / DRb[:, None] / DLb[None, :] \
        + (DRs[:, None] * (right.T @ left.T.T)) * DLs[None, :]
    rhs = QRh / DRb[:, None]
    Y = np.linalg.solve(X, rhs)
    G = (QLc / DLb[None, :]) @ Y
    sign, logabs = np.linalg.slogdet(X)
    logdet = float(np.sum(np.log(DRb)) + np.sum(np.log(DLb)) + logabs)
    return G, logdet


def _chunks(lo: int, hi: int, n_wrap: int):
    """Split (lo, hi] into chunks of at most n_wrap slices aligned to multiples
    of n_wrap."""
    edges = [lo]
    nxt = (lo // n_wrap + 1) * n_wrap
    while nxt < hi:
        edges.append(nxt)
        nxt += n_wrap
    edges.append(hi)
    return edges


def right_udv(model, field, tau: int) -> Optional[UDV]:
    """Stabilised B'(tau, 0) from scratch."""
    if tau == 0:
        return None
    udv = None
    e = _chunks(0, tau, model.n_wrap)
    for a, b in zip(e[:-1], e[1:]):
        udv = right_step(model, field, udv, a, b)
    return udv


def left_udv(model, field, tau: int) -> Optional[UDV]:
    """Stabilised B'(beta, tau)^T from scratch."""
    if tau == model.L:
        return None
    udv = None
    e = _chunks(tau, model.L, model.n_wrap)
    for a, b in reversed(list(zip(e[:-1], e[1:]))):
        udv = left_step(model, field, udv, a, b)
    return udv


def green_scratch(model, field, tau: int = 0) -> np.ndarray:
    """G(tau) = (1 + B'(tau,0) B'(beta,tau))^-1 recomputed stably (Eq. (Green_eq)
    evaluated with Eq. (green_stable))."""
    G, _ = merge(right_udv(model, field, tau), left_udv(model, field, tau), model.N)
    return G


def logdet_scratch(model, field) -> float:
    """log|det(1 + B'(beta, 0))|."""
    _, ld = merge(None, left_udv(model, field, 0), model.N)
    return ld


def log_weight(model, field) -> float:
    """log W(C) of Eq. (partition_2) with N_fl = 1: the field prefactor plus
    N_col log|det(1 + B'(beta,0))| (the determinant power is real and
    non-negative in the sampling frame, so the sign is one)."""
    return model.prefactor_log(field) + model.n_col * logdet_scratch(model, field)


def weight_ratio(model, field, tau: int, i: int, s_new: float) -> float:
    """W(C') / W(C) for the field of site i on slice tau changed to s_new, from
    the two weights (Eq. (partition_2)) evaluated from scratch."""
    f2 = np.array(field, dtype=np.float64)
    f2[tau - 1, i] = s_new
    return float(np.exp(log_weight(model, f2) - log_weight(model, field)))
