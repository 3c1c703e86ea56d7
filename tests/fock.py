"""Fock-space evaluation of Trotterised Hubbard expectation values (a pin).

Independent of the oracle: the repulsive Hubbard Hamiltonian
H = sum_sigma c^+ K_sigma c - h sum_i (n_i,up - n_i,dn) + (U/2) sum_i (n_i - 1)^2
(h an optional Zeeman field, part of the one-body H_T; K_up = K_dn = K unless
a separate down-spin hopping is given) is built as a 4^N-dimensional
matrix from Jordan-Wigner fermions, and the symmetric Trotter product
S = exp(-dtau H_T/2) exp(-dtau H_U) exp(-dtau H_T/2) of the section
"The partition function" gives

    <O> = Tr(S^L O) / Tr(S^L),
    <A(tau) B(0)> = Tr(S^(L-n) A S^n B) / Tr(S^L)   (tau = n dtau).

Only the physics (not the determinant method) enters, so agreement with the
oracle's enumeration pins the HS constants, the weight, the particle-hole
frame map and the measured Green's function together.
"""
import numpy as np


def _expmh(H, x):
    w, V = np.linalg.eigh(H)
    return (V * np.exp(x * w)[None, :]) @ V.T


class Fock:
    def __init__(self, K, U, h=0.0, K_dn=None):
        K = np.asarray(K, dtype=float)
        Ks = (K, K if K_dn is None else np.asarray(K_dn, dtype=float))
        self.N = N = K.shape[0]
        nm = 2 * N
        dim = 2 ** nm
        a = np.array([[0.0, 1.0], [0.0, 0.0]])    # annihilator on one mode
        Z = np.diag([1.0, -1.0])
        I2 = np.eye(2)
        self.c = []
        for m in range(nm):
            op = np.array([[1.0]])
            for j in range(nm):
                op = np.kron(op, Z if j < m else (a if j == m else I2))
            self.c.append(op)
        self.dim = dim

        def mode(i, s):
            return 2 * i + s

        HT = np.zeros((dim, dim))
        for s in range(2):
            for i in range(N):
                for j in range(N):
                    if Ks[s][i, j] != 0.0:
                        HT += Ks[s][i, j] * self.c[mode(i, s)].T @ self.c[mode(j, s)]
        self.n = [[self.c[mode(i, s)].T @ self.c[mode(i, s)] for s in range(2)] for i in range(N)]
        for i in range(N):
            HT -= h * (self.n[i][0] - self.n[i][1])
        HU = np.zeros((dim, dim))
        for i in range(N):
            ni = self.n[i][0] + self.n[i][1] - np.eye(dim)
            HU += 0.5 * U * ni @ ni
        self.HT, self.HU = HT, HU

    def trotter(self, dtau):
        Th = _expmh(self.HT, -dtau / 2)
        return Th @ _expmh(self.HU, -dtau) @ Th

    def trotter_asym(self, dtau):
        """exp(-dtau H_U) exp(-dtau H_T): the split whose equal-time Green's
        function at a slice boundary is the sampling-frame G'."""
        return _expmh(self.HU, -dtau) @ _expmh(self.HT, -dtau)

    def double_occ(self):
        return sum(self.n[i][0] @ self.n[i][1] for i in range(self.N)) / self.N

    def kinetic(self):
        return self.HT / self.N

    def potential(self):
        return self.HU / self.N

    def sz(self, i):
        return 0.5 * (self.n[i][0] - self.n[i][1])

    def expect(self, O, dtau, L):
        return self.expect_with(self.trotter(dtau), O, L)

    def expect_with(self, S, O, L):
        P = np.linalg.matrix_power(S, L)
        return float(np.trace(P @ O) / np.trace(P))

    def expect_tau(self, A, B, dtau, L, n):
        return self.expect_tau_with(self.trotter(dtau), A, B, L, n)

    def expect_tau_with(self, S, A, B, L, n):
        Z = np.trace(np.linalg.matrix_power(S, L))
        return float(np.trace(np.linalg.matrix_power(S, L - n) @ A @ np.linalg.matrix_power(S, n) @ B) / Z)
