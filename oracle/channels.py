"""Single-qubit error channels of the paper, written from their definitions.

SRX (Eq. 1): a coherent over-rotation about X.  The paper writes e^{-i theta X};
this build's parameter is the full rotation angle, U = exp(-i theta X / 2)
(so theta_paper = theta / 2).

AD (Eq. 2-3): Kraus operators K0 = diag(1, sqrt(1-gamma)), K1 = sqrt(gamma)|0><1|.

Pauli twirl (Sec. IV.C, Eq. 9): expand a channel in the Pauli basis,
E[rho] = sum_ij eta_ij P_i rho P_j, and keep only the diagonal eta_ii.
For a channel with Kraus operators K_k, K_k = sum_i c_ki P_i with
c_ki = Tr(P_i K_k) / 2, hence eta_ij = sum_k c_ki conj(c_kj).
"""
from __future__ import annotations

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
PAULIS = (I2, X, Y, Z)


def srx_unitary(theta: float) -> np.ndarray:
    """exp(-i theta X / 2), from the power series of a Pauli exponential."""
    return np.cos(theta / 2.0) * I2 - 1j * np.sin(theta / 2.0) * X


def ad_kraus(gamma: float) -> tuple:
    k0 = np.array([[1.0, 0.0], [0.0, np.sqrt(1.0 - gamma)]], dtype=np.complex128)
    k1 = np.array([[0.0, np.sqrt(gamma)], [0.0, 0.0]], dtype=np.complex128)
    return k0, k1


def ad_trotter_nojump(gamma: float) -> np.ndarray:
    """The no-jump gate of the Trotterised effective Hamiltonian (Sec. III.C):
    with the single jump operator L1 = K1 / sqrt(dt) of Eq. 3 the factor
    exp(-(dt/2) L1^dag L1) is exp(-(gamma/2) |1><1|) = diag(1, e^{-gamma/2}).
    It agrees with K0 = diag(1, sqrt(1 - gamma)) only to first order in gamma;
    the jump itself (K1, probability gamma <n1>) is the same in both readings."""
    return np.array([[1.0, 0.0], [0.0, np.exp(-gamma / 2.0)]], dtype=np.complex128)


def pauli_process_matrix(kraus) -> np.ndarray:
    """eta_ij of Eq. 9's Pauli-basis expansion (4x4, Hermitian)."""
    c = np.array([[np.trace(P @ K) / 2.0 for P in PAULIS] for K in kraus])
    return np.einsum("ki,kj->ij", c, c.conj())


def twirl_probs(kraus) -> np.ndarray:
    """(p_I, p_X, p_Y, p_Z) = diag(eta) of Eq. 9."""
    eta = pauli_process_matrix(kraus)
    return np.real(np.diag(eta)).copy()


def pta_srx_probs(theta: float) -> np.ndarray:
    return twirl_probs([srx_unitary(theta)])


def pta_ad_probs(gamma: float) -> np.ndarray:
    return twirl_probs(list(ad_kraus(gamma)))
