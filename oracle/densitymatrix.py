"""Exact channel evolution on a dense density matrix (complex128).

The quantity the trajectories approximate (Sec. III.C): rho evolved by the
gates and by the channels themselves (Eq. 1: U rho U^dag; Eq. 2:
sum_k K_k rho K_k^dag; Eq. 9: sum_i eta_ii P_i rho P_i).  A measurement is
either unconditioned (the qubit is traced out, which is what an unread
measurement followed by a reset does) or conditioned on a given outcome m
(rho -> Pi_m rho Pi_m, unnormalised, so that Tr rho at the end is the
probability of the conditioning outcomes).

Lazy ancillas as in the state-vector oracle: a measured qubit leaves the
register; its initialisation brings it back.  The live register is n + P
qubits, so d=3 needs a 1024 x 1024 matrix.
"""
from __future__ import annotations

import numpy as np

from . import channels

OP_INIT, OP_CNOT, OP_SRX, OP_AD, OP_PAULI, OP_MEAS = 0, 1, 2, 3, 4, 5
C_OP, C_Q0, C_Q1, C_ARG, C_LOC, C_DRAW, C_REC, C_PREV, C_TICK = range(9)


class DMState:
    def __init__(self, initial_live):
        self.live = list(initial_live)
        n = len(self.live)
        self.rho = np.zeros((2,) * (2 * n), dtype=np.complex128)
        self.rho[(0,) * (2 * n)] = 1.0

    @property
    def n(self):
        return len(self.live)

    def _axes(self, q):
        i = self.live.index(q)
        return i, self.n + i

    def apply_1q(self, q, m):
        """rho -> m rho m^dag on qubit q."""
        ka, ba = self._axes(q)
        r = np.moveaxis(self.rho, ka, -1)
        r = np.einsum("...j,ij->...i", r, m)
        r = np.moveaxis(r, -1, ka)
        r = np.moveaxis(r, ba, -1)
        r = np.einsum("...j,ij->...i", r, m.conj())
        self.rho = np.moveaxis(r, -1, ba)

    def apply_channel(self, q, kraus):
        acc = None
        saved = self.rho
        for K in kraus:
            self.rho = saved
            self.apply_1q(q, K)
            acc = self.rho if acc is None else acc + self.rho
        self.rho = acc

    def apply_pauli_channel(self, q, probs):
        acc = None
        saved = self.rho
        for p, P in zip(probs, channels.PAULIS):
            self.rho = saved
            self.apply_1q(q, P)
            term = p * self.rho
            acc = term if acc is None else acc + term
        self.rho = acc

    def apply_cnot(self, c, t):
        g = np.eye(4, dtype=np.complex128)[[0, 1, 3, 2]].reshape(2, 2, 2, 2)
        kc, bc = self._axes(c)
        kt, bt = self._axes(t)
        r = np.moveaxis(self.rho, (kc, kt), (-2, -1))
        r = np.einsum("...ab,xyab->...xy", r, g)
        r = np.moveaxis(r, (-2, -1), (kc, kt))
        r = np.moveaxis(r, (bc, bt), (-2, -1))
        r = np.einsum("...ab,xyab->...xy", r, g.conj())
        self.rho = np.moveaxis(r, (-2, -1), (bc, bt))

    def add_qubit(self, q, vec):
        n = self.n
        proj = np.outer(vec, vec.conj())
        r = np.multiply.outer(self.rho, proj)          # axes: ket(n) bra(n) k_new b_new
        r = np.moveaxis(r, 2 * n, n)                    # ket(n) k_new bra(n) b_new
        self.rho = r
        self.live.append(q)

    def drop_qubit(self, q, outcome=None):
        """Trace out q (outcome None) or keep its (m, m) block."""
        ka, ba = self._axes(q)
        if outcome is None:
            r = np.trace(self.rho, axis1=ka, axis2=ba)
        else:
            r = np.moveaxis(self.rho, (ka, ba), (0, 1))[outcome, outcome]
        self.rho = r
        self.live.remove(q)

    def trace(self) -> float:
        n = self.n
        return float(np.real(np.trace(self.rho.reshape(2 ** n, 2 ** n))))

    def diag_probs(self, order) -> np.ndarray:
        """Z-basis probabilities over `order` (first = most significant)."""
        n = self.n
        m = self.rho.reshape(2 ** n, 2 ** n)
        d = np.real(np.diag(m)).reshape((2,) * n)
        perm = [self.live.index(q) for q in order]
        return np.transpose(d, perm).reshape(-1)


def evolve(circ, theta, gamma, record=None, stop_before_final=True):
    """Evolve the op list exactly.

    theta, gamma: [n_loc] per-location parameters.
    record: optional [n_rec] outcomes; measurements whose record index is
    given (>= 0 entry) are conditioned on it, the others are traced out.
    Returns the DMState, stopped before the final data measurements when
    `stop_before_final` (the data qubits are then the live register).
    """
    ops = np.asarray(circ.ops)
    theta = np.broadcast_to(np.asarray(theta, dtype=np.float64), (circ.n_loc,))
    gamma = np.broadcast_to(np.asarray(gamma, dtype=np.float64), (circ.n_loc,))
    data = [int(q) for q in circ.code.data_label]
    final_recs = set(int(r) for r in circ.data_rec)
    st = DMState(data)
    for row in ops:
        op, q0, q1, arg, loc, rec = (int(row[C_OP]), int(row[C_Q0]), int(row[C_Q1]),
                                     int(row[C_ARG]), int(row[C_LOC]), int(row[C_REC]))
        if op == OP_INIT:
            if q0 in st.live:
                if arg == 1:
                    st.apply_1q(q0, channels.H)
            else:
                vec = np.array([1.0, 0.0], dtype=np.complex128) if arg == 0 else \
                    np.array([1.0, 1.0], dtype=np.complex128) / np.sqrt(2.0)
                st.add_qubit(q0, vec)
        elif op == OP_CNOT:
            st.apply_cnot(q0, q1)
        elif op == OP_SRX:
            st.apply_1q(q0, channels.srx_unitary(theta[loc]))
        elif op == OP_AD:
            st.apply_channel(q0, channels.ad_kraus(gamma[loc]))
        elif op == OP_PAULI:
            pr = channels.pta_srx_probs(theta[loc]) if arg == 0 else channels.pta_ad_probs(gamma[loc])
            st.apply_pauli_channel(q0, pr)
        elif op == OP_MEAS:
            if stop_before_final and rec in final_recs:
                break
            if arg == 1:
                st.apply_1q(q0, channels.H)
            out = None
            if record is not None and int(record[rec]) >= 0:
                out = int(record[rec])
            st.drop_qubit(q0, out)
        else:
            raise ValueError(op)
    return st


def final_data_distribution(circ, theta, gamma, record=None) -> np.ndarray:
    """Distribution of the final data bits over data index order (data 0 most
    significant).  With `record`, it is the joint probability with the
    conditioned syndrome bits (unnormalised)."""
    st = evolve(circ, theta, gamma, record=record, stop_before_final=True)
    return st.diag_probs([int(q) for q in circ.code.data_label])
