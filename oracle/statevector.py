"""Quantum-trajectory simulation on a dense state vector (complex128).

Follows Sec. III.C: the mixed state is approximated by an average over pure
trajectories.  Unitary gates and coherent errors (SRX, Eq. 1) act directly.
Amplitude damping (Eq. 2-3) is unravelled exactly by its Kraus operators: with
p1 = <psi|K1^dag K1|psi> = gamma <n_q>, the trajectory jumps (psi -> K1 psi /
sqrt(p1)) when its uniform draw u < p1 and otherwise evolves by K0 (psi ->
K0 psi / sqrt(1 - p1)), so the trajectory average reproduces Eq. 2 exactly.
(The paper's Trotterised no-jump gate, diag(1, e^{-gamma/2}) from the
effective Hamiltonian of Sec. III.C, equals K0 only to first order in gamma;
the exact unravelling is the default reading, the Trotterised one is
ad_mode="trotter": same jump probability gamma <n_q> and jump K1 psi / sqrt(p1),
but no jump evolves by the Trotter gate M, psi -> M psi / |M psi|, with
probability 1 - p1.)

Measurements follow the Born rule: p0 = <psi|Pi_0|psi>, outcome 0 iff u < p0,
psi -> Pi_m psi / sqrt(p_m); outcome 0 is the +1 eigenvector (|0> or |+>).
Each trajectory accumulates log P = sum log p of every sampled event.

Ancillas are held only between their initialisation and their measurement
("lazy ancillas"): after a measurement the qubit is a known product factor and
is dropped from the register; a later initialisation adds it back in the
requested state, which is exactly the reset.  The live register is therefore
n + P qubits (10 at d=3, 28 at d=5).

All trajectories of a batch are evolved together as one array [T, 2, ..., 2].
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import channels
from .rng import uniforms

OP_INIT, OP_CNOT, OP_SRX, OP_AD, OP_PAULI, OP_MEAS = 0, 1, 2, 3, 4, 5
C_OP, C_Q0, C_Q1, C_ARG, C_LOC, C_DRAW, C_REC, C_PREV, C_TICK = range(9)


@dataclass
class TrajResult:
    records: np.ndarray     # [T, n_rec] uint8
    branches: np.ndarray    # [T, n_ad] int8 (Kraus index of each AD op)
    logp: np.ndarray        # [T] float64
    probs: np.ndarray       # [T, n_draws] probability of each sampled event (nan if none)


class SVState:
    """Dense state of the live qubits of T trajectories."""

    def __init__(self, T: int, initial_live):
        self.live = list(initial_live)
        self.psi = np.zeros((T,) + (2,) * len(self.live), dtype=np.complex128)
        self.psi[(slice(None),) + (0,) * len(self.live)] = 1.0
        self.T = T
        # known product state of dropped qubits: qubit -> 2-vector
        self.known = {}

    def axis(self, q: int) -> int:
        return 1 + self.live.index(q)

    def apply_1q(self, q: int, m: np.ndarray):
        """m: [2,2] or [T,2,2] acting on qubit q."""
        ax = self.axis(q)
        p = np.moveaxis(self.psi, ax, -1)
        if m.ndim == 2:
            p = np.einsum("...j,ij->...i", p, m)
        else:
            mm = m.reshape((self.T,) + (1,) * (p.ndim - 2) + (2, 2))
            p = np.einsum("...j,...ij->...i", p, mm)
        self.psi = np.moveaxis(p, -1, ax)

    def apply_cnot(self, c: int, t: int):
        ac, at = self.axis(c), self.axis(t)
        p = np.moveaxis(self.psi, (ac, at), (1, 2)).copy()
        p[:, 1] = p[:, 1, ::-1]
        self.psi = np.moveaxis(p, (1, 2), (ac, at))

    def prob_one(self, q: int) -> np.ndarray:
        """<n_q> per trajectory (state assumed normalised)."""
        ax = self.axis(q)
        sl = [slice(None)] * self.psi.ndim
        sl[ax] = 1
        a = self.psi[tuple(sl)]
        return np.sum(np.abs(a.reshape(self.T, -1)) ** 2, axis=1)

    def add_qubit(self, q: int, vec: np.ndarray):
        self.psi = np.multiply.outer(self.psi, vec)
        self.live.append(q)
        self.known.pop(q, None)

    def drop_qubit(self, q: int, outcome: np.ndarray, vec_of_outcome):
        """Keep slice `outcome` (per trajectory) of qubit q and drop its axis."""
        ax = self.axis(q)
        p = np.moveaxis(self.psi, ax, 1)
        idx = np.asarray(outcome, dtype=np.int64)
        self.psi = p[np.arange(self.T), idx]
        self.live.remove(q)
        self.known[q] = vec_of_outcome

    def norm2(self) -> np.ndarray:
        return np.sum(np.abs(self.psi.reshape(self.T, -1)) ** 2, axis=1)

    def full_state(self, n_qubits: int) -> np.ndarray:
        """Amplitudes over all qubits [T, 2**n_qubits], qubit 0 the most
        significant bit; dropped / untouched qubits are their known product
        factor (|0> if never initialised)."""
        psi = self.psi
        order = list(self.live)
        for q in range(n_qubits):
            if q not in order:
                v = self.known.get(q)
                if v is None:
                    v = np.array([1.0, 0.0], dtype=np.complex128)
                if np.ndim(v) == 1:
                    psi = np.multiply.outer(psi, v)
                else:   # per-trajectory vector [T, 2]
                    psi = psi[..., None] * v.reshape((self.T,) + (1,) * (psi.ndim - 1) + (2,))
                order.append(q)
        perm = [0] + [1 + order.index(q) for q in range(n_qubits)]
        return np.transpose(psi, perm).reshape(self.T, -1)


def _col(params, T, n_loc):
    a = np.asarray(params, dtype=np.float64)
    if a.ndim == 1:
        a = a.reshape(1, -1)
    return np.broadcast_to(a, (T, n_loc))


def _pta(kind: int, values: np.ndarray) -> np.ndarray:
    """[T, 4] twirled Pauli probabilities for per-trajectory parameters."""
    out = np.empty((values.size, 4))
    cache = {}
    for i, v in enumerate(values):
        key = float(v)
        if key not in cache:
            cache[key] = channels.pta_srx_probs(key) if kind == 0 else channels.pta_ad_probs(key)
        out[i] = cache[key]
    return out


def run(circ, theta, gamma, seed: int, traj_ids, forced_records=None,
        forced_branches=None, stop_after_op: int | None = None,
        uniforms_override=None, ad_mode: str = "kraus"):
    """Run the op list for the trajectories `traj_ids`.

    theta, gamma: [n_loc] or [T, n_loc] per-location parameters.
    forced_records / forced_branches: if given, outcomes are taken from them
    instead of sampled (log P of a given record, A12 reading).
    stop_after_op: return (result, state) after executing op index k.
    ad_mode: "kraus" (exact unravelling) or "trotter" (the no-jump branch
    evolves by the Trotterised gate diag(1, e^{-gamma/2}), renormalised).
    """
    if ad_mode not in ("kraus", "trotter"):
        raise ValueError("ad_mode must be 'kraus' or 'trotter'")
    traj_ids = np.asarray(traj_ids, dtype=np.uint64).reshape(-1)
    T = traj_ids.size
    ops = np.asarray(circ.ops)
    th = _col(theta, T, circ.n_loc)
    ga = _col(gamma, T, circ.n_loc)
    U = uniforms_override if uniforms_override is not None else uniforms(seed, traj_ids, circ.n_draws)
    data = [int(q) for q in circ.code.data_label]
    st = SVState(T, data)
    records = np.zeros((T, circ.n_rec), dtype=np.uint8)
    branches = np.zeros((T, circ.n_ad), dtype=np.int8)
    probs = np.full((T, circ.n_draws), np.nan)
    logp = np.zeros(T)
    ad_j = 0
    ar = np.arange(T)
    for k, row in enumerate(ops):
        op, q0, q1, arg, loc, draw, rec = (int(row[C_OP]), int(row[C_Q0]), int(row[C_Q1]),
                                            int(row[C_ARG]), int(row[C_LOC]), int(row[C_DRAW]),
                                            int(row[C_REC]))
        if op == OP_INIT:
            vec = np.array([1.0, 0.0], dtype=np.complex128) if arg == 0 else \
                np.array([1.0, 1.0], dtype=np.complex128) / np.sqrt(2.0)
            if q0 in st.live:
                # a qubit that was never measured is still |0>: prepare by H if |+> is asked
                if arg == 1:
                    st.apply_1q(q0, channels.H)
            else:
                st.add_qubit(q0, vec)
        elif op == OP_CNOT:
            st.apply_cnot(q0, q1)
        elif op == OP_SRX:
            m = np.stack([channels.srx_unitary(t) for t in th[:, loc]])
            st.apply_1q(q0, m)
        elif op == OP_AD:
            g = ga[:, loc]
            p1 = np.clip(g * st.prob_one(q0), 0.0, 1.0)
            if forced_branches is not None:
                jump = np.asarray(forced_branches)[:, ad_j].astype(bool)
            else:
                jump = U[:, draw] < p1
            p = np.where(jump, p1, 1.0 - p1)
            m = np.zeros((T, 2, 2), dtype=np.complex128)
            with np.errstate(divide="ignore", invalid="ignore"):
                if ad_mode == "kraus":
                    # K1 / sqrt(p1) on jump, K0 / sqrt(1 - p1) otherwise
                    m[:, 0, 1] = np.where(jump, np.sqrt(g) / np.sqrt(p), 0.0)
                    m[:, 0, 0] = np.where(jump, 0.0, 1.0 / np.sqrt(p))
                    m[:, 1, 1] = np.where(jump, 0.0, np.sqrt(1.0 - g) / np.sqrt(p))
                else:
                    # K1 / sqrt(p1) on jump; otherwise the Trotter gate
                    # diag(1, e^{-g/2}) over the norm it leaves, which is
                    # sqrt(1 - <n_q> (1 - e^{-g})), not sqrt(1 - p1)
                    n1 = st.prob_one(q0)
                    nrm = np.sqrt(1.0 - n1 * (1.0 - np.exp(-g)))
                    m[:, 0, 1] = np.where(jump, np.sqrt(g) / np.sqrt(p), 0.0)
                    m[:, 0, 0] = np.where(jump, 0.0, 1.0 / nrm)
                    m[:, 1, 1] = np.where(jump, 0.0, np.exp(-g / 2.0) / nrm)
                logp += np.log(p)
            st.apply_1q(q0, m)
            branches[:, ad_j] = jump
            probs[:, draw] = p
            ad_j += 1
        elif op == OP_PAULI:
            vals = th[:, loc] if arg == 0 else ga[:, loc]
            pr = _pta(arg, vals)
            cum = np.cumsum(pr, axis=1)
            u = U[:, draw]
            choice = np.argmax(u[:, None] < cum, axis=1)
            choice[u >= cum[:, -1]] = 3
            m = np.stack([channels.PAULIS[c] for c in choice])
            st.apply_1q(q0, m)
            probs[:, draw] = pr[ar, choice]
        elif op == OP_MEAS:
            if arg == 1:
                st.apply_1q(q0, channels.H)
            p0 = np.clip(1.0 - st.prob_one(q0), 0.0, 1.0)
            if forced_records is not None:
                mres = np.asarray(forced_records)[:, rec].astype(np.int64)
            else:
                mres = (U[:, draw] >= p0).astype(np.int64)
            p = np.where(mres == 0, p0, 1.0 - p0)
            with np.errstate(divide="ignore"):
                logp += np.log(p)
            if arg == 0:
                vecs = np.where(mres[:, None] == 0, np.array([1.0, 0.0]), np.array([0.0, 1.0]))
            else:
                s = 1.0 / np.sqrt(2.0)
                vecs = np.where(mres[:, None] == 0, np.array([s, s]), np.array([s, -s]))
            st.drop_qubit(q0, mres, vecs.astype(np.complex128))
            with np.errstate(divide="ignore", invalid="ignore"):
                st.psi = st.psi / np.sqrt(p).reshape((T,) + (1,) * (st.psi.ndim - 1))
            records[:, rec] = mres
            probs[:, draw] = p
        else:
            raise ValueError(f"unknown op {op}")
        if stop_after_op is not None and k == stop_after_op:
            return TrajResult(records, branches, logp, probs), st
    res = TrajResult(records, branches, logp, probs)
    if stop_after_op is not None:
        return res, st
    return res
