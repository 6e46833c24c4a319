"""Stabilizer tableau simulator (Aaronson & Gottesman, PRA 70, 052328, 2004 --
the efficient Clifford simulation the paper cites in Sec. I and uses for the
Pauli-twirled comparison of Sec. IV.C).

The tableau holds n destabilizer rows, n stabilizer rows and one scratch row,
each a Pauli string (x bits, z bits) with a sign bit r.  Pauli errors only flip
signs, and a measurement's random/deterministic structure depends only on the
x/z bits, so for a batch of trajectories that run the same Clifford circuit
with different Pauli errors and outcomes the x/z bits are shared and only the
signs r[T, 2n+1] differ.  That is how the batch is stored here.

Random measurement outcomes use the trajectory's uniform u: outcome 0 iff
u < 1/2 (the Born probability of a random stabilizer outcome).
"""
from __future__ import annotations

import numpy as np

from . import channels
from .rng import uniforms

OP_INIT, OP_CNOT, OP_SRX, OP_AD, OP_PAULI, OP_MEAS = 0, 1, 2, 3, 4, 5
C_OP, C_Q0, C_Q1, C_ARG, C_LOC, C_DRAW, C_REC, C_PREV, C_TICK = range(9)


class Tableau:
    def __init__(self, n: int, T: int):
        self.n, self.T = n, T
        self.x = np.zeros((2 * n + 1, n), dtype=np.uint8)
        self.z = np.zeros((2 * n + 1, n), dtype=np.uint8)
        self.r = np.zeros((T, 2 * n + 1), dtype=np.uint8)
        for i in range(n):
            self.x[i, i] = 1          # destabilizer X_i
            self.z[n + i, i] = 1      # stabilizer Z_i  (state |0...0>)

    # --- Clifford gates (Sec. III of Aaronson-Gottesman) ---
    def h(self, a):
        self.r ^= (self.x[:, a] & self.z[:, a])[None, :]
        self.x[:, a], self.z[:, a] = self.z[:, a].copy(), self.x[:, a].copy()

    def s(self, a):
        self.r ^= (self.x[:, a] & self.z[:, a])[None, :]
        self.z[:, a] ^= self.x[:, a]

    def cnot(self, a, b):
        self.r ^= (self.x[:, a] & self.z[:, b] & (self.x[:, b] ^ self.z[:, a] ^ 1))[None, :]
        self.x[:, b] ^= self.x[:, a]
        self.z[:, a] ^= self.z[:, b]

    # --- Pauli errors on a subset of trajectories ---
    def pauli(self, a, which: np.ndarray):
        """which[T] in {0:I, 1:X, 2:Y, 3:Z}."""
        fx = (which == 1) | (which == 2)     # X or Y part anticommutes with Z-type rows
        fz = (which == 3) | (which == 2)
        self.r ^= (fx[:, None] & self.z[None, :, a].astype(bool)).astype(np.uint8)
        self.r ^= (fz[:, None] & self.x[None, :, a].astype(bool)).astype(np.uint8)

    def flip_x(self, a, mask):
        self.pauli(a, np.where(mask, 1, 0))

    def flip_z(self, a, mask):
        self.pauli(a, np.where(mask, 3, 0))

    # --- measurement ---
    @staticmethod
    def _g(x1, z1, x2, z2):
        x1 = x1.astype(np.int64); z1 = z1.astype(np.int64)
        x2 = x2.astype(np.int64); z2 = z2.astype(np.int64)
        return np.where((x1 == 0) & (z1 == 0), 0,
               np.where((x1 == 1) & (z1 == 1), z2 - x2,
               np.where((x1 == 1) & (z1 == 0), z2 * (2 * x2 - 1), x2 * (1 - 2 * z2))))

    def rowsum(self, h, i):
        gsum = int(self._g(self.x[i], self.z[i], self.x[h], self.z[h]).sum())
        tot = 2 * self.r[:, h].astype(np.int64) + 2 * self.r[:, i].astype(np.int64) + gsum
        self.r[:, h] = ((tot % 4) // 2).astype(np.uint8)
        self.x[h] ^= self.x[i]
        self.z[h] ^= self.z[i]

    def measure_z(self, a, u: np.ndarray) -> np.ndarray:
        n = self.n
        rows = np.nonzero(self.x[n:2 * n, a])[0]
        if rows.size:
            p = n + int(rows[0])
            for i in range(2 * n):
                if i != p and self.x[i, a]:
                    self.rowsum(i, p)
            self.x[p - n] = self.x[p]
            self.z[p - n] = self.z[p]
            self.r[:, p - n] = self.r[:, p]
            self.x[p] = 0
            self.z[p] = 0
            self.z[p, a] = 1
            out = (u >= 0.5).astype(np.uint8)
            self.r[:, p] = out
            return out
        s = 2 * n
        self.x[s] = 0
        self.z[s] = 0
        self.r[:, s] = 0
        for i in range(n):
            if self.x[i, a]:
                self.rowsum(s, i + n)
        return self.r[:, s].copy()

    def stabilizers(self) -> np.ndarray:
        """[n, 2n] generator matrix (x bits | z bits)."""
        n = self.n
        return np.concatenate([self.x[n:2 * n], self.z[n:2 * n]], axis=1)


def run(circ, theta, gamma, seed: int, traj_ids, stop_after_op=None, on_tick=None):
    """Run a Clifford + Pauli op list (channels "none", "pta_*").

    Returns (records [T, n_rec], tableau).  `on_tick(tick, tableau)` is called
    after the last op of every tick (used for bond-dimension pins)."""
    traj_ids = np.asarray(traj_ids, dtype=np.uint64).reshape(-1)
    T = traj_ids.size
    ops = np.asarray(circ.ops)
    th = np.broadcast_to(np.asarray(theta, dtype=np.float64).reshape(-1, circ.n_loc) if np.ndim(theta) else
                         np.full((1, circ.n_loc), float(theta)), (T, circ.n_loc))
    ga = np.broadcast_to(np.asarray(gamma, dtype=np.float64).reshape(-1, circ.n_loc) if np.ndim(gamma) else
                         np.full((1, circ.n_loc), float(gamma)), (T, circ.n_loc))
    U = uniforms(seed, traj_ids, circ.n_draws)
    tab = Tableau(circ.n_qubits, T)
    records = np.zeros((T, circ.n_rec), dtype=np.uint8)
    for k, row in enumerate(ops):
        op, q0, q1, arg, loc, draw, rec, prev = (int(row[C_OP]), int(row[C_Q0]), int(row[C_Q1]),
                                                 int(row[C_ARG]), int(row[C_LOC]), int(row[C_DRAW]),
                                                 int(row[C_REC]), int(row[C_PREV]))
        if op == OP_INIT:
            # known previous state -> requested basis state (the reset)
            if prev == 0:
                tab.flip_x(q0, records[:, rec] == 1)
                if arg == 1:
                    tab.h(q0)
            elif prev == 1:
                tab.flip_z(q0, records[:, rec] == 1)
                if arg == 0:
                    tab.h(q0)
            else:
                if arg == 1:
                    tab.h(q0)
        elif op == OP_CNOT:
            tab.cnot(q0, q1)
        elif op == OP_PAULI:
            cache = {}
            vals = th[:, loc] if arg == 0 else ga[:, loc]
            pr = np.empty((T, 4))
            for t in range(T):
                key = float(vals[t])
                if key not in cache:
                    cache[key] = channels.pta_srx_probs(key) if arg == 0 else channels.pta_ad_probs(key)
                pr[t] = cache[key]
            cum = np.cumsum(pr, axis=1)
            u = U[:, draw]
            choice = np.argmax(u[:, None] < cum, axis=1)
            choice[u >= cum[:, -1]] = 3
            tab.pauli(q0, choice)
        elif op == OP_MEAS:
            if arg == 1:
                tab.h(q0)
            m = tab.measure_z(q0, U[:, draw])
            if arg == 1:
                tab.h(q0)
            records[:, rec] = m
        elif op in (OP_SRX, OP_AD):
            raise ValueError("non-Clifford channel in a stabilizer run")
        else:
            raise ValueError(op)
        if on_tick is not None and (k + 1 == len(ops) or int(ops[k + 1][C_TICK]) != int(row[C_TICK])):
            on_tick(int(row[C_TICK]), tab)
        if stop_after_op is not None and k == stop_after_op:
            break
    return records, tab
